"""Benchmark: block-Lanczos kernel columns phi(L) E_W on one MI355X.

Workload (default): random geometric graph, N = 100,000 points uniform in the
unit square, symmetrised 8-NN, Gaussian weights with sigma = median 8-NN
distance; spline kernel (0.01 I + L)^(-2); s = 64 samples; m = 40 blocks;
classical block Lanczos.  One step = one krylov_kernel_columns call (all
stages: start block, SpMM + orthogonalisation per block, phi of the projected
matrix, assembly of the n x s columns) with the Laplacian and samples resident
on the device and the columns written to device memory.

Metric: kernel columns per second of the mixed-precision path, valid only if
its columns match the float64 GPU path to 1e-5 relative Frobenius error
(checked in the same run).  Printed as one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Roof of each kernel class: (bound, peak, unit, source file or files).  Peaks are the
# MI355X datasheet figures: HBM3E 8 TB/s, FP64 vector and FP64 matrix
# 78.6 TFLOP/s, FP32 matrix 157.3 TFLOP/s (dense).
ROOFS = {
    "spmm_diff": ("hbm", HBM_PEAK_GBS, "GB/s", "spmm.hip"),
    "reduce_parts": ("hbm", HBM_PEAK_GBS, "GB/s", "ortho.hip"),
    "panel_gramv": ("mfma", 78.6, "TFLOP/s", "panel.hip"),
    "panel_update_self": ("mfma", 78.6, "TFLOP/s", "panel.hip"),
    "panel_apply_self": ("mfma", 78.6, "TFLOP/s", "panel.hip"),
    "panel_apply_write": ("mfma", 78.6, "TFLOP/s", "panel.hip"),
    "arch_gram": ("mfma", 157.3, "TFLOP/s", "arch.hip"),
    "arch_update": ("mfma", 157.3, "TFLOP/s", "arch.hip"),
    "gram": ("mfma", 78.6, "TFLOP/s", "ortho.hip"),
    "tsgemm": ("mfma", 78.6, "TFLOP/s", "ortho.hip"),
    "assemble": ("mfma", 157.3, "TFLOP/s", "arch.hip"),
    "predict": ("hbm", HBM_PEAK_GBS, "GB/s", "ortho.hip"),
    "cholqr": ("alu", 78.6, "TFLOP/s", ("small.hip", "tile64.h")),
    "omega": ("alu", 78.6, "TFLOP/s", ("small.hip", "tile64.h")),
    "banded_factor": ("alu", 78.6, "TFLOP/s", ("bcr.hip", "tile64.h")),
    "banded_solve": ("alu", 78.6, "TFLOP/s", ("bcr.hip", "tile64.h")),
    "cheb_step": ("alu", 78.6, "TFLOP/s", ("small.hip", "tile64.h")),
    "jacobi_eig": ("alu", 78.6, "TFLOP/s", ("small.hip", "tile64.h")),
}


def _kernel_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2301_06384_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_from_profile(kernel: str, workload: str, src_hash: str):
    """HBM bytes per launch of a kernel from a committed rocprofv3 --pmc
    summary, only if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(p):
        return None
    vals = {}
    with open(p) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != src_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _achieved(k):
    bound, peak, unit, _ = ROOFS.get(k["name"], ("alu", 78.6, "TFLOP/s", ""))
    t = k["total_ms"] * 1e-3
    if t <= 0:
        return bound, peak, unit, 0.0
    a = k["alg_bytes"] / t / 1e9 if unit == "GB/s" else k["alg_flops"] / t / 1e12
    return bound, peak, unit, a


def cpu_baseline(L, W, phi, m, s_sample: int):
    """The FP64 oracle on a bounded sample: the same graph, phi and m, the
    first s_sample of the samples."""
    from oracle import krylov
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas_threads = max([i.get("num_threads", 1) for i in info] or [1])
    except Exception:
        blas_threads = None
    A = L.to_scipy()
    t0 = time.perf_counter()
    krylov.cbl(A, W[:s_sample], phi, m)
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    return dict(value=s_sample / dt, unit="cols/s", cores=blas_threads or cores, host_cores=cores,
                kind="oracle", seconds=dt,
                sample=f"float64 CPU oracle cbl on the full graph with the first {s_sample} of the "
                       f"{len(W)} samples, same phi and m (BLAS threads {blas_threads}; scipy sparse "
                       f"products single-threaded)")


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def serving_bench(gk, I, n_req: int, seed: int = 0, max_active: int = 8, n_streams: int = 8):
    """Serving workload: 8 resident random geometric graphs (N 10k..500k),
    requests with s ~ U{4..128}, diffusion or spline kernels, m = 30, cbl,
    mixed precision, fit + predict on all N nodes.  A closed-loop warm-up
    measures the saturated throughput; the timed stream has Poisson arrivals
    at 0.7 x that rate.  Latency = completion - scheduled arrival."""
    t_gen = time.perf_counter()
    pool = I.serving_pool()
    graphs = [gk.Graph.from_laplacian(L, flags=gk.REORDER) for L in pool]
    sizes = [L.n for L in pool]
    t_gen = time.perf_counter() - t_gen
    srv = gk.Server(max_active=max_active, hbm_budget=0, n_streams=n_streams)
    try:
        warm = I.serving_requests(min(64, n_req), sizes, seed=seed + 1)
        t0 = time.perf_counter()
        tk = [srv.submit(graphs[r["graph"]], r["samples"], r["y"], r["phi"], r["m"], r["gamma"]) for r in warm]
        for t in tk:
            res = srv.poll(t, -1)
            if res["status"] != 0:
                raise RuntimeError(f"warm-up request failed with status {res['status']}")
        sat = len(warm) / (time.perf_counter() - t0)
        lam = 0.7 * sat
        _progress(f"serving: saturated {sat:.2f} req/s, arrivals at {lam:.2f} req/s")
        reqs = I.serving_requests(n_req, sizes, seed=seed)
        arrivals = np.cumsum(np.random.default_rng(seed + 2).exponential(1.0 / lam, n_req))
        start = time.perf_counter()
        subs = []
        for r, ta in zip(reqs, arrivals):
            now = time.perf_counter() - start
            if ta > now:
                time.sleep(ta - now)
            t_host = time.perf_counter() - start
            if len(subs) % 64 == 63:
                _progress(f"serving: {len(subs) + 1}/{n_req} submitted")
            subs.append((srv.submit(graphs[r["graph"]], r["samples"], r["y"], r["phi"], r["m"], r["gamma"]), ta,
                         t_host))
        _progress(f"serving: {n_req} requests submitted")
        lat, fails, done_at = [], 0, []
        for ticket, ta, t_host in subs:
            res = srv.poll(ticket, -1)
            if res["status"] != 0:
                fails += 1
                continue
            service = (res["t_complete_ms"] - res["t_submit_ms"]) * 1e-3
            lat.append(service + (t_host - ta))
            done_at.append(t_host + service)
        span = max(done_at) - arrivals[0] if done_at else float("nan")
    finally:
        srv.stop()
    lat = np.sort(np.asarray(lat))
    return {"requests": n_req, "failed": fails, "graphs_n": sizes, "max_active": max_active,
            "streams": n_streams, "saturated_req_per_s": sat, "arrival_rate_req_per_s": lam,
            "throughput_req_per_s": len(lat) / span, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)), "mean_ms": 1e3 * float(lat.mean()),
            "pool_build_s": t_gen,
            "workload": "8 RGG 8-NN graphs N=10k..500k (seeds 100+i); s~U{4..128}; diffusion t~U[0.1,2] or "
                        "spline eps~U[0.001,0.1] k=2; m=30; cbl mixed; gamma=1e-3; Poisson arrivals at 0.7x "
                        "saturated closed-loop throughput"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rgg100k_spline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--reorder", type=int, default=1)
    ap.add_argument("--serving-requests", type=int, default=512,
                    help="requests of the serving leg (0 skips it)")
    ap.add_argument("--counters", action="store_true",
                    help="for hardware-counter runs: one mixed step, then a 1 GiB device-to-device copy of "
                         "known size (calibration of the byte counters); prints no benchmark line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2301_06384_amd import gk
    from paper_2301_06384_amd import inputs as I

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L, W, phi, m = I.workload(args.workload)
    s = len(W)
    flags_g = gk.REORDER if args.reorder else 0
    g = gk.Graph.from_laplacian(L, flags=flags_g)
    stream = torch.cuda.current_stream()
    gk.set_stream(stream)
    Wd = torch.as_tensor(W, device=dev)
    out = {p: torch.empty((s, L.n), dtype=torch.float64, device=dev) for p in ("mixed", "fp64")}
    kout = {p: torch.empty((s, s), dtype=torch.float64, device=dev) for p in ("mixed", "fp64")}

    def step(prec, flags=0):
        gk.krylov_kernel_columns(g, Wd, phi, m, "cbl", prec, flags=gk.IO_DEVICE | flags,
                                 out_cols=out[prec], out_kww=kout[prec])

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step(prec)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    if args.counters:
        step("mixed")
        torch.cuda.synchronize()
        nbytes = 1 << 30
        x = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"counters_run": True, "copy_bytes": nbytes}), flush=True)
        return

    _progress("timing the mixed path")
    ms_mixed = timed("mixed", args.steps, args.warmup)
    _progress(f"mixed {ms_mixed:.2f} ms/step; timing the float64 path")
    ms_fp64 = timed("fp64", max(2, args.steps // 2), 1)
    P_m = out["mixed"].cpu().numpy()
    P_d = out["fp64"].cpu().numpy()
    err = float(np.linalg.norm(P_m - P_d) / np.linalg.norm(P_d))

    _progress("per-kernel timing pass")
    # per-phase and per-kernel device times of the mixed step, from HIP events
    # the library records on the stream the kernels run on (same K steps)
    agg = {}
    stats = None
    for _ in range(args.steps):
        _, _, st = gk.krylov_kernel_columns(g, Wd, phi, m, "cbl", "mixed", flags=gk.IO_DEVICE | gk.TIMING,
                                            out_cols=out["mixed"], out_kww=kout["mixed"])
        d = st.as_dict()
        if stats is not None:
            for f in ("t_spmm_ms", "t_orth_ms", "t_reorth_ms", "t_phi_ms", "t_asm_ms", "t_total_ms"):
                d[f] += stats[f]
        stats = d
        for k in gk.kernel_timings():
            if k["launches"] == 0:
                continue
            a_ = agg.setdefault(k["name"], dict(name=k["name"], launches=0, total_ms=0.0, alg_bytes=0.0,
                                                alg_flops=0.0))
            for f in ("launches", "total_ms", "alg_bytes", "alg_flops"):
                a_[f] += k[f]
    K = float(args.steps)
    kernels = {}
    for name, k in sorted(agg.items(), key=lambda kv: -kv[1]["total_ms"]):
        bound, peak, unit, ach = _achieved(k)
        kernels[name] = {"launches_per_step": k["launches"] / K, "ms_per_step": k["total_ms"] / K,
                         "avg_launch_us": 1e3 * k["total_ms"] / k["launches"], "bound": bound,
                         "achieved": ach, "unit": unit, "frac": ach / peak}
    dom = max(agg.values(), key=lambda k: k["total_ms"])
    bound, peak, unit, ach = _achieved(dom)
    src = ROOFS.get(dom["name"], (None, None, None, "small.hip"))[3]
    traffic = _traffic_from_profile(dom["name"], "rgg100k_s64", _kernel_hash([src] if isinstance(src, str) else src))
    value = s / (ms_mixed * 1e-3)
    res = {
        "metric": "kernel cols/s at 1e-5 rel err vs FP64 path",
        "value": value if err <= 1e-5 else None,
        "unit": "cols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "rgg100k_knn8_spline_eps0.01_k2_s64_m40_cbl", "n": L.n, "nnz": L.nnz,
                   "s": s, "m": m, "reorder": bool(args.reorder)},
        "rel_err_vs_fp64_path": err,
        "fp64_path": {"ms_per_step": ms_fp64, "cols_per_s": s / (ms_fp64 * 1e-3),
                      "speedup_mixed_over_fp64": ms_fp64 / ms_mixed},
        "phase_ms": {k: stats[k] / K for k in ("t_spmm_ms", "t_orth_ms", "t_reorth_ms", "t_phi_ms", "t_asm_ms",
                                               "t_total_ms")},
        "phi_method": stats["phi_method"],
        "mixed_reorth_steps": stats["n_reorth"],
        "mixed_orth_estimate": stats["orth_est"],
        "mixed_qr2_series_steps": stats["n_qr2_series"],
        "roofline": {"kernel": dom["name"], "bound": bound, "achieved": ach, "peak": peak, "unit": unit,
                     "frac": ach / peak, "traffic": traffic,
                     "avg_launch_ms": dom["total_ms"] / dom["launches"],
                     "alg_bytes_per_launch": dom["alg_bytes"] / dom["launches"],
                     "alg_flops_per_launch": dom["alg_flops"] / dom["launches"]},
        "kernels": kernels,
    }
    if args.serving_requests > 0:
        _progress("serving leg")
        res["serving"] = serving_bench(gk, I, args.serving_requests)
    if not args.no_cpu:
        _progress("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(L, W, phi, m, args.cpu_sample)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
