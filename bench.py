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
# MI355X datasheet peaks (dense): FP64 vector and matrix 78.6 TFLOP/s, FP32
# matrix 157.3 TFLOP/s, BF16 matrix 2.5 PFLOP/s.  "bf16x6": float32-accurate
# products formed as six BF16 part products each (a three-part split of both
# operands), so a sixth of the BF16 peak.
PEAK_TF = {"fp64": 78.6, "fp32": 157.3, "bf16x6": 2500.0 / 6}

# Kernel class -> (arithmetic of its flops, runs on the matrix cores, source
# files).  Single-workgroup classes form latency chains: no chip-wide roof.
CLASSES = {
    "spmm_diff": ("fp64", False, "spmm.hip"),
    "reduce_parts": ("fp64", False, "ortho.hip"),
    "panel_gramv": ("fp64", True, "panel.hip"),
    "panel_update_self": ("fp64", True, "panel.hip"),
    "panel_apply_self": ("fp64", True, "panel.hip"),
    "panel_apply_write": ("fp64", True, "panel.hip"),
    "arch_gram": ("fp32", True, ("arch.hip", "ortho.hip")),     # ld <= 64 / wider blocks
    # widths 64 k (every benchmark workload) run on the BF16 cores; 16, 32
    # and 48, and wide blocks of other widths, keep the FP32 kernels
    "arch_update": ("bf16x6", True, ("arch.hip", "ortho.hip")),
    "gram": ("fp64", True, "ortho.hip"),
    "tsgemm": ("fp64", True, "ortho.hip"),
    "assemble": ("fp32", True, ("arch.hip", "ortho.hip")),
    "predict": ("fp64", False, "ortho.hip"),
}
LATENCY = {"cholqr": ("small.hip", "tile64.h", "wide.hip"), "omega": ("small.hip", "tile64.h", "wide.hip"),
           "banded_factor": ("bcr.hip", "tile64.h"), "banded_solve": ("bcr.hip", "tile64.h"),
           "cheb_step": ("small.hip", "tile64.h"), "jacobi_eig": ("small.hip", "tile64.h"),
           # rocprofv3 names of both banded phases (bcr_*, banded_*) map to one class
           "banded": ("bcr.hip", "small.hip", "tile64.h", "wide.hip")}


def _kernel_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2301_06384_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _sources(name):
    src = CLASSES[name][2] if name in CLASSES else LATENCY.get(name, "small.hip")
    return [src] if isinstance(src, str) else list(src)


def _traffic_from_profile(kernel: str, workload: str, src_hash: str, prof_dir=None):
    """HBM bytes per launch of a kernel from a committed rocprofv3 --pmc
    summary, only if it was taken on the current kernel source."""
    p = os.path.join(prof_dir or os.path.join(ROOT, "profiles"), f"{kernel}_{workload}_traffic.txt")
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


def classify(k, assemble_dtype="fp32"):
    """Roofline of one kernel class from its algorithmic bytes and flops: the
    bound is the roof its intensity reaches first (HBM below the ridge point
    peak / 8 TB/s of its arithmetic, the compute roof above it); single
    workgroup classes are latency chains and carry no chip-wide fraction."""
    name, t = k["name"], k["total_ms"] * 1e-3
    if name in LATENCY or name not in CLASSES:
        return dict(bound="latency", achieved=None, peak=None, unit=None, frac=None, intensity=None)
    dtype, mfma, _ = CLASSES[name]
    if name == "assemble":
        dtype = assemble_dtype
    inten = k["alg_flops"] / k["alg_bytes"] if k["alg_bytes"] > 0 else float("inf")
    ridge = PEAK_TF[dtype] * 1e12 / (HBM_PEAK_GBS * 1e9)
    if t <= 0:
        return dict(bound="hbm", achieved=0.0, peak=HBM_PEAK_GBS, unit="GB/s", frac=0.0, intensity=inten)
    if inten < ridge:
        a = k["alg_bytes"] / t / 1e9
        return dict(bound="hbm", achieved=a, peak=HBM_PEAK_GBS, unit="GB/s", frac=a / HBM_PEAK_GBS,
                    intensity=inten, ridge=ridge)
    a = k["alg_flops"] / t / 1e12
    return dict(bound="mfma" if mfma else "alu", achieved=a, peak=PEAK_TF[dtype], unit="TFLOP/s",
                frac=a / PEAK_TF[dtype], intensity=inten, ridge=ridge)


def kernel_table(agg, steps, assemble_dtype="fp32"):
    """Per-class table and the whole-solve roofline of `steps` solves."""
    K = float(steps)
    table = {}
    t_bound = lat = byt = fl = 0.0
    for name, k in sorted(agg.items(), key=lambda kv: -kv[1]["total_ms"]):
        c = classify(k, assemble_dtype)
        row = {"launches_per_step": k["launches"] / K, "ms_per_step": k["total_ms"] / K,
               "avg_launch_us": 1e3 * k["total_ms"] / k["launches"],
               "alg_bytes_per_step": k["alg_bytes"] / K, "alg_flops_per_step": k["alg_flops"] / K, **c}
        table[name] = row
        if c["bound"] == "latency":
            lat += row["ms_per_step"]
            continue
        dtype = assemble_dtype if name == "assemble" else CLASSES[name][0]
        byt += row["alg_bytes_per_step"]
        fl += row["alg_flops_per_step"]
        t_bound += 1e3 * max(row["alg_bytes_per_step"] / (HBM_PEAK_GBS * 1e9),
                             row["alg_flops_per_step"] / (PEAK_TF[dtype] * 1e12))
    return table, {"alg_bytes_per_solve": byt, "alg_flops_per_solve": fl, "t_bound_ms": t_bound,
                   "latency_chain_ms": lat}


def collect_timings(run_timed, steps):
    """Aggregate gk_kernel_timings over `steps` calls made with GK_TIMING."""
    from paper_2301_06384_amd import gk
    agg, stats = {}, None
    for _ in range(steps):
        st = run_timed()
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
    return agg, stats


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


# ------------------------------------------------ rocprofv3 summaries (host)
# descriptive names of the workloads (graph, kernel, block width, depth, variant)
WORKLOAD_NAMES = {
    "rgg100k_spline": "rgg100k_knn8_spline_eps0.01_k2_s64_m40_cbl",
    "ba1m_diffusion": "ba1m_m4_diffusion_t0.5_s256_m30_cbl",
    "grid128c_spline": "grid128cube_uniform_spline_eps0.05_k1_s512_m30_cbl",
    "grid32_diffusion": "grid32x32_diffusion_t1_s8_m20_cbl",
}


def kernel_class_of(name: str):
    """Kernel class (as the library's own timings name them) of a rocprofv3
    kernel name, or None for kernels outside the path."""
    base = name.split("(")[0]
    args = []
    if "<" in base:
        args = [a.strip() for a in base[base.index("<") + 1:base.rindex(">")].split(",")]
        base = base[:base.index("<")]
    base = base.split("::")[-1]
    if base.startswith("panel_kernel") and len(args) >= 8:
        upd, app, grv, slf = (a == "true" for a in args[2:6])
        return ("panel_gramv" if grv else "panel_update_self" if upd else
                "panel_apply_self" if (app and slf) else "panel_apply_write")
    if base.startswith("tsgemm_mfma_kernel"):
        return "assemble" if len(args) >= 2 and args[1] == "true" else "tsgemm"
    table = [("spmm_", "spmm_diff"), ("reduce_parts", "reduce_parts"), ("arch_gram", "arch_gram"),
             ("arch_update", "arch_update"), ("update_bf3", "arch_update"), ("arch_assemble", "assemble"),
             ("gram_f32mma", "arch_gram"),
             ("tsgemm_f32mma", "arch_update"), ("assemble_f32mma", "assemble"), ("gram_", "gram"),
             ("tsgemm", "tsgemm"), ("predict", "predict"), ("cholqr", "cholqr"), ("omega", "omega"),
             ("bcr_", "banded"), ("banded_", "banded"), ("btd_cheb", "cheb_step"), ("jacobi", "jacobi_eig")]
    for pre, cls in table:
        if base.startswith(pre):
            return cls
    return None


def _csv_rows(d, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    with open(files[-1], newline="") as fh:
        return list(csv.DictReader(fh))


def summarize_profiles(stats_dir, fetch_dir, write_dir, workload, tag, cmd_stats, cmd_pmc, out_dir=None):
    """Write profiles/kernel_stats_<tag>.txt from a `rocprofv3 --kernel-trace
    --stats` run and profiles/<class>_<tag>_traffic.txt from two `--pmc` runs
    (FETCH_SIZE, WRITE_SIZE) of `bench.py --counters`, whose 1 GiB copy
    calibrates the byte counters."""
    out = out_dir or os.path.join(ROOT, "profiles")
    if stats_dir:
        rows = _csv_rows(stats_dir, "kernel_stats.csv")
        # register and LDS use per kernel from the trace of the same run:
        # waves per SIMD = min(8, 512 // (VGPR + AGPR), LDS-limited
        # workgroups per CU (160 KiB) x waves per workgroup / 4 SIMDs).
        # The trace's VGPR_Count is half the unified register allocation on
        # gfx950 (it equals the compiler's .amdhsa_next_free_vgpr, rounded to
        # the granule of 8, divided by 2), so it is doubled here.
        res = {}
        for t in _csv_rows(stats_dir, "kernel_trace.csv"):
            if t["Kernel_Name"] in res:
                continue
            v, a, lds = 2 * int(t["VGPR_Count"]), int(t["Accum_VGPR_Count"]), int(t["LDS_Block_Size"])
            wg = int(t["Workgroup_Size_X"]) * int(t["Workgroup_Size_Y"]) * int(t["Workgroup_Size_Z"])
            wpg = max(1, (wg + 63) // 64)
            occ = min(8, 512 // max(1, v + a))
            if lds > 0:
                occ = min(occ, (163840 // lds) * wpg // 4)
            res[t["Kernel_Name"]] = (v, a, lds, occ)
        lines = [f"# rocprofv3 kernel statistics, benchmark workload {workload}",
                 f"# command: {cmd_stats}",
                 "# vgpr/agpr: registers per lane (vgpr: the unified allocation, twice the trace's VGPR_Count); "
                 "lds: bytes per workgroup; w/simd: waves per SIMD the registers and LDS allow (at most 8)",
                 f"# {'kernel':<62} {'calls':>6} {'total_ms':>10} {'avg_us':>10} {'min_us':>9} {'max_us':>9} "
                 f"{'vgpr':>5} {'agpr':>5} {'lds':>6} {'w/simd':>6}"]
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        for r in rows:
            v, a, lds, occ = res.get(r["Name"], (-1, -1, -1, -1))
            lines.append(f"{r['Name'][:62]:<64} {int(r['Calls']):>6} {float(r['TotalDurationNs']) * 1e-6:>10.3f} "
                         f"{float(r['AverageNs']) * 1e-3:>10.2f} {float(r['MinNs']) * 1e-3:>9.2f} "
                         f"{float(r['MaxNs']) * 1e-3:>9.2f} {v:>5} {a:>5} {lds:>6} {occ:>6}")
        with open(os.path.join(out, f"kernel_stats_{tag}.txt"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    if not (fetch_dir and write_dir):
        return
    per = {}
    calib = {}
    for ctr, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        disp = {}
        for r in _csv_rows(d, "counter_collection.csv"):
            if r.get("Counter_Name") != ctr:
                continue
            key = (r["Dispatch_Id"], r["Kernel_Name"])
            disp[key] = disp.get(key, 0.0) + float(r["Counter_Value"])
        copies = [v for (i, nm), v in disp.items() if "copyBuffer" in nm or "copy" in nm.lower()]
        if not copies:
            raise SystemExit(f"{ctr}: the calibration copy is missing")
        calib[ctr] = max(copies)
        for (i, nm), v in disp.items():
            cls = kernel_class_of(nm)
            if cls is None:
                continue
            e = per.setdefault(cls, {}).setdefault(ctr, [])
            e.append(v)
    nbytes = float(1 << 30)
    fs = nbytes / 1024.0 / calib["FETCH_SIZE"]   # KiB counted per KiB moved
    ws = nbytes / 1024.0 / calib["WRITE_SIZE"]
    for cls, c in sorted(per.items()):
        if "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
            continue
        fk = sum(c["FETCH_SIZE"]) / len(c["FETCH_SIZE"])
        wk = sum(c["WRITE_SIZE"]) / len(c["WRITE_SIZE"])
        srcs = _sources(cls) if (cls in CLASSES or cls in LATENCY) else ["small.hip"]
        lines = [f"# HBM traffic of {cls} per dispatch, benchmark workload {workload} (one mixed step)",
                 f"# commands: {cmd_pmc.format(ctr='FETCH_SIZE')}  ;  {cmd_pmc.format(ctr='WRITE_SIZE')}",
                 f"# calibration: bench.py --counters copies 1 GiB device-to-device after the step; the counters "
                 f"read FETCH_SIZE {calib['FETCH_SIZE']:.1f} KiB and WRITE_SIZE {calib['WRITE_SIZE']:.1f} KiB for it",
                 f"kernel: {cls}",
                 f"source_files: {' '.join(srcs)}",
                 f"source_hash: {_kernel_hash(srcs)}",
                 f"dispatches: {len(c['FETCH_SIZE'])}",
                 f"fetch_kib_per_dispatch: {fk:.3f}",
                 f"write_kib_per_dispatch: {wk:.3f}",
                 f"fetch_scale: {fs:.5f}",
                 f"write_scale: {ws:.5f}",
                 f"hbm_bytes_per_launch: {1024.0 * (fk * fs + wk * ws):.1f}"]
        with open(os.path.join(out, f"{cls}_{tag}_traffic.txt"), "w") as fh:
            fh.write("\n".join(lines) + "\n")


def serving_bench(gk, I, n_req: int, seed: int = 0, max_active: int = 8, n_streams: int = 16):
    """Serving workload: 8 resident random geometric graphs (N 10k..500k),
    requests with s ~ U{4..128}, diffusion or spline kernels, m = 30, cbl,
    mixed precision, fit + predict on all N nodes.  The server batches the
    requests of each graph at the iteration level (one grouped SpMM and one
    batched launch per CholQR pass per round).  A closed-loop warm-up
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


def stream_copy_gbps(torch, dev, nbytes=1 << 30, reps=5):
    """Measured device-to-device copy rate (read + write bytes per second):
    the practical HBM ceiling beside the 8 TB/s datasheet figure."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * nbytes / t / 1e9


def config_leg(torch, gk, I, name, variants, fp64=True):
    """One full-size configuration: per variant, one timed call in each
    precision (device-resident inputs and outputs), the mixed-vs-float64
    error, and the per-kernel split of the mixed classical block Lanczos."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    L, W, phi, m = I.workload(name)
    g = gk.Graph.from_laplacian(L, flags=gk.REORDER)
    t_gen = time.perf_counter() - t0
    s = len(W)
    Wd = torch.as_tensor(W, device=dev)
    stream = torch.cuda.current_stream()
    out = {"workload": name, "n": L.n, "nnz": L.nnz, "s": s, "m": m, "graph_build_s": t_gen}
    gk.trim()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    foot64 = gk.request_footprint(L.n, s, m, "cbl", "fp64")
    out["fp64_footprint_GB"] = foot64 / 1e9
    out["mixed_footprint_GB"] = gk.request_footprint(L.n, s, m, "cbl", "mixed") / 1e9
    run64 = fp64 and foot64 < 0.9 * free

    def call(variant, prec, P, K, flags=0):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, _, st = gk.krylov_kernel_columns(g, Wd, phi, m, variant, prec, flags=gk.IO_DEVICE | flags,
                                            out_cols=P, out_kww=K)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), st

    Pm = torch.empty((s, L.n), dtype=torch.float64, device=dev)
    Km = torch.empty((s, s), dtype=torch.float64, device=dev)
    call("cbl", "mixed", Pm, Km)   # warm-up (allocations, code objects)
    for variant in variants:
        ms_m, st_m = call(variant, "mixed", Pm, Km)
        row = {"mixed_ms": ms_m, "mixed_cols_per_s": s / (ms_m * 1e-3), "mixed_reorth_steps": st_m.n_reorth}
        if run64:
            P64 = torch.empty_like(Pm)
            K64 = torch.empty_like(Km)
            ms_d, _ = call(variant, "fp64", P64, K64)
            row.update(fp64_ms=ms_d, fp64_cols_per_s=s / (ms_d * 1e-3), speedup_mixed_over_fp64=ms_d / ms_m,
                       rel_err_mixed_vs_fp64=float(torch.linalg.norm(Pm - P64) / torch.linalg.norm(P64)))
            del P64, K64
            torch.cuda.empty_cache()
        else:
            row["fp64"] = (f"refused by admission: float64 footprint {foot64 / 1e9:.1f} GB above 0.9 x "
                           f"free device memory {free / 1e9:.1f} GB")
        if variant == "cbl":
            Wi = torch.as_tensor(W, device=dev, dtype=torch.int64)
            Kh = Km.cpu().numpy()
            row["kww_min_eig"] = float(np.linalg.eigvalsh(0.5 * (Kh + Kh.T)).min())
            row["corollary1_gap"] = float(torch.linalg.norm(Pm[:, Wi] - Km) / torch.linalg.norm(Km))
        out[variant] = row
        _progress(f"{name} {variant}: {row}")
    agg, _ = collect_timings(lambda: call("cbl", "mixed", Pm, Km, gk.TIMING)[1], 1)
    ld = s if s <= 8 else 16 * ((s + 15) // 16)
    table, whole = kernel_table(agg, 1, "fp32")
    out["cbl_mixed_kernels"] = {k: {f: v[f] for f in ("launches_per_step", "ms_per_step", "avg_launch_us", "bound",
                                                      "achieved", "unit", "frac")} for k, v in table.items()}
    # measured HBM-side traffic (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)
    # per launch from a committed profile of this workload taken on the
    # current kernel sources, over the launch time measured here (per-launch
    # averages include the gated launches of steps that do not project)
    for k, v in out["cbl_mixed_kernels"].items():
        srcs = _sources(k) if (k in CLASSES or k in LATENCY) else None
        tb = _traffic_from_profile(k, name, _kernel_hash(srcs)) if srcs else None
        v["traffic_bytes_per_launch"] = tb
        v["traffic_GBps"] = (tb / (v["avg_launch_us"] * 1e-6) / 1e9) if (tb and v["avg_launch_us"]) else None
    out["cbl_mixed_whole_solve"] = whole
    del Pm, Km
    g.release()
    torch.cuda.empty_cache()
    return out


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
    ap.add_argument("--legs", default="ba1m_diffusion,grid128c_spline",
                    help="full-size configuration legs reported beside the benchmark ('' skips them)")
    ap.add_argument("--counters", action="store_true",
                    help="for hardware-counter runs: one mixed step, then a 1 GiB device-to-device copy of "
                         "known size (calibration of the byte counters); prints no benchmark line")
    ap.add_argument("--summarize", nargs=3, metavar=("STATS_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="host only: write the profiles/ summaries from rocprofv3 output directories "
                         "('-' skips one) and exit")
    args = ap.parse_args()
    if args.summarize:
        sd, fd, wd = (None if x == "-" else x for x in args.summarize)
        tag = {"rgg100k_spline": "rgg100k_s64"}.get(args.workload, args.workload)
        pre = "cd /tmp && export TMPDIR=/tmp && "
        wl = "" if args.workload == "rgg100k_spline" else f"--workload {args.workload} "
        steps = "--steps 3 --warmup 1" if not wl else "--steps 1 --warmup 1"
        summarize_profiles(sd, fd, wd, args.workload, tag,
                           pre + "rocprofv3 --kernel-trace --stats --output-format csv -d <out>/prof_stats -o stats "
                                 f"-- python3 <repo>/bench.py {wl}{steps} --no-cpu --serving-requests 0 --legs ''",
                           pre + "rocprofv3 --pmc {ctr} --output-format csv -d <out>/pmc -o pmc -- python3 "
                                 f"<repo>/bench.py {wl}--counters")
        return
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
        return gk.krylov_kernel_columns(g, Wd, phi, m, "cbl", prec, flags=gk.IO_DEVICE | flags,
                                        out_cols=out[prec], out_kww=kout[prec])

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
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
    ms_mixed = timed(lambda: step("mixed"), args.steps, args.warmup)
    _progress(f"mixed {ms_mixed:.2f} ms/step; timing the float64 path")
    ms_fp64 = timed(lambda: step("fp64"), max(2, args.steps // 2), 1)
    P_m = out["mixed"].cpu().numpy()
    P_d = out["fp64"].cpu().numpy()
    err = float(np.linalg.norm(P_m - P_d) / np.linalg.norm(P_d))

    # the same call with host (pinned) samples and outputs: adds the n x s
    # float64 device-to-host copy of the columns
    _progress("timing with host outputs (D2H included)")
    Wh = np.ascontiguousarray(W)
    Ph = torch.empty((s, L.n), dtype=torch.float64, pin_memory=True)
    Kh = torch.empty((s, s), dtype=torch.float64, pin_memory=True)
    ms_d2h = timed(lambda: gk.krylov_kernel_columns(g, Wh, phi, m, "cbl", "mixed", out_cols=Ph, out_kww=Kh),
                   args.steps, 1)

    _progress("per-kernel timing pass")
    # per-phase and per-kernel device times of the mixed step, from HIP events
    # the library records on the stream the kernels run on (same K steps)
    agg, stats = collect_timings(lambda: step("mixed", gk.TIMING)[2], args.steps)
    K = float(args.steps)
    kernels, whole = kernel_table(agg, args.steps, "fp32")
    copy_gbps = stream_copy_gbps(torch, dev)
    dom_name = max((k for k in kernels if kernels[k]["bound"] != "latency"), key=lambda k: kernels[k]["ms_per_step"])
    dom = kernels[dom_name]
    traffic = _traffic_from_profile(dom_name, "rgg100k_s64", _kernel_hash(_sources(dom_name)))
    value = s / (ms_mixed * 1e-3)
    whole.update(ms_per_step=ms_mixed, frac=whole["t_bound_ms"] / ms_mixed,
                 achieved_GBps=whole["alg_bytes_per_solve"] / (ms_mixed * 1e-3) / 1e9)
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
        "config": {"workload": WORKLOAD_NAMES.get(args.workload, args.workload), "n": L.n, "nnz": L.nnz,
                   "s": s, "m": m, "reorder": bool(args.reorder)},
        "rel_err_vs_fp64_path": err,
        "value_with_d2h": {"cols_per_s": s / (ms_d2h * 1e-3), "ms_per_step": ms_d2h,
                           "note": "samples on the host, columns and K_WW copied to pinned host memory"},
        "fp64_path": {"ms_per_step": ms_fp64, "cols_per_s": s / (ms_fp64 * 1e-3),
                      "speedup_mixed_over_fp64": ms_fp64 / ms_mixed},
        "phase_ms": {k: stats[k] / K for k in ("t_spmm_ms", "t_orth_ms", "t_reorth_ms", "t_phi_ms", "t_asm_ms",
                                               "t_total_ms")},
        "phi_method": stats["phi_method"],
        "mixed_reorth_steps": stats["n_reorth"],
        "mixed_orth_estimate": stats["orth_est"],
        "mixed_qr2_series_steps": stats["n_qr2_series"],
        "mixed_qr2_skipped_steps": stats["n_qr2_skipped"],
        "stream_copy_GBps": copy_gbps,
        "roofline": {"kernel": dom_name, "bound": dom["bound"], "achieved": dom["achieved"], "peak": dom["peak"],
                     "unit": dom["unit"], "frac": dom["frac"], "traffic": traffic,
                     "frac_of_stream_copy": (dom["achieved"] / copy_gbps) if dom["unit"] == "GB/s" else None,
                     "intensity_flop_per_byte": dom["intensity"], "ridge_flop_per_byte": dom.get("ridge"),
                     "avg_launch_ms": dom["avg_launch_us"] * 1e-3,
                     "alg_bytes_per_launch": dom["alg_bytes_per_step"] / dom["launches_per_step"],
                     "alg_flops_per_launch": dom["alg_flops_per_step"] / dom["launches_per_step"]},
        "whole_solve_roofline": whole,
        "kernels": kernels,
    }
    del Ph, Kh
    if args.serving_requests > 0:
        _progress("serving leg")
        res["serving"] = serving_bench(gk, I, args.serving_requests)
    g.release()
    del out, kout
    torch.cuda.empty_cache()
    legs = [x for x in args.legs.split(",") if x]
    if legs:
        res["configs"] = {}
        for name in legs:
            _progress(f"configuration leg {name}")
            variants = ("cbl", "gbl") if name.startswith("ba") else ("cbl",)
            res["configs"][name] = config_leg(torch, gk, I, name, variants)
    if not args.no_cpu:
        _progress("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(L, W, phi, m, args.cpu_sample)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
