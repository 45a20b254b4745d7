"""Serving loop: continuous admission by device-memory footprint and
iteration-level batching (classical block Lanczos requests advance one
Lanczos step per round together: one grouped SpMM per graph, one batched
launch of their CholQR factors per pass), other variants on a worker of
their own.  Each result is bitwise identical to the same request run alone
through kernel_machine_fit_predict, and matches the float64 oracle."""
import numpy as np
import pytest

from oracle import krylov
from paper_2301_06384_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
gk = pytest.importorskip("paper_2301_06384_amd.gk")


@pytest.fixture(scope="module")
def pool():
    Ls = [I.rgg_knn(n, 8, seed=200 + i) for i, n in enumerate([3000, 7000, 12000])]
    return Ls, [gk.Graph.from_laplacian(L, flags=gk.REORDER) for L in Ls]


def _mix(Ls, n_req, seed):
    reqs = I.serving_requests(n_req, [L.n for L in Ls], seed=seed, s_range=(4, 128), m=12)
    rng = np.random.default_rng(seed + 11)
    for r in reqs:   # mostly mixed cbl (batched), some float64 cbl, some gbl / sbl (whole)
        u = rng.random()
        r["variant"], r["precision"] = ("cbl", "mixed") if u < 0.6 else (("cbl", "fp64") if u < 0.8 else
                                                                          (("gbl", "mixed") if u < 0.9 else
                                                                           ("sbl", "fp64")))
    return reqs


def test_mix_equals_alone(pool):
    Ls, gs = pool
    reqs = _mix(Ls, 32, 5)
    assert max(len(r["samples"]) for r in reqs) > 64   # the wide (65..128) path is in the mix
    srv = gk.Server(max_active=8, hbm_budget=0, n_streams=3)
    try:
        tickets = [srv.submit(gs[r["graph"]], r["samples"], r["y"], r["phi"], r["m"], r["gamma"], r["variant"],
                              r["precision"]) for r in reqs]
        res = [srv.poll(t, -1) for t in tickets]
    finally:
        srv.stop()
    for r, out in zip(reqs, res):
        assert out["status"] == 0, (r["variant"], r["precision"], len(r["samples"]), out["status"])
        c, pred, _ = gk.kernel_machine_fit_predict(gs[r["graph"]], r["samples"], r["y"], r["phi"], r["m"],
                                                   r["gamma"], r["variant"], r["precision"])
        assert np.array_equal(out["coef"], c), (r["variant"], r["precision"], len(r["samples"]))
        assert np.array_equal(out["pred"], pred)
        assert out["t_complete_ms"] >= out["t_start_ms"] >= out["t_submit_ms"]


def test_served_results_match_oracle(pool):
    Ls, gs = pool
    L, g = Ls[0], gs[0]
    A = L.to_scipy()
    cases = [(100, dict(kind="diffusion", t=0.7), "cbl", "mixed"), (24, dict(kind="spline", eps=0.05, k=2.0), "cbl",
                                                                   "mixed"),
             (72, dict(kind="spline", eps=0.02, k=2.0), "cbl", "fp64"), (16, dict(kind="diffusion", t=1.5), "gbl",
                                                                        "mixed")]
    srv = gk.Server(max_active=4, hbm_budget=0, n_streams=3)
    try:
        subs = []
        for i, (s, phi, v, p) in enumerate(cases):
            W, y = I.samples(L.n, s, 50 + i), I.labels(s, 50 + i)
            subs.append((W, y, phi, v, p, srv.submit(g, W, y, phi, 12, 1e-3, v, p)))
        outs = [(W, y, phi, v, p, srv.poll(t, -1)) for W, y, phi, v, p, t in subs]
    finally:
        srv.stop()
    for W, y, phi, v, p, out in outs:
        assert out["status"] == 0
        c0, y0, K0 = krylov.fit_predict(A, W, y, phi, 12, 1e-3, v)
        kappa = np.linalg.cond(K0 + 1e-3 * np.eye(len(W)))
        tol = (1e-10 if p == "fp64" else 1e-5) * max(1.0, kappa)
        assert np.linalg.norm(out["coef"] - c0) / np.linalg.norm(c0) < tol, (v, p, len(W))
        assert np.linalg.norm(out["pred"] - y0) / np.linalg.norm(y0) < tol, (v, p, len(W))


def test_poll_eagain_and_shutdown(pool):
    Ls, gs = pool
    W, y = I.samples(Ls[2].n, 64, 9), I.labels(64, 9)
    srv = gk.Server(max_active=2, hbm_budget=0, n_streams=2)
    stopped = False
    try:
        t = srv.submit(gs[2], W, y, dict(kind="diffusion", t=1.0), 30, 1e-3, "cbl", "mixed")
        assert srv.poll(t, 0) is None            # GK_EAGAIN right after submission
        out = srv.poll(t, -1)
        assert out["status"] == 0
        with pytest.raises(gk.GKError) as ei:
            srv.poll(t, 0)                       # a consumed ticket is unknown
        assert ei.value.code == gk.EINVAL
        srv.stop()
        stopped = True
        with pytest.raises(gk.GKError) as ei:
            srv.submit(gs[2], W, y, dict(kind="diffusion", t=1.0), 30, 1e-3, "cbl", "mixed")
        assert ei.value.code == gk.ESHUTDOWN
    finally:
        if not stopped:
            srv.stop()


def test_admission_refuses_oversized(pool):
    Ls, gs = pool
    r = I.serving_requests(1, [Ls[2].n], seed=1, s_range=(32, 32), m=12)[0]
    foot = gk.request_footprint(Ls[2].n, 32, 12, "cbl", "mixed")
    srv = gk.Server(max_active=2, hbm_budget=foot // 2, n_streams=2)
    try:
        t = srv.submit(gs[2], r["samples"], r["y"], r["phi"], r["m"], r["gamma"], "cbl", "mixed")
        out = srv.poll(t, -1)
    finally:
        srv.stop()
    assert out["status"] == gk.ENOMEM


@pytest.mark.parametrize("variant,precision", [("cbl", "mixed"), ("cbl", "fp64"), ("gbl", "mixed"), ("gbl", "fp64"),
                                               ("sbl", "mixed"), ("sbl", "fp64")])
def test_footprint_bounds_actual_use(pool, variant, precision):
    # admission arithmetic must not under-estimate what a request holds
    Ls, gs = pool
    for s, phi in [(8, dict(kind="diffusion", t=1.0)), (40, dict(kind="spline", eps=0.01, k=2.0)),
                   (100, dict(kind="spline", eps=0.05, k=2.0))]:
        W = I.samples(Ls[1].n, s, 3)
        c, pred, st = gk.kernel_machine_fit_predict(gs[1], W, I.labels(s, 3), phi, 12, 1e-3, variant, precision)
        assert st.footprint_bytes <= gk.request_footprint(Ls[1].n, s, 12, variant, precision), (s, variant)


def test_hub_graph_served_equals_alone_and_oracle():
    # a heavy-tailed graph: rows above 256 entries are summed by workgroups of
    # their own (hub rows) in both the lone and the grouped product launches,
    # at whole-row widths and in 64-column strips (widths 128, 192)
    L = I.barabasi_albert(20000, 4, seed=7)
    assert int((np.diff(L.row_ptr) - 1 > 256).sum()) >= 4
    g = gk.Graph.from_laplacian(L, flags=gk.REORDER)
    A = L.to_scipy()
    phi = dict(kind="diffusion", t=0.6)
    cases = [(24, "cbl", "mixed"), (100, "cbl", "fp64"), (128, "cbl", "mixed"), (192, "cbl", "fp64"),
             (64, "cbl", "fp64"), (64, "cbl", "mixed"), (16, "gbl", "mixed")]
    srv = gk.Server(max_active=7, hbm_budget=0, n_streams=3)
    try:
        subs = []
        for i, (s, v, p) in enumerate(cases):
            W, y = I.samples(L.n, s, 70 + i), I.labels(s, 70 + i)
            subs.append((W, y, v, p, srv.submit(g, W, y, phi, 10, 1e-3, v, p)))
        outs = [(W, y, v, p, srv.poll(t, -1)) for W, y, v, p, t in subs]
    finally:
        srv.stop()
    for W, y, v, p, out in outs:
        assert out["status"] == 0, (v, p, len(W))
        c, pred, _ = gk.kernel_machine_fit_predict(g, W, y, phi, 10, 1e-3, v, p)
        assert np.array_equal(out["coef"], c) and np.array_equal(out["pred"], pred), (v, p, len(W))
        c0, y0, K0 = krylov.fit_predict(A, W, y, phi, 10, 1e-3, v)
        kappa = np.linalg.cond(K0 + 1e-3 * np.eye(len(W)))
        tol = (1e-10 if p == "fp64" else 1e-5) * max(1.0, kappa)
        assert np.linalg.norm(out["pred"] - y0) / np.linalg.norm(y0) < tol, (v, p, len(W))
    g.release()
