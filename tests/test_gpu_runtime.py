"""Runtime hooks of the C ABI: a caller-installed device allocator
(gk_set_allocator) and torch's caching allocator behind it
(gk.use_torch_allocator).  The library's own arithmetic does not depend on
where its memory comes from, so results are bitwise those of the default
allocator."""
import ctypes as C

import numpy as np
import pytest

from paper_2301_06384_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
gk = pytest.importorskip("paper_2301_06384_amd.gk")


@pytest.fixture(scope="module")
def case():
    L = I.rgg_knn(5000, 8, seed=31)
    g = gk.Graph.from_laplacian(L, flags=gk.REORDER)
    W = I.samples(L.n, 40, 3)
    yield L, g, W
    g.release()


def _reset():
    gk.reset_allocator()


def test_counting_allocator_bitwise_and_balanced(case):
    L, g, W = case
    phi = dict(kind="spline", eps=0.02, k=2.0)
    runs = {}
    for prec in ("fp64", "mixed"):
        runs[prec] = gk.krylov_kernel_columns(g, W, phi, 10, "cbl", prec)
    fa, ff, live, log, bad = _counting_hooks()
    assert gk._lib.gk_set_allocator(fa, ff, None) == gk.OK
    try:
        for prec in ("fp64", "mixed"):
            before = log["bytes"]
            P, K, st = gk.krylov_kernel_columns(g, W, phi, 10, "cbl", prec)
            P0, K0, _ = runs[prec]
            assert np.array_equal(P, P0) and np.array_equal(K, K0), prec
            # everything the call held came through the hook
            assert log["bytes"] - before >= st.footprint_bytes > 0, prec
    finally:
        _reset()
    assert not bad, bad
    assert log["alloc"] > 0 and log["alloc"] == log["free"] and not live


def test_hooks_changed_while_requests_run(case):
    # a request that started on the library's cache keeps returning its
    # blocks there after a hook is installed, and the hook only ever sees
    # its own blocks
    L, g, W = case
    phi = dict(kind="spline", eps=0.02, k=2.0)
    y = I.labels(len(W), 4)
    c0, p0, _ = gk.kernel_machine_fit_predict(g, W, y, phi, 30, 1e-3, "cbl", "mixed")
    fa, ff, live, log, bad = _counting_hooks()
    srv = gk.Server(max_active=4, hbm_budget=0, n_streams=2)
    try:
        t1 = srv.submit(g, W, y, phi, 30, 1e-3, "cbl", "mixed")
        assert gk._lib.gk_set_allocator(fa, ff, None) == gk.OK
        t2 = srv.submit(g, W, y, phi, 30, 1e-3, "cbl", "mixed")
        r1, r2 = srv.poll(t1, -1), srv.poll(t2, -1)
        gk.reset_allocator()
        t3 = srv.submit(g, W, y, phi, 30, 1e-3, "cbl", "mixed")
        r3 = srv.poll(t3, -1)
    finally:
        srv.stop()
        _reset()
    assert not bad, bad
    assert log["alloc"] == log["free"] and not live
    for r in (r1, r2, r3):
        assert r["status"] == 0
        assert np.array_equal(r["coef"], c0) and np.array_equal(r["pred"], p0)


def _counting_hooks():
    # device allocations through torch's caching allocator, counted; a free
    # of a block the hook did not make is recorded (exceptions raised inside
    # a ctypes callback would not reach the test)
    dev = torch.cuda.current_device()
    live, log, bad = {}, {"alloc": 0, "free": 0, "bytes": 0}, []

    def _alloc(nbytes, ctx):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), dev, torch.cuda.current_stream(dev))
        live[p] = int(nbytes)
        log["alloc"] += 1
        log["bytes"] += int(nbytes)
        if p % 256:
            bad.append(("misaligned", p))
        return p

    def _free(ptr, ctx):
        if ptr not in live:
            bad.append(("foreign free", ptr))
            return
        del live[ptr]
        log["free"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    fa, ff = gk._ALLOC_T(_alloc), gk._FREE_T(_free)
    gk._alloc_keep[:] = [fa, ff]
    return fa, ff, live, log, bad


def test_torch_allocator_hook(case):
    L, g, W = case
    phi = dict(kind="diffusion", t=0.8)
    P0, K0, _ = gk.krylov_kernel_columns(g, W, phi, 12, "cbl", "mixed")
    gk.use_torch_allocator()
    try:
        P1, K1, _ = gk.krylov_kernel_columns(g, W, phi, 12, "cbl", "mixed")
    finally:
        _reset()
    assert np.array_equal(P1, P0) and np.array_equal(K1, K0)
    P2, _, _ = gk.krylov_kernel_columns(g, W, phi, 12, "cbl", "mixed")   # default allocator again
    assert np.array_equal(P2, P0)


def test_allocator_hooks_come_in_pairs():
    fa = gk._ALLOC_T(lambda nbytes, ctx: 0)
    assert gk._lib.gk_set_allocator(fa, gk._FREE_T(), None) == gk.EINVAL
    assert gk._lib.gk_set_allocator(gk._ALLOC_T(), gk._FREE_T(), None) == gk.OK
