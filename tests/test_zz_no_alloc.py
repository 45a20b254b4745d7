"""The allocation-free entry point krylov_kernel_columns_noalloc against
krylov_kernel_columns, through the C ABI: same inputs, two calls in a row
(the second smaller, on the scratch the first left behind), results equal to
the allocating entry point's (the same kernels in the same order, so
bitwise), and a request beyond the static scratch refused."""
import ctypes as C

import numpy as np
import pytest

from paper_2301_06384_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
gk = pytest.importorskip("paper_2301_06384_amd.gk")

DEV = torch.device("cuda:0")
TOL = {"fp64": 1e-10, "mixed": 1e-5}


def _both(g, n, W, phi, m, variant, prec):
    Wd = torch.as_tensor(np.asarray(W, dtype=np.int64), device=DEV)
    s = len(W)
    out = []
    for fn in (gk.krylov_kernel_columns, gk.krylov_kernel_columns_noalloc):
        P = torch.full((s, n), float("nan"), dtype=torch.float64, device=DEV)
        K = torch.full((s, s), float("nan"), dtype=torch.float64, device=DEV)
        if fn is gk.krylov_kernel_columns:
            fn(g, Wd, phi, m, variant, prec, flags=gk.IO_DEVICE, out_cols=P, out_kww=K)
        else:
            fn(g, Wd, phi, m, variant, prec, P, K)
        torch.cuda.synchronize()
        out.append((P.cpu().numpy(), K.cpu().numpy()))
    return out


@pytest.mark.parametrize("variant,prec", [("cbl", "mixed"), ("cbl", "fp64"), ("gbl", "mixed"), ("cheb", "fp64")])
def test_noalloc_matches_allocating_entry_point(variant, prec):
    big = I.grid((32, 32))
    small = I.grid((16, 16))
    gb, gs = gk.Graph.from_laplacian(big), gk.Graph.from_laplacian(small)
    phi = dict(kind="diffusion", t=1.0)
    cases = [(gb, big.n, I.samples(big.n, 8, 0), 20), (gs, small.n, I.samples(small.n, 5, 1), 10)]
    for g, n, W, m in cases:   # second call smaller than the first
        (P0, K0), (P1, K1) = _both(g, n, W, phi, m, variant, prec)
        assert np.all(np.isfinite(P1)) and np.all(np.isfinite(K1))
        assert np.linalg.norm(P1 - P0) / np.linalg.norm(P0) < TOL[prec]
        assert np.array_equal(P1, P0) and np.array_equal(K1, K0), (variant, prec, n)
    gb.release()
    gs.release()


def test_noalloc_rejects_oversized_and_host_io():
    L = I.grid((200, 200))
    g = gk.Graph.from_laplacian(L)
    W = I.samples(L.n, 64, 0)
    Wd = torch.as_tensor(W, device=DEV)
    P = torch.empty((64, L.n), dtype=torch.float64, device=DEV)
    K = torch.empty((64, 64), dtype=torch.float64, device=DEV)
    with pytest.raises(gk.GKError) as ei:
        gk.krylov_kernel_columns_noalloc(g, Wd, dict(kind="diffusion", t=1.0), 40, "cbl", "fp64", P, K)
    assert ei.value.code == gk.ENOMEM
    # without GK_IO_DEVICE the call is refused before any pointer is touched
    phi, keep = gk.make_phi(dict(kind="diffusion", t=1.0))
    Wh = np.ascontiguousarray(W[:4])
    rc = gk._lib.krylov_kernel_columns_noalloc(g.handle, Wh.ctypes.data, 4, C.byref(phi), 5, 0, 0, 0, None, None,
                                               None)
    assert rc == gk.EINVAL
    g.release()
