"""The paper's experiments (Sec. 8) as GPU regression workloads, through the
C ABI against the float64 oracle.

* Sec. 8.1: path graph, 201 nodes, normalised Laplacian (GK_ASSUME_PSD: its
  rows do not sum to zero), central sample v_101, exp(-200 L) and
  (L + 0.001 I)^(-2): GPU Lanczos and Chebyshev columns match the oracle for
  each m, and the Lanczos uniform error stays below the Chebyshev one.
* Sec. 8.2: synthetic stand-in of the 900-point planar graph (7325 closest
  pairs of 900 uniform points; the paper's point set is not available),
  normalised Laplacian, N = 20, binary labels, gamma = 0: the five GPU
  interpolants match the oracle's, and their uniform errors against the
  exact interpolant rank cbl < gbl, sbl < cheb, cheb2.
* Sec. 8.3: N = 40, exp(-20 L), m = 6: the GPU collocation matrices match the
  oracle's, with positive eigenvalues for cbl and cheb2, negative ones for
  gbl and cheb and complex ones for sbl.
"""
import numpy as np
import pytest

from oracle import cheb as ocheb
from oracle import dense, krylov
from paper_2301_06384_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
gk = pytest.importorskip("paper_2301_06384_amd.gk")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _oracle(variant, A, W, phi, m):
    if variant == "cheb":
        return ocheb.cheb(A, W, phi, m)
    if variant == "cheb2":
        return ocheb.cheb2(A, W, phi, m)
    return getattr(krylov, variant)(A, W, phi, m)


@pytest.fixture(scope="module")
def path201():
    L = I.normalized_laplacian(I.path(201))
    return L, gk.Graph.from_laplacian(L, flags=gk.ASSUME_PSD)


@pytest.mark.parametrize("phi", [dict(kind="diffusion", t=200.0), dict(kind="spline", eps=0.001, k=2.0)])
def test_sec81_path_lanczos_vs_chebyshev(path201, phi):
    L, g = path201
    A = L.to_scipy()
    W = [100]
    ref = dense.phi_columns(A, W, phi)
    for m in (5, 10, 20, 40, 60):
        Pl, _, _ = gk.krylov_kernel_columns(g, W, phi, m, "cbl", "fp64")
        Pc, _, _ = gk.krylov_kernel_columns(g, W, phi, m, "cheb", "fp64")
        assert rel(Pl, krylov.cbl(A, W, phi, m)["P"]) < 1e-10, m
        assert rel(Pc, ocheb.cheb(A, W, phi, m)["P"]) < 1e-10, m
        e_l, e_c = np.max(np.abs(Pl - ref)), np.max(np.abs(Pc - ref))
        print(f"{phi['kind']} m={m}: uniform error Lanczos {e_l:.2e}, Chebyshev {e_c:.2e}")
        assert e_l < e_c, (m, e_l, e_c)


@pytest.fixture(scope="module")
def planar():
    L = I.normalized_laplacian(I.planar_radius_standin())
    return L, gk.Graph.from_laplacian(L, flags=gk.ASSUME_PSD)


@pytest.mark.parametrize("phi", [dict(kind="diffusion", t=20.0), dict(kind="spline", eps=0.05, k=2.0)])
def test_sec82_interpolants_and_ranking(planar, phi):
    L, g = planar
    A = L.to_scipy()
    W = I.samples(900, 20, 1)
    y = (np.random.default_rng(3).random(20) < 0.5).astype(float)
    _, y0, _, _ = dense.fit_predict(A, W, y, phi, 0.0)
    for m in (12, 16, 24):
        err = {}
        for v in ("cbl", "gbl", "sbl", "cheb", "cheb2"):
            c, pred, _ = gk.kernel_machine_fit_predict(g, W, y, phi, m, 0.0, v, "fp64")
            r = _oracle(v, A, W, phi, m)
            K = r["Kww"] if v == "cbl" else r["Kww_gathered"]
            c_ref = np.linalg.solve(K, y)
            pred_ref = (r["P"] @ c_ref)
            kappa = np.linalg.cond(K)
            assert rel(c, c_ref) < 1e-10 * kappa and rel(pred, pred_ref) < 1e-10 * kappa, (v, m)
            err[v] = np.max(np.abs(pred - y0))
        print(f"{phi['kind']} m={m}: " + ", ".join(f"{k} {e:.2e}" for k, e in err.items()))
        assert err["cbl"] < min(err["gbl"], err["sbl"]), (m, err)
        assert max(err["gbl"], err["sbl"]) < min(err["cheb"], err["cheb2"]), (m, err)


def test_sec83_collocation_eigenvalue_signs(planar):
    L, g = planar
    A = L.to_scipy()
    W = I.samples(900, 40, 1)
    phi = dict(kind="diffusion", t=20.0)
    ev = {}
    for v in ("cbl", "gbl", "sbl", "cheb", "cheb2"):
        _, K, _ = gk.krylov_kernel_columns(g, W, phi, 6, v, "fp64", want_cols=False)
        r = _oracle(v, A, W, phi, 6)
        assert rel(K, r["Kww"] if v == "cbl" else r["Kww_gathered"]) < 1e-10, v
        ev[v] = np.linalg.eigvals(K)
    assert ev["cbl"].real.min() > 0 and ev["cheb2"].real.min() > 0
    assert ev["gbl"].real.min() < 0 and ev["cheb"].real.min() < 0
    assert np.abs(ev["sbl"].imag).max() > 0
