"""The wide-block configurations against the float64 oracle, through the C
ABI, at graph sizes the oracle can hold: fixtures written by
tests/golden/make_wide_fixtures.py (oracle and input generators only) hold
seeded rows of K_WW and of the kernel columns P, and the Frobenius norms of
the whole K_WW and P.

* Barabasi-Albert, 200,000 nodes (hub degrees in the thousands), exp(-0.5 L),
  s = 256, m = 30: cbl (float64 1e-10, mixed 1e-5).  gbl at m = 30, where
  float64 runs that differ only in summation order already disagree by
  ~6e-5 (the Alg. 2 coefficients are forward-unstable at this depth): the
  mixed path must be as close to the oracle as the float64 path is; gbl at
  m = 20 to 1e-10 / 1e-5.
* 3-D grid 48^3 with weights U[0.5, 1.5], (0.05 I + L)^(-1), s = 512, m = 30
  (the widest block, on the tiled 65..512 kernels): 1e-10 / 1e-5.
"""
import os

import numpy as np
import pytest

from paper_2301_06384_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
gk = pytest.importorskip("paper_2301_06384_amd.gk")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = {"fp64": 1e-10, "mixed": 1e-5}


def load(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            tag, rest = line.split(" ", 1)
            meth, kind = tag.split("_", 1)
            d = out.setdefault(meth, {"K": {}, "P": {}})
            if kind in ("normK", "normP"):
                d[kind] = float(rest)
            elif kind in ("krows", "prows"):
                d[kind] = [int(x) for x in rest.split()]
            else:
                r, vals = rest.split(" ", 1)
                d[kind][int(r)] = np.array([float(v) for v in vals.split()])
    for d in out.values():
        d["Kmat"] = np.stack([d["K"][r] for r in d["krows"]])
        d["Pmat"] = np.stack([d["P"][r] for r in d["prows"]])
    return out


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def compare(ref, P, K):
    """Largest relative error over the sampled rows of P and K_WW and the
    norms of the whole P and K_WW."""
    errs = [rel(P[ref["prows"]], ref["Pmat"]), rel(K[ref["krows"]], ref["Kmat"]),
            abs(np.linalg.norm(P) - ref["normP"]) / ref["normP"], abs(np.linalg.norm(K) - ref["normK"]) / ref["normK"]]
    return max(errs)


@pytest.fixture(scope="module")
def ba200k():
    L = I.barabasi_albert(200_000, 4, seed=0)
    g = gk.Graph.from_laplacian(L, flags=gk.REORDER)
    yield L, g
    g.release()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ba200k_cbl_against_oracle(ba200k, prec):
    L, g = ba200k
    ref = load("ba200k_diffusion_oracle.txt")["cbl"]
    W = I.samples(L.n, 256, 0)
    P, K, st = gk.krylov_kernel_columns(g, W, dict(kind="diffusion", t=0.5), 30, "cbl", prec)
    err = compare(ref, P, K)
    print(f"BA200k cbl {prec}: {err:.3e} (archive projections {st.n_reorth})")
    assert err < TOL[prec]


def test_ba200k_gbl_m30_against_oracle(ba200k):
    # At m = 30 the Alg. 2 coefficients on this graph amplify any rounding
    # difference by about 6x per step: the float64 GPU path and the float64
    # oracle (another Gram-Schmidt order) end 1.7e-2 apart, and the path's own
    # node-order noise is 6e-5, while Theorem 4.2 bounds the approximation
    # error only by ~2e3 here (t Lambda = 1526, far from converged).  Checked:
    # the mixed path is as close to the oracle as the float64 path is.
    L, g = ba200k
    ref = load("ba200k_diffusion_oracle.txt")["gbl"]
    W = I.samples(L.n, 256, 0)
    phi = dict(kind="diffusion", t=0.5)
    P64, K64, _ = gk.krylov_kernel_columns(g, W, phi, 30, "gbl", "fp64")
    Pm, Km, _ = gk.krylov_kernel_columns(g, W, phi, 30, "gbl", "mixed")
    e64, em = compare(ref, P64, K64), compare(ref, Pm, Km)
    print(f"BA200k gbl m=30: fp64 {e64:.3e}, mixed {em:.3e} against the oracle")
    assert em < 1.5 * e64 + 1e-5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ba200k_gbl_m20_against_oracle(ba200k, prec):
    L, g = ba200k
    ref = load("ba200k_gbl_m20_oracle.txt")["gbl"]
    W = I.samples(L.n, 256, 0)
    P, K, st = gk.krylov_kernel_columns(g, W, dict(kind="diffusion", t=0.5), 20, "gbl", prec)
    err = compare(ref, P, K)
    print(f"BA200k gbl m=20 {prec}: {err:.3e} (archive projections {st.n_reorth})")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_grid48_s512_against_oracle(prec):
    # the widest block (s = 512, tiled 65..512 kernels) on a 3-D grid
    L = I.grid((48, 48, 48), weights="uniform", seed=0)
    g = gk.Graph.from_laplacian(L, flags=gk.REORDER)
    try:
        ref = load("grid48_spline_oracle.txt")["cbl"]
        W = I.samples(L.n, 512, 0)
        P, K, st = gk.krylov_kernel_columns(g, W, dict(kind="spline", eps=0.05, k=1.0), 30, "cbl", prec)
    finally:
        g.release()
    err = compare(ref, P, K)
    print(f"grid48 s=512 cbl {prec}: {err:.3e} (archive projections {st.n_reorth})")
    assert err < TOL[prec]
