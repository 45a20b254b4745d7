"""Writes the float64 oracle fixtures of the wide-block configurations at
reduced graph size (the oracle must hold the whole float64 basis on the host):

  ba200k_diffusion_oracle.txt -- Barabasi-Albert graph, 200,000 nodes, 4 edges
      per new node (seed 0), unit weights; exp(-0.5 L); s = 256 samples
      (seed 0); m = 30; classical block Lanczos (Alg. 1) and global block
      Lanczos (Alg. 2), both with full two-pass reorthogonalisation.
  ba200k_gbl_m20_oracle.txt -- the same graph and samples, Alg. 2 at m = 20.
  grid48_spline_oracle.txt -- 3-D grid 48^3 with edge weights U[0.5, 1.5]
      (seed 0); (0.05 I + L)^(-1); s = 512 samples (seed 0); m = 30; Alg. 1.

Each file holds, per method, seeded rows of the sampled block K_WW and of the
kernel columns P, and the Frobenius norms of the whole K_WW and P.  Calls only
the oracle and the input generators.

    python tests/golden/make_wide_fixtures.py [ba|ba_gbl20|grid]   (tens of minutes, ~30 GB)
"""
import gc
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import krylov  # noqa: E402
from paper_2301_06384_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROW_SEED = 2024


def _rows(n, count, salt):
    return np.sort(np.random.default_rng(ROW_SEED + salt).choice(n, count, replace=False))


def _write_method(fh, tag, P, K, krows, prows):
    fh.write(f"{tag}_normK {float(np.linalg.norm(K))!r}\n")
    fh.write(f"{tag}_normP {float(np.linalg.norm(P))!r}\n")
    fh.write(f"{tag}_krows " + " ".join(str(int(x)) for x in krows) + "\n")
    fh.write(f"{tag}_prows " + " ".join(str(int(x)) for x in prows) + "\n")
    for r in krows:
        fh.write(f"{tag}_K {int(r)} " + " ".join(repr(float(v)) for v in K[r]) + "\n")
    for r in prows:
        fh.write(f"{tag}_P {int(r)} " + " ".join(repr(float(v)) for v in P[r]) + "\n")


def make_ba():
    L = I.barabasi_albert(200_000, 4, seed=0)
    W = I.samples(L.n, 256, 0)
    phi = dict(kind="diffusion", t=0.5)
    A = L.to_scipy()
    out = os.path.join(HERE, "ba200k_diffusion_oracle.txt")
    with open(out, "w") as fh:
        fh.write("# float64 oracle, Barabasi-Albert n=200000 (4 edges/node, seed 0), exp(-0.5 L), "
                 "s=256 (seed 0), m=30\n")
        fh.write(f"# written by tests/golden/make_wide_fixtures.py; row seed {ROW_SEED}\n")
        r = krylov.cbl(A, W, phi, 30)
        P, K = r["P"], r["Kww"]
        del r
        gc.collect()
        _write_method(fh, "cbl", P, K, _rows(256, 16, 1), _rows(L.n, 48, 2))
        del P, K
        gc.collect()
        r = krylov.gbl(A, W, phi, 30)
        P, K = r["P"], r["Kww_gathered"]
        del r
        gc.collect()
        _write_method(fh, "gbl", P, K, _rows(256, 16, 1), _rows(L.n, 48, 2))
    print("wrote", out)


def make_ba_gbl20():
    # global block Lanczos at depth 20: at m = 30 its coefficients are
    # forward-unstable on this hub graph (float64 runs that differ only in
    # summation order disagree by ~1e-5), at m = 20 they agree to ~1e-11
    L = I.barabasi_albert(200_000, 4, seed=0)
    W = I.samples(L.n, 256, 0)
    phi = dict(kind="diffusion", t=0.5)
    r = krylov.gbl(L.to_scipy(), W, phi, 20)
    P, K = r["P"], r["Kww_gathered"]
    del r
    gc.collect()
    out = os.path.join(HERE, "ba200k_gbl_m20_oracle.txt")
    with open(out, "w") as fh:
        fh.write("# float64 oracle gbl, Barabasi-Albert n=200000 (4 edges/node, seed 0), exp(-0.5 L), "
                 "s=256 (seed 0), m=20\n")
        fh.write(f"# written by tests/golden/make_wide_fixtures.py; row seed {ROW_SEED}\n")
        _write_method(fh, "gbl", P, K, _rows(256, 16, 1), _rows(L.n, 48, 2))
    print("wrote", out)


def make_grid():
    L = I.grid((48, 48, 48), weights="uniform", seed=0)
    W = I.samples(L.n, 512, 0)
    phi = dict(kind="spline", eps=0.05, k=1.0)
    r = krylov.cbl(L.to_scipy(), W, phi, 30)
    P, K = r["P"], r["Kww"]
    del r
    gc.collect()
    out = os.path.join(HERE, "grid48_spline_oracle.txt")
    with open(out, "w") as fh:
        fh.write("# float64 oracle, 3-D grid 48^3 weights U[0.5,1.5] (seed 0), (0.05 I + L)^(-1), "
                 "s=512 (seed 0), m=30\n")
        fh.write(f"# written by tests/golden/make_wide_fixtures.py; row seed {ROW_SEED}\n")
        _write_method(fh, "cbl", P, K, _rows(512, 12, 3), _rows(L.n, 24, 4))
    print("wrote", out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["ba", "ba_gbl20", "grid"]
    if "ba" in which:
        make_ba()
    if "ba_gbl20" in which:
        make_ba_gbl20()
    if "grid" in which:
        make_grid()
