"""Writes rgg100k_spline_oracle.txt: float64 oracle (classical block Lanczos,
Alg. 1, full two-pass reorthogonalisation) on the benchmark workload -- the
100,000-point 8-NN random geometric graph (seed 1), spline kernel
(0.01 I + L)^(-2), s = 64 samples (seed 0), m = 40 -- reduced to what a test
can compare against: the sampled block K_WW and the kernel columns at 96
seeded rows.  Calls only the oracle and the input generators.

    python tests/golden/make_rgg100k_fixture.py   (about two minutes)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import krylov  # noqa: E402
from paper_2301_06384_amd import inputs as I  # noqa: E402

ROW_SEED = 12345
N_ROWS = 96


def main():
    L, W, phi, m = I.workload("rgg100k_spline")
    r = krylov.cbl(L.to_scipy(), W, phi, m)
    rows = np.sort(np.random.default_rng(ROW_SEED).choice(L.n, N_ROWS, replace=False))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rgg100k_spline_oracle.txt")
    with open(out, "w") as fh:
        fh.write("# float64 oracle cbl, rgg100k_spline workload (n=100000, s=64, m=40, eps=0.01, k=2)\n")
        fh.write(f"# written by tests/golden/make_rgg100k_fixture.py; rows seed {ROW_SEED}\n")
        fh.write("rows " + " ".join(str(int(x)) for x in rows) + "\n")
        for i, row in enumerate(r["Kww"]):
            fh.write(f"K {i} " + " ".join(repr(float(v)) for v in row) + "\n")
        for ri in rows:
            fh.write(f"P {int(ri)} " + " ".join(repr(float(v)) for v in r["P"][ri]) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
