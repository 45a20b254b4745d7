"""Kernel functions phi (Sec. 2.4): the kernel matrix is phi(L).

Test infrastructure only (see the oracle package docstring).

  diffusion   phi(lam) = exp(-t lam),       t >= 0
  spline      phi(lam) = (eps + lam)^(-k),  eps > 0, k > 0
              (the paper calls the exponent s; k avoids the clash with the
              block width)
  polynomial  phi(lam) = sum_j c_j lam^j    (not a kernel of the paper; used
              to check polynomial exactness of the Krylov approximants,
              Lemma 4.1)
"""
from __future__ import annotations

import numpy as np


def make(spec: dict):
    """Return a vectorised float64 function lam -> phi(lam) for a phi spec."""
    kind = spec["kind"]
    if kind == "diffusion":
        t = float(spec["t"])
        if not (t >= 0 and np.isfinite(t)):
            raise ValueError("diffusion needs finite t >= 0")
        return lambda lam: np.exp(-t * np.asarray(lam, dtype=np.float64))
    if kind == "spline":
        eps, k = float(spec["eps"]), float(spec["k"])
        if not (eps > 0 and k > 0):
            raise ValueError("spline needs eps > 0 and k > 0")

        def f(lam):
            z = eps + np.asarray(lam, dtype=np.float64)
            if np.any(z <= 0):
                raise ValueError("eps + lambda must stay positive")
            return z ** (-k)
        return f
    if kind == "polynomial":
        c = np.asarray(spec["coef"], dtype=np.float64)

        def p(lam):
            lam = np.asarray(lam, dtype=np.float64)
            acc = np.zeros_like(lam)
            for cj in c[::-1]:          # Horner
                acc = acc * lam + cj
            return acc
        return p
    raise ValueError(f"unknown phi kind {kind!r}")


def apply_polynomial_sparse(L, coef, B):
    """p(L) B by Horner's rule with sparse products (no eigendecomposition)."""
    acc = np.zeros_like(B, dtype=np.float64)
    for cj in np.asarray(coef, dtype=np.float64)[::-1]:
        acc = L @ acc + cj * B
    return acc
