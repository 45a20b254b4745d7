"""Chebyshev interpolation methods of Sec. 3.4.

Test infrastructure only (see the oracle package docstring).

p_{phi,m}(lam) interpolates phi on the shifted Chebyshev-Lobatto grid
lam_j = (Lambda/2)(1 - cos(pi j/m)), j = 0..m, written as a Chebyshev series
in x = 1 - 2 lam / Lambda.  The block p(L) E_W follows from the three-term
recurrence of the T_k applied to E_W.

Readings (the printed formulas are garbled): the interpolant is the standard
Lobatto one, i.e. c_k = (2/m) sum_j'' phi(lam_j) cos(pi j k / m) where the
double prime halves the j = 0 and j = m terms (the printed correction term
carries the wrong sign), the series halves c_0 and c_m, and T_1(x) = x.
cheb2 approximates sqrt(phi) with degree floor(m/2) and squares it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import phi as _phi
from .dense import unit_block
from .krylov import gershgorin_bound


def lobatto_nodes(m: int, Lam: float) -> np.ndarray:
    j = np.arange(m + 1)
    return 0.5 * Lam * (1.0 - np.cos(np.pi * j / m))


def coefficients(f, m: int, Lam: float) -> np.ndarray:
    """Series coefficients a_k with p(lam) = sum_k a_k T_k(1 - 2 lam/Lam);
    the endpoint halvings are folded into a_0 and a_m."""
    fj = f(lobatto_nodes(m, Lam))
    j = np.arange(m + 1)
    w = np.ones(m + 1)
    w[0] = w[-1] = 0.5
    c = (2.0 / m) * np.array([np.sum(w * fj * np.cos(np.pi * j * k / m)) for k in range(m + 1)])
    c[0] *= 0.5
    c[-1] *= 0.5
    return c


def eval_scalar(a: np.ndarray, lam, Lam: float) -> np.ndarray:
    """Evaluate sum_k a_k T_k(x), x = 1 - 2 lam / Lam, by the recurrence."""
    x = 1.0 - 2.0 * np.asarray(lam, dtype=np.float64) / Lam
    t0, t1 = np.ones_like(x), x
    acc = a[0] * t0
    if a.size > 1:
        acc = acc + a[1] * t1
    for k in range(2, a.size):
        t0, t1 = t1, 2.0 * x * t1 - t0
        acc = acc + a[k] * t1
    return acc


def apply_series(L, a: np.ndarray, B: np.ndarray, Lam: float) -> np.ndarray:
    """sum_k a_k T_k(I - 2L/Lam) B by the three-term recurrence."""
    def A(Y):
        return Y - (2.0 / Lam) * (L @ Y)
    Y0 = B.copy()
    acc = a[0] * Y0
    if a.size == 1:
        return acc
    Y1 = A(B)
    acc = acc + a[1] * Y1
    for k in range(2, a.size):
        Y0, Y1 = Y1, 2.0 * A(Y1) - Y0
        acc = acc + a[k] * Y1
    return acc


def cheb(L, samples, phi_spec, m: int, Lam: float | None = None):
    """Chebyshev interpolation method: p_{phi,m}(L) E_W (m block products)."""
    L = sp.csr_matrix(L)
    Lam = gershgorin_bound(L) if Lam is None else Lam
    a = coefficients(_phi.make(phi_spec), m, Lam)
    W = np.asarray(samples, dtype=np.int64)
    P = apply_series(L, a, unit_block(L.shape[0], W), Lam)
    return dict(P=P, coef=a, Lam=Lam, Kww_gathered=P[W, :])


def cheb2(L, samples, phi_spec, m: int, Lam: float | None = None):
    """Squared Chebyshev method: (p_{sqrt(phi), floor(m/2)}(L))^2 E_W."""
    L = sp.csr_matrix(L)
    Lam = gershgorin_bound(L) if Lam is None else Lam
    f = _phi.make(phi_spec)
    half = max(m // 2, 1)
    a = coefficients(lambda lam: np.sqrt(f(lam)), half, Lam)
    W = np.asarray(samples, dtype=np.int64)
    E = unit_block(L.shape[0], W)
    P = apply_series(L, a, apply_series(L, a, E, Lam), Lam)
    return dict(P=P, coef=a, Lam=Lam, Kww_gathered=P[W, :])
