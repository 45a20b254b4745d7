"""Exact kernel columns and kernel machine by full spectral decomposition.

Test infrastructure only (see the oracle package docstring).

Follows Sec. 2.4 (kernel columns K(., w_i) = phi(L) e_{w_i}, eq. of the
kernel matrix function), the naive approach at the start of Sec. 3
(spectral decomposition of L, then phi on the spectrum, then the product with
E_W), and Sec. 2.3 (representer form and the RLS coefficient system).
Feasible only for small graphs (dense n x n eigendecomposition).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import phi as _phi


def _dense(L):
    if sp.issparse(L):
        return L.toarray()
    return np.asarray(L, dtype=np.float64)


def unit_block(n: int, samples) -> np.ndarray:
    """E_W = [e_{w_1}, ..., e_{w_N}] (Sec. 3)."""
    E = np.zeros((n, len(samples)))
    E[np.asarray(samples), np.arange(len(samples))] = 1.0
    return E


def phi_of_L(L, phi_spec) -> np.ndarray:
    """phi(L) = U phi(Lambda) U^T from L = U Lambda U^T (LAPACK eigh)."""
    A = _dense(L)
    lam, U = np.linalg.eigh(A)
    return (U * _phi.make(phi_spec)(lam)) @ U.T


def phi_columns(L, samples, phi_spec) -> np.ndarray:
    """phi(L) E_W, computed as U phi(Lambda) U[W,:]^T (n x N)."""
    A = _dense(L)
    lam, U = np.linalg.eigh(A)
    f = _phi.make(phi_spec)(lam)
    return U @ (f[:, None] * U[np.asarray(samples), :].T)


def fit_predict(L, samples, y, phi_spec, gamma: float):
    """Exact RLS kernel machine (Sec. 2.3).

    K_W = E_W^T phi(L) E_W; solve (K_W + gamma I) c = y; y(v) = sum_i c_i
    K(v, w_i).  `gamma` is the full diagonal shift (the paper writes it as
    gamma_paper * N with N samples).
    Returns (c, yhat, P, K_W).
    """
    P = phi_columns(L, samples, phi_spec)
    K = P[np.asarray(samples), :]
    s = K.shape[0]
    c = np.linalg.solve(K + gamma * np.eye(s), np.asarray(y, dtype=np.float64))
    return c, P @ c, P, K
