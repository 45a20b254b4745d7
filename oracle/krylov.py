"""Block Krylov approximations of phi(L) E_W and the Krylov RLS predictor.

Test infrastructure only (see the oracle package docstring).

Implements, in float64 with numpy/scipy:
  cbl  -- classical block Lanczos, Alg. 1 (Sec. 3.1)
  gbl  -- global block Lanczos, Alg. 2 (Sec. 3.2)
  sbl  -- sequential Lanczos (Sec. 3.3): Alg. 1 with block width 1 per column
  fit_predict -- kernel RLS predictor, Alg. 3 (Sec. 6) for cbl, and the
          collocation system of Sec. 5 for gbl / sbl.

Readings of the paper taken here (each also listed in the design notes):
  * Alg. 1 sets H_{k,k+1} from H_{k+1,k}; the text of Sec. 3.1 states
    H_{k+1,k} = H_{k,k+1}^*, so the transpose is used.
  * The basis is stated to be orthonormal (Sec. 3.1, Sec. 6); in floating
    point this is realised by reorthogonalising each new block twice against
    all stored blocks (classical block Gram-Schmidt, two passes).  The
    projection coefficients of these passes are discarded: they vanish in
    exact arithmetic.
  * H_{k+1,k} is assumed invertible.  When the QR factor of X is numerically
    rank deficient (min |R_ii| < tau * ||L||_1) the block is factorised by an
    SVD instead and the deflated directions become zero columns of Q_{k+1}
    and zero rows of H_{k+1,k}; the block width stays fixed.
  * The QR factor of the last iteration (k = m) is never used; the residual
    norm ||X||_F of that iteration is returned as a diagnostic.
  * H_kk is symmetrised before it enters H_m.
  * The sequential formulas omit phi; p(L) e_w = [q_1..q_m] phi(H_m^(w)) f_1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import phi as _phi
from .dense import unit_block

DEFAULT_TAU = 1e-12


def gershgorin_bound(L) -> float:
    """Upper bound Lambda of spec(L): max_i sum_j |L_ij| (the paper leaves
    Lambda unspecified; any bound with spec(L) in [0, Lambda] works)."""
    A = L if sp.issparse(L) else sp.csr_matrix(L)
    return float(np.max(np.asarray(abs(A).sum(axis=1)).ravel()))


def _qr_deflating(X, thresh, flip_signs=False):
    """Reduced QR X = Q R with diag(R) >= 0; rank-revealing fallback.

    Returns (Q, R, n_deflated).  `flip_signs` selects the opposite sign
    convention (diag(R) <= 0); outputs of the method must not depend on it.
    """
    n, s = X.shape
    Q, R = np.linalg.qr(X, mode="reduced")          # Householder (LAPACK geqrf)
    sg = np.sign(np.diag(R))
    sg[sg == 0] = 1.0
    if flip_signs:
        sg = -sg
    Q, R = Q * sg, sg[:, None] * R
    if np.min(np.abs(np.diag(R))) >= thresh:
        return Q, R, 0
    Us, sig, Wt = np.linalg.svd(X, full_matrices=False)
    keep = sig > thresh
    r = int(np.count_nonzero(keep))
    Q = np.zeros((n, s))
    R = np.zeros((s, s))
    Q[:, :r] = Us[:, keep]
    R[:r, :] = sig[keep, None] * Wt[keep, :]
    return Q, R, s - r


def _phi_projected(T, f, s):
    """Spectral decomposition T = S Theta S^T; returns (U, S, theta, ftheta)
    with U = phi(T) F_1 = S phi(Theta) S[:s,:]^T."""
    theta, S = np.linalg.eigh(T)
    ft = f(theta)
    U = S @ (ft[:, None] * S[:s, :].T)
    return U, S, theta, ft


def cbl(L, samples, phi_spec, m: int, tau: float = DEFAULT_TAU, flip_signs=False):
    """Classical block Lanczos, Alg. 1.

    Q_1 = E_W; for k = 1..m: X = L Q_k - Q_{k-1} H_{k-1,k}; H_kk = Q_k^T X;
    X -= Q_k H_kk; QR X = Q_{k+1} H_{k+1,k}.  Then U = phi(H_m) F_1 and the
    approximation is [Q_1..Q_m] U.

    Returns a dict with P (n x s), U (ms x s), T (= H_m), Q (n x ms),
    Kww (F_1^T phi(H_m) F_1 formed as a Gram, Theorem 3.1 / Sec. 6),
    Kww_gathered (E_W^T P), theta (Ritz values), resid, n_deflated.
    """
    L = sp.csr_matrix(L)
    n = L.shape[0]
    W = np.asarray(samples, dtype=np.int64)
    s = W.size
    f = _phi.make(phi_spec)
    thresh = tau * gershgorin_bound(L)
    Qs = [unit_block(n, W)]
    T = np.zeros((m * s, m * s))
    B_prev = None
    n_defl = 0
    resid = 0.0
    for k in range(m):
        Qk = Qs[k]
        X = L @ Qk
        if k > 0:
            X -= Qs[k - 1] @ B_prev.T               # H_{k-1,k} = H_{k,k-1}^T
        H = Qk.T @ X
        H = 0.5 * (H + H.T)
        X -= Qk @ H
        Qall = np.hstack(Qs)
        for _ in range(2):
            X -= Qall @ (Qall.T @ X)
        T[k * s:(k + 1) * s, k * s:(k + 1) * s] = H
        if k + 1 < m:
            Qn, R, d = _qr_deflating(X, thresh, flip_signs)
            n_defl += d
            Qs.append(Qn)
            T[(k + 1) * s:(k + 2) * s, k * s:(k + 1) * s] = R
            T[k * s:(k + 1) * s, (k + 1) * s:(k + 2) * s] = R.T
            B_prev = R
        else:
            resid = float(np.linalg.norm(X))
    Qcat = np.hstack(Qs)
    U, S, theta, ft = _phi_projected(T, f, s)
    P = Qcat @ U
    if np.all(ft >= 0):
        G = np.sqrt(ft)[:, None] * S[:s, :].T      # SPD by construction
        Kww = G.T @ G
    else:                                            # e.g. a polynomial phi
        Kww = S[:s, :] @ (ft[:, None] * S[:s, :].T)
    return dict(P=P, U=U, T=T, Q=Qcat, S=S, theta=theta, ftheta=ft, Kww=Kww,
                Kww_gathered=P[W, :], resid=resid, n_deflated=n_defl)


def gbl(L, samples, phi_spec, m: int, tau: float = DEFAULT_TAU):
    """Global block Lanczos, Alg. 2 (Frobenius inner product).

    Q_1 = E_W / sqrt(N); X = L Q_k - h_{k-1,k} Q_{k-1}; h_kk = tr(Q_k^T X);
    X -= h_kk Q_k; h_{k+1,k} = ||X||_F; Q_{k+1} = X / h_{k+1,k}.
    u = sqrt(N) phi(H_m) f_1 and the approximation is sum_k u_k Q_k.
    On breakdown (h_{k+1,k} < tau ||L||_1) the Krylov space is invariant and
    the iteration stops with the current H.
    """
    L = sp.csr_matrix(L)
    n = L.shape[0]
    W = np.asarray(samples, dtype=np.int64)
    s = W.size
    f = _phi.make(phi_spec)
    thresh = tau * gershgorin_bound(L)
    Qs = [unit_block(n, W) / np.sqrt(s)]
    alpha, beta = [], []
    resid = 0.0
    for k in range(m):
        X = L @ Qs[k]
        if k > 0:
            X -= beta[k - 1] * Qs[k - 1]
        a = float(np.sum(Qs[k] * X))
        X -= a * Qs[k]
        for _ in range(2):
            coef = [float(np.sum(Qj * X)) for Qj in Qs]
            for cj, Qj in zip(coef, Qs):
                X -= cj * Qj
        alpha.append(a)
        h = float(np.linalg.norm(X))
        if k + 1 < m:
            if h < thresh:
                break
            beta.append(h)
            Qs.append(X / h)
        else:
            resid = h
    mm = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:mm - 1], 1) + np.diag(beta[:mm - 1], -1)
    theta, S = np.linalg.eigh(T)
    u = np.sqrt(s) * (S @ (f(theta) * S[0, :]))
    P = sum(uk * Qk for uk, Qk in zip(u, Qs))
    return dict(P=P, u=u, T=T, theta=theta, Kww_gathered=P[W, :], resid=resid, m_eff=mm,
                Q_blocks=Qs)


def sbl(L, samples, phi_spec, m: int, tau: float = DEFAULT_TAU):
    """Sequential Lanczos (Sec. 3.3): an ordinary Lanczos run (Alg. 1 with
    block width 1) on each column e_{w_i} separately; H_m is the block
    diagonal of the per-column tridiagonal matrices."""
    W = np.asarray(samples, dtype=np.int64)
    cols, Ts = [], []
    for w in W:
        r = cbl(L, [int(w)], phi_spec, m, tau)
        cols.append(r["P"][:, 0])
        Ts.append(r["T"])
    P = np.stack(cols, axis=1)
    return dict(P=P, T_list=Ts, Kww_gathered=P[W, :])


def fit_predict(L, samples, y, phi_spec, m: int, gamma: float, variant: str = "cbl",
                tau: float = DEFAULT_TAU):
    """Krylov RLS predictor.

    cbl (Alg. 3): K = F_1^T phi(H_m) F_1 (Theorem 3.1: SPD), c from a Cholesky
    solve of (K + gamma I) c = y, prediction [Q_1..Q_m] phi(H_m) F_1 c
    (Corollary 1).  gbl / sbl: K = E_W^T P (symmetric but possibly indefinite,
    resp. non-symmetric, Sec. 8.3), c from an LU solve, prediction P c.
    `gamma` is the full diagonal shift.
    Returns (c, yhat, K).
    """
    y = np.asarray(y, dtype=np.float64)
    s = y.size
    if variant == "cbl":
        r = cbl(L, samples, phi_spec, m, tau)
        K = r["Kww"]
        c = sla.cho_solve(sla.cho_factor(K + gamma * np.eye(s), lower=False), y)
        return c, r["Q"] @ (r["U"] @ c), K
    r = {"gbl": gbl, "sbl": sbl}[variant](L, samples, phi_spec, m, tau)
    K = r["Kww_gathered"]
    c = sla.lu_solve(sla.lu_factor(K + gamma * np.eye(s)), y)
    return c, r["P"] @ c, K


def rel_fro(A, A_ref) -> float:
    """||A - A_ref||_F / ||A_ref||_F."""
    return float(np.linalg.norm(np.asarray(A) - np.asarray(A_ref)) / np.linalg.norm(A_ref))
