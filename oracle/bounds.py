"""Error bounds of Sec. 4 used to pin the Krylov oracle.

Test infrastructure only (see the oracle package docstring).

Theorem 4.2: for the three Lanczos variants,
    ||phi(L) E_W - p_{phi,m}(L) E_W||_F <= 2 sqrt(N) E_m(phi),
with E_m the best uniform polynomial approximation error of degree m on
[0, Lambda].  The approximant built from m blocks has degree m-1 (Alg. 1
returns p_{phi,m-1}), so with m blocks the bound reads 2 sqrt(N) E_{m-1}(phi)
(the form Remark 2 uses).

Example 3 gives an explicit bound for E_m(exp(-t lam)) with the constants
b = (sqrt 5 - 1)/2 and d = (sqrt 5 - 2) e^b.
"""
from __future__ import annotations

import math

B_CONST = (math.sqrt(5.0) - 1.0) / 2.0
D_CONST = (math.sqrt(5.0) - 2.0) * math.exp(B_CONST)


def exp_best_approx_bound(m: int, t: float, Lam: float) -> float:
    """Upper bound for E_m(exp(-t lam)) on [0, Lam] (Example 3)."""
    tl = t * Lam
    b, d = B_CONST, D_CONST
    if m <= tl:
        return (2.0 * math.exp(-b * (m + 1) ** 2 / tl) * (1.0 + math.sqrt(tl * math.pi / (4.0 * b)))
                + 2.0 * d ** tl / (1.0 - d))
    return 2.0 * d ** m / (1.0 - d)


def lanczos_column_bound(n_samples: int, m_blocks: int, t: float, Lam: float) -> float:
    """2 sqrt(N) E_{m-1}(exp(-t lam)): bound on the Frobenius error of the
    Lanczos kernel columns after m blocks (Theorem 4.2 with Example 3)."""
    return 2.0 * math.sqrt(n_samples) * exp_best_approx_bound(m_blocks - 1, t, Lam)


def predictor_bound(y_norm: float, phi_min: float, phi_max: float, gamma_total: float,
                    kernel_err_2: float) -> float:
    """First-order bound of Theorem 5.1 on ||y - y^(kr)||_2 (gamma_total is
    the full diagonal shift gamma * N)."""
    a = phi_min + gamma_total
    return y_norm / a * (1.0 + phi_max / a) * kernel_err_2
