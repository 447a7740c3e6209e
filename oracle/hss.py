"""The gamma=k HSS iteration and the shifted-HSS preconditioner.

Literal form (Definition "gamma=k HSS iteration in primal form",
eq. (primal-hss-system), and Definition "Shifted HSS iteration for the primal
system", eq. (HSSpc primal), which is the same iteration with delta_hat):

    L u_{n+1} = ((k-1)/(k+1)) N u_n + (2k/(k+1)) R,     u_0 = 0,
    n = 0, ..., m ceil(k) - 1,   and  B~^{-1} R = u_{m ceil(k)}.

Correction form.  From (k+1) L - (k-1) N = 2k B_delta (a consequence of the
definitions of L, N and B_delta, asserted by the tests) the same step reads

    u_{n+1} = u_n + L^{-1} [ (2k/(k+1)) (R - B_delta u_n) ].

The two agree exactly when L^{-1} is applied exactly.  When L^{-1} is
replaced by one multigrid cycle (Sec. 5.3) the correction form is the one
used: the cycle then approximates the correction, starting from zero, which
equals a cycle warm-started at u_n.
"""

import numpy as np


def hss_literal(L, N, R, k, steps, inner_solve, history=None):
    """`steps` iterations of eq. (HSSpc primal) from u_0 = 0."""
    u = np.zeros_like(R, dtype=np.complex128)
    for _ in range(steps):
        rhs = ((k - 1.0) / (k + 1.0)) * (N @ u) + (2.0 * k / (k + 1.0)) * R
        u = inner_solve(rhs)
        if history is not None:
            history.append(u.copy())
    return u


def hss_correction(B_shift, R, k, steps, inner_solve, history=None):
    """`steps` iterations of the correction form from u_0 = 0."""
    u = np.zeros_like(R, dtype=np.complex128)
    c = 2.0 * k / (k + 1.0)
    for _ in range(steps):
        rho = c * (R - B_shift @ u)
        u = u + inner_solve(rho)
        if history is not None:
            history.append(u.copy())
    return u


def contraction_factor(k):
    """nu_s = (1 - 1/k)/(1 + 1/k) = (k-1)/(k+1), eq. (primal-hss-contraction)."""
    return (k - 1.0) / (k + 1.0)


def h_norm(H, e):
    """||e||_H = sqrt(e^H H e) for the H_primal Gram matrix."""
    return float(np.sqrt(np.real(np.vdot(e, H @ e))))
