"""Outer iterations for B_0 u = G (Sec. 5.1): flexible GMRES and
preconditioned Richardson.

FGMRES is Saad's flexible, right-preconditioned GMRES: it stores the
preconditioned directions z_j so that x = x_0 + Z y holds even when the
preconditioner varies between applications.  Orthogonalisation here is
modified Gram-Schmidt (one pass) and the least-squares problem is reduced
with Givens rotations.  Convergence is declared on the 2-norm of the
residual relative to ||b||, then re-checked on the true residual.

Richardson is the stationary iteration  B~ x^{n+1} = (B~ - B_0) x^n + G
of Sec. 4, i.e.  x^{n+1} = x^n + B~^{-1} (G - B_0 x^n).
"""

import numpy as np


def fgmres(apply_A, b, precond, tol=1e-8, restart=200, maxiter=1000, x0=None):
    """Returns (x, info) with info = {'its', 'history', 'converged'}.

    `history` lists the Arnoldi residual norms relative to ||b||, one per
    iteration (entry 0 is the initial residual).
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), {"its": 0, "history": [0.0], "converged": True}
    history = []
    its = 0
    converged = False
    while its < maxiter:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if not history:
            history.append(beta / bnorm)
        if beta <= tol * bnorm:
            converged = True
            break
        m = min(restart, maxiter - its)
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        Z = np.zeros((m, b.size), dtype=np.complex128)
        Hs = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = apply_A(Z[j])
            for i in range(j + 1):               # modified Gram-Schmidt
                Hs[i, j] = np.vdot(V[i], w)
                w = w - Hs[i, j] * V[i]
            Hs[j + 1, j] = np.linalg.norm(w)
            if Hs[j + 1, j] != 0.0:
                V[j + 1] = w / Hs[j + 1, j]
            for i in range(j):                   # previous rotations
                t = cs[i] * Hs[i, j] + sn[i] * Hs[i + 1, j]
                Hs[i + 1, j] = -np.conj(sn[i]) * Hs[i, j] + np.conj(cs[i]) * Hs[i + 1, j]
                Hs[i, j] = t
            a, bb = Hs[j, j], Hs[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            # rotation [c s; -s* c*] with c = conj(a)/den, s = conj(bb)/den
            # maps (a, bb) to (den, 0)
            cs[j] = np.conj(a) / den if den != 0 else 1.0
            sn[j] = np.conj(bb) / den if den != 0 else 0.0
            Hs[j, j] = cs[j] * a + sn[j] * bb
            Hs[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or its >= maxiter:
                break
        y = np.linalg.solve(np.triu(Hs[:j_done, :j_done]), g[:j_done])
        x = x + Z[:j_done].T @ y
    r = b - apply_A(x)
    true_rel = np.linalg.norm(r) / bnorm
    converged = converged or true_rel <= tol * (1 + 1e-6)
    return x, {"its": its, "history": history, "converged": bool(converged),
               "true_rel_residual": float(true_rel)}


def richardson(apply_A, b, precond, tol=1e-8, maxiter=1000, x0=None):
    """Preconditioned Richardson; returns (x, info) like `fgmres`."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    history = []
    its = 0
    while True:
        r = b - apply_A(x)
        history.append(np.linalg.norm(r) / bnorm)
        if history[-1] <= tol or its >= maxiter:
            break
        x = x + precond(r)
        its += 1
    return x, {"its": its, "history": history, "converged": history[-1] <= tol,
               "true_rel_residual": float(history[-1])}
