"""CSR geometric multigrid for the shifted operator L of the HSS iteration.

The paper approximates each HSS solve with multigrid using standard
transfer operators and a scaled-Jacobi smoother (Sec. 1 and Sec. 5.3).  The
schedule here is the textbook V(nu1, nu2) cycle with zero initial guess:

    x = 0;  nu1 sweeps  x <- x + omega D^{-1} (b - A x),  D = diag(A);
    b_c = P^T (b - A x);  e_c = cycle(level + 1, b_c);  x <- x + P e_c;
    nu2 sweeps as above;  on the coarsest level x = A^{-1} b (dense LU).

The coarse operators are rediscretised on each mesh (equal to the Galerkin
product P^T A P for nested conforming spaces; asserted by the tests).  P is
finite-element interpolation from `oracle.fem`.
"""

import numpy as np
import scipy.linalg as sla

from . import fem
from .operators import combine


class Level:
    def __init__(self, n, A, P=None):
        self.n = n
        self.A = A                      # CSR operator on this level
        self.D = A.diagonal().copy()    # Jacobi diagonal
        self.P = P                      # interpolation from level+1 to here


class Hierarchy:
    """Levels 0 (finest, n cells per side) to levels-1 (n / 2^(levels-1))."""

    def __init__(self, dim, n, levels, abc, faces=None):
        if n % (2 ** (levels - 1)) != 0:
            raise ValueError("n must be divisible by 2^(levels-1)")
        self.dim = dim
        self.levels = []
        for l in range(levels):
            nl = n // (2 ** l)
            K, M, MG = fem.assemble(dim, nl, faces)
            A = combine(K, M, MG, abc)
            P = fem.prolongation(dim, nl) if l < levels - 1 else None
            self.levels.append(Level(nl, A, P))
        coarse = self.levels[-1].A.toarray()
        self.coarse_lu = sla.lu_factor(coarse)

    def coarse_solve(self, b):
        return sla.lu_solve(self.coarse_lu, b)


def jacobi_sweep(level, x, b, omega):
    """One scaled-Jacobi sweep x + omega D^{-1} (b - A x)."""
    return x + omega * (b - level.A @ x) / level.D


def vcycle(hier, b, l=0, nu1=2, nu2=2, omega=2.0 / 3.0):
    """One V(nu1, nu2) cycle for A_l x = b with zero initial guess."""
    lev = hier.levels[l]
    if l == len(hier.levels) - 1:
        return hier.coarse_solve(b)
    x = np.zeros_like(b, dtype=np.complex128)
    for _ in range(nu1):
        x = jacobi_sweep(lev, x, b, omega)
    r = b - lev.A @ x
    bc = lev.P.T @ r
    ec = vcycle(hier, bc, l + 1, nu1, nu2, omega)
    x = x + lev.P @ ec
    for _ in range(nu2):
        x = jacobi_sweep(lev, x, b, omega)
    return x


def cycles(hier, b, count, nu1=2, nu2=2, omega=2.0 / 3.0):
    """`count` V-cycles used as a stationary iteration from x = 0:
    x <- x + V(b - A x).  This is how "one or more multigrid cycles"
    approximate an inner solve (Sec. 1, Sec. 5.3)."""
    A = hier.levels[0].A
    x = np.zeros_like(b, dtype=np.complex128)
    for _ in range(count):
        x = x + vcycle(hier, b - A @ x, 0, nu1, nu2, omega)
    return x


def error_propagator(hier, l=0, nu1=2, nu2=2, omega=2.0 / 3.0):
    """Dense error-propagation matrix of the cycle on level l, built by
    composition of its factors (used only on tiny meshes by the tests):

        E_l = S^nu2 (I - P (I - E_{l+1}) A_{l+1}^{-1} P^T A_l) S^nu1,
        S   = I - omega D^{-1} A_l,   E_coarsest = 0.
    """
    lev = hier.levels[l]
    A = lev.A.toarray()
    nl = A.shape[0]
    if l == len(hier.levels) - 1:
        return np.zeros((nl, nl), dtype=np.complex128)
    S = np.eye(nl) - omega * (A / lev.D[:, None])
    Ac = hier.levels[l + 1].A.toarray()
    Ec = error_propagator(hier, l + 1, nu1, nu2, omega)
    P = lev.P.toarray()
    Bc = (np.eye(Ac.shape[0]) - Ec) @ np.linalg.inv(Ac)   # approximate coarse inverse
    C = np.eye(nl) - P @ Bc @ P.T @ A
    return np.linalg.matrix_power(S, nu2) @ C @ np.linalg.matrix_power(S, nu1)
