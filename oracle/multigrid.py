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

The paper's own multigrid variant (Sec. 5.3) is also here: a W-cycle whose
smoother on every level, the coarsest included, is a few iterations of
GMRES preconditioned by Jacobi (no coarse factorisation):

    x <- GMRES_m(x; b) on level l;  b_c = P^T (b - A x);  e_c = 0;
    e_c <- W(l + 1; b_c, e_c) twice;  x <- x + P e_c;  x <- GMRES_m(x; b),

and on the coarsest level x <- GMRES_m(x; b).  GMRES_m is m iterations of
left-preconditioned GMRES from the current x: with r = D^{-1}(b - A x) it
returns x + V y, V an orthonormal basis of the Krylov space
span{r, (D^{-1}A) r, ..., (D^{-1}A)^{m-1} r} and y minimising
|D^{-1}(b - A (x + V y))|_2 (the minimal-residual property that defines
GMRES; the basis is built by Arnoldi with modified Gram-Schmidt and the
small least-squares problem is solved by numpy).  Left preconditioning is a
reading: the paper names GMRES with a Jacobi preconditioner, not the side.
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
    """Levels 0 (finest, n cells per side) to levels-1 (n / 2^(levels-1)).

    `dirichlet` names faces with u = 0 (e.g. ("x0", "x1")): on every level
    their nodes are eliminated (`fem.eliminate`), the boundary term stays on
    the other faces, and P interpolates between the reduced spaces
    (`fem.restrict_prolongation`)."""

    def __init__(self, dim, n, levels, abc, faces=None, dirichlet=()):
        if n % (2 ** (levels - 1)) != 0:
            raise ValueError("n must be divisible by 2^(levels-1)")
        self.dim = dim
        self.levels = []
        if dirichlet and faces is None:
            faces = fem.impedance_faces(dim, dirichlet)
        for l in range(levels):
            nl = n // (2 ** l)
            K, M, MG = fem.assemble(dim, nl, faces)
            A = combine(K, M, MG, abc)
            P = fem.prolongation(dim, nl) if l < levels - 1 else None
            if dirichlet:
                A = fem.eliminate(A, fem.dirichlet_node_mask(dim, nl, dirichlet))
                if P is not None:
                    P = fem.restrict_prolongation(P, fem.dirichlet_node_mask(dim, nl, dirichlet),
                                                  fem.dirichlet_node_mask(dim, nl // 2, dirichlet))
            self.levels.append(Level(nl, A, P))
        self._coarse_lu = None

    def coarse_solve(self, b):
        if self._coarse_lu is None:   # dense LU of the coarsest operator
            self._coarse_lu = sla.lu_factor(self.levels[-1].A.toarray())
        return sla.lu_solve(self._coarse_lu, b)


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


def gmres_jacobi(level, x, b, its):
    """`its` iterations of Jacobi-left-preconditioned GMRES for A x = b
    from the given x (see the module notes); returns the new x."""
    A, D = level.A, level.D
    r = (b - A @ x) / D
    beta = np.linalg.norm(r)
    if beta == 0.0:
        return x.copy()
    V = np.zeros((its + 1, b.size), dtype=np.complex128)
    H = np.zeros((its + 1, its), dtype=np.complex128)
    V[0] = r / beta
    m = its
    for j in range(its):                       # Arnoldi, modified Gram-Schmidt
        w = (A @ V[j]) / D
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:                 # the Krylov space is invariant
            m = j + 1
            break
        V[j + 1] = w / H[j + 1, j]
    g = np.zeros(m + 1, dtype=np.complex128)
    g[0] = beta
    y = np.linalg.lstsq(H[:m + 1, :m], g, rcond=None)[0]
    return x + V[:m].T @ y


def wcycle(hier, b, x, l=0, its=5):
    """One W-cycle for A_l x = b from the given x, GMRES_its smoothing on
    every level (the coarsest: one GMRES_its application); returns x."""
    lev = hier.levels[l]
    if l == len(hier.levels) - 1:
        return gmres_jacobi(lev, x, b, its)
    x = gmres_jacobi(lev, x, b, its)
    bc = lev.P.T @ (b - lev.A @ x)
    ec = np.zeros_like(bc)
    for _ in range(2):
        ec = wcycle(hier, bc, ec, l + 1, its)
    x = x + lev.P @ ec
    return gmres_jacobi(lev, x, b, its)


def w_cycles(hier, b, count, its=5):
    """`count` W-cycles from x = 0 (each after the first continues from the
    previous iterate): the paper's inner HSS solve with multigrid."""
    x = np.zeros_like(b, dtype=np.complex128)
    for _ in range(count):
        x = wcycle(hier, b, x, 0, its)
    return x
