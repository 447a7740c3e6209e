"""End-to-end reference solve: outer FGMRES on B_0 preconditioned by the
shifted-HSS preconditioner (Sec. 4), whose inner solves with L are either
exact (sparse LU, Sec. 5.2) or a fixed number of V-cycles each (Sec. 5.3;
default two: with one V(2,2)-Jacobi cycle the inexact HSS iteration has
error modes that grow, see the tests).

`Problem` assembles everything once for a mesh and parameter set; the
methods return plain numpy arrays.  The direct solution B_0^{-1} b is the
unique discrete solution the iterative method converges to (the paper
assumes the discrete problem is well posed, Sec. 2).
"""

import numpy as np
import scipy.sparse.linalg as spla

from . import fem, operators as ops, hss, multigrid, krylov


class Problem:
    def __init__(self, dim, n, k, delta_hat, delta=0.0, levels=1, faces=None,
                 nu1=2, nu2=2, omega=2.0 / 3.0, m=1, cycles=2, cycle="v", smooth_its=5):
        self.dim, self.n, self.k = dim, n, float(k)
        self.delta, self.delta_hat = float(delta), float(delta_hat)
        self.nu1, self.nu2, self.omega, self.m = nu1, nu2, omega, m
        self.cycles = cycles            # cycles per inner HSS solve
        self.cycle = cycle              # "v": V(nu1, nu2) Jacobi; "w": the
        self.smooth_its = smooth_its    # paper's W-cycle, GMRES_its smoothing
        self.K, self.M, self.MG = fem.assemble(dim, n, faces)
        K, M, MG = self.K, self.M, self.MG
        self.B0 = ops.b_delta(K, M, MG, k, delta).tocsr()
        self.Bdh = ops.b_delta(K, M, MG, k, delta_hat).tocsr()
        self.L = ops.hss_lhs(K, M, MG, k, delta_hat).tocsr()
        self.N = ops.hss_rhs(K, M, MG, k, delta_hat).tocsr()
        self.H = ops.h_gram(M, MG, k, delta_hat).tocsr()
        self.levels = levels
        self._lu_L = None
        self._lu_B0 = None
        self._hier = None
        self.faces = faces

    # -- exact solves -------------------------------------------------------
    def solve_L(self, r):
        if self._lu_L is None:
            self._lu_L = spla.splu(self.L.tocsc())
        return self._lu_L.solve(np.asarray(r, dtype=np.complex128))

    def solve_direct(self, b):
        """u = B_0^{-1} b by sparse LU."""
        if self._lu_B0 is None:
            self._lu_B0 = spla.splu(self.B0.tocsc())
        return self._lu_B0.solve(np.asarray(b, dtype=np.complex128))

    # -- multigrid ------------------------------------------------------------
    @property
    def hierarchy(self):
        if self._hier is None:
            abc = ops.coefficients("L", self.k, self.delta_hat)
            self._hier = multigrid.Hierarchy(self.dim, self.n, self.levels, abc, self.faces)
        return self._hier

    def vcycle(self, b):
        return multigrid.vcycle(self.hierarchy, np.asarray(b, dtype=np.complex128),
                                0, self.nu1, self.nu2, self.omega)

    def mg_solve(self, b):
        """Inner HSS solve by `cycles` V-cycles (x <- x + V(b - L x), x0 = 0),
        or by `cycles` of the paper's W-cycles (cycle = "w")."""
        b = np.asarray(b, dtype=np.complex128)
        if self.cycle == "w":
            return multigrid.w_cycles(self.hierarchy, b, self.cycles, self.smooth_its)
        return multigrid.cycles(self.hierarchy, b, self.cycles, self.nu1, self.nu2, self.omega)

    # -- preconditioner -------------------------------------------------------
    def hss_steps(self):
        return ops.inner_iterations(self.k, self.m)

    def precond(self, R, inner="mg", steps=None):
        """B~^{-1} R: shifted-HSS preconditioner in correction form."""
        solve = self.mg_solve if inner == "mg" else self.solve_L
        nsteps = self.hss_steps() if steps is None else steps
        return hss.hss_correction(self.Bdh, np.asarray(R, dtype=np.complex128),
                                  self.k, nsteps, solve)

    # -- outer solve ------------------------------------------------------------
    def solve(self, b, tol=1e-8, inner="mg", restart=200, maxiter=2000, x0=None,
              method="fgmres"):
        A = lambda x: self.B0 @ x
        P = lambda r: self.precond(r, inner)
        if method == "fgmres":
            return krylov.fgmres(A, b, P, tol=tol, restart=restart, maxiter=maxiter, x0=x0)
        return krylov.richardson(A, b, P, tol=tol, maxiter=maxiter, x0=x0)


def load_from_nodal(M, f_nodal):
    """Load vector b = M f for a source given by its nodal values
    (b_i = int I_h f phi_i); used for the Gaussian sources."""
    return M @ np.asarray(f_nodal, dtype=np.complex128)
