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


def nested_dissection_2d(n1, leaf=6):
    """Nested-dissection order of the n1 x n1 nodes of a 2D mesh (node index
    i + n1 j).  A box of nodes is split by its middle grid line across the
    longer side: the two halves are ordered (recursively) first and the
    line last.  No P1 edge of the right-diagonal triangulation crosses a
    grid line (edges join nodes at most one row and one column apart), so
    the two halves of every split are uncoupled in B_0 and their factors
    fill in only within each half and the separator.  Returns p with
    p[new] = old."""
    out = []

    def split(i0, i1, j0, j1):
        wi, wj = i1 - i0, j1 - j0
        if wi * wj <= leaf * leaf or min(wi, wj) < 3:
            I, J = np.meshgrid(np.arange(i0, i1), np.arange(j0, j1), indexing="xy")
            out.append((I + n1 * J).ravel())
        elif wi >= wj:
            m = (i0 + i1) // 2
            split(i0, m, j0, j1)
            split(m + 1, i1, j0, j1)
            out.append(m + n1 * np.arange(j0, j1))
        else:
            m = (j0 + j1) // 2
            split(i0, i1, j0, m)
            split(i0, i1, m + 1, j1)
            out.append(np.arange(i0, i1) + n1 * m)

    split(0, n1, 0, n1)
    return np.concatenate(out)


class Problem:
    def __init__(self, dim, n, k, delta_hat, delta=0.0, levels=1, faces=None,
                 nu1=2, nu2=2, omega=2.0 / 3.0, m=1, cycles=2, cycle="v", smooth_its=5,
                 dirichlet=()):
        self.dim, self.n, self.k = dim, n, float(k)
        self.delta, self.delta_hat = float(delta), float(delta_hat)
        self.nu1, self.nu2, self.omega, self.m = nu1, nu2, omega, m
        self.cycles = cycles            # cycles per inner HSS solve
        self.cycle = cycle              # "v": V(nu1, nu2) Jacobi; "w": the
        self.smooth_its = smooth_its    # paper's W-cycle, GMRES_its smoothing
        # faces with u = 0: their nodes are eliminated from every operator
        # and the boundary term lives on the remaining faces
        self.dirichlet = tuple(dirichlet)
        if self.dirichlet and faces is None:
            faces = fem.impedance_faces(dim, self.dirichlet)
        self.fixed = fem.dirichlet_node_mask(dim, n, self.dirichlet)
        self.K, self.M, self.MG = fem.assemble(dim, n, faces)
        K, M, MG = self.K, self.M, self.MG
        elim = (lambda A: fem.eliminate(A, self.fixed)) if self.dirichlet else (lambda A: A)
        self.B0 = elim(ops.b_delta(K, M, MG, k, delta).tocsr())
        self.Bdh = elim(ops.b_delta(K, M, MG, k, delta_hat).tocsr())
        self.L = elim(ops.hss_lhs(K, M, MG, k, delta_hat).tocsr())
        self.N = elim(ops.hss_rhs(K, M, MG, k, delta_hat).tocsr())
        self.H = elim(ops.h_gram(M, MG, k, delta_hat).tocsr())
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
        """u = B_0^{-1} b by sparse LU.  On 2D meshes the unknowns are first
        put in nested-dissection order (`nested_dissection_2d`), which keeps
        the factor of a 2049^2-node mesh within a few GB; the solution is
        the same vector in the original order."""
        b = np.asarray(b, dtype=np.complex128)
        if self._lu_B0 is None:
            if self.dim == 2:
                p = nested_dissection_2d(self.n + 1)
                A = self.B0[p][:, p].tocsc()
                self._lu_B0 = (spla.splu(A, permc_spec="NATURAL", diag_pivot_thresh=0.01,
                                         options=dict(SymmetricMode=True)), p)
            else:
                self._lu_B0 = (spla.splu(self.B0.tocsc()), None)
        lu, p = self._lu_B0
        if p is None:
            return lu.solve(b)
        u = np.empty_like(b)
        u[p] = lu.solve(b[p])
        return u

    # -- multigrid ------------------------------------------------------------
    @property
    def hierarchy(self):
        if self._hier is None:
            abc = ops.coefficients("L", self.k, self.delta_hat)
            self._hier = multigrid.Hierarchy(self.dim, self.n, self.levels, abc, self.faces,
                                             self.dirichlet)
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
