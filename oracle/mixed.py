"""The mixed formulation of Sec. 2 and its shifted-HSS preconditioner
(Definition "Shifted HSS preconditioner for the mixed system"), 2D.

Spaces: sigma in [DG0]^2 (one constant vector per triangle of the
right-diagonal mesh), u in CG1 = P1, so that grad u lies in the sigma space
(the embedding property of Sec. 2).  With a real basis the forms of the
mixed system a_delta((v, tau), (u, sigma)) become the block matrix

    A_delta = [ (delta - i k) M_s    -G                         ]   sigma rows
              [  G^T                 (delta - i k) M + M_Gamma   ]   u rows

with M_s the DG0 mass (area times identity per triangle and component),
G the matrix of <tau, grad u> (G^T that of <grad v, sigma>), M the P1 mass
and M_Gamma the boundary mass.  The right-hand side is F_sigma = 0 and
F_u[v] = int f v / (delta - i k), i.e. the load vector b = M f divided by
(delta - i k).

Unknown vectors are stacked as [u (N nodes) | sigma], sigma ordered by
triangle (the order of `fem.triangles_2d`) with its two components
interleaved.

The HSS step with gamma = k in the H_mixed inner product
delta<sigma, tau> + delta<u, v> + <<u, v>> (whose skew part S_mixed is
skew-Hermitian in that inner product) is written literally as one block
solve per step (`hss_step_literal`), and in the form the paper derives by
eliminating sigma_{n+1} with the embedding property (`hss_step_eliminated`):
a scalar shifted system K + k^2 (dh - i)^2 M + k^2 (dh - i) M_Gamma for
u_{n+1}, then sigma_{n+1} recovered triangle by triangle.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


def dg0_gradient(n):
    """G (2 E x N, E = 2 n^2 triangles): row (e, c) holds |T_e| times the
    c-th component of the gradient of each P1 basis function on T_e, so
    (G u)[e, c] = int_{T_e} d_c u  =  <tau_{e,c}, grad u>."""
    xy = fem.nodes_2d(n)
    tri = fem.triangles_2d(n)
    E = tri.shape[0]
    P = xy[tri]                                                  # (E, 3, 2)
    B = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=2)  # (E, 2, 2)
    area = 0.5 * np.abs(np.linalg.det(B))
    gref = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    grad = np.einsum("as,est->eat", gref, np.linalg.inv(B))      # (E, 3, 2)
    rows, cols, vals = [], [], []
    for a in range(3):
        for c in range(2):
            rows.append(2 * np.arange(E) + c)
            cols.append(tri[:, a])
            vals.append(area * grad[:, a, c])
    G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * E, xy.shape[0]))
    return G, np.repeat(area, 2)


class MixedProblem:
    """Matrices of the mixed system on the n x n right-diagonal mesh."""

    def __init__(self, n, k, delta_hat, delta=0.0):
        self.n, self.k, self.delta, self.delta_hat = n, float(k), float(delta), float(delta_hat)
        self.K, self.M, self.MG = fem.assemble_2d(n)
        self.G, self.ms = dg0_gradient(n)          # ms: diagonal of M_s
        self.N = self.K.shape[0]
        self.E2 = self.G.shape[0]                  # 2 * triangles
        self.A0 = self.system(delta)
        self._lu = None
        self._lm = None

    def system(self, delta):
        """A_delta as a sparse block matrix on [u | sigma]."""
        s = delta - 1j * self.k
        Ms = sp.diags(self.ms)
        return sp.bmat([[s * self.M + self.MG, self.G.T],
                        [-self.G, s * Ms]], format="csr").astype(np.complex128)

    def h_gram(self, delta):
        """Gram matrix of the H_mixed inner product on [u | sigma]."""
        return sp.block_diag([delta * self.M + self.MG, delta * sp.diags(self.ms)],
                             format="csr").astype(np.complex128)

    def skew(self):
        """The matrix of <S_mixed U, V>_H_mixed (the form that defines S)."""
        k = self.k
        Ms = sp.diags(self.ms)
        return sp.bmat([[-1j * k * self.M, self.G.T],
                        [-self.G, -1j * k * Ms]], format="csr").astype(np.complex128)

    def rhs(self, b_load, delta=None):
        """F = (F_u, F_sigma) = (b / (delta - i k), 0) for a P1 load vector b."""
        d = self.delta if delta is None else delta
        return np.concatenate([np.asarray(b_load, complex) / (d - 1j * self.k),
                               np.zeros(self.E2, complex)])

    def solve_direct(self, F):
        if self._lu is None:
            self._lu = spla.splu(self.A0.tocsc())
        return self._lu.solve(np.asarray(F, dtype=np.complex128))

    # -- the HSS step of the shifted-HSS preconditioner --------------------
    def hss_step_literal(self, U, R):
        """(k H + S) U' = nu (k H - S) U + c R  in the H_mixed inner product
        with delta_hat (the two equations of the mixed preconditioner's
        definition), solved as one sparse block system."""
        k, dh = self.k, self.delta_hat
        nu, c = (k - 1.0) / (k + 1.0), 2.0 * k / (k + 1.0)
        H, S = self.h_gram(dh), self.skew()
        lhs = (k * H + S).tocsc()
        return spla.spsolve(lhs, nu * ((k * H - S) @ U) + c * R)

    def lmix(self):
        """The scalar operator of the eliminated step:
        K + k^2 (dh - i)^2 M + k^2 (dh - i) M_Gamma."""
        k, dh = self.k, self.delta_hat
        s = dh - 1j
        return (self.K + (k * k * s * s) * self.M + (k * k * s) * self.MG).tocsr()

    def _lmix_csr(self):
        if self._lm is None:
            self._lm = self.lmix()
        return self._lm

    def hss_step_eliminated(self, U, R, solve_lmix):
        """The same step with sigma_{n+1} eliminated: from the sigma rows,
        k (dh - i) sigma' = grad u' + g with
        g = nu (k (dh + i) sigma + grad u) + c M_s^{-1} R_sigma;
        substituted into the u rows (and multiplied by k (dh - i)),
        Lmix u' = k (dh - i) [nu (k (dh + i) M u - G^T sigma + k M_Gamma u)
                               + c R_u] - G^T g.
        The scalar solve is taken in correction form, u' = u + Lmix^{-1}
        (rhs - Lmix u), as for the primal preconditioner (identical with an
        exact solve; with multigrid it is a cycle warm-started at u)."""
        k, dh = self.k, self.delta_hat
        nu, c = (k - 1.0) / (k + 1.0), 2.0 * k / (k + 1.0)
        N = self.N
        u, sig = U[:N], U[N:]
        Ru, Rs = R[:N], R[N:]
        grad = lambda w: (self.G @ w) / self.ms          # grad u per triangle
        g = nu * (k * (dh + 1j) * sig + grad(u)) + c * Rs / self.ms
        ru = nu * (k * (dh + 1j) * (self.M @ u) - self.G.T @ sig + k * (self.MG @ u)) + c * Ru
        rhs = k * (dh - 1j) * ru - self.G.T @ g
        u1 = u + solve_lmix(rhs - self._lmix_csr() @ u)
        s1 = (grad(u1) + g) / (k * (dh - 1j))
        return np.concatenate([u1, s1])

    def precond(self, R, steps=None, solve_lmix=None):
        """A~^{-1} R: m ceil(k) eliminated HSS steps from (0, 0); the scalar
        solves exact (sparse LU) unless `solve_lmix` is given."""
        if solve_lmix is None:
            lu = spla.splu(self.lmix().tocsc())
            solve_lmix = lu.solve
        S = int(np.ceil(self.k)) if steps is None else steps
        U = np.zeros(self.N + self.E2, complex)
        for _ in range(S):
            U = self.hss_step_eliminated(U, R, solve_lmix)
        return U
