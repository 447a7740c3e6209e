"""Pins for the oracle's assembly and transfer operators (Sec. 2).

Each check comes from outside the oracle: an invariant of the continuous
forms (constants are in the kernel of the gradient, the mass of 1 is the
area, the boundary mass of 1 is the perimeter), the textbook O(h^2) L2 rate
of CG1/Q1 on a manufactured solution, nestedness of the spaces (Galerkin
identity), and the closed-form P1 stencil values derived by hand.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, operators as ops


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_2d_invariants(n):
    K, M, MG = fem.assemble_2d(n)
    one = np.ones(K.shape[0])
    assert np.abs(K @ one).max() < 1e-13            # constants are harmonic
    assert abs(one @ M @ one - 1.0) < 1e-13         # area of the unit square
    assert abs(one @ MG @ one - 4.0) < 1e-13        # perimeter
    for A in (K, M, MG):
        assert abs(A - A.T).max() < 1e-15
    x, y = fem.nodes_2d(n).T
    # int grad x . grad x = 1, int x^2 = 1/3 (P1 reproduces linears exactly in K)
    assert abs(x @ K @ x - 1.0) < 1e-12
    assert abs(y @ K @ y - 1.0) < 1e-12


@pytest.mark.parametrize("n", [1, 2, 4])
def test_3d_invariants(n):
    K, M, MG = fem.assemble_3d(n)
    one = np.ones(K.shape[0])
    assert np.abs(K @ one).max() < 1e-13
    assert abs(one @ M @ one - 1.0) < 1e-13
    assert abs(one @ MG @ one - 6.0) < 1e-13
    x, y, z = fem.nodes_3d(n).T
    assert abs(z @ K @ z - 1.0) < 1e-12
    assert abs(x @ M @ x - 1.0 / 3.0) < 1e-12       # Q1 integrates x^2 exactly


def test_2d_k_positive_semidefinite_with_constant_kernel():
    K, M, MG = fem.assemble_2d(4)
    w = np.linalg.eigvalsh(K.toarray())
    assert w[0] > -1e-12 and abs(w[0]) < 1e-12 and w[1] > 1e-3


def _class_rows_2d(n):
    """Hand-derived rows of K, M (times 24/h^2) and MG (times 6/h) for the
    right-diagonal mesh.  c_pq flags whether the cell whose corner is the
    node sits at offset (p-1, q-1) lies in the domain."""
    rows = {}
    for j in range(n + 1):
        for i in range(n + 1):
            c00 = int(i > 0 and j > 0)
            c10 = int(i < n and j > 0)
            c01 = int(i > 0 and j < n)
            c11 = int(i < n and j < n)
            K = {(0, 0): c00 + c10 + c01 + c11,
                 (1, 0): -(c11 + c10) / 2, (-1, 0): -(c01 + c00) / 2,
                 (0, 1): -(c11 + c01) / 2, (0, -1): -(c00 + c10) / 2}
            M = {(0, 0): 2 * (2 * c11 + c01 + 2 * c00 + c10),
                 (1, 0): c11 + c10, (-1, 0): c01 + c00,
                 (0, 1): c11 + c01, (0, -1): c00 + c10,
                 (1, 1): 2 * c11, (-1, -1): 2 * c00}
            hor = int(j == 0) + int(j == n)
            ver = int(i == 0) + int(i == n)
            G = {(1, 0): hor * int(i < n), (-1, 0): hor * int(i > 0),
                 (0, 1): ver * int(j < n), (0, -1): ver * int(j > 0)}
            G[(0, 0)] = 2 * sum(G.values())
            rows[(i, j)] = (K, M, G)
    return rows


@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_2d_rows_match_hand_derived_classes(n):
    h = 1.0 / n
    K, M, MG = (A.toarray() for A in fem.assemble_2d(n))
    for (i, j), (kr, mr, gr) in _class_rows_2d(n).items():
        r = i + (n + 1) * j
        for A, want, scale in ((K, kr, 1.0), (M, mr, h * h / 24), (MG, gr, h / 6)):
            expect = np.zeros(A.shape[1])
            for (di, dj), v in want.items():
                ii, jj = i + di, j + dj
                if 0 <= ii <= n and 0 <= jj <= n:
                    expect[ii + (n + 1) * jj] += v * scale
            assert np.abs(A[r] - expect).max() < 1e-14, (i, j)


@pytest.mark.parametrize("dim,n", [(2, 2), (2, 8), (3, 2), (3, 4)])
def test_galerkin_identity_and_interpolation(dim, n):
    Kf, Mf, Gf = fem.assemble(dim, n)
    Kc, Mc, Gc = fem.assemble(dim, n // 2)
    P = fem.prolongation(dim, n)
    for Af, Ac in ((Kf, Kc), (Mf, Mc), (Gf, Gc)):
        assert abs(P.T @ Af @ P - Ac).max() < 1e-13
    xf = fem.nodes(dim, n)
    xc = fem.nodes(dim, n // 2)
    assert np.abs(P @ np.ones(P.shape[1]) - 1).max() < 1e-14
    for d in range(dim):                              # linears are reproduced
        assert np.abs(P @ xc[:, d] - xf[:, d]).max() < 1e-14
    assert P.shape == ((n + 1) ** dim, (n // 2 + 1) ** dim)


def _mms_error(dim, n, k, delta, wave):
    """Discrete solution of the plane-wave manufactured problem vs the
    nodal interpolant, in the M-norm."""
    s = -delta + 1j * k
    wv = np.asarray(wave, dtype=float)
    lam = s * s + wv @ wv                     # f = ((-delta+ik)^2 + |w|^2) u

    def u(*x):
        return np.exp(1j * sum(wi * xi for wi, xi in zip(wv, x)))

    def f(*x):
        return lam * u(*x)

    def g(*args):                              # d_n u - (-delta + ik) u
        x, nrm = args[:-1], np.asarray(args[-1])
        return (1j * (wv @ nrm) - s) * u(*x)

    K, M, MG = fem.assemble(dim, n)
    B = ops.b_delta(K, M, MG, k, delta).tocsc()
    b = (fem.load_vector_2d(n, f, g) if dim == 2 else fem.load_vector_3d(n, f, g))
    uh = spla.spsolve(B, b)
    e = uh - u(*fem.nodes(dim, n).T)
    return float(np.sqrt(np.real(np.vdot(e, M @ e))))


def test_mms_p1_second_order():
    errs = [_mms_error(2, n, 4.0, 0.5, (2.0, 1.5)) for n in (8, 16, 32, 64)]
    rates = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.6 < r < 4.4 for r in rates[1:]), rates


def test_mms_p1_second_order_no_absorption():
    errs = [_mms_error(2, n, 3.0, 0.0, (1.0, -2.5)) for n in (16, 32, 64)]
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.6 < r < 4.4 for r in rates), rates


def test_mms_q1_second_order():
    errs = [_mms_error(3, n, 2.0, 0.5, (1.5, 1.0, -0.5)) for n in (4, 8, 16)]
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.4 < r < 4.6 for r in rates), rates


def test_sampled_q1_rows_match_assembled_b0():
    """The row-at-a-time 3D B_0 used to check meshes too large to assemble
    equals the assembled operator on every row of a small mesh."""
    from gpu_util import q1_b0_rows, oracle_matrix
    n, k = 5, 3.5
    B = oracle_matrix(3, n, "B0", k, k).toarray()
    allpts = [(i, j, l) for l in range(n + 1) for j in range(n + 1) for i in range(n + 1)]
    for r, (cols, vals) in enumerate(q1_b0_rows(n, k, allpts)):
        row = np.zeros(B.shape[1], complex)
        row[cols] = vals
        assert np.abs(row - B[r]).max() < 1e-14 * np.abs(B).max()


def test_sampled_q1_rows_match_assembled_operators():
    """The row builder for any a K + b M + c M_Gamma (here L and B_shift of
    the HSS step) equals the assembled operator on every row of a small mesh,
    and its diagonal is the Jacobi diagonal."""
    from gpu_util import q1_rows, row_apply, row_diag
    from oracle import operators as ops
    n, k, dh = 4, 3.5, 2.0
    K, M, MG = fem.assemble(3, n)
    allpts = [(i, j, l) for l in range(n + 1) for j in range(n + 1) for i in range(n + 1)]
    x = np.random.default_rng(5).standard_normal((n + 1) ** 3) * (1 + 1j)
    for name, delta in (("L", dh), ("B", dh)):
        abc = ops.coefficients(name, k, delta)
        A = ops.combine(K, M, MG, abc)
        rows = q1_rows(n, abc, allpts)
        assert np.abs(row_apply(rows, x) - A @ x).max() < 1e-13 * np.abs(A @ x).max()
        assert np.abs(row_diag(rows, allpts, n) - A.diagonal()).max() < 1e-14 * np.abs(A.diagonal()).max()


def test_sampled_q1_transfer_rows_match_prolongation():
    """Rows of P from the oracle's Q1 basis, and rows of P^T gathered from
    them, equal the oracle's assembled trilinear prolongation."""
    from gpu_util import q1_prolong_row, q1_restrict_rows
    n = 6
    nc = n // 2
    P = fem.prolongation_3d(n).toarray()
    for l in range(n + 1):
        for j in range(n + 1):
            for i in range(n + 1):
                cols, w = q1_prolong_row(n, (i, j, l))
                row = np.zeros(P.shape[1])
                row[cols] = w
                assert np.abs(row - P[i + (n + 1) * (j + (n + 1) * l)]).max() < 1e-15
    cpts = [(I, J, L) for L in range(nc + 1) for J in range(nc + 1) for I in range(nc + 1)]
    for C, (fine, w) in enumerate(q1_restrict_rows(n, cpts)):
        col = np.zeros(P.shape[0])
        col[[f[0] + (n + 1) * (f[1] + (n + 1) * f[2]) for f in fine]] = w
        assert np.abs(col - P[:, C]).max() < 1e-15


def test_sampled_p1_rows_match_assembled_b0():
    """The row-at-a-time 2D B_0 equals the assembled operator on every row
    of a small mesh."""
    from gpu_util import p1_b0_rows, oracle_matrix
    n, k = 7, 2.5
    B = oracle_matrix(2, n, "B0", k, k).toarray()
    allpts = [(i, j) for j in range(n + 1) for i in range(n + 1)]
    for r, (cols, vals) in enumerate(p1_b0_rows(n, k, allpts)):
        row = np.zeros(B.shape[1], complex)
        row[cols] = vals
        assert np.abs(row - B[r]).max() < 1e-14 * np.abs(B).max()
