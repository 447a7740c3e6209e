"""Pins for the oracle's Dirichlet faces (u = 0 on some faces, the impedance
condition of Sec. 2 on the rest).

What fixes them from outside the oracle: the textbook O(h^2) L2 rate of
CG1/Q1 on manufactured solutions that vanish on the Dirichlet faces and
carry impedance data on the others (a boundary term left on a Dirichlet
face, a wrong node on an edge or corner, or a sign slip in the elimination
breaks the rate or the solution), node counts of the faces, the fact that
a face's boundary mass couples only that face's nodes, the Galerkin
identity of the reduced spaces, and convergence of the V-cycle iteration
and of the HSS iteration to the direct solve.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, multigrid, operators as ops, solver as osolver


def _grad_dot_n(grad, normal):
    return sum(gd * nd for gd, nd in zip(grad, normal))


def _mms(dim, n, k, delta, dirichlet, u, grad_u, lap_u):
    """Discrete solution with `dirichlet` faces vs the nodal interpolant of
    u, in the M-norm.  -lap u + (-delta + ik)^2 u = f inside, u = 0 on the
    Dirichlet faces, d_n u - (-delta + ik) u = g on the others (the strong
    form of b_delta, Sec. 2)."""
    s = -delta + 1j * k
    f = lambda *x: -lap_u(*x) + s * s * u(*x)

    def g(*args):
        x, nrm = args[:-1], args[-1]
        return _grad_dot_n(grad_u(*x), nrm) - s * u(*x)

    pr = osolver.Problem(dim, n, k, k, delta=delta, dirichlet=dirichlet)
    imp = fem.impedance_faces(dim, dirichlet)
    b = (fem.load_vector_2d(n, f, g, faces=imp) if dim == 2
         else fem.load_vector_3d(n, f, g, faces=imp))
    b[pr.fixed] = 0.0
    uh = spla.spsolve(pr.B0.tocsc(), b)
    assert np.abs(uh[pr.fixed]).max() == 0.0
    e = uh - u(*fem.nodes(dim, n).T)
    return float(np.sqrt(np.real(np.vdot(e, pr.M @ e))))


def _rates(errs):
    return [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]


def test_mms_p1_opposite_dirichlet_faces():
    # u vanishes on x = 0 and x = 1; travelling wave in y with impedance data
    a, w = np.pi, 2.5
    u = lambda x, y: np.sin(a * x) * np.exp(1j * w * y)
    grad = lambda x, y: (a * np.cos(a * x) * np.exp(1j * w * y), 1j * w * u(x, y))
    lap = lambda x, y: -(a * a + w * w) * u(x, y)
    errs = [_mms(2, n, 4.0, 0.0, ("x0", "x1"), u, grad, lap) for n in (8, 16, 32, 64)]
    assert all(3.6 < r < 4.4 for r in _rates(errs)[1:]), errs


def test_mms_p1_adjacent_dirichlet_faces():
    # u vanishes on x = 0 and y = 0 (the corner node lies on both); impedance
    # on x = 1 and y = 1
    a, c = 2.0, 1.5
    u = lambda x, y: np.sin(a * x) * np.sin(c * y) * (1.0 + 0.5j)
    grad = lambda x, y: (a * np.cos(a * x) * np.sin(c * y) * (1.0 + 0.5j),
                         c * np.sin(a * x) * np.cos(c * y) * (1.0 + 0.5j))
    lap = lambda x, y: -(a * a + c * c) * u(x, y)
    errs = [_mms(2, n, 3.0, 0.5, ("x0", "y0"), u, grad, lap) for n in (8, 16, 32, 64)]
    assert all(3.6 < r < 4.4 for r in _rates(errs)[1:]), errs


def test_mms_q1_three_dirichlet_faces():
    # u vanishes on x = 0, y = 1 and z = 0; impedance on x = 1, y = 0, z = 1
    a, c, d = 1.5, 2.0, 1.0
    u = lambda x, y, z: np.sin(a * x) * np.sin(c * (1 - y)) * np.sin(d * z) + 0j
    grad = lambda x, y, z: (a * np.cos(a * x) * np.sin(c * (1 - y)) * np.sin(d * z),
                            -c * np.sin(a * x) * np.cos(c * (1 - y)) * np.sin(d * z),
                            d * np.sin(a * x) * np.sin(c * (1 - y)) * np.cos(d * z))
    lap = lambda x, y, z: -(a * a + c * c + d * d) * u(x, y, z)
    errs = [_mms(3, n, 2.0, 0.5, ("x0", "y1", "z0"), u, grad, lap) for n in (4, 8, 16)]
    assert all(3.4 < r < 4.6 for r in _rates(errs)), errs


@pytest.mark.parametrize("dim,n,faces,count", [
    (2, 6, ("x0",), 7), (2, 6, ("x0", "x1"), 14), (2, 6, ("x0", "y0"), 13),
    (2, 6, ("x0", "x1", "y0", "y1"), 24), (3, 4, ("z1",), 25), (3, 4, ("x0", "y0", "z0"), 61),
    (3, 4, ("x0", "x1", "y0", "y1", "z0", "z1"), 98)])
def test_face_node_counts(dim, n, faces, count):
    assert int(fem.dirichlet_node_mask(dim, n, faces).sum()) == count


@pytest.mark.parametrize("dim,n,faces", [(2, 8, ("x0", "y1")), (3, 4, ("x1", "z0"))])
def test_free_rows_equal_all_impedance_rows(dim, n, faces):
    """A face's boundary mass couples only nodes of that face, so on the
    nodes off the Dirichlet faces every operator equals the operator with
    the impedance term on every face."""
    k, dh = 5.0, 5.0
    pr = osolver.Problem(dim, n, k, dh, dirichlet=faces)
    full = osolver.Problem(dim, n, k, dh)
    free = ~pr.fixed
    for A, F in ((pr.B0, full.B0), (pr.Bdh, full.Bdh), (pr.L, full.L), (pr.N, full.N),
                 (pr.H, full.H)):
        D = (A[free][:, free] - F[free][:, free]).toarray()
        assert np.abs(D).max() < 1e-14
        # the Dirichlet rows and columns are the identity's
        assert np.abs((A[pr.fixed] - fem.eliminate(F, pr.fixed)[pr.fixed]).toarray()).max() == 0
        assert np.allclose(A[pr.fixed][:, pr.fixed].toarray(), np.eye(int(pr.fixed.sum())))
        assert abs(A[pr.fixed][:, free]).max() == 0 and abs(A[free][:, pr.fixed]).max() == 0


@pytest.mark.parametrize("dim,n,faces", [(2, 8, ("x0", "x1")), (2, 8, ("y1",)),
                                         (3, 4, ("x0", "y0", "z1"))])
def test_reduced_spaces_are_nested(dim, n, faces):
    """P maps coarse functions that vanish on the Dirichlet faces to fine
    functions that vanish there, and the Galerkin product of the reduced
    fine operator is the reduced coarse operator on the free nodes."""
    abc = ops.coefficients("L", 4.0, 4.0)
    hier = multigrid.Hierarchy(dim, n, 2, abc, dirichlet=faces)
    P = hier.levels[0].P
    ff = ~fem.dirichlet_node_mask(dim, n, faces)
    fc = ~fem.dirichlet_node_mask(dim, n // 2, faces)
    G = (P.T @ hier.levels[0].A @ P).toarray()
    Ac = hier.levels[1].A.toarray()
    assert np.abs(G[np.ix_(fc, fc)] - Ac[np.ix_(fc, fc)]).max() < 1e-13
    assert np.abs(G[~fc]).max() == 0 and np.abs(G[:, ~fc]).max() == 0
    # P restricted to the free nodes is the unreduced interpolation there
    Pfull = fem.prolongation(dim, n).toarray()
    assert np.abs(P.toarray()[np.ix_(ff, fc)] - Pfull[np.ix_(ff, fc)]).max() == 0


@pytest.mark.parametrize("dim,n,levels,faces", [(2, 32, 3, ("x0", "x1")), (2, 32, 3, ("x0", "y0")),
                                                (3, 8, 2, ("x0", "y0", "z0"))])
def test_vcycles_converge_to_direct_solve(dim, n, levels, faces):
    k = 3.0
    pr = osolver.Problem(dim, n, k, k, levels=levels, dirichlet=faces)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(pr.L.shape[0]) + 1j * rng.standard_normal(pr.L.shape[0])
    b[pr.fixed] = 0.0
    x = multigrid.cycles(pr.hierarchy, b, 40)
    ref = spla.spsolve(pr.L.tocsc(), b)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-10
    assert np.abs(multigrid.vcycle(pr.hierarchy, b)[pr.fixed]).max() == 0.0


@pytest.mark.parametrize("dim,n,faces", [(2, 16, ("x0", "x1", "y0", "y1")), (2, 16, ("y0",)),
                                         (3, 4, ("x1", "z0"))])
def test_hss_iteration_converges_to_shifted_solve(dim, n, faces):
    """With exact inner solves the HSS iteration converges to the solution
    of the shifted system (Sec. 3.1 and Sec. 4), Dirichlet faces included."""
    k = 4.0
    pr = osolver.Problem(dim, n, k, k, dirichlet=faces)
    rng = np.random.default_rng(9)
    R = rng.standard_normal(pr.L.shape[0]) + 1j * rng.standard_normal(pr.L.shape[0])
    R[pr.fixed] = 0.0
    z = pr.precond(R, inner="lu", steps=80)
    ref = spla.spsolve(pr.Bdh.tocsc(), R)
    assert np.linalg.norm(z - ref) / np.linalg.norm(ref) < 1e-9
    assert np.abs(z[pr.fixed]).max() == 0.0
