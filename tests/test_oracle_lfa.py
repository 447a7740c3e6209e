"""Pin of the oracle's multigrid contraction by local Fourier analysis.

For the interior 7-point P1 stencil of L (right-diagonal mesh: E, W, N, S,
NE, SW neighbours) the two-grid cycle V(2,2) with damped Jacobi (omega =
2/3), FE interpolation P, restriction P^T and the Galerkin coarse operator
acts on the four harmonics theta, theta + (pi, 0), theta + (0, pi),
theta + (pi, pi) of every low frequency theta as a 4 x 4 matrix

    M(theta) = S^2 (I - p (r L p)^{-1} r L) S^2,
    L = diag(L(theta^a)),  S = I - omega L / L_C,
    r = [r(theta^a)],  p = r^H,
    L(t) = w_C + 2 w_A (cos t1 + cos t2) + 2 w_D cos(t1 + t2),
    r(t) = 1 + cos t1 + cos t2 + cos(t1 + t2)

(the symbol of P^T: weight 1 at the node and 1/2 at its six neighbours), and
max_theta rho(M(theta)) is the two-grid contraction of an infinite mesh
(Trottenberg, Oosterlee and Schuller, Multigrid, ch. 4).  With every face
Dirichlet the oracle's mesh carries only that stencil, and its two-grid
error propagator (built from its own CSR operators) must contract at the
LFA rate up to the boundary's effect (a few per cent, the finite mesh
slightly faster).  A wrong damping, sweep count, transfer weight or coarse
operator moves the rate far outside that band.
"""

import numpy as np
import pytest

from oracle import fem, multigrid, operators as ops

FACES = ("x0", "x1", "y0", "y1")


def lfa_two_grid(wC, wA, wD, omega=2.0 / 3.0, nu1=2, nu2=2, m=48):
    def sym_L(t1, t2):
        return wC + 2.0 * wA * (np.cos(t1) + np.cos(t2)) + 2.0 * wD * np.cos(t1 + t2)

    def sym_r(t1, t2):
        return 1.0 + np.cos(t1) + np.cos(t2) + np.cos(t1 + t2)

    worst = 0.0
    ts = -np.pi / 2 + np.pi * (np.arange(m) + 0.5) / m   # low frequencies, avoiding 0
    for t1 in ts:
        for t2 in ts:
            ang = [(t1, t2), (t1 + np.pi, t2), (t1, t2 + np.pi), (t1 + np.pi, t2 + np.pi)]
            L = np.diag([sym_L(*a) for a in ang]).astype(complex)
            r = np.array([[sym_r(*a) for a in ang]], dtype=complex)
            p = r.conj().T
            K = np.eye(4) - p @ np.linalg.solve(r @ L @ p, r @ L)
            S = np.eye(4) - omega * L / wC
            M = np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)
            worst = max(worst, float(np.abs(np.linalg.eigvals(M)).max()))
    return worst


def interior_stencil(A, n):
    c = n // 2 + (n + 1) * (n // 2)
    wC, wE, wW = A[c, c], A[c, c + 1], A[c, c - 1]
    wN, wS = A[c, c + n + 1], A[c, c - n - 1]
    wNE, wSW = A[c, c + n + 2], A[c, c - n - 2]
    assert np.allclose([wW, wN, wS], wE) and np.isclose(wSW, wNE)
    assert abs(A[c, c + n]) == 0 and abs(A[c, c - n]) == 0          # no NW, SE coupling
    return wC, wE, wNE


def oracle_two_grid(n, k, omega=2.0 / 3.0):
    hier = multigrid.Hierarchy(2, n, 2, ops.coefficients("L", k, k), dirichlet=FACES)
    E = multigrid.error_propagator(hier, omega=omega)
    free = ~fem.dirichlet_node_mask(2, n, FACES)
    rho = float(np.abs(np.linalg.eigvals(E[np.ix_(free, free)])).max())
    return rho, interior_stencil(hier.levels[0].A.toarray(), n)


@pytest.mark.parametrize("k", [1.0, 3.0, 6.0])
def test_two_grid_rate_matches_lfa(k):
    rho, (wC, wA, wD) = oracle_two_grid(32, k)
    lfa = lfa_two_grid(wC, wA, wD)
    assert 0.2 < lfa < 0.3          # the textbook range of damped Jacobi V(2,2) for P1
    assert lfa - 0.015 < rho <= lfa * 1.005, (rho, lfa)


def test_lfa_separates_wrong_settings():
    """The band is narrow enough to catch a wrong damping or sweep count."""
    rho, (wC, wA, wD) = oracle_two_grid(32, 3.0)
    for bad in (lfa_two_grid(wC, wA, wD, omega=0.5), lfa_two_grid(wC, wA, wD, nu1=1, nu2=1)):
        assert abs(bad - rho) > 0.03, (bad, rho)
    rho_half, _ = oracle_two_grid(32, 3.0, omega=0.5)
    assert abs(rho_half - lfa_two_grid(wC, wA, wD, omega=0.5)) < 0.02


def lfa_two_grid_q1(wts, omega=2.0 / 3.0, nu1=2, nu2=2, m=16):
    """The same analysis for the 27-point Q1 stencil `wts` (offset -> weight)
    with trilinear interpolation: eight harmonics per low frequency, and the
    restriction symbol prod_j (1 + cos t_j) (weights 1/2, 1, 1/2 per axis)."""
    import itertools
    wC = wts[(0, 0, 0)]

    def sym_L(t):
        return sum(w * np.exp(1j * (d[0] * t[0] + d[1] * t[1] + d[2] * t[2])) for d, w in wts.items())

    def sym_r(t):
        return float(np.prod([1.0 + np.cos(x) for x in t]))

    worst = 0.0
    ts = -np.pi / 2 + np.pi * (np.arange(m) + 0.5) / m
    shifts = list(itertools.product((0, 1), repeat=3))
    for t in itertools.product(ts, ts, ts):
        ang = [tuple(t[j] + np.pi * a[j] for j in range(3)) for a in shifts]
        L = np.diag([sym_L(a) for a in ang]).astype(complex)
        r = np.array([[sym_r(a) for a in ang]], dtype=complex)
        p = r.conj().T
        K = np.eye(8) - p @ np.linalg.solve(r @ L @ p, r @ L)
        S = np.eye(8) - omega * L / wC
        M = np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)
        worst = max(worst, float(np.abs(np.linalg.eigvals(M)).max()))
    return worst


def test_q1_two_grid_rate_matches_lfa():
    """3D Q1, every face Dirichlet, 16^3: the oracle's two-grid rate is the
    LFA rate up to the boundary's effect (which shrinks as the mesh grows:
    0.157, 0.179, 0.187 at 8^3, 12^3, 16^3 against 0.195)."""
    import itertools
    faces3 = ("x0", "x1", "y0", "y1", "z0", "z1")
    n, k = 16, 3.0
    hier = multigrid.Hierarchy(3, n, 2, ops.coefficients("L", k, k), dirichlet=faces3)
    A = hier.levels[0].A.tocsr()
    n1 = n + 1
    c = n // 2 + n1 * (n // 2 + n1 * (n // 2))
    wts = {d: A[c, c + d[0] + n1 * (d[1] + n1 * d[2])] for d in itertools.product((-1, 0, 1), repeat=3)}
    E = multigrid.error_propagator(hier)
    free = ~fem.dirichlet_node_mask(3, n, faces3)
    rho = float(np.abs(np.linalg.eigvals(E[np.ix_(free, free)])).max())
    lfa = lfa_two_grid_q1(wts)
    assert 0.15 < lfa < 0.25
    assert lfa - 0.015 < rho <= lfa * 1.005, (rho, lfa)
