"""Pins for the oracle's multigrid cycle and outer Krylov iteration.

Multigrid: a one-level cycle is the coarse direct solve; the cycle is a
linear map whose error propagator equals the product of its factors
(smoother powers and the coarse-grid correction, composed recursively); on
the SPD limit k -> 0 of the shifted operator the V(2,2)-Jacobi contraction
lies in the textbook range; on the benchmark's shifted operator the
two-grid factor is small.
Krylov: with the identity preconditioner FGMRES is GMRES, so its residual
history must equal scipy's GMRES; it reaches the direct solution; and the
HSS-preconditioned FGMRES converges on the workload operators.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import multigrid, krylov, operators as ops, solver
import workloads as W


def _hier(dim, n, levels, k, dh):
    return multigrid.Hierarchy(dim, n, levels, ops.coefficients("L", k, dh))


def test_one_level_cycle_is_direct_solve():
    h = _hier(2, 8, 1, 5.0, 5.0)
    b = W.random_complex(81, 0)
    x = multigrid.vcycle(h, b)
    assert np.linalg.norm(h.levels[0].A @ x - b) < 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("dim,n,levels,k", [(2, 8, 2, 4.0), (2, 8, 3, 6.0), (3, 4, 2, 3.0)])
def test_cycle_error_propagator(dim, n, levels, k):
    h = _hier(dim, n, levels, k, k)
    A = h.levels[0].A.toarray()
    E = multigrid.error_propagator(h)
    Nn = A.shape[0]
    xtrue = W.random_complex(Nn, 5)
    x = multigrid.vcycle(h, A @ xtrue)
    assert np.linalg.norm((xtrue - x) - E @ xtrue) < 1e-10 * np.linalg.norm(xtrue)
    # q cycles as a stationary iteration propagate the error by E^q
    for q in (2, 3):
        xq = multigrid.cycles(h, A @ xtrue, q)
        Eq = np.linalg.matrix_power(E, q)
        assert np.linalg.norm((xtrue - xq) - Eq @ xtrue) < 1e-10 * np.linalg.norm(xtrue)
    # linearity
    b1, b2 = W.random_complex(Nn, 6), W.random_complex(Nn, 7)
    lhs = multigrid.vcycle(h, (2 - 1j) * b1 + b2)
    rhs = (2 - 1j) * multigrid.vcycle(h, b1) + multigrid.vcycle(h, b2)
    assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(lhs)


def test_spd_limit_textbook_contraction():
    """k -> 0 with delta_hat = 1: L = K + M + MG is SPD; V(2,2) with
    omega = 2/3 Jacobi contracts by a mesh-independent factor ~0.1-0.3."""
    rhos = []
    for n in (16, 32):
        h = multigrid.Hierarchy(2, n, 3, (1.0, 1.0, 1.0))
        E = multigrid.error_propagator(h)
        rhos.append(max(abs(np.linalg.eigvals(E))))
    assert all(0.03 < r < 0.4 for r in rhos), rhos
    assert abs(rhos[0] - rhos[1]) < 0.1


def test_shifted_operator_cycle_contracts():
    """On L with delta_hat = k (the benchmark setting) the cycle converges
    as a stationary iteration at a rate well below 1."""
    pr = solver.Problem(2, 64, 10.0, 10.0, levels=3)
    b = W.random_complex(pr.L.shape[0], 8)
    xs = pr.solve_L(b)
    x = np.zeros_like(b)
    errs = []
    for _ in range(4):
        x = x + pr.vcycle(b - pr.L @ x)
        errs.append(np.linalg.norm(x - xs) / np.linalg.norm(xs))
    rates = np.array(errs[1:]) / np.array(errs[:-1])
    assert rates.max() < 0.35, rates


def test_fgmres_identity_matches_scipy_gmres():
    rng = np.random.default_rng(0)
    n = 40
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) * 0.3 + 1j * rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = krylov.fgmres(lambda v: A @ v, b, lambda v: v, tol=1e-10, restart=n, maxiter=n)
    ref = []
    spla.gmres(sp.csr_matrix(A), b, rtol=1e-10, restart=n, maxiter=1,
               callback=lambda r: ref.append(r), callback_type="pr_norm")
    ours = info["history"][1:]
    m = min(len(ours), len(ref))
    assert m >= 5
    np.testing.assert_allclose(ours[:m], ref[:m], rtol=1e-7, atol=1e-14)
    assert np.linalg.norm(A @ x - b) <= 1.01e-10 * np.linalg.norm(b)


def test_fgmres_reaches_direct_solution_with_restart():
    rng = np.random.default_rng(1)
    n = 60
    A = np.diag(np.linspace(1, 4, n)).astype(complex) + 0.2j * rng.standard_normal((n, n))
    b = rng.standard_normal(n).astype(complex)
    x, info = krylov.fgmres(lambda v: A @ v, b, lambda v: v, tol=1e-12, restart=7, maxiter=400)
    assert info["converged"]
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-10 * np.linalg.norm(x)


def test_richardson_exact_preconditioner_one_step():
    rng = np.random.default_rng(2)
    A = np.eye(8) + 0.1 * rng.standard_normal((8, 8))
    b = rng.standard_normal(8).astype(complex)
    x, info = krylov.richardson(lambda v: A @ v, b, lambda r: np.linalg.solve(A, r), tol=1e-12)
    assert info["its"] == 1


def test_small_workload_solve_matches_direct():
    """The 64 x 64, k = 10 workload: FGMRES + shifted HSS + V(2,2) reaches
    the unique discrete solution (u = B_0^{-1} b)."""
    w = W.WORKLOADS["p1-64-k10"]
    pr = solver.Problem(2, w["n"], w["k"], w["delta_hat"], levels=w["levels"])
    b = solver.load_from_nodal(pr.M, W.workload_sources("p1-64-k10")[0])
    x, info = pr.solve(b, tol=1e-10, inner="mg")
    u = pr.solve_direct(b)
    assert info["converged"] and info["true_rel_residual"] < 1e-10
    assert np.linalg.norm(x - u) / np.linalg.norm(u) < 1e-8
    assert 15 <= info["its"] <= 40


# ---- the paper's multigrid variant: W-cycle, GMRES-Jacobi smoothing --------

def test_gmres_jacobi_is_the_minimal_residual_vector():
    """GMRES_m from x returns the vector of x + K_m minimising the Jacobi-
    preconditioned residual, K_m = span{r, Mr, ..., M^{m-1} r} with
    M = D^{-1}A and r = D^{-1}(b - A x): checked against the least-squares
    problem over the monomial Krylov basis, solved directly."""
    lev = _hier(2, 4, 1, 3.0, 3.0).levels[0]
    A, D = lev.A.toarray(), lev.D
    b = W.random_complex(A.shape[0], 31)
    x0 = W.random_complex(A.shape[0], 32)
    for m in (1, 2, 4):
        x = multigrid.gmres_jacobi(lev, x0, b, m)
        Mop = A / D[:, None]
        r = (b - A @ x0) / D
        K = np.stack([np.linalg.matrix_power(Mop, i) @ r for i in range(m)], axis=1)
        c = np.linalg.lstsq(Mop @ K, r, rcond=None)[0]
        xb = x0 + K @ c
        assert np.linalg.norm(x - xb) <= 1e-9 * np.linalg.norm(xb)


def test_gmres_jacobi_full_space_is_exact():
    """With as many iterations as unknowns (or an invariant Krylov space,
    detected as breakdown) GMRES returns A^{-1} b."""
    lev = _hier(2, 3, 1, 2.0, 2.0).levels[0]
    b = W.random_complex(lev.A.shape[0], 33)
    x = multigrid.gmres_jacobi(lev, np.zeros_like(b), b, lev.A.shape[0] + 3)
    xe = np.linalg.solve(lev.A.toarray(), b)
    assert np.linalg.norm(x - xe) <= 1e-9 * np.linalg.norm(xe)
    # a zero residual returns the iterate unchanged
    assert np.array_equal(multigrid.gmres_jacobi(lev, xe, lev.A @ xe, 5), xe)


def test_two_level_wcycle_with_exact_coarse_level_is_two_grid():
    """On two levels with a coarsest level small enough for GMRES to solve
    exactly, the W-cycle is the two-grid cycle: smoothing, exact coarse
    correction (the second coarse visit starts from the exact solution and
    leaves it), smoothing."""
    hier = _hier(2, 6, 2, 3.0, 3.0)
    f, c = hier.levels
    its = c.A.shape[0] + 2
    b = W.random_complex(f.A.shape[0], 34)
    x0 = W.random_complex(f.A.shape[0], 35)
    x = multigrid.wcycle(hier, b, x0, 0, its)
    y = multigrid.gmres_jacobi(f, x0, b, its)
    ec = np.linalg.solve(c.A.toarray(), f.P.T @ (b - f.A @ y))
    y = multigrid.gmres_jacobi(f, y + f.P @ ec, b, its)
    assert np.linalg.norm(x - y) <= 1e-9 * np.linalg.norm(y)


def test_wcycle_visits_each_level_twice_as_often_as_the_one_above(monkeypatch):
    calls = {}
    orig = multigrid.gmres_jacobi

    def counting(level, x, b, its):
        calls[level.n] = calls.get(level.n, 0) + 1
        return orig(level, x, b, its)

    monkeypatch.setattr(multigrid, "gmres_jacobi", counting)
    hier = _hier(2, 16, 4, 2.0, 2.0)
    multigrid.wcycle(hier, W.random_complex(17 * 17, 36), np.zeros(17 * 17, complex), 0, 2)
    # levels 16, 8, 4 smooth twice per visit (visits 1, 2, 4); the coarsest
    # (2 cells) is visited 8 times, one GMRES application each
    assert calls == {16: 2, 8: 4, 4: 8, 2: 8}


def test_paper_wcycle_contracts_strongly():
    """The paper's cycle (4 levels, GMRES(5)-Jacobi on every level) on the
    shifted operator at its k = 16 setting: one cycle reduces the residual
    of a random right-hand side by more than 100 (the paper's measured
    multigrid rates at k = 64..1024 are 0.0034 to 0.0006)."""
    pr = solver.Problem(2, 64, 16.0, 2.0, levels=4, cycles=1, cycle="w")
    b = W.random_complex(pr.L.shape[0], 37)
    x = pr.mg_solve(b)
    assert np.linalg.norm(b - pr.L @ x) < 0.01 * np.linalg.norm(b)


@pytest.mark.parametrize("n1", [1, 2, 7, 13, 21, 64])
def test_nested_dissection_is_a_permutation(n1):
    p = solver.nested_dissection_2d(n1)
    assert np.array_equal(np.sort(p), np.arange(n1 * n1))


def test_nested_dissection_first_split_decouples_the_halves():
    """The two halves ordered before the first separator line share no
    nonzero of B_0 (so the split is a true vertex separator of the P1 mesh)."""
    n = 20
    w = solver.Problem(2, n, 5.0, 5.0)
    n1 = n + 1
    m = n1 // 2                                      # first split: i = m
    I = np.arange(n1 * n1) % n1
    left, right = np.flatnonzero(I < m), np.flatnonzero(I > m)
    assert abs(w.B0[left][:, right]).max() == 0
    assert abs(w.B0[left][:, I == m]).max() > 0


@pytest.mark.parametrize("n,k", [(7, 3.0), (12, 6.0), (20, 9.0)])
def test_direct_solve_in_nested_dissection_order_is_the_dense_solve(n, k):
    """u = B_0^{-1} b through the reordered sparse LU equals numpy's dense
    LU of the assembled matrix in the original node order."""
    pr = solver.Problem(2, n, k, k)
    rng = np.random.default_rng(n)
    b = rng.standard_normal(pr.B0.shape[0]) + 1j * rng.standard_normal(pr.B0.shape[0])
    u = pr.solve_direct(b)
    ud = np.linalg.solve(pr.B0.toarray(), b)
    assert np.linalg.norm(u - ud) <= 1e-12 * np.linalg.norm(ud)
