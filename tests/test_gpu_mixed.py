"""The mixed formulation ([DG0]^2 x P1, Sec. 2) on the GPU against the
oracle (`oracle.mixed`): the mixed operator and right-hand side, the
sigma-eliminated shifted-HSS preconditioner with multigrid (or exact,
one-level) inner solves, its per-step residual history, FGMRES and
Richardson solves whose u equals the primal discrete solution, and the
paper's measured outer rate for the mixed formulation at k = 16.
"""

import numpy as np
import pytest

from oracle import krylov, mixed, multigrid, solver as osolver
import workloads as W
from gpu_util import to_dev, to_host, rel_l2

pytestmark = pytest.mark.gpu


def _gpu(n, levels, k, dh, **kw):
    from paper_2506_18694_amd import Solver
    return Solver(2, n, levels, k, 0.0, dh, mixed=True, **kw)


def _lmix_solver(mp, levels, cycles):
    k, dh = mp.k, mp.delta_hat
    s = dh - 1j
    hier = multigrid.Hierarchy(2, mp.n, levels, (1.0, k * k * s * s, k * k * s))
    return lambda b: multigrid.cycles(hier, np.asarray(b, complex), cycles)


@pytest.mark.parametrize("n", [16, 24])
def test_mixed_operator_and_rhs_match_oracle(n):
    import torch
    mp = mixed.MixedProblem(n, 6.0, 2.0)
    s = _gpu(n, 2, 6.0, 2.0, restart=4)
    assert s.NV == mp.N + mp.E2
    X = W.random_complex((2, mp.N + mp.E2), 51)
    for op, A in (("MIXED", mp.A0), ("MIXED_SHIFT", mp.system(2.0))):
        y = to_host(s.apply(op, to_dev(X)))
        ref = np.stack([A @ x for x in X])
        assert rel_l2(y, ref) < 1e-13
    f = W.gaussian_nodal(2, n, (0.4, 0.5), 0.1)
    b = to_host(s.load_nodal(torch.from_numpy(f[None]).cuda()))[0]
    assert rel_l2(b, mp.rhs(mp.M @ f)) < 1e-13


@pytest.mark.parametrize("levels,cycles,prec,tol", [(1, 1, "fp64", 1e-11), (3, 2, "fp64", 1e-11),
                                                   (3, 2, "fp32", 2e-4)])
def test_mixed_preconditioner_matches_oracle(levels, cycles, prec, tol):
    n, k, dh = 32, 8.0, 2.0
    mp = mixed.MixedProblem(n, k, dh)
    solve = _lmix_solver(mp, levels, cycles)
    R = W.random_complex((2, mp.N + mp.E2), 52)
    s = _gpu(n, levels, k, dh, restart=4, mg_cycles=cycles, precision=prec)
    z = to_host(s.precondition(to_dev(R)))
    ref = np.stack([mp.precond(r, solve_lmix=solve) for r in R])
    assert rel_l2(z, ref) < tol


def test_mixed_hss_history_matches_oracle():
    n, k, dh = 32, 8.0, 2.0
    mp = mixed.MixedProblem(n, k, dh)
    solve = _lmix_solver(mp, 3, 2)
    R = W.random_complex(mp.N + mp.E2, 53)
    U = np.zeros_like(R)
    Bd = mp.system(dh)
    ref = [np.linalg.norm(R)]
    for _ in range(8):
        U = mp.hss_step_eliminated(U, R, solve)
        ref.append(np.linalg.norm(R - Bd @ U))
    z, res = _gpu(n, 3, k, dh, restart=4, mg_cycles=2).hss_history(to_dev(R[None]))
    assert np.abs(res[0] - np.array(ref)).max() < 1e-10 * ref[0]
    assert rel_l2(to_host(z)[0], U) < 1e-11


@pytest.mark.parametrize("outer,prec", [("fgmres", "fp64"), ("richardson", "fp64"),
                                        ("fgmres", "fp32")])
def test_mixed_solve_gives_the_primal_solution(outer, prec):
    import torch
    n, k, dh, levels = 64, 16.0, 2.0, 3
    mp = mixed.MixedProblem(n, k, dh)
    f = W.box_source(n)
    F = mp.rhs(mp.M @ f)
    solve = _lmix_solver(mp, levels, 2)
    P = lambda r: mp.precond(r, solve_lmix=solve)
    A = lambda v: mp.A0 @ v
    if outer == "fgmres":
        _, info = krylov.fgmres(A, F, P, tol=1e-10, restart=100, maxiter=100)
    else:
        _, info = krylov.richardson(A, F, P, tol=1e-10, maxiter=200)
    s = _gpu(n, levels, k, dh, mg_cycles=2, outer=outer, precision=prec)
    Fd = s.load_nodal(torch.from_numpy(f[None]).cuda())
    x, st = s.solve(Fd, tol=1e-10)
    x = to_host(x)[0]
    assert st["converged"] == 1
    slack = 1 if prec == "fp64" else 2
    assert abs(st["outer_its"] - info["its"]) <= slack, (st["outer_its"], info["its"])
    assert np.linalg.norm(F - mp.A0 @ x) <= 1e-10 * 1.01 * np.linalg.norm(F)
    u = osolver.Problem(2, n, k, dh).solve_direct(mp.M @ f)
    assert rel_l2(x[:mp.N], u) < 1e-6
    grad = (mp.G @ u) / mp.ms
    assert rel_l2(x[mp.N:], grad / (-1j * k)) < 1e-6


def test_paper_mixed_rate_at_k16():
    """The paper's mixed FGMRES rate with multigrid inner solves at k = 16
    (0.2806 / 0.2830 with direct / multigrid inner solves, uniform source),
    from the random guess's residual with the tolerance relative to it.  As
    in the paper, the mixed form needs a more accurate inner solve than the
    primal one: four V(2,2) cycles per HSS step."""
    n, k, dh = 64, 16.0, 2.0
    mp = mixed.MixedProblem(n, k, dh)
    r0 = mp.rhs(mp.M @ W.uniform_source(2, n)) - mp.A0 @ W.paper_initial_guess(mp.N + mp.E2, 3)
    _, st = _gpu(n, 3, k, dh, mg_cycles=4).solve(to_dev(r0[None]), tol=1e-6)
    assert st["converged"] == 1
    assert abs(st["outer_rate"] - 0.2806) < 0.01, st["outer_rate"]


@pytest.mark.parametrize("mixed_form,n,levels,k,steps", [(True, 32, 3, 8.0, 1500),
                                                         (False, 32, 2, 4.0, 4000)])
def test_long_hss_loop_graphs_equal_eager(mixed_form, n, levels, k, steps):
    """A preconditioner whose HSS loop launches more work than one captured
    graph holds (~20000 launches) is replayed as a head graph plus a body
    graph of a block of steps launched several times: the result equals the
    eager launches bit for bit."""
    from paper_2506_18694_amd import Solver
    outs = []
    for graphs in (True, False):
        s = Solver(2, n, levels, k, 0.0, 2.0, mixed=mixed_form, hss_steps=steps, mg_cycles=2,
                   restart=4, graphs=graphs)
        v = W.random_complex((2, s.NV), 54)
        outs.append(to_host(s.precondition(to_dev(v))))
        s.close()
    assert np.array_equal(outs[0], outs[1])


def test_mixed_columns_batch_equals_single_solves():
    """Mixed columns share every launch but not their arithmetic: a batch of
    three (one of them zero) equals the single-column solves."""
    import torch
    n, k, dh, levels = 32, 8.0, 2.0, 2
    s = _gpu(n, levels, k, dh, mg_cycles=2)
    f = np.stack([W.gaussian_nodal(2, n, c, 0.08) for c in ((0.3, 0.4), (0.6, 0.7))])
    F = s.load_nodal(torch.from_numpy(np.stack([f[0], np.zeros_like(f[0]), f[1]])).cuda())
    xb, st = s.solve(F, tol=1e-10)
    xb = to_host(xb)
    assert st["converged"] == 1
    assert np.abs(xb[1]).max() == 0.0
    for c in (0, 2):
        x1, _ = s.solve(F[c:c + 1].contiguous(), tol=1e-10)
        assert rel_l2(to_host(x1)[0], xb[c]) < 1e-12
