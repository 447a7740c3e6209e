"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (all right-hand sides in one batch on one stream, the
preconditioner run eagerly with the dominant kernel's launches bracketed
by events, register-streaming kernels on every level down to the
LDS-resident small levels).

2D P1 1024 x 1024, k = delta_hat = 100, 8 levels, four right-hand sides:
every output of the operator apply, of one V-cycle and of two shifted-HSS
steps is compared with the oracle element by element; the full solve to
1e-8 is checked through its true residual, recomputed with the oracle's
assembled B_0, and through its error against the oracle's sparse direct
solution (1e-6 FP64, 1e-5 FP32 multigrid); the FP32-multigrid
preconditioner is shown to compute in FP32.  3D Q1 256^3, k = 40: the
operator apply on sampled nodes (corners, edges, faces and random interior
nodes), the rows built from the oracle's element matrices (the other 3D
steps and the 3D solve: test_gpu_full_size_3d.py).  2D P1 2048 x 2048, k = 200 (too large
for the oracle's assembly in a test): the B_0 apply on sampled rows, and
the FP32-multigrid solve through the residual of the library's B_0 apply,
whose sampled rows are checked against the oracle on the solution itself.
Tolerances as in the per-step tests.
"""

import numpy as np
import pytest

from oracle import solver as osolver
import workloads as W
from gpu_util import (p1_b0_rows, q1_b0_rows, rel_err, rel_l2, sample_nodes_2d, sample_nodes_3d,
                      to_dev, to_host)

pytestmark = pytest.mark.gpu

HEAD = "p1-1024-k100"
DT = {"fp64": "complex128", "fp32": "complex64"}


def _bench_solver(name, prec, **kw):
    """A solver with the options the benchmark's timed solves use."""
    from paper_2506_18694_amd import Solver
    w = W.WORKLOADS[name]
    return Solver(w["dim"], w["n"], w["levels"], w["k"], w["delta"], w["delta_hat"],
                  precision=prec, profile=True, streaming=True, split=False, **kw)


@pytest.fixture(scope="module")
def head():
    w = W.WORKLOADS[HEAD]
    pr = osolver.Problem(2, w["n"], w["k"], w["delta_hat"], levels=w["levels"], cycles=3)
    _ = pr.hierarchy
    return w, pr


def _inputs(N, nrhs, seed, prec):
    x = W.random_complex((nrhs, N), seed)
    if prec == "fp32":
        x = x.astype(np.complex64).astype(np.complex128)
    return x


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_headline_operator_apply(head, prec, tol):
    w, pr = head
    s = _bench_solver(HEAD, prec)
    x = _inputs(s.N, w["nrhs"], 41, prec)
    for op, A in (("B0", pr.B0), ("L", pr.L)):
        y = to_host(s.apply(op, to_dev(x, DT[prec])))
        ref = np.stack([A @ xi for xi in x])
        assert rel_err(y, ref) < tol, op
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-4)])
def test_headline_vcycle(head, prec, tol):
    w, pr = head
    s = _bench_solver(HEAD, prec, mg_cycles=3)
    b = _inputs(s.N, w["nrhs"], 43, prec)
    x = to_host(s.vcycle(to_dev(b, DT[prec])))
    for xi, bi in zip(x, b):
        assert rel_l2(xi, pr.vcycle(bi)) < tol
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 5e-4)])
def test_headline_two_hss_steps(head, prec, tol):
    """Two HSS steps with three V-cycles each: the step whose residual is
    c R (u = 0) and one with the residual of a nonzero iterate."""
    w, pr = head
    s = _bench_solver(HEAD, prec, mg_cycles=3, hss_steps=2)
    v = W.random_complex((w["nrhs"], s.N), 45)
    z = to_host(s.precondition(to_dev(v)))
    for zi, vi in zip(z, v):
        assert rel_l2(zi, pr.precond(vi, inner="mg", steps=2)) < tol
    s.close()


@pytest.fixture(scope="module")
def head_direct(head):
    """The oracle's sparse direct solutions u = B_0^{-1} b of the four
    right-hand sides (about a minute of one core)."""
    w, pr = head
    return np.stack([pr.solve_direct((pr.M @ fi).astype(np.complex128))
                     for fi in W.workload_sources(HEAD)])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,err_tol", [("fp64", 1e-6), ("fp32", 1e-5)])
def test_headline_solve_true_residual(head, head_direct, prec, err_tol):
    """The 1e-8 solve: converged, true residual with the oracle's CSR B_0,
    and each column's relative l2 error against the oracle's direct
    solution (1e-6 for the FP64 path, 1e-5 for FP32 multigrid)."""
    import torch
    w, pr = head
    s = _bench_solver(HEAD, prec)
    f = torch.from_numpy(W.workload_sources(HEAD)).cuda().contiguous()
    b = s.load_nodal(f)
    x, st = s.solve(b, tol=1e-8)
    assert st["converged"]
    bh, xh = to_host(b), to_host(x)
    errs = []
    for bi, xi, ui in zip(bh, xh, head_direct):
        assert np.linalg.norm(bi - pr.B0 @ xi) / np.linalg.norm(bi) <= 1.01e-8
        errs.append(rel_l2(xi, ui))
    print("%s %s rel l2 error vs oracle direct per column: %s"
          % (HEAD, prec, " ".join("%.3e" % e for e in errs)))
    assert max(errs) <= err_tol
    # the load vector itself against the oracle's mass matrix
    fh = W.workload_sources(HEAD)
    assert rel_err(bh, np.stack([pr.M @ fi for fi in fh])) < 1e-12
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_3d_full_size_apply_sampled(prec, tol):
    name = "q1-256-k40"
    w = W.WORKLOADS[name]
    s = _bench_solver(name, prec)
    n, k = w["n"], w["k"]
    x = _inputs(s.N, 1, 47, prec)
    y = to_host(s.apply("B0", to_dev(x, DT[prec])))[0]
    pts = sample_nodes_3d(n, 400, 48)
    rows = q1_b0_rows(n, k, pts)
    ref = np.array([vals @ x[0][cols] for cols, vals in rows])
    got = np.array([y[i + (n + 1) * (j + (n + 1) * l)] for (i, j, l) in pts])
    assert rel_err(got, ref) < tol
    s.close()


def _sampled_2d(n, k, v, y, seed):
    pts = sample_nodes_2d(n, 400, seed)
    rows = p1_b0_rows(n, k, pts)
    ref = np.array([vals @ v[cols] for cols, vals in rows])
    got = np.array([y[i + (n + 1) * j] for (i, j) in pts])
    return rel_err(got, ref)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_2048_apply_sampled(prec, tol):
    name = "p1-2048-k200"
    w = W.WORKLOADS[name]
    s = _bench_solver(name, prec)
    x = _inputs(s.N, 1, 49, prec)
    y = to_host(s.apply("B0", to_dev(x, DT[prec])))[0]
    assert _sampled_2d(w["n"], w["k"], x[0], y, 50) < tol
    s.close()


@pytest.mark.timeout(900)
def test_2048_fp32_solve_residual():
    """The 2048^2, k = 200 solve with FP32 multigrid: converged to 1e-8, the
    true residual through the FP64 apply, sampled rows of that apply against
    the oracle's element matrices, and the relative l2 error against the
    oracle's FP64 sparse direct solution (<= 1e-5; printed)."""
    import torch
    name = "p1-2048-k200"
    w = W.WORKLOADS[name]
    s = _bench_solver(name, "fp32")
    f = torch.from_numpy(W.workload_sources(name)).cuda().contiguous()
    b = s.load_nodal(f)
    x, st = s.solve(b, tol=1e-8)
    assert st["converged"]
    # the residual through the FP64 apply of an FP64 handle on the same mesh
    s64 = _bench_solver(name, "fp64")
    y = to_host(s64.apply("B0", x))[0]
    bh, xh = to_host(b)[0], to_host(x)[0]
    assert np.linalg.norm(bh - y) / np.linalg.norm(bh) <= 1.01e-8
    # B_0 x ~ b is about 1e3 times smaller than sum |w_ij x_j| here, so the
    # summation-order difference is relatively larger than on random input
    assert _sampled_2d(w["n"], w["k"], xh, y, 51) < 1e-10
    s.close()
    s64.close()
    del b, x, y, f
    torch.cuda.empty_cache()
    # the oracle's direct solve (nested-dissection sparse LU, ~1-2 min)
    pr = osolver.Problem(2, w["n"], w["k"], w["delta_hat"], levels=1)
    fh = W.workload_sources(name)[0]
    assert rel_l2(bh, pr.M @ fh) < 1e-12
    u = pr.solve_direct(pr.M @ fh.astype(np.complex128))
    assert np.linalg.norm(pr.M @ fh - pr.B0 @ u) <= 1e-10 * np.linalg.norm(pr.M @ fh)
    err = rel_l2(xh, u)
    print("p1-2048-k200 fp32-mg rel l2 error vs oracle direct: %.3e" % err)
    assert err <= 1e-5


def test_headline_fp32_mg_runs_in_fp32(head):
    """The FP32-multigrid preconditioner really computes in FP32: on the same
    input its output differs from the FP64 preconditioner's by FP32 rounding
    (far above FP64 round-off, far below the method's own error), and every
    value it returns is an FP32 number (the directions are stored in FP32
    and promoted exactly)."""
    import torch
    w, pr = head
    v = to_dev(W.random_complex((w["nrhs"], (w["n"] + 1) ** 2), 53))
    z = {}
    for prec in ("fp64", "fp32"):
        s = _bench_solver(HEAD, prec, mg_cycles=3)
        z[prec] = s.precondition(v)
        torch.cuda.synchronize()
        s.close()
    d = float(torch.linalg.vector_norm(z["fp32"] - z["fp64"]) / torch.linalg.vector_norm(z["fp64"]))
    assert 1e-9 < d < 1e-3, d
    z32 = z["fp32"]
    assert torch.equal(z32.to(torch.complex64).to(torch.complex128), z32)
    assert not torch.equal(z["fp64"].to(torch.complex64).to(torch.complex128), z["fp64"])
