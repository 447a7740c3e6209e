"""The 3D Q1 workload at its full size (256^3 hexahedra, k = delta_hat = 40,
6 levels) against the oracle, in the launch configuration the benchmark
times (register-streaming / z-marching kernels, eager preconditioner with
the dominant kernel's launches bracketed by events).

A mesh of 257^3 nodes is too large for the oracle's assembly in a test, so
every step is checked on sampled nodes (the 8 corners, a node on edges and
faces, random nodes) whose rows are built one at a time from the oracle's
element and face matrices and its Q1 basis (tests/gpu_util.py; the row
builders are pinned against the assembled operators and prolongation on
small meshes in tests/test_oracle_fem.py):

  * the operator L of the HSS step (its Jacobi diagonal from the same rows),
  * one scaled-Jacobi sweep from a zero and from a nonzero guess,
  * the HSS residual c (R - B_shift u), with u = 0 and u nonzero,
  * the residual restriction P^T (b - L x) on sampled coarse nodes,
  * the prolongation and correction x + P e on sampled fine nodes,
  * the complete solve to 1e-8 in both precision modes, through the true
    residual of an FP64 handle's B_0 apply on the solution, whose sampled
    rows are themselves checked against the oracle on that solution.

Tolerances: FP64 1e-12 relative to the sampled reference's max-norm, FP32
2e-5 (a few FP32 ulps of sum |w| |x|), on inputs rounded to FP32 first.
"""

import numpy as np
import pytest

from oracle import operators as ops
import workloads as W
from gpu_util import (q1_prolong_row, q1_restrict_rows, q1_rows, q1_b0_rows, rel_err, row_apply,
                      row_diag, sample_nodes_3d, to_dev, to_host)

pytestmark = pytest.mark.gpu

NAME = "q1-256-k40"
DT = {"fp64": "complex128", "fp32": "complex64"}
TOL = {"fp64": 1e-12, "fp32": 2e-5}
OMEGA = 2.0 / 3.0


def _solver(prec, **kw):
    from paper_2506_18694_amd import Solver
    w = W.WORKLOADS[NAME]
    return Solver(3, w["n"], w["levels"], w["k"], w["delta"], w["delta_hat"], precision=prec,
                  profile=True, streaming=True, split=False, **kw)


def _rand(N, seed, prec):
    x = W.random_complex(N, seed)
    if prec == "fp32":
        x = x.astype(np.complex64).astype(np.complex128)
    return x


def _idx(n, pts):
    return np.array([i + (n + 1) * (j + (n + 1) * l) for (i, j, l) in pts])


@pytest.fixture(scope="module")
def sampled():
    w = W.WORKLOADS[NAME]
    n, k, dh = w["n"], w["k"], w["delta_hat"]
    pts = sample_nodes_3d(n, 300, 71)
    Lrows = q1_rows(n, ops.coefficients("L", k, dh), pts)
    return dict(n=n, k=k, dh=dh, pts=pts, t=_idx(n, pts), Lrows=Lrows,
                D=row_diag(Lrows, pts, n))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_3d_full_size_L_apply_sampled(sampled, prec):
    s = _solver(prec)
    x = _rand(s.N, 72, prec)
    y = to_host(s.apply("L", to_dev(x, DT[prec])))
    assert rel_err(y[sampled["t"]], row_apply(sampled["Lrows"], x)) < TOL[prec]
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("guess", [False, True])
def test_3d_full_size_jacobi_sampled(sampled, prec, guess):
    s = _solver(prec)
    b = _rand(s.N, 73, prec)
    x = _rand(s.N, 74, prec) if guess else None
    out = to_host(s.jacobi(to_dev(b, DT[prec]), x_in=to_dev(x, DT[prec]) if guess else None))
    t, D = sampled["t"], sampled["D"]
    if guess:
        ref = x[t] + OMEGA / D * (b[t] - row_apply(sampled["Lrows"], x))
    else:
        ref = OMEGA / D * b[t]
    assert rel_err(out[t], ref) < TOL[prec]
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("with_u", [False, True])
def test_3d_full_size_hss_residual_sampled(sampled, prec, with_u):
    s = _solver(prec)
    R = _rand(s.N, 75, prec)
    u = _rand(s.N, 76, prec) if with_u else None
    rho = to_host(s.hss_residual(to_dev(R, DT[prec]), to_dev(u, DT[prec]) if with_u else None))
    k, t = sampled["k"], sampled["t"]
    c = 2.0 * k / (k + 1.0)
    if with_u:
        Brows = q1_rows(sampled["n"], ops.coefficients("B", k, sampled["dh"]), sampled["pts"])
        ref = c * (R[t] - row_apply(Brows, u))
    else:
        ref = c * R[t]
    assert rel_err(rho[t], ref) < TOL[prec]
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_3d_full_size_restrict_residual_sampled(sampled, prec):
    n = sampled["n"]
    s = _solver(prec)
    x = _rand(s.N, 77, prec)
    b = _rand(s.N, 78, prec)
    bc = to_host(s.restrict_residual(to_dev(x, DT[prec]), to_dev(b, DT[prec])))
    cpts = sample_nodes_3d(n // 2, 120, 79)
    ref = []
    for fine, wts in q1_restrict_rows(n, cpts):
        Lf = q1_rows(n, ops.coefficients("L", sampled["k"], sampled["dh"]), fine)
        r = b[_idx(n, fine)] - row_apply(Lf, x)
        ref.append(wts @ r)
    assert rel_err(bc[_idx(n // 2, cpts)], np.array(ref)) < TOL[prec]
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_3d_full_size_prolong_correct_sampled(sampled, prec):
    n = sampled["n"]
    s = _solver(prec)
    x = _rand(s.N, 80, prec)
    e = _rand((n // 2 + 1) ** 3, 81, prec)
    out = to_host(s.prolong_correct(to_dev(e, DT[prec]), to_dev(x, DT[prec])))
    ref = []
    for p in sampled["pts"]:
        cols, wts = q1_prolong_row(n, p)
        ref.append(wts @ e[cols])
    t = sampled["t"]
    assert rel_err(out[t], x[t] + np.array(ref)) < TOL[prec]
    s.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_3d_full_size_solve(sampled, prec):
    """The 256^3 solve to 1e-8 (FP64, and FP32 multigrid with FP64 outer
    iteration): converged, with the true relative residual <= 1e-8 (1%
    slack for the recomputation) through an FP64 handle's B_0 apply."""
    import torch
    n, k = sampled["n"], sampled["k"]
    s = _solver(prec)
    f = torch.from_numpy(W.workload_sources(NAME)).cuda().contiguous()
    b = s.load_nodal(f)
    x, st = s.solve(b, tol=1e-8)
    assert st["converged"] and st["true_rel_residual"] <= 1e-8
    s64 = s if prec == "fp64" else _solver("fp64")
    y = to_host(s64.apply("B0", x))[0]
    bh, xh = to_host(b)[0], to_host(x)[0]
    assert np.linalg.norm(bh - y) / np.linalg.norm(bh) <= 1.01e-8
    # that apply against the oracle's rows on the solution itself
    rows = q1_b0_rows(n, k, sampled["pts"])
    assert rel_err(y[sampled["t"]], row_apply(rows, xh)) < 1e-10
    if s64 is not s:
        s64.close()
    s.close()
