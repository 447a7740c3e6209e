"""Dirichlet faces on the GPU (helm_bc.dirichlet_faces): every step of the
hot path, the cycle, the preconditioner and the solve against the oracle's
eliminated operators (Dirichlet nodes removed from the unknowns, impedance
term on the other faces), 2D and 3D, FP64 and FP32 multigrid.

Inputs of the per-step calls are zero on the Dirichlet nodes (the calls'
contract); the solve and the preconditioner receive inputs that are not,
and must ignore those values.  Every output must be exactly zero there.
Tolerances as in the per-step parity tests (summation order and, in FP32,
a few ulps per pass).
"""

import numpy as np
import pytest

from oracle import fem, multigrid, operators as ops, solver as osolver
import workloads as W
from gpu_util import to_dev, to_host, rel_err, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5}
FACES = ("x0", "x1", "y0", "y1", "z0", "z1")


def _names(bits):
    return tuple(FACES[f] for f in range(6) if (bits >> f) & 1)


def _solver(dim, n, levels, k, dh, bits, precision="fp64", **kw):
    from paper_2506_18694_amd import Solver
    return Solver(dim, n, levels, k, 0.0, dh, precision=precision, dirichlet_faces=bits, **kw)


def _masked(N, nrhs, seed, prec, fixed):
    x = W.random_complex((nrhs, N), seed)
    if prec == "fp32":
        x = x.astype(np.complex64).astype(np.complex128)
    x[:, fixed] = 0.0
    return x


def _op(dim, n, op, k, dh, faces):
    """The oracle operator with the Dirichlet nodes of `faces` eliminated
    and the boundary term on the other faces."""
    imp = fem.impedance_faces(dim, faces)
    K, M, MG = fem.assemble(dim, n, imp)
    A = {"B0": lambda: ops.b_delta(K, M, MG, k, 0.0), "BSHIFT": lambda: ops.b_delta(K, M, MG, k, dh),
         "L": lambda: ops.hss_lhs(K, M, MG, k, dh), "N": lambda: ops.hss_rhs(K, M, MG, k, dh),
         "H": lambda: ops.h_gram(M, MG, k, dh).astype(np.complex128),
         "M": lambda: M.astype(np.complex128)}[op]().tocsr()
    return fem.eliminate(A, fem.dirichlet_node_mask(dim, n, faces))


CASES = [(2, 24, 3, 0b0011), (2, 33, 1, 0b0101), (2, 64, 3, 0b1111), (2, 64, 4, 0b1000),
         (3, 16, 3, 0b000011), (3, 7, 1, 0b010101), (3, 32, 3, 0b111111), (3, 24, 2, 0b100100)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim,n,levels,bits", CASES)
def test_operator_apply(dim, n, levels, bits, prec):
    k, dh = 7.5, 7.5
    faces = _names(bits)
    s = _solver(dim, n, levels, k, dh, bits, prec)
    dt = "complex128" if prec == "fp64" else "complex64"
    for l in range(levels):
        nl = n >> l
        fixed = fem.dirichlet_node_mask(dim, nl, faces)
        x = _masked(fixed.size, 2, 11 + l, prec, fixed)
        for op in ("B0", "BSHIFT", "L", "N", "H", "M"):
            if l > 0 and op in ("B0", "H", "M"):
                continue
            y = to_host(s.apply(op, to_dev(x, dt), level=l))
            A = _op(dim, nl, op, k, dh, faces)
            ref = np.stack([A @ xi for xi in x])
            assert rel_err(y, ref) < TOL[prec], (op, l)
            assert np.abs(y[:, fixed]).max() == 0.0, (op, l)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim,n,levels,bits", [c for c in CASES if c[2] > 1])
def test_transfer_smoother_and_coarse_steps(dim, n, levels, bits, prec):
    k, dh = 6.0, 6.0
    faces = _names(bits)
    dt = "complex128" if prec == "fp64" else "complex64"
    s = _solver(dim, n, levels, k, dh, bits, prec)
    hier = multigrid.Hierarchy(dim, n, levels, ops.coefficients("L", k, dh), dirichlet=faces)
    for l in range(levels):
        lev = hier.levels[l]
        fixed = fem.dirichlet_node_mask(dim, lev.n, faces)
        x = _masked(fixed.size, 2, 30 + l, prec, fixed)
        b = _masked(fixed.size, 2, 40 + l, prec, fixed)
        y = to_host(s.jacobi(to_dev(b, dt), to_dev(x, dt), level=l))
        ref = np.stack([multigrid.jacobi_sweep(lev, xi, bi, 2.0 / 3.0) for xi, bi in zip(x, b)])
        assert rel_err(y, ref) < TOL[prec], ("jacobi", l)
        y0 = to_host(s.jacobi(to_dev(b, dt), None, level=l))
        ref0 = np.stack([multigrid.jacobi_sweep(lev, np.zeros(fixed.size), bi, 2.0 / 3.0) for bi in b])
        assert rel_err(y0, ref0) < TOL[prec], ("jacobi0", l)
        assert np.abs(y[:, fixed]).max() == 0.0 and np.abs(y0[:, fixed]).max() == 0.0
        if l == levels - 1:
            xc = to_host(s.coarse_solve(to_dev(b, dt)))
            refc = np.linalg.solve(lev.A.toarray(), b.T).T
            assert rel_err(xc, refc) < (1e-11 if prec == "fp64" else 1e-5), "coarse"
            assert np.abs(xc[:, fixed]).max() == 0.0
            continue
        bc = to_host(s.restrict_residual(to_dev(x, dt), to_dev(b, dt), level=l))
        refc = np.stack([lev.P.T @ (bi - lev.A @ xi) for xi, bi in zip(x, b)])
        assert rel_err(bc, refc) < TOL[prec], ("restrict", l)
        cfix = fem.dirichlet_node_mask(dim, lev.n // 2, faces)
        assert np.abs(bc[:, cfix]).max() == 0.0
        e = _masked(cfix.size, 2, 50 + l, prec, cfix)
        xd = to_dev(x, dt)
        s.prolong_correct(to_dev(e, dt), xd, level=l)
        refp = np.stack([xi + lev.P @ ei for xi, ei in zip(x, e)])
        xp = to_host(xd)
        assert rel_err(xp, refp) < TOL[prec], ("prolong", l)
        assert np.abs(xp[:, fixed]).max() == 0.0
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hss_residual(prec):
    k, dh, n, bits = 12.0, 12.0, 40, 0b0110
    faces = _names(bits)
    dt = "complex128" if prec == "fp64" else "complex64"
    s = _solver(2, n, 1, k, dh, bits, prec)
    fixed = fem.dirichlet_node_mask(2, n, faces)
    R = _masked(fixed.size, 2, 3, prec, fixed)
    u = _masked(fixed.size, 2, 4, prec, fixed)
    B = _op(2, n, "BSHIFT", k, dh, faces)
    c = 2 * k / (k + 1)
    rho = to_host(s.hss_residual(to_dev(R, dt), to_dev(u, dt)))
    ref = np.stack([c * (Ri - B @ ui) for Ri, ui in zip(R, u)])
    assert rel_err(rho, ref) < TOL[prec]
    assert np.abs(rho[:, fixed]).max() == 0.0
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-4)])
@pytest.mark.parametrize("dim,n,levels,k,bits", [(2, 64, 3, 10.0, 0b0011), (2, 96, 4, 15.0, 0b1111),
                                                 (3, 16, 3, 4.0, 0b010101), (3, 32, 3, 6.0, 0b000011)])
def test_vcycle_matches_oracle(dim, n, levels, k, bits, prec, tol):
    faces = _names(bits)
    dt = "complex128" if prec == "fp64" else "complex64"
    s = _solver(dim, n, levels, k, k, bits, prec, restart=4)
    pr = osolver.Problem(dim, n, k, k, levels=levels, dirichlet=faces)
    b = _masked(s.nodes(0), 2, 21, prec, pr.fixed)
    x = to_host(s.vcycle(to_dev(b, dt)))
    ref = np.stack([pr.vcycle(bi) for bi in b])
    assert rel_l2(x, ref) < tol
    assert np.abs(x[:, pr.fixed]).max() == 0.0
    # the cycle without a workspace gives the same bits
    xn = to_host(s.vcycle_noalloc(to_dev(b, dt)))
    assert np.array_equal(xn, x)
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 5e-4)])
@pytest.mark.parametrize("dim,n,levels,k,cycles,bits", [
    (2, 64, 3, 10.0, 2, 0b0011), (2, 48, 2, 7.3, 3, 0b1001), (2, 96, 4, 12.0, 1, 0b1111),
    (3, 16, 3, 4.0, 2, 0b111111), (3, 8, 2, 3.0, 2, 0b000110)])
def test_preconditioner_matches_oracle(dim, n, levels, k, cycles, bits, prec, tol):
    faces = _names(bits)
    s = _solver(dim, n, levels, k, k, bits, prec, restart=4, mg_cycles=cycles)
    pr = osolver.Problem(dim, n, k, k, levels=levels, cycles=cycles, dirichlet=faces)
    v = W.random_complex((3, s.nodes(0)), 5)      # not zero on the Dirichlet nodes
    z = to_host(s.precondition(to_dev(v)))
    vm = v.copy()
    vm[:, pr.fixed] = 0.0
    ref = np.stack([pr.precond(vi, inner="mg") for vi in vm])
    assert rel_l2(z, ref) < tol
    assert np.abs(z[:, pr.fixed]).max() == 0.0
    # the diagnostic path computes the same preconditioner, and its first
    # entry is the norm of v without its Dirichlet-node values
    zh, res = s.hss_history(to_dev(v))
    assert rel_l2(to_host(zh), z) < (1e-13 if prec == "fp64" else 1e-6)
    assert np.abs(res[:, 0] / np.linalg.norm(vm, axis=1) - 1).max() < 1e-12
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("dim,n,levels,k,bits", [(2, 128, 5, 16.0, 0b0011), (2, 64, 4, 10.0, 0b1111),
                                                 (3, 32, 3, 6.0, 0b010101), (3, 16, 3, 4.0, 0b111111)])
def test_solve_matches_direct_solve(dim, n, levels, k, bits, precision):
    faces = _names(bits)
    s = _solver(dim, n, levels, k, k, bits, precision)
    pr = osolver.Problem(dim, n, k, k, dirichlet=faces)
    b = W.random_complex((2, s.nodes(0)), 31)     # not zero on the Dirichlet nodes
    x, st = s.solve(to_dev(b), tol=1e-10)
    assert st["status"] == 0, st
    xh = to_host(x)
    bm = b.copy()
    bm[:, pr.fixed] = 0.0
    ref = np.stack([pr.solve_direct(bi) for bi in bm])
    assert rel_l2(xh, ref) < 1e-7, (rel_l2(xh, ref), st)
    assert np.abs(xh[:, pr.fixed]).max() == 0.0
    s.close()


def test_richardson_outer_with_dirichlet_faces():
    """Preconditioned Richardson (x <- x + B~^{-1}(b - B_0 x)) with two
    Dirichlet faces: the iterate after a fixed number of iterations equals
    the oracle's (this case contracts slowly, about 0.98 per iteration, so
    the comparison is on the iterate, not on convergence)."""
    dim, n, levels, k, bits, its = 2, 64, 4, 6.0, 0b0101, 60
    faces = _names(bits)
    s = _solver(dim, n, levels, k, k, bits, outer="richardson", max_outer=its)
    pr = osolver.Problem(dim, n, k, k, levels=levels, dirichlet=faces)
    b = W.random_complex((1, s.nodes(0)), 41)
    b[:, pr.fixed] = 0.0
    x, st = s.solve(to_dev(b), tol=1e-12)
    ref, info = pr.solve(b[0], tol=1e-12, method="richardson", maxiter=its)
    assert info["its"] == its
    assert rel_l2(to_host(x)[0], ref) < 1e-9
    assert abs(st["true_rel_residual"] / info["true_rel_residual"] - 1) < 1e-6
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_3d_128_matches_masked_impedance_rows(prec, tol):
    """At 128^3 a handle with Dirichlet faces runs the column-tile kernel and
    the face mask, one with impedance on every face the fused z-marching
    passes (pinned to the oracle at full size).  On inputs that vanish on
    the Dirichlet nodes, the operator rows of the other nodes are the same
    (a face's boundary mass couples only that face's nodes; pinned in the
    oracle), so the applies and the Jacobi sweeps agree there, and the
    Dirichlet handle's outputs are exactly zero on the faces."""
    import torch
    n, levels, k, bits = 128, 5, 9.0, 0b010110
    faces = _names(bits)
    dt = "complex128" if prec == "fp64" else "complex64"
    sd = _solver(3, n, levels, k, k, bits, prec)
    si = _solver(3, n, levels, k, k, 0, prec)
    fixed = fem.dirichlet_node_mask(3, n, faces)
    free = torch.from_numpy(~fixed).cuda()
    x = to_dev(_masked(fixed.size, 2, 81, prec, fixed), dt)
    b = to_dev(_masked(fixed.size, 2, 82, prec, fixed), dt)
    pairs = [(sd.apply(op, x), si.apply(op, x)) for op in ("L", "B0", "BSHIFT")]
    pairs += [(sd.jacobi(b, x), si.jacobi(b, x)), (sd.jacobi(b, None), si.jacobi(b, None))]
    for yd, yi in pairs:
        a, r = to_host(yd), to_host(yi * free)
        assert rel_err(a, r) < tol
        assert np.abs(a[:, fixed]).max() == 0.0
    sd.close()
    si.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 5e-4)])
@pytest.mark.parametrize("dim,n,levels,k,bits", [(3, 24, 3, 4.0, 0b101001), (2, 96, 4, 9.0, 0b1001),
                                                 (2, 64, 3, 7.0, 0b0111)])
def test_fused_and_one_pass_paths_agree(dim, n, levels, k, bits, prec, tol):
    """Handles with Dirichlet faces run the fused passes (3D z-marching, 2D
    register streaming on the levels of at least 16 cells) with the faces
    cleared inside every stage; with the fused passes switched off they run
    one pass per launch and a mask after each.  Both compute the oracle's
    preconditioner, and the cycle of each matches the oracle's."""
    cycles = 2
    faces = _names(bits)
    pr = osolver.Problem(dim, n, k, k, levels=levels, cycles=cycles, dirichlet=faces)
    v = W.random_complex((2, (n + 1) ** dim), 23)
    vm = v.copy()
    vm[:, pr.fixed] = 0.0
    ref = np.stack([pr.precond(vi, inner="mg") for vi in vm])
    refc = np.stack([pr.vcycle(vi) for vi in vm])
    dt = "complex128" if prec == "fp64" else "complex64"
    bc = vm.astype(np.complex64).astype(np.complex128) if prec == "fp32" else vm
    for streaming in (True, False):
        s = _solver(dim, n, levels, k, k, bits, prec, restart=4, mg_cycles=cycles, streaming=streaming)
        z = to_host(s.precondition(to_dev(v)))
        assert rel_l2(z, ref) < tol, streaming
        assert np.abs(z[:, pr.fixed]).max() == 0.0
        x = to_host(s.vcycle(to_dev(bc, dt)))
        refx = np.stack([pr.vcycle(vi) for vi in bc]) if prec == "fp32" else refc
        assert rel_l2(x, refx) < (1e-12 if prec == "fp64" else 2e-4), streaming
        s.close()
