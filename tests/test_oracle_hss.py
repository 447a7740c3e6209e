"""Pins for the oracle's HSS operators, iteration and preconditioner
(Sec. 3.1 and Sec. 4).

  * the splitting identities: i B = H + i A_S, L - N = 2 A_S,
    L + N = -2ik H, (k+1) L - (k-1) N = 2k B  (so the fixed point is B u = R);
  * H is symmetric positive definite for delta > 0 and A_S is real
    symmetric, so S = H^{-1} i A_S is skew-adjoint in H and its Cayley
    transform is H-unitary;
  * with exact inner solves the H-norm error contracts by exactly
    (k-1)/(k+1) per step (the proposition's bound holds with equality
    because the Cayley transform is H-unitary); the paper's printed nu_s
    values are this formula (golden file);
  * the preconditioner equals (I - T^s) B^{-1} with T = (k-1)/(k+1) L^{-1} N;
  * k = 1 makes T = 0 so one step solves B u = R exactly (gamma = 1 is the
    "optimal" choice the paper mentions).
"""

import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem, operators as ops, hss

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mats(n=4, dim=2):
    return fem.assemble(dim, n)


@pytest.mark.parametrize("k,delta", [(3.0, 0.7), (10.0, 10.0), (7.3, 2.0), (1.0, 0.5)])
def test_splitting_identities(k, delta):
    K, M, MG = _mats(5)
    B = ops.b_delta(K, M, MG, k, delta).toarray()
    H = ops.h_gram(M, MG, k, delta).toarray()
    AS = ops.a_skew(K, M, MG, k, delta).toarray()
    L = ops.hss_lhs(K, M, MG, k, delta).toarray()
    N = ops.hss_rhs(K, M, MG, k, delta).toarray()
    assert np.abs(1j * B - (H + 1j * AS)).max() < 1e-12
    assert np.abs((L - N) - 2 * AS).max() < 1e-12
    assert np.abs((L + N) + 2j * k * H).max() < 1e-12
    assert np.abs((k + 1) * L - (k - 1) * N - 2 * k * B).max() < 1e-11
    assert np.isrealobj(AS) and np.abs(AS - AS.T).max() < 1e-14
    sla.cholesky(H)                                   # raises unless SPD
    # Cayley transform of S/k is H-unitary
    S = np.linalg.solve(H, 1j * AS)
    I = np.eye(S.shape[0])
    C = np.linalg.solve(k * I + S, k * I - S)
    assert np.abs(C.conj().T @ H @ C - H).max() < 1e-10 * np.abs(H).max()


def test_shift_reading_matches_squared_form():
    """eq. (primal-hss-system) has +delta^2 on the mass term; the remark
    after it prints -delta^2 (a sign slip).  Re-deriving from eq. (HSS) with
    gamma = k gives L = A_S - i k H, which the oracle's L matches."""
    K, M, MG = _mats(3)
    k, d = 5.0, 1.25
    AS = ops.a_skew(K, M, MG, k, d)
    H = ops.h_gram(M, MG, k, d)
    L = ops.hss_lhs(K, M, MG, k, d)
    assert abs(L - (AS - 1j * k * H)).max() < 1e-12
    a, b, c = ops.coefficients("L", k, d)
    assert a == 1 and abs(b - (d * d - k * k - 2j * d * k * k)) < 1e-12
    assert abs(c - (d - 1j * k * k)) < 1e-12


@pytest.mark.parametrize("k,delta", [(4.0, 0.8), (7.3, 7.3), (16.0, 2.0), (1.5, 3.0)])
def test_hss_contraction_is_exact(k, delta):
    n = 6
    K, M, MG = _mats(n)
    B = ops.b_delta(K, M, MG, k, delta).toarray()
    H = ops.h_gram(M, MG, k, delta).toarray()
    L = ops.hss_lhs(K, M, MG, k, delta).toarray()
    N = ops.hss_rhs(K, M, MG, k, delta).toarray()
    rng = np.random.default_rng(1)
    R = rng.standard_normal(B.shape[0]) + 1j * rng.standard_normal(B.shape[0])
    ustar = np.linalg.solve(B, R)
    hist = []
    hss.hss_literal(L, N, R, k, 12, lambda r: np.linalg.solve(L, r), hist)
    errs = [hss.h_norm(H, ustar)] + [hss.h_norm(H, u - ustar) for u in hist]
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    assert np.abs(ratios - hss.contraction_factor(k)).max() < 1e-9


def test_literal_and_correction_forms_agree():
    K, M, MG = _mats(7)
    k, d = 6.0, 6.0
    B = ops.b_delta(K, M, MG, k, d)
    L = ops.hss_lhs(K, M, MG, k, d).toarray()
    N = ops.hss_rhs(K, M, MG, k, d)
    R = np.random.default_rng(2).standard_normal(B.shape[0]) * (1 + 0.5j)
    solve = lambda r: np.linalg.solve(L, r)
    u1 = hss.hss_literal(L, N, R, k, 6, solve)
    u2 = hss.hss_correction(B, R, k, 6, solve)
    assert np.linalg.norm(u1 - u2) < 1e-12 * np.linalg.norm(u1)


@pytest.mark.parametrize("k,steps", [(5.0, 5), (2.5, 3), (9.0, 1)])
def test_preconditioner_closed_form(k, steps):
    K, M, MG = _mats(4)
    d = 1.5
    B = ops.b_delta(K, M, MG, k, d).toarray()
    L = ops.hss_lhs(K, M, MG, k, d).toarray()
    N = ops.hss_rhs(K, M, MG, k, d).toarray()
    T = (k - 1) / (k + 1) * np.linalg.solve(L, N)
    Pc = (np.eye(B.shape[0]) - np.linalg.matrix_power(T, steps)) @ np.linalg.inv(B)
    rng = np.random.default_rng(3)
    R = rng.standard_normal(B.shape[0]) + 1j * rng.standard_normal(B.shape[0])
    u = hss.hss_correction(B, R, k, steps, lambda r: np.linalg.solve(L, r))
    assert np.linalg.norm(u - Pc @ R) < 1e-11 * np.linalg.norm(u)


def test_k_equal_one_single_step_is_exact():
    K, M, MG = _mats(5)
    k, d = 1.0, 0.3
    B = ops.b_delta(K, M, MG, k, d).toarray()
    L = ops.hss_lhs(K, M, MG, k, d).toarray()
    N = ops.hss_rhs(K, M, MG, k, d).toarray()
    R = np.arange(B.shape[0]) * (1 - 2j)
    u = hss.hss_literal(L, N, R, k, 1, lambda r: np.linalg.solve(L, r))
    assert np.linalg.norm(B @ u - R) < 1e-12 * np.linalg.norm(R)


def test_inner_iteration_count():
    assert ops.inner_iterations(10.0) == 10
    assert ops.inner_iterations(12.8) == 13
    assert ops.inner_iterations(16.0, m=2) == 32


def test_paper_nu_s_values():
    """Every nu_s the paper prints equals (k-1)/(k+1) to its 4 digits, and
    exp(-m) bounds nu_s^(m ceil k) (the corollary after the proposition)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "nu_s.txt"), comments="#")
    for k, nu in rows:
        assert abs(round(hss.contraction_factor(k), 4) - nu) < 1e-12, (k, nu)
        for m in (1, 2):
            assert hss.contraction_factor(k) ** (m * np.ceil(k)) <= np.exp(-m)
