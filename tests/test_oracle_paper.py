"""Paper-level behaviour of the oracle at the paper's own settings
(Sec. 5.1-5.2): delta_hat = 2, uniform and box sources, c0 k^(3/2) cells
per direction, exact inner HSS solves, outer relative tolerance 1e-6.

The paper's absolute counts come from PETSc runs with a random initial
guess and PETSc's residual-norm conventions, which the paper does not fully
state; the oracle uses x0 = 0 and ||b - B_0 x|| <= tol ||b||.  Its counts
are about 1.5x the printed ones, so the pins here are the qualitative
claims the paper draws from its tables (Sec. 5.2), plus the measured HSS
residual rate against nu_s (Table "tab:hss-direct-rate"):
  * theta = 1: outer counts essentially independent of k;
  * theta = 1/2: counts grow with k; theta = 3/2: fewer than theta = 1;
  * FGMRES needs fewer iterations than Richardson;
  * uniform and box sources give (nearly) the same counts;
  * the measured HSS residual rate is within 2% of nu_s = (k-1)/(k+1).
"""

import numpy as np
import pytest

from oracle import solver, hss, krylov
import workloads as W


def _counts(k, n, source):
    pr = solver.Problem(2, n, k, 2.0, levels=1)
    f = W.uniform_source(2, n) if source == "uniform" else W.box_source(n)
    b = pr.M @ f
    out = {}
    for theta in (0.5, 1.0, 1.5):
        steps = int(np.ceil(k ** theta))
        P = lambda r: hss.hss_correction(pr.Bdh, r, k, steps, pr.solve_L)
        A = lambda x: pr.B0 @ x
        _, fi = krylov.fgmres(A, b, P, tol=1e-6, restart=400, maxiter=400)
        _, ri = krylov.richardson(A, b, P, tol=1e-6, maxiter=400)
        out[theta] = (fi["its"], ri["its"])
    return out


@pytest.fixture(scope="module")
def counts():
    return {(k, s): _counts(k, n, s)
            for (k, n) in ((8.0, 23), (16.0, 64)) for s in ("uniform", "box")}


def test_theta_one_is_k_robust(counts):
    f8, f16 = counts[(8.0, "uniform")][1.0][0], counts[(16.0, "uniform")][1.0][0]
    assert 6 <= f8 <= 16 and 6 <= f16 <= 16
    assert abs(f8 - f16) <= 3


def test_theta_ordering_and_growth(counts):
    for key, c in counts.items():
        assert c[1.5][0] <= c[1.0][0] < c[0.5][0], key
        assert c[1.5][1] <= c[1.0][1] < c[0.5][1], key
        for th in c:
            assert c[th][0] < c[th][1], (key, th)     # FGMRES beats Richardson
    assert counts[(16.0, "uniform")][0.5][0] > counts[(8.0, "uniform")][0.5][0] + 5


def test_uniform_and_box_agree(counts):
    for k in (8.0, 16.0):
        for th in (0.5, 1.0, 1.5):
            u, b = counts[(k, "uniform")][th], counts[(k, "box")][th]
            assert abs(u[0] - b[0]) <= max(2, 0.1 * u[0])


@pytest.mark.parametrize("source,paper_eta", [("uniform", 0.8789), ("box", 0.8789)])
def test_hss_rate_from_random_guess(source, paper_eta):
    """With the paper's random initial guess every frequency is present in
    the residual R = b - B_0 x_0 that the preconditioner first receives;
    the HSS residual then contracts at nu_s from the first step, and the
    measured rate matches the paper's table of HSS rates with direct inner
    solves (k = 16: nu_s = 0.8824, eta_s = 0.8789 for both sources)."""
    k, n = 16.0, 64
    pr = solver.Problem(2, n, k, 2.0, levels=1)
    f = W.uniform_source(2, n) if source == "uniform" else W.box_source(n)
    R = pr.M @ f - pr.B0 @ W.random_complex((pr.B0.shape[0],), 7)
    hist = []
    hss.hss_correction(pr.Bdh, R, k, 16, pr.solve_L, hist)
    res = np.array([np.linalg.norm(R)] + [np.linalg.norm(R - pr.Bdh @ u) for u in hist])
    eta_s = (res[-1] / res[0]) ** (1.0 / 16)
    assert abs(eta_s - hss.contraction_factor(k)) < 0.002
    assert abs(eta_s - paper_eta) < 0.005
    steps = res[1:] / res[:-1]
    assert np.all(np.abs(steps - hss.contraction_factor(k)) < 0.005)


def test_hss_residual_rate_near_nu_s():
    k, n = 16.0, 64
    pr = solver.Problem(2, n, k, 2.0, levels=1)
    R = pr.M @ W.uniform_source(2, n)
    hist = []
    hss.hss_correction(pr.Bdh, R, k, 16, pr.solve_L, hist)
    res = [np.linalg.norm(R)] + [np.linalg.norm(R - pr.Bdh @ u) for u in hist]
    eta_s = (res[-1] / res[0]) ** (1.0 / 16)
    assert abs(eta_s - hss.contraction_factor(k)) < 0.02


@pytest.mark.parametrize("source", ["uniform", "box"])
def test_outer_rate_matches_paper_table_from_random_guess(source):
    """The paper's setting with its random initial guess x_0 and the 1e-6
    tolerance read relative to the initial residual (run as B_0 e = r_0 from
    e = 0, which gives the same Krylov spaces): at k = 16 the measured FGMRES
    rate with exact inner solves is the paper's (table of FGMRES rates with
    direct inner solves: 0.2271 uniform, 0.2265 box), and the counts are
    within two of its 8 (29 at theta = 1/2, 6 at theta = 3/2)."""
    k, n = 16.0, 64
    pr = solver.Problem(2, n, k, 2.0, levels=1)
    f = W.uniform_source(2, n) if source == "uniform" else W.box_source(n)
    r0 = pr.M @ f - pr.B0 @ W.paper_initial_guess(pr.B0.shape[0], 3)
    A = lambda x: pr.B0 @ x
    its = {}
    for theta in (0.5, 1.0, 1.5):
        steps = int(np.ceil(k ** theta))
        P = lambda r, s=steps: hss.hss_correction(pr.Bdh, r, k, s, pr.solve_L)
        _, fi = krylov.fgmres(A, r0, P, tol=1e-6, restart=400, maxiter=400)
        its[theta] = fi["its"]
        if theta == 1.0:
            h = fi["history"]
            rate = (h[-1] / h[0]) ** (1.0 / fi["its"])
            assert abs(rate - (0.2271 if source == "uniform" else 0.2265)) < 0.005, rate
    assert 8 <= its[1.0] <= 10 and 6 <= its[1.5] <= 8 and 29 <= its[0.5] <= 40, its


@pytest.mark.parametrize("source,paper_rate", [("uniform", 0.4955), ("box", 0.4960)])
def test_richardson_rate_matches_paper_in_preconditioned_norm(source, paper_rate):
    """The paper's measured Richardson rate with exact inner solves at k = 16
    (its table of Richardson rates: 0.4955 uniform, 0.4960 box) is the mean
    contraction of the preconditioned residual |B~^{-1}(b - B_0 x_n)| from
    the paper's random initial guess until it falls below 1e-6 of its
    initial value: the norm a left-preconditioned Richardson iteration
    monitors.  The true-residual rate over the same iterations is well below
    it (about 0.40).
    The count under this norm is 20 here against the paper's 16 (a reading
    recorded, not pinned: no stopping reference reproduces both)."""
    k, n = 16.0, 64
    pr = solver.Problem(2, n, k, 2.0, levels=1)
    f = W.uniform_source(2, n) if source == "uniform" else W.box_source(n)
    b = pr.M @ f
    x = W.paper_initial_guess(pr.B0.shape[0], 3)
    P = lambda r: hss.hss_correction(pr.Bdh, r, k, int(np.ceil(k)), pr.solve_L)
    zs, rs = [], []
    for _ in range(40):
        r = b - pr.B0 @ x
        z = P(r)
        zs.append(np.linalg.norm(z))
        rs.append(np.linalg.norm(r))
        if zs[-1] <= 1e-6 * zs[0]:
            break
        x = x + z
    J = len(zs) - 1
    rate = (zs[-1] / zs[0]) ** (1.0 / J)
    assert abs(rate - paper_rate) < 0.01, rate
    assert 16 <= J <= 22, J
    true_rate = (rs[-1] / rs[0]) ** (1.0 / J)
    assert true_rate < rate - 0.05
