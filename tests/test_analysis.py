"""Pins for the host analysis (App. A, B, C; Sec. IV.D): closed forms,
brute force, the paper's own piecewise formula and processes with known
autocorrelation."""
import math

import numpy as np
import pytest
from scipy import special

from paper_1510_04675_amd import analysis as an


def paper_g(n, nj, j, lag):
    """The piecewise degeneracy of App. B as printed, with m_1..m_5 the sorted
    {N_J, (j-1) N_J, j N_J, N - j N_J, N - (j-1) N_J}."""
    m = sorted([nj, (j - 1) * nj, j * nj, n - j * nj, n - (j - 1) * nj])
    if lag < m[0]:
        return n - nj - 2 * lag
    if lag < m[1]:
        return n - nj - m[0] - lag
    if lag < m[2]:
        return n - nj - m[0] - m[1]
    if lag < m[3]:
        return n - nj - m[0] - m[1] + m[2] - lag
    if lag < m[4]:
        return n - nj - m[0] - m[1] + m[2] - m[3]
    return n - lag


@pytest.mark.parametrize("n,nj", [(40, 8), (60, 10), (48, 16), (100, 10), (90, 30)])
def test_pair_count_matches_paper_formula(n, nj):
    """The degeneracy is the number of pairs with both members kept (brute
    force).  The printed piecewise form equals it for every block except one
    sitting exactly in the middle of the series ((j-1) N_J = N - j N_J), where
    the tied m's make it miscount; pairs are counted directly."""
    for j in range(1, n // nj + 1):
        lo, hi = (j - 1) * nj, j * nj
        for lag in range(0, n):
            brute = sum(1 for t in range(1, n - lag + 1) if not (lo < t <= hi or lo < t + lag <= hi))
            assert an.pair_count(n, nj, j, lag) == brute
            if (j - 1) * nj != n - j * nj:
                assert brute == paper_g(n, nj, j, lag), (n, nj, j, lag)


def test_autocovariance_estimator_is_the_definition():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(257)
    dx = x - x.mean()
    g = an.autocov_hat(dx, 40)
    brute = np.array([np.sum(dx[: x.size - d] * dx[d:]) / x.size for d in range(41)])
    assert np.max(np.abs(g - brute)) < 1e-13


def test_tau_int_of_ar1_process():
    """x_t = a x_{t-1} + sqrt(1 - a^2) eta_t has rho_Delta = a^Delta and
    tau_int = (1 + a) / (2 (1 - a))."""
    rng = np.random.default_rng(11)
    for a in (0.0, 0.5, 0.8):
        n = 1 << 15
        eta = rng.standard_normal(n)
        x = np.empty(n)
        x[0] = eta[0]
        for t in range(1, n):
            x[t] = a * x[t - 1] + math.sqrt(1 - a * a) * eta[t]
        tau, dtau, w = an.tau_int(x, nj=512, max_lag=200)
        exact = (1 + a) / (2 * (1 - a))
        assert abs(tau - exact) < 4 * dtau + 0.02, (a, tau, dtau, exact, w)
        assert 0.2 * exact * math.sqrt(2 * (2 * w + 1) / n) < dtau < 5 * exact * math.sqrt(2 * (2 * w + 1) / n) + 0.01
        rho, err, _ = an.autocorrelation(x, 512, 6)
        assert np.all(np.abs(rho - a ** np.arange(7)) < 5 * err + 1e-12)


def test_varpro_recovers_constrained_two_exponential_model():
    t = np.arange(0, 40, dtype=float)
    E = np.array([0.04, 0.35])
    z = np.array([[1.0, 0.5], [-1.0, 2.0]])  # constraint: z^0_0 + z^1_0 = 0
    phi = np.array([[1.0, 0.0, 1.0, 0.0]])
    y = z @ np.exp(-np.outer(E, t))
    sig = 0.01 * np.ones(y.size)
    cov = np.diag(sig**2)
    Ef, zf, c2 = an.varpro_fit(t, y, cov, [0.1, 0.5], phi)
    assert np.max(np.abs(Ef - E)) < 1e-6 and np.max(np.abs(zf - z)) < 1e-5 and c2 < 1e-8
    assert abs(zf[0, 0] + zf[1, 0]) < 1e-10
    rng = np.random.default_rng(5)
    chis = []
    for _ in range(20):
        yn = y + rng.normal(0, 0.01, y.shape)
        Ef, zf, c2 = an.varpro_fit(t, yn, cov, [0.1, 0.5], phi)
        assert abs(zf[0, 0] + zf[1, 0]) < 1e-9
        chis.append(c2)
    dof = y.size - (2 + 4 - 1)
    assert abs(np.mean(chis) - dof) < 5 * math.sqrt(2 * dof / 20)


def test_acceptance_fit_and_eps_q():
    om = 762.0
    dtau = 1.0 / np.array([24, 30, 37, 48, 64])
    acc = an.acceptance_model(dtau, om)
    fit, err, inv70 = an.fit_acceptance(dtau, acc, 10**8)
    assert abs(fit - om) < 1e-4 * om
    assert abs(special.erfc(0.5 * om / inv70**2) - 0.7) < 1e-9
    rng = np.random.default_rng(2)
    assert abs(an.eps_q(rng.uniform(0, 10, 200000)) - 1 / math.sqrt(12)) < 0.005
    assert an.eps_q([1.0, -2.0, 3.0]) == 0.0
