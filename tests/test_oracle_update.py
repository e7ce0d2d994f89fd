"""Oracle pins for the Cabibbo-Marinari heat bath, the SU(2) samplers,
overrelaxation and the checkerboard schedule (Sec. IV.A)."""
import numpy as np
import pytest
from scipy import integrate, optimize, stats

import synth_inputs as si


def _g0_bins(alpha, nbins):
    dens = lambda x: np.sqrt(max(0.0, 1 - x * x)) * np.exp(alpha * (x - 1))
    tot = integrate.quad(dens, -1, 1, points=[1 - 1 / alpha] if alpha > 1 else None, limit=200)[0]
    cdf = lambda x: integrate.quad(dens, -1, x, limit=200)[0] / tot
    edges = [-1.0]
    for k in range(1, nbins):
        edges.append(optimize.brentq(lambda x: cdf(x) - k / nbins, -1, 1, xtol=1e-13))
    edges.append(1.0)
    return np.array(edges)


@pytest.mark.parametrize("sampler", [0, 1])
@pytest.mark.parametrize("alpha", [0.3, 1.0, 4.0, 12.0, 30.0])
def test_su2_sampler_distribution(orc, alpha, sampler):
    """g0 has density proportional to sqrt(1-g0^2) exp(alpha g0) on [-1,1]
    (the SU(2) heat-bath law), checked by chi^2 on equal-probability bins."""
    n, nb = 200_000, 40
    g, fails = orc.sample_g0(alpha, n, seed=1000 + int(alpha * 10), sampler=sampler, max_tries=4096)
    assert fails == 0
    edges = _g0_bins(alpha, nb)
    cnt, _ = np.histogram(g, bins=edges)
    chi2 = np.sum((cnt - n / nb) ** 2 / (n / nb))
    assert stats.chi2.sf(chi2, nb - 1) > 1e-3, chi2


def test_kp_acceptance_and_exhaustion(orc):
    """With one trial the KP sampler reports exhausted draws at a rate equal
    to 1 - acceptance, where acceptance = (integral of the target) /
    (integral of the Gamma(3/2) proposal) is computed by quadrature."""
    alpha = 1.0
    n = 100_000
    g, fails = orc.sample_g0(alpha, n, seed=5, sampler=0, max_tries=1)
    target = integrate.quad(lambda d: np.sqrt(d * (2 - d)) * np.exp(-alpha * d), 0, 2)[0]
    proposal = integrate.quad(lambda d: np.sqrt(2 * d) * np.exp(-alpha * d), 0, np.inf)[0]
    acc = target / proposal
    assert abs((n - fails) / n - acc) < 5 * np.sqrt(acc * (1 - acc) / n)
    assert np.all(np.isnan(g) | ((g >= -1) & (g <= 1)))


@pytest.mark.parametrize("alpha", [1.0, 4.0, 30.0])
def test_creutz_acceptance_and_exhaustion(orc, alpha):
    """Creutz's sampler proposes g0 from exp(alpha g0) on [-1, 1] and accepts
    with probability sqrt(1 - g0^2): with one trial the exhausted draws occur
    at 1 - acceptance, acceptance = (integral of sqrt(1-x^2) e^{alpha x}) /
    (integral of e^{alpha x}) by quadrature (0.76, 0.56 and 0.23 here)."""
    n = 100_000
    g, fails = orc.sample_g0(alpha, n, seed=11, sampler=1, max_tries=1)
    target = integrate.quad(lambda x: np.sqrt(1 - x * x) * np.exp(alpha * (x - 1)), -1, 1, limit=200)[0]
    proposal = integrate.quad(lambda x: np.exp(alpha * (x - 1)), -1, 1, limit=200)[0]
    acc = target / proposal
    assert abs((n - fails) / n - acc) < 5 * np.sqrt(acc * (1 - acc) / n), ((n - fails) / n, acc)
    assert np.all(np.isnan(g) | ((g >= -1) & (g <= 1)))


def test_or_conserves_action_and_is_reversible(orc):
    """Each OR pass leaves the Wilson action unchanged (links of one phase
    share no plaquette, and each subgroup reflection keeps Re Tr(U A)); the
    reversed pass undoes it."""
    d = [4, 4, 4, 4]
    U = orc.init_hot(d, 2, 0)
    orc.sweep_hb_or(d, U, 6.0, 2, 0, 0, 3, n_or=0)
    s0 = orc.action(d, U, 6.0)
    U0 = U.copy()
    orc.or_pass(d, U)
    assert abs(orc.action(d, U, 6.0) - s0) < 1e-12 * s0
    assert np.max(np.abs(U - U0)) > 1e-2  # it did move
    assert orc.max_su3_dev(d, U) < 1e-13
    orc.or_pass_reversed(d, U)
    assert np.max(np.abs(U - U0)) < 1e-12


@pytest.mark.parametrize("sampler", [0, 1])
def test_beta_zero_heat_bath_is_exhausted(orc, sampler):
    """At beta = 0 the draw's weight exp(alpha g0) has alpha = 0 (Sec. IV.A):
    the Kennedy-Pendleton proposal delta = e / alpha is infinite and the
    Creutz inversion 0 / 0, so no trial is accepted.  Every subgroup draw of
    every hit is then counted exhausted and the links are left as they were;
    overrelaxation, which does not involve beta, still moves them."""
    d = [4, 2, 4, 2]
    U = orc.init_hot(d, 4, 0)
    U0 = U.copy()
    n_links = 4 * int(np.prod(d))
    _, ex = orc.sweep_hb_or(d, U, 0.0, 4, 0, 0, 2, n_or=0, n_hb_hits=2, hb_max_tries=3, sampler=sampler)
    assert ex == 2 * 2 * 3 * n_links
    assert np.array_equal(U, U0)
    _, ex = orc.sweep_hb_or(d, U, 0.0, 4, 0, 2, 1, n_or=1, hb_max_tries=3, sampler=sampler)
    assert ex == 3 * n_links
    assert np.max(np.abs(U - U0)) > 1e-2


def test_hb_lowers_action_from_hot_start(orc):
    d = [4, 4, 4, 4]
    U = orc.init_hot(d, 1, 0)
    hist, ex = orc.sweep_hb_or(d, U, 6.0, 1, 0, 0, 10)
    assert ex == 0
    assert hist[-1] > 0.5 and np.all(np.diff(hist[:4]) > 0)
    assert orc.max_su3_dev(d, U) < 1e-12


def _weyl_single_link(beta):
    """<(1/3) Re Tr U> under weight exp((beta/3) Re Tr U) on Haar SU(3),
    integrated over the eigenphase torus with the Vandermonde density."""
    n = 256
    th = 2 * np.pi * np.arange(n) / n
    t1, t2 = np.meshgrid(th, th, indexing="ij")
    t3 = -t1 - t2
    z = [np.exp(1j * t) for t in (t1, t2, t3)]
    vdm = np.abs(z[0] - z[1]) ** 2 * np.abs(z[0] - z[2]) ** 2 * np.abs(z[1] - z[2]) ** 2
    tr = (np.cos(t1) + np.cos(t2) + np.cos(t3)) / 3
    w = vdm * np.exp(beta * tr)
    return float(np.sum(w * tr) / np.sum(w))


@pytest.mark.slow
@pytest.mark.parametrize("beta", [0.5, 1.0])
def test_strong_coupling_plaquette(orc, beta):
    """At strong coupling the plaquette equals the single-plaquette value
    <(1/3)ReTr U> with weight exp((beta/3) ReTr U) up to O((beta/18)^5);
    pins the heat-bath coupling alpha = 2 beta k / 3 (a factor 2 in alpha
    would double the plaquette)."""
    d = [4, 4, 4, 4]
    U = orc.init_hot(d, 31, 0)
    hist, _ = orc.sweep_hb_or(d, U, beta, 31, 0, 0, 1600, n_or=0)
    x = hist[100:]
    b = x.reshape(50, -1).mean(axis=1)
    mean, err = b.mean(), b.std(ddof=1) / np.sqrt(len(b))
    exact = _weyl_single_link(beta)
    assert abs(exact - {0.5: 0.02893167, 1.0: 0.06012655}[beta]) < 1e-7
    assert abs(mean - exact) < 4 * err + 1e-4, (mean, err, exact)


@pytest.mark.slow
def test_weak_coupling_equipartition(orc):
    """At weak coupling beta (1 - <P>) -> 2 (1 - 1/V): (N^2-1) = 8 quadratic
    modes per link with gauge and constant modes removed share the action
    equally."""
    d = [4, 4, 4, 4]
    V = np.prod(d)
    beta = 100.0
    U = orc.init_cold(d)
    hist, _ = orc.sweep_hb_or(d, U, beta, 41, 0, 0, 300, n_or=2)
    val = beta * (1 - hist[100:].mean())
    assert abs(val - 2 * (1 - 1 / V)) < 0.03 * 2, val


def test_schedule_is_deterministic_and_resumable(orc):
    """Counter-based draws: N sweeps equal N/2 + N/2 sweeps with the sweep
    index carried over, and the thread count does not change any bit."""
    d = [4, 2, 4, 2]
    U1 = orc.init_hot(d, 3, 2)
    U2 = U1.copy()
    h1, _ = orc.sweep_hb_or(d, U1, 5.8, 3, 2, 10, 6, reunit_every=4)
    ha, _ = orc.sweep_hb_or(d, U2, 5.8, 3, 2, 10, 3, reunit_every=4)
    hb, _ = orc.sweep_hb_or(d, U2, 5.8, 3, 2, 13, 3, reunit_every=4)
    assert np.array_equal(U1, U2)
    assert np.array_equal(h1, np.concatenate([ha, hb]))
    nt = orc.max_threads()
    orc.set_threads(1)
    try:
        U3 = orc.init_hot(d, 3, 2)
        orc.sweep_hb_or(d, U3, 5.8, 3, 2, 10, 6, reunit_every=4)
    finally:
        orc.set_threads(nt)
    assert np.array_equal(U1, U3)


def test_hb_is_gauge_covariant_in_distribution(orc):
    """A sweep from a gauge-transformed start gives the same plaquette
    history up to rounding for the OR passes alone (OR is a deterministic
    function of gauge-invariant data: U' = R U with R conjugated along)."""
    d = [4, 4, 2, 2]
    U = orc.init_hot(d, 8, 0)
    orc.sweep_hb_or(d, U, 6.0, 8, 0, 0, 2, n_or=0)
    W = U.copy()
    orc.gauge_transform(d, W, 99)
    for _ in range(3):
        orc.or_pass(d, U)
        orc.or_pass(d, W)
    assert abs(orc.plaquette(d, U) - orc.plaquette(d, W)) < 1e-12
