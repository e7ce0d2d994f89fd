"""Oracle pins for HMC (Sec. IV.E, App. A): force = derivative of the
Wilson action, leapfrog error scaling, reversibility, Creutz equality."""
import numpy as np
import pytest
from scipy.linalg import expm

import synth_inputs as si


def _gellmann():
    l = np.zeros((8, 3, 3), dtype=complex)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return l


def test_gellmann_normalization():
    l = _gellmann()
    for a in range(8):
        assert abs(np.trace(l[a])) < 1e-15
        for b in range(8):
            assert abs(np.trace(l[a] @ l[b]) - 2 * (a == b)) < 1e-14


@pytest.mark.parametrize("dims", [[2, 2, 2, 2], [4, 2, 2, 4]])
def test_force_is_action_derivative(orc, dims):
    """F^a(n,mu) equals the central difference of S(exp(i h T^a) U_mu(n))."""
    beta = 5.5
    U = si.random_field(dims, 13)
    F = orc.hmc_force(dims, U, beta)
    T = _gellmann() / 2
    h = 1e-5
    rng = np.random.Generator(np.random.PCG64(4))
    for _ in range(5):
        site, mu = int(rng.integers(0, np.prod(dims))), int(rng.integers(0, 4))
        u = U[site, mu, ..., 0] + 1j * U[site, mu, ..., 1]
        for a in range(8):
            vals = []
            for s in (+1, -1):
                W = U.copy()
                m = expm(1j * s * h * T[a]) @ u
                W[site, mu] = np.stack([m.real, m.imag], axis=-1)
                vals.append(orc.action(dims, W, beta))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - F[site, mu, a]) < 1e-6 * (1 + abs(fd)), (a, fd, F[site, mu, a])


def _thermal(orc, dims, beta, seed):
    U = orc.init_hot(dims, seed, 0)
    orc.sweep_hb_or(dims, U, beta, seed, 0, 0, 20)
    return U


def test_leapfrog_error_is_second_order(orc):
    """|dH| at fixed trajectory length falls by 4 when the step halves."""
    d = [4, 4, 2, 4]
    beta = 6.0
    U0 = _thermal(orc, d, beta, 6)
    p0 = orc.hmc_momenta(d, 6, 0, 0)
    H0 = orc.hmc_kinetic(d, p0) + orc.action(d, U0, beta)
    dh = []
    for n in (48, 96, 192):
        U, p = U0.copy(), p0.copy()
        orc.md_leapfrog(d, U, p, beta, 0.5 / n, n)
        dh.append(orc.hmc_kinetic(d, p) + orc.action(d, U, beta) - H0)
    r1, r2 = dh[0] / dh[1], dh[1] / dh[2]
    assert abs(r1 - 4) < 0.3 and abs(r2 - 4) < 0.15, dh


def test_leapfrog_is_reversible_and_keeps_su3(orc):
    d = [4, 4, 2, 2]
    beta = 6.0
    U0 = _thermal(orc, d, beta, 7)
    p0 = orc.hmc_momenta(d, 7, 0, 3)
    U, p = U0.copy(), p0.copy()
    orc.md_leapfrog(d, U, p, beta, 0.05, 20)
    assert np.max(np.abs(U - U0)) > 1e-2
    assert orc.max_su3_dev(d, U) < 1e-12
    p = np.ascontiguousarray(-p)
    orc.md_leapfrog(d, U, p, beta, 0.05, 20)
    assert np.max(np.abs(U - U0)) < 1e-11
    assert np.max(np.abs(p + p0)) < 1e-10


def test_zero_length_trajectory_and_flow_are_identities(orc):
    """tau = 0 and flow steps of 0: exp(0) is the identity and every kick is
    zero, so the links come back unchanged bit for bit and dH is 0 exactly
    (the same sums over the same values)."""
    d = [4, 2, 2, 4]
    U = orc.init_hot(d, 9, 0)
    U0 = U.copy()
    acc, dH = orc.hmc_trajectory(d, U, 6.0, 0.0, 5, 9, 0, 0, 1)
    assert acc and dH == 0.0
    assert np.array_equal(U, U0)
    orc.wilson_flow(d, U, 0.0, 3)
    assert np.array_equal(U, U0)


def test_momenta_are_standard_normal(orc):
    p = orc.hmc_momenta([8, 8, 8, 8], 3, 1, 5)
    x = p.ravel()
    assert abs(x.mean()) < 5 / np.sqrt(x.size)
    assert abs(x.var() - 1) < 5 * np.sqrt(2 / x.size)
    assert not np.array_equal(p, orc.hmc_momenta([8, 8, 8, 8], 3, 1, 6))


def test_rejection_restores_field(orc):
    """A huge step is rejected and the field is restored bit for bit."""
    d = [2, 2, 2, 2]
    U = _thermal(orc, d, 6.0, 9)
    U0 = U.copy()
    acc, dH = orc.hmc_trajectory(d, U, 6.0, 3.0, 2, 9, 0, 0, 1)
    assert not acc and dH > 50
    assert np.array_equal(U, U0)
    acc, dH = orc.hmc_trajectory(d, U, 6.0, 3.0, 2, 9, 0, 0, 0)
    assert acc and not np.array_equal(U, U0)


@pytest.mark.slow
def test_creutz_equality_and_hb_hmc_agreement(orc):
    """<exp(-dH)> = 1 in equilibrium, and HMC and HB+OR give the same
    average plaquette (two algorithms for the same distribution) on 2^4."""
    d = [2, 2, 2, 2]
    beta = 3.0
    U = _thermal(orc, d, beta, 12)
    e, pl, nacc = [], [], 0
    for t in range(1500):
        acc, dH = orc.hmc_trajectory(d, U, beta, 1.0, 8, 12, 0, t, 1)
        nacc += acc
        if t >= 100:
            e.append(np.exp(-dH))
            pl.append(orc.plaquette(d, U))
    e = np.array(e)
    be = e.reshape(35, -1).mean(axis=1)
    assert abs(be.mean() - 1) < 4 * be.std(ddof=1) / np.sqrt(len(be)) + 1e-3
    assert nacc > 300
    W = _thermal(orc, d, beta, 13)
    hist, _ = orc.sweep_hb_or(d, W, beta, 13, 0, 100, 4000, n_or=1)
    bh = hist.reshape(40, -1).mean(axis=1)
    bm = np.array(pl).reshape(35, -1).mean(axis=1)
    diff = bm.mean() - bh.mean()
    err = np.hypot(bm.std(ddof=1) / np.sqrt(35), bh.std(ddof=1) / np.sqrt(40))
    assert abs(diff) < 4 * err, (bm.mean(), bh.mean(), err)
