"""Oracle pins for the Wilson flow (Sec. IV.B) and the clover topological
charge (Sec. IV.D; clover reading of the charge density)."""
import numpy as np
import pytest
from scipy.linalg import expm

import synth_inputs as si


def _thermal(orc, dims, beta, seed, n=10):
    U = orc.init_hot(dims, seed, 0)
    orc.sweep_hb_or(dims, U, beta, seed, 0, 0, n)
    return U


def test_flow_keeps_cold_field(orc):
    d = [4, 4, 4, 4]
    U = orc.init_cold(d)
    orc.wilson_flow(d, U, 0.01, 3)
    assert np.array_equal(U, orc.init_cold(d))


def test_flow_lowers_action_monotonically(orc):
    d = [4, 4, 4, 4]
    U = _thermal(orc, d, 6.0, 3)
    s = [orc.action(d, U, 1.0)]
    for _ in range(6):
        orc.wilson_flow(d, U, 0.02, 2)
        s.append(orc.action(d, U, 1.0))
    assert np.all(np.diff(s) < 0)
    assert orc.max_su3_dev(d, U) < 1e-12


def test_flow_initial_slope(orc):
    """dS/dt at t = 0 equals -(beta/3) sum_links Re Tr(Z Om) with
    Z = -(1/2)(Om - Om^+)_traceless, Om = U A: the flow generator is the
    negative action gradient (with beta = 1 for S)."""
    d = [4, 2, 2, 4]
    U = _thermal(orc, d, 6.0, 4)
    s0 = orc.action(d, U, 3.0)  # beta = 3 so that S = -sum ReTr U_p + const
    slope = 0.0
    for site in range(int(np.prod(d))):
        for mu in range(4):
            A = orc.staple(d, U, site, mu)
            Om = (U[site, mu, ..., 0] + 1j * U[site, mu, ..., 1]) @ (A[..., 0] + 1j * A[..., 1])
            X = Om - Om.conj().T
            Z = -0.5 * (X - np.trace(X) / 3 * np.eye(3))
            slope -= np.trace(Z @ Om).real
    h = 1e-4
    W = U.copy()
    orc.wilson_flow(d, W, h, 1)
    W2 = U.copy()
    orc.wilson_flow(d, W2, -h, 1)
    fd = (orc.action(d, W, 3.0) - orc.action(d, W2, 3.0)) / (2 * h)
    assert slope < 0
    assert abs(fd - slope) < 1e-5 * abs(slope), (fd, slope)


@pytest.mark.slow
def test_flow_is_third_order(orc):
    """The RK3 integrator's global error at fixed flow time scales as eps^3."""
    d = [4, 4, 2, 2]
    U0 = _thermal(orc, d, 6.0, 5)
    res = []
    for n in (16, 32, 64):
        U = U0.copy()
        orc.wilson_flow(d, U, 0.4 / n, n)
        res.append(U)
    e1 = np.max(np.abs(res[0] - res[1]))
    e2 = np.max(np.abs(res[1] - res[2]))
    assert abs(e1 / e2 - 8) < 1.6, e1 / e2


def test_flow_is_gauge_covariant(orc):
    d = [4, 4, 2, 2]
    U = _thermal(orc, d, 6.0, 6)
    W = U.copy()
    orc.gauge_transform(d, W, 12)
    orc.wilson_flow(d, U, 0.02, 3)
    orc.wilson_flow(d, W, 0.02, 3)
    assert abs(orc.plaquette(d, U) - orc.plaquette(d, W)) < 1e-13
    assert abs(orc.topological_charge(d, U) - orc.topological_charge(d, W)) < 1e-12
    assert abs(orc.clover_energy(d, U) - orc.clover_energy(d, W)) < 1e-12


def _flux_field(dims, n01, n23, H01, H23):
    """Constant abelian flux: plaquette angles phi01 H01 in every 01 plaquette
    and phi23 H23 in every 23 plaquette, phi = 2 pi n / (area), made periodic
    by a twist on the last slice."""
    L0, L1, L2, L3 = dims
    V = L0 * L1 * L2 * L3
    p01 = 2 * np.pi * n01 / (L0 * L1)
    p23 = 2 * np.pi * n23 / (L2 * L3)
    U = np.zeros((V, 4, 3, 3), dtype=complex)
    e = lambda a, H: np.diag(np.exp(1j * a * np.asarray(H, dtype=float)))
    for i in range(V):
        x0, r = i % L0, i // L0
        x1, r = r % L1, r // L1
        x2, x3 = r % L2, r // L2
        U[i, 0] = e(-p01 * x1, H01)
        U[i, 1] = e(p01 * L1 * x0, H01) if x1 == L1 - 1 else np.eye(3)
        U[i, 2] = e(-p23 * x3, H23)
        U[i, 3] = e(p23 * L3 * x2, H23) if x3 == L3 - 1 else np.eye(3)
    return np.ascontiguousarray(np.stack([U.real, U.imag], -1)), p01, p23


@pytest.mark.parametrize("H01,H23", [((1, -1, 0), (1, 0, -1)), ((1, 1, -2), (1, 1, -2)), ((1, -1, 0), (0, 1, -1))])
def test_q_constant_flux_closed_form(orc, H01, H23):
    """For constant diagonal flux every clover leaf equals exp(i phi H), so
    F = i (sin(phi h) - mean) and Q = V/(2 pi^2) sum_i f01_i f23_i exactly;
    it tends to the continuum integer 2 Tr(H01 H23) n01 n23 as L grows."""
    d = [8, 8, 6, 6]
    U, p01, p23 = _flux_field(d, 1, 1, H01, H23)
    assert orc.max_su3_dev(d, U) < 1e-13
    f = np.sin(p01 * np.array(H01, float))
    f -= f.mean()
    g = np.sin(p23 * np.array(H23, float))
    g -= g.mean()
    exact = np.prod(d) / (2 * np.pi**2) * np.sum(f * g)
    q = orc.topological_charge(d, U)
    assert abs(q - exact) < 1e-11, (q, exact)
    big = [24, 24, 24, 24]
    pb01, pb23 = 2 * np.pi / 576, 2 * np.pi / 576
    fb = np.sin(pb01 * np.array(H01, float)); fb -= fb.mean()
    gb = np.sin(pb23 * np.array(H23, float)); gb -= gb.mean()
    integer = 2 * np.dot(H01, H23)
    assert abs(np.prod(big) / (2 * np.pi**2) * np.sum(fb * gb) - integer) < 1e-3 * max(1, abs(integer))


@pytest.mark.parametrize("H01,H23", [((1, -1, 0), (1, 0, -1)), ((1, 1, -2), (0, 1, -1))])
def test_clover_energy_constant_flux_closed_form(orc, H01, H23):
    """Clover energy density on constant diagonal flux: F_01 = i diag(f),
    f = sin(phi01 H01) minus its mean, likewise F_23 = i diag(g), all other
    planes zero, so -sum_{mu<nu} Re Tr(F F) per site = sum f^2 + sum g^2."""
    d = [8, 8, 6, 6]
    U, p01, p23 = _flux_field(d, 1, 1, H01, H23)
    f = np.sin(p01 * np.array(H01, float))
    f -= f.mean()
    g = np.sin(p23 * np.array(H23, float))
    g -= g.mean()
    exact = float(np.sum(f * f) + np.sum(g * g))
    e = orc.clover_energy(d, U)
    assert abs(e - exact) < 1e-13, (e, exact)
    # doubling the flux quantum changes the energy as the closed form says
    U2, q01, q23 = _flux_field(d, 2, 1, H01, H23)
    f2 = np.sin(q01 * np.array(H01, float))
    f2 -= f2.mean()
    assert abs(orc.clover_energy(d, U2) - float(np.sum(f2 * f2) + np.sum(g * g))) < 1e-13


def test_q_vanishes_on_pure_gauge_and_is_parity_odd(orc):
    d = [4, 4, 4, 4]
    U = orc.init_cold(d)
    orc.gauge_transform(d, U, 3)
    assert abs(orc.topological_charge(d, U)) < 1e-13
    U = _thermal(orc, d, 6.0, 9)
    orc.wilson_flow(d, U, 0.05, 4)
    q = orc.topological_charge(d, U)
    # reflection x0 -> -x0: U'_0(x) = U_0(Px - e0)^+, U'_k(x) = U_k(Px)
    M = orc.as_complex(U).reshape(d[3], d[2], d[1], d[0], 4, 3, 3)
    x0 = np.arange(d[0])
    R = np.empty_like(M)
    R[..., 0, :, :] = np.conj(np.swapaxes(M[:, :, :, (-x0 - 1) % d[0], 0], -1, -2))
    for k in range(1, 4):
        R[..., k, :, :] = M[:, :, :, (-x0) % d[0], k]
    W = orc.from_complex(R.reshape(-1, 4, 3, 3))
    assert abs(orc.plaquette(d, W) - orc.plaquette(d, U)) < 1e-13
    assert abs(q) > 1e-3
    assert abs(orc.topological_charge(d, W) + q) < 1e-12
