"""Oracle pins for the adaptive-step Wilson flow, the flow scale t0 and the
admissibility measure h = max s_p (Sec. IV.B and IV.D)."""
import numpy as np
import pytest

import synth_inputs as si


def _thermal(orc, dims, beta, seed, n=8):
    U = orc.init_hot(dims, seed, 0)
    orc.sweep_hb_or(dims, U, beta, seed, 0, 0, n)
    return U


def _fixed_curve(orc, dims, U, eps, t_meas):
    """E(t) at t_meas from the fixed-step flow (each t a multiple of eps)."""
    W = U.copy()
    out, t = [], 0.0
    for tm in t_meas:
        n = int(round((tm - t) / eps))
        if n:
            orc.wilson_flow(dims, W, eps, n)
        t = tm
        out.append(orc.clover_energy(dims, W))
    return np.array(out), W


def test_embedded_estimate_is_second_order(orc):
    """The embedded result W~ = exp(2 Z1 - Z0) W0 is second order, so its
    distance to the third-order step shrinks as h^3 (ratio 8 per halving);
    a first-order estimate would give ratio 2."""
    d = [4, 4, 4, 4]
    U = _thermal(orc, d, 6.0, 4)
    orc.wilson_flow(d, U, 0.02, 5)
    dist = []
    for h in (0.08, 0.04, 0.02):
        W = U.copy()
        dist.append(orc.flow_step_distance(d, W, h))
    r1, r2 = dist[0] / dist[1], dist[1] / dist[2]
    assert 6.5 < r1 < 9.5 and 6.5 < r2 < 9.5, (dist, r1, r2)
    # the step itself is the fixed-step RK3 step
    W = U.copy()
    orc.flow_step_distance(d, W, 0.05)
    V = U.copy()
    orc.wilson_flow(d, V, 0.05, 1)
    assert np.max(np.abs(W - V)) < 1e-14


def test_adaptive_flow_tracks_fine_fixed_step_flow(orc):
    """E(t) from the adaptive flow against a fine fixed-step flow: the
    deviation is small and shrinks with the tolerance; the field lands on
    every measurement time."""
    d = [4, 4, 4, 6]
    U = _thermal(orc, d, 5.8, 6)
    t_meas = [0.0, 0.25, 0.5, 1.0, 1.5, 2.0]
    Eref, Wref = _fixed_curve(orc, d, U, 0.0025, t_meas)
    devs = []
    for tol in (1e-2, 1e-4):
        W = U.copy()
        E, Q, na, nr = orc.wilson_flow_adaptive(d, W, 2.0, tol, 0.2, 0.01, t_meas)
        devs.append(np.max(np.abs(E - Eref) / Eref))
        assert E[0] == orc.clover_energy(d, U)
    assert devs[0] < 5e-4, devs  # the paper quotes up to 2e-4 at this tolerance
    assert devs[1] < devs[0] / 20, devs


def test_adaptive_flow_rejects_and_grows_steps(orc):
    """A first step far too large for a rough field is rejected and
    repeated smaller; on a smooth field steps grow to the maximum."""
    d = [4, 4, 4, 4]
    U = si.random_field(d, 8)
    W = U.copy()
    E, Q, na, nr = orc.wilson_flow_adaptive(d, W, 0.4, 1e-3, 0.2, 0.2, [0.4])
    assert nr >= 1 and na >= 2
    # accepted steps: every one within tolerance, result equals a fixed-step flow
    # of the same total length to the tolerance level
    V = U.copy()
    orc.wilson_flow(d, V, 0.002, 200)
    assert abs(E[0] - orc.clover_energy(d, V)) < 5e-3 * abs(E[0])
    C = orc.init_cold(d)
    orc.gauge_transform(d, C, 5)
    E, Q, na, nr = orc.wilson_flow_adaptive(d, C, 2.0, 1e-2, 0.2, 0.01, [2.0])
    assert nr == 0 and na <= 12 and abs(E[0]) < 1e-12


def test_flow_t0_interpolation(orc):
    """t0 solves t^2 E(t) = 0.3 by linear interpolation between the two
    bracketing measurements: exact when t^2 E is linear in t."""
    t = np.linspace(0.1, 2.0, 20)
    y = 0.05 + 0.2 * t  # crosses 0.3 at t = 1.25
    E = y / t**2
    assert abs(orc.flow_t0(t, E) - 1.25) < 1e-14
    y2 = 0.3 * (t / 1.3) ** 2  # quadratic: interpolation error (h^2/8) |y''|
    t0 = orc.flow_t0(t, y2 / t**2)
    assert abs(t0 - 1.3) < 0.1**2 / 8 * 2 * 0.3 / 1.3**2 / (2 * 0.3 / 1.3) + 1e-12
    assert np.isnan(orc.flow_t0(t, 0.01 * np.ones_like(t)))


def test_max_splaq_closed_forms(orc):
    """h = max_p 3 [1 - (1/3) Re Tr U_p]: 0 on pure gauge, 3 - sum cos of the
    flux angles on constant abelian flux, and the maximum of a numpy
    evaluation of every plaquette on a random field."""
    d = [4, 4, 4, 4]
    C = orc.init_cold(d)
    orc.gauge_transform(d, C, 2)
    assert orc.max_splaq(d, C) < 1e-13
    from test_oracle_flow_q import _flux_field
    d2 = [8, 8, 6, 6]
    H01, H23 = (1, -1, 0), (1, 1, -2)
    U, p01, p23 = _flux_field(d2, 1, 1, H01, H23)
    exact = max(3 - np.cos(p01 * np.array(H01, float)).sum(), 3 - np.cos(p23 * np.array(H23, float)).sum())
    assert abs(orc.max_splaq(d2, U) - exact) < 1e-13
    d3 = [4, 4, 2, 6]
    R = si.random_field(d3, 13)
    M = orc.as_complex(R).reshape(d3[3], d3[2], d3[1], d3[0], 4, 3, 3)

    def shift(A, mu):
        return np.roll(A, -1, axis=3 - mu)

    hmax = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = M[..., mu, :, :]
            b = shift(M[..., nu, :, :], mu)
            c = np.conj(np.swapaxes(shift(M[..., mu, :, :], nu), -1, -2))
            e = np.conj(np.swapaxes(M[..., nu, :, :], -1, -2))
            hmax = max(hmax, float((3 - np.trace(a @ b @ c @ e, axis1=-2, axis2=-1).real).max()))
    assert abs(orc.max_splaq(d3, R) - hmax) < 1e-12
