"""Oracle pins for the m x n Wilson loops of Sec. III (their average over
sites and planes, and the displaced averages by site class), including
loops with m != n, whose two legs a plain square-loop check cannot tell
apart."""
from math import comb

import numpy as np
import pytest

import synth_inputs as si


def _graded_flux(dims, mu, nu, phi, H):
    """Abelian field with flux only in the plane (mu, nu), varying along mu:
    U_nu(x) = exp(i Phi(x_mu) H) with Phi(x) = sum_{a<x} phi(a), every other
    link 1.  The plaquette at x in that plane is exp(i phi(x_mu) H); with
    sum(phi) a multiple of 2 pi and integer H the field is periodic."""
    V = int(np.prod(dims))
    Phi = np.concatenate([[0.0], np.cumsum(phi)[:-1]])
    U = np.zeros((V, 4, 3, 3), dtype=complex)
    U[:] = np.eye(3)
    i = np.arange(V)
    x = []
    for L in dims:
        x.append(i % L)
        i = i // L
    ph = Phi[x[mu]]
    U[:, nu] = np.exp(1j * ph[:, None] * np.asarray(H, float)[None, :])[:, :, None] * np.eye(3)[None]
    return np.ascontiguousarray(np.stack([U.real, U.imag], -1))


def _graded_closed_form(L, mu, nu, phi, H, m, n):
    """Average m x n loop of _graded_flux: 5 of the 6 planes give 1.  In the
    flux plane the loop runs m steps along its lower direction first.  If
    that is mu, the loop holds the flux of n columns of width m,
    exp(i n D_m(x) H) with D_m(x) = sum_{a<m} phi(x+a); if it is nu, the
    legs exchange roles and the phase is -m D_n(x) H."""
    h = np.asarray(H, float)

    def D(w):
        return np.array([sum(phi[(x + a) % L] for a in range(w)) for x in range(L)])

    if mu < nu:
        t = np.mean(np.cos(n * D(m)[:, None] * h[None, :]))
    else:
        t = np.mean(np.cos(m * D(n)[:, None] * h[None, :]))
    return (t + 5.0) / 6.0


@pytest.mark.parametrize("mu,nu", [(0, 1), (1, 3), (3, 2)])
@pytest.mark.parametrize("H", [(1, -1, 0), (2, -1, -1)])
def test_wilson_loop_graded_flux_closed_form(orc, mu, nu, H):
    """A flux that varies across the plane makes W(m, n) != W(n, m), so this
    fixes which leg takes m steps and that the path closes."""
    d = [6, 4, 4, 8]
    L = d[mu]
    rng = np.random.Generator(np.random.PCG64(100 + 10 * mu + nu))
    phi = 2 * np.pi / L + 1.2 * (rng.random(L) - 0.5)
    phi[-1] = 2 * np.pi - np.sum(phi[:-1])  # one flux quantum in total
    U = _graded_flux(d, mu, nu, phi, H)
    assert orc.max_su3_dev(d, U) < 1e-13
    for m, n in [(1, 1), (1, 2), (2, 1), (2, 3), (3, 1), (1, 3)]:
        w = orc.wilson_loop(d, U, m, n)
        exact = _graded_closed_form(L, mu, nu, phi, H, m, n)
        assert abs(w - exact) < 1e-13, (m, n, w, exact)
    # the field is anisotropic enough that exchanging the legs is visible
    assert abs(orc.wilson_loop(d, U, 1, 2) - orc.wilson_loop(d, U, 2, 1)) > 1e-4


def test_wilson_loop_gauge_invariant(orc):
    d = [4, 4, 4, 4]
    U = orc.init_hot(d, 21, 0)
    orc.sweep_hb_or(d, U, 6.0, 21, 0, 0, 3)
    W = U.copy()
    orc.gauge_transform(d, W, 77)
    assert np.max(np.abs(W - U)) > 0.1
    for m, n in [(1, 2), (2, 1), (2, 3), (3, 1)]:
        a, b = orc.wilson_loop(d, U, m, n), orc.wilson_loop(d, W, m, n)
        assert abs(a - b) < 1e-13, (m, n, a, b)
        for c in range(5):
            a, b = orc.displaced_loop(d, U, c, m, n), orc.displaced_loop(d, W, c, m, n)
            assert abs(a - b) < 1e-13, (c, m, n)


def test_displaced_loops_recombine(orc):
    """Sites of class chi = d are a fraction C(D,d)/2^D of the lattice, so
    the displaced m x n averages recombine to the full average."""
    d = [4, 2, 4, 6]
    U = si.random_field(d, 13)
    for m, n in [(1, 2), (2, 1), (3, 2)]:
        tot = sum(comb(4, c) / 16.0 * orc.displaced_loop(d, U, c, m, n) for c in range(5))
        assert abs(tot - orc.wilson_loop(d, U, m, n)) < 1e-13
    for c in range(5):
        assert orc.displaced_loop(d, U, c, 2, 2) == orc.displaced_2x2(d, U, c)


def test_prolongation_preserves_even_loops(orc):
    """Sec. III: after the transfer every even-sided loop from an even fine
    site equals the coarse loop of half the size; the interpolation only
    moves bonds with chi_mu > 0, none of which lies on such a loop."""
    dc = [4, 2, 4, 2]
    df = [2 * x for x in dc]
    Uc = si.random_field(dc, 41)
    pairs = [(1, 1), (1, 2), (2, 1), (2, 3), (3, 1)]
    Uf = orc.prolong_transfer(dc, Uc)
    for m, n in pairs:
        assert abs(orc.displaced_loop(df, Uf, 0, 2 * m, 2 * n) - orc.wilson_loop(dc, Uc, m, n)) < 1e-13, (m, n)
    Up, _ = orc.prolongate(dc, Uc, max_iter=20)
    for m, n in pairs:
        assert abs(orc.displaced_loop(df, Up, 0, 2 * m, 2 * n) - orc.wilson_loop(dc, Uc, m, n)) < 1e-13, (m, n)
    # odd-sided loops are not preserved (the interpolated bonds enter them)
    assert abs(orc.displaced_loop(df, Up, 0, 1, 2) - orc.wilson_loop(dc, Uc, 1, 1)) > 1e-3
