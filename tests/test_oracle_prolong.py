"""Oracle pins for restriction, prolongation (transfer + APE interpolation)
and the partial averages of Sec. III."""
from math import comb

import numpy as np
import pytest

import synth_inputs as si


def _chi_mu(dims):
    """chi_mu(n) = number of odd coordinates of n other than n_mu, [V,4]."""
    V = int(np.prod(dims))
    i = np.arange(V)
    n = []
    for L in dims:
        n.append(i % L)
        i = i // L
    odd = np.stack(n, axis=1) & 1
    return odd.sum(axis=1)[:, None] - odd


def test_restrict_of_transfer_is_identity(orc):
    dc = [2, 4, 2, 2]
    Uc = si.random_field(dc, 1)
    Uf = orc.prolong_transfer(dc, Uc)
    df = [2 * x for x in dc]
    assert np.array_equal(orc.restrict(df, Uf), Uc)
    chi = _chi_mu(df)
    # every bond not transferred from the coarse lattice starts at 1
    one = orc.init_cold(df)
    moved = np.any(Uf != one, axis=(2, 3, 4))
    assert np.all(chi[moved] == 0)


def test_normalizations_of_partial_averages(orc):
    """N^{1x1}_d = 2(D-d)(D-d-1) C(D,d) N0/2^D and N^{2x2}_d = C(D,2) C(D,d)
    N0/2^D weight the partial averages into the full ones; both sum to the
    number of plaquettes C(D,2) N0."""
    D = 4
    dims = [4, 2, 4, 2]
    N0 = np.prod(dims)
    n11 = [2 * (D - d) * (D - d - 1) * comb(D, d) * N0 / 2**D for d in range(D + 1)]
    n22 = [comb(D, 2) * comb(D, d) * N0 / 2**D for d in range(D + 1)]
    assert sum(n11) == sum(n22) == comb(D, 2) * N0
    U = si.random_field(dims, 8)
    p = orc.plaquette(dims, U)
    tot = sum(n11[d] * orc.partial_plaquette(dims, U, d) for d in range(D - 1))
    assert abs(tot / (comb(D, 2) * N0) - p) < 1e-13
    w22 = orc.wilson_loop(dims, U, 2, 2)
    tot = sum(n22[d] * orc.displaced_2x2(dims, U, d) for d in range(D + 1))
    assert abs(tot / (comb(D, 2) * N0) - w22) < 1e-13


def test_ape_step_touches_only_active_bonds(orc):
    df = [4, 4, 4, 4]
    U = si.random_field(df, 2)
    chi = _chi_mu(df)
    for d in range(3):
        W = U.copy()
        orc.ape_step(df, W, d, 0.05)
        changed = np.any(W != U, axis=(2, 3, 4))
        assert np.all(changed == (chi == d + 1))
        assert orc.max_su3_dev(df, W) < 1e-13


def test_projection_maximizes_overlap(orc):
    """P_SU(3)(M) is in SU(3), fixes SU(3) elements, and beats random SU(3)
    elements and the unitarized M on Re Tr(X^+ M)."""
    rng = np.random.Generator(np.random.PCG64(3))
    for k in range(20):
        M = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        X = orc.project_su3(np.stack([M.real, M.imag], -1))
        X = X[..., 0] + 1j * X[..., 1]
        assert np.allclose(X @ X.conj().T, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(X) - 1) < 1e-13
        f = np.trace(X.conj().T @ M).real
        for R in si.random_su3(200, k):
            assert np.trace(R.conj().T @ M).real <= f + 1e-12
            # local optimality: small SU(3) moves do not improve
        for a in range(8):
            H = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
            H = H + H.conj().T
            H -= np.trace(H) / 3 * np.eye(3)
            from scipy.linalg import expm
            Y = expm(1e-4j * H) @ X
            assert np.trace(Y.conj().T @ M).real <= f + 1e-12
    G = si.random_su3(1, 99)[0]
    X = orc.project_su3(np.stack([G.real, G.imag], -1))
    assert np.allclose(X[..., 0] + 1j * X[..., 1], G, atol=1e-14)


@pytest.mark.slow
def test_prolongation_properties(orc):
    """After prolongation: restriction returns the coarse field exactly;
    chi_mu = 0 bonds are untouched; 2x2 loops from even sites are the coarse
    plaquettes; each stage's active bonds are stationary points of S_d."""
    dc = [2, 2, 2, 2]
    df = [4, 4, 4, 4]
    Uc = orc.init_hot(dc, 7, 0)
    orc.sweep_hb_or(dc, Uc, 5.8, 7, 0, 0, 30)
    Uf, iters = orc.prolongate(dc, Uc, 0.05, 1e-12, 20000)
    assert all(1 <= k < 20000 for k in iters), iters
    assert np.array_equal(orc.restrict(df, Uf), Uc)
    T0 = orc.prolong_transfer(dc, Uc)
    chi = _chi_mu(df)
    assert np.array_equal(Uf[chi == 0], T0[chi == 0])
    assert abs(orc.displaced_2x2(df, Uf, 0) - orc.plaquette(dc, Uc)) < 1e-13
    assert orc.max_su3_dev(df, Uf) < 1e-12
    # stationarity: (U^+ sum_T)_AT ~ 0 on active bonds of each stage
    M = orc.as_complex(Uf).reshape(df[3], df[2], df[1], df[0], 4, 3, 3)
    chi4 = chi.reshape(df[3], df[2], df[1], df[0], 4)
    odd = [(np.arange(L) & 1) for L in df]
    par = np.zeros((df[3], df[2], df[1], df[0], 4), dtype=int)
    for m in range(4):
        shape = [1, 1, 1, 1]
        shape[3 - m] = df[m]
        par[..., m] = np.broadcast_to(odd[m].reshape(shape), par.shape[:4])

    def sh(A, mu, s):
        return np.roll(A, -s, axis=3 - mu)

    dag = lambda A: np.conj(np.swapaxes(A, -1, -2))
    worst = 0.0
    for d in range(3):
        for mu in range(4):
            S = np.zeros(M.shape[:4] + (3, 3), dtype=complex)
            for nu in range(4):
                if nu == mu:
                    continue
                Unu, Umu = M[..., nu, :, :], M[..., mu, :, :]
                tp = Unu @ sh(Umu, nu, 1) @ dag(sh(Unu, mu, 1))
                tm = dag(sh(Unu, nu, -1)) @ sh(Umu, nu, -1) @ sh(sh(Unu, nu, -1), mu, 1)
                # staples of plaquettes with chi_munu = d: nu an odd transverse direction
                w = (par[..., nu] == 1) & (chi4[..., mu] == d + 1)
                S += np.where(w[..., None, None], tp + tm, 0)
            act = chi4[..., mu] == d + 1
            X = dag(M[..., mu, :, :]) @ S
            A = X - dag(X)
            A -= np.trace(A, axis1=-2, axis2=-1)[..., None, None] / 3 * np.eye(3)
            worst = max(worst, np.max(np.abs(A[act])))
    assert worst < 1e-4, worst
