"""Host-side analysis of Monte Carlo histories (numpy / scipy).

- Autocorrelations and the integrated autocorrelation time with jackknife
  errors (App. B: autocovariance estimator, jackknife over blocks with the
  pair-count correction, windowed tau_int).
- Constrained multi-exponential fits by variable projection (App. C).
- HMC acceptance model P_acc = erfc(Omega^(1/2) dtau^2 / 2) (App. A) and the
  topological-charge integrality measure eps(Q) (Sec. IV.D).

These operate on measurement arrays returned by the library; no lattice
data passes through them.
"""
from __future__ import annotations

import numpy as np
from scipy import optimize, special

# ---------------------------------------------------------------------------
# App. B: autocorrelations
# ---------------------------------------------------------------------------


def autocov_hat(dx: np.ndarray, max_lag: int) -> np.ndarray:
    """Gamma_hat_Delta = (1/N) sum_{tau=1}^{N-Delta} dx_tau dx_{tau+Delta} for
    Delta = 0..max_lag, through a zero-padded FFT (O(N log N))."""
    dx = np.asarray(dx, dtype=np.float64)
    n = dx.size
    m = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(dx, m)
    c = np.fft.irfft(f * np.conj(f), m)[: max_lag + 1]
    return c / n


def pair_count(n: int, nj: int, j: int, lag: int) -> int:
    """Number of pairs (tau, tau + lag), 1 <= tau <= n - lag, with neither
    member in the omitted block ((j-1) nj, j nj] (the degeneracy g_Delta of a
    jackknife ensemble); j = 0 omits nothing."""
    if j == 0:
        return n - lag
    lo, hi = (j - 1) * nj, j * nj  # omitted: lo < tau <= hi
    tau = np.arange(1, n - lag + 1)
    keep = ~(((tau > lo) & (tau <= hi)) | ((tau + lag > lo) & (tau + lag <= hi)))
    return int(np.count_nonzero(keep))


def _rho(x: np.ndarray, omit: tuple | None, max_lag: int) -> np.ndarray:
    n = x.size
    if omit is None:
        dx = x - x.mean()
        g = n - np.arange(max_lag + 1)
    else:
        nj, j = omit
        mask = np.ones(n, bool)
        mask[(j - 1) * nj: j * nj] = False
        dx = np.where(mask, x - x[mask].mean(), 0.0)
        g = np.array([pair_count(n, nj, j, d) for d in range(max_lag + 1)], dtype=np.float64)
    gam = n / g * autocov_hat(dx, max_lag)
    return gam / gam[0]


def autocorrelation(x, nj: int, max_lag: int | None = None):
    """rho_Delta and its jackknife error for Delta = 0..max_lag, from blocks of
    nj consecutive measurements (len(x) must be a multiple of nj)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n % nj:
        raise ValueError("the number of measurements must be a multiple of the block size")
    max_lag = n // 2 if max_lag is None else max_lag
    rho = _rho(x, None, max_lag)
    nb = n // nj
    jk = np.array([_rho(x, (nj, j), max_lag) for j in range(1, nb + 1)])
    err = np.sqrt(n / (n - nj) * np.sum((jk - rho) ** 2, axis=0))
    return rho, err, jk


def tau_int(x, nj: int, max_lag: int | None = None):
    """Integrated autocorrelation time tau_int = 1/2 + sum_{Delta=1}^{W} rho_Delta
    with the window W the first lag where rho_Delta is no longer above its
    error, and its jackknife error.  Returns (tau_int, error, W)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    rho, err, jk = autocorrelation(x, nj, max_lag)
    w = len(rho) - 1
    for d in range(1, len(rho)):
        if not rho[d] > err[d]:
            w = d
            break
    tau = 0.5 + rho[1: w + 1].sum()
    tj = 0.5 + jk[:, 1: w + 1].sum(axis=1)
    dtau = float(np.sqrt(n / (n - nj) * np.sum((tj - tau) ** 2)))
    return float(tau), dtau, w


# ---------------------------------------------------------------------------
# App. C: constrained multi-exponential fits by variable projection
# ---------------------------------------------------------------------------


def _design(E: np.ndarray, t: np.ndarray, n_obs: int) -> np.ndarray:
    """Basis of f = sum_n z^alpha_n exp(-E_n tau) for the stacked data vector
    (alpha major, tau minor) and the stacked amplitudes (alpha major, n
    minor): block-diagonal copies of exp(-E_n tau)."""
    b = np.exp(-np.outer(t, E))  # [T, N]
    return np.kron(np.eye(n_obs), b)


def varpro_amplitudes(E, t, y, Vinv, phi=None):
    """Amplitudes z(E) minimizing chi^2 at fixed decay constants under the
    linear constraint phi z = 0 (App. C, amplitude equation), and chi^2 there.
    y: [n_obs, T]; Vinv: inverse covariance of the stacked data [n_obs T]^2;
    phi: [n_con, n_obs N] or None."""
    y = np.asarray(y, dtype=np.float64)
    n_obs = y.shape[0]
    B = _design(np.asarray(E, float), np.asarray(t, float), n_obs)
    yv = y.reshape(-1)
    u = B.T @ Vinv @ yv
    W = B.T @ Vinv @ B
    Wi_u = np.linalg.solve(W, u)
    if phi is not None and len(phi):
        phi = np.asarray(phi, dtype=np.float64)
        Wi_pT = np.linalg.solve(W, phi.T)
        z = Wi_u - Wi_pT @ np.linalg.solve(phi @ Wi_pT, phi @ Wi_u)
    else:
        z = Wi_u
    r = yv - B @ z
    return z.reshape(n_obs, -1), float(r @ Vinv @ r)


def varpro_fit(t, y, cov, E0, phi=None):
    """Fit y^alpha(tau) = sum_n z^alpha_n exp(-E_n tau) with shared decay
    constants E_n and constraint phi z = 0 by minimizing the reduced chi^2(E)
    (App. C).  cov: covariance of the stacked data.  Returns (E, z, chi2)."""
    t = np.asarray(t, dtype=np.float64)
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    Vinv = np.linalg.inv(np.asarray(cov, dtype=np.float64))

    def chi2(logE):
        return varpro_amplitudes(np.exp(logE), t, y, Vinv, phi)[1]

    res = optimize.minimize(chi2, np.log(np.asarray(E0, dtype=np.float64)), method="Nelder-Mead",
                            options={"xatol": 1e-10, "fatol": 1e-12, "maxiter": 20000, "maxfev": 40000})
    E = np.exp(res.x)
    order = np.argsort(E)
    E = E[order]
    z, c2 = varpro_amplitudes(E, t, y, Vinv, phi)
    return E, z, c2


# ---------------------------------------------------------------------------
# App. A and Sec. IV.D
# ---------------------------------------------------------------------------


def acceptance_model(dtau, omega_half):
    """P_acc = erfc(Omega^(1/2) dtau^2 / 2)."""
    return special.erfc(0.5 * omega_half * np.asarray(dtau, dtype=np.float64) ** 2)


def fit_acceptance(dtau, acc, n_traj):
    """Least-squares fit of Omega^(1/2) to measured acceptance rates (binomial
    weights).  Returns (Omega^(1/2), its error, 1/dtau at 70 % acceptance)."""
    dtau = np.asarray(dtau, dtype=np.float64)
    acc = np.asarray(acc, dtype=np.float64)
    n = np.broadcast_to(np.asarray(n_traj, dtype=np.float64), acc.shape)
    sig = np.sqrt(np.clip(acc * (1 - acc), 0.25 / n, None) / n)
    p0 = 2 * special.erfcinv(np.clip(np.median(acc), 0.05, 0.95)) / np.median(dtau) ** 2
    (om,), cov = optimize.curve_fit(acceptance_model, dtau, acc, p0=[p0], sigma=sig, absolute_sigma=True)
    inv70 = 1.0 / np.sqrt(2 * special.erfcinv(0.7) / om)
    return float(om), float(np.sqrt(cov[0, 0])), float(inv70)


def eps_q(Q):
    """eps(Q) = sqrt(mean((Q_i - [Q_i])^2)), [Q] the nearest integer."""
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.sqrt(np.mean((Q - np.rint(Q)) ** 2)))
