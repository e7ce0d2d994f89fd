"""Oracle pins for the complete Cabibbo-Marinari heat-bath update of one link
(Sec. IV.A): the SU(2) draw of every subgroup, its direction, the embedding
into SU(3), the order of the subgroups and the exhausted-draw count, taken
from the full update with the staple frozen (only the one link changes).

The SU(2) part of each subgroup is recomputed here from its defining
property, Re Tr(r w) = k Re Tr(r v) for every r in SU(2) (w the 2x2 block
of W = U A), and the laws are those of the local weight
exp((beta/3) Re Tr(U A)): g = r v has density exp(alpha g0) on the Haar
measure of SU(2) with alpha = 2 beta k / 3, i.e. g0 with density
sqrt(1 - g0^2) exp(alpha g0) and a direction uniform on the sphere."""
import numpy as np
import pytest
from scipy import integrate, stats

import synth_inputs as si

SUBGROUPS = [(0, 1), (1, 2), (0, 2)]


def _cx(a):
    return a[..., 0] + 1j * a[..., 1]


def _su2_part(W, i, j):
    """k and the unit quaternion v (as a 2x2 matrix [[x0+ix3, x2+ix1],
    [-x2+ix1, x0-ix3]]/k) of the (i, j) block of W."""
    w = np.array([[W[i, i], W[i, j]], [W[j, i], W[j, j]]])
    x0 = (w[0, 0] + w[1, 1]).real / 2
    x3 = (w[0, 0] - w[1, 1]).imag / 2
    x1 = (w[0, 1] + w[1, 0]).imag / 2
    x2 = (w[0, 1] - w[1, 0]).real / 2
    k = np.sqrt(x0 * x0 + x1 * x1 + x2 * x2 + x3 * x3)
    v = np.array([[x0 + 1j * x3, x2 + 1j * x1], [-x2 + 1j * x1, x0 - 1j * x3]]) / k
    return k, v, w


def _embed(r, i, j):
    R = np.eye(3, dtype=complex)
    R[i, i], R[i, j], R[j, i], R[j, j] = r[0, 0], r[0, 1], r[1, 0], r[1, 1]
    return R


def _g0_cdf(g0, alpha):
    """P(G0 <= g0) for the density sqrt(1-x^2) exp(alpha x) on [-1, 1], per
    sample: with x = cos(t) the integrand sin(t)^2 exp(alpha (cos t - 1)) is
    smooth, integrated by 64-point Gauss-Legendre over [arccos g0, pi]."""
    xs, ws = np.polynomial.legendre.leggauss(64)
    a = np.arccos(np.clip(g0, -1, 1))[:, None]
    t = a + (np.pi - a) * (xs[None, :] + 1) / 2
    f = np.sin(t) ** 2 * np.exp(alpha[:, None] * (np.cos(t) - 1))
    part = (np.pi - a[:, 0]) / 2 * np.sum(ws[None, :] * f, axis=1)
    t = np.pi * (xs + 1) / 2
    tot = np.pi / 2 * np.sum(ws[None, :] * np.sin(t)[None, :] ** 2 * np.exp(alpha[:, None] * (np.cos(t)[None, :] - 1)),
                             axis=1)
    return part / tot


def _uniform_chi2_p(x, lo, hi, nb=20):
    cnt, _ = np.histogram(x, bins=np.linspace(lo, hi, nb + 1))
    e = len(x) / nb
    return stats.chi2.sf(np.sum((cnt - e) ** 2 / e), nb - 1)


def _run_link(orc, d, U0, site, mu, beta, n, **kw):
    """n full updates of link (site, mu) from the same start (sweep counter
    s = 0..n-1); returns the new links, the step records and the counts."""
    U = U0.copy()
    out = np.empty((n, 3, 3), dtype=complex)
    recs = np.empty((n, 3, 11))
    exs = np.empty(n, dtype=np.int64)
    for s in range(n):
        U[site, mu] = U0[site, mu]
        exs[s], recs[s] = orc.hb_link(d, U, site, mu, beta, 7, 0, s, record=True, **kw)
        out[s] = _cx(U[site, mu])
    return out, recs, exs


def test_su2_part_property(orc):
    """The projection used below is the SU(2) part: Re Tr(r w) = k Re Tr(r v)
    for random r in SU(2) (so its convention cannot be wrong in the same way
    as the oracle's without failing here)."""
    rng = np.random.Generator(np.random.PCG64(3))
    W = si.random_su3(1, 5)[0] @ (si.random_su3(1, 6)[0] + 0.7 * si.random_su3(1, 7)[0])
    for i, j in SUBGROUPS:
        k, v, w = _su2_part(W, i, j)
        assert abs(np.linalg.det(v) - 1) < 1e-14 and np.allclose(v @ v.conj().T, np.eye(2), atol=1e-14)
        for _ in range(5):
            q = rng.standard_normal(4)
            q /= np.linalg.norm(q)
            r = np.array([[q[0] + 1j * q[3], q[2] + 1j * q[1]], [-q[2] + 1j * q[1], q[0] - 1j * q[3]]])
            assert abs(np.trace(r @ w).real - k * np.trace(r @ v).real) < 1e-13


@pytest.mark.slow
@pytest.mark.parametrize("sampler", [0, 1])
def test_full_heat_bath_update_laws(orc, sampler):
    """Through the full one-link update on a 2^4 lattice with a frozen
    staple: the new link is R_(0,2) R_(1,2) R_(0,1) U with each R the
    identity but for its 2x2 block r; g = r v is in SU(2); g0 follows
    sqrt(1-x^2) exp(alpha x) with alpha = 2 beta k / 3 (k recomputed from W
    after the earlier subgroups); the direction of g is uniform."""
    d = [2, 2, 2, 2]
    U0 = si.random_field(d, 31)
    site, mu, beta = 5, 2, 6.0
    n = 40_000
    out, recs, exs = _run_link(orc, d, U0, site, mu, beta, n, sampler=sampler, max_tries=4096)
    assert np.all(exs == 0) and np.all(recs[:, :, 1] == 1)
    A = _cx(orc.staple(d, U0, site, mu))
    g0s = np.empty((n, 3))
    alphas = np.empty((n, 3))
    dirs = np.empty((n, 3, 3))
    for s in range(n):
        u = _cx(U0[site, mu]).copy()
        W = u @ A
        for sg, (i, j) in enumerate(SUBGROUPS):
            k, v, _ = _su2_part(W, i, j)
            rc = recs[s, sg]
            assert abs(rc[0] - k) < 1e-12 * k
            r = (rc[3::2] + 1j * rc[4::2]).reshape(2, 2)
            g = r @ v
            assert abs(g[1, 1] - np.conj(g[0, 0])) < 1e-13 and abs(g[1, 0] + np.conj(g[0, 1])) < 1e-13
            assert abs(abs(g[0, 0]) ** 2 + abs(g[0, 1]) ** 2 - 1) < 1e-13
            g0s[s, sg] = g[0, 0].real
            alphas[s, sg] = 2 * beta * k / 3
            gv = np.array([g[0, 1].imag, g[0, 1].real, g[0, 0].imag])
            dirs[s, sg] = gv / np.linalg.norm(gv)
            R = _embed(r, i, j)
            u = R @ u
            W = R @ W
        assert np.max(np.abs(u - out[s])) < 1e-13
    assert np.allclose(alphas[:, 0], recs[:, 0, 2], rtol=1e-13)
    for sg in range(3):
        pit = _g0_cdf(g0s[:, sg], alphas[:, sg])
        assert _uniform_chi2_p(pit, 0, 1) > 1e-3, sg
        assert _uniform_chi2_p(dirs[:, sg, 2], -1, 1) > 1e-3, sg
        assert _uniform_chi2_p(np.arctan2(dirs[:, sg, 1], dirs[:, sg, 0]), -np.pi, np.pi) > 1e-3, sg
    # alpha varies from sample to sample after the first subgroup
    assert np.std(alphas[:, 1]) > 0.01 and np.std(alphas[:, 0]) == 0


@pytest.mark.slow
def test_full_update_exhaustion_count(orc):
    """With one KP trial per draw, a subgroup whose trial is rejected keeps
    its value: the count returned is the number of such steps, and for the
    first subgroup (fixed alpha) their rate is 1 - acceptance, with the
    acceptance the ratio of the target and proposal integrals."""
    d = [2, 2, 2, 2]
    U0 = si.random_field(d, 32)
    site, mu, beta = 11, 1, 1.0
    n = 40_000
    out, recs, exs = _run_link(orc, d, U0, site, mu, beta, n, max_tries=1)
    assert np.array_equal(exs, np.sum(recs[:, :, 1] == 0, axis=1))
    assert np.all(recs[:, :, 1] >= 0)
    rej = recs[:, :, 1] == 0
    # steps that were rejected apply nothing
    assert np.all(recs[rej][:, 3:] == 0)
    none = np.all(rej, axis=1)
    assert np.all(np.abs(out[none] - _cx(U0[site, mu])) == 0)
    alpha = recs[0, 0, 2]
    target = integrate.quad(lambda x: np.sqrt(x * (2 - x)) * np.exp(-alpha * x), 0, 2)[0]
    proposal = integrate.quad(lambda x: np.sqrt(2 * x) * np.exp(-alpha * x), 0, np.inf)[0]
    acc = target / proposal
    rate = 1 - rej[:, 0].mean()
    assert abs(rate - acc) < 5 * np.sqrt(acc * (1 - acc) / n), (rate, acc)


def _weyl_retr_bins(c, nb=20, n=1024):
    """Equal-probability bins of x = Re Tr U and their edges under the weight
    exp(c x) on Haar SU(3), from the eigenphase torus with the Vandermonde
    density (periodic trapezoid rule)."""
    th = 2 * np.pi * np.arange(n) / n
    t1, t2 = np.meshgrid(th, th, indexing="ij")
    t3 = -t1 - t2
    z = [np.exp(1j * t) for t in (t1, t2, t3)]
    vdm = np.abs(z[0] - z[1]) ** 2 * np.abs(z[0] - z[2]) ** 2 * np.abs(z[1] - z[2]) ** 2
    x = (np.cos(t1) + np.cos(t2) + np.cos(t3)).ravel()
    w = (vdm.ravel() * np.exp(c * (x - 3)))
    o = np.argsort(x)
    cw = np.cumsum(w[o]) / np.sum(w)
    edges = np.concatenate([[-1.6], np.interp(np.arange(1, nb) / nb, cw, x[o]), [3.0]])
    mean = float(np.sum(w * x) / np.sum(w))
    return edges, mean, vdm, x


def test_weyl_quadrature_reproduces_haar_moments():
    """The quadrature used for the single-link law: <Re Tr U> = 0 and
    <|Tr U|^2> = 1 on Haar SU(3)."""
    _, mean, vdm, x = _weyl_retr_bins(0.0, n=256)
    n = 256
    th = 2 * np.pi * np.arange(n) / n
    t1, t2 = np.meshgrid(th, th, indexing="ij")
    tr = np.exp(1j * t1) + np.exp(1j * t2) + np.exp(-1j * (t1 + t2))
    assert abs(mean) < 1e-12
    assert abs(np.sum(vdm * np.abs(tr) ** 2) / np.sum(vdm) - 1) < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("beta", [0.5, 2.0])
def test_single_link_chain_samples_the_local_law(orc, beta):
    """On a cold 2^4 lattice the staple of any link is 6 times the identity,
    so repeated full heat-bath updates of one link (independent streams per
    chain) sample exp((beta/3) Re Tr(U A)) = exp(2 beta Re Tr U) on SU(3):
    the histogram of Re Tr U matches that law, computed by Weyl's
    integration formula, on equal-probability bins."""
    d = [2, 2, 2, 2]
    site, mu = 3, 1
    U = orc.init_cold(d)
    A = _cx(orc.staple(d, U, site, mu))
    assert np.allclose(A, 6 * np.eye(3), atol=1e-14)
    nchain, steps = 12_000, 6
    starts = si.random_su3(nchain, 91)
    x = np.empty(nchain)
    for c in range(nchain):
        U[site, mu, ..., 0] = starts[c].real
        U[site, mu, ..., 1] = starts[c].imag
        for s in range(steps):
            orc.hb_link(d, U, site, mu, beta, 5, c, s)
        x[c] = np.trace(_cx(U[site, mu])).real
    edges, mean, _, _ = _weyl_retr_bins(2 * beta)
    cnt, _ = np.histogram(x, bins=edges)
    e = nchain / (len(edges) - 1)
    p = stats.chi2.sf(np.sum((cnt - e) ** 2 / e), len(edges) - 2)
    assert p > 1e-3, (p, cnt)
    assert abs(x.mean() - mean) < 4 * x.std() / np.sqrt(nchain), (x.mean(), mean)
