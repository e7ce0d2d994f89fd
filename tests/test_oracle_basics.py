"""Oracle pins: Philox, uniform map, Haar start, SU(3) arithmetic, plaquette,
staple orientation and gauge invariance (Sec. III definitions)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth_inputs as si

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_blocks(tuples, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers or g++ not available")
    exe = str(tmp_path / "probe")
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           os.path.join(HERE, "rocrand_philox_probe.cpp"), "-o", exe])
    args = [str(x) for t in tuples for x in t]
    out = subprocess.check_output([exe] + args, text=True).split("\n")
    return [list(map(int, line.split())) for line in out if line.strip()]


def test_philox_matches_rocrand(orc, tmp_path):
    """The oracle's Philox4x32-10 equals rocRAND's block function (an
    independent implementation of the same published generator)."""
    rng = np.random.Generator(np.random.PCG64(11))
    tuples = [(0, 0, 0, 0, 0, 0), (1, 2, 3, 4, 5, 6), (0xFFFFFFFF,) * 6]
    tuples += [tuple(int(x) for x in rng.integers(0, 2**32, 6, dtype=np.uint64)) for _ in range(40)]
    ref = _rocrand_blocks(tuples, tmp_path)
    for t, r in zip(tuples, ref):
        assert list(orc.philox(t[:4], t[4:])) == r


def test_philox_bits_uniform(orc):
    """Counter sweep gives unbiased bits (mean of each of the 32 bits)."""
    bits = np.zeros(32)
    n = 4000
    for c in range(n):
        o = orc.philox([c, 7, 0, 0], [3, 0])
        for w in o:
            bits += (int(w) >> np.arange(32)) & 1
    frac = bits / (4 * n)
    assert np.all(np.abs(frac - 0.5) < 5 * 0.5 / np.sqrt(4 * n))


def test_u01_map(orc):
    """u = (2*(x>>9)+1) 2^-24: open interval, exactly representable in fp32."""
    assert orc.u01(0) == 2.0**-24
    assert orc.u01(0xFFFFFFFF) == 1.0 - 2.0**-24
    for x in [0, 1, 511, 512, 12345678, 0x80000000, 0xFFFFFFFF]:
        u = orc.u01(x)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u


def test_cold_start(orc):
    d = [4, 4, 4, 4]
    U = orc.init_cold(d)
    assert orc.plaquette(d, U) == 1.0
    assert orc.action(d, U, 6.0) == 0.0
    assert orc.max_su3_dev(d, U) == 0.0


def test_hot_start_is_su3_and_haar(orc):
    """Haar moments of SU(3): <Tr U> = 0, <|Tr U|^2> = 1, <(Tr U)^3> = 1
    (det = 1; it would be 0 for U(3)), <|Tr U|^4> = 2."""
    d = [16, 16, 8, 8]
    U = orc.init_hot(d, 5, 0)
    assert orc.max_su3_dev(d, U) < 1e-14
    t = np.trace(orc.as_complex(U), axis1=2, axis2=3).ravel()
    n = t.size
    assert abs(np.mean(t)) < 5 * np.sqrt(1.0 / n)
    assert abs(np.mean(np.abs(t) ** 2) - 1.0) < 5 * np.sqrt(1.0 / n)
    m3 = np.mean(t**3)
    assert abs(m3.real - 1.0) < 5 * np.sqrt(6.0 / n) and abs(m3.imag) < 5 * np.sqrt(6.0 / n)
    assert abs(np.mean(np.abs(t) ** 4) - 2.0) < 5 * np.sqrt(22.0 / n)
    # different seeds and lattice ids give different fields, same seed the same
    assert np.array_equal(U, orc.init_hot(d, 5, 0))
    assert not np.array_equal(U[:10], orc.init_hot(d, 5, 1)[:10])


def test_hot_start_rows_are_gram_schmidt_of_gaussians(orc):
    """Rows 0,1 of a hot-start link are Gram-Schmidt orthonormalized complex
    Gaussians drawn from Philox (purpose INIT); checked for one link from
    the raw Philox words through Box-Muller written out here."""
    d = [2, 2, 2, 2]
    U = orc.as_complex(orc.init_hot(d, 9, 3))
    site, mu = 5, 2
    z = []
    for draw in range(3):
        w = orc.philox([site, (1 << 28) | (mu << 24) | draw, 0, 0], [9, 3])
        u = [orc.u01(int(x)) for x in w]
        for h in range(2):
            r = np.sqrt(-2 * np.log(u[2 * h]))
            z += [r * np.cos(2 * np.pi * u[2 * h + 1]), r * np.sin(2 * np.pi * u[2 * h + 1])]
    r0 = np.array(z[0:6:2]) + 1j * np.array(z[1:6:2])
    r1 = np.array(z[6:12:2]) + 1j * np.array(z[7:12:2])
    q, _ = np.linalg.qr(np.stack([r0, r1], axis=1))
    # QR gives the same orthonormal rows up to a phase per row
    for k in range(2):
        ph = np.vdot(q[:, k], U[site, mu, k])
        assert abs(abs(ph) - 1) < 1e-12
        np.testing.assert_allclose(U[site, mu, k], ph * q[:, k], atol=1e-12)
    assert abs(np.linalg.det(U[site, mu]) - 1) < 1e-13


def test_plaquette_numpy_and_gauge_invariance(orc):
    """Plaquette and action are gauge invariant; the plaquette equals a
    vectorized numpy evaluation via np.roll."""
    d = [4, 4, 2, 6]
    U = si.random_field(d, 3)
    p0 = orc.plaquette(d, U)
    s0 = orc.action(d, U, 5.7)
    assert abs(s0 - 5.7 * 6 * np.prod(d) * (1 - p0)) < 1e-9
    M = orc.as_complex(U).reshape(d[3], d[2], d[1], d[0], 4, 3, 3)

    def shift(A, mu):  # A(n + e_mu)
        ax = 3 - mu
        return np.roll(A, -1, axis=ax)

    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = M[..., mu, :, :]
            b = shift(M[..., nu, :, :], mu)
            c = np.conj(np.swapaxes(shift(M[..., mu, :, :], nu), -1, -2))
            e = np.conj(np.swapaxes(M[..., nu, :, :], -1, -2))
            tot += np.trace(a @ b @ c @ e, axis1=-2, axis2=-1).real.sum() / 3
    assert abs(tot / (6 * np.prod(d)) - p0) < 1e-13
    orc.gauge_transform(d, U, 77)
    assert orc.max_su3_dev(d, U) < 1e-13
    assert abs(orc.plaquette(d, U) - p0) < 1e-13
    assert abs(orc.action(d, U, 5.7) - s0) < 1e-9 * abs(s0)


def test_staple_gives_local_action(orc):
    """Re Tr(U_mu(n) A_mu(n)) equals the sum of the six plaquettes that
    contain U_mu(n) (found by differencing the action), and the staple is
    gauge covariant: A -> Om(n+mu) A Om(n)^+, checked through Re Tr(U A)."""
    d = [4, 2, 4, 2]
    U = si.random_field(d, 21)
    rng = np.random.Generator(np.random.PCG64(2))
    for _ in range(6):
        site, mu = int(rng.integers(0, np.prod(d))), int(rng.integers(0, 4))
        A = orc.staple(d, U, site, mu)
        A = A[..., 0] + 1j * A[..., 1]
        u = U[site, mu, ..., 0] + 1j * U[site, mu, ..., 1]
        loc = np.trace(u @ A).real
        # action difference when the link is replaced by a random SU(3) element
        V2 = U.copy()
        r = si.random_su3(1, site + 17 * mu)[0]
        V2[site, mu] = np.stack([r.real, r.imag], axis=-1)
        dS = orc.action(d, V2, 3.0) - orc.action(d, U, 3.0)
        loc2 = np.trace(r @ A).real
        assert abs(dS - (-(3.0 / 3.0) * (loc2 - loc))) < 1e-11
    W = U.copy()
    orc.gauge_transform(d, W, 5)
    for site in range(0, np.prod(d), 7):
        for mu in range(4):
            a0 = orc.staple(d, U, site, mu)
            a1 = orc.staple(d, W, site, mu)
            u0 = orc.as_complex(U[site, mu][None])[0]
            u1 = orc.as_complex(W[site, mu][None])[0]
            t0 = np.trace(u0 @ (a0[..., 0] + 1j * a0[..., 1])).real
            t1 = np.trace(u1 @ (a1[..., 0] + 1j * a1[..., 1])).real
            assert abs(t0 - t1) < 1e-12


def test_reunitarize_restores_su3(orc):
    d = [2, 2, 2, 2]
    U = si.random_field(d, 4)
    U2 = U * (1 + 1e-3)
    U2[..., 2, :, :] += 1e-3
    orc.reunitarize(d, U2)
    assert orc.max_su3_dev(d, U2) < 1e-14
    orc.reunitarize(d, U)
    # a field already in SU(3) is unchanged to rounding, row 2 rebuilt from rows 0,1
    np.testing.assert_allclose(U, si.random_field(d, 4), atol=1e-14)


def test_fixed_sequence_elementary_functions(orc):
    """The oracle's own ln, exp and (cos, sin)(2 pi u), used for every random
    draw, agree with the C library to a few ulp over their ranges of use."""
    rng = np.random.Generator(np.random.PCG64(17))
    xs = np.concatenate([rng.random(4000), 2.0 ** -rng.uniform(0, 24, 2000), [2.0**-24, 0.5, 1 - 2.0**-24, 1.0]])
    for x in xs:
        ref = np.log(x)
        assert abs(orc.det_ln(x) - ref) <= 4 * np.spacing(max(abs(ref), 1e-300)) + 1e-300, x
    for y in np.concatenate([-rng.uniform(0, 60, 3000), [0.0, -1e-12, -700.0]]):
        ref = np.exp(y)
        assert abs(orc.det_exp(y) - ref) <= 4 * np.spacing(ref), y
    us = np.concatenate([rng.random(4000), [0.0, 0.125, 0.25, 0.5, 0.75, 1.0 - 2.0**-24]])
    two_pi = 2 * np.longdouble("3.14159265358979323846264338327950288")
    for u in us:
        c, s = orc.det_cossin_2pi(u)
        ang = two_pi * np.longdouble(u)  # x87 extended precision reference
        assert abs(c - float(np.cos(ang))) < 2.3e-16 and abs(s - float(np.sin(ang))) < 2.3e-16, u
