/*
 * su3_oracle.c -- plain, slow, FP64 CPU reference for the rethermalization
 * path of the multiscale thermalization method for pure SU(3) Yang-Mills
 * theory (Endres, Brower, Detmold, Orginos, Pochinsky, arXiv:1510.04675).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code with the HIP library:
 * every routine below is written out again from the paper's definitions
 * (and, where the paper is silent, from the readings listed in the design
 * notes), in sequential loops with C99 complex arithmetic.
 *
 * Field layout (host exchange format): double[V][4][3][3][2], site index
 * i = n0 + L0*(n1 + L1*(n2 + L2*n3)) with n0 fastest, then direction mu,
 * then the 3x3 matrix row-major, then (re, im).
 *
 * Parity notes: every function is pinned by the tests under tests/ against
 * closed forms, invariants, brute force or an independent library; one with
 * no such check would say "parity unpinned" in its comment.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cx;
typedef struct { cx e[3][3]; } mat3;
typedef struct { int L[4]; int64_t V; } geom;

#define PI 3.14159265358979323846

/* RNG purposes (counter word 1, bits 28..31). */
enum { P_INIT = 1, P_HB = 2, P_HB_DIR = 3, P_MOM = 4, P_ACCEPT = 5, P_GAUGE = 6, P_PARAM = 7 };
enum { SAMPLER_KP = 0, SAMPLER_CREUTZ = 1 };

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the  */
/* 4x32 round function; the key is bumped by the two Weyl constants     */
/* between rounds.                                                       */
/* ------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform in (0,1) from the top 23 bits: (2*(x>>9)+1) * 2^-24. */
double orc_u01(uint32_t x) { return ((double)(x >> 9) * 2.0 + 1.0) * 0x1p-24; }

/* ------------------------------------------------------------------ */
/* Elementary functions of the random draws.  Each is a fixed sequence  */
/* of IEEE-754 double operations (no fused multiply-add), so that any   */
/* implementation taking the same steps produces the same bits:         */
/*  ln x:   x = m 2^e with m in [sqrt(1/2), sqrt(2)), s = (m-1)/(m+1),   */
/*          ln m = 2 s (1 + s^2/3 + ... + s^22/23) summed by Horner in   */
/*          s^2, ln x = e ln2_hi + (e ln2_lo + ln m).                    */
/*  cos, sin of 2 pi u (u in [0,1]): q = nearest integer to 4u,          */
/*          v = u - q/4, t = 2 pi v in [-pi/4, pi/4], Taylor series of   */
/*          cos t to t^18 and sin t to t^19 by Horner in t^2, then q     */
/*          quarter turns.                                               */
/*  exp y:  n = nearest integer to y/ln2, r = (y - n ln2_hi) - n ln2_lo, */
/*          Taylor series to r^17 by Horner, times 2^n.                  */
/* ------------------------------------------------------------------ */
/* ln 2 split so that n * LN2_HI is exact for |n| < 2^11 (Cody-Waite). */
static const double LN2_HI = 0x1.62e42feep-1;
static const double LN2_LO = 0x1.a39ef35793c76p-33;
static const double INV_LN2 = 1.44269504088896340736;
static const double TWO_PI = 6.28318530717958647693;
static const double SQRT_HALF = 0.70710678118654752440;
static const double FACT[21] = { 1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0, 5040.0, 40320.0, 362880.0, 3628800.0,
                                 39916800.0, 479001600.0, 6227020800.0, 87178291200.0, 1307674368000.0,
                                 20922789888000.0, 355687428096000.0, 6402373705728000.0,
                                 121645100408832000.0, 2432902008176640000.0 };

double orc_ln(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < SQRT_HALF) {
        m = 2.0 * m;
        e -= 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 23.0;
    for (int k = 10; k >= 0; k--) p = p * z + 1.0 / (double)(2 * k + 1);
    double de = (double)e;
    return de * LN2_HI + (de * LN2_LO + 2.0 * s * p);
}

void orc_cossin_2pi(double u, double* c, double* s)
{
    double q = floor(4.0 * u + 0.5);
    double v = u - 0.25 * q;
    double t = TWO_PI * v;
    double t2 = t * t;
    double ps = -1.0 / FACT[19];
    for (int k = 8; k >= 0; k--) ps = ps * t2 + ((k & 1) ? -1.0 : 1.0) / FACT[2 * k + 1];
    double pc = -1.0 / FACT[18];
    for (int k = 8; k >= 0; k--) pc = pc * t2 + ((k & 1) ? -1.0 : 1.0) / FACT[2 * k];
    double s0 = t * ps, c0 = pc;
    switch (((int)q) & 3) {
    case 0: *c = c0; *s = s0; break;
    case 1: *c = -s0; *s = c0; break;
    case 2: *c = -c0; *s = -s0; break;
    default: *c = s0; *s = -c0; break;
    }
}

double orc_exp(double y)
{
    if (y < -745.0) return 0.0;
    double n = floor(y * INV_LN2 + 0.5);
    double r = (y - n * LN2_HI) - n * LN2_LO;
    double p = 1.0 / FACT[17];
    for (int k = 16; k >= 0; k--) p = p * r + 1.0 / FACT[k];
    return ldexp(p, (int)n);
}

static uint32_t word1(int purpose, int mu, int sub, int hit, int draw)
{
    return ((uint32_t)purpose << 28) | ((uint32_t)mu << 24) | ((uint32_t)sub << 20) |
           ((uint32_t)hit << 12) | (uint32_t)draw;
}

/* Four uniforms from one Philox call. */
static void uniforms4(uint32_t seed, uint32_t lid, uint32_t c0, uint32_t c1, uint64_t c23, double u[4])
{
    uint32_t ctr[4] = { c0, c1, (uint32_t)c23, (uint32_t)(c23 >> 32) };
    uint32_t key[2] = { seed, lid };
    uint32_t o[4];
    orc_philox(ctr, key, o);
    for (int k = 0; k < 4; k++) u[k] = orc_u01(o[k]);
}

/* Four standard normals from one Philox call (two Box-Muller pairs). */
static void normals4(uint32_t seed, uint32_t lid, uint32_t c0, uint32_t c1, uint64_t c23, double z[4])
{
    double u[4];
    uniforms4(seed, lid, c0, c1, c23, u);
    for (int h = 0; h < 2; h++) {
        double r = sqrt(-2.0 * orc_ln(u[2 * h]));
        double c, s;
        orc_cossin_2pi(u[2 * h + 1], &c, &s);
        z[2 * h] = r * c;
        z[2 * h + 1] = r * s;
    }
}

/* ------------------------------------------------------------------ */
/* Geometry: periodic hypercubic lattice (Sec. III).                   */
/* ------------------------------------------------------------------ */
static geom mkgeom(const int32_t L[4])
{
    geom g;
    g.V = 1;
    for (int m = 0; m < 4; m++) { g.L[m] = L[m]; g.V *= L[m]; }
    return g;
}

static void coords(const geom* g, int64_t i, int n[4])
{
    for (int m = 0; m < 4; m++) { n[m] = (int)(i % g->L[m]); i /= g->L[m]; }
}

static int64_t index_of(const geom* g, const int n[4])
{
    int64_t i = 0;
    for (int m = 3; m >= 0; m--) {
        int c = ((n[m] % g->L[m]) + g->L[m]) % g->L[m];
        i = i * g->L[m] + c;
    }
    return i;
}

/* Site index of n + s*e_mu. */
static int64_t hop(const geom* g, int64_t i, int mu, int s)
{
    int n[4];
    coords(g, i, n);
    n[mu] += s;
    return index_of(g, n);
}

static int parity_of(const geom* g, int64_t i)
{
    int n[4];
    coords(g, i, n);
    return (n[0] + n[1] + n[2] + n[3]) & 1;
}

/* ------------------------------------------------------------------ */
/* 3x3 complex matrices.                                               */
/* ------------------------------------------------------------------ */
static mat3 ld(const double* U, int64_t i, int mu)
{
    mat3 m;
    const double* p = U + (i * 4 + mu) * 18;
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) m.e[r][c] = p[(r * 3 + c) * 2] + I * p[(r * 3 + c) * 2 + 1];
    return m;
}

static void st(double* U, int64_t i, int mu, const mat3* m)
{
    double* p = U + (i * 4 + mu) * 18;
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            p[(r * 3 + c) * 2] = creal(m->e[r][c]);
            p[(r * 3 + c) * 2 + 1] = cimag(m->e[r][c]);
        }
}

static mat3 m_zero(void) { mat3 m; memset(&m, 0, sizeof m); return m; }
static mat3 m_one(void) { mat3 m = m_zero(); for (int k = 0; k < 3; k++) m.e[k][k] = 1.0; return m; }

static mat3 m_mul(mat3 a, mat3 b)
{
    mat3 c;
    for (int r = 0; r < 3; r++)
        for (int s = 0; s < 3; s++) {
            cx t = 0;
            for (int k = 0; k < 3; k++) t += a.e[r][k] * b.e[k][s];
            c.e[r][s] = t;
        }
    return c;
}

static mat3 m_dag(mat3 a)
{
    mat3 c;
    for (int r = 0; r < 3; r++)
        for (int s = 0; s < 3; s++) c.e[r][s] = conj(a.e[s][r]);
    return c;
}

static mat3 m_add(mat3 a, mat3 b)
{
    for (int r = 0; r < 3; r++)
        for (int s = 0; s < 3; s++) a.e[r][s] += b.e[r][s];
    return a;
}

static mat3 m_sub(mat3 a, mat3 b)
{
    for (int r = 0; r < 3; r++)
        for (int s = 0; s < 3; s++) a.e[r][s] -= b.e[r][s];
    return a;
}

static mat3 m_scale(mat3 a, cx f)
{
    for (int r = 0; r < 3; r++)
        for (int s = 0; s < 3; s++) a.e[r][s] *= f;
    return a;
}

static cx m_tr(mat3 a) { return a.e[0][0] + a.e[1][1] + a.e[2][2]; }

static cx m_det(mat3 a)
{
    return a.e[0][0] * (a.e[1][1] * a.e[2][2] - a.e[1][2] * a.e[2][1]) -
           a.e[0][1] * (a.e[1][0] * a.e[2][2] - a.e[1][2] * a.e[2][0]) +
           a.e[0][2] * (a.e[1][0] * a.e[2][1] - a.e[1][1] * a.e[2][0]);
}

static double m_norm(mat3 a)
{
    double s = 0;
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) s += creal(a.e[r][c] * conj(a.e[r][c]));
    return sqrt(s);
}

/* Unitarize from the first two rows: normalize row 0, orthogonalize row 1
 * against it and normalize, row 2 = complex conjugate of row0 x row1.
 * This is the unique SU(3) completion of two orthonormal rows. */
static mat3 m_reunit(mat3 a)
{
    double n0 = 0;
    for (int c = 0; c < 3; c++) n0 += creal(a.e[0][c] * conj(a.e[0][c]));
    n0 = 1.0 / sqrt(n0);
    for (int c = 0; c < 3; c++) a.e[0][c] *= n0;
    cx ip = 0;
    for (int c = 0; c < 3; c++) ip += conj(a.e[0][c]) * a.e[1][c];
    for (int c = 0; c < 3; c++) a.e[1][c] -= ip * a.e[0][c];
    double n1 = 0;
    for (int c = 0; c < 3; c++) n1 += creal(a.e[1][c] * conj(a.e[1][c]));
    n1 = 1.0 / sqrt(n1);
    for (int c = 0; c < 3; c++) a.e[1][c] *= n1;
    for (int c = 0; c < 3; c++) {
        int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        a.e[2][c] = conj(a.e[0][c1] * a.e[1][c2] - a.e[0][c2] * a.e[1][c1]);
    }
    return a;
}

/* exp(X) by its Taylor series, summed until the term is below 1e-17
 * relative to the running sum (at most 200 terms). */
static mat3 m_exp(mat3 X)
{
    mat3 s = m_one(), t = m_one();
    for (int k = 1; k <= 200; k++) {
        t = m_scale(m_mul(t, X), 1.0 / k);
        s = m_add(s, t);
        if (m_norm(t) < 1e-17 * m_norm(s)) break;
    }
    return s;
}

/* Gell-Mann matrices lambda^a, a = 1..8 (index a-1). T^a = lambda^a / 2. */
static mat3 gellmann(int a)
{
    mat3 m = m_zero();
    switch (a) {
    case 1: m.e[0][1] = 1; m.e[1][0] = 1; break;
    case 2: m.e[0][1] = -I; m.e[1][0] = I; break;
    case 3: m.e[0][0] = 1; m.e[1][1] = -1; break;
    case 4: m.e[0][2] = 1; m.e[2][0] = 1; break;
    case 5: m.e[0][2] = -I; m.e[2][0] = I; break;
    case 6: m.e[1][2] = 1; m.e[2][1] = 1; break;
    case 7: m.e[1][2] = -I; m.e[2][1] = I; break;
    case 8: {
        double f = 1.0 / sqrt(3.0);
        m.e[0][0] = f; m.e[1][1] = f; m.e[2][2] = -2.0 * f;
        break;
    }
    }
    return m;
}

/* ------------------------------------------------------------------ */
/* Field initialisation.                                               */
/* ------------------------------------------------------------------ */
void orc_init_cold(const int32_t L[4], double* U)
{
    geom g = mkgeom(L);
    mat3 one = m_one();
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++) st(U, i, mu, &one);
}

/* Haar-random SU(3) element from twelve normals: rows 0 and 1 are complex
 * Gaussian vectors, orthonormalized; row 2 completes to det = 1. */
static mat3 haar_from_normals(const double z[12])
{
    mat3 m = m_zero();
    for (int c = 0; c < 3; c++) {
        m.e[0][c] = z[2 * c] + I * z[2 * c + 1];
        m.e[1][c] = z[6 + 2 * c] + I * z[6 + 2 * c + 1];
    }
    return m_reunit(m);
}

void orc_init_hot(const int32_t L[4], double* U, uint32_t seed, uint32_t lid)
{
    geom g = mkgeom(L);
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++) {
            double z[12];
            for (int d = 0; d < 3; d++) normals4(seed, lid, (uint32_t)i, word1(P_INIT, mu, 0, 0, d), 0, z + 4 * d);
            mat3 m = haar_from_normals(z);
            st(U, i, mu, &m);
        }
}

void orc_reunitarize(const int32_t L[4], double* U)
{
    geom g = mkgeom(L);
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++) {
            mat3 m = m_reunit(ld(U, i, mu));
            st(U, i, mu, &m);
        }
}

/* Random gauge transformation U_mu(n) -> Om(n) U_mu(n) Om(n+mu)^dagger with
 * Haar-random Om(n) from Philox purpose GAUGE (a test utility). */
void orc_gauge_transform(const int32_t L[4], double* U, uint32_t seed)
{
    geom g = mkgeom(L);
    mat3* om = (mat3*)malloc(sizeof(mat3) * (size_t)g.V);
    for (int64_t i = 0; i < g.V; i++) {
        double z[12];
        for (int d = 0; d < 3; d++) normals4(seed, 0, (uint32_t)i, word1(P_GAUGE, 0, 0, 0, d), 0, z + 4 * d);
        om[i] = haar_from_normals(z);
    }
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++) {
            mat3 m = m_mul(m_mul(om[i], ld(U, i, mu)), m_dag(om[hop(&g, i, mu, +1)]));
            st(U, i, mu, &m);
        }
    free(om);
}

/* ------------------------------------------------------------------ */
/* Wilson action and plaquettes (Sec. III, Wilson action and loops).   */
/* ------------------------------------------------------------------ */
static mat3 plaq_mat(const geom* g, const double* U, int64_t i, int mu, int nu)
{
    int64_t ipm = hop(g, i, mu, +1), ipn = hop(g, i, nu, +1);
    return m_mul(m_mul(m_mul(ld(U, i, mu), ld(U, ipm, nu)), m_dag(ld(U, ipn, mu))), m_dag(ld(U, i, nu)));
}

/* Average plaquette: (1/(6V)) sum_n sum_{mu<nu} (1/3) Re Tr U_munu(n). */
/* Compensated (Neumaier) summation.  Plaquette, action and kinetic energy
 * add up 10^6 - 10^8 terms, and the Metropolis test needs the difference of
 * two such sums: plain accumulation would lose about sqrt(n) ulps of the
 * total, a compensated sum keeps the error near one ulp. */
typedef struct {
    double s, c;
} ksum;

static void ks_add(ksum* k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x))
        k->c += (k->s - t) + x;
    else
        k->c += (x - t) + k->s;
    k->s = t;
}

static double ks_val(const ksum* k) { return k->s + k->c; }

double orc_plaquette(const int32_t L[4], const double* U)
{
    geom g = mkgeom(L);
    ksum s = { 0, 0 };
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) ks_add(&s, creal(m_tr(plaq_mat(&g, U, i, mu, nu))) / 3.0);
    return ks_val(&s) / (6.0 * (double)g.V);
}

/* Wilson action S = beta sum_n sum_{mu<nu} [1 - (1/3) Re Tr U_munu(n)]. */
double orc_action(const int32_t L[4], const double* U, double beta)
{
    geom g = mkgeom(L);
    ksum s = { 0, 0 };
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) ks_add(&s, 1.0 - creal(m_tr(plaq_mat(&g, U, i, mu, nu))) / 3.0);
    return beta * ks_val(&s);
}

/* Staple sum A_mu(n): for nu != mu ascending, the forward term
 * U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+ then the backward term
 * U_nu(n+mu-nu)^+ U_mu(n-nu)^+ U_nu(n-nu), so that Re Tr(U_mu(n) A_mu(n)) is
 * the sum of the six plaquettes that contain U_mu(n).  These are the
 * daggered staples T^+ and T^- of the APE step in Sec. III (with the
 * gauge-covariant reading of T^-). */
static mat3 staple(const geom* g, const double* U, int64_t i, int mu)
{
    mat3 A = m_zero();
    int64_t ipm = hop(g, i, mu, +1);
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        int64_t ipn = hop(g, i, nu, +1);
        int64_t imn = hop(g, i, nu, -1);
        int64_t ipm_mn = hop(g, ipm, nu, -1);
        mat3 f = m_mul(m_mul(ld(U, ipm, nu), m_dag(ld(U, ipn, mu))), m_dag(ld(U, i, nu)));
        mat3 b = m_mul(m_mul(m_dag(ld(U, ipm_mn, nu)), m_dag(ld(U, imn, mu))), ld(U, imn, nu));
        A = m_add(A, f);
        A = m_add(A, b);
    }
    return A;
}

void orc_staple(const int32_t L[4], const double* U, int64_t site, int mu, double* out)
{
    geom g = mkgeom(L);
    mat3 A = staple(&g, U, site, mu);
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            out[(r * 3 + c) * 2] = creal(A.e[r][c]);
            out[(r * 3 + c) * 2 + 1] = cimag(A.e[r][c]);
        }
}

/* ------------------------------------------------------------------ */
/* Cabibbo-Marinari heat bath and overrelaxation (Sec. IV.A).          */
/* ------------------------------------------------------------------ */
static const int SUB_I[3] = { 0, 1, 0 };
static const int SUB_J[3] = { 1, 2, 2 };

/* Draw g0 with density proportional to sqrt(1-g0^2) exp(alpha g0) on [-1,1].
 * Kennedy-Pendleton: delta = 1 - g0 is proposed from a Gamma(3/2) law with
 * rate alpha (an exponential plus a squared half-normal) and accepted with
 * probability sqrt(1 - delta/2).  Creutz: g0 from the truncated exponential
 * exp(alpha g0) by inversion, accepted with probability sqrt(1 - g0^2).
 * Trial t uses the Philox counter (c0, word(P_HB, mu, sub, hit, t), sweep).
 * Returns 1 and sets *g0 on acceptance; 0 if max_tries trials all failed. */
static int sample_g0(double alpha, int sampler, int max_tries, uint32_t seed, uint32_t lid, uint32_t c0,
                     int mu, int sub, int hit, uint64_t sweep, double* g0)
{
    for (int t = 0; t < max_tries; t++) {
        double u[4];
        uniforms4(seed, lid, c0, word1(P_HB, mu, sub, hit, t), sweep, u);
        if (sampler == SAMPLER_KP) {
            double c, sn;
            orc_cossin_2pi(u[1], &c, &sn);
            double delta = -(orc_ln(u[0]) + c * c * orc_ln(u[2])) / alpha;
            if (u[3] * u[3] <= 1.0 - 0.5 * delta) { *g0 = 1.0 - delta; return 1; }
        } else {
            double e = orc_exp(-2.0 * alpha);
            double x = 1.0 + orc_ln(e + u[0] * (1.0 - e)) / alpha;
            if (u[1] * u[1] <= 1.0 - x * x) { *g0 = x; return 1; }
        }
    }
    return 0;
}

/* Draws of g0 alone, for checking the sampler's distribution: sample k uses
 * the counter of a link at site k, mu = 0, subgroup 0, hit 0, sweep 0. */
int64_t orc_sample_g0(double alpha, int32_t sampler, int32_t max_tries, uint32_t seed, int64_t n, double* out)
{
    int64_t fails = 0;
    for (int64_t k = 0; k < n; k++) {
        double g0 = NAN;
        if (!sample_g0(alpha, sampler, max_tries, seed, 0, (uint32_t)k, 0, 0, 0, 0, &g0)) fails++;
        out[k] = g0;
    }
    return fails;
}

/* The SU(2) part k*v of the (i,j) block of W, with v in SU(2) written as
 * [[x0 + i x3, x2 + i x1], [-x2 + i x1, x0 - i x3]] / k. */
static double su2_part(const mat3* W, int i, int j, cx v[2][2])
{
    double x0 = creal(W->e[i][i] + W->e[j][j]) * 0.5;
    double x3 = cimag(W->e[i][i] - W->e[j][j]) * 0.5;
    double x1 = cimag(W->e[i][j] + W->e[j][i]) * 0.5;
    double x2 = creal(W->e[i][j] - W->e[j][i]) * 0.5;
    double k = sqrt(x0 * x0 + x1 * x1 + x2 * x2 + x3 * x3);
    if (k == 0.0) return 0.0;
    v[0][0] = (x0 + I * x3) / k;
    v[0][1] = (x2 + I * x1) / k;
    v[1][0] = (-x2 + I * x1) / k;
    v[1][1] = (x0 - I * x3) / k;
    return k;
}

/* M <- R M where R is the identity with its (i,j) block replaced by r. */
static void left_apply(mat3* M, int i, int j, cx r[2][2])
{
    for (int c = 0; c < 3; c++) {
        cx a = M->e[i][c], b = M->e[j][c];
        M->e[i][c] = r[0][0] * a + r[0][1] * b;
        M->e[j][c] = r[1][0] * a + r[1][1] * b;
    }
}

/* One link update.  kind 0 = heat bath (hits 0..n_hits-1), 1 = OR.
 * Heat bath for subgroup (i,j): the local weight is exp((beta/3) Re Tr(U A));
 * with W = U A and the new link R U, Re Tr(R W) depends on r only through
 * k Re Tr(r v), so g = r v is drawn with weight exp(alpha g0) on the Haar
 * measure of SU(2), alpha = 2 beta k / 3, and r = g v^+.
 * Overrelaxation: r = (v^+)^2, which leaves Re Tr(r v) and hence the action
 * unchanged.  Returns the number of subgroup draws left unchanged because
 * no trial was accepted. */
static int update_link(const geom* g, double* U, int64_t i, int mu, int kind, double beta, uint32_t seed,
                       uint32_t lid, uint64_t sweep, int n_hits, int max_tries, int sampler, double* rec)
{
    mat3 A = staple(g, U, i, mu);
    mat3 u = ld(U, i, mu);
    mat3 W = m_mul(u, A);
    int exhausted = 0;
    int nh = (kind == 0) ? n_hits : 1;
    for (int h = 0; h < nh; h++)
        for (int s = 0; s < 3; s++) {
            int a = SUB_I[s], b = SUB_J[s];
            cx v[2][2];
            double k = su2_part(&W, a, b, v);
            double* rc = rec ? rec + 11 * (3 * h + s) : NULL;
            if (rc) { memset(rc, 0, 11 * sizeof(double)); rc[0] = k; rc[1] = -1.0; }
            if (k == 0.0) continue;
            cx vd[2][2] = { { conj(v[0][0]), conj(v[1][0]) }, { conj(v[0][1]), conj(v[1][1]) } };
            cx r[2][2];
            if (kind == 0) {
                double alpha = 2.0 * beta * k / 3.0;
                double g0;
                if (rc) rc[2] = alpha;
                if (!sample_g0(alpha, sampler, max_tries, seed, lid, (uint32_t)i, mu, s, h, sweep, &g0)) {
                    exhausted++;
                    if (rc) rc[1] = 0.0;
                    continue;
                }
                double u[4];
                uniforms4(seed, lid, (uint32_t)i, word1(P_HB_DIR, mu, s, h, 0), sweep, u);
                double ct = 2.0 * u[0] - 1.0;
                double stt = sqrt(fmax(0.0, 1.0 - ct * ct));
                double cp, sp;
                orc_cossin_2pi(u[1], &cp, &sp);
                double sr = sqrt(fmax(0.0, 1.0 - g0 * g0));
                double g1 = sr * stt * cp, g2 = sr * stt * sp, g3 = sr * ct;
                cx gm[2][2] = { { g0 + I * g3, g2 + I * g1 }, { -g2 + I * g1, g0 - I * g3 } };
                for (int p = 0; p < 2; p++)
                    for (int q = 0; q < 2; q++) r[p][q] = gm[p][0] * vd[0][q] + gm[p][1] * vd[1][q];
            } else {
                for (int p = 0; p < 2; p++)
                    for (int q = 0; q < 2; q++) r[p][q] = vd[p][0] * vd[0][q] + vd[p][1] * vd[1][q];
            }
            if (rc) {
                rc[1] = 1.0;
                for (int p = 0; p < 2; p++)
                    for (int q = 0; q < 2; q++) {
                        rc[3 + 2 * (2 * p + q)] = creal(r[p][q]);
                        rc[4 + 2 * (2 * p + q)] = cimag(r[p][q]);
                    }
            }
            left_apply(&u, a, b, r);
            left_apply(&W, a, b, r);
        }
    st(U, i, mu, &u);
    return exhausted;
}

/* One checkerboard pass: for mu = 0..3, even sites then odd sites.  Links of
 * one direction and one parity share no plaquette, so within a phase the
 * order of sites is immaterial. */
static int64_t pass(const geom* g, double* U, int kind, double beta, uint32_t seed, uint32_t lid, uint64_t sweep,
                    int n_hits, int max_tries, int sampler)
{
    int64_t exhausted = 0;
    for (int mu = 0; mu < 4; mu++)
        for (int par = 0; par < 2; par++) {
#pragma omp parallel for reduction(+ : exhausted) schedule(static)
            for (int64_t i = 0; i < g->V; i++) {
                if (parity_of(g, i) != par) continue;
                exhausted += update_link(g, U, i, mu, kind, beta, seed, lid, sweep, n_hits, max_tries, sampler, NULL);
            }
        }
    return exhausted;
}

int64_t orc_hb_pass(const int32_t L[4], double* U, double beta, uint32_t seed, uint32_t lid, uint64_t sweep,
                    int32_t n_hits, int32_t max_tries, int32_t sampler)
{
    geom g = mkgeom(L);
    return pass(&g, U, 0, beta, seed, lid, sweep, n_hits, max_tries, sampler);
}

/* The full update of the single link (site, mu) -- heat bath (kind 0, hits
 * 0..n_hits-1) or overrelaxation (kind 1) -- with the counters a pass would
 * use, leaving every other link unchanged (so its staple stays frozen).  If
 * rec is not NULL it receives 11 doubles per (hit, subgroup) step, in step
 * order: k, the outcome (1 applied, 0 all trials rejected, -1 skipped with
 * k = 0), alpha, and the applied 2x2 factor r as (re, im) of r00, r01, r10,
 * r11 (zero unless applied).  Returns the number of exhausted draws. */
int64_t orc_hb_link(const int32_t L[4], double* U, int64_t site, int32_t mu, int32_t kind, double beta,
                    uint32_t seed, uint32_t lid, uint64_t sweep, int32_t n_hits, int32_t max_tries, int32_t sampler,
                    double* rec)
{
    geom g = mkgeom(L);
    return update_link(&g, U, site, mu, kind, beta, seed, lid, sweep, n_hits, max_tries, sampler, rec);
}

void orc_or_pass(const int32_t L[4], double* U)
{
    geom g = mkgeom(L);
    pass(&g, U, 1, 0.0, 0, 0, 0, 1, 1, 0);
}

/* One OR pass with the subgroup order reversed and the reflection applied in
 * reverse; it undoes orc_or_pass link by link (used as a test of OR). */
void orc_or_pass_reversed(const int32_t L[4], double* U)
{
    geom g = mkgeom(L);
    for (int mu = 3; mu >= 0; mu--)
        for (int par = 1; par >= 0; par--)
            for (int64_t i = 0; i < g.V; i++) {
                if (parity_of(&g, i) != par) continue;
                mat3 A = staple(&g, U, i, mu);
                mat3 u = ld(U, i, mu);
                mat3 W = m_mul(u, A);
                for (int s = 2; s >= 0; s--) {
                    int a = SUB_I[s], b = SUB_J[s];
                    cx v[2][2];
                    if (su2_part(&W, a, b, v) == 0.0) continue;
                    cx vd[2][2] = { { conj(v[0][0]), conj(v[1][0]) }, { conj(v[0][1]), conj(v[1][1]) } };
                    cx r[2][2];
                    for (int p = 0; p < 2; p++)
                        for (int q = 0; q < 2; q++) r[p][q] = vd[p][0] * vd[0][q] + vd[p][1] * vd[1][q];
                    left_apply(&u, a, b, r);
                    left_apply(&W, a, b, r);
                }
                st(U, i, mu, &u);
            }
}

/* Sweeps s = first_sweep .. first_sweep+n_sweeps-1; each is one heat-bath
 * pass followed by n_or overrelaxation passes.  With reunit_every > 0 the
 * field is reunitarized after every sweep s with (s+1) % reunit_every == 0,
 * before that sweep's plaquette is recorded.  Returns the number of
 * exhausted subgroup draws. */
int64_t orc_sweep_hb_or(const int32_t L[4], double* U, double beta, uint32_t seed, uint32_t lid,
                        uint64_t first_sweep, int32_t n_sweeps, int32_t n_or, int32_t n_hits,
                        int32_t max_tries, int32_t reunit_every, int32_t sampler, double* plaq_hist)
{
    geom g = mkgeom(L);
    int64_t exhausted = 0;
    for (int32_t k = 0; k < n_sweeps; k++) {
        uint64_t s = first_sweep + (uint64_t)k;
        exhausted += pass(&g, U, 0, beta, seed, lid, s, n_hits, max_tries, sampler);
        for (int o = 0; o < n_or; o++) pass(&g, U, 1, beta, seed, lid, s, 1, 1, sampler);
        if (reunit_every > 0 && (s + 1) % (uint64_t)reunit_every == 0) orc_reunitarize(L, U);
        if (plaq_hist) plaq_hist[k] = orc_plaquette(L, U);
    }
    return exhausted;
}

/* ------------------------------------------------------------------ */
/* HMC (Sec. IV.E and App. A): PQP leapfrog, unit trajectories.         */
/* Momenta p^a (a = 1..8) per link, P = sum_a p^a T^a, T^a = lambda^a/2, */
/* H = (1/2) sum p^a p^a + S(U), dU/dtau = i P U.                       */
/* ------------------------------------------------------------------ */
void orc_hmc_momenta(const int32_t L[4], double* p, uint32_t seed, uint32_t lid, uint64_t traj)
{
    geom g = mkgeom(L);
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++) {
            double z[8];
            normals4(seed, lid, (uint32_t)i, word1(P_MOM, mu, 0, 0, 0), traj, z);
            normals4(seed, lid, (uint32_t)i, word1(P_MOM, mu, 0, 0, 1), traj, z + 4);
            for (int a = 0; a < 8; a++) p[(i * 4 + mu) * 8 + a] = z[a];
        }
}

/* F^a = dS/d omega^a with U -> exp(i omega^a T^a) U.  Since S contains
 * -(beta/3) Re Tr(U A) for the link, F^a = (beta/3) Im Tr(T^a U A). */
void orc_hmc_force(const int32_t L[4], const double* U, double beta, double* F)
{
    geom g = mkgeom(L);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++) {
            mat3 Om = m_mul(ld(U, i, mu), staple(&g, U, i, mu));
            for (int a = 1; a <= 8; a++) {
                mat3 T = m_scale(gellmann(a), 0.5);
                F[(i * 4 + mu) * 8 + a - 1] = beta / 3.0 * cimag(m_tr(m_mul(T, Om)));
            }
        }
}

double orc_hmc_kinetic(const int32_t L[4], const double* p)
{
    geom g = mkgeom(L);
    ksum k = { 0, 0 };
    for (int64_t j = 0; j < g.V * 4 * 8; j++) ks_add(&k, 0.5 * p[j] * p[j]);
    return ks_val(&k);
}

/* U <- exp(i eps P) U for every link. */
static void drift(const geom* g, double* U, const double* p, double eps)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->V; i++)
        for (int mu = 0; mu < 4; mu++) {
            mat3 P = m_zero();
            for (int a = 1; a <= 8; a++) P = m_add(P, m_scale(gellmann(a), 0.5 * p[(i * 4 + mu) * 8 + a - 1]));
            mat3 m = m_mul(m_exp(m_scale(P, I * eps)), ld(U, i, mu));
            st(U, i, mu, &m);
        }
}

static void kick(const int32_t L[4], const double* U, double* p, double beta, double eps, double* F)
{
    geom g = mkgeom(L);
    orc_hmc_force(L, U, beta, F);
    for (int64_t j = 0; j < g.V * 4 * 8; j++) p[j] -= eps * F[j];
}

/* Kick-drift-kick leapfrog with n_steps steps of size eps. */
void orc_md_leapfrog(const int32_t L[4], double* U, double* p, double beta, double eps, int32_t n_steps)
{
    geom g = mkgeom(L);
    double* F = (double*)malloc(sizeof(double) * (size_t)(g.V * 32));
    kick(L, U, p, beta, 0.5 * eps, F);
    for (int32_t k = 0; k < n_steps; k++) {
        drift(&g, U, p, eps);
        kick(L, U, p, beta, (k == n_steps - 1) ? 0.5 * eps : eps, F);
    }
    free(F);
}

/* One trajectory: momenta from Philox (purpose MOM, counter words 2-3 =
 * traj), H0, leapfrog with eps = tau/n_steps, H1, Metropolis with the
 * uniform of Philox purpose ACCEPT (counter word 0 = 0) against exp(-dH);
 * metropolis = 0 accepts unconditionally.  On rejection U is restored. */
int32_t orc_hmc_trajectory(const int32_t L[4], double* U, double beta, double tau, int32_t n_steps, uint32_t seed,
                           uint32_t lid, uint64_t traj, int32_t metropolis, double* dH_out)
{
    geom g = mkgeom(L);
    size_t nU = (size_t)g.V * 72, np = (size_t)g.V * 32;
    double* U0 = (double*)malloc(sizeof(double) * nU);
    double* p = (double*)malloc(sizeof(double) * np);
    memcpy(U0, U, sizeof(double) * nU);
    orc_hmc_momenta(L, p, seed, lid, traj);
    double H0 = orc_hmc_kinetic(L, p) + orc_action(L, U, beta);
    orc_md_leapfrog(L, U, p, beta, tau / n_steps, n_steps);
    double H1 = orc_hmc_kinetic(L, p) + orc_action(L, U, beta);
    double dH = H1 - H0;
    int acc = 1;
    if (metropolis) {
        double u[4];
        uniforms4(seed, lid, 0, word1(P_ACCEPT, 0, 0, 0, 0), traj, u);
        acc = (u[0] < exp(-dH));
    }
    if (!acc) memcpy(U, U0, sizeof(double) * nU);
    if (dH_out) *dH_out = dH;
    free(U0);
    free(p);
    return acc;
}

/* ------------------------------------------------------------------ */
/* Restriction and prolongation (Sec. III, restriction and prolongation */
/* equations, partial actions S_d and the APE step).                    */
/* ------------------------------------------------------------------ */
static int chi_excl(const int n[4], int m1, int m2)
{
    int c = 0;
    for (int m = 0; m < 4; m++)
        if (m != m1 && m != m2) c += n[m] & 1;
    return c;
}

/* U^c_mu(n/2) = U^f_mu(n) U^f_mu(n+e_mu) for every fine site with all
 * coordinates even; fine dims = 2 x coarse dims. */
void orc_restrict(const int32_t Lf[4], const double* Uf, double* Uc)
{
    geom gf = mkgeom(Lf);
    int32_t Lc[4] = { Lf[0] / 2, Lf[1] / 2, Lf[2] / 2, Lf[3] / 2 };
    geom gc = mkgeom(Lc);
    for (int64_t ic = 0; ic < gc.V; ic++) {
        int nc[4], nf[4];
        coords(&gc, ic, nc);
        for (int m = 0; m < 4; m++) nf[m] = 2 * nc[m];
        int64_t i = index_of(&gf, nf);
        for (int mu = 0; mu < 4; mu++) {
            mat3 m = m_mul(ld(Uf, i, mu), ld(Uf, hop(&gf, i, mu, +1), mu));
            st(Uc, ic, mu, &m);
        }
    }
}

/* Transfer: U^f_mu(n) = U^c_mu(n/2), U^f_mu(n+e_mu) = 1 on sites with all
 * coordinates even; every other fine bond starts at 1. */
void orc_prolong_transfer(const int32_t Lc[4], const double* Uc, double* Uf)
{
    int32_t Lf[4] = { 2 * Lc[0], 2 * Lc[1], 2 * Lc[2], 2 * Lc[3] };
    geom gc = mkgeom(Lc), gf = mkgeom(Lf);
    orc_init_cold(Lf, Uf);
    for (int64_t ic = 0; ic < gc.V; ic++) {
        int nc[4], nf[4];
        coords(&gc, ic, nc);
        for (int m = 0; m < 4; m++) nf[m] = 2 * nc[m];
        int64_t i = index_of(&gf, nf);
        for (int mu = 0; mu < 4; mu++) {
            mat3 m = ld(Uc, ic, mu);
            st(Uf, i, mu, &m);
        }
    }
}

/* Partial action S_d = beta sum_n sum_{mu<nu} delta(d, chi_munu(n)) (1 - W_munu(n)). */
double orc_partial_action(const int32_t L[4], const double* U, int32_t d, double beta)
{
    geom g = mkgeom(L);
    /* the six plane terms of every site (in parallel; 0 where chi_munu != d),
     * then summed in site and plane order */
    double* term = (double*)malloc(sizeof(double) * (size_t)g.V * 6);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g.V; i++) {
        int n[4], k = 0;
        coords(&g, i, n);
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++, k++)
                term[i * 6 + k] = (chi_excl(n, mu, nu) == d) ? 1.0 - creal(m_tr(plaq_mat(&g, U, i, mu, nu))) / 3.0 : 0.0;
    }
    double s = 0;
    for (int64_t j = 0; j < g.V * 6; j++) s += term[j];
    free(term);
    return beta * s;
}

/* Projection onto SU(3): the X maximizing Re Tr(X^+ M), found by starting
 * from the unitarized M and repeatedly maximizing over the three SU(2)
 * subgroups (X <- R X, R the SU(2) part of M X^+ in that subgroup), until a
 * round improves Re Tr(X^+ M) by no more than 1e-15 relative, at most 100
 * rounds. */
static mat3 project_su3(mat3 M)
{
    mat3 X = m_reunit(M);
    double f_prev = creal(m_tr(m_mul(m_dag(X), M)));
    for (int it = 0; it < 100; it++) {
        for (int s = 0; s < 3; s++) {
            mat3 Y = m_mul(M, m_dag(X));
            cx v[2][2];
            if (su2_part(&Y, SUB_I[s], SUB_J[s], v) == 0.0) continue;
            left_apply(&X, SUB_I[s], SUB_J[s], v);
        }
        double f = creal(m_tr(m_mul(m_dag(X), M)));
        if (f - f_prev <= 1e-15 * fabs(f)) break;
        f_prev = f;
    }
    return X;
}

void orc_project_su3(const double* Min, double* Xout)
{
    mat3 M;
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) M.e[r][c] = Min[(r * 3 + c) * 2] + I * Min[(r * 3 + c) * 2 + 1];
    mat3 X = project_su3(M);
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            Xout[(r * 3 + c) * 2] = creal(X.e[r][c]);
            Xout[(r * 3 + c) * 2 + 1] = cimag(X.e[r][c]);
        }
}

/* One APE step of stage d on every active bond (chi_mu(n) = d+1) at once:
 * U' = P_SU(3)[U + c sum_{nu: chi_munu(n) = d} (T^+_munu + T^-_munu)] with
 * T^+ = U_nu(n) U_mu(n+nu) U_nu(n+mu)^+ and
 * T^- = U_nu(n-nu)^+ U_mu(n-nu) U_nu(n-nu+mu). */
void orc_ape_step(const int32_t L[4], double* U, int32_t d, double c)
{
    geom g = mkgeom(L);
    size_t nU = (size_t)g.V * 72;
    double* Uold = (double*)malloc(sizeof(double) * nU);
    memcpy(Uold, U, sizeof(double) * nU);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < g.V; i++) {
        int n[4];
        coords(&g, i, n);
        for (int mu = 0; mu < 4; mu++) {
            if (chi_excl(n, mu, mu) != d + 1) continue;
            mat3 M = ld(Uold, i, mu);
            for (int nu = 0; nu < 4; nu++) {
                if (nu == mu || chi_excl(n, mu, nu) != d) continue;
                int64_t ipm = hop(&g, i, mu, +1), ipn = hop(&g, i, nu, +1), imn = hop(&g, i, nu, -1);
                int64_t imn_pm = hop(&g, imn, mu, +1);
                mat3 tp = m_mul(m_mul(ld(Uold, i, nu), ld(Uold, ipn, mu)), m_dag(ld(Uold, ipm, nu)));
                mat3 tm = m_mul(m_mul(m_dag(ld(Uold, imn, nu)), ld(Uold, imn, mu)), ld(Uold, imn_pm, nu));
                M = m_add(M, m_scale(m_add(tp, tm), c));
            }
            mat3 X = project_su3(M);
            st(U, i, mu, &X);
        }
    }
    free(Uold);
}

/* Prolongation: transfer, then for d = 0, 1, 2 repeated APE steps until the
 * partial action S_d changes by no more than rel_tol relative to its previous
 * value (or max_iter steps).  iters[d] receives the number of steps taken. */
int32_t orc_prolongate(const int32_t Lc[4], const double* Uc, double* Uf, double c, double rel_tol,
                       int32_t max_iter, int32_t iters[3])
{
    int32_t Lf[4] = { 2 * Lc[0], 2 * Lc[1], 2 * Lc[2], 2 * Lc[3] };
    orc_prolong_transfer(Lc, Uc, Uf);
    for (int d = 0; d < 3; d++) {
        double s_prev = orc_partial_action(Lf, Uf, d, 1.0);
        int k = 0;
        while (k < max_iter) {
            orc_ape_step(Lf, Uf, d, c);
            k++;
            double s = orc_partial_action(Lf, Uf, d, 1.0);
            int done = fabs(s - s_prev) <= rel_tol * s_prev;
            s_prev = s;
            if (done) break;
        }
        iters[d] = k;
    }
    return 0;
}

/* (1/3) Re Tr of the m x n Wilson loop at site i in the plane (mu, nu):
 * m steps along +mu, n along +nu, m back along mu, n back along nu (Sec. III,
 * Wilson loops of the plaquette and of its 2x2 and larger relatives). */
static double loop_retr(const geom* g, const double* U, int64_t i, int mu, int nu, int m, int n)
{
    mat3 P = m_one();
    int64_t j = i;
    for (int a = 0; a < m; a++) { P = m_mul(P, ld(U, j, mu)); j = hop(g, j, mu, +1); }
    for (int b = 0; b < n; b++) { P = m_mul(P, ld(U, j, nu)); j = hop(g, j, nu, +1); }
    for (int a = 0; a < m; a++) { j = hop(g, j, mu, -1); P = m_mul(P, m_dag(ld(U, j, mu))); }
    for (int b = 0; b < n; b++) { j = hop(g, j, nu, -1); P = m_mul(P, m_dag(ld(U, j, nu))); }
    return creal(m_tr(P)) / 3.0;
}

/* Average m x n Wilson loop over all sites and planes mu<nu (Sec. III);
 * the m steps go along the lower direction mu of each plane. */
double orc_wilson_loop(const int32_t L[4], const double* U, int32_t m, int32_t n)
{
    geom g = mkgeom(L);
    double s = 0;
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) s += loop_retr(&g, U, i, mu, nu, m, n);
    return s / (6.0 * (double)g.V);
}

/* Partially averaged plaquette W^{1x1}_d: plaquettes with chi_munu(n) = d
 * (normalized by their count).  Displaced 2x2 loops W^{2x2}_d: 2x2 loops from
 * sites with chi(n) = d.  Both from the partial-average equations of Sec. III. */
double orc_partial_plaquette(const int32_t L[4], const double* U, int32_t d)
{
    geom g = mkgeom(L);
    double s = 0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < g.V; i++) {
        int n[4];
        coords(&g, i, n);
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++)
                if (chi_excl(n, mu, nu) == d) { s += creal(m_tr(plaq_mat(&g, U, i, mu, nu))) / 3.0; cnt++; }
    }
    return cnt ? s / (double)cnt : NAN;
}

/* Displaced m x n loops: the loops of orc_wilson_loop from the sites with
 * chi(n) = d only (Sec. III, displaced-loop average; its 2x2 case is
 * W^{2x2}_d, and even-sided loops from chi = 0 sites are the ones the
 * prolongation preserves). */
double orc_displaced_loop(const int32_t L[4], const double* U, int32_t d, int32_t m, int32_t n)
{
    geom g = mkgeom(L);
    double s = 0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < g.V; i++) {
        int x[4];
        coords(&g, i, x);
        if (chi_excl(x, -1, -1) != d) continue;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                s += loop_retr(&g, U, i, mu, nu, m, n);
                cnt++;
            }
    }
    return cnt ? s / (double)cnt : NAN;
}

double orc_displaced_2x2(const int32_t L[4], const double* U, int32_t d) { return orc_displaced_loop(L, U, d, 2, 2); }

/* ------------------------------------------------------------------ */
/* Wilson flow (Sec. IV.B), fixed-step third-order Runge-Kutta.         */
/* Z(U) = -(1/2)(Om - Om^+) + (1/6) Tr(Om - Om^+), Om = U A, the flow   */
/* generator for the Wilson action (independent of beta).               */
/* ------------------------------------------------------------------ */
static mat3 flow_generator(mat3 Om)
{
    mat3 X = m_sub(Om, m_dag(Om));
    cx t = m_tr(X);
    mat3 Z = m_scale(X, -0.5);
    for (int k = 0; k < 3; k++) Z.e[k][k] += t / 6.0;
    return Z;
}

static void flow_Z(const geom* g, const double* U, mat3* Z, double eps)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->V; i++)
        for (int mu = 0; mu < 4; mu++)
            Z[i * 4 + mu] = m_scale(flow_generator(m_mul(ld(U, i, mu), staple(g, U, i, mu))), eps);
}

/* W1 = exp(Z0/4) W0, W2 = exp(8/9 Z1 - 17/36 Z0) W1,
 * W3 = exp(3/4 Z2 - 8/9 Z1 + 17/36 Z0) W2, Z_i = eps Z(W_i). */
void orc_wilson_flow(const int32_t L[4], double* U, double eps, int32_t n_steps)
{
    geom g = mkgeom(L);
    size_t nl = (size_t)g.V * 4;
    mat3* Z0 = (mat3*)malloc(sizeof(mat3) * nl);
    mat3* Z1 = (mat3*)malloc(sizeof(mat3) * nl);
    mat3* Z2 = (mat3*)malloc(sizeof(mat3) * nl);
    for (int32_t s = 0; s < n_steps; s++) {
        flow_Z(&g, U, Z0, eps);
#pragma omp parallel for schedule(static)
        for (size_t l = 0; l < nl; l++) {
            mat3 m = m_mul(m_exp(m_scale(Z0[l], 0.25)), ld(U, (int64_t)(l / 4), (int)(l % 4)));
            st(U, (int64_t)(l / 4), (int)(l % 4), &m);
        }
        flow_Z(&g, U, Z1, eps);
#pragma omp parallel for schedule(static)
        for (size_t l = 0; l < nl; l++) {
            mat3 X = m_sub(m_scale(Z1[l], 8.0 / 9.0), m_scale(Z0[l], 17.0 / 36.0));
            mat3 m = m_mul(m_exp(X), ld(U, (int64_t)(l / 4), (int)(l % 4)));
            st(U, (int64_t)(l / 4), (int)(l % 4), &m);
        }
        flow_Z(&g, U, Z2, eps);
#pragma omp parallel for schedule(static)
        for (size_t l = 0; l < nl; l++) {
            mat3 X = m_add(m_sub(m_scale(Z2[l], 0.75), m_scale(Z1[l], 8.0 / 9.0)), m_scale(Z0[l], 17.0 / 36.0));
            mat3 m = m_mul(m_exp(X), ld(U, (int64_t)(l / 4), (int)(l % 4)));
            st(U, (int64_t)(l / 4), (int)(l % 4), &m);
        }
    }
    free(Z0);
    free(Z1);
    free(Z2);
}

/* ------------------------------------------------------------------ */
/* Adaptive-step flow.  Sec. IV.B uses the adaptive integrator of      */
/* Fritzsch and Ramos with a tolerance and a maximum step; the error   */
/* estimate and the step rule here are this implementation's reading:  */
/* a step of size h is the RK3 step above, W3 its result; the embedded */
/* second-order result is W~ = exp(2 Z1 - Z0) W0 (Z_i = h Z(W_i)), and  */
/* d = max over links and matrix elements of |W3 - W~|.  d <= tol      */
/* accepts the step; either way the next step size is                   */
/* min(max_step, 0.95 h (tol / d)^(1/3)).  A step is shortened to land */
/* on the next measurement time; at each measurement time the clover   */
/* energy density E and charge Q are recorded.                          */
/* ------------------------------------------------------------------ */
double orc_clover_energy(const int32_t L[4], const double* U);
double orc_topological_charge(const int32_t L[4], const double* U);

static double flow_step_embedded(const geom* g, double* U, double* W0, mat3* Z0, mat3* Z1, mat3* Z2, double h)
{
    size_t nl = (size_t)g->V * 4;
    memcpy(W0, U, sizeof(double) * (size_t)g->V * 72);
    flow_Z(g, U, Z0, h);
#pragma omp parallel for schedule(static)
    for (size_t l = 0; l < nl; l++) {
        mat3 m = m_mul(m_exp(m_scale(Z0[l], 0.25)), ld(U, (int64_t)(l / 4), (int)(l % 4)));
        st(U, (int64_t)(l / 4), (int)(l % 4), &m);
    }
    flow_Z(g, U, Z1, h);
#pragma omp parallel for schedule(static)
    for (size_t l = 0; l < nl; l++) {
        mat3 X = m_sub(m_scale(Z1[l], 8.0 / 9.0), m_scale(Z0[l], 17.0 / 36.0));
        mat3 m = m_mul(m_exp(X), ld(U, (int64_t)(l / 4), (int)(l % 4)));
        st(U, (int64_t)(l / 4), (int)(l % 4), &m);
    }
    flow_Z(g, U, Z2, h);
    double* dl = (double*)malloc(sizeof(double) * nl);
#pragma omp parallel for schedule(static)
    for (size_t l = 0; l < nl; l++) {
        int64_t i = (int64_t)(l / 4);
        int mu = (int)(l % 4);
        mat3 X = m_add(m_sub(m_scale(Z2[l], 0.75), m_scale(Z1[l], 8.0 / 9.0)), m_scale(Z0[l], 17.0 / 36.0));
        mat3 w3 = m_mul(m_exp(X), ld(U, i, mu));
        st(U, i, mu, &w3);
        mat3 w2 = m_mul(m_exp(m_sub(m_scale(Z1[l], 2.0), Z0[l])), ld(W0, i, mu));
        double worst = 0;
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) worst = fmax(worst, cabs(w3.e[r][c] - w2.e[r][c]));
        dl[l] = worst;
    }
    double d = 0;
    for (size_t l = 0; l < nl; l++) d = fmax(d, dl[l]);
    free(dl);
    return d;
}

int32_t orc_wilson_flow_adaptive(const int32_t L[4], double* U, double t_end, double tol, double max_step, double eps0,
                                 const double* t_meas, int32_t n_meas, double* E_out, double* Q_out,
                                 int32_t* n_accepted, int32_t* n_rejected)
{
    geom g = mkgeom(L);
    size_t nl = (size_t)g.V * 4;
    double* W0 = (double*)malloc(sizeof(double) * (size_t)g.V * 72);
    mat3* Z0 = (mat3*)malloc(sizeof(mat3) * nl);
    mat3* Z1 = (mat3*)malloc(sizeof(mat3) * nl);
    mat3* Z2 = (mat3*)malloc(sizeof(mat3) * nl);
    double t = 0, eps = fmin(eps0, max_step);
    int32_t k = 0, acc = 0, rej = 0, rc = 0;
    while (k < n_meas && t_meas[k] <= 0) {
        E_out[k] = orc_clover_energy(L, U);
        Q_out[k] = orc_topological_charge(L, U);
        k++;
    }
    while (t < t_end) {
        double target = (k < n_meas && t_meas[k] < t_end) ? t_meas[k] : t_end;
        int lands = eps >= target - t;
        double h = lands ? target - t : eps;
        double d = flow_step_embedded(&g, U, W0, Z0, Z1, Z2, h);
        if (d <= tol) {
            acc++;
            t = lands ? target : t + h;
            while (k < n_meas && t_meas[k] <= t) {
                E_out[k] = orc_clover_energy(L, U);
                Q_out[k] = orc_topological_charge(L, U);
                k++;
            }
        } else {
            rej++;
            memcpy(U, W0, sizeof(double) * (size_t)g.V * 72);
        }
        eps = d > 0 ? fmin(max_step, 0.95 * h * cbrt(tol / d)) : max_step;
        if (rej > 100000 || !(eps > 1e-12)) {
            rc = -1;
            break;
        }
    }
    if (n_accepted) *n_accepted = acc;
    if (n_rejected) *n_rejected = rej;
    free(W0);
    free(Z0);
    free(Z1);
    free(Z2);
    return rc;
}

/* One RK3 step of size h (U <- W3), returning its embedded-error distance d. */
double orc_flow_step_distance(const int32_t L[4], double* U, double h)
{
    geom g = mkgeom(L);
    size_t nl = (size_t)g.V * 4;
    double* W0 = (double*)malloc(sizeof(double) * (size_t)g.V * 72);
    mat3* Z0 = (mat3*)malloc(sizeof(mat3) * nl);
    mat3* Z1 = (mat3*)malloc(sizeof(mat3) * nl);
    mat3* Z2 = (mat3*)malloc(sizeof(mat3) * nl);
    double d = flow_step_embedded(&g, U, W0, Z0, Z1, Z2, h);
    free(W0);
    free(Z0);
    free(Z1);
    free(Z2);
    return d;
}

/* Flow scale: the t at which t^2 E(t) crosses `target` (0.3 for t0, Sec.  */
/* IV.B), by linear interpolation between the two bracketing measurements. */
/* Returns 0, or -1 when no measurement pair brackets the target.          */
int32_t orc_flow_t0(const double* t, const double* E, int32_t n, double target, double* t0)
{
    for (int32_t k = 1; k < n; k++) {
        double y0 = t[k - 1] * t[k - 1] * E[k - 1], y1 = t[k] * t[k] * E[k];
        if (y0 < target && y1 >= target) {
            *t0 = t[k - 1] + (target - y0) * (t[k] - t[k - 1]) / (y1 - y0);
            return 0;
        }
    }
    return -1;
}

/* Admissibility measure (Sec. IV.D): h = max over plaquettes of          */
/* s_p = 3 [1 - (1/3) Re Tr U_p].                                        */
double orc_max_splaq(const int32_t L[4], const double* U)
{
    geom g = mkgeom(L);
    double h = 0;
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) h = fmax(h, 3.0 - creal(m_tr(plaq_mat(&g, U, i, mu, nu))));
    return h;
}

/* ------------------------------------------------------------------ */
/* Clover field strength and topological charge (Sec. IV.D uses an      */
/* improved definition; this is the clover one).                        */
/* Q_munu(x) = sum of the four counter-clockwise leaves in the munu     */
/* plane at x; F_munu = traceless part of (Q_munu - Q_munu^+)/8;        */
/* q(x) = -(1/(2 pi^2)) Re Tr[F01 F23 + F02 F31 + F03 F12].             */
/* ------------------------------------------------------------------ */
static mat3 clover_F(const geom* g, const double* U, int64_t x, int mu, int nu)
{
    int64_t xpm = hop(g, x, mu, +1), xpn = hop(g, x, nu, +1);
    int64_t xmm = hop(g, x, mu, -1), xmn = hop(g, x, nu, -1);
    int64_t xmm_pn = hop(g, xmm, nu, +1), xmm_mn = hop(g, xmm, nu, -1), xpm_mn = hop(g, xpm, nu, -1);
    mat3 Q = m_zero();
    Q = m_add(Q, m_mul(m_mul(m_mul(ld(U, x, mu), ld(U, xpm, nu)), m_dag(ld(U, xpn, mu))), m_dag(ld(U, x, nu))));
    Q = m_add(Q, m_mul(m_mul(m_mul(ld(U, x, nu), m_dag(ld(U, xmm_pn, mu))), m_dag(ld(U, xmm, nu))), ld(U, xmm, mu)));
    Q = m_add(Q, m_mul(m_mul(m_mul(m_dag(ld(U, xmm, mu)), m_dag(ld(U, xmm_mn, nu))), ld(U, xmm_mn, mu)), ld(U, xmn, nu)));
    Q = m_add(Q, m_mul(m_mul(m_mul(m_dag(ld(U, xmn, nu)), ld(U, xmn, mu)), ld(U, xpm_mn, nu)), m_dag(ld(U, x, mu))));
    mat3 F = m_scale(m_sub(Q, m_dag(Q)), 0.125);
    cx t = m_tr(F) / 3.0;
    for (int k = 0; k < 3; k++) F.e[k][k] -= t;
    return F;
}

double orc_topological_charge(const int32_t L[4], const double* U)
{
    geom g = mkgeom(L);
    double q = 0;
    for (int64_t x = 0; x < g.V; x++) {
        mat3 F01 = clover_F(&g, U, x, 0, 1), F23 = clover_F(&g, U, x, 2, 3);
        mat3 F02 = clover_F(&g, U, x, 0, 2), F13 = clover_F(&g, U, x, 1, 3);
        mat3 F03 = clover_F(&g, U, x, 0, 3), F12 = clover_F(&g, U, x, 1, 2);
        cx t = m_tr(m_mul(F01, F23)) - m_tr(m_mul(F02, F13)) + m_tr(m_mul(F03, F12));
        q += -creal(t) / (2.0 * PI * PI);
    }
    return q;
}

/* Clover energy density summed over sites: E = -(1/2) sum_{mu,nu} Tr(F F)
 * per site, averaged over the volume.  Pinned by the closed form on constant
 * abelian flux fields and by gauge invariance. */
double orc_clover_energy(const int32_t L[4], const double* U)
{
    geom g = mkgeom(L);
    double e = 0;
    for (int64_t x = 0; x < g.V; x++)
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                mat3 F = clover_F(&g, U, x, mu, nu);
                e += -creal(m_tr(m_mul(F, F)));
            }
    return e / (double)g.V;
}

/* ------------------------------------------------------------------ */
/* Diagnostics.                                                        */
/* ------------------------------------------------------------------ */
/* Largest deviation from SU(3) over all links: max of ||U U^+ - 1||_max
 * and |det U - 1|. */
double orc_max_su3_dev(const int32_t L[4], const double* U)
{
    geom g = mkgeom(L);
    double worst = 0;
    for (int64_t i = 0; i < g.V; i++)
        for (int mu = 0; mu < 4; mu++) {
            mat3 u = ld(U, i, mu);
            mat3 d = m_sub(m_mul(u, m_dag(u)), m_one());
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) worst = fmax(worst, cabs(d.e[r][c]));
            worst = fmax(worst, cabs(m_det(u) - 1.0));
        }
    return worst;
}

void orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
