// device.hpp -- device-side building blocks for the SU(3) rethermalization
// kernels on gfx950: SU(3) matrices in registers, the tiled link layout,
// checkerboard geometry, the Philox4x32-10 generator and the fixed-sequence
// fp64 elementary functions.
//
// Link layout (one allocation per lattice): 8 slabs, slab = mu * 2 + parity,
// each holding the V/2 link records of that direction and parity indexed by
// cb = (lexicographic site index) >> 1.  A record is NC reals, NC = 18 (full
// matrix) or 12 (rows 0 and 1; row 2 rebuilt on load), ordered (re, im) per
// entry, row-major.  Records are grouped in tiles of 32 consecutive cb and
// cut into 16-byte chunks; chunk c of the 32 records of a tile is contiguous
// (see load_reals).  A thread loads a record with 16-byte vector loads at
// fixed offsets from one address; a wavefront's load covers contiguous
// 512-byte runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace msmc {

// ---------------------------------------------------------------------------
// Lattice geometry.  Site index i = n0 + L0*(n1 + L1*(n2 + L2*n3)); extents
// are even, so the two sites 2c and 2c+1 have opposite parity and c = i >> 1
// enumerates each parity exactly once.
// ---------------------------------------------------------------------------
struct Geo {
    int L[4];
    int h0;   // L0 / 2
    int Vh;   // sites per parity
};

__device__ __forceinline__ void cb_coords(const Geo& g, int cb, int par, int n[4])
{
    int x0h = cb % g.h0;
    int r = cb / g.h0;
    n[1] = r % g.L[1];
    r /= g.L[1];
    n[2] = r % g.L[2];
    n[3] = r / g.L[2];
    int b = (par + n[1] + n[2] + n[3]) & 1;
    n[0] = 2 * x0h + b;
}

__device__ __forceinline__ int lex_index(const Geo& g, const int n[4])
{
    return n[0] + g.L[0] * (n[1] + g.L[1] * (n[2] + g.L[2] * n[3]));
}

__device__ __forceinline__ int wrap_add(int x, int s, int L)
{
    x += s;
    return x < 0 ? x + L : (x >= L ? x - L : x);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the uniform / Gaussian maps.
// Counter words: c0 = lexicographic site, c1 = purpose<<28 | mu<<24 |
// subgroup<<20 | hit<<12 | draw, (c2, c3) = 64-bit sweep or trajectory index.
// Key = (seed, lattice id).
// ---------------------------------------------------------------------------
enum Purpose : uint32_t { P_INIT = 1, P_HB = 2, P_HB_DIR = 3, P_MOM = 4, P_ACCEPT = 5, P_GAUGE = 6, P_PARAM = 7 };

__device__ __forceinline__ uint32_t ctr_word(uint32_t purpose, int mu, int sub, int hit, int draw)
{
    return (purpose << 28) | ((uint32_t)mu << 24) | ((uint32_t)sub << 20) | ((uint32_t)hit << 12) | (uint32_t)draw;
}

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32 x 32 -> 64-bit product per multiplier (v_mad_u64_u32) and
        // one three-input XOR per output word (v_bitop3_b32, table 0x96)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96), lo1,
                       __builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96), lo0);
    }
    return c;
}

template <typename R> __device__ __forceinline__ R u01(uint32_t x);
template <> __device__ __forceinline__ double u01<double>(uint32_t x)
{
    return ((double)(x >> 9) * 2.0 + 1.0) * 0x1p-24;
}
// fp32: 1 + (x >> 9) 2^-23 built from its bits, minus (1 - 2^-24); both
// steps are exact, so the value is the same (2 (x >> 9) + 1) 2^-24.
template <> __device__ __forceinline__ float u01<float>(uint32_t x)
{
    return __uint_as_float(0x3F800000u | (x >> 9)) - 0x1.fffffep-1f;
}

struct Rng {
    uint32_t k0, k1;
    uint32_t site;
    uint64_t step;
    __device__ __forceinline__ uint4 draw(uint32_t w1) const
    {
        return philox10(make_uint4(site, w1, (uint32_t)step, (uint32_t)(step >> 32)), k0, k1);
    }
};

// ---------------------------------------------------------------------------
// fp64 elementary functions of the random draws, each a fixed sequence of
// IEEE-754 operations (the translation units using them are compiled without
// floating-point contraction), so the fp64 chain is reproducible bit for bit
// by any implementation that takes the same steps:
//  ln x:  x = m 2^e, m in [sqrt(1/2), sqrt(2)), s = (m-1)/(m+1),
//         ln m = 2 s sum_{k=0..11} s^{2k}/(2k+1) (Horner), ln x = e ln2_hi +
//         (e ln2_lo + ln m) with the Cody-Waite split of ln 2;
//  cos, sin of 2 pi u: q = nearest integer to 4u, t = 2 pi (u - q/4) in
//         [-pi/4, pi/4], Taylor series to t^18 / t^19, q quarter turns;
//  exp y: n = nearest integer to y/ln2, r = (y - n ln2_hi) - n ln2_lo,
//         Taylor series to r^17, scaled by 2^n.
// fp32 uses the device library functions.
// ---------------------------------------------------------------------------
struct FixedSeq {
    static constexpr double ln2_hi = 0x1.62e42feep-1;
    static constexpr double ln2_lo = 0x1.a39ef35793c76p-33;
    static constexpr double inv_ln2 = 1.44269504088896340736;
    static constexpr double two_pi = 6.28318530717958647693;
    static constexpr double sqrt_half = 0.70710678118654752440;
};

__device__ __forceinline__ double fact_d(int n)
{
    constexpr double F[21] = { 1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0, 5040.0, 40320.0, 362880.0, 3628800.0,
                               39916800.0, 479001600.0, 6227020800.0, 87178291200.0, 1307674368000.0,
                               20922789888000.0, 355687428096000.0, 6402373705728000.0,
                               121645100408832000.0, 2432902008176640000.0 };
    return F[n];
}

__device__ __forceinline__ double fs_ln(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < FixedSeq::sqrt_half) {
        m = 2.0 * m;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 23.0;
#pragma unroll
    for (int k = 10; k >= 0; k--) p = p * z + 1.0 / (double)(2 * k + 1);
    const double de = (double)e;
    return de * FixedSeq::ln2_hi + (de * FixedSeq::ln2_lo + 2.0 * s * p);
}

__device__ __forceinline__ void fs_cossin_2pi(double u, double* c, double* s)
{
    const double q = floor(4.0 * u + 0.5);
    const double v = u - 0.25 * q;
    const double t = FixedSeq::two_pi * v;
    const double t2 = t * t;
    double ps = -1.0 / fact_d(19);
#pragma unroll
    for (int k = 8; k >= 0; k--) ps = ps * t2 + ((k & 1) ? -1.0 : 1.0) / fact_d(2 * k + 1);
    double pc = -1.0 / fact_d(18);
#pragma unroll
    for (int k = 8; k >= 0; k--) pc = pc * t2 + ((k & 1) ? -1.0 : 1.0) / fact_d(2 * k);
    const double s0 = t * ps, c0 = pc;
    switch (((int)q) & 3) {
    case 0: *c = c0; *s = s0; break;
    case 1: *c = -s0; *s = c0; break;
    case 2: *c = -c0; *s = -s0; break;
    default: *c = s0; *s = -c0; break;
    }
}

__device__ __forceinline__ double fs_exp(double y)
{
    if (y < -745.0) return 0.0;
    const double n = floor(y * FixedSeq::inv_ln2 + 0.5);
    const double r = (y - n * FixedSeq::ln2_hi) - n * FixedSeq::ln2_lo;
    double p = 1.0 / fact_d(17);
#pragma unroll
    for (int k = 16; k >= 0; k--) p = p * r + 1.0 / fact_d(k);
    return ldexp(p, (int)n);
}

// math wrappers per precision.  fp32 uses the hardware instructions directly
// (the fp32 chain is never compared with fp64 bit for bit, and its draws
// only need the accuracy of the uniforms, 2^-24): log2 times ln 2 (the
// arguments are normal numbers in (0, 1]), square root, and sine / cosine of
// 2 pi u, which the hardware takes in revolutions (u in (0, 1)).
__device__ __forceinline__ double m_log(double x) { return fs_ln(x); }
__device__ __forceinline__ float m_log(float x) { return __builtin_amdgcn_logf(x) * 0.69314718056f; }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// 1 / sqrt(x): the fp64 form is the exact IEEE sequence; fp32 the hardware
// reciprocal square root and one Newton step.  The hardware value alone is
// low on average (rows normalized with it came out short by 6e-8 in |row|^2
// on average over all links of a 32^4 field).
__device__ __forceinline__ double m_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float m_rsqrt(float x)
{
    const float r = __builtin_amdgcn_rsqf(x);
    const float e = fmaf(-x, r * r, 1.0f);
    return fmaf(r * 0.5f, e, r);
}
__device__ __forceinline__ double m_exp(double x) { return fs_exp(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
// (cos 2 pi u, sin 2 pi u)
__device__ __forceinline__ void m_cossin2pi(double u, double* c, double* s) { fs_cossin_2pi(u, c, s); }
__device__ __forceinline__ void m_cossin2pi(float u, float* c, float* s)
{
    *c = __builtin_amdgcn_cosf(u);
    *s = __builtin_amdgcn_sinf(u);
}
__device__ __forceinline__ double m_max(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float m_max(float a, float b) { return fmaxf(a, b); }

// Four normals from one Philox call (Box-Muller on two uniform pairs).
template <typename R> __device__ __forceinline__ void normals4(uint4 w, R z[4])
{
    R u[4] = { u01<R>(w.x), u01<R>(w.y), u01<R>(w.z), u01<R>(w.w) };
#pragma unroll
    for (int h = 0; h < 2; h++) {
        R r = m_sqrt(R(-2) * m_log(u[2 * h]));
        R c, s;
        m_cossin2pi(u[2 * h + 1], &c, &s);
        z[2 * h] = r * c;
        z[2 * h + 1] = r * s;
    }
}

// ---------------------------------------------------------------------------
// 3x3 complex matrices in registers, row-major, separate re / im.
// ---------------------------------------------------------------------------
template <typename R> struct M3 {
    R re[9], im[9];
};

template <typename R> __device__ __forceinline__ void m_set_zero(M3<R>& a)
{
#pragma unroll
    for (int k = 0; k < 9; k++) a.re[k] = a.im[k] = R(0);
}

template <typename R> __device__ __forceinline__ void m_set_one(M3<R>& a)
{
    m_set_zero(a);
    a.re[0] = a.re[4] = a.re[8] = R(1);
}

// 3x3 complex products with either factor optionally daggered.
// fp64: each complex product is formed as (ac - bd, ad + bc) and added to
// the running sum in k order, with no contraction -- the order the fp64 chain
// is specified in.  fp32: the same sums as chains of fused multiply-adds
// (four per complex multiply-accumulate).
template <bool DA, bool DB, typename R>
__device__ __forceinline__ void mm_acc(M3<R>& c, const M3<R>& a, const M3<R>& b)
{
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int s = 0; s < 3; s++) {
            R xr = c.re[r * 3 + s], xi = c.im[r * 3 + s];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const R ar = DA ? a.re[k * 3 + r] : a.re[r * 3 + k];
                const R ai = DA ? -a.im[k * 3 + r] : a.im[r * 3 + k];
                const R br = DB ? b.re[s * 3 + k] : b.re[k * 3 + s];
                const R bi = DB ? -b.im[s * 3 + k] : b.im[k * 3 + s];
                if constexpr (std::is_same<R, float>::value) {
                    xr = fmaf(ar, br, xr);
                    xr = fmaf(-ai, bi, xr);
                    xi = fmaf(ar, bi, xi);
                    xi = fmaf(ai, br, xi);
                } else {
                    xr += ar * br - ai * bi;
                    xi += ar * bi + ai * br;
                }
            }
            c.re[r * 3 + s] = xr;
            c.im[r * 3 + s] = xi;
        }
}

template <bool DA, bool DB, typename R> __device__ __forceinline__ M3<R> mm(const M3<R>& a, const M3<R>& b)
{
    M3<R> c;
#pragma unroll
    for (int k = 0; k < 9; k++) c.re[k] = c.im[k] = R(0);
    mm_acc<DA, DB>(c, a, b);
    return c;
}

// C = A B, A B^+, A^+ B, A^+ B^+
template <typename R> __device__ __forceinline__ M3<R> m_mul(const M3<R>& a, const M3<R>& b) { return mm<false, false>(a, b); }
template <typename R> __device__ __forceinline__ M3<R> m_mul_nd(const M3<R>& a, const M3<R>& b) { return mm<false, true>(a, b); }
template <typename R> __device__ __forceinline__ M3<R> m_mul_dn(const M3<R>& a, const M3<R>& b) { return mm<true, false>(a, b); }
template <typename R> __device__ __forceinline__ M3<R> m_mul_dd(const M3<R>& a, const M3<R>& b) { return mm<true, true>(a, b); }

template <typename R> __device__ __forceinline__ void m_acc(M3<R>& a, const M3<R>& b)
{
#pragma unroll
    for (int k = 0; k < 9; k++) {
        a.re[k] += b.re[k];
        a.im[k] += b.im[k];
    }
}

template <typename R> __device__ __forceinline__ M3<R> m_dag(const M3<R>& a)
{
    M3<R> c;
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int s = 0; s < 3; s++) {
            c.re[r * 3 + s] = a.re[s * 3 + r];
            c.im[r * 3 + s] = -a.im[s * 3 + r];
        }
    return c;
}

template <typename R> __device__ __forceinline__ R m_retr(const M3<R>& a) { return a.re[0] + a.re[4] + a.re[8]; }

template <typename R, typename S> __device__ __forceinline__ M3<S> m_cast(const M3<R>& a)
{
    M3<S> c;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        c.re[k] = (S)a.re[k];
        c.im[k] = (S)a.im[k];
    }
    return c;
}

// row 2 = complex conjugate of (row 0 x row 1)
template <typename R> __device__ __forceinline__ void m_complete_row2(M3<R>& a)
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        if constexpr (std::is_same<R, float>::value) {
            R xr = a.re[c1] * a.re[3 + c2];
            xr = fmaf(-a.im[c1], a.im[3 + c2], xr);
            xr = fmaf(-a.re[c2], a.re[3 + c1], xr);
            xr = fmaf(a.im[c2], a.im[3 + c1], xr);
            R ni = -(a.re[c1] * a.im[3 + c2]);
            ni = fmaf(-a.im[c1], a.re[3 + c2], ni);
            ni = fmaf(a.re[c2], a.im[3 + c1], ni);
            ni = fmaf(a.im[c2], a.re[3 + c1], ni);
            a.re[6 + c] = xr;
            a.im[6 + c] = ni;
        } else {
            R xr = a.re[c1] * a.re[3 + c2] - a.im[c1] * a.im[3 + c2] - (a.re[c2] * a.re[3 + c1] - a.im[c2] * a.im[3 + c1]);
            R xi = a.re[c1] * a.im[3 + c2] + a.im[c1] * a.re[3 + c2] - (a.re[c2] * a.im[3 + c1] + a.im[c2] * a.re[3 + c1]);
            a.re[6 + c] = xr;
            a.im[6 + c] = -xi;
        }
    }
}

// Gram-Schmidt of rows 0 and 1, then row 2 completes to SU(3).
template <typename R> __device__ __forceinline__ void m_reunit(M3<R>& a)
{
    R n0 = R(0);
#pragma unroll
    for (int c = 0; c < 3; c++) n0 += a.re[c] * a.re[c] + a.im[c] * a.im[c];
    n0 = m_rsqrt(n0);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        a.re[c] *= n0;
        a.im[c] *= n0;
    }
    R pr = R(0), pi = R(0);  // <row0, row1> = sum conj(r0) r1
#pragma unroll
    for (int c = 0; c < 3; c++) {
        pr += a.re[c] * a.re[3 + c] + a.im[c] * a.im[3 + c];
        pi += a.re[c] * a.im[3 + c] - a.im[c] * a.re[3 + c];
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        a.re[3 + c] -= pr * a.re[c] - pi * a.im[c];
        a.im[3 + c] -= pr * a.im[c] + pi * a.re[c];
    }
    R n1 = R(0);
#pragma unroll
    for (int c = 0; c < 3; c++) n1 += a.re[3 + c] * a.re[3 + c] + a.im[3 + c] * a.im[3 + c];
    n1 = m_rsqrt(n1);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        a.re[3 + c] *= n1;
        a.im[3 + c] *= n1;
    }
    m_complete_row2(a);
}

// ---------------------------------------------------------------------------
// SU(2) subgroups of SU(3) in quaternion form: q = q0 + i q.sigma is the
// 2x2 block [[q0 + i q3, q2 + i q1], [-q2 + i q1, q0 - i q3]].
// ---------------------------------------------------------------------------
// subgroup s = 0, 1, 2 acts on rows (0,1), (1,2), (0,2), in that order
__host__ __device__ constexpr int sub_i(int s) { return s == 1 ? 1 : 0; }
__host__ __device__ constexpr int sub_j(int s) { return s == 0 ? 1 : 2; }

template <typename R> struct Q4 {
    R q0, q1, q2, q3;
};

// SU(2) part of the (i,j) block of W: returns k and the unit quaternion v.
template <typename R> __device__ __forceinline__ R su2_part(const M3<R>& W, int i, int j, Q4<R>& v)
{
    const int ii = i * 3 + i, jj = j * 3 + j, ij = i * 3 + j, ji = j * 3 + i;
    R x0 = (W.re[ii] + W.re[jj]) * R(0.5);
    R x3 = (W.im[ii] - W.im[jj]) * R(0.5);
    R x1 = (W.im[ij] + W.im[ji]) * R(0.5);
    R x2 = (W.re[ij] - W.re[ji]) * R(0.5);
    const R k2 = x0 * x0 + x1 * x1 + x2 * x2 + x3 * x3;
    const R ik = (k2 > R(0)) ? m_rsqrt(k2) : R(0);
    const R k = k2 * ik;
    v.q0 = x0 * ik;
    v.q1 = x1 * ik;
    v.q2 = x2 * ik;
    v.q3 = x3 * ik;
    return k;
}

// rows i, j of M <- r applied from the left
template <typename R> __device__ __forceinline__ void left_apply(M3<R>& M, int i, int j, const Q4<R>& r)
{
    const R a_re = r.q0, a_im = r.q3;   // r00
    const R b_re = r.q2, b_im = r.q1;   // r01
    const R c_re = -r.q2, c_im = r.q1;  // r10
    const R d_re = r.q0, d_im = -r.q3;  // r11
#pragma unroll
    for (int c = 0; c < 3; c++) {
        R xr = M.re[i * 3 + c], xi = M.im[i * 3 + c];
        R yr = M.re[j * 3 + c], yi = M.im[j * 3 + c];
        M.re[i * 3 + c] = a_re * xr - a_im * xi + b_re * yr - b_im * yi;
        M.im[i * 3 + c] = a_re * xi + a_im * xr + b_re * yi + b_im * yr;
        M.re[j * 3 + c] = c_re * xr - c_im * xi + d_re * yr - d_im * yi;
        M.im[j * 3 + c] = c_re * xi + c_im * xr + d_re * yi + d_im * yr;
    }
}

// quaternion product a b
template <typename R> __device__ __forceinline__ Q4<R> q_mul(const Q4<R>& a, const Q4<R>& b)
{
    Q4<R> c;
    c.q0 = a.q0 * b.q0 - a.q1 * b.q1 - a.q2 * b.q2 - a.q3 * b.q3;
    // vector part: a0 b + b0 a - a x b
    c.q1 = a.q0 * b.q1 + b.q0 * a.q1 - (a.q2 * b.q3 - a.q3 * b.q2);
    c.q2 = a.q0 * b.q2 + b.q0 * a.q2 - (a.q3 * b.q1 - a.q1 * b.q3);
    c.q3 = a.q0 * b.q3 + b.q0 * a.q3 - (a.q1 * b.q2 - a.q2 * b.q1);
    return c;
}

template <typename R> __device__ __forceinline__ Q4<R> q_conj(const Q4<R>& a) { return Q4<R>{ a.q0, -a.q1, -a.q2, -a.q3 }; }

// ---------------------------------------------------------------------------
// fp64 SU(2) steps as explicit complex 2x2 arithmetic with products
// (ac - bd, ad + bc) and sums taken in a fixed order: the form the fp64
// chain is specified in, so that it is reproducible bit for bit.
// ---------------------------------------------------------------------------
struct Cx {
    double re, im;
};
__device__ __forceinline__ Cx c_mul(Cx a, Cx b) { return Cx{ a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re }; }
__device__ __forceinline__ Cx c_add(Cx a, Cx b) { return Cx{ a.re + b.re, a.im + b.im }; }
__device__ __forceinline__ Cx c_conj(Cx a) { return Cx{ a.re, -a.im }; }

// v = unit SU(2) part of the (i,j) block of W as [[x0+i x3, x2+i x1],
// [-x2+i x1, x0-i x3]]/k (each component divided by k); returns k.
__device__ __forceinline__ double su2_part_c(const M3<double>& W, int i, int j, Cx v[2][2])
{
    const int ii = i * 3 + i, jj = j * 3 + j, ij = i * 3 + j, ji = j * 3 + i;
    const double x0 = (W.re[ii] + W.re[jj]) * 0.5;
    const double x3 = (W.im[ii] - W.im[jj]) * 0.5;
    const double x1 = (W.im[ij] + W.im[ji]) * 0.5;
    const double x2 = (W.re[ij] - W.re[ji]) * 0.5;
    const double k = sqrt(x0 * x0 + x1 * x1 + x2 * x2 + x3 * x3);
    if (k == 0.0) return 0.0;
    // four quotients; negating one equals dividing the negated numerator
    const double q0 = x0 / k, q1 = x1 / k, q2 = x2 / k, q3 = x3 / k;
    v[0][0] = Cx{ q0, q3 };
    v[0][1] = Cx{ q2, q1 };
    v[1][0] = Cx{ -q2, q1 };
    v[1][1] = Cx{ q0, -q3 };
    return k;
}

// rows i, j of M <- r applied from the left: M_i = r00 M_i + r01 M_j, ...
__device__ __forceinline__ void left_apply_c(M3<double>& M, int i, int j, const Cx r[2][2])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const Cx a{ M.re[i * 3 + c], M.im[i * 3 + c] };
        const Cx b{ M.re[j * 3 + c], M.im[j * 3 + c] };
        const Cx x = c_add(c_mul(r[0][0], a), c_mul(r[0][1], b));
        const Cx y = c_add(c_mul(r[1][0], a), c_mul(r[1][1], b));
        M.re[i * 3 + c] = x.re;
        M.im[i * 3 + c] = x.im;
        M.re[j * 3 + c] = y.re;
        M.im[j * 3 + c] = y.im;
    }
}

// C = A B for 2x2 complex matrices
__device__ __forceinline__ void mul2_c(const Cx a[2][2], const Cx b[2][2], Cx c[2][2])
{
#pragma unroll
    for (int p = 0; p < 2; p++)
#pragma unroll
        for (int q = 0; q < 2; q++) c[p][q] = c_add(c_mul(a[p][0], b[0][q]), c_mul(a[p][1], b[1][q]));
}

// Rows 0 and 1 made orthonormal for a 12-real store, computed in fp64 and
// rounded once.  An fp32 Gram-Schmidt without contracted arithmetic leaves the
// row norms off by a fraction of an ulp with the same sign on every link;
// summed over millions of links that shifts the action by whole units (one
// 32^4 HMC trajectory gave an energy difference of 13.3 where fp64 gives
// 9.45), whereas a single rounding of exact rows is unbiased.
//
// The fp64 normalizations use the hardware fp64 reciprocal square root and one
// Newton step (relative error about 2^-44, far below the fp32 rounding that
// follows), not the IEEE sequence the fp64 chain needs.
__device__ __forceinline__ double rsqrt_d_for_f32(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    return r + 0.5 * r * (1.0 - x * r * r);
}

template <typename R> __device__ __forceinline__ void m_reunit_for_store(M3<R>& a)
{
    if constexpr (std::is_same<R, double>::value) {
        m_reunit(a);
    } else {
        M3<double> d = m_cast<R, double>(a);
        double n0 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++) n0 += d.re[c] * d.re[c] + d.im[c] * d.im[c];
        n0 = rsqrt_d_for_f32(n0);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            d.re[c] *= n0;
            d.im[c] *= n0;
        }
        double pr = 0.0, pi = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            pr += d.re[c] * d.re[3 + c] + d.im[c] * d.im[3 + c];
            pi += d.re[c] * d.im[3 + c] - d.im[c] * d.re[3 + c];
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            d.re[3 + c] -= pr * d.re[c] - pi * d.im[c];
            d.im[3 + c] -= pr * d.im[c] + pi * d.re[c];
        }
        double n1 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++) n1 += d.re[3 + c] * d.re[3 + c] + d.im[3 + c] * d.im[3 + c];
        n1 = rsqrt_d_for_f32(n1);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            d.re[3 + c] *= n1;
            d.im[3 + c] *= n1;
        }
        m_complete_row2(d);
        a = m_cast<double, R>(d);
    }
}

// ---------------------------------------------------------------------------
// Link field views.
// ---------------------------------------------------------------------------
// Records of N reals (a link: N = 18 or 12; momenta / flow generators:
// N = 8) live in slabs, one per (direction, parity), sb bytes apart.  A slab
// is a sequence of tiles of 32 consecutive checkerboard sites; inside a tile
// the records are cut into 16-byte chunks and chunk c of all 32 sites is
// contiguous (512 bytes), followed by an 8-byte tail chunk (256 bytes) when
// the record is not a multiple of 16 bytes (fp32, N = 18).  Record reals are
// ordered (re, im) per matrix entry, row-major.  A thread computes one
// address per record and loads it with 16-byte vector loads at fixed
// offsets; a wavefront's load is two or three contiguous 512-byte runs.
// ---------------------------------------------------------------------------
template <typename R, int N> struct Rec {
    static constexpr int BYTES = N * (int)sizeof(R);
    static constexpr int NF = BYTES / 16;
    static constexpr bool TAIL = (BYTES % 16) != 0;
    static constexpr int TB = 32 * BYTES;
};

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) v4f g_v4f;
typedef __attribute__((address_space(1))) v2f g_v2f;
typedef __attribute__((address_space(1))) v2d g_v2d;

// Vector load / store; NT marks data used once (nontemporal hint, so the
// caches keep the neighbour links that other threads still need).
template <bool NT, typename V> __device__ __forceinline__ V vload(uintptr_t a)
{
    typedef __attribute__((address_space(1))) V GV;
    if constexpr (NT)
        return __builtin_nontemporal_load((const GV*)a);
    else
        return *(const GV*)a;
}

template <bool NT, typename V> __device__ __forceinline__ void vstore(uintptr_t a, V v)
{
    typedef __attribute__((address_space(1))) V GV;
    if constexpr (NT)
        __builtin_nontemporal_store(v, (GV*)a);
    else
        *(GV*)a = v;
}

template <typename R, int N, bool NT = false> __device__ __forceinline__ void load_reals(uintptr_t slab, int cb, R out[N])
{
    using L = Rec<R, N>;
    const uintptr_t t = slab + (uintptr_t)(cb >> 5) * L::TB;
    const uintptr_t q = t + (uintptr_t)(cb & 31) * 16;
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int c = 0; c < L::NF; c++) {
            const v4f v = vload<NT, v4f>(q + c * 512);
            out[4 * c] = v.x;
            out[4 * c + 1] = v.y;
            out[4 * c + 2] = v.z;
            out[4 * c + 3] = v.w;
        }
        if constexpr (L::TAIL) {
            const v2f v = vload<NT, v2f>(t + L::NF * 512 + (uintptr_t)(cb & 31) * 8);
            out[4 * L::NF] = v.x;
            out[4 * L::NF + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int c = 0; c < L::NF; c++) {
            const v2d v = vload<NT, v2d>(q + c * 512);
            out[2 * c] = v.x;
            out[2 * c + 1] = v.y;
        }
    }
}

template <typename R, int N, bool NT = false> __device__ __forceinline__ void store_reals(uintptr_t slab, int cb, const R in[N])
{
    using L = Rec<R, N>;
    const uintptr_t t = slab + (uintptr_t)(cb >> 5) * L::TB;
    const uintptr_t q = t + (uintptr_t)(cb & 31) * 16;
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int c = 0; c < L::NF; c++)
            vstore<NT, v4f>(q + c * 512, v4f{ in[4 * c], in[4 * c + 1], in[4 * c + 2], in[4 * c + 3] });
        if constexpr (L::TAIL)
            vstore<NT, v2f>(t + L::NF * 512 + (uintptr_t)(cb & 31) * 8, v2f{ in[4 * L::NF], in[4 * L::NF + 1] });
    } else {
#pragma unroll
        for (int c = 0; c < L::NF; c++) vstore<NT, v2d>(q + c * 512, v2d{ in[2 * c], in[2 * c + 1] });
    }
}

template <typename R, int NC> struct Links {
    uintptr_t p;
    size_t sb;  // bytes per slab
    __device__ __forceinline__ uintptr_t slab(int mu, int par) const { return p + (uintptr_t)(mu * 2 + par) * sb; }
    __device__ __forceinline__ uintptr_t slab_at(int s) const { return p + (uintptr_t)s * sb; }
};

template <typename R, int NC, bool NT = false> __device__ __forceinline__ M3<R> load_link(uintptr_t slab, int cb)
{
    R b[NC];
    load_reals<R, NC, NT>(slab, cb, b);
    M3<R> m;
#pragma unroll
    for (int k = 0; k < NC / 2; k++) {
        m.re[k] = b[2 * k];
        m.im[k] = b[2 * k + 1];
    }
    if constexpr (NC == 12) m_complete_row2(m);
    return m;
}

template <typename R, int NC, bool NT = false> __device__ __forceinline__ void store_link(uintptr_t slab, int cb, const M3<R>& m)
{
    R b[NC];
#pragma unroll
    for (int k = 0; k < NC / 2; k++) {
        b[2 * k] = m.re[k];
        b[2 * k + 1] = m.im[k];
    }
    store_reals<R, NC, NT>(slab, cb, b);
}

// Convenience: load U_mu at site coordinates n (any parity).
template <typename R, int NC> __device__ __forceinline__ M3<R> load_at(const Links<R, NC>& U, const Geo& g, int mu, const int n[4])
{
    int i = lex_index(g, n);
    int par = (n[0] + n[1] + n[2] + n[3]) & 1;
    return load_link<R, NC>(U.slab(mu, par), i >> 1);
}

// ---------------------------------------------------------------------------
// fp32 staples.  Every staple term is a product of SU(3) matrices, hence
// itself in SU(3): its rows 0 and 1 are formed by products and its row 2 is
// conj(row0 x row1).  Of a term's first factor only rows 0 and 1 are loaded
// (its row-2 entries where the backward term reads them); a 12-real link's
// third row is rebuilt only where a product reads it.
// ---------------------------------------------------------------------------
struct Rows2 {
    float re[6], im[6];  // rows 0 and 1
};

// rows 0 and 1 of a record of NC = 12 or 18 reals: its first three 16-byte
// chunks
template <int NC> __device__ __forceinline__ Rows2 load_rows2(uintptr_t slab, int cb)
{
    const uintptr_t q = slab + (uintptr_t)(cb >> 5) * Rec<float, NC>::TB + (uintptr_t)(cb & 31) * 16;
    Rows2 r;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const v4f v = vload<false, v4f>(q + c * 512);
        r.re[2 * c] = v.x;
        r.im[2 * c] = v.y;
        r.re[2 * c + 1] = v.z;
        r.im[2 * c + 1] = v.w;
    }
    return r;
}

template <int NC>
__device__ __forceinline__ Rows2 load_rows2_at(const Links<float, NC>& U, const Geo& g, int mu, const int n[4])
{
    const int i = lex_index(g, n);
    return load_rows2<NC>(U.slab(mu, (n[0] + n[1] + n[2] + n[3]) & 1), i >> 1);
}

// entry (2, c) of an SU(3) matrix from rows 0, 1: conj(row0 x row1)_c, the
// arithmetic of m_complete_row2
__device__ __forceinline__ void row2_entry(const float re[6], const float im[6], int c, float& xr, float& ni)
{
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    xr = re[c1] * re[3 + c2];
    xr = fmaf(-im[c1], im[3 + c2], xr);
    xr = fmaf(-re[c2], re[3 + c1], xr);
    xr = fmaf(im[c2], im[3 + c1], xr);
    ni = -(re[c1] * im[3 + c2]);
    ni = fmaf(-im[c1], re[3 + c2], ni);
    ni = fmaf(re[c2], im[3 + c1], ni);
    ni = fmaf(im[c2], re[3 + c1], ni);
}

__device__ __forceinline__ M3<float> full_of(const Rows2& r)
{
    M3<float> m;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        m.re[k] = r.re[k];
        m.im[k] = r.im[k];
    }
#pragma unroll
    for (int c = 0; c < 3; c++) row2_entry(r.re, r.im, c, m.re[6 + c], m.im[6 + c]);
    return m;
}

// A += S for S in SU(3) given by its rows 0, 1
__device__ __forceinline__ void acc_su3_rows(M3<float>& A, const Rows2& S)
{
#pragma unroll
    for (int k = 0; k < 6; k++) {
        A.re[k] += S.re[k];
        A.im[k] += S.im[k];
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        float xr, xi;
        row2_entry(S.re, S.im, c, xr, xi);
        A.re[6 + c] += xr;
        A.im[6 + c] += xi;
    }
}

// rows 0, 1 of X Y^+ from rows 0, 1 of X and all of Y
__device__ __forceinline__ Rows2 rows_mul_nd(const Rows2& x, const M3<float>& y)
{
    Rows2 t;
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int s = 0; s < 3; s++) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const float ar = x.re[3 * r + k], ai = x.im[3 * r + k];
                const float br = y.re[3 * s + k], bi = y.im[3 * s + k];
                re = fmaf(ar, br, re);
                re = fmaf(ai, bi, re);
                im = fmaf(ai, br, im);
                im = fmaf(-ar, bi, im);
            }
            t.re[3 * r + s] = re;
            t.im[3 * r + s] = im;
        }
    return t;
}

// rows 0, 1 of (B A)^+ C: columns 0, 1 of B A need B whole and rows 0..2 of
// A at columns 0, 1 only; then conj(BA)_{k r} C_{k s} summed over k.
__device__ __forceinline__ Rows2 rows_bwd(const Rows2& a, const float a2r[2], const float a2i[2], const M3<float>& b,
                                          const M3<float>& c)
{
    float xr[3][2], xi[3][2];  // (B A)_{k r}, r = 0, 1
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
        for (int r = 0; r < 2; r++) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const float br = b.re[3 * k + j], bi = b.im[3 * k + j];
                const float ar = j < 2 ? a.re[3 * j + r] : a2r[r];
                const float ai = j < 2 ? a.im[3 * j + r] : a2i[r];
                re = fmaf(br, ar, re);
                re = fmaf(-bi, ai, re);
                im = fmaf(br, ai, im);
                im = fmaf(bi, ar, im);
            }
            xr[k][r] = re;
            xi[k][r] = im;
        }
    Rows2 t;
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int s = 0; s < 3; s++) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const float cr = c.re[3 * k + s], ci = c.im[3 * k + s];
                re = fmaf(xr[k][r], cr, re);
                re = fmaf(xi[k][r], ci, re);
                im = fmaf(xr[k][r], ci, im);
                im = fmaf(-xi[k][r], cr, im);
            }
            t.re[3 * r + s] = re;
            t.im[3 * r + s] = im;
        }
    return t;
}

// a link whole: 12-real records rebuild row 2, 18-real ones load it
template <int NC>
__device__ __forceinline__ M3<float> load_full_at(const Links<float, NC>& U, const Geo& g, int mu, const int n[4])
{
    if constexpr (NC == 12)
        return full_of(load_rows2_at<12>(U, g, mu, n));
    else
        return load_at(U, g, mu, n);
}

// Where a staple link sits relative to the updated link's site n: n itself,
// n + e_0, n - e_0, or elsewhere (a loader may serve the first three from
// on-chip copies).
enum NbKind { NB_SAME = 0, NB_XP = 1, NB_XM = 2, NB_OTHER = 3 };

// Staple links straight from the field.
template <int NC> struct GlobalLd {
    const Links<float, NC>& U;
    const Geo& g;
    __device__ __forceinline__ Rows2 rows(int dir, const int m[4], int) const { return load_rows2_at<NC>(U, g, dir, m); }
    __device__ __forceinline__ M3<float> full(int dir, const int m[4], int) const { return load_full_at<NC>(U, g, dir, m); }
    // rows 0, 1 and the row-2 entries of columns 0, 1
    __device__ __forceinline__ void rows_c01(int dir, const int m[4], int, Rows2& a, float a2r[2], float a2i[2]) const
    {
        if constexpr (NC == 12) {
            a = load_rows2_at<12>(U, g, dir, m);
            row2_entry(a.re, a.im, 0, a2r[0], a2i[0]);
            row2_entry(a.re, a.im, 1, a2r[1], a2i[1]);
        } else {
            const M3<float> af = load_at(U, g, dir, m);
#pragma unroll
            for (int k = 0; k < 6; k++) {
                a.re[k] = af.re[k];
                a.im[k] = af.im[k];
            }
            a2r[0] = af.re[6];
            a2i[0] = af.im[6];
            a2r[1] = af.re[7];
            a2i[1] = af.im[7];
        }
    }
};

template <int NC, bool SNAP, class LD>
__device__ __forceinline__ M3<float> staple_sum_rows(const LD& ld, const Geo& g, int mu, const int n[4], M3<float>* lo)
{
    M3<float> A;
    m_set_zero(A);
    int npm[4];
#pragma unroll
    for (int k = 0; k < 4; k++) npm[k] = (k == mu) ? wrap_add(n[k], 1, g.L[k]) : n[k];
#pragma unroll
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) {
            if constexpr (SNAP) *lo = A;
            continue;
        }
        int npn[4] = { n[0], n[1], n[2], n[3] };
        npn[nu] = wrap_add(n[nu], 1, g.L[nu]);
        int nmn[4] = { n[0], n[1], n[2], n[3] };
        nmn[nu] = wrap_add(n[nu], -1, g.L[nu]);
        int npm_mn[4] = { npm[0], npm[1], npm[2], npm[3] };
        npm_mn[nu] = nmn[nu];
        {
            // U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+
            const Rows2 a = ld.rows(nu, npm, mu == 0 ? NB_XP : NB_OTHER);
            const M3<float> b = ld.full(mu, npn, nu == 0 ? NB_XP : NB_OTHER);
            const M3<float> c = ld.full(nu, n, NB_SAME);
            acc_su3_rows(A, rows_mul_nd(rows_mul_nd(a, b), c));
        }
        {
            // U_nu(n+mu-nu)^+ U_mu(n-nu)^+ U_nu(n-nu) = (U_mu(n-nu) U_nu(n+mu-nu))^+ U_nu(n-nu):
            // of the first factor rows 0, 1 and the row-2 entries of columns 0, 1
            Rows2 a;
            float a2r[2], a2i[2];
            ld.rows_c01(nu, npm_mn, NB_OTHER, a, a2r, a2i);
            const M3<float> b = ld.full(mu, nmn, nu == 0 ? NB_XM : NB_OTHER);
            const M3<float> c = ld.full(nu, nmn, nu == 0 ? NB_XM : NB_OTHER);
            acc_su3_rows(A, rows_bwd(a, a2r, a2i, b, c));
        }
    }
    return A;
}

// Staple sum A_mu(n): for nu != mu ascending, the forward term
// U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+ then the backward term
// U_nu(n+mu-nu)^+ U_mu(n-nu)^+ U_nu(n-nu); Re Tr(U_mu(n) A) is the sum of the
// six plaquettes containing U_mu(n).  Computed in precision C from links of
// precision R.
//
// With SNAP, *lo receives the partial sum of the terms nu < mu (the staples
// of the plaquettes in the planes (nu, mu), nu < mu).  In fp32 the terms are
// formed from their rows 0 and 1 (staple_sum_rows), which takes every term to
// be in SU(3): exact for 12-real links; 18-real HMC and flow links are off
// SU(3) only by rounding, and the difference is of that order (HMC energy
// differences against fp64 stay within their bars).
template <typename R, int NC, typename C, bool SNAP = false>
__device__ __forceinline__ M3<C> staple_sum(const Links<R, NC>& U, const Geo& g, int mu, const int n[4],
                                           M3<C>* lo = nullptr)
{
    if constexpr (std::is_same<R, float>::value && std::is_same<C, float>::value)
        return staple_sum_rows<NC, SNAP>(GlobalLd<NC>{ U, g }, g, mu, n, lo);
    M3<C> A;
    m_set_zero(A);
    // n + mu with mu known only at run time: selects over the unrolled
    // components keep the coordinates in registers (no indexed array)
    int npm[4];
#pragma unroll
    for (int k = 0; k < 4; k++) npm[k] = (k == mu) ? wrap_add(n[k], 1, g.L[k]) : n[k];
#pragma unroll
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) {
            if constexpr (SNAP) *lo = A;
            continue;
        }
        int npn[4] = { n[0], n[1], n[2], n[3] };
        npn[nu] = wrap_add(n[nu], 1, g.L[nu]);
        int nmn[4] = { n[0], n[1], n[2], n[3] };
        nmn[nu] = wrap_add(n[nu], -1, g.L[nu]);
        int npm_mn[4] = { npm[0], npm[1], npm[2], npm[3] };
        npm_mn[nu] = nmn[nu];
        {
            M3<C> a = m_cast<R, C>(load_at(U, g, nu, npm));
            M3<C> b = m_cast<R, C>(load_at(U, g, mu, npn));
            M3<C> c = m_cast<R, C>(load_at(U, g, nu, n));
            if constexpr (std::is_same<C, float>::value)
                mm_acc<false, true>(A, m_mul_nd(a, b), c);
            else
                m_acc(A, m_mul_nd(m_mul_nd(a, b), c));
        }
        {
            M3<C> a = m_cast<R, C>(load_at(U, g, nu, npm_mn));
            M3<C> b = m_cast<R, C>(load_at(U, g, mu, nmn));
            M3<C> c = m_cast<R, C>(load_at(U, g, nu, nmn));
            if constexpr (std::is_same<C, float>::value)
                mm_acc<false, false>(A, m_mul_dd(a, b), c);
            else
                m_acc(A, m_mul(m_mul_dd(a, b), c));
        }
    }
    return A;
}

// Thread index w -> site of the given parity, walking the lattice in tiles of
// L0 x ty x tz x tt sites (tiles ordered y, z, t; inside a tile x-halves
// fastest, then y, z, t).  Whole x rows keep each wavefront's loads
// contiguous; the tile shape sets which neighbours are in flight together on
// one XCD.  ty = L1, tz = L2, tt = 1 is the plain lexicographic order.
__device__ __forceinline__ void tiled_coords(const Geo& g, const int tile[3], int w, int par, int n[4])
{
    const int ty = tile[0], tz = tile[1], tt = tile[2];
    const int th = g.h0 * ty * tz * tt;
    const int tid = w / th, j = w - tid * th;
    const int ny = g.L[1] / ty, nz = g.L[2] / tz;
    const int iy = tid % ny, r = tid / ny;
    const int iz = r % nz, it = r / nz;
    const int x0h = j % g.h0;
    int q = j / g.h0;
    const int ly = q % ty;
    q /= ty;
    const int lz = q % tz, lt = q / tz;
    n[1] = iy * ty + ly;
    n[2] = iz * tz + lz;
    n[3] = it * tt + lt;
    n[0] = 2 * x0h + ((par + n[1] + n[2] + n[3]) & 1);
}

// Largest v over a block of 256 threads; the result is valid in thread 0.
__device__ __forceinline__ double block_max_256(double v)
{
    __shared__ double sh[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) v = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    return v;
}

// Logical block id with XCD-aware remapping: the hardware deals workgroups
// round-robin over the 8 XCDs, so logical blocks are renumbered to give each
// XCD one contiguous range of sites (neighbouring sites then share an L2).
__device__ __forceinline__ int logical_block(int b, int nblocks, int remap)
{
    if (!remap) return b;
    const int x = b & 7, y = b >> 3;
    const int q = nblocks >> 3, r = nblocks & 7;
    return (x < r) ? x * (q + 1) + y : r * (q + 1) + (x - r) * q + y;
}

// For anti-hermitian Y: Y^2 is hermitian and Y Y^2 anti-hermitian, so only
// their upper triangles are formed (half the multiply-adds of a product) and
// the lower ones mirrored.  (Y^2)_ij = -sum_k Y_ik conj(Y_jk).
template <typename R> __device__ __forceinline__ M3<R> m_sq_ah(const M3<R>& Y)
{
    M3<R> H;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        R d = R(0);
#pragma unroll
        for (int k = 0; k < 3; k++) d -= Y.re[3 * i + k] * Y.re[3 * i + k] + Y.im[3 * i + k] * Y.im[3 * i + k];
        H.re[4 * i] = d;
        H.im[4 * i] = R(0);
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = i + 1; j < 3; j++) {
            R re = R(0), im = R(0);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                re -= Y.re[3 * i + k] * Y.re[3 * j + k] + Y.im[3 * i + k] * Y.im[3 * j + k];
                im -= Y.im[3 * i + k] * Y.re[3 * j + k] - Y.re[3 * i + k] * Y.im[3 * j + k];
            }
            H.re[3 * i + j] = re;
            H.im[3 * i + j] = im;
            H.re[3 * j + i] = re;
            H.im[3 * j + i] = -im;
        }
    return H;
}

// Exponential of an anti-hermitian traceless 3x3 matrix X: Taylor series of
// order N of X / 2^s followed by s squarings, with s chosen so that the
// Frobenius norm of X / 2^s is at most 2^-L (the remainder is then below
// 2^(-L (N+1)) / (N+1)!).
//
// The polynomial is evaluated through the Cayley-Hamilton identity of a
// traceless 3x3 matrix, Y^3 = q Y + d 1 with q = tr(Y^2) / 2 (real for
// anti-hermitian Y) and d = det Y (imaginary): every power is
// Y^k = a_k 1 + b_k Y + c_k Y^2 with a_k+1 = c_k d, b_k+1 = a_k + c_k q and
// c_k+1 = b_k, so E = 1 + (Y + Y^2/2) + (A 1 + B Y + C Y^2) with the complex
// scalars A, B, C the sums over k = 3..N of (a_k, b_k, c_k) / k!.  One half
// product (Y^2) and a determinant take the place of N - 1 matrix products
// (Horner).  The bracket is summed at its own scale, small terms first, and
// the identity added last: added first, small terms of one sign (the real
// diagonal of Y^4/24 is positive) are each rounded on the grid of 1, which in
// fp32 biases E's unitarity the same way on every link.
template <typename R, int N, int L = 2> __device__ __forceinline__ M3<R> m_exp_ah(const M3<R>& X)
{
    R nrm = R(0);
#pragma unroll
    for (int k = 0; k < 9; k++) nrm += X.re[k] * X.re[k] + X.im[k] * X.im[k];
    nrm = m_sqrt(nrm);
    const R lim = R(1) / R(1 << L);
    int s = 0;
    R sc = R(1);
    while (nrm * sc > lim && s < 40) {
        sc *= R(0.5);
        s++;
    }
    M3<R> Y;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        Y.re[k] = X.re[k] * sc;
        Y.im[k] = X.im[k] * sc;
    }
    static_assert(N >= 3, "Cayley-Hamilton form from order 3");
    const M3<R> Y2 = m_sq_ah(Y);
    const R q = R(0.5) * (Y2.re[0] + Y2.re[4] + Y2.re[8]);
    // Im det Y by cofactors along row 0
    R dl;
    {
        const R m0r = Y.re[4] * Y.re[8] - Y.im[4] * Y.im[8] - (Y.re[5] * Y.re[7] - Y.im[5] * Y.im[7]);
        const R m0i = Y.re[4] * Y.im[8] + Y.im[4] * Y.re[8] - (Y.re[5] * Y.im[7] + Y.im[5] * Y.re[7]);
        const R m1r = Y.re[3] * Y.re[8] - Y.im[3] * Y.im[8] - (Y.re[5] * Y.re[6] - Y.im[5] * Y.im[6]);
        const R m1i = Y.re[3] * Y.im[8] + Y.im[3] * Y.re[8] - (Y.re[5] * Y.im[6] + Y.im[5] * Y.re[6]);
        const R m2r = Y.re[3] * Y.re[7] - Y.im[3] * Y.im[7] - (Y.re[4] * Y.re[6] - Y.im[4] * Y.im[6]);
        const R m2i = Y.re[3] * Y.im[7] + Y.im[3] * Y.re[7] - (Y.re[4] * Y.im[6] + Y.im[4] * Y.re[6]);
        dl = (Y.re[0] * m0i + Y.im[0] * m0r) - (Y.re[1] * m1i + Y.im[1] * m1r) + (Y.re[2] * m2i + Y.im[2] * m2r);
    }
    // (A, B, C) = sum_k v_k / k! for v_k = (a_k, b_k, c_k) = M^(k-3) v_3,
    // v_3 = (d, q, 0), M v = (c d, a + c q, b): by Horner in M,
    // (1/3!) [v_3 + M/4 (v_3 + M/5 (... (v_3 + M/N v_3)))], smallest
    // terms first and six scalars live.
    R wAr = R(0), wAi = dl, wBr = q, wBi = R(0), wCr = R(0), wCi = R(0);
#pragma unroll
    for (int k = N; k >= 4; k--) {
        const R f = R(1.0 / k);
        const R mAr = -wCi * dl, mAi = wCr * dl;
        const R mBr = wAr + wCr * q, mBi = wAi + wCi * q;
        const R mCr = wBr, mCi = wBi;
        wAr = mAr * f;
        wAi = dl + mAi * f;
        wBr = q + mBr * f;
        wBi = mBi * f;
        wCr = mCr * f;
        wCi = mCi * f;
    }
    const R sixth = R(1.0 / 6);
    const R Ar = wAr * sixth, Ai = wAi * sixth, Br = wBr * sixth, Bi = wBi * sixth, Cr = wCr * sixth,
            Ci = wCi * sixth;
    M3<R> E;
#pragma unroll
    for (int e = 0; e < 9; e++) {
        R sr = Br * Y.re[e] - Bi * Y.im[e] + (Cr * Y2.re[e] - Ci * Y2.im[e]);
        R si = Br * Y.im[e] + Bi * Y.re[e] + (Cr * Y2.im[e] + Ci * Y2.re[e]);
        if (e % 4 == 0) {
            sr += Ar;
            si += Ai;
        }
        E.re[e] = (Y.re[e] + Y2.re[e] * R(0.5)) + sr;
        E.im[e] = (Y.im[e] + Y2.im[e] * R(0.5)) + si;
    }
#pragma unroll
    for (int e = 0; e < 9; e += 4) E.re[e] += R(1);
    for (int k = 0; k < s; k++) E = m_mul(E, E);
    return E;
}

}  // namespace msmc
