// k_measure.hip -- fp64 reductions: Wilson action density (plaquette), clover
// topological charge and clover energy density.  Every reduction uses blocks
// of 256 threads, one site per thread, a wavefront shuffle tree, then one
// final block per lattice that adds the block partials in a fixed order, so
// results are bitwise reproducible and independent of the launch shapes
// chosen for the update kernels and of the hardware block order.
#include "kernels.hpp"

namespace msmc {

__device__ __forceinline__ int find_lattice_m(const int* __restrict__ bbeg, int nlat, int lb)
{
    int lo = 0, hi = nlat - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (bbeg[mid] <= lb)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Sum over a block of 256 threads; the result is valid in thread 0.
__device__ __forceinline__ double block_sum_256(double v)
{
    __shared__ double sh[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) v = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return v;
}

struct SiteIdx {
    int l, lb, n[4];
    bool valid;
};

// Site of this thread.  Both parities are interleaved: sites are walked in
// tiles of L0 x ty x tz x tt (tiles ordered y, z, t; inside a tile x fastest,
// then y, z, t), so the forward neighbours a site reads are the own links of
// threads that run at nearly the same time on the same XCD.  The mapping
// depends only on the logical block, and block partials are stored by
// logical block, so sums do not depend on the hardware block order.
__device__ __forceinline__ SiteIdx site_index(const Grid& gr, int b)
{
    SiteIdx s;
    s.lb = logical_block(b, gr.nblocks, gr.remap);
    s.l = find_lattice_m(gr.bbeg, gr.nlat, s.lb);
    const LatDesc& d = gr.descs[s.l];
    const Geo g = d.g;
    const int e = (s.lb - gr.bbeg[s.l]) * 256 + (int)threadIdx.x;
    s.valid = e < 2 * g.Vh;
    if (s.valid) {
        const int ty = d.mtile[0], tz = d.mtile[1], tt = d.mtile[2];
        const int th = g.L[0] * ty * tz * tt;
        const int tid = e / th, j = e - tid * th;
        const int ny = g.L[1] / ty, nz = g.L[2] / tz;
        const int iy = tid % ny, r = tid / ny;
        const int iz = r % nz, it = r / nz;
        s.n[0] = j % g.L[0];
        int q = j / g.L[0];
        const int ly = q % ty;
        q /= ty;
        const int lz = q % tz, lt = q / tz;
        s.n[1] = iy * ty + ly;
        s.n[2] = iz * tz + lz;
        s.n[3] = it * tt + lt;
    }
    return s;
}

template <typename R, int NC>
__device__ __forceinline__ M3<double> ld_d(const Links<R, NC>& U, const Geo& g, int mu, const int n[4])
{
    return m_cast<R, double>(load_at(U, g, mu, n));
}

__device__ __forceinline__ void shifted(const int n[4], const Geo& g, int mu, int smu, int nu, int snu, int out[4])
{
    out[0] = n[0];
    out[1] = n[1];
    out[2] = n[2];
    out[3] = n[3];
    if (smu) out[mu] = wrap_add(out[mu], smu, g.L[mu]);
    if (snu) out[nu] = wrap_add(out[nu], snu, g.L[nu]);
}

// Rows 0 and 1 of X = A B for a 12-real A (rows 0, 1 only) and a full B,
// in fp32 with explicit fused multiply-adds.
__device__ __forceinline__ void rows01_mul(const float a[12], const M3<float>& b, float xr[6], float xi[6])
{
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const float ar = a[6 * r + 2 * k], ai = a[6 * r + 2 * k + 1];
                re = fmaf(ar, b.re[3 * k + c], re);
                re = fmaf(-ai, b.im[3 * k + c], re);
                im = fmaf(ar, b.im[3 * k + c], im);
                im = fmaf(ai, b.re[3 * k + c], im);
            }
            xr[3 * r + c] = re;
            xi[3 * r + c] = im;
        }
}

// Re Tr(X Y^+) for X, Y in SU(3) from their rows 0 and 1 alone.  With
// s_ij = sum_k X_ik conj(Y_jk) (i, j = 0, 1) the third rows, being
// conj(row0 x row1), contribute conj(s00 s11 - s01 s10); hence
// Re Tr(X Y^+) = Re(s00 + s11 + s00 s11 - s01 s10).
__device__ __forceinline__ float retr_rows01(const float xr[6], const float xi[6], const float yr[6], const float yi[6])
{
    float sr[2][2], si[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                re = fmaf(xr[3 * i + k], yr[3 * j + k], re);
                re = fmaf(xi[3 * i + k], yi[3 * j + k], re);
                im = fmaf(xi[3 * i + k], yr[3 * j + k], im);
                im = fmaf(-xr[3 * i + k], yi[3 * j + k], im);
            }
            sr[i][j] = re;
            si[i][j] = im;
        }
    float t = sr[0][0] + sr[1][1];
    t = fmaf(sr[0][0], sr[1][1], t);
    t = fmaf(-si[0][0], si[1][1], t);
    t = fmaf(-sr[0][1], sr[1][0], t);
    t = fmaf(si[0][1], si[1][0], t);
    return t;
}

// X = A B in fp32 with explicit fused multiply-adds (this unit is compiled
// without contraction).
__device__ __forceinline__ M3<float> mul_fma(const M3<float>& a, const M3<float>& b)
{
    M3<float> x;
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                re = fmaf(a.re[3 * r + k], b.re[3 * k + c], re);
                re = fmaf(-a.im[3 * r + k], b.im[3 * k + c], re);
                im = fmaf(a.re[3 * r + k], b.im[3 * k + c], im);
                im = fmaf(a.im[3 * r + k], b.re[3 * k + c], im);
            }
            x.re[3 * r + c] = re;
            x.im[3 * r + c] = im;
        }
    return x;
}

// sum_{mu<nu} [1 - (1/3) Re Tr U_mu(n) U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+]
// Each plane term is formed per site and summed in fp64.  fp64 fields
// multiply in fp64; 18-real fp32 fields form the two half-plaquettes in fp32
// (no SU(3) property assumed) and trace them in fp64; 12-real fields, whose
// third rows are by construction conj(row0 x row1), form only rows 0 and 1 of
// the two half-plaquettes in fp32 (the SU(3) identity above).
template <typename R, int NC, bool GATED = false>
__global__ void __launch_bounds__(256) k_plaq(Grid gr, double* __restrict__ partials,
                                              const uint64_t* __restrict__ sweep_base = nullptr, int sweep_off = 0,
                                              int every = 0)
{
    if constexpr (GATED) {
        const uint64_t sw = *sweep_base + (uint64_t)sweep_off;
        if ((sw + 1) % (uint64_t)every != 0) return;
    }
    // blocks loop over the logical blocks, so that a gated launch can use a
    // small grid (most sweeps it exits at once)
    for (int b = blockIdx.x; b < gr.nblocks; b += gridDim.x) {
    const SiteIdx s = site_index(gr, b);
    double acc = 0.0;
    if (s.valid) {
        const LatDesc& d = gr.descs[s.l];
        const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
        if constexpr (NC == 12) {
            const int cb = lex_index(d.g, s.n) >> 1;
            const int par = (s.n[0] + s.n[1] + s.n[2] + s.n[3]) & 1;
            float own[4][12];
#pragma unroll
            for (int mu = 0; mu < 4; mu++) load_reals<float, 12>(U.slab(mu, par), cb, own[mu]);
#pragma unroll
            for (int mu = 0; mu < 4; mu++) {
                int npm[4];
                shifted(s.n, d.g, mu, 1, 0, 0, npm);
#pragma unroll
                for (int nu = mu + 1; nu < 4; nu++) {
                    int npn[4];
                    shifted(s.n, d.g, nu, 1, 0, 0, npn);
                    float xr[6], xi[6], yr[6], yi[6];
                    rows01_mul(own[mu], load_at(U, d.g, nu, npm), xr, xi);
                    rows01_mul(own[nu], load_at(U, d.g, mu, npn), yr, yi);
                    acc += 1.0 - (double)retr_rows01(xr, xi, yr, yi) / 3.0;
                }
            }
        } else if constexpr (std::is_same<R, float>::value) {
            const int cb = lex_index(d.g, s.n) >> 1;
            const int par = (s.n[0] + s.n[1] + s.n[2] + s.n[3]) & 1;
            M3<float> own[4];
#pragma unroll
            for (int mu = 0; mu < 4; mu++) own[mu] = load_link<float, NC>(U.slab(mu, par), cb);
#pragma unroll
            for (int mu = 0; mu < 4; mu++) {
                int npm[4];
                shifted(s.n, d.g, mu, 1, 0, 0, npm);
#pragma unroll
                for (int nu = mu + 1; nu < 4; nu++) {
                    int npn[4];
                    shifted(s.n, d.g, nu, 1, 0, 0, npn);
                    const M3<float> X = mul_fma(own[mu], load_at(U, d.g, nu, npm));
                    const M3<float> Y = mul_fma(own[nu], load_at(U, d.g, mu, npn));
                    double t = 0.0;
#pragma unroll
                    for (int k = 0; k < 9; k++) t += (double)fmaf(X.re[k], Y.re[k], X.im[k] * Y.im[k]);
                    acc += 1.0 - t / 3.0;
                }
            }
        } else {
#pragma unroll
            for (int mu = 0; mu < 4; mu++) {
                int npm[4];
                shifted(s.n, d.g, mu, 1, 0, 0, npm);
                const M3<double> umu = ld_d(U, d.g, mu, s.n);
#pragma unroll
                for (int nu = mu + 1; nu < 4; nu++) {
                    int npn[4];
                    shifted(s.n, d.g, nu, 1, 0, 0, npn);
                    const M3<double> X = m_mul(umu, ld_d(U, d.g, nu, npm));
                    const M3<double> Y = m_mul(ld_d(U, d.g, nu, s.n), ld_d(U, d.g, mu, npn));
                    double t = 0.0;
#pragma unroll
                    for (int k = 0; k < 9; k++) t += X.re[k] * Y.re[k] + X.im[k] * Y.im[k];
                    acc += 1.0 - t / 3.0;
                }
            }
        }
    }
    acc = block_sum_256(acc);
    if (threadIdx.x == 0) partials[s.lb] = acc;
    __syncthreads();  // the shared slots of block_sum_256 are reused
    }
}

// Clover field strength: traceless part of (Q - Q^+)/8, Q the sum of the
// four counter-clockwise leaves of the mu-nu plane at x.
template <typename R, int NC>
__device__ __forceinline__ M3<double> clover_F(const Links<R, NC>& U, const Geo& g, const int x[4], int mu, int nu)
{
    int xpm[4], xpn[4], xmm[4], xmn[4], xmm_pn[4], xmm_mn[4], xpm_mn[4];
    shifted(x, g, mu, 1, nu, 0, xpm);
    shifted(x, g, mu, 0, nu, 1, xpn);
    shifted(x, g, mu, -1, nu, 0, xmm);
    shifted(x, g, mu, 0, nu, -1, xmn);
    shifted(x, g, mu, -1, nu, 1, xmm_pn);
    shifted(x, g, mu, -1, nu, -1, xmm_mn);
    shifted(x, g, mu, 1, nu, -1, xpm_mn);
    M3<double> Q;
    {
        const M3<double> a = m_mul(ld_d(U, g, mu, x), ld_d(U, g, nu, xpm));
        const M3<double> b = m_mul(ld_d(U, g, nu, x), ld_d(U, g, mu, xpn));
        Q = m_mul_nd(a, b);
    }
    {
        const M3<double> a = m_mul_nd(ld_d(U, g, nu, x), ld_d(U, g, mu, xmm_pn));
        const M3<double> b = m_mul_dn(ld_d(U, g, nu, xmm), ld_d(U, g, mu, xmm));
        m_acc(Q, m_mul(a, b));
    }
    {
        const M3<double> a = m_mul_dd(ld_d(U, g, mu, xmm), ld_d(U, g, nu, xmm_mn));
        const M3<double> b = m_mul(ld_d(U, g, mu, xmm_mn), ld_d(U, g, nu, xmn));
        m_acc(Q, m_mul(a, b));
    }
    {
        const M3<double> a = m_mul_dn(ld_d(U, g, nu, xmn), ld_d(U, g, mu, xmn));
        const M3<double> b = m_mul_nd(ld_d(U, g, nu, xpm_mn), ld_d(U, g, mu, x));
        m_acc(Q, m_mul(a, b));
    }
    M3<double> F;
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            F.re[r * 3 + c] = 0.125 * (Q.re[r * 3 + c] - Q.re[c * 3 + r]);
            F.im[r * 3 + c] = 0.125 * (Q.im[r * 3 + c] + Q.im[c * 3 + r]);
        }
    const double ti = (F.im[0] + F.im[4] + F.im[8]) / 3.0;
    F.im[0] -= ti;
    F.im[4] -= ti;
    F.im[8] -= ti;
    return F;
}

__device__ __forceinline__ double retr_prod(const M3<double>& a, const M3<double>& b)
{
    double t = 0.0;
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int k = 0; k < 3; k++) t += a.re[r * 3 + k] * b.re[k * 3 + r] - a.im[r * 3 + k] * b.im[k * 3 + r];
    return t;
}

// q(x) = -(1/(2 pi^2)) Re Tr[F01 F23 - F02 F13 + F03 F12]
template <typename R, int NC> __global__ void __launch_bounds__(256) k_qtop(Grid gr, double* __restrict__ partials)
{
    const SiteIdx s = site_index(gr, blockIdx.x);
    double acc = 0.0;
    if (s.valid) {
        const LatDesc& d = gr.descs[s.l];
        const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
        double t = 0.0;
        {
            const M3<double> a = clover_F(U, d.g, s.n, 0, 1);
            const M3<double> b = clover_F(U, d.g, s.n, 2, 3);
            t += retr_prod(a, b);
        }
        {
            const M3<double> a = clover_F(U, d.g, s.n, 0, 2);
            const M3<double> b = clover_F(U, d.g, s.n, 1, 3);
            t -= retr_prod(a, b);
        }
        {
            const M3<double> a = clover_F(U, d.g, s.n, 0, 3);
            const M3<double> b = clover_F(U, d.g, s.n, 1, 2);
            t += retr_prod(a, b);
        }
        acc = -t / (2.0 * M_PI * M_PI);
    }
    acc = block_sum_256(acc);
    if (threadIdx.x == 0) partials[s.lb] = acc;
}

// sum_{mu<nu} -Re Tr(F_munu F_munu) per site
template <typename R, int NC> __global__ void __launch_bounds__(256) k_energy(Grid gr, double* __restrict__ partials)
{
    const SiteIdx s = site_index(gr, blockIdx.x);
    double acc = 0.0;
    if (s.valid) {
        const LatDesc& d = gr.descs[s.l];
        const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                const M3<double> F = clover_F(U, d.g, s.n, mu, nu);
                acc -= retr_prod(F, F);
            }
    }
    acc = block_sum_256(acc);
    if (threadIdx.x == 0) partials[s.lb] = acc;
}

// Wilson loops (Sec. III, loop and partial-average equations).  For every
// site n and plane mu < nu the m x n loop
//   W = (1/3) Re Tr L_mu^m(n) L_nu^n(n + m mu) L_mu^m(n + n nu)^+ L_nu^n(n)^+,
// L_mu^m(n) the product of m links along mu, is added to a class:
//   mode 0: one class (all loops);
//   mode 1: class chi_munu(n) in 0..2, the number of odd coordinates of n
//           other than n_mu, n_nu (partially averaged plaquettes, m = n = 1);
//   mode 2: class chi(n) in 0..4, the number of odd coordinates of n
//           (displaced loops, m = n = 2).
// Block partials of class c go to partials[c * nblocks + logical block].
template <typename R, int NC>
__global__ void __launch_bounds__(256) k_loops(Grid gr, int lm, int ln, int mode, double* __restrict__ partials)
{
    const SiteIdx s = site_index(gr, blockIdx.x);
    double acc[5] = { 0.0, 0.0, 0.0, 0.0, 0.0 };
    if (s.valid) {
        const LatDesc& d = gr.descs[s.l];
        const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
        const int odd[4] = { s.n[0] & 1, s.n[1] & 1, s.n[2] & 1, s.n[3] & 1 };
#pragma unroll
        for (int mu = 0; mu < 4; mu++)
#pragma unroll
            for (int nu = mu + 1; nu < 4; nu++) {
                int x[4] = { s.n[0], s.n[1], s.n[2], s.n[3] };
                M3<double> P = ld_d(U, d.g, mu, x);
                x[mu] = wrap_add(x[mu], 1, d.g.L[mu]);
                for (int a = 1; a < lm; a++) {
                    P = m_mul(P, ld_d(U, d.g, mu, x));
                    x[mu] = wrap_add(x[mu], 1, d.g.L[mu]);
                }
                for (int b = 0; b < ln; b++) {
                    P = m_mul(P, ld_d(U, d.g, nu, x));
                    x[nu] = wrap_add(x[nu], 1, d.g.L[nu]);
                }
                for (int a = 0; a < lm; a++) {
                    x[mu] = wrap_add(x[mu], -1, d.g.L[mu]);
                    P = m_mul_nd(P, ld_d(U, d.g, mu, x));
                }
                for (int b = 0; b < ln; b++) {
                    x[nu] = wrap_add(x[nu], -1, d.g.L[nu]);
                    P = m_mul_nd(P, ld_d(U, d.g, nu, x));
                }
                const double w = (P.re[0] + P.re[4] + P.re[8]) / 3.0;
                const int all = odd[0] + odd[1] + odd[2] + odd[3];
                const int c = mode == 0 ? 0 : (mode == 1 ? all - odd[mu] - odd[nu] : all);
#pragma unroll
                for (int k = 0; k < 5; k++)
                    if (k == c) acc[k] += w;
            }
    }
    const int nclass = mode == 0 ? 1 : (mode == 1 ? 3 : 5);
    for (int k = 0; k < nclass; k++) {
        const double v = block_sum_256(acc[k]);
        if (threadIdx.x == 0) partials[(size_t)k * gr.nblocks + s.lb] = v;
        __syncthreads();  // the next block sum reuses the shared slots
    }
}

// Admissibility measure (Sec. IV.D): per site the largest
// s_p = 3 [1 - (1/3) Re Tr U_p] over its six plaquettes, block maxima into
// partials[logical block] (0 for padding threads).
template <typename R, int NC> __global__ void __launch_bounds__(256) k_max_splaq(Grid gr, double* __restrict__ partials)
{
    const SiteIdx s = site_index(gr, blockIdx.x);
    double h = 0.0;
    if (s.valid) {
        const LatDesc& d = gr.descs[s.l];
        const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            int npm[4];
            shifted(s.n, d.g, mu, 1, 0, 0, npm);
            const M3<double> umu = ld_d(U, d.g, mu, s.n);
#pragma unroll
            for (int nu = mu + 1; nu < 4; nu++) {
                int npn[4];
                shifted(s.n, d.g, nu, 1, 0, 0, npn);
                const M3<double> X = m_mul(umu, ld_d(U, d.g, nu, npm));
                const M3<double> Y = m_mul(ld_d(U, d.g, nu, s.n), ld_d(U, d.g, mu, npn));
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < 9; k++) t += X.re[k] * Y.re[k] + X.im[k] * Y.im[k];
                h = fmax(h, 3.0 - t);
            }
        }
    }
    h = block_max_256(h);
    if (threadIdx.x == 0) partials[s.lb] = h;
}

// Block partials of the plaquette site values that the last overrelaxation
// pass of a sweep wrote (3 Vh doubles per lattice): block b of a lattice adds
// values [1024 b, 1024 b + 1024), four consecutive ones per thread, in a
// fixed order that does not depend on any launch shape.
__global__ void __launch_bounds__(256) k_psite(Grid gr, double* __restrict__ partials)
{
    const int lb = blockIdx.x;
    const int l = find_lattice_m(gr.bbeg, gr.nlat, lb);
    const LatDesc& d = gr.descs[l];
    const size_t n = (size_t)3 * d.g.Vh;
    const size_t i0 = (size_t)(lb - gr.bbeg[l]) * 1024 + 4 * (size_t)threadIdx.x;
    double v = 0.0;
    if (i0 + 4 <= n) {
        // 3 Vh is a multiple of 4 and every lattice's values start 32-byte
        // aligned: two 16-byte loads
        const v2d a = vload<true, v2d>((uintptr_t)(d.psite + i0));
        const v2d b = vload<true, v2d>((uintptr_t)(d.psite + i0 + 2));
        v = ((a.x + a.y) + b.x) + b.y;
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (i0 + k < n) v += d.psite[i0 + k];
    }
    v = block_sum_256(v);
    if (threadIdx.x == 0) partials[lb] = v;
}

// One block per lattice: the partials of (bbeg_a, pa) in sweeps that
// reunitarize, else those of (bbeg_b, pb), added in a fixed order.
__global__ void __launch_bounds__(256) k_reduce_pick(const int* __restrict__ bbeg_a, const double* __restrict__ pa,
                                                     const int* __restrict__ bbeg_b, const double* __restrict__ pb,
                                                     const uint64_t* __restrict__ sweep_base, int sweep_off, int every,
                                                     double* __restrict__ out, int stride, int off)
{
    const int l = blockIdx.x;
    bool use_a = false;
    if (every > 0) {
        const uint64_t sw = *sweep_base + (uint64_t)sweep_off;
        use_a = (sw + 1) % (uint64_t)every == 0;
    }
    const int* bbeg = use_a ? bbeg_a : bbeg_b;
    const double* p = use_a ? pa : pb;
    const int b0 = bbeg[l], b1 = bbeg[l + 1];
    double v = 0.0;
    for (int k = b0 + (int)threadIdx.x; k < b1; k += 256) v += p[k];
    v = block_sum_256(v);
    if (threadIdx.x == 0) out[(size_t)l * stride + off] = v;
}

// One block per lattice: out[l * stride + off] = sum of its partials.
__global__ void __launch_bounds__(256) k_reduce_final(const int* __restrict__ bbeg, const double* __restrict__ partials,
                                                      double* __restrict__ out, int stride, int off)
{
    const int l = blockIdx.x;
    const int b0 = bbeg[l], b1 = bbeg[l + 1];
    double v = 0.0;
    for (int k = b0 + (int)threadIdx.x; k < b1; k += 256) v += partials[k];
    v = block_sum_256(v);
    if (threadIdx.x == 0) out[(size_t)l * stride + off] = v;
}

#define DISPATCH_PREC_M(prec, CALL)                                              \
    switch (prec) {                                                              \
    case PREC_F64: { using R = double; constexpr int NC = 18; CALL; } break;     \
    case PREC_F32: { using R = float; constexpr int NC = 18; CALL; } break;      \
    case PREC_F32_R12: { using R = float; constexpr int NC = 12; CALL; } break;  \
    default: return hipErrorInvalidValue;                                        \
    }

hipError_t launch_plaq_partial(int prec, const Grid& gr, double* partials, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    DISPATCH_PREC_M(prec, (k_plaq<R, NC><<<gr.nblocks, 256, 0, st>>>(gr, partials)));
    return hipGetLastError();
}

hipError_t launch_plaq_partial_gated(int prec, const Grid& gr, double* partials, const uint64_t* sweep_base,
                                     int sweep_off, int every, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    if (every <= 0) return hipErrorInvalidValue;
    const int nb = gr.nblocks < 2048 ? gr.nblocks : 2048;
    DISPATCH_PREC_M(prec, (k_plaq<R, NC, true><<<nb, 256, 0, st>>>(gr, partials, sweep_base, sweep_off, every)));
    return hipGetLastError();
}

hipError_t launch_psite_partial(const Grid& gr, double* partials, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    k_psite<<<gr.nblocks, 256, 0, st>>>(gr, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_pick(int nlat, const int* bbeg_a, const double* pa, const int* bbeg_b, const double* pb,
                              const uint64_t* sweep_base, int sweep_off, int every, double* out, int stride, int off,
                              hipStream_t st)
{
    if (nlat <= 0) return hipSuccess;
    k_reduce_pick<<<nlat, 256, 0, st>>>(bbeg_a, pa, bbeg_b, pb, sweep_base, sweep_off, every, out, stride, off);
    return hipGetLastError();
}

hipError_t launch_qtop_partial(int prec, const Grid& gr, double* partials, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    DISPATCH_PREC_M(prec, (k_qtop<R, NC><<<gr.nblocks, 256, 0, st>>>(gr, partials)));
    return hipGetLastError();
}

hipError_t launch_energy_partial(int prec, const Grid& gr, double* partials, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    DISPATCH_PREC_M(prec, (k_energy<R, NC><<<gr.nblocks, 256, 0, st>>>(gr, partials)));
    return hipGetLastError();
}

hipError_t launch_loops_partial(int prec, const Grid& gr, int m, int n, int mode, double* partials, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    DISPATCH_PREC_M(prec, (k_loops<R, NC><<<gr.nblocks, 256, 0, st>>>(gr, m, n, mode, partials)));
    return hipGetLastError();
}

hipError_t launch_max_splaq_partial(int prec, const Grid& gr, double* partials, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    DISPATCH_PREC_M(prec, (k_max_splaq<R, NC><<<gr.nblocks, 256, 0, st>>>(gr, partials)));
    return hipGetLastError();
}

hipError_t launch_reduce_final(const Grid& gr, const double* partials, double* out, int stride, int off, hipStream_t st)
{
    if (gr.nlat <= 0) return hipSuccess;
    k_reduce_final<<<gr.nlat, 256, 0, st>>>(gr.bbeg, partials, out, stride, off);
    return hipGetLastError();
}

}  // namespace msmc
