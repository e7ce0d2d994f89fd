// k_measure.hip -- fp64 reductions: Wilson action density (plaquette), clover
// topological charge and clover energy density.  Every reduction uses blocks
// of 256 threads, one site per thread, a wavefront shuffle tree, then one
// final block per lattice that adds the block partials in a fixed order, so
// results are bitwise reproducible and independent of the launch shapes
// chosen for the update kernels.
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
    int l, n[4];
    bool valid;
};

__device__ __forceinline__ SiteIdx site_index(const Grid& gr)
{
    SiteIdx s;
    const int lb = blockIdx.x;  // reductions are not remapped
    s.l = find_lattice_m(gr.bbeg, gr.nlat, lb);
    const Geo g = gr.descs[s.l].g;
    const int e = (lb - gr.bbeg[s.l]) * 256 + (int)threadIdx.x;
    s.valid = e < 2 * g.Vh;
    if (s.valid) {
        const int par = e >= g.Vh ? 1 : 0;
        cb_coords(g, e - par * g.Vh, par, s.n);
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

// sum_{mu<nu} [1 - (1/3) Re Tr U_mu(n) U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+]
template <typename R, int NC> __global__ void __launch_bounds__(256) k_plaq(Grid gr, double* __restrict__ partials)
{
    const SiteIdx s = site_index(gr);
    double acc = 0.0;
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
                acc += 1.0 - t / 3.0;
            }
        }
    }
    acc = block_sum_256(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
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
    const SiteIdx s = site_index(gr);
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
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// sum_{mu<nu} -Re Tr(F_munu F_munu) per site
template <typename R, int NC> __global__ void __launch_bounds__(256) k_energy(Grid gr, double* __restrict__ partials)
{
    const SiteIdx s = site_index(gr);
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
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
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

hipError_t launch_reduce_final(const Grid& gr, const double* partials, double* out, int stride, int off, hipStream_t st)
{
    if (gr.nlat <= 0) return hipSuccess;
    k_reduce_final<<<gr.nlat, 256, 0, st>>>(gr.bbeg, partials, out, stride, off);
    return hipGetLastError();
}

}  // namespace msmc
