// k_hmc.hip -- HMC momentum refresh, fused kick-drift leapfrog step and the
// kinetic-energy reduction (Sec. IV.E, App. A).
//
// Momenta: p^a, a = 1..8, per link, P = sum_a p^a lambda^a / 2, stored as 8
// reals per link in the same structure-of-arrays scheme as the links:
// one 8-real record per link in the tiled record layout (slabs cs8 bytes
// apart), p^1..p^8 in order.
// Equations of motion dU/dtau = i P U, dp^a/dtau = -F^a with
// F^a = dS/d omega^a = (beta/6) Im Tr(lambda^a U A) for U -> exp(i omega T) U.
//
// One leapfrog step is fused into one kernel: p <- p - eps_kick F(U_src) and
// then U_dst = exp(i eps_drift P) U_src; U_src and U_dst are different
// buffers because the staples of other threads read U_src.
#include "kernels.hpp"
#include "pair_walk.hpp"

namespace msmc {

__device__ __forceinline__ int find_lattice_h(const int* __restrict__ bbeg, int nlat, int lb)
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

struct LinkIdxH {
    int l, mu, par, cb;
    bool valid;
};

__device__ __forceinline__ LinkIdxH link_index_h(const Grid& gr)
{
    LinkIdxH x;
    const int lb = logical_block(blockIdx.x, gr.nblocks, gr.remap);
    x.l = find_lattice_h(gr.bbeg, gr.nlat, lb);
    const int Vh = gr.descs[x.l].g.Vh;
    const int e = (lb - gr.bbeg[x.l]) * (int)blockDim.x + (int)threadIdx.x;
    x.valid = e < 8 * Vh;
    const int slab = e / Vh;
    x.cb = e - slab * Vh;
    x.mu = slab >> 1;
    x.par = slab & 1;
    return x;
}

template <typename R> __global__ void __launch_bounds__(256) k_mom(Grid gr, uint64_t traj)
{
    const LinkIdxH x = link_index_h(gr);
    if (!x.valid) return;
    const LatDesc& d = gr.descs[x.l];
    int n[4];
    cb_coords(d.g, x.cb, x.par, n);
    const Rng rng{ d.seed, d.lid, (uint32_t)lex_index(d.g, n), traj };
    double z[8];
    normals4<double>(rng.draw(ctr_word(P_MOM, x.mu, 0, 0, 0)), z);
    normals4<double>(rng.draw(ctr_word(P_MOM, x.mu, 0, 0, 1)), z + 4);
    R p[8];
#pragma unroll
    for (int a = 0; a < 8; a++) p[a] = (R)z[a];
    store_reals<R, 8>((uintptr_t)d.aux + (uintptr_t)(x.mu * 2 + x.par) * d.cs8, x.cb, p);
}

// i eps P as a 3x3 matrix (anti-hermitian, traceless)
template <typename R> __device__ __forceinline__ M3<R> i_eps_P(const R p[8], R eps)
{
    const R s3 = R(0.57735026918962576451);  // 1/sqrt(3)
    // hermitian P
    R pre[9], pim[9];
    pre[0] = R(0.5) * (p[2] + p[7] * s3);
    pim[0] = R(0);
    pre[4] = R(0.5) * (-p[2] + p[7] * s3);
    pim[4] = R(0);
    pre[8] = -p[7] * s3;
    pim[8] = R(0);
    pre[1] = R(0.5) * p[0];
    pim[1] = -R(0.5) * p[1];
    pre[3] = R(0.5) * p[0];
    pim[3] = R(0.5) * p[1];
    pre[2] = R(0.5) * p[3];
    pim[2] = -R(0.5) * p[4];
    pre[6] = R(0.5) * p[3];
    pim[6] = R(0.5) * p[4];
    pre[5] = R(0.5) * p[5];
    pim[5] = -R(0.5) * p[6];
    pre[7] = R(0.5) * p[5];
    pim[7] = R(0.5) * p[6];
    M3<R> X;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        X.re[k] = -eps * pim[k];
        X.im[k] = eps * pre[k];
    }
    return X;
}

template <typename R> struct ExpOrder;
template <> struct ExpOrder<double> { static constexpr int N = 12; };
// fp32: the argument is scaled to norm <= 1/4, where the order-6 remainder
// (< 1/4^7/7!, about 1.2e-8) is below fp32 rounding.
template <> struct ExpOrder<float> { static constexpr int N = 6; };

// The kick of link U_mu at (par, cb) from its staple A, then the drift into
// the destination buffer.
template <typename R, int NC>
__device__ __forceinline__ void kick_drift_link(const LatDesc& d, int mu, int par, int cb, const M3<R>& u,
                                                const M3<R>& A, double eps_kick, double eps_drift, int drift)
{
    const M3<R> Om = m_mul(u, A);
    const R b6 = (R)(d.beta / 6.0);
    const R s3 = R(0.57735026918962576451);
    R F[8];
    F[0] = b6 * (Om.im[1] + Om.im[3]);
    F[1] = b6 * (Om.re[1] - Om.re[3]);
    F[2] = b6 * (Om.im[0] - Om.im[4]);
    F[3] = b6 * (Om.im[2] + Om.im[6]);
    F[4] = b6 * (Om.re[2] - Om.re[6]);
    F[5] = b6 * (Om.im[5] + Om.im[7]);
    F[6] = b6 * (Om.re[5] - Om.re[7]);
    F[7] = b6 * s3 * (Om.im[0] + Om.im[4] - R(2) * Om.im[8]);
    const uintptr_t pslab = (uintptr_t)d.aux + (uintptr_t)(mu * 2 + par) * d.cs8;
    R p[8];
    load_reals<R, 8>(pslab, cb, p);
    const R ek = (R)eps_kick;
#pragma unroll
    for (int a = 0; a < 8; a++) p[a] = p[a] - ek * F[a];
    store_reals<R, 8>(pslab, cb, p);
    if (drift) {
        const M3<R> E = m_exp_ah<R, ExpOrder<R>::N, 2, true>(i_eps_P(p, (R)eps_drift));
        const Links<R, NC> D{ (uintptr_t)d.aux2, d.cs };
        M3<R> un = m_mul(E, u);
        // fp32 links are re-orthonormalized in fp64 and rounded once at every
        // drift: for 12-real records row 2 is rebuilt from rows 0 and 1, whose
        // rounding would otherwise feed back; for 18-real records the rounding
        // of the product leaves a drift away from SU(3) that grows with the
        // number of steps, and with it an energy error that no longer falls
        // with the step size (+0.5 in dH after 182 steps at 32^3 x 72).
        if constexpr (std::is_same<R, float>::value) m_reunit_for_store(un);
        store_link<R, NC>(D.slab(mu, par), cb, un);
    }
}

// fp64: one link per thread in the link walk of four directions of 64 sites.
template <typename R, int NC>
__global__ void __launch_bounds__(256) k_kick_drift(Grid gr, double eps_kick, double eps_drift, int drift)
{
    const LinkWalk x = link_walk(gr);
    if (!x.valid) return;
    const LatDesc& d = gr.descs[x.l];
    const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
    const M3<R> A = staple_sum<R, NC, R>(U, d.g, x.mu, x.n);
    const M3<R> u = load_link<R, NC>(U.slab(x.mu, x.par), x.cb);
    kick_drift_link<R, NC>(d, x.mu, x.par, x.cb, u, A, eps_kick, eps_drift, drift);
}

// fp32: the pair walk (PairWalk), 512 threads per block.
template <int NC>
__global__ void __launch_bounds__(512, 4) k_kick_drift_pair(Grid gr, double eps_kick, double eps_drift, int drift)
{
    __shared__ PairLds lds;
    const PairWalk<NC> pw = pair_walk<NC>(gr, lds);
    if (!pw.valid) return;
    const PairLd<NC> ld = pw.loader(lds);
    const M3<float> A = staple_sum_rows<NC, false>(ld, pw.g, pw.mu, pw.n, nullptr);
    // the own link again from LDS rather than held in registers through the staple
    kick_drift_link<float, NC>(*pw.d, pw.mu, pw.par, pw.cb, ld.from_lds(pw.own), A, eps_kick, eps_drift, drift);
}

__device__ __forceinline__ double block_sum_256h(double v)
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

// (1/2) sum_a p^a p^a per link, summed per block of 256 links (not remapped)
template <typename R> __global__ void __launch_bounds__(256) k_kinetic(Grid gr, double* __restrict__ partials)
{
    const int lb = blockIdx.x;
    const int l = find_lattice_h(gr.bbeg, gr.nlat, lb);
    const LatDesc& d = gr.descs[l];
    const int e = (lb - gr.bbeg[l]) * 256 + (int)threadIdx.x;
    double k = 0.0;
    if (e < 8 * d.g.Vh) {
        const int slab = e / d.g.Vh, cb = e - slab * d.g.Vh;
        R pv[8];
        load_reals<R, 8>((uintptr_t)d.aux + (uintptr_t)slab * d.cs8, cb, pv);
#pragma unroll
        for (int a = 0; a < 8; a++) {
            const double v = (double)pv[a];
            k += 0.5 * v * v;
        }
    }
    k = block_sum_256h(k);
    if (threadIdx.x == 0) partials[blockIdx.x] = k;
}

hipError_t launch_mom_refresh(int prec, const Grid& gr, uint64_t traj, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    if (prec == PREC_F64)
        k_mom<double><<<gr.nblocks, gr.block, 0, st>>>(gr, traj);
    else
        k_mom<float><<<gr.nblocks, gr.block, 0, st>>>(gr, traj);
    return hipGetLastError();
}

hipError_t launch_kick_drift(int prec, const Grid& gr, double eps_kick, double eps_drift, int drift, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    switch (prec) {
    case PREC_F64: k_kick_drift<double, 18><<<gr.nblocks, gr.block, 0, st>>>(gr, eps_kick, eps_drift, drift); break;
    case PREC_F32:
        k_kick_drift_pair<18><<<gr.nblocks / 2, 512, 0, st>>>(gr, eps_kick, eps_drift, drift);
        break;
    case PREC_F32_R12:
        k_kick_drift_pair<12><<<gr.nblocks / 2, 512, 0, st>>>(gr, eps_kick, eps_drift, drift);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_kinetic_partial(int prec, const Grid& gr, double* partials, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    if (prec == PREC_F64)
        k_kinetic<double><<<gr.nblocks, 256, 0, st>>>(gr, partials);
    else
        k_kinetic<float><<<gr.nblocks, 256, 0, st>>>(gr, partials);
    return hipGetLastError();
}

}  // namespace msmc
