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
//
// Fused multiply-adds are allowed in this unit (the pragma precedes the
// headers so that their inline arithmetic is contracted too): a trajectory
// is not chaotic at its length, and contraction saves 4 % of the fp32 step's
// instructions.  The kick and the drift generator are formed in fp64 with the
// exact step (hmc_step.hpp), which keeps dH unbiased either way.
#pragma clang fp contract(fast)
#include "hmc_step.hpp"
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

// fp32: the pair walk (PairWalk), 512 threads per block.
template <int NC>
__global__ void __launch_bounds__(512, 4) k_kick_drift_pair(Grid gr, double eps_kick, double eps_drift, int drift)
{
    __shared__ PairLds lds;
    __shared__ PairQLds qlds;
    const PairWalk<NC> pw = pair_walk<NC>(gr, lds);
    const PairLd<NC> ld = pw.loader(lds);
    const M3<float> A = pair_staple<NC>(pw, ld, qlds);
    if (!pw.valid) return;
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
    case PREC_F64: return launch_kick_drift_f64(gr, eps_kick, eps_drift, drift, st);
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
