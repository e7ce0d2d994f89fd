// k_flow.hip -- one stage of the third-order Runge-Kutta Wilson flow
// (Sec. IV.B) in 2N-storage form.
//
// Z(W) = -(1/2)(Om - Om^+) + (1/6) Tr(Om - Om^+), Om = W A (A the staple
// sum); the three stages are W1 = exp(Z0/4) W0, W2 = exp(8/9 Z1 - 17/36 Z0) W1,
// W3 = exp(3/4 Z2 - 8/9 Z1 + 17/36 Z0) W2 with Z_i = eps Z(W_i).  With the
// running generator X (8 reals per link): X <- cz * eps * Z + ca * X using
// (cz, ca) = (1/4, 0), (8/9, -17/9), (3/4, -1), then W <- exp(X) W.
// X is anti-hermitian traceless, stored as (Im X00, Im X11, Re X01, Im X01,
// Re X02, Im X02, Re X12, Im X12).
//
// Adaptive steps (see su3_wilson_flow_adaptive): the second stage also forms
// the embedded second-order result exp(2 Z1 - Z0) W0 = exp(9/4 X1 + 1/4 X0) W0
// (X0 = Z0/4, X1 = 8/9 Z1 - 17/9 X0), the third stage its distance to W3.
//
// Fused multiply-adds are allowed in this unit (the pragma precedes the
// headers so that their inline arithmetic is contracted too): the flow
// smooths rather than amplifies rounding, and contraction saves 6 % of the
// fp32 stage's instructions.
#pragma clang fp contract(fast)
#include "flow_stage.hpp"
#include "kernels.hpp"
#include "pair_walk.hpp"

namespace msmc {

__device__ __forceinline__ double block_max_512(double v)
{
    __shared__ double sh[8];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        v = fmax(fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3])), fmax(fmax(sh[4], sh[5]), fmax(sh[6], sh[7])));
    return v;
}

// fp32: the pair walk (PairWalk), 512 threads per block.  mode 2 stores the
// block maximum of the distance into partials[2p] and 0 into partials[2p + 1]
// for pair block p (the two link-walk blocks it covers).
template <int NC>
__global__ void __launch_bounds__(512, 4) k_flow_stage_pair(Grid gr, double eps, double cz, double ca, int first,
                                                            int mode, double* __restrict__ partials)
{
    __shared__ PairLds lds;
    __shared__ PairQLds qlds;
    const PairWalk<NC> pw = pair_walk<NC>(gr, lds);
    const PairLd<NC> ld = pw.loader(lds);
    const M3<float> A = pair_staple<NC>(pw, ld, qlds);
    double dist = 0.0;
    if (pw.valid) {
        dist = flow_stage_link<float, NC>(*pw.d, pw.mu, pw.par, pw.cb, ld.from_lds(pw.own), A, eps, cz, ca, first,
                                          mode);
    }
    if (mode == 2) {
        dist = block_max_512(dist);
        if (threadIdx.x == 0) {
            partials[2 * pw.pb] = dist;
            partials[2 * pw.pb + 1] = 0.0;
        }
    }
}

// Largest of a lattice's block partials (one block per lattice).
__global__ void __launch_bounds__(256) k_reduce_max(const int* __restrict__ bbeg, const double* __restrict__ partials,
                                                    double* __restrict__ out)
{
    const int l = blockIdx.x;
    double v = 0.0;
    for (int k = bbeg[l] + (int)threadIdx.x; k < bbeg[l + 1]; k += 256) v = fmax(v, partials[k]);
    v = block_max_256(v);
    if (threadIdx.x == 0) out[l] = v;
}

hipError_t launch_reduce_max(const Grid& gr, const double* partials, double* out, hipStream_t st)
{
    if (gr.nlat <= 0) return hipSuccess;
    k_reduce_max<<<gr.nlat, 256, 0, st>>>(gr.bbeg, partials, out);
    return hipGetLastError();
}

hipError_t launch_flow_stage(int prec, const Grid& gr, double eps, double cz, double ca, int first, int mode,
                             double* partials, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    switch (prec) {
    case PREC_F64:
        return launch_flow_stage_f64(gr, eps, cz, ca, first, mode, partials, st);
    case PREC_F32:
        k_flow_stage_pair<18><<<gr.nblocks / 2, 512, 0, st>>>(gr, eps, cz, ca, first, mode, partials);
        break;
    case PREC_F32_R12:
        k_flow_stage_pair<12><<<gr.nblocks / 2, 512, 0, st>>>(gr, eps, cz, ca, first, mode, partials);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace msmc
