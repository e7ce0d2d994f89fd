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
#include "kernels.hpp"
#include "pair_walk.hpp"

namespace msmc {

template <typename R> struct FlowExpOrder;
template <> struct FlowExpOrder<double> { static constexpr int N = 12; };
// fp32: X is scaled to norm <= 1/4, where the order-6 remainder (< 1/4^7/7!,
// about 1.2e-8) is below fp32 rounding.
template <> struct FlowExpOrder<float> { static constexpr int N = 6; };

// X in 8-real form as a 3x3 anti-hermitian traceless matrix.
template <typename R> __device__ __forceinline__ M3<R> ah_from8(const R x[8])
{
    M3<R> X;
    X.re[0] = R(0);
    X.im[0] = x[0];
    X.re[4] = R(0);
    X.im[4] = x[1];
    X.re[8] = R(0);
    X.im[8] = -(x[0] + x[1]);
    X.re[1] = x[2];
    X.im[1] = x[3];
    X.re[3] = -x[2];
    X.im[3] = x[3];
    X.re[2] = x[4];
    X.im[2] = x[5];
    X.re[6] = -x[4];
    X.im[6] = x[5];
    X.re[5] = x[6];
    X.im[5] = x[7];
    X.re[7] = -x[6];
    X.im[7] = x[7];
    return X;
}

// One stage for the link (mu, par, cb) of lattice d, whose value is w and
// staple sum A.  mode 0: plain stage.  mode 1 (the second stage, X = X1
// built from the stored X0): also the embedded second-order result
// W~ = exp(2 Z1 - Z0) W0 = exp(9/4 X1 + 1/4 X0) W0 into aux3, W0 read from
// aux4.  mode 2 (the third stage): returns the distance max_ij |W3 - W~| of
// the link (else 0).
template <typename R, int NC>
__device__ __forceinline__ double flow_stage_link(const LatDesc& d, int mu, int par, int cb, const M3<R>& w,
                                                  const M3<R>& A, double eps, double cz, double ca, int first,
                                                  int mode)
{
    const int slab = 2 * mu + par;
    const M3<R> Om = m_mul(w, A);
    // Z in 8-real form
    const R tr3 = (Om.im[0] + Om.im[4] + Om.im[8]) / R(3);
    R z[8];
    z[0] = -Om.im[0] + tr3;
    z[1] = -Om.im[4] + tr3;
    z[2] = R(-0.5) * (Om.re[1] - Om.re[3]);
    z[3] = R(-0.5) * (Om.im[1] + Om.im[3]);
    z[4] = R(-0.5) * (Om.re[2] - Om.re[6]);
    z[5] = R(-0.5) * (Om.im[2] + Om.im[6]);
    z[6] = R(-0.5) * (Om.re[5] - Om.re[7]);
    z[7] = R(-0.5) * (Om.im[5] + Om.im[7]);
    const uintptr_t xslab = (uintptr_t)d.aux + (uintptr_t)slab * d.cs8;
    R x[8], xo[8];
    const R fz = (R)(cz * eps), fa = (R)ca;
    if (!first) load_reals<R, 8>(xslab, cb, xo);
#pragma unroll
    for (int a = 0; a < 8; a++) {
        x[a] = fz * z[a];
        if (!first) x[a] += fa * xo[a];
    }
    store_reals<R, 8>(xslab, cb, x);
    const M3<R> E = m_exp_ah<R, FlowExpOrder<R>::N, 2, true>(ah_from8(x));
    const Links<R, NC> D{ (uintptr_t)d.aux2, d.cs };
    M3<R> wn = m_mul(E, w);
    // fp32 links are re-orthonormalized (in fp64, rounded once) before the
    // store: a 12-real record rebuilds row 2 from rows 0 and 1, so their
    // rounding would feed back through every later product, and an 18-real
    // one would drift away from SU(3) step by step.
    if constexpr (std::is_same<R, float>::value) m_reunit_for_store(wn);
    store_link<R, NC>(D.slab(mu, par), cb, wn);
    double dist = 0.0;
    if (mode == 1) {
        R y[8];
#pragma unroll
        for (int a = 0; a < 8; a++) y[a] = R(2.25) * x[a] + R(0.25) * xo[a];
        const Links<R, NC> W0{ (uintptr_t)d.aux4, d.cs };
        M3<R> wt = m_mul(m_exp_ah<R, FlowExpOrder<R>::N, 2, true>(ah_from8(y)), load_link<R, NC>(W0.slab(mu, par), cb));
        if constexpr (std::is_same<R, float>::value) m_reunit_for_store(wt);
        const Links<R, NC> T{ (uintptr_t)d.aux3, d.cs };
        store_link<R, NC>(T.slab(mu, par), cb, wt);
    } else if (mode == 2) {
        const Links<R, NC> T{ (uintptr_t)d.aux3, d.cs };
        M3<R> wt = load_link<R, NC>(T.slab(mu, par), cb);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const double dr = (double)wn.re[k] - (double)wt.re[k], di = (double)wn.im[k] - (double)wt.im[k];
            dist = fmax(dist, sqrt(dr * dr + di * di));
        }
    }
    return dist;
}

// fp64: one link per thread in the link walk of four directions of 64 sites;
// mode 2 stores the block maxima of the distance into partials[logical
// block] (0 for the padding threads).  Held at 3 wavefronts per SIMD (168
// VGPRs): at 170 the compiler would leave it 2.
template <typename R, int NC>
__global__ void __launch_bounds__(256, 3) k_flow_stage(Grid gr, double eps, double cz, double ca, int first, int mode,
                                                    double* __restrict__ partials)
{
    const LinkWalk lw = link_walk(gr);
    double dist = 0.0;
    if (lw.valid) {
        const LatDesc& d = gr.descs[lw.l];
        const Links<R, NC> W{ (uintptr_t)d.U, d.cs };
        const M3<R> A = staple_sum<R, NC, R>(W, d.g, lw.mu, lw.n);
        const M3<R> w = load_link<R, NC>(W.slab(lw.mu, lw.par), lw.cb);
        dist = flow_stage_link<R, NC>(d, lw.mu, lw.par, lw.cb, w, A, eps, cz, ca, first, mode);
    }
    if (mode == 2) {
        dist = block_max_256(dist);
        if (threadIdx.x == 0) partials[logical_block(blockIdx.x, gr.nblocks, gr.remap)] = dist;
    }
}

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
    const PairWalk<NC> pw = pair_walk<NC>(gr, lds);
    double dist = 0.0;
    if (pw.valid) {
        const PairLd<NC> ld = pw.loader(lds);
        const M3<float> A = staple_sum_rows<NC, false>(ld, pw.g, pw.mu, pw.n, nullptr);
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
        k_flow_stage<double, 18><<<gr.nblocks, gr.block, 0, st>>>(gr, eps, cz, ca, first, mode, partials);
        break;
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
