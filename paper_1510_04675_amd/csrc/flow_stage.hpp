// flow_stage.hpp -- the per-link stage of the third-order Runge-Kutta
// Wilson flow (Sec. IV.B), shared by the fp32 kernels (k_flow.hip) and the
// fp64 kernel (k_flow_f64.hip).  Notation as in k_flow.hip.
#pragma once

#include <type_traits>

#include "kernels.hpp"

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
    const M3<R> E = m_exp_ah<R, FlowExpOrder<R>::N, 2>(ah_from8(x));
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
        M3<R> wt = m_mul(m_exp_ah<R, FlowExpOrder<R>::N, 2>(ah_from8(y)), load_link<R, NC>(W0.slab(mu, par), cb));
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

// fp64 stage launch (k_flow_f64.hip): one link per thread in the link walk
// (bbeg counts 2 ceil(Vh / 64) blocks of 256 per lattice).
hipError_t launch_flow_stage_f64(const Grid& gr, double eps, double cz, double ca, int first, int mode,
                                 double* partials, hipStream_t st);

}  // namespace msmc
