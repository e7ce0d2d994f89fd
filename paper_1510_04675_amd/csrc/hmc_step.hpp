// hmc_step.hpp -- the per-link leapfrog step of the HMC (Sec. IV.E, App. A),
// shared by the fp32 kernels (k_hmc.hip) and the fp64 kernel (k_hmc_f64.hip).
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace msmc {

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
    // The kick is formed in fp64 with the step as given and rounded once, and
    // so is the drift's generator eps P below.  In fp32 the step itself rounds
    // (1/40 to 1/40 (1 + 1.5e-8)), and a kick that far from the drift's step
    // unbalances the second-order terms the leapfrog cancels between them
    // (about 1e4 per step at 32^4): dH then shifted systematically against
    // fp64 from the same start, -0.010 +- 0.001 per 32^4 trajectory of 40
    // steps (+0.041 with a fused multiply-add), against -0.002 +- 0.001 now.
#pragma unroll
    for (int a = 0; a < 8; a++) p[a] = (R)((double)p[a] - eps_kick * (double)F[a]);
    store_reals<R, 8>(pslab, cb, p);
    if (drift) {
        double pd[8];
#pragma unroll
        for (int a = 0; a < 8; a++) pd[a] = (double)p[a];
        const M3<R> E = m_exp_ah<R, ExpOrder<R>::N, 2>(m_cast<double, R>(i_eps_P(pd, eps_drift)));
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

// fp64 kick-drift launch (k_hmc_f64.hip): one link per thread in the link
// walk (bbeg counts 2 ceil(Vh / 64) blocks of 256 per lattice).
hipError_t launch_kick_drift_f64(const Grid& gr, double eps_kick, double eps_drift, int drift, hipStream_t st);

}  // namespace msmc
