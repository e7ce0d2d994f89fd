// k_hmc_f64.hip -- the fp64 leapfrog step of the HMC (Sec. IV.E, App. A).
//
// Fused multiply-adds are allowed in this unit, the pragma coming before the
// headers so that their inline arithmetic is contracted here too.  Unlike the
// heat-bath and overrelaxation chain, whose fp64 results follow the oracle's
// operation order because overrelaxation amplifies any rounding difference,
// a trajectory is not chaotic at its length: contraction cuts a fifth of the
// fp64 instructions and leaves the links within 1e-15 and dH within 1e-8 of
// the uncontracted step.
#pragma clang fp contract(fast)
#include "hmc_step.hpp"
#include "pair_walk.hpp"

namespace msmc {

// One link per thread in the link walk of four directions of 64 sites, the
// forward staple products shared within a site (walk_staple_f64), held at 3
// wavefronts per SIMD (168 VGPRs).
template <typename R, int NC>
__global__ void __launch_bounds__(256, 3) k_kick_drift(Grid gr, double eps_kick, double eps_drift, int drift)
{
    __shared__ WalkQLds qlds;
    const LinkWalk x = link_walk(gr);
    const LatDesc& d = gr.descs[x.l];
    const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
    const M3<R> A = walk_staple_f64<NC>(x, U, d.g, qlds);
    if (!x.valid) return;
    const M3<R> u = load_link<R, NC>(U.slab(x.mu, x.par), x.cb);
    kick_drift_link<R, NC>(d, x.mu, x.par, x.cb, u, A, eps_kick, eps_drift, drift);
}

hipError_t launch_kick_drift_f64(const Grid& gr, double eps_kick, double eps_drift, int drift, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    k_kick_drift<double, 18><<<gr.nblocks, 256, 0, st>>>(gr, eps_kick, eps_drift, drift);
    return hipGetLastError();
}

}  // namespace msmc
