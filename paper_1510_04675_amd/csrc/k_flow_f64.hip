// k_flow_f64.hip -- the fp64 stage of the third-order Runge-Kutta Wilson
// flow (Sec. IV.B).
//
// Fused multiply-adds are allowed in this unit, the pragma coming before the
// headers so that their inline arithmetic is contracted here too: the flow
// smooths the field rather than amplifying rounding, so contraction (a fifth
// fewer fp64 instructions, 3.13 -> 2.81 ms per 32^4 step) leaves the links
// within 1e-15 of the oracle's per step.
#pragma clang fp contract(fast)
#include "flow_stage.hpp"
#include "pair_walk.hpp"

namespace msmc {

// One link per thread in the link walk of four directions of 64 sites, the
// forward staple products shared within a site (walk_staple_f64);
// mode 2 stores the block maxima of the distance into partials[logical
// block] (0 for the padding threads).  Held at 3 wavefronts per SIMD (168
// VGPRs): at 170 the compiler would leave it 2.
template <typename R, int NC>
__global__ void __launch_bounds__(256, 3) k_flow_stage(Grid gr, double eps, double cz, double ca, int first, int mode,
                                                    double* __restrict__ partials)
{
    __shared__ WalkQLds qlds;
    const LinkWalk lw = link_walk(gr);
    const LatDesc& d = gr.descs[lw.l];
    const Links<R, NC> W{ (uintptr_t)d.U, d.cs };
    const M3<R> A = walk_staple_f64<NC>(lw, W, d.g, qlds);
    double dist = 0.0;
    if (lw.valid) {
        const M3<R> w = load_link<R, NC>(W.slab(lw.mu, lw.par), lw.cb);
        dist = flow_stage_link<R, NC>(d, lw.mu, lw.par, lw.cb, w, A, eps, cz, ca, first, mode);
    }
    if (mode == 2) {
        dist = block_max_256(dist);
        if (threadIdx.x == 0) partials[logical_block(blockIdx.x, gr.nblocks, gr.remap)] = dist;
    }
}

hipError_t launch_flow_stage_f64(const Grid& gr, double eps, double cz, double ca, int first, int mode,
                                 double* partials, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    k_flow_stage<double, 18><<<gr.nblocks, 256, 0, st>>>(gr, eps, cz, ca, first, mode, partials);
    return hipGetLastError();
}

}  // namespace msmc
