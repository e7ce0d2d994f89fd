// k_phase_f32.hip -- fp32 instantiations (full 18-real and 12-real link
// records) of the checkerboard phase kernel, compiled with fused
// multiply-add contraction.
#include "phase.hpp"

namespace msmc {

hipError_t launch_phase_f32(int prec, int kind, const Grid& gr, int mu, int par, const uint64_t* sweep_base,
                            int sweep_off, HbArgs hb, unsigned long long* exhausted, hipStream_t st)
{
    if (prec == PREC_F32) {
        if (kind == 0) return launch_phase_t<float, 18, 0>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
        if (kind == 2) return launch_phase_t<float, 18, 2>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
        return launch_phase_t<float, 18, 1>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
    }
    if (kind == 0) return launch_phase_t<float, 12, 0>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
    if (kind == 2) return launch_phase_t<float, 12, 2>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
    return launch_phase_t<float, 12, 1>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
}

}  // namespace msmc
