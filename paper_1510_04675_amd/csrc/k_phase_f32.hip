// k_phase_f32.hip -- fp32 instantiations (full 18-real and 12-real link
// records) of the checkerboard phase kernel, compiled with fused
// multiply-add contraction.
#include "phase.hpp"

namespace msmc {

hipError_t launch_phase_f32(int prec, int kind, const Grid& gr, int mu, int par, const uint64_t* sweep_base,
                            int sweep_off, HbArgs hb, unsigned long long* exhausted, hipStream_t st)
{
#define PHASE_F32(NC)                                                                                          \
    switch (kind) {                                                                                            \
    case 0: return launch_phase_t<float, NC, 0>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);        \
    case PH_STORE64:                                                                                           \
        return launch_phase_t<float, NC, PH_STORE64>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);   \
    case PH_OR: return launch_phase_t<float, NC, PH_OR>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st); \
    case PH_OR | PH_STORE64:                                                                                   \
        return launch_phase_t<float, NC, PH_OR | PH_STORE64>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, \
                                                              st);                                              \
    case PH_OR | PH_PLAQ | PH_STORE64:                                                                         \
        return launch_phase_t<float, NC, PH_OR | PH_PLAQ | PH_STORE64>(gr, mu, par, sweep_base, sweep_off, hb,  \
                                                                        exhausted, st);                         \
    default: return hipErrorInvalidValue;                                                                      \
    }
    if (prec == PREC_F32) PHASE_F32(18)
    PHASE_F32(12)
#undef PHASE_F32
}

}  // namespace msmc
