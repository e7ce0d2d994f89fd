// k_phase_f64.hip -- fp64 instantiations of the checkerboard phase kernel.
// Compiled without floating-point contraction: every operation of the fp64
// chain is a separately rounded IEEE-754 operation in a fixed order.
#include "phase.hpp"

namespace msmc {

hipError_t launch_phase_f64(int kind, const Grid& gr, int mu, int par, const uint64_t* sweep_base, int sweep_off,
                            HbArgs hb, unsigned long long* exhausted, hipStream_t st)
{
    // fp64 stores need no re-orthonormalization: the store bit is dropped
    switch (kind & (PH_OR | PH_PLAQ)) {
    case 0: return launch_phase_t<double, 18, 0>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
    case PH_OR: return launch_phase_t<double, 18, PH_OR>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
    case PH_OR | PH_PLAQ:
        return launch_phase_t<double, 18, PH_OR | PH_PLAQ>(gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace msmc
