// kernels.hpp -- host-visible launch interface of the HIP kernels.  The
// C-ABI layer (capi.cpp) builds descriptor tables and calls these launchers;
// each launcher dispatches on the storage precision to a kernel template.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device.hpp"

namespace msmc {

enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_F32_R12 = 2 };

inline int prec_ncomp(int p) { return p == PREC_F32_R12 ? 12 : 18; }
inline size_t prec_real_bytes(int p) { return p == PREC_F64 ? 8 : 4; }

// Per-lattice descriptor read by the batched kernels.
struct LatDesc {
    void* U;       // link field
    void* aux;     // second buffer (momenta, flow generator, ping-pong links)
    void* aux2;
    void* aux3;    // adaptive flow: embedded second-order links W~
    void* aux4;    // adaptive flow: links at the start of the step W0
    size_t cs;     // bytes per slab of U, aux2, aux3, aux4 (link records)
    size_t cs8;    // bytes per slab of aux (8-real records)
    Geo g;
    double beta;
    uint32_t seed, lid;
    int tile[3];   // (ty, tz, tt): site tile of the phase kernels (divisors of L1, L2, L3)
    int mtile[3];  // (ty, tz, tt): site tile of the measurement kernels, fixed by the extents
    double* psite; // plaquette site values of the last overrelaxation pass (3 x Vh), or NULL
};

// Block partition: lattice l owns logical blocks [bbeg[l], bbeg[l+1]).
// All launchers take (descs, bbeg, nlat, nblocks) and a block size.
struct Grid {
    const LatDesc* descs;
    const int* bbeg;
    int nlat;
    int nblocks;
    int block;
    int remap;
};

// Thread -> link for the kernels that update all 4V links at once and read
// neighbour links (HMC kick-drift, flow stage).  Blocks of 256 threads: the
// four wavefronts of a block take directions mu = 0..3 of the same 64 sites of
// one parity, consecutive blocks alternate parity, and the sites follow the
// tiled checkerboard order of the phase kernels, so the links a staple reads
// were loaded by nearby threads.  bbeg counts 2 ceil(Vh / 64) blocks per
// lattice.
struct LinkWalk {
    int l, mu, par, cb, n[4];
    bool valid;
};

__device__ __forceinline__ LinkWalk link_walk(const Grid& gr)
{
    LinkWalk x;
    const int lb = logical_block(blockIdx.x, gr.nblocks, gr.remap);
    int lo = 0, hi = gr.nlat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (gr.bbeg[mid] <= lb)
            lo = mid;
        else
            hi = mid - 1;
    }
    x.l = lo;
    const LatDesc& d = gr.descs[x.l];
    const int b = lb - gr.bbeg[x.l];
    x.par = b & 1;
    x.mu = (int)threadIdx.x >> 6;
    const int w = (b >> 1) * 64 + ((int)threadIdx.x & 63);
    x.valid = w < d.g.Vh;
    x.cb = 0;
    if (x.valid) {
        tiled_coords(d.g, d.tile, w, x.par, x.n);
        x.cb = lex_index(d.g, x.n) >> 1;
    }
    return x;
}

struct HbArgs {
    int n_hits;
    int max_tries;
    int sampler;  // 0 = Kennedy-Pendleton, 1 = Creutz
};

// --- update kernels (k_update.hip) -----------------------------------------
// One checkerboard phase (mu, parity).  kind is a set of bits (phase.hpp):
// 1 overrelaxation (else heat bath); 2 also write, for the odd-parity phases
// mu = 1, 2, 3 of a sweep's last pass, each site's share of the plaquette sum
// into psite (see k_phase); 4 re-orthonormalize fp32 stores in fp64 (a
// sweep's last pass).  Work unit: one link of that direction and parity per
// thread, bbeg counts ceil(Vh / block) blocks per lattice.
hipError_t launch_phase(int prec, int kind, const Grid& gr, int mu, int par, const uint64_t* sweep_base,
                        int sweep_off, HbArgs hb, unsigned long long* exhausted, hipStream_t st);
hipError_t launch_phase_f64(int kind, const Grid& gr, int mu, int par, const uint64_t* sweep_base, int sweep_off,
                            HbArgs hb, unsigned long long* exhausted, hipStream_t st);
hipError_t launch_phase_f32(int prec, int kind, const Grid& gr, int mu, int par, const uint64_t* sweep_base,
                            int sweep_off, HbArgs hb, unsigned long long* exhausted, hipStream_t st);

// Per-link kernels: bbeg counts ceil(8*Vh / 256) blocks per lattice.
hipError_t launch_init(int prec, int hot, const Grid& gr, hipStream_t st);
hipError_t launch_reunit(int prec, const Grid& gr, const uint64_t* sweep_base, int sweep_off, int every,
                         hipStream_t st);
hipError_t launch_gauge(int prec, const Grid& gr, uint32_t seed, hipStream_t st);
// host exchange layout <-> structure of arrays (one lattice, staging in fp64)
hipError_t launch_to_aos(int prec, const LatDesc* d, const Geo& g, const void* U, size_t cs, double* aos,
                         hipStream_t st);
hipError_t launch_from_aos(int prec, const Geo& g, void* U, size_t cs, const double* aos, hipStream_t st);
// copy with precision conversion between two fields of the same shape
hipError_t launch_convert(int pdst, void* dst, size_t cs_dst, int psrc, const void* src, size_t cs_src, int Vh,
                          hipStream_t st);
// largest deviation from SU(3) per block (max of |UU^+ - 1| and |det U - 1|)
hipError_t launch_check(int prec, const Geo& g, const void* U, size_t cs, double* block_max, int* block_arg,
                        int nblk, hipStream_t st);

// --- reductions (k_measure.hip) --------------------------------------------
// Sum over sites and planes of 1 - (1/3) Re Tr U_munu(n) in fp64.  Work unit:
// one site per thread, bbeg counts ceil(V / 256) blocks per lattice.
hipError_t launch_plaq_partial(int prec, const Grid& gr, double* partials, hipStream_t st);
// The same, done only in sweeps s = *sweep_base + sweep_off with
// (s + 1) % every == 0 (those that reunitarize); other sweeps exit at once.
hipError_t launch_plaq_partial_gated(int prec, const Grid& gr, double* partials, const uint64_t* sweep_base,
                                     int sweep_off, int every, hipStream_t st);
// Block partials of the plaquette site values psite of each lattice (3 Vh
// doubles, 1024 per block in a fixed order): bbeg counts ceil(3 Vh / 1024)
// blocks per lattice.
hipError_t launch_psite_partial(const Grid& gr, double* partials, hipStream_t st);
// out[l * stride + off] = sum of lattice l's partials from (bbeg_a, pa) if
// sweep *sweep_base + sweep_off reunitarizes (every > 0), else from
// (bbeg_b, pb).
hipError_t launch_reduce_pick(int nlat, const int* bbeg_a, const double* pa, const int* bbeg_b, const double* pb,
                              const uint64_t* sweep_base, int sweep_off, int every, double* out, int stride, int off,
                              hipStream_t st);
// out[l * stride + off] = sum of partials of lattice l (fixed order).
hipError_t launch_reduce_final(const Grid& gr, const double* partials, double* out, int stride, int off,
                               hipStream_t st);
// Clover topological charge density summed per block (fp64).
// Wilson loop sums by class (mode 0: all; 1: chi_munu, 3 classes; 2: chi,
// 5 classes); partials hold nclass x nblocks doubles.
hipError_t launch_loops_partial(int prec, const Grid& gr, int m, int n, int mode, double* partials, hipStream_t st);
// per-block maxima of s_p = 3 - Re Tr U_p (admissibility)
hipError_t launch_max_splaq_partial(int prec, const Grid& gr, double* partials, hipStream_t st);
hipError_t launch_qtop_partial(int prec, const Grid& gr, double* partials, hipStream_t st);
// Clover energy density summed per block (fp64).
hipError_t launch_energy_partial(int prec, const Grid& gr, double* partials, hipStream_t st);

// --- HMC (k_hmc.hip) ---------------------------------------------------------
// aux = momenta (8 reals per link, stride cs8), aux2 = destination links.
// Per-link work unit over all 4V links: bbeg counts ceil(8*Vh / block).
hipError_t launch_mom_refresh(int prec, const Grid& gr, uint64_t traj, hipStream_t st);
hipError_t launch_kick_drift(int prec, const Grid& gr, double eps_kick, double eps_drift, int drift,
                             hipStream_t st);
hipError_t launch_kinetic_partial(int prec, const Grid& gr, double* partials, hipStream_t st);

// --- Wilson flow (k_flow.hip) ------------------------------------------------
// aux = 2N-storage generator (8 reals per link), aux2 = destination links.
hipError_t launch_flow_stage(int prec, const Grid& gr, double eps, double cz, double ca, int first, int mode,
                             double* partials, hipStream_t st);
// out[l] = max of lattice l's block partials
hipError_t launch_reduce_max(const Grid& gr, const double* partials, double* out, hipStream_t st);

// --- restriction / prolongation (k_prolong.hip), fp64 fine field ------------
hipError_t launch_restrict(int pf, const Geo& gf, const void* Uf, size_t csf, int pc, const Geo& gc, void* Uc,
                           size_t csc, hipStream_t st);
hipError_t launch_transfer(int pc, const Geo& gc, const void* Uc, size_t csc, const Geo& gf, double* Uf,
                           size_t csf, hipStream_t st);
// One interpolation step j of stage d (Uold = iterate j-1 -> Unew = iterate j)
// plus the device-side stopping rule; state (ape_state_bytes() bytes) is
// reset at the stage start, block_sums holds ape_blocks(gf, d) doubles.
int ape_blocks(const Geo& gf, int d);
size_t ape_state_bytes();
hipError_t launch_ape_reset(void* state, hipStream_t st);
hipError_t launch_ape_step(const Geo& gf, const double* Uold, double* Unew, size_t csf, int d, double c, int j,
                           double rel_tol, int max_iter, void* state, double* block_sums, int nblk, hipStream_t st);
// waits for the stream, then reads whether the stage is done and its step count
hipError_t read_ape_state(const void* state, int* done, int* iters, hipStream_t st);

}  // namespace msmc
