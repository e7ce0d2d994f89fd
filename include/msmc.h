/*
 * msmc.h -- C ABI of the MI355X (gfx950) library for the rethermalization
 * path of the multiscale thermalization method for pure SU(3) Yang-Mills
 * theory (Endres, Brower, Detmold, Orginos, Pochinsky, arXiv:1510.04675).
 *
 * The calls follow the paper's four-step procedure (Sec. I): coarse
 * configurations come from init + sweeps on a coarse field, refinement is
 * su3_prolongate, rethermalization / evolution is su3_sweep_hb_or,
 * su3_batch_sweep_hb_or or su3_hmc_trajectory on fine fields, measurement is
 * su3_plaquette, su3_action, su3_wilson_flow and su3_topological_charge.
 *
 * Conventions
 *  - Every call returns an int32 status (SU3_OK = 0) and never throws.  On
 *    an error the reason is available from su3_last_error() (thread-local)
 *    and, for validation errors, no device work was enqueued and the field
 *    is unchanged.
 *  - A field is an opaque handle to one periodic L0 x L1 x L2 x L3 lattice of
 *    SU(3) links U_mu(n), mu = 0..3.  Every extent must be even and >= 2
 *    (SU3_ERR_SHAPE otherwise), and the volume at most 2^28 sites.
 *  - Device memory: su3_field_create allocates and owns it; su3_field_wrap
 *    borrows caller memory (e.g. a torch tensor's storage) that must stay
 *    valid until su3_field_destroy, which never frees borrowed memory.  The
 *    library also allocates per-field scratch (momenta, ping-pong buffers,
 *    reduction partials) on first use and frees it in su3_field_destroy.
 *  - Streams: all work of a field is enqueued on the HIP stream given at
 *    create/wrap time (NULL = the default stream) or by su3_field_set_stream.
 *    Calls that return host values synchronize that stream before returning.
 *  - Random numbers are counter based (Philox4x32-10): key = (seed,
 *    lattice_id), counter = (lexicographic site, purpose/direction/subgroup/
 *    hit/draw word, 64-bit sweep or trajectory index), so results do not
 *    depend on launch shapes, batching or how a run is split into calls.
 *  - Handles are not thread-safe; distinct handles may be used concurrently
 *    on distinct streams.
 *
 * Host exchange layout: double[V][4][3][3][2] with site index
 * i = n0 + L0*(n1 + L1*(n2 + L2*n3)) (n0 fastest), direction mu, row-major
 * 3x3 matrix, (re, im).
 */
#ifndef MSMC_H
#define MSMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum su3_status {
    SU3_OK = 0,
    SU3_ERR_ARG = 1,         /* invalid argument (NULL pointer, bad enum, bad count) */
    SU3_ERR_SHAPE = 2,       /* odd or too small extent, coarse/fine mismatch, mixed shapes */
    SU3_ERR_NOMEM = 3,       /* device allocation failed */
    SU3_ERR_HIP = 4,         /* a HIP runtime call failed */
    SU3_ERR_NUMERIC = 5,     /* a link is not in SU(3) within tolerance, or NaN */
    SU3_ERR_UNSUPPORTED = 6  /* valid request the library does not implement */
};

/* Link storage precision.  SU3_FP32_R12 stores rows 0 and 1 only and
 * rebuilds row 2 = conj(row0 x row1) on every load. */
enum su3_prec { SU3_FP64 = 0, SU3_FP32 = 1, SU3_FP32_R12 = 2 };

/* SU(2) subgroup sampler of the heat bath. */
enum su3_sampler { SU3_SAMPLER_KP = 0, SU3_SAMPLER_CREUTZ = 1 };

typedef struct su3_field_s* su3_field;

/* Heat-bath / overrelaxation schedule (Sec. IV.A).
 *  n_or          overrelaxation passes after each heat-bath pass (paper: 10)
 *  n_hb_hits     heat-bath hits per SU(2) subgroup per link (default 1)
 *  hb_max_tries  rejection trials per draw; if all fail the subgroup is left
 *                unchanged (the paper's "attempted updates"), 1..4096
 *  reunit_every  fp64 fields: reunitarize after every sweep s with
 *                (s+1) % reunit_every == 0 (0 = never).  fp32 and 12-real
 *                fields leave every sweep re-orthonormalized in fp64 (the
 *                stores of its last pass), which subsumes it
 *  sampler       SU3_SAMPLER_KP or SU3_SAMPLER_CREUTZ */
typedef struct {
    int32_t n_or;
    int32_t n_hb_hits;
    int32_t hb_max_tries;
    int32_t reunit_every;
    int32_t sampler;
} su3_hb_params;

/* Bytes of device memory a field of these dimensions and precision needs. */
int32_t su3_field_bytes(const int32_t dims[4], int32_t prec, size_t* out);

/* Create a field that owns its device memory (contents undefined). */
int32_t su3_field_create(const int32_t dims[4], int32_t prec, void* hip_stream, su3_field* out);

/* Wrap caller-owned device memory of at least su3_field_bytes() bytes,
 * 256-byte aligned.  The memory is borrowed, never freed by the library. */
int32_t su3_field_wrap(const int32_t dims[4], int32_t prec, void* dev_ptr, size_t bytes, void* hip_stream,
                       su3_field* out);

/* Release the handle, owned memory and scratch.  NULL is accepted. */
int32_t su3_field_destroy(su3_field f);

int32_t su3_field_set_stream(su3_field f, void* hip_stream);

/* dims[4], precision and byte size of a field. */
int32_t su3_field_info(su3_field f, int32_t dims[4], int32_t* prec, size_t* bytes);

/* The two starts of the thermalization studies (Sec. IV.F: an ordered,
 * delta-function start and a random one).  Cold start: every link = 1.  Hot
 * start: every link Haar-random from Philox purpose INIT (rows 0,1 complex
 * Gaussians, Gram-Schmidt, row 2 the SU(3) completion), computed in fp64 and
 * rounded to the storage precision.  Errors: SU3_ERR_ARG for a NULL handle,
 * SU3_ERR_HIP if a launch fails. */
int32_t su3_init_cold(su3_field f);
int32_t su3_init_hot(su3_field f, uint32_t seed, uint32_t lattice_id);

/* Copy to / from the host exchange layout (V*4*18 doubles).  from_host
 * rounds to the storage precision; R12 fields keep rows 0 and 1. */
int32_t su3_field_to_host(su3_field f, double* out);
int32_t su3_field_from_host(su3_field f, const double* in);

/* dst <- src for fields of equal dims, converting the precision. */
int32_t su3_field_copy(su3_field dst, su3_field src);

/* Restriction (Sec. III): U^c_mu(n/2) = U^f_mu(n) U^f_mu(n+e_mu) for fine
 * sites with all coordinates even.  fine dims must be 2 x coarse dims. */
int32_t su3_restrict(su3_field fine, su3_field coarse);

/* Prolongation (Sec. III): transfer U^f_mu(n) = U^c_mu(n/2), U^f_mu(n+e_mu)
 * = 1 for even n, all other bonds 1; then for d = 0, 1, 2 APE steps with
 * coefficient c on the bonds with chi_mu(n) = d+1 (all at once), repeated
 * until the partial action S_d changes by at most rel_tol relative to the
 * previous step, or max_iter steps.  The interpolation runs in fp64; the
 * result is rounded into fine's precision.  Paper values: c = 0.05,
 * rel_tol = 1e-5 (Sec. IV.C).  iters_out (3 ints, may be NULL) receives
 * the steps taken per stage.  The call allocates and frees two fp64 copies of
 * the fine field and block sums (8 bytes per 256 bonds), applies the rule on
 * the device (steps past the stopping point of a run of 16 do nothing) and
 * returns after the result is in fine.  c > 0, rel_tol >= 0 and
 * max_iter >= 0 (0: transfer only) or SU3_ERR_ARG; SU3_ERR_NOMEM if the
 * copies do not fit. */
int32_t su3_prolongate(su3_field coarse, su3_field fine, double c, double rel_tol, int32_t max_iter,
                       int32_t iters_out[3]);

/* n_sweeps sweeps s = first_sweep, ..., each one heat-bath pass then p->n_or
 * overrelaxation passes; each pass runs mu = 0..3, even sites then odd sites
 * (Sec. IV.A).  Wilson action at coupling beta.  plaq_hist (n_sweeps
 * doubles, may be NULL) receives the average plaquette after each sweep
 * (after reunitarization when that sweep reunitarizes).  p = NULL uses
 * {n_or 4, n_hb_hits 1, hb_max_tries 64, reunit_every 10, KP}; on fp64
 * fields, whose links stay in SU(3) to rounding, pass reunit_every = 0 to
 * follow the paper's schedule exactly.  The count of exhausted draws is
 * kept per field (su3_last_exhausted).  At beta = 0 the draw's weight
 * exp(alpha g0) has alpha = 0, where neither sampler proposes an acceptable
 * g0: every heat-bath draw is exhausted and leaves its link unchanged (the
 * beta = 0 ensemble is the Haar measure of su3_init_hot); overrelaxation does
 * not depend on beta. */
int32_t su3_sweep_hb_or(su3_field f, double beta, uint32_t seed, uint32_t lattice_id, uint64_t first_sweep,
                        int32_t n_sweeps, const su3_hb_params* p, double* plaq_hist);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sweeps
 * of su3_sweep_hb_or, same arguments and update kernels, bitwise the same
 * links and exhausted-draw counts, with no allocation of any kind.  Its
 * plaquette history comes from the standalone plaquette kernel rather than
 * from the last overrelaxation pass, so it agrees with su3_sweep_hb_or's to
 * rounding (1e-13 in fp64, 1e-7 in fp32).  The tables, counters, plaquette
 * partials and history it needs live in a fixed device array of 557,824
 * bytes that each GPU the library runs on holds until the process ends;
 * the field itself is the caller's (su3_field_wrap allocates nothing).
 * Limits: at most 2^24 sites (SU3_ERR_UNSUPPORTED beyond) and at most 4096
 * sweeps per call when plaq_hist is given (SU3_ERR_ARG beyond).  It uses the
 * default launch shape or the one forced by su3_set_launch / su3_set_tile,
 * never runs the autotuner and is not timed by su3_profile_enable.  Every
 * call on one GPU shares that GPU's array: calls that overlap in time on one
 * GPU (other threads, other streams) race and must be serialized by the
 * caller.  Like su3_sweep_hb_or it synchronizes the field's stream before
 * returning. */
int32_t su3_sweep_hb_or_noalloc(su3_field f, double beta, uint32_t seed, uint32_t lattice_id, uint64_t first_sweep,
                                int32_t n_sweeps, const su3_hb_params* p, double* plaq_hist);

/* Parallel rethermalization of many prolongated lattices (Sec. II, the
 * strategy in which refined configurations are rethermalized independently,
 * which the paper notes is embarrassingly parallel): the schedule of
 * su3_sweep_hb_or on n independent lattices of equal precision (any shapes)
 * in one batched launch per phase, recorded once into a HIP graph and
 * replayed.  Per lattice: fs[i], betas[i], seeds[i], lattice_ids[i].
 * Results are bitwise equal to n separate su3_sweep_hb_or calls, the
 * exhausted-draw count of each field included.  plaq_out (n_sweeps * n
 * doubles, [sweep][lattice], may be NULL).  The fields must share one
 * stream and appear once each (SU3_ERR_ARG), and share one precision
 * (SU3_ERR_UNSUPPORTED). */
int32_t su3_batch_sweep_hb_or(const su3_field* fs, int32_t n, const double* betas, const uint32_t* seeds,
                              const uint32_t* lattice_ids, uint64_t first_sweep, int32_t n_sweeps,
                              const su3_hb_params* p, double* plaq_out);

/* One HMC trajectory (Sec. IV.E, App. A): momenta p^a ~ N(0,1) from Philox
 * purpose MOM with the 64-bit trajectory index traj; H = (1/2) sum p^2 + S in
 * fp64; kick-drift-kick leapfrog with eps = tau / n_steps, U <- exp(i eps P)
 * U, in the storage precision; Metropolis with the uniform of Philox purpose
 * ACCEPT (site word 0) against exp(-dH).  metropolis = 0 accepts always
 * (warm-up trajectories).  On rejection the field is unchanged.  12-real
 * links are re-orthonormalized (in fp64, rounded once) at every drift store;
 * 18-real fp32 links are not, so their distance from SU(3) grows slowly over
 * many trajectories: long runs call su3_reunitarize between trajectories. */
int32_t su3_hmc_trajectory(su3_field f, double beta, double tau, int32_t n_steps, uint32_t seed,
                           uint32_t lattice_id, uint64_t traj, int32_t metropolis, double* dH, int32_t* accepted);

/* Sec. III, the Wilson action and the 1 x 1 Wilson loops W_munu(n):
 * su3_plaquette gives the average plaquette
 * (1/(6V)) sum_n sum_{mu<nu} (1/3) Re Tr U_munu(n), su3_action the Wilson
 * action beta sum_n sum_{mu<nu} [1 - (1/3) Re Tr U_munu(n)].  Both are
 * summed in fp64 in a fixed order (the same bits for any launch shape). */
int32_t su3_plaquette(su3_field f, double* out);
int32_t su3_action(su3_field f, double beta, double* out);

/* n_steps fixed steps eps of the third-order Runge-Kutta Wilson flow, in
 * place, in the storage precision (Sec. IV.B). */
int32_t su3_wilson_flow(su3_field f, double eps, int32_t n_steps);

/* Adaptive-step Wilson flow (Sec. IV.B: the adaptive integrator with a
 * tolerance and a maximum step; the paper's runs use tol = 0.01,
 * max_step = 0.2).  Each step of size h is the RK3 step of su3_wilson_flow;
 * its error estimate is d = max over links and matrix elements of
 * |W3 - W~|, W~ = exp(2 Z1 - Z0) W0 the embedded second-order result.
 * d <= tol accepts the step, otherwise the field returns to W0; the next
 * size is min(max_step, 0.95 h (tol/d)^(1/3)), starting from eps0.  Steps
 * are shortened to land exactly on each of the n_meas ascending times
 * t_meas[k] in [0, t_end], where E_out[k] (clover energy density,
 * su3_clover_energy) and Q_out[k] (clover charge) are recorded.  The field
 * is flowed in place to t_end.  n_accepted / n_rejected (may be NULL)
 * receive the step counts.  SU3_ERR_NUMERIC if the step size collapses.
 * Allocates three link-sized scratch fields on first use. */
int32_t su3_wilson_flow_adaptive(su3_field f, double t_end, double tol, double max_step, double eps0,
                                 const double* t_meas, int32_t n_meas, double* E_out, double* Q_out,
                                 int32_t* n_accepted, int32_t* n_rejected);

/* Flow scale (Sec. IV.B): the t where t^2 E(t) crosses `target` (0.3 for
 * t0), linearly interpolated between the two bracketing points of the host
 * arrays t[0..n), E[0..n).  SU3_ERR_NUMERIC if no pair brackets it. */
int32_t su3_flow_t0(const double* t, const double* E, int32_t n, double target, double* t0);

/* Admissibility measure (Sec. IV.D): h = max over plaquettes of
 * s_p = 3 [1 - (1/3) Re Tr U_p]; fields with h < 0.067 fall into distinct
 * topological sectors. */
int32_t su3_max_plaquette_action(su3_field f, double* h);

/* Topological charge of the current field (Sec. IV.D).  The paper measures
 * it with a three-loop improved gluonic operator whose coefficients it does
 * not give; this library uses the clover definition: F_munu = traceless
 * part of (Q_munu - Q_munu^+)/8 with Q_munu the four-leaf clover,
 * q(x) = -(1/(2 pi^2)) Re Tr[F01 F23 - F02 F13 + F03 F12] (epsilon_0123 =
 * +1), Q = sum_x q(x), in fp64.  Like it, Q approaches integers along the
 * Wilson flow. */
int32_t su3_topological_charge(su3_field f, double* Q);
/* Clover energy density (Sec. IV.B, the E(t) that defines the flow scale
 * t0): (1/V) sum_x sum_{mu<nu} -Re Tr(F_munu F_munu) with the F_munu of
 * su3_topological_charge, fp64. */
int32_t su3_clover_energy(su3_field f, double* E);

/* Wilson loops (Sec. III, the m x n loop, its plane/site average and the
 * partial averages).  W_munu^{m x n}(n) = (1/3) Re Tr L_mu^m(n)
 * L_nu^n(n + m e_mu) L_mu^m(n + n e_nu)^+ L_nu^n(n)^+ with L_mu^m the product
 * of m links along mu, for mu < nu (m steps along the lower direction).
 *   su3_wilson_loop: the average over all sites and the 6 planes,
 *     1 <= m, n <= 1024 (su3_wilson_loop(f, 1, 1) is the plaquette);
 *   su3_partial_plaquettes: out[d], d = 0, 1, 2, the average of the 1 x 1
 *     loops with chi_munu(n) = d, chi_munu counting the odd coordinates of n
 *     other than n_mu, n_nu (the partial average of Sec. III);
 *   su3_displaced_loops: out[d], d = 0..4, the average of the 2 x 2 loops
 *     from sites with chi(n) = d odd coordinates (after prolongation out[0]
 *     equals the coarse plaquette).
 * Computed in fp64 from the stored links, summed in a fixed order. */
int32_t su3_wilson_loop(su3_field f, int32_t m, int32_t n, double* out);
int32_t su3_partial_plaquettes(su3_field f, double out[3]);
int32_t su3_displaced_loops(su3_field f, double out[5]);

/* Reunitarize every link (Gram-Schmidt of rows 0,1 in fp64).  Not a step of
 * the paper, whose precision is unstated: it returns reduced-precision links
 * to SU(3) (the sweeps do it for fp64 fields every reunit_every sweeps, and
 * for fp32 fields at the end of every sweep). */
int32_t su3_reunitarize(su3_field f);

/* Random gauge transformation U_mu(n) -> Om(n) U_mu(n) Om(n+mu)^+ with Om
 * Haar-random per site from Philox purpose GAUGE, key (seed, 0): the gauge
 * freedom of the action (Sec. III), used to check that measurements are
 * gauge invariant. */
int32_t su3_gauge_transform(su3_field f, uint32_t seed);

/* Largest deviation of any link from SU(3) (the largest entry modulus of
 * U U^+ - 1, or |det U - 1|, NaN counting as infinite) and the index of that
 * link, (2*mu + parity) * (V/2) + (lexicographic site >> 1).  Returns
 * SU3_ERR_NUMERIC when the deviation exceeds tol (outputs still written). */
int32_t su3_check_field(su3_field f, double tol, double* max_dev, int64_t* worst);

/* Heat-bath draws left unchanged because every trial was rejected (the
 * paper's cap on attempted updates, Sec. IV.A), summed over the last
 * su3_sweep_hb_or, su3_sweep_hb_or_noalloc or su3_batch_sweep_hb_or call
 * that named f: after a batch each field holds its own lattice's count, and
 * after a call of no sweeps the count is 0. */
int32_t su3_last_exhausted(su3_field f, int64_t* count);

/* Launch shape of the checkerboard phase kernels: block in {64, 128, 256,
 * 512}, xcd_remap in {0, 1}; block = 0 restores automatic choice.
 * Results do not depend on it.  su3_autotune(1) makes the next sweep call
 * time the candidates (3 blocks x 2 remaps x 7 tiles) on cold-start scratch
 * fields of the same shapes, swept at that call's couplings and options, and
 * keep the fastest for those shapes; the default (256, remap, tile 8 x 8 x 8) is kept unless
 * another shape is faster by more than 1.5 %.  The scratch fields are
 * allocated and freed inside that call. */
int32_t su3_set_launch(int32_t block, int32_t xcd_remap);
int32_t su3_autotune(int32_t enable);
int32_t su3_get_launch(int32_t* block, int32_t* xcd_remap);

/* Batched sweeps run lattice groups one after another, each group's
 * links at most `bytes` (a larger lattice forms a group alone), all passes
 * of a sweep per group, so that a group stays in the last-level cache
 * (256 MB on MI355X) between phases.  0 sweeps the whole batch phase by
 * phase.  Default 224 MiB.  Results do not depend on it. */
int32_t su3_set_group_bytes(uint64_t bytes);

/* Site tile of the checkerboard phase kernels: threads walk each lattice in
 * tiles of L0 x ty x tz x tt sites (each extent clamped to the largest
 * divisor of L1, L2, L3 not above it; 0 = whole extent).  (0, 0, 0) restores
 * the automatic choice (autotuned, else 8 x 8 x 8).  Results do not depend
 * on it; it sets which neighbour links are loaded together into one L2. */
int32_t su3_set_tile(int32_t ty, int32_t tz, int32_t tt);

/* The launch shape the next sweep on these n fields would use:
 * out = {block, xcd_remap, ty, tz, tt} (tile before clamping). */
int32_t su3_get_config(const su3_field* fs, int32_t n, int32_t out[5]);

/* Kernel timing with HIP events recorded on the field's stream around each
 * run of consecutive launches of one kind (the 8 heat-bath phases of a
 * lattice group, its 8 n_or overrelaxation phases, the plaquette kernel);
 * su3_profile_read returns the summed time and the number of launches.
 * While enabled, su3_batch_sweep_hb_or launches the same kernels eagerly
 * instead of replaying its graph.  kind 0 = heat-bath phases,
 * 1 = overrelaxation phases, 2 = the per-sweep plaquette kernel.  Enabling
 * resets the accumulators. */
int32_t su3_profile_enable(int32_t enable);
int32_t su3_profile_read(int32_t kind, double* total_ms, int64_t* launches);

/* Message of the last failed call on this thread ("" if none). */
const char* su3_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MSMC_H */
