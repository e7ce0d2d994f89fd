// phase.hpp -- one checkerboard phase of the Cabibbo-Marinari heat bath or of
// overrelaxation (Sec. IV.A); included by k_phase_f64.hip (fp64, compiled
// without floating-point contraction) and k_phase_f32.hip (fp32).
//
// For the link U_mu(n) the local weight is exp((beta/3) Re Tr(U A)), A the
// staple sum.  With W = U A, each SU(2) subgroup (0,1), (1,2), (0,2) in turn
// is updated by U <- R U (and W <- R W): R's 2x2 block is r = g v^+, v the
// unit SU(2) part k v of W's block, g drawn with density exp(alpha g0) on the
// SU(2) Haar measure, alpha = 2 beta k / 3 (Kennedy-Pendleton: delta = 1 - g0
// proposed from Gamma(3/2) with rate alpha and accepted with probability
// sqrt(1 - delta/2); Creutz: g0 from exp(alpha g0) on [-1, 1] by inversion,
// accepted with probability sqrt(1 - g0^2)); the direction of g is uniform on
// the sphere.  A draw whose trials all fail leaves the subgroup unchanged.
// Overrelaxation uses r = (v^+)^2, which keeps Re Tr(U A) and the action.
//
// One thread per link of direction mu and the given parity; no two links of
// one phase share a plaquette, so the phase is a single data-parallel launch.
// exhausted (may be NULL) holds one counter per lattice of the launch, indexed
// like its descriptors.
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace msmc {

__device__ __forceinline__ int find_lattice_p(const int* __restrict__ bbeg, int nlat, int lb)
{
    int lo = 0, hi = nlat - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (bbeg[mid] <= lb)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Draw g0 (trial t uses Philox word (P_HB, mu, sub, hit, t)); false if all
// max_tries trials were rejected.
template <typename R>
__device__ __forceinline__ bool draw_g0(const Rng& rng, R alpha, int mu, int sg, int h, const HbArgs& hb, R& g0)
{
    // fp64 divides by alpha exactly as the reference order does; fp32 scales
    // by the hardware reciprocal
    R ia;
    if constexpr (std::is_same<R, double>::value)
        ia = R(1) / alpha;
    else
        ia = __builtin_amdgcn_rcpf(alpha);
    for (int t = 0; t < hb.max_tries; t++) {
        const uint4 w = rng.draw(ctr_word(P_HB, mu, sg, h, t));
        const R u0 = u01<R>(w.x), u1 = u01<R>(w.y), u2 = u01<R>(w.z), u3 = u01<R>(w.w);
        if (hb.sampler == 0) {
            R cs, sn;
            m_cossin2pi(u1, &cs, &sn);
            R delta;
            if constexpr (std::is_same<R, double>::value)
                delta = -(m_log(u0) + cs * cs * m_log(u2)) / alpha;
            else
                delta = -(m_log(u0) + cs * cs * m_log(u2)) * ia;
            if (u3 * u3 <= R(1) - R(0.5) * delta) {
                g0 = R(1) - delta;
                return true;
            }
        } else {
            const R e = m_exp(R(-2) * alpha);
            R x;
            if constexpr (std::is_same<R, double>::value)
                x = R(1) + m_log(e + u0 * (R(1) - e)) / alpha;
            else
                x = R(1) + m_log(e + u0 * (R(1) - e)) * ia;
            if (u1 * u1 <= R(1) - x * x) {
                g0 = x;
                return true;
            }
        }
    }
    return false;
}

// fp32 Kennedy-Pendleton heat bath: the link-independent part of the first
// kPreTrials trials of every subgroup (hit 0) and of their directions is
// computed before the staple, while its loads are in flight.  Per trial:
// e = -(ln u0 + cos^2(2 pi u1) ln u2), so that delta = e / alpha, and u3^2;
// per direction: cos(theta), sin(theta) cos(phi), sin(theta) sin(phi).
constexpr int kPreTrials = 2;
struct KpPre {
    float e[3][kPreTrials > 0 ? kPreTrials : 1], a[3][kPreTrials > 0 ? kPreTrials : 1];
    float ct[3], sc[3], ss[3];
};

__device__ __forceinline__ void kp_trial_parts(const Rng& rng, int mu, int sg, int t, float& e, float& a)
{
    const uint4 w = rng.draw(ctr_word(P_HB, mu, sg, 0, t));
    float cs, sn;
    m_cossin2pi(u01<float>(w.y), &cs, &sn);
    e = -(m_log(u01<float>(w.x)) + cs * cs * m_log(u01<float>(w.z)));
    const float u3 = u01<float>(w.w);
    a = u3 * u3;
}

__device__ __forceinline__ void kp_precompute(const Rng& rng, int mu, KpPre& p)
{
#pragma unroll
    for (int sg = 0; sg < 3; sg++) {
#pragma unroll
        for (int t = 0; t < kPreTrials; t++) kp_trial_parts(rng, mu, sg, t, p.e[sg][t], p.a[sg][t]);
        const uint4 w = rng.draw(ctr_word(P_HB_DIR, mu, sg, 0, 0));
        const float ct = 2.0f * u01<float>(w.x) - 1.0f;
        const float stt = m_sqrt(m_max(0.0f, 1.0f - ct * ct));
        float cp, sp;
        m_cossin2pi(u01<float>(w.y), &cp, &sp);
        p.ct[sg] = ct;
        p.sc[sg] = stt * cp;
        p.ss[sg] = stt * sp;
    }
}

// g0 for the precomputed case: the same trials in the same order as draw_g0.
__device__ __forceinline__ bool draw_g0_pre(const Rng& rng, float alpha, int mu, int sg, const HbArgs& hb,
                                            const KpPre& p, float& g0)
{
    const float ia = __builtin_amdgcn_rcpf(alpha);
#pragma unroll
    for (int t = 0; t < kPreTrials; t++) {
        if (t >= hb.max_tries) return false;
        const float delta = p.e[sg][t] * ia;
        if (p.a[sg][t] <= 1.0f - 0.5f * delta) {
            g0 = 1.0f - delta;
            return true;
        }
    }
    for (int t = kPreTrials; t < hb.max_tries; t++) {
        float e, a;
        kp_trial_parts(rng, mu, sg, t, e, a);
        const float delta = e * ia;
        if (a <= 1.0f - 0.5f * delta) {
            g0 = 1.0f - delta;
            return true;
        }
    }
    return false;
}

// Direction of g: cos(theta) = 2 u0 - 1, phi = 2 pi u1 (Philox word
// (P_HB_DIR, mu, sub, hit, 0)); g = (g0, s sin(theta) cos(phi),
// s sin(theta) sin(phi), s cos(theta)), s = sqrt(1 - g0^2).
template <typename R>
__device__ __forceinline__ void draw_dir(const Rng& rng, int mu, int sg, int h, R g0, R g[4])
{
    const uint4 w = rng.draw(ctr_word(P_HB_DIR, mu, sg, h, 0));
    const R ct = R(2) * u01<R>(w.x) - R(1);
    const R stt = m_sqrt(m_max(R(0), R(1) - ct * ct));
    R cp, sp;
    m_cossin2pi(u01<R>(w.y), &cp, &sp);
    const R sr = m_sqrt(m_max(R(0), R(1) - g0 * g0));
    g[0] = g0;
    g[1] = sr * stt * cp;
    g[2] = sr * stt * sp;
    g[3] = sr * ct;
}

// KIND bits: 1 overrelaxation (else heat bath), 2 plaquette site values,
// 4 fp64 re-orthonormalization of fp32 stores (the last pass of a sweep).
constexpr int PH_OR = 1, PH_PLAQ = 2, PH_STORE64 = 4;

template <typename R, int NC, int KIND>
__global__ void __launch_bounds__(512) k_phase(Grid gr, int mu, int par, const uint64_t* __restrict__ sweep_base,
                                               int sweep_off, HbArgs hb, unsigned long long* exhausted)
{
    constexpr bool kF64 = std::is_same<R, double>::value;
    constexpr bool kHB = (KIND & PH_OR) == 0;
    constexpr bool kPlaq = (KIND & PH_PLAQ) != 0;
    const int lb = logical_block(blockIdx.x, gr.nblocks, gr.remap);
    const int l = find_lattice_p(gr.bbeg, gr.nlat, lb);
    const LatDesc& d = gr.descs[l];
    const Geo g = d.g;
    const int w = (lb - gr.bbeg[l]) * (int)blockDim.x + (int)threadIdx.x;
    if (w >= g.Vh) return;

    const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
    int n[4];
    tiled_coords(g, d.tile, w, par, n);
    const int cb = lex_index(g, n) >> 1;
    Rng rng{ d.seed, d.lid, (uint32_t)lex_index(g, n), 0 };
    if (kHB) rng.step = *sweep_base + (uint64_t)sweep_off;
    // fp32 KP: draws of hit 0 ahead of the staple (uniform branch)
    constexpr bool kPre = !kF64 && kHB && kPreTrials >= 0;
    const bool pre = kPre && hb.sampler == 0 && kPreTrials > 0;
    KpPre kp;
    if constexpr (kPre)
        if (pre) kp_precompute(rng, mu, kp);

    M3<R> Alo;  // kind 2: the staples of the planes (nu, mu), nu < mu
    const M3<R> A = staple_sum<R, NC, R, kPlaq>(U, g, mu, n, &Alo);
    const uintptr_t s = U.slab(mu, par);
    M3<R> u = load_link<R, NC, true>(s, cb);
    M3<R> W = m_mul(u, A);
    const R beta = (R)d.beta;
    const float b23 = (float)(d.beta * (2.0 / 3.0));  // fp32 alpha = (2 beta / 3) k
    const int nh = kHB ? hb.n_hits : 1;

    for (int h = 0; h < nh; h++) {
#pragma unroll
        for (int sg = 0; sg < 3; sg++) {
            const int i = sub_i(sg), j = sub_j(sg);
            if constexpr (kF64) {
                Cx v[2][2];
                const double k = su2_part_c(W, i, j, v);
                if (k == 0.0) continue;
                const Cx vd[2][2] = { { c_conj(v[0][0]), c_conj(v[1][0]) }, { c_conj(v[0][1]), c_conj(v[1][1]) } };
                Cx r[2][2];
                if (kHB) {
                    const double alpha = 2.0 * beta * k / 3.0;
                    double g0;
                    if (!draw_g0<double>(rng, alpha, mu, sg, h, hb, g0)) {
                        if (exhausted) atomicAdd(exhausted + l, 1ull);
                        continue;
                    }
                    double q[4];
                    draw_dir<double>(rng, mu, sg, h, g0, q);
                    const Cx gm[2][2] = { { Cx{ q[0], q[3] }, Cx{ q[2], q[1] } }, { Cx{ -q[2], q[1] }, Cx{ q[0], -q[3] } } };
                    mul2_c(gm, vd, r);
                } else {
                    mul2_c(vd, vd, r);
                }
                left_apply_c(u, i, j, r);
                left_apply_c(W, i, j, r);
            } else {
                Q4<R> v;
                const R k = su2_part(W, i, j, v);
                if (!(k > R(0))) continue;
                Q4<R> r;
                if (kHB) {
                    const R alpha = b23 * k;
                    R g0;
                    R q[4];
                    if (pre && h == 0) {
                        if (!draw_g0_pre(rng, alpha, mu, sg, hb, kp, g0)) {
                            if (exhausted) atomicAdd(exhausted + l, 1ull);
                            continue;
                        }
                        const R sr = m_sqrt(m_max(R(0), R(1) - g0 * g0));
                        q[0] = g0;
                        q[1] = sr * kp.sc[sg];
                        q[2] = sr * kp.ss[sg];
                        q[3] = sr * kp.ct[sg];
                    } else {
                        if (!draw_g0<R>(rng, alpha, mu, sg, h, hb, g0)) {
                            if (exhausted) atomicAdd(exhausted + l, 1ull);
                            continue;
                        }
                        draw_dir<R>(rng, mu, sg, h, g0, q);
                    }
                    r = q_mul(Q4<R>{ q[0], q[1], q[2], q[3] }, q_conj(v));
                } else {
                    const Q4<R> vd = q_conj(v);
                    r = q_mul(vd, vd);
                }
                left_apply(u, i, j, r);
                left_apply(W, i, j, r);
            }
        }
    }
    // fp32 links are re-orthonormalized (rows 0, 1; row 2 their completion)
    // before every store: rounding in a 12-real record would otherwise grow,
    // because the rebuilt third row feeds back into rows 0 and 1.  In fp32,
    // rows already within an ulp of unit length are not rescaled at all, and
    // sub-ulp drifts of one sign (the hardware square roots of the draws) left
    // |row|^2 - 1 at -1.7e-8 on average (0.2 of an ulp; the plaquette 3e-8
    // low).  The last pass of a sweep, which stores every link once, does it
    // in fp64 and rounds once, so the field at the end of every sweep has
    // unbiased rows (mean 1e-11).
    if constexpr (!kF64) {
        if constexpr ((KIND & PH_STORE64) != 0)
            m_reunit_for_store(u);
        else
            m_reunit(u);
    }
    if constexpr (kPlaq) {
        // Plaquette sum of the sweep, formed in its last pass: a phase (mu,
        // odd) with mu >= 1 is the last update of every plaquette in the
        // planes (nu, mu), nu < mu, and each of those plaquettes holds
        // exactly one odd-site link U_mu, whose staple has it as a term.  So
        // Re Tr(U_mu A_lo) over the odd sites, A_lo the staples with nu < mu,
        // counts each plaquette of those planes once, and the phases mu = 1,
        // 2, 3 cover all six planes.  Per site: the 2 mu plaquettes'
        // sum of 1 - (1/3) Re Tr U_p, traced in fp64 from the stored link.
        if (par == 1 && mu >= 1 && d.psite) {
            const M3<double> ud = m_cast<R, double>(u);
            const M3<double> ad = m_cast<R, double>(Alo);
            double t = 0.0;
#pragma unroll
            for (int r = 0; r < 3; r++)
#pragma unroll
                for (int k = 0; k < 3; k++) t += ud.re[3 * r + k] * ad.re[3 * k + r] - ud.im[3 * r + k] * ad.im[3 * k + r];
            d.psite[(size_t)(mu - 1) * g.Vh + cb] = (double)(2 * mu) - t / 3.0;
        }
    }
    store_link<R, NC, true>(s, cb, u);
}

// Overrelaxation phases keep at most 12 wavefronts per CU in flight: with
// more, the links of their sites and neighbours overflow the XCD's 4 MB L2
// before the other readers of a record run (a 32^4 R12 phase took 47.0 us at
// 20 wavefronts per CU and 45.0 us at 12; 8 and 16 were slower, and the heat
// bath, with more arithmetic per load, is faster uncapped).  The cap reserves
// LDS per block, which the kernel does not use: 144 KB shared by the blocks
// allowed (three blocks of 54.5 KB did not fit together on a CU, three of 48
// KB did).  Blocks of 512 threads are left alone (a cap there would exceed 64
// KB per block).
// fp64 records are three times larger: its overrelaxation phases keep at most
// 4 wavefronts per CU (a 32^4 phase 173.8 -> 166.5 us; its heat bath, again,
// is faster uncapped at the 8 its registers allow).  18-real fp32 records,
// 1.5 times the 12-real ones, keep at most 8 in both kinds of phase (32^4:
// overrelaxation 72.2 -> 66.1 us, heat bath 78.2 -> 72.1 us; 4 per CU gave
// 85 us for overrelaxation).
constexpr int kOrWavesPerCu = 12;
constexpr int kOrWavesPerCuF64 = 4;
constexpr int kWavesPerCuF32x18 = 8;

static size_t or_lds_bytes(int block, int waves_per_cu)
{
    const int waves = block / 64;
    if (waves < 1 || waves > 4) return 0;
    const int blocks_per_cu = waves_per_cu / waves > 0 ? waves_per_cu / waves : 1;
    return (size_t)(147456 / blocks_per_cu) & ~(size_t)255;
}

template <typename R, int NC, int KIND>
static hipError_t launch_phase_t(const Grid& gr, int mu, int par, const uint64_t* sb, int so, HbArgs hb,
                                 unsigned long long* ex, hipStream_t st)
{
    constexpr bool kOr = (KIND & PH_OR) != 0;
    constexpr int cap = std::is_same<R, double>::value ? (kOr ? kOrWavesPerCuF64 : 0)
                        : NC == 18                      ? kWavesPerCuF32x18
                                                        : (kOr ? kOrWavesPerCu : 0);
    const size_t lds = cap > 0 ? or_lds_bytes(gr.block, cap) : 0;
    k_phase<R, NC, KIND><<<gr.nblocks, gr.block, lds, st>>>(gr, mu, par, sb, so, hb, ex);
    return hipGetLastError();
}

}  // namespace msmc
