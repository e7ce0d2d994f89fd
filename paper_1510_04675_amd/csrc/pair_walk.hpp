// pair_walk.hpp -- the thread -> link walk of the fp32 kernels that update
// all 4V links at once and read neighbour links (HMC step, flow stage), with
// the block's own links in LDS; and the staple sums of these kernels, fp32
// and fp64, with the forward products shared within a site.
#pragma once

#include "kernels.hpp"

namespace msmc {

// The pair walk of the fp32 kernels over all 4V links (HMC step, flow
// stage): a block of 512 threads takes the four directions of the same 64
// checkerboard positions in both parities (wavefront w: parity w >> 2,
// direction w & 3), i.e. whole x rows when L0 / 2 divides 64.  Each thread
// puts its own link into LDS; a staple then reads from there the links at its
// own site and at n +- e_0 (a third of its links at 32^4), which are own links
// of the block, and the rest from memory.  It is the link walk taken two
// blocks at a time (launch nblocks / 2 blocks): pair block p covers the link
// walk's logical blocks 2p (even sites) and 2p + 1 (odd sites).
constexpr int kPairSlots = 512;
typedef v2f PairLds[9][kPairSlots];

template <int NC> struct PairLd {
    GlobalLd<NC> gl;
    const PairLds& lds;
    int par, lane, w, w0, Vh, x0h;
    // slot of the link (dir, m) if it is in the block, else -1
    __device__ __forceinline__ int slot(int kind, int dir, const int m[4]) const
    {
        if (kind == NB_SAME) return par * 256 + dir * 64 + lane;
        if (kind == NB_OTHER) return -1;
        const int wn = w - x0h + (m[0] >> 1);  // same row, other parity
        if (wn < w0 || wn >= w0 + 64 || wn >= Vh) return -1;
        return (1 - par) * 256 + dir * 64 + (wn - w0);
    }
    __device__ __forceinline__ M3<float> from_lds(int sl) const
    {
        M3<float> m;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const v2f v = lds[k][sl];
            m.re[k] = v.x;
            m.im[k] = v.y;
        }
        return m;
    }
    __device__ __forceinline__ M3<float> full(int dir, const int m[4], int kind) const
    {
        const int sl = slot(kind, dir, m);
        return sl >= 0 ? from_lds(sl) : gl.full(dir, m, kind);
    }
    __device__ __forceinline__ Rows2 rows(int dir, const int m[4], int kind) const
    {
        const int sl = slot(kind, dir, m);
        if (sl < 0) return gl.rows(dir, m, kind);
        Rows2 r;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const v2f v = lds[k][sl];
            r.re[k] = v.x;
            r.im[k] = v.y;
        }
        return r;
    }
    __device__ __forceinline__ void rows_c01(int dir, const int m[4], int kind, Rows2& a, float a2r[2],
                                             float a2i[2]) const
    {
        gl.rows_c01(dir, m, kind, a, a2r, a2i);
    }
};

template <int NC> struct PairWalk {
    const LatDesc* d;
    Geo g;  // a copy: the loaders keep references to it
    Links<float, NC> U;
    int pb, lane, par, mu, w0, w, own, cb, n[4];
    bool valid;
    __device__ __forceinline__ PairLd<NC> loader(const PairLds& lds) const
    {
        return PairLd<NC>{ GlobalLd<NC>{ U, g }, lds, par, lane, w, w0, g.Vh, n[0] >> 1 };
    }
};

// Locates the thread's link and stores it into its LDS slot; every thread of
// the block reaches the barrier, so callers may return early afterwards only
// if they hold no later barrier.
template <int NC> __device__ __forceinline__ PairWalk<NC> pair_walk(const Grid& gr, PairLds& lds)
{
    PairWalk<NC> x;
    const int nb2 = gr.nblocks >> 1;
    x.pb = logical_block(blockIdx.x, nb2, gr.remap);
    int lo = 0, hi = gr.nlat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (gr.bbeg[mid] <= 2 * x.pb)
            lo = mid;
        else
            hi = mid - 1;
    }
    x.d = &gr.descs[lo];
    x.g = x.d->g;
    x.U = Links<float, NC>{ (uintptr_t)x.d->U, x.d->cs };
    x.lane = (int)threadIdx.x & 63;
    const int wv = (int)threadIdx.x >> 6;
    x.par = wv >> 2;
    x.mu = wv & 3;
    x.w0 = (x.pb - (gr.bbeg[lo] >> 1)) * 64;
    x.w = x.w0 + x.lane;
    x.valid = x.w < x.g.Vh;
    x.own = x.par * 256 + x.mu * 64 + x.lane;
    x.n[0] = x.n[1] = x.n[2] = x.n[3] = 0;
    x.cb = 0;
    if (x.valid) {
        tiled_coords(x.g, x.d->tile, x.w, x.par, x.n);
        x.cb = lex_index(x.g, x.n) >> 1;
        const M3<float> u = load_link<float, NC>(x.U.slab(x.mu, x.par), x.cb);
#pragma unroll
        for (int k = 0; k < 9; k++) lds[k][x.own] = v2f{ u.re[k], u.im[k] };
    }
    __syncthreads();
    return x;
}

// Staple sum of the pair walk.  In the plaquette of the plane (a, b), a < b,
// at site n the forward staples of U_a(n) and U_b(n) share one product,
// Q = U_b(n+a) U_a(n+b)^+: they are Q U_b(n)^+ and Q^+ U_a(n)^+.  The block
// holds all four directions of its sites, so one thread per site forms each
// plane's Q (directions 0, 0, 3, 1, 1, 2 for the planes (0,1), (0,2), (0,3),
// (1,2), (1,3), (2,3), at most two per thread), puts its rows 0 and 1 in LDS,
// and both threads take it from there after a barrier: 6 of a site's 48
// staple products and 12 of its 72 staple link reads fewer.  Every thread of
// the block must call it (it holds a barrier); the result is meaningful only
// where pw.valid.
constexpr int kPairPlanes = 6;
typedef v4f PairQLds[kPairPlanes][3][2 * 64];

__device__ __forceinline__ int plane_of(int a, int b)  // a < b
{
    return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}

template <int NC>
__device__ __forceinline__ M3<float> pair_staple(const PairWalk<NC>& pw, const PairLd<NC>& ld, PairQLds& qlds)
{
    constexpr int pa[kPairPlanes] = { 0, 0, 0, 1, 1, 2 }, pb[kPairPlanes] = { 1, 2, 3, 2, 3, 3 };
    constexpr int owner[kPairPlanes] = { 0, 0, 3, 1, 1, 2 };
    const Geo& g = pw.g;
    const int mu = pw.mu, qs = pw.par * 64 + pw.lane;
    if (pw.valid) {
#pragma unroll
        for (int p = 0; p < kPairPlanes; p++) {
            if (owner[p] != mu) continue;
            const int a = pa[p], b = pb[p];
            int na[4] = { pw.n[0], pw.n[1], pw.n[2], pw.n[3] };
            na[a] = wrap_add(pw.n[a], 1, g.L[a]);
            int nb[4] = { pw.n[0], pw.n[1], pw.n[2], pw.n[3] };
            nb[b] = wrap_add(pw.n[b], 1, g.L[b]);
            const Rows2 q = rows_mul_nd(ld.rows(b, na, a == 0 ? NB_XP : NB_OTHER), ld.full(a, nb, NB_OTHER));
#pragma unroll
            for (int c = 0; c < 3; c++)
                qlds[p][c][qs] = v4f{ q.re[2 * c], q.im[2 * c], q.re[2 * c + 1], q.im[2 * c + 1] };
        }
    }
    __syncthreads();
    M3<float> A;
    m_set_zero(A);
    if (!pw.valid) return A;
    int npm[4];
#pragma unroll
    for (int k = 0; k < 4; k++) npm[k] = (k == mu) ? wrap_add(pw.n[k], 1, g.L[k]) : pw.n[k];
#pragma unroll
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        {
            // U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+: Q U_nu(n)^+ for mu < nu, else Q^+ U_nu(n)^+
            Rows2 q;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const v4f v = qlds[mu < nu ? plane_of(mu, nu) : plane_of(nu, mu)][c][qs];
                q.re[2 * c] = v.x;
                q.im[2 * c] = v.y;
                q.re[2 * c + 1] = v.z;
                q.im[2 * c + 1] = v.w;
            }
            Rows2 x;
            if (mu < nu) {
                x = q;
            } else {
                // rows 0, 1 of Q^+: conj of Q's columns 0, 1, whose row-2
                // entries come from rows 0 and 1 (Q is in SU(3))
                float q2r[2], q2i[2];
                row2_entry(q.re, q.im, 0, q2r[0], q2i[0]);
                row2_entry(q.re, q.im, 1, q2r[1], q2i[1]);
#pragma unroll
                for (int r = 0; r < 2; r++) {
                    x.re[3 * r] = q.re[r];
                    x.im[3 * r] = -q.im[r];
                    x.re[3 * r + 1] = q.re[3 + r];
                    x.im[3 * r + 1] = -q.im[3 + r];
                    x.re[3 * r + 2] = q2r[r];
                    x.im[3 * r + 2] = -q2i[r];
                }
            }
            acc_su3_rows(A, rows_mul_nd(x, ld.full(nu, pw.n, NB_SAME)));
        }
        {
            // U_nu(n+mu-nu)^+ U_mu(n-nu)^+ U_nu(n-nu), as in staple_sum_rows
            int nmn[4] = { pw.n[0], pw.n[1], pw.n[2], pw.n[3] };
            nmn[nu] = wrap_add(pw.n[nu], -1, g.L[nu]);
            int npm_mn[4] = { npm[0], npm[1], npm[2], npm[3] };
            npm_mn[nu] = nmn[nu];
            Rows2 a;
            float a2r[2], a2i[2];
            ld.rows_c01(nu, npm_mn, NB_OTHER, a, a2r, a2i);
            const M3<float> b = ld.full(mu, nmn, nu == 0 ? NB_XM : NB_OTHER);
            const M3<float> c = ld.full(nu, nmn, nu == 0 ? NB_XM : NB_OTHER);
            acc_su3_rows(A, rows_bwd(a, a2r, a2i, b, c));
        }
    }
    return A;
}

// The fp64 kernels' link walk (one parity, the four directions of 64 sites
// per block of 256) shares the forward products the same way.  Q is passed
// whole (its adjoint is then exactly that of the computed Q, so no property
// of the links is assumed) and in two rounds of three planes, (0,1), (0,2),
// (0,3) and then (1,2), (1,3), (2,3), formed by directions 1, 2, 3 and then
// 0, 3, 2, so that three blocks still share a CU (27.6 KB of LDS each).
// Every thread of the block must call it (it holds barriers); the result is
// meaningful only where lw.valid.
typedef v2d WalkQLds[3][9][64];

template <int NC>
__device__ __forceinline__ M3<double> walk_staple_f64(const LinkWalk& lw, const Links<double, NC>& U, const Geo& g,
                                                      WalkQLds& qlds)
{
    constexpr int pa[kPairPlanes] = { 0, 0, 0, 1, 1, 2 }, pb[kPairPlanes] = { 1, 2, 3, 2, 3, 3 };
    constexpr int owner[kPairPlanes] = { 1, 2, 3, 0, 3, 2 };
    const int mu = lw.mu, lane = (int)threadIdx.x & 63;
    M3<double> A;
    m_set_zero(A);
#pragma unroll
    for (int r = 0; r < 2; r++) {
        if (r) __syncthreads();  // the first round's Q are read before they are overwritten
        if (lw.valid) {
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const int p = 3 * r + k;
                if (owner[p] != mu) continue;
                const int a = pa[p], b = pb[p];
                int na[4] = { lw.n[0], lw.n[1], lw.n[2], lw.n[3] };
                na[a] = wrap_add(lw.n[a], 1, g.L[a]);
                int nb[4] = { lw.n[0], lw.n[1], lw.n[2], lw.n[3] };
                nb[b] = wrap_add(lw.n[b], 1, g.L[b]);
                const M3<double> q = m_mul_nd(load_at(U, g, b, na), load_at(U, g, a, nb));
#pragma unroll
                for (int e = 0; e < 9; e++) qlds[k][e][lane] = v2d{ q.re[e], q.im[e] };
            }
        }
        __syncthreads();
        if (lw.valid) {
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const int p = 3 * r + k, a = pa[p], b = pb[p];
                if (mu != a && mu != b) continue;
                M3<double> q;
#pragma unroll
                for (int e = 0; e < 9; e++) {
                    const v2d v = qlds[k][e][lane];
                    q.re[e] = v.x;
                    q.im[e] = v.y;
                }
                const int nu = mu == a ? b : a;
                const M3<double> un = load_at(U, g, nu, lw.n);
                // U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+: Q U_nu(n)^+ for mu < nu, else Q^+ U_nu(n)^+
                if (mu == a)
                    mm_acc<false, true>(A, q, un);
                else
                    mm_acc<true, true>(A, q, un);
            }
        }
    }
    if (!lw.valid) return A;
    int npm[4];
#pragma unroll
    for (int k = 0; k < 4; k++) npm[k] = (k == mu) ? wrap_add(lw.n[k], 1, g.L[k]) : lw.n[k];
#pragma unroll
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        // U_nu(n+mu-nu)^+ U_mu(n-nu)^+ U_nu(n-nu)
        int nmn[4] = { lw.n[0], lw.n[1], lw.n[2], lw.n[3] };
        nmn[nu] = wrap_add(lw.n[nu], -1, g.L[nu]);
        int npm_mn[4] = { npm[0], npm[1], npm[2], npm[3] };
        npm_mn[nu] = nmn[nu];
        mm_acc<false, false>(A, m_mul_dd(load_at(U, g, nu, npm_mn), load_at(U, g, mu, nmn)), load_at(U, g, nu, nmn));
    }
    return A;
}

}  // namespace msmc
