// pair_walk.hpp -- the thread -> link walk of the fp32 kernels that update
// all 4V links at once and read neighbour links (HMC step, flow stage), with
// the block's own links in LDS.
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

}  // namespace msmc
