// k_update.hip -- dispatch of the checkerboard phase kernels (phase.hpp),
// field initialisation, reunitarization, gauge transformation, layout
// conversion and the SU(3) check, for gfx950.  Compiled without
// floating-point contraction (fp64 hot starts and reunitarization are part
// of the bit-reproducible fp64 chain).
#include "kernels.hpp"

namespace msmc {

__device__ __forceinline__ int find_lattice(const int* __restrict__ bbeg, int nlat, int lb)
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

hipError_t launch_phase(int prec, int kind, const Grid& gr, int mu, int par, const uint64_t* sweep_base,
                        int sweep_off, HbArgs hb, unsigned long long* exhausted, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    if (kind < 0 || kind > 7) return hipErrorInvalidValue;
    if (prec == PREC_F64) return launch_phase_f64(kind, gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
    if (prec == PREC_F32 || prec == PREC_F32_R12)
        return launch_phase_f32(prec, kind, gr, mu, par, sweep_base, sweep_off, hb, exhausted, st);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Per-link kernels over the index space link = slab * Vh + cb,
// slab = mu * 2 + parity.
// ---------------------------------------------------------------------------
struct LinkIdx {
    int l, mu, par, cb;
    bool valid;
};

__device__ __forceinline__ LinkIdx link_index(const Grid& gr, int b)
{
    LinkIdx x;
    const int lb = logical_block(b, gr.nblocks, gr.remap);
    x.l = find_lattice(gr.bbeg, gr.nlat, lb);
    const int Vh = gr.descs[x.l].g.Vh;
    const int e = (lb - gr.bbeg[x.l]) * (int)blockDim.x + (int)threadIdx.x;
    x.valid = e < 8 * Vh;
    const int slab = e / Vh;
    x.cb = e - slab * Vh;
    x.mu = slab >> 1;
    x.par = slab & 1;
    return x;
}

// Haar element from twelve normals (rows 0,1 complex Gaussian, then
// Gram-Schmidt and completion), in fp64.
__device__ __forceinline__ M3<double> haar_from_rng(const Rng& rng, uint32_t purpose, int mu)
{
    double z[12];
#pragma unroll
    for (int dd = 0; dd < 3; dd++) normals4<double>(rng.draw(ctr_word(purpose, mu, 0, 0, dd)), z + 4 * dd);
    M3<double> m;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        m.re[c] = z[2 * c];
        m.im[c] = z[2 * c + 1];
        m.re[3 + c] = z[6 + 2 * c];
        m.im[3 + c] = z[6 + 2 * c + 1];
    }
    m_reunit(m);
    return m;
}

template <typename R, int NC> __global__ void __launch_bounds__(256) k_init(Grid gr, int hot)
{
    const LinkIdx x = link_index(gr, blockIdx.x);
    if (!x.valid) return;
    const LatDesc& d = gr.descs[x.l];
    const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
    M3<double> m;
    if (hot) {
        int n[4];
        cb_coords(d.g, x.cb, x.par, n);
        Rng rng{ d.seed, d.lid, (uint32_t)lex_index(d.g, n), 0 };
        m = haar_from_rng(rng, P_INIT, x.mu);
    } else {
        m_set_one(m);
    }
    store_link<R, NC>(U.slab(x.mu, x.par), x.cb, m_cast<double, R>(m));
}

template <typename R, int NC>
__global__ void __launch_bounds__(256) k_reunit(Grid gr, const uint64_t* __restrict__ sweep_base, int sweep_off,
                                                int every)
{
    if (every > 0) {
        const uint64_t s = *sweep_base + (uint64_t)sweep_off;
        if ((s + 1) % (uint64_t)every != 0) return;
    }
    // a small grid loops over the logical blocks (most sweeps exit above)
    for (int b = blockIdx.x; b < gr.nblocks; b += gridDim.x) {
        const LinkIdx x = link_index(gr, b);
        if (!x.valid) continue;
        const LatDesc& d = gr.descs[x.l];
        const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
        const uintptr_t s = U.slab(x.mu, x.par);
        M3<double> m = m_cast<R, double>(load_link<R, NC>(s, x.cb));
        m_reunit(m);
        store_link<R, NC>(s, x.cb, m_cast<double, R>(m));
    }
}

// U_mu(n) -> Om(n) U_mu(n) Om(n+mu)^+, Om Haar-random per site from Philox
// purpose GAUGE with key (seed, 0); every thread recomputes the two Om it
// needs, so the update is in place.
template <typename R, int NC> __global__ void __launch_bounds__(256) k_gauge(Grid gr, uint32_t seed)
{
    const LinkIdx x = link_index(gr, blockIdx.x);
    if (!x.valid) return;
    const LatDesc& d = gr.descs[x.l];
    const Links<R, NC> U{ (uintptr_t)d.U, d.cs };
    int n[4];
    cb_coords(d.g, x.cb, x.par, n);
    int np[4] = { n[0], n[1], n[2], n[3] };
    np[x.mu] = wrap_add(n[x.mu], 1, d.g.L[x.mu]);
    const Rng r0{ seed, 0u, (uint32_t)lex_index(d.g, n), 0 };
    const Rng r1{ seed, 0u, (uint32_t)lex_index(d.g, np), 0 };
    const M3<double> o0 = haar_from_rng(r0, P_GAUGE, 0);
    const M3<double> o1 = haar_from_rng(r1, P_GAUGE, 0);
    const uintptr_t s = U.slab(x.mu, x.par);
    const M3<double> u = m_cast<R, double>(load_link<R, NC>(s, x.cb));
    store_link<R, NC>(s, x.cb, m_cast<double, R>(m_mul_nd(m_mul(o0, u), o1)));
}

#define DISPATCH_PREC(prec, CALL)                                 \
    switch (prec) {                                               \
    case PREC_F64: { using R = double; constexpr int NC = 18; CALL; } break; \
    case PREC_F32: { using R = float; constexpr int NC = 18; CALL; } break;  \
    case PREC_F32_R12: { using R = float; constexpr int NC = 12; CALL; } break; \
    default: return hipErrorInvalidValue;                         \
    }

hipError_t launch_init(int prec, int hot, const Grid& gr, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    DISPATCH_PREC(prec, (k_init<R, NC><<<gr.nblocks, gr.block, 0, st>>>(gr, hot)));
    return hipGetLastError();
}

hipError_t launch_reunit(int prec, const Grid& gr, const uint64_t* sweep_base, int sweep_off, int every,
                         hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    const int nb = (every > 0 && gr.nblocks > 4096) ? 4096 : gr.nblocks;
    DISPATCH_PREC(prec, (k_reunit<R, NC><<<nb, gr.block, 0, st>>>(gr, sweep_base, sweep_off, every)));
    return hipGetLastError();
}

hipError_t launch_gauge(int prec, const Grid& gr, uint32_t seed, hipStream_t st)
{
    if (gr.nblocks <= 0) return hipSuccess;
    DISPATCH_PREC(prec, (k_gauge<R, NC><<<gr.nblocks, gr.block, 0, st>>>(gr, seed)));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Layout conversion.  Host exchange layout: double [V][4][3][3][2].
// ---------------------------------------------------------------------------
template <typename R, int NC>
__global__ void __launch_bounds__(256) k_to_aos(Geo g, const R* __restrict__ U, size_t cs, double* __restrict__ aos)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 8 * g.Vh) return;
    const int slab = e / g.Vh, cb = e - slab * g.Vh, mu = slab >> 1, par = slab & 1;
    int n[4];
    cb_coords(g, cb, par, n);
    const size_t i = (size_t)lex_index(g, n);
    const M3<R> m = load_link<R, NC>((uintptr_t)U + (uintptr_t)slab * cs, cb);
    double* o = aos + (i * 4 + mu) * 18;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        o[2 * k] = (double)m.re[k];
        o[2 * k + 1] = (double)m.im[k];
    }
}

template <typename R, int NC>
__global__ void __launch_bounds__(256) k_from_aos(Geo g, R* __restrict__ U, size_t cs, const double* __restrict__ aos)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 8 * g.Vh) return;
    const int slab = e / g.Vh, cb = e - slab * g.Vh, mu = slab >> 1, par = slab & 1;
    int n[4];
    cb_coords(g, cb, par, n);
    const size_t i = (size_t)lex_index(g, n);
    const double* o = aos + (i * 4 + mu) * 18;
    M3<R> m;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        m.re[k] = (R)o[2 * k];
        m.im[k] = (R)o[2 * k + 1];
    }
    store_link<R, NC>((uintptr_t)U + (uintptr_t)slab * cs, cb, m);
}

hipError_t launch_to_aos(int prec, const LatDesc*, const Geo& g, const void* U, size_t cs, double* aos, hipStream_t st)
{
    const int nb = (8 * g.Vh + 255) / 256;
    DISPATCH_PREC(prec, (k_to_aos<R, NC><<<nb, 256, 0, st>>>(g, (const R*)U, cs, aos)));
    return hipGetLastError();
}

hipError_t launch_from_aos(int prec, const Geo& g, void* U, size_t cs, const double* aos, hipStream_t st)
{
    const int nb = (8 * g.Vh + 255) / 256;
    DISPATCH_PREC(prec, (k_from_aos<R, NC><<<nb, 256, 0, st>>>(g, (R*)U, cs, aos)));
    return hipGetLastError();
}

template <typename RD, int ND, typename RS, int NS>
__global__ void __launch_bounds__(256) k_convert(RD* __restrict__ dst, size_t csd, const RS* __restrict__ src,
                                                 size_t css, int Vh)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 8 * Vh) return;
    const int slab = e / Vh, cb = e - slab * Vh;
    const M3<RS> m = load_link<RS, NS>((uintptr_t)src + (uintptr_t)slab * css, cb);
    store_link<RD, ND>((uintptr_t)dst + (uintptr_t)slab * csd, cb, m_cast<RS, RD>(m));
}

template <typename RD, int ND>
static hipError_t convert_from(void* dst, size_t csd, int psrc, const void* src, size_t css, int Vh, hipStream_t st)
{
    const int nb = (8 * Vh + 255) / 256;
    switch (psrc) {
    case PREC_F64: k_convert<RD, ND, double, 18><<<nb, 256, 0, st>>>((RD*)dst, csd, (const double*)src, css, Vh); break;
    case PREC_F32: k_convert<RD, ND, float, 18><<<nb, 256, 0, st>>>((RD*)dst, csd, (const float*)src, css, Vh); break;
    case PREC_F32_R12: k_convert<RD, ND, float, 12><<<nb, 256, 0, st>>>((RD*)dst, csd, (const float*)src, css, Vh); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_convert(int pdst, void* dst, size_t cs_dst, int psrc, const void* src, size_t cs_src, int Vh,
                          hipStream_t st)
{
    switch (pdst) {
    case PREC_F64: return convert_from<double, 18>(dst, cs_dst, psrc, src, cs_src, Vh, st);
    case PREC_F32: return convert_from<float, 18>(dst, cs_dst, psrc, src, cs_src, Vh, st);
    case PREC_F32_R12: return convert_from<float, 12>(dst, cs_dst, psrc, src, cs_src, Vh, st);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// SU(3) check: per block the largest of max|U U^+ - 1| and |det U - 1| and
// the link index (slab * Vh + cb) where it occurs.
// ---------------------------------------------------------------------------
template <typename R, int NC>
__global__ void __launch_bounds__(256) k_check(Geo g, const R* __restrict__ U, size_t cs, double* bmax, int* barg)
{
    __shared__ double sv[256];
    __shared__ int si[256];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double dev = -1.0;
    if (e < 8 * g.Vh) {
        const int slab = e / g.Vh, cb = e - slab * g.Vh;
        const M3<double> m = m_cast<R, double>(load_link<R, NC>((uintptr_t)U + (uintptr_t)slab * cs, cb));
        const M3<double> p = m_mul_nd(m, m);
        dev = 0.0;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const double dr = p.re[k] - ((k % 4 == 0) ? 1.0 : 0.0);
            dev = fmax(dev, sqrt(dr * dr + p.im[k] * p.im[k]));
        }
        // det by expansion along row 0
        double dr = 0.0, di = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            const double mr = m.re[3 + c1] * m.re[6 + c2] - m.im[3 + c1] * m.im[6 + c2] -
                              (m.re[3 + c2] * m.re[6 + c1] - m.im[3 + c2] * m.im[6 + c1]);
            const double mi = m.re[3 + c1] * m.im[6 + c2] + m.im[3 + c1] * m.re[6 + c2] -
                              (m.re[3 + c2] * m.im[6 + c1] + m.im[3 + c2] * m.re[6 + c1]);
            dr += m.re[c] * mr - m.im[c] * mi;
            di += m.re[c] * mi + m.im[c] * mr;
        }
        dev = fmax(dev, sqrt((dr - 1.0) * (dr - 1.0) + di * di));
        double any = 0.0;  // NaN or infinite entries count as the worst
#pragma unroll
        for (int k = 0; k < 9; k++) any += m.re[k] + m.im[k];
        if (!(any - any == 0.0)) dev = 1e300;
    }
    sv[threadIdx.x] = dev;
    si[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            if (sv[threadIdx.x + o] > sv[threadIdx.x]) {
                sv[threadIdx.x] = sv[threadIdx.x + o];
                si[threadIdx.x] = si[threadIdx.x + o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bmax[blockIdx.x] = sv[0];
        barg[blockIdx.x] = si[0];
    }
}

hipError_t launch_check(int prec, const Geo& g, const void* U, size_t cs, double* block_max, int* block_arg, int nblk,
                        hipStream_t st)
{
    DISPATCH_PREC(prec, (k_check<R, NC><<<nblk, 256, 0, st>>>(g, (const R*)U, cs, block_max, block_arg)));
    return hipGetLastError();
}

}  // namespace msmc
