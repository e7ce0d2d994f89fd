// k_prolong.hip -- restriction, prolongation transfer, the APE interpolation
// step and the partial action S_d (Sec. III, restriction / prolongation /
// interpolation equations).  The interpolation works on an fp64 fine field.
//
// chi(n) = number of odd coordinates of n; chi_mu(n) and chi_munu(n) count
// them with mu (and nu) left out.  Stage d updates the bonds with
// chi_mu(n) = d + 1 all at once from the previous iterate:
//   U' = P_SU(3)[U + c sum_{nu: chi_munu(n) = d} (T^+_munu + T^-_munu)],
// where chi_munu(n) = d exactly when n_nu is odd, and P_SU(3) maximizes
// Re Tr(X^+ M) by repeated SU(2)-subgroup maximization.
#include "kernels.hpp"

namespace msmc {

__device__ __forceinline__ int n_odd_excl(const int n[4], int a, int b)
{
    int c = 0;
#pragma unroll
    for (int m = 0; m < 4; m++)
        if (m != a && m != b) c += n[m] & 1;
    return c;
}

__device__ __forceinline__ void link_of(const Geo& g, int e, int& mu, int& par, int& cb, int n[4])
{
    const int slab = e / g.Vh;
    cb = e - slab * g.Vh;
    mu = slab >> 1;
    par = slab & 1;
    cb_coords(g, cb, par, n);
}

// U^c_mu(n/2) = U^f_mu(n) U^f_mu(n + e_mu) on fine sites with all coordinates even
template <typename RF, int NF, typename RC, int NCc>
__global__ void __launch_bounds__(256) k_restrict(Geo gf, const RF* __restrict__ Uf, size_t csf, Geo gc,
                                                  RC* __restrict__ Uc, size_t csc)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 8 * gc.Vh) return;
    int mu, par, cb, nc[4];
    link_of(gc, e, mu, par, cb, nc);
    int nf[4] = { 2 * nc[0], 2 * nc[1], 2 * nc[2], 2 * nc[3] };
    const Links<RF, NF> F{ (uintptr_t)Uf, csf };
    const M3<double> a = m_cast<RF, double>(load_at(F, gf, mu, nf));
    nf[mu] = wrap_add(nf[mu], 1, gf.L[mu]);
    const M3<double> b = m_cast<RF, double>(load_at(F, gf, mu, nf));
    const Links<RC, NCc> C{ (uintptr_t)Uc, csc };
    store_link<RC, NCc>(C.slab(mu, par), cb, m_cast<double, RC>(m_mul(a, b)));
}

// Fine bond U^f_mu(n) = U^c_mu(n/2) where all coordinates of n are even, 1 elsewhere.
template <typename RC, int NCc>
__global__ void __launch_bounds__(256) k_transfer(Geo gc, const RC* __restrict__ Uc, size_t csc, Geo gf,
                                                  double* __restrict__ Uf, size_t csf)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 8 * gf.Vh) return;
    int mu, par, cb, n[4];
    link_of(gf, e, mu, par, cb, n);
    M3<double> m;
    if (((n[0] | n[1] | n[2] | n[3]) & 1) == 0) {
        const int nc[4] = { n[0] >> 1, n[1] >> 1, n[2] >> 1, n[3] >> 1 };
        const Links<RC, NCc> C{ (uintptr_t)Uc, csc };
        m = m_cast<RC, double>(load_at(C, gc, mu, nc));
    } else {
        m_set_one(m);
    }
    store_link<double, 18>((uintptr_t)Uf + (uintptr_t)(mu * 2 + par) * csf, cb, m);
}

// Re Tr(X^+ M) summed as the trace of the product X^+ M: diagonal element r
// is sum_k conj(X_kr) M_kr (k ascending), then (d0 + d1) + d2.
__device__ __forceinline__ double retr_dn(const M3<double>& x, const M3<double>& m)
{
    double d[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < 3; k++) t += x.re[k * 3 + r] * m.re[k * 3 + r] + x.im[k * 3 + r] * m.im[k * 3 + r];
        d[r] = t;
    }
    return (d[0] + d[1]) + d[2];
}

// Plaquette trace Re Tr(X Y^+) for the partial action.
__device__ __forceinline__ double retr_nd(const M3<double>& x, const M3<double>& y)
{
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 9; k++) t += x.re[k] * y.re[k] + x.im[k] * y.im[k];
    return t;
}

// argmax over X in SU(3) of Re Tr(X^+ M): start from the unitarized M, then
// rounds of SU(2)-subgroup maximization (X <- R X, R the SU(2) part of M X^+)
// until a round gains no more than 1e-15 relative (at most 100 rounds).  The
// fp64 operations follow a fixed order, so the stopping round is reproducible.
__device__ M3<double> project_su3(const M3<double>& M)
{
    M3<double> X = M;
    m_reunit(X);
    double f_prev = retr_dn(X, M);
    for (int it = 0; it < 100; it++) {
#pragma unroll
        for (int s = 0; s < 3; s++) {
            const M3<double> Y = m_mul_nd(M, X);
            Cx v[2][2];
            if (su2_part_c(Y, sub_i(s), sub_j(s), v) == 0.0) continue;
            left_apply_c(X, sub_i(s), sub_j(s), v);
        }
        const double f = retr_dn(X, M);
        if (f - f_prev <= 1e-15 * fabs(f)) break;
        f_prev = f;
    }
    return X;
}

// The bonds a stage updates, grouped in classes: a direction mu and the set
// of other coordinates that are odd (a bit mask, bit m for coordinate m).
// Each class holds V/8 sites: n_mu takes every value, each other coordinate
// the values of its parity, numbered with coordinate 0 fastest so that a
// wavefront reads consecutive checkerboard sites.  A block takes 256
// consecutive sites of one class; blocks run chunk-major and class-minor,
// renumbered so that each XCD gets a contiguous range, so the classes of one
// region of the lattice are updated together and share its links in L2.
struct BondClasses {
    int n;
    int mu[12];
    int odd[12];
};

// Site r of a class: coordinates in the mask `free` take every value, the
// others the values of the parity given by `odd`; coordinate 0 fastest.
__device__ __forceinline__ void class_site(const Geo& g, int free, int odd, int r, int n[4])
{
#pragma unroll
    for (int m = 0; m < 4; m++) {
        if ((free >> m) & 1) {
            n[m] = r % g.L[m];
            r /= g.L[m];
        } else {
            const int h = g.L[m] >> 1;
            n[m] = 2 * (r % h) + ((odd >> m) & 1);
            r /= h;
        }
    }
}

__device__ __forceinline__ double block_sum_256p(double v)
{
    __shared__ double sh[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) v = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return v;
}

// Progress of one interpolation stage, kept on the device so that steps can
// be enqueued without a host round trip per step: s_prev is the partial
// action of the last iterate seen, done is set (with iters, the number of
// steps of the result) once the stopping rule holds or max_iter is reached.
struct ApeState {
    double s_prev;
    int done;
    int iters;
};

// Step j of stage d (reads iterate j-1, writes iterate j) on the bonds with
// chi_mu(n) = d + 1 only; Unew must already hold every other bond (they do
// not change in a stage).  It also returns, as block sums, the partial action
// S_d of iterate j-1: each plaquette of S_d contains exactly two updated bonds
// and is the staple term of both, so summing 1 - Re Tr(U T^+)/6 over the
// bonds and staple directions (T = T+ + T-, two plaquettes) counts each
// plaquette's 1 - Re Tr/3 once.  A finished stage makes the launch a no-op.
__global__ void __launch_bounds__(256) k_ape(Geo g, const double* __restrict__ Uold, double* __restrict__ Unew,
                                             size_t cs, int d, double c, BondClasses bc,
                                             const ApeState* __restrict__ st, double* __restrict__ bsum)
{
    if (st->done) return;
    const int per = g.Vh >> 2;  // V / 8
    const int lb = logical_block(blockIdx.x, gridDim.x, 1);
    const int k = lb % bc.n;
    const int r = (lb / bc.n) * 256 + threadIdx.x;
    double acc = 0.0;
    if (r < per) {
        const int mu = bc.mu[k];
        int n[4];
        class_site(g, 1 << mu, bc.odd[k], r, n);
        const Links<double, 18> U{ (uintptr_t)Uold, cs };
        const M3<double> u = load_at(U, g, mu, n);
        // M = U + c (T+ + T-) added direction by direction, nu ascending
        M3<double> M = u;
        for (int nu = 0; nu < 4; nu++) {
            if (nu == mu || n_odd_excl(n, mu, nu) != d) continue;
            int npn[4] = { n[0], n[1], n[2], n[3] }, npm[4] = { n[0], n[1], n[2], n[3] },
                nmn[4] = { n[0], n[1], n[2], n[3] };
            npn[nu] = wrap_add(n[nu], 1, g.L[nu]);
            npm[mu] = wrap_add(n[mu], 1, g.L[mu]);
            nmn[nu] = wrap_add(n[nu], -1, g.L[nu]);
            int nmn_pm[4] = { nmn[0], nmn[1], nmn[2], nmn[3] };
            nmn_pm[mu] = npm[mu];
            // T+ = U_nu(n) U_mu(n+nu) U_nu(n+mu)^+
            M3<double> T = m_mul_nd(m_mul(load_at(U, g, nu, n), load_at(U, g, mu, npn)), load_at(U, g, nu, npm));
            // T- = U_nu(n-nu)^+ U_mu(n-nu) U_nu(n-nu+mu)
            m_acc(T, m_mul(m_mul_dn(load_at(U, g, nu, nmn), load_at(U, g, mu, nmn)), load_at(U, g, nu, nmn_pm)));
            acc += 1.0 - retr_nd(u, T) / 6.0;
#pragma unroll
            for (int k2 = 0; k2 < 9; k2++) {
                M.re[k2] += T.re[k2] * c;
                M.im[k2] += T.im[k2] * c;
            }
        }
        const int par = (n[0] + n[1] + n[2] + n[3]) & 1;
        store_link<double, 18>((uintptr_t)Unew + (uintptr_t)(mu * 2 + par) * cs, lex_index(g, n) >> 1,
                               project_su3(M));
    }
    acc = block_sum_256p(acc);
    if (threadIdx.x == 0) bsum[blockIdx.x] = acc;
}

// After step j: S_d of iterate j-1 from the block sums (each thread a strided
// share in block order, then a fixed tree); step j-1 ends the stage when S_d
// changed by no more than rel_tol relative to iterate j-2, else step j ends
// it when j = max_iter.
__global__ void __launch_bounds__(256) k_ape_check(const double* __restrict__ bsum, int nblk, ApeState* st, int j,
                                                   double rel_tol, int max_iter)
{
    if (st->done) return;
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) v += bsum[b];
    v = block_sum_256p(v);
    if (threadIdx.x == 0) {
        if (j >= 2 && fabs(v - st->s_prev) <= rel_tol * st->s_prev) {
            st->done = 1;
            st->iters = j - 1;
        } else if (j >= max_iter) {
            st->done = 1;
            st->iters = j;
        }
        st->s_prev = v;
    }
}

__global__ void k_ape_reset(ApeState* st)
{
    st->s_prev = 0.0;
    st->done = 0;
    st->iters = 0;
}

template <typename RF, int NF>
static hipError_t restrict_to(const Geo& gf, const void* Uf, size_t csf, int pc, const Geo& gc, void* Uc, size_t csc,
                              hipStream_t st)
{
    const int nb = (8 * gc.Vh + 255) / 256;
    switch (pc) {
    case PREC_F64: k_restrict<RF, NF, double, 18><<<nb, 256, 0, st>>>(gf, (const RF*)Uf, csf, gc, (double*)Uc, csc); break;
    case PREC_F32: k_restrict<RF, NF, float, 18><<<nb, 256, 0, st>>>(gf, (const RF*)Uf, csf, gc, (float*)Uc, csc); break;
    case PREC_F32_R12: k_restrict<RF, NF, float, 12><<<nb, 256, 0, st>>>(gf, (const RF*)Uf, csf, gc, (float*)Uc, csc); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_restrict(int pf, const Geo& gf, const void* Uf, size_t csf, int pc, const Geo& gc, void* Uc,
                           size_t csc, hipStream_t st)
{
    switch (pf) {
    case PREC_F64: return restrict_to<double, 18>(gf, Uf, csf, pc, gc, Uc, csc, st);
    case PREC_F32: return restrict_to<float, 18>(gf, Uf, csf, pc, gc, Uc, csc, st);
    case PREC_F32_R12: return restrict_to<float, 12>(gf, Uf, csf, pc, gc, Uc, csc, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_transfer(int pc, const Geo& gc, const void* Uc, size_t csc, const Geo& gf, double* Uf, size_t csf,
                           hipStream_t st)
{
    const int nb = (8 * gf.Vh + 255) / 256;
    switch (pc) {
    case PREC_F64: k_transfer<double, 18><<<nb, 256, 0, st>>>(gc, (const double*)Uc, csc, gf, Uf, csf); break;
    case PREC_F32: k_transfer<float, 18><<<nb, 256, 0, st>>>(gc, (const float*)Uc, csc, gf, Uf, csf); break;
    case PREC_F32_R12: k_transfer<float, 12><<<nb, 256, 0, st>>>(gc, (const float*)Uc, csc, gf, Uf, csf); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static BondClasses bond_classes(int d)
{
    BondClasses bc;
    bc.n = 0;
    for (int mu = 0; mu < 4; mu++)
        for (int odd = 0; odd < 16; odd++)
            if (!((odd >> mu) & 1) && __builtin_popcount(odd) == d + 1) {
                bc.mu[bc.n] = mu;
                bc.odd[bc.n] = odd;
                bc.n++;
            }
    return bc;
}

int ape_blocks(const Geo& gf, int d)
{
    return bond_classes(d).n * (((gf.Vh >> 2) + 255) / 256);
}

size_t ape_state_bytes() { return sizeof(ApeState); }

hipError_t launch_ape_reset(void* state, hipStream_t st)
{
    k_ape_reset<<<1, 1, 0, st>>>((ApeState*)state);
    return hipGetLastError();
}

hipError_t launch_ape_step(const Geo& gf, const double* Uold, double* Unew, size_t csf, int d, double c, int j,
                           double rel_tol, int max_iter, void* state, double* block_sums, int nblk, hipStream_t st)
{
    for (int m = 0; m < 4; m++)
        if (gf.L[m] & 1) return hipErrorInvalidValue;
    if (nblk != ape_blocks(gf, d) || nblk == 0) return hipErrorInvalidValue;
    k_ape<<<nblk, 256, 0, st>>>(gf, Uold, Unew, csf, d, c, bond_classes(d), (const ApeState*)state, block_sums);
    k_ape_check<<<1, 256, 0, st>>>(block_sums, nblk, (ApeState*)state, j, rel_tol, max_iter);
    return hipGetLastError();
}

hipError_t read_ape_state(const void* state, int* done, int* iters, hipStream_t st)
{
    ApeState h;
    hipError_t e = hipMemcpyAsync(&h, state, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    *done = h.done;
    *iters = h.iters;
    return e;
}

}  // namespace msmc
