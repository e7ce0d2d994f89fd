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

__global__ void __launch_bounds__(256) k_ape(Geo g, const double* __restrict__ Uold, double* __restrict__ Unew,
                                             size_t cs, int d, double c)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 8 * g.Vh) return;
    int mu, par, cb, n[4];
    link_of(g, e, mu, par, cb, n);
    const Links<double, 18> U{ (uintptr_t)Uold, cs };
    const M3<double> u = load_link<double, 18>(U.slab(mu, par), cb);
    const uintptr_t dst = (uintptr_t)Unew + (uintptr_t)(mu * 2 + par) * cs;
    if (n_odd_excl(n, mu, mu) != d + 1) {
        store_link<double, 18>(dst, cb, u);
        return;
    }
    // M = U + c (T+ + T-) added direction by direction, nu ascending
    M3<double> M = u;
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu || n_odd_excl(n, mu, nu) != d) continue;
        int npn[4] = { n[0], n[1], n[2], n[3] }, npm[4] = { n[0], n[1], n[2], n[3] }, nmn[4] = { n[0], n[1], n[2], n[3] };
        npn[nu] = wrap_add(n[nu], 1, g.L[nu]);
        npm[mu] = wrap_add(n[mu], 1, g.L[mu]);
        nmn[nu] = wrap_add(n[nu], -1, g.L[nu]);
        int nmn_pm[4] = { nmn[0], nmn[1], nmn[2], nmn[3] };
        nmn_pm[mu] = npm[mu];
        // T+ = U_nu(n) U_mu(n+nu) U_nu(n+mu)^+
        M3<double> T = m_mul_nd(m_mul(load_at(U, g, nu, n), load_at(U, g, mu, npn)), load_at(U, g, nu, npm));
        // T- = U_nu(n-nu)^+ U_mu(n-nu) U_nu(n-nu+mu)
        m_acc(T, m_mul(m_mul_dn(load_at(U, g, nu, nmn), load_at(U, g, mu, nmn)), load_at(U, g, nu, nmn_pm)));
#pragma unroll
        for (int k = 0; k < 9; k++) {
            M.re[k] += T.re[k] * c;
            M.im[k] += T.im[k] * c;
        }
    }
    store_link<double, 18>(dst, cb, project_su3(M));
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

// sum over plaquettes with chi_munu(n) = d of 1 - (1/3) Re Tr U_munu(n)
__global__ void __launch_bounds__(256) k_partial_action(Geo g, const double* __restrict__ Ud, size_t cs, int d,
                                                        double* __restrict__ bsum)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (e < 2 * g.Vh) {
        const int par = e >= g.Vh ? 1 : 0;
        int n[4];
        cb_coords(g, e - par * g.Vh, par, n);
        const Links<double, 18> U{ (uintptr_t)Ud, cs };
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                if (n_odd_excl(n, mu, nu) != d) continue;
                int npm[4] = { n[0], n[1], n[2], n[3] }, npn[4] = { n[0], n[1], n[2], n[3] };
                npm[mu] = wrap_add(n[mu], 1, g.L[mu]);
                npn[nu] = wrap_add(n[nu], 1, g.L[nu]);
                const M3<double> X = m_mul(load_at(U, g, mu, n), load_at(U, g, nu, npm));
                const M3<double> Y = m_mul(load_at(U, g, nu, n), load_at(U, g, mu, npn));
                acc += 1.0 - retr_nd(X, Y) / 3.0;
            }
    }
    acc = block_sum_256p(acc);
    if (threadIdx.x == 0) bsum[blockIdx.x] = acc;
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

hipError_t launch_ape(const Geo& gf, const double* Uold, double* Unew, size_t csf, int d, double c, hipStream_t st)
{
    const int nb = (8 * gf.Vh + 255) / 256;
    k_ape<<<nb, 256, 0, st>>>(gf, Uold, Unew, csf, d, c);
    return hipGetLastError();
}

hipError_t launch_partial_action(const Geo& gf, const double* U, size_t csf, int d, double* block_sums, int nblk,
                                 hipStream_t st)
{
    k_partial_action<<<nblk, 256, 0, st>>>(gf, U, csf, d, block_sums);
    return hipGetLastError();
}

}  // namespace msmc
