// Discrete adjoint of one dSDC step (transpose of every linear map of the forward step, at the
// recomputed stages), with respect to the real inner product over (Re, Im) of every coefficient.
//
// f_E(u) = Analysis(Products(Synthesis(u))) has the Jacobian transpose
//   J^T = Synthesis^T . Products'^T . Analysis^T.
// * Analysis^T (the synthesis kernel in adjoint mode + the first half of k_grid_adj): the analysis of a grid
//   field is c_nm = sum_j w_j Pbar (1/nlon) DFT_m; its transpose is a synthesis with unit m-weights
//   scaled per latitude.  For the tendencies zeta_t = -div(A,B), delta_t = curl(A,B) + c_n KE,
//   Phi'_t = -div(C,D), with div/curl weights g'_j = w_j/(1-mu_j^2):
//     A^ = i m Pbar.zeta_adj + H.delta_adj,   B^ = H.zeta_adj - i m Pbar.delta_adj,
//     C^ = i m Pbar.Phi_adj,  D^ = H.Phi_adj,  E^ = Pbar.(c_n delta_adj)
//   and on the grid A_adj = g'_j/(a nlon) sum_m Re(A^_m e^{i m lambda}) (unit m-weights; E with
//   w_j/nlon).
// * Products'^T (k_grid_adj): at the stage's grid fields (zeta, Phi', U, V), q = zeta + f,
//     zeta_g_adj = A U + B V, Phi_g_adj = C U + D V,
//     U_adj = A q + C Phi' + E U/(1-mu^2), V_adj = B q + D Phi' + E V/(1-mu^2).
// * Synthesis^T (second half of k_grid_adj + analysis kernel in adjoint mode): for a scalar field
//   (Synthesis^T g)_nm = s_m sum_j Pbar DFT_m(g) (unnormalised, no quadrature weight); for the winds
//   psi_adj = (s_m/a) sum_j [-i m V^ Pbar - U^ H], chi_adj = (s_m/a) sum_j [-i m U^ Pbar + V^ H],
//   zeta_adj += -a^2/(n(n+1)) psi_adj, delta_adj += -a^2/(n(n+1)) chi_adj.
// The node update and solve are per-coefficient linear maps with constant real coefficients; their
// transposes are written out in k_update_adj.
#include "adj_update.h"

__device__ __forceinline__ double2 ld2a(const double* p) { return *(const double2*)p; }
__device__ __forceinline__ void st2a(double* p, double2 v) { *(double2*)p = v; }

// ---------------------------------------------------------------------------------------------
// Coefficient-major layout of adjoint tendencies: (zeta_adj, delta_adj, Phi_adj, c_n delta_adj).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_prep_cml_adj(const double* __restrict__ ebar, int nstates,
                                                         double* __restrict__ cml, int cml32,
                                                         const int* __restrict__ n_of,
                                                         const int* __restrict__ m_of,
                                                         const int* __restrict__ rowoff,
                                                         const double* __restrict__ neg_lap, int ncoef,
                                                         int T) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (idx >= ncoef) return;
    const int n = n_of[idx], mo = m_of[idx], par = (n - mo) & 1, kk = (n - mo) >> 1;
    const size_t fs = (size_t)ncoef * 2;
    const double* e = ebar + (size_t)s * 3 * fs + (size_t)idx * 2;
    const double2 phi = ld2a(e), zeta = ld2a(e + fs), dv = ld2a(e + 2 * fs);
    const double c = neg_lap[n];
    const size_t ci = (((size_t)rowoff[2 * mo + par] + kk) * nstates + s) * kCmlVals;
    if (cml32) {
        float4* o = reinterpret_cast<float4*>(reinterpret_cast<float*>(cml) + ci);
        o[0] = make_float4((float)zeta.x, (float)zeta.y, (float)dv.x, (float)dv.y);
        o[1] = make_float4((float)phi.x, (float)phi.y, (float)(c * dv.x), (float)(c * dv.y));
    } else {
        double* o = cml + ci;
        st2a(o, zeta);
        st2a(o + 2, dv);
        st2a(o + 4, phi);
        st2a(o + 6, make_double2(c * dv.x, c * dv.y));
    }
    cml_clear_pad(cml, cml32, rowoff[2 * mo + par], kk, npk_of(T, mo, par), nstates, s);
}

void launch_prep_cml_adj(const double* ebar, int nstates, double* cml, bool cml32, const int* n_of,
                         const int* m_of,
                         const int* rowoff, const double* neg_lap, int ncoef, int T, hipStream_t st) {
    dim3 grid((ncoef + kBlock - 1) / kBlock, nstates);
    k_prep_cml_adj<<<grid, kBlock, 0, st>>>(ebar, nstates, cml, cml32 ? 1 : 0, n_of, m_of, rowoff, neg_lap,
                                            ncoef, T);
}

// Node-update adjoint (adj_update_part), one thread per (coefficient, Re/Im part, member): every
// map here has real coefficients.
template <int M>
__global__ __launch_bounds__(64) void k_update_adj(AdjUpdateArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= 2 * a.ncoef) return;
    const size_t fs = (size_t)a.ncoef * 2;
    const double* u = a.ubar + (size_t)b * a.ubar_member + (size_t)t;
    adj_update_part<M>(a, t, b, [&](int m, int f) {
        return u[(size_t)(a.last ? 0 : m) * a.ubar_node + f * fs];
    });
}

void launch_update_adj(const AdjUpdateArgs& a, hipStream_t st) {
    dim3 grid((2 * a.ncoef + 63) / 64, a.batch);
    switch (a.M) {
    case 1: k_update_adj<1><<<grid, 64, 0, st>>>(a); break;
    case 2: k_update_adj<2><<<grid, 64, 0, st>>>(a); break;
    case 3: k_update_adj<3><<<grid, 64, 0, st>>>(a); break;
    case 4: k_update_adj<4><<<grid, 64, 0, st>>>(a); break;
    case 5: k_update_adj<5><<<grid, 64, 0, st>>>(a); break;
    case 6: k_update_adj<6><<<grid, 64, 0, st>>>(a); break;
    case 7: k_update_adj<7><<<grid, 64, 0, st>>>(a); break;
    default: k_update_adj<8><<<grid, 64, 0, st>>>(a); break;
    }
}

// Copy the accumulated adjoint to the output with the m = 0 imaginary parts set to zero.
__global__ __launch_bounds__(kBlock) void k_finish_adj(const double* __restrict__ src,
                                                       double* __restrict__ dst,
                                                       const int* __restrict__ m_of, int ncoef,
                                                       long long total) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;   // one double2 each
    if (k >= total) return;
    const int idx = (int)(k % ncoef);
    double2 v = ld2a(src + 2 * k);
    if (m_of[idx] == 0) v.y = 0.0;
    st2a(dst + 2 * k, v);
}

void launch_finish_adj(const double* src, double* dst, const int* m_of, int ncoef, int nstates,
                       hipStream_t st) {
    const long long total = (long long)nstates * 3 * ncoef;
    k_finish_adj<<<(int)((total + kBlock - 1) / kBlock), kBlock, 0, st>>>(src, dst, m_of, ncoef, total);
}
