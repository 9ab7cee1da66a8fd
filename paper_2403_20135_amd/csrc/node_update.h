// The node update of the dSDC sweep (Section 4.2) for one (coefficient, Re/Im part, member),
// shared by the update kernel and the analysis kernel's fused epilogue so that both form exactly
// the same arithmetic:
//   beta_m = u_n + dt sum_j Q[m][j] (L_g(u_j) + E_j) - alpha_m L_g(u_m);  u_m <- solve(alpha_m, beta_m)
// alpha_m = dt tau_m / min(sweep, M) (MIN-SR-FLEX; MIN-SR-NS passes sweep = M).  ep(j, field)
// returns E_j of this coefficient and part (field 0 Phi', 1 zeta, 2 delta).  When last_only, only
// node M is updated and written (to the state), with a non-finite check.
#pragma once
#include "common.h"

template <int M, typename EP>
__device__ __forceinline__ void node_update_part(const UpdateArgs& a, int idx, int c, int b, EP ep) {
    const int nc = a.ncoef;
    const int n = a.n_of[idx];
    const double cn = n * (n + 1.0) * a.inv_a2;
    const size_t o = (size_t)(2 * idx + c);
    const size_t fs = (size_t)nc * 2;             // field stride in doubles
    const double* un = a.un + (size_t)b * 3 * fs + o;
    const double u0p = un[0], u0z = un[fs], u0d = un[2 * fs];
    double Fphi[M], Fzeta[M], Fdiv[M];
    double Lphi[M], Ldiv[M];                      // L_g(u_j) (zeta component is zero)
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double* uj = a.uprev + (size_t)b * a.uprev_member + (size_t)j * a.uprev_node + o;
        Lphi[j] = -a.phibar * uj[2 * fs];
        Ldiv[j] = cn * uj[0];
        Fphi[j] = Lphi[j] + ep(j, 0);
        Fzeta[j] = ep(j, 1);
        Fdiv[j] = Ldiv[j] + ep(j, 2);
    }
    const int sdiv = a.sweep < M ? a.sweep : M;
    const int m_begin = a.last_only ? M - 1 : 0;
    bool bad = false;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (m < m_begin) continue;
        const double* Qm = a.Q + m * kMaxNodes;
        double sp = 0.0, sz = 0.0, sd = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const double qj = Qm[j];
            sp += qj * Fphi[j];
            sz += qj * Fzeta[j];
            sd += qj * Fdiv[j];
        }
        const double alpha = a.dt * a.tau[m] / sdiv;
        const double bphi = u0p + a.dt * sp - alpha * Lphi[m];
        const double bzeta = u0z + a.dt * sz;
        const double bdiv = u0d + a.dt * sd - alpha * Ldiv[m];
        const double den = 1.0 / (1.0 + alpha * alpha * a.phibar * cn);
        const double phi = (bphi - alpha * a.phibar * bdiv) * den;
        const double dv = bdiv + alpha * cn * phi;
        double* out = a.uout + (size_t)b * a.out_member + (size_t)(a.last_only ? 0 : m) * a.out_node + o;
        out[0] = phi;
        out[fs] = bzeta;
        out[2 * fs] = dv;
        if (a.last_only) bad = !(isfinite(phi) && isfinite(bzeta) && isfinite(dv));
    }
    if (bad) a.flag[0] = 1;
}
