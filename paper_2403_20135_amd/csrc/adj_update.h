// The transposed node update of one dSDC sweep (the adjoint of the Section 4.2 node update and
// its 2x2 solve) for one (coefficient, Re/Im part, member), shared by the adjoint update kernel
// and the transposed analysis kernel's fused epilogue so that both form exactly the same
// arithmetic.  Per node m of sweep s:
//   beta_adj_m = A_{m,s}^T ubar_m,  A = (I - alpha L)^{-1},  A^T(a, b, d) = ((a + alpha c d)/D, b,
//   (d - alpha Phi_bar a)/D), D = 1 + alpha^2 Phi_bar c;  L^T(a, b, d) = (c d, 0, -Phi_bar a).
//   u_n_adj += beta_adj_m
//   E_adj_j (previous sweep) = dt sum_m q_mj beta_adj_m
//   u_adj_j (previous sweep) = dt sum_m q_mj L^T beta_adj_m - alpha_{j,s} L^T beta_adj_j
// For the last sweep only node M carries ubar (the incoming adjoint state).  When the previous
// sweep is the initial one (all nodes equal u_n, all tendencies E_0) the node sums are folded
// into u_n_adj and E_0_adj.  ub(m, field) returns ubar of node m (field 0 Phi', 1 zeta, 2 delta).
// The E adjoints go to ebar_prev, or (cml set) straight into the synthesis-adjoint input layout
// (zeta, delta, Phi', c_n delta) of the next transposed tendency: state b M + j, or b for E_0.
#pragma once
#include "common.h"

template <int M, typename UB>
__device__ __forceinline__ void adj_update_part(const AdjUpdateArgs& a, int t, int b, UB ub) {
    const int idx = t >> 1, part = t & 1;
    const int n = a.n_of[idx];
    const double c = n * (n + 1.0) * a.inv_a2;
    const size_t o = (size_t)t;
    const size_t fs = (size_t)a.ncoef * 2;
    const int sdiv = a.sweep < M ? a.sweep : M;
    double bp[M], bz[M], bd[M];                               // beta_adj per node
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (a.last && m != M - 1) {
            bp[m] = bz[m] = bd[m] = 0.0;
            continue;
        }
        const double up = ub(m, 0), uz = ub(m, 1), ud = ub(m, 2);
        const double alpha = a.dt * a.tau[m] / sdiv;
        const double den = 1.0 / (1.0 + alpha * alpha * a.phibar * c);
        bp[m] = (up + alpha * c * ud) * den;
        bz[m] = uz;
        bd[m] = (ud - alpha * a.phibar * up) * den;
    }
    // E adjoint (Phi', zeta, delta) of state st of a layout of S states
    auto put_e = [&](size_t st, size_t S, double ep, double ez, double ed) {
        if (a.cml) {
            const int mo = a.m_of[idx], par = (n - mo) & 1, kk = (n - mo) >> 1;
            const size_t ci = (((size_t)a.rowoff[2 * mo + par] + kk) * S + st) * kCmlVals + part;
            cml_put(a.cml, a.cml32, ci, ez);
            cml_put(a.cml, a.cml32, ci + 2, ed);
            cml_put(a.cml, a.cml32, ci + 4, ep);
            cml_put(a.cml, a.cml32, ci + 6, a.neg_lap[n] * ed);
            if (part == 0)
                cml_clear_pad(a.cml, a.cml32, a.rowoff[2 * mo + par], kk, npk_of(a.T, mo, par), S, st);
        } else {
            double* e = a.ebar_prev + st * 3 * fs + o;
            e[0] = ep;
            e[fs] = ez;
            e[2 * fs] = ed;
        }
    };
    double sp = 0.0, sz = 0.0, sd = 0.0;                      // u_n adjoint contributions
    double ep0 = 0.0, ez0 = 0.0, ed0 = 0.0;                   // E_0 adjoint when first_stage
#pragma unroll
    for (int m = 0; m < M; ++m) {
        sp += bp[m];
        sz += bz[m];
        sd += bd[m];
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double qp = 0.0, qz = 0.0, qd = 0.0;                  // sum_m q_mj beta_adj_m
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const double qmj = a.Q[m * kMaxNodes + j];
            qp += qmj * bp[m];
            qz += qmj * bz[m];
            qd += qmj * bd[m];
        }
        const double aj = a.dt * a.tau[j] / sdiv;
        // E_adj_j = dt * qsum;  u_adj_j = dt L^T qsum - alpha_j L^T beta_adj_j
        const double ep = a.dt * qp, ez = a.dt * qz, ed = a.dt * qd;
        const double wp = c * (ed - aj * bd[j]);
        const double wd = -a.phibar * (ep - aj * bp[j]);
        if (a.first_stage) {
            ep0 += ep;
            ez0 += ez;
            ed0 += ed;
            sp += wp;
            sd += wd;
        } else {
            put_e((size_t)b * M + j, (size_t)a.batch * M, ep, ez, ed);
            double* u = a.ubar_prev + ((size_t)b * M + j) * 3 * fs + o;
            u[0] = wp;
            u[fs] = 0.0;
            u[2 * fs] = wd;
        }
    }
    if (a.first_stage) put_e((size_t)b, (size_t)a.batch, ep0, ez0, ed0);
    double* un = a.ubar_n + (size_t)b * 3 * fs + o;
    if (a.init_un) {
        un[0] = sp;
        un[fs] = sz;
        un[2 * fs] = sd;
    } else {
        un[0] += sp;
        un[fs] += sz;
        un[2 * fs] += sd;
    }
}
