// The split with the linear Coriolis term on the implicit side (the change of implicit and
// explicit terms the paper's outlook names, Section 6): f_I = L_g + L_c, f_E = N_a + N_r.
//
// L_c(u) = (0, -div(f U, f V), curl(f U, f V)), f = 2 Omega mu, in spectral space couples degree
// k of order m with k - 1 and k + 1 (mu P and (1 - mu^2) dP/dmu of orthonormal functions are
// combinations of the neighbouring degrees), per coefficient:
//   d zeta_k  = i b_k zeta_k - 2 Omega (e-_k delta_{k-1} + e+_k delta_{k+1})
//   d delta_k = i b_k delta_k + 2 Omega (e-_k zeta_{k-1} + e+_k zeta_{k+1})
// with b_k = 2 Omega m / (k (k + 1)) (0 at k = 0), e-_k = eps_k (k + 1) / k (0 at k = 0),
// e+_k = eps_{k+1} k / (k + 1), eps_k = sqrt((k^2 - m^2) / (4 k^2 - 1)), and degrees outside
// m..T dropped (the truncation).  Together with L_g (d Phi' = -Phi_bar delta, d delta = c_k Phi',
// c_k = k (k + 1) / a^2) the solve of u - alpha f_I(u) = beta splits, per order m, into two
// independent chains over k = m..T: chain c holds zeta at the degrees with k - m = c (mod 2) and
// delta and Phi' at the others, Phi' eliminated (Phi'_k = beta_Phi,k - alpha Phi_bar delta_k).
// Each chain is a complex tridiagonal system, diagonally dominant for the step sizes of the
// shallow-water configurations (off-diagonals 2 Omega alpha e <~ 0.1, diagonals of modulus >= 1),
// solved without pivoting: up to T = 511 by one wave per chain (segments per lane, cyclic
// reduction over the lanes for the segment boundaries; k_solve_lc_wave), beyond that by forward
// elimination and back substitution with one thread per chain (k_solve_lc), whose elimination
// coefficients go to a scratch buffer.
#include "common.h"

// (e-_k, e+_k) per coefficient of the m-major triangular layout
__global__ __launch_bounds__(kBlock) void k_lc_coefs(double2* __restrict__ lc, const int* __restrict__ n_of,
                                                     const int* __restrict__ m_of, int ncoef) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncoef) return;
    const double k = n_of[idx], m = m_of[idx];
    auto eps = [&](double n) { return n > m ? sqrt((n * n - m * m) / (4.0 * n * n - 1.0)) : 0.0; };
    const double em = k > 0.0 ? eps(k) * (k + 1.0) / k : 0.0;
    const double ep = eps(k + 1.0) * k / (k + 1.0);
    lc[idx] = make_double2(em, ep);
}

void launch_lc_coefs(double2* lc, const int* n_of, const int* m_of, int ncoef, hipStream_t st) {
    k_lc_coefs<<<(ncoef + kBlock - 1) / kBlock, kBlock, 0, st>>>(lc, n_of, m_of, ncoef);
}

namespace {

__device__ __forceinline__ double2 ld(const double* p) { return *(const double2*)p; }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 rmul(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 imul(double s, double2 a) { return make_double2(-s * a.y, s * a.x); }  // i s a
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cinv(double2 a) {
    const double r = 1.0 / (a.x * a.x + a.y * a.y);
    return make_double2(a.x * r, -a.y * r);
}

// f_I = L_g + L_c of the state u ([3][ncoef] complex) at degree k of order m (coefficient idx,
// first coefficient of the order at idx0); fields (Phi', zeta, delta).
struct FI {
    double2 phi, zeta, div;
};
__device__ __forceinline__ FI f_implicit_at(const double* __restrict__ u, size_t fs, int idx, int k, int m,
                                            int T, double2 e, double two_omega, double phibar, double cn) {
    const double2 z = ld(u + fs + 2 * (size_t)idx), d = ld(u + 2 * fs + 2 * (size_t)idx);
    const double2 p = ld(u + 2 * (size_t)idx);
    double2 zm = make_double2(0.0, 0.0), zp = zm, dm = zm, dp = zm;
    if (k > m) {
        zm = ld(u + fs + 2 * (size_t)(idx - 1));
        dm = ld(u + 2 * fs + 2 * (size_t)(idx - 1));
    }
    if (k < T) {
        zp = ld(u + fs + 2 * (size_t)(idx + 1));
        dp = ld(u + 2 * fs + 2 * (size_t)(idx + 1));
    }
    const double b = k > 0 ? two_omega * m / (k * (k + 1.0)) : 0.0;
    FI r;
    r.phi = rmul(-phibar, d);
    r.zeta = csub(imul(b, z), rmul(two_omega, cadd(rmul(e.x, dm), rmul(e.y, dp))));
    r.div = cadd(cadd(imul(b, d), rmul(cn, p)), rmul(two_omega, cadd(rmul(e.x, zm), rmul(e.y, zp))));
    return r;
}

}  // namespace

// Right-hand sides of the node update (Section 4.2, with f_I = L_g + L_c) for every coefficient,
// output node and member: beta_i = u_n + dt sum_j Q[i][j] (f_I(u_j) + E_j) - alpha_i f_I(u_i),
// written to the workspace the chain solve reads ([output state][3][ncoef]).  One thread per
// (coefficient, member) forms f_I(u_j) and reads E_j once for all its output nodes (M is a template
// parameter so that the per-node sums stay in registers); each beta_i is summed over j in order.
template <int M>
__global__ __launch_bounds__(kBlock) void k_lc_rhs(LcArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;                       // member
    if (idx >= a.ncoef) return;
    const int i0 = a.last_only ? M - 1 : 0;         // output nodes i0 .. M-1
    const int T = a.T;
    const size_t fs = (size_t)a.ncoef * 2;
    const int k = a.n_of[idx], m = a.m_of[idx];
    const double cn = k * (k + 1.0) * a.inv_a2;
    const double2 e = a.lc[idx];
    const int sdiv = a.sweep < M ? a.sweep : M;
    const double* un = a.un + (size_t)b * 3 * fs;
    const double2 u0p = ld(un + 2 * (size_t)idx), u0z = ld(un + fs + 2 * (size_t)idx),
                  u0d = ld(un + 2 * fs + 2 * (size_t)idx);
    double2 bphi[M], bzeta[M], bdiv[M];
    FI own[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        bphi[i] = u0p;
        bzeta[i] = u0z;
        bdiv[i] = u0d;
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double* uj = a.uprev + (size_t)b * a.uprev_member + (size_t)j * a.uprev_node;
        const double* ej = a.E + (size_t)b * a.E_member + (size_t)j * a.E_node;
        const FI fi = f_implicit_at(uj, fs, idx, k, m, T, e, a.two_omega, a.phibar, cn);
        const double2 sp = cadd(fi.phi, ld(ej + 2 * (size_t)idx));
        const double2 sz = cadd(fi.zeta, ld(ej + fs + 2 * (size_t)idx));
        const double2 sd = cadd(fi.div, ld(ej + 2 * fs + 2 * (size_t)idx));
        own[j] = fi;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (i < i0) continue;
            const double q = a.dt * a.Q[i * kMaxNodes + j];
            bphi[i] = cadd(bphi[i], rmul(q, sp));
            bzeta[i] = cadd(bzeta[i], rmul(q, sz));
            bdiv[i] = cadd(bdiv[i], rmul(q, sd));
        }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
        if (i < i0) continue;
        const double alpha = a.dt * a.tau[i] / sdiv;
        const int ostate = a.last_only ? b : b * M + i;
        double* out = a.beta_ws + (size_t)ostate * 3 * fs + 2 * (size_t)idx;
        *(double2*)out = csub(bphi[i], rmul(alpha, own[i].phi));
        *(double2*)(out + fs) = csub(bzeta[i], rmul(alpha, own[i].zeta));
        *(double2*)(out + 2 * fs) = csub(bdiv[i], rmul(alpha, own[i].div));
    }
}

// The chain solve of u - alpha f_I(u) = beta for one chain of one order of one output state:
// mode 0, beta from k_lc_rhs (node update of a sweep, output node i of member b); mode 1, beta
// given (imex_solve, member b; u may alias beta).  The elimination and the back substitution are
// the only serial dependences; the loads they need are issued several degrees ahead.
__global__ __launch_bounds__(64) void k_solve_lc(LcArgs a) {
    const int nodes = a.mode == 0 ? (a.last_only ? 1 : a.M) : 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int per_m = 2 * nodes * a.batch;
    if (t >= (a.T + 1) * per_m) return;
    const int m = t / per_m;
    int r = t - m * per_m;
    const int c = r / (nodes * a.batch);
    r -= c * nodes * a.batch;
    const int i = a.mode == 0 ? (a.last_only ? a.M - 1 : r / a.batch) : 0;   // output node
    const int b = r % a.batch;
    const int T = a.T;
    const size_t fs = (size_t)a.ncoef * 2;
    const int idx0 = coef_offset(T, m);
    const int J = T + 1 - m;
    const int sdiv = a.sweep < a.M ? a.sweep : a.M;
    const double alpha = a.mode == 0 ? a.dt * a.tau[i] / sdiv : a.alpha;
    const double two_omega = a.two_omega;
    const int ostate = a.mode == 0 ? (a.last_only ? b : b * a.M + i) : b;
    // scratch: 3 complex per (output state, chain, coefficient)
    double2* __restrict__ sc = a.scratch + ((size_t)ostate * 2 + c) * a.ncoef * 3;
    const double* __restrict__ be = (a.mode == 0 ? a.beta_ws + (size_t)ostate * 3 * fs
                                                 : a.beta + (size_t)b * 3 * fs);
    const double2* __restrict__ lc = a.lc;
    // the right-hand side this chain needs at position j: zeta at its zeta degrees, the combination
    // beta_delta + alpha c_k beta_Phi (Phi' eliminated) and beta_Phi at its delta degrees
    struct Pos {
        double2 r, bphi, e;
    };
    auto fetch = [&](int j) {
        Pos p;
        const int idx = idx0 + j;
        p.e = lc[idx];
        if (((j & 1) == c)) {
            p.r = ld(be + fs + 2 * (size_t)idx);
            p.bphi = make_double2(0.0, 0.0);
        } else {
            p.bphi = ld(be + 2 * (size_t)idx);
            p.r = ld(be + 2 * fs + 2 * (size_t)idx);          // beta_delta (combined below)
        }
        return p;
    };
    // The loads of a chain are independent of its elimination: they are requested kQ positions
    // ahead (two alternating register sets of kQ), so their latency overlaps kQ eliminations.
    constexpr int kQ = 8;
    double2 cp = make_double2(0.0, 0.0), dp = cp;
    Pos q0[kQ], q1[kQ];
#pragma unroll
    for (int u = 0; u < kQ; ++u) q0[u] = fetch(u < J ? u : J - 1);
    auto eliminate = [&](const Pos& cur, int j) {
        const int k = m + j, idx = idx0 + j;
        const double cn = k * (k + 1.0) * a.inv_a2;
        const double bk = k > 0 ? two_omega * m / (k * (k + 1.0)) : 0.0;
        double2 D, rr;
        double Lo, Up;
        if ((j & 1) == c) {
            D = make_double2(1.0, -alpha * bk);
            Lo = two_omega * alpha * cur.e.x;
            Up = two_omega * alpha * cur.e.y;
            rr = cur.r;
        } else {
            D = make_double2(1.0 + alpha * alpha * a.phibar * cn, -alpha * bk);
            Lo = -two_omega * alpha * cur.e.x;
            Up = -two_omega * alpha * cur.e.y;
            rr = cadd(cur.r, rmul(alpha * cn, cur.bphi));
        }
        if (j == J - 1) Up = 0.0;                       // degree T + 1 is truncated
        const double2 den = j == 0 ? D : csub(D, rmul(Lo, cp));
        const double2 inv = cinv(den);
        cp = rmul(Up, inv);
        dp = cmul(csub(rr, rmul(Lo, dp)), inv);
        sc[3 * (size_t)idx] = cp;
        sc[3 * (size_t)idx + 1] = dp;
        sc[3 * (size_t)idx + 2] = cur.bphi;
    };
    for (int j0 = 0; j0 < J; j0 += 2 * kQ) {
#pragma unroll
        for (int u = 0; u < kQ; ++u) {                 // next set while this one is eliminated
            const int jn = j0 + kQ + u;
            q1[u] = fetch(jn < J ? jn : J - 1);
        }
#pragma unroll
        for (int u = 0; u < kQ; ++u)
            if (j0 + u < J) eliminate(q0[u], j0 + u);
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const int jn = j0 + 2 * kQ + u;
            q0[u] = fetch(jn < J ? jn : J - 1);
        }
#pragma unroll
        for (int u = 0; u < kQ; ++u)
            if (j0 + kQ + u < J) eliminate(q1[u], j0 + kQ + u);
    }
    // back substitution and output
    double* __restrict__ out =
        a.uout + (size_t)b * a.out_member + (size_t)(a.mode == 0 && !a.last_only ? i : 0) * a.out_node;
    bool bad = false;
    double2 x = make_double2(0.0, 0.0);
    struct Back {
        double2 cp, dp, bphi;
    };
    auto fetch_back = [&](int j) {
        const size_t idx = (size_t)(idx0 + (j >= 0 ? j : 0));
        return Back{sc[3 * idx], sc[3 * idx + 1], sc[3 * idx + 2]};
    };
    auto substitute = [&](const Back& bb, int j) {
        const int idx = idx0 + j;
        x = csub(bb.dp, cmul(bb.cp, x));
        const bool zeta_pos = ((j & 1) == c);
        const double2 xv = x;
        if (zeta_pos) {
            *(double2*)(out + fs + 2 * (size_t)idx) = xv;
            bad = bad || !(isfinite(xv.x) && isfinite(xv.y));
        } else {
            const double2 phi = csub(bb.bphi, rmul(alpha * a.phibar, xv));
            *(double2*)(out + 2 * fs + 2 * (size_t)idx) = xv;
            *(double2*)(out + 2 * (size_t)idx) = phi;
            bad = bad || !(isfinite(xv.x) && isfinite(xv.y) && isfinite(phi.x) && isfinite(phi.y));
        }
    };
    Back b0[kQ], b1[kQ];
#pragma unroll
    for (int u = 0; u < kQ; ++u) b0[u] = fetch_back(J - 1 - u);
    for (int j0 = J - 1; j0 >= 0; j0 -= 2 * kQ) {
#pragma unroll
        for (int u = 0; u < kQ; ++u) b1[u] = fetch_back(j0 - kQ - u);
#pragma unroll
        for (int u = 0; u < kQ; ++u)
            if (j0 - u >= 0) substitute(b0[u], j0 - u);
#pragma unroll
        for (int u = 0; u < kQ; ++u) b0[u] = fetch_back(j0 - 2 * kQ - u);
#pragma unroll
        for (int u = 0; u < kQ; ++u)
            if (j0 - kQ - u >= 0) substitute(b1[u], j0 - kQ - u);
    }
    if (a.last_only && bad) a.flag[0] = 1;
}

// The same chain solve with one wave per chain (orders up to T = 511): the J = T + 1 - m
// positions are cut into 64 segments of L consecutive positions (L = 1, 2, 4 or 8, the chain
// padded with identity rows to 64 L), one segment per lane and held in registers.
//  1. Each lane eliminates its segment's interior (all positions but the last) with the two
//     boundary unknowns moved to the right-hand side: x_q = g_q + hl_q X_{p-1} + hr_q X_p, X_p the
//     last unknown of segment p (three right-hand sides, one Thomas sweep each way).
//  2. Substituting these into each segment's last equation leaves a tridiagonal system in the 64
//     X_p (the first interior representation of segment p + 1 comes from the next lane), solved
//     by parallel cyclic reduction over the lanes: six steps of combining each equation with the
//     ones h = 1, 2, 4, .., 32 lanes away (shuffles), after which every equation holds one unknown.
//  3. Every lane forms its interior values from X_{p-1} (the previous lane's) and X_p.
// The chains are diagonally dominant (see above), for which cyclic reduction and the segment
// eliminations need no pivoting; the result equals the sequential elimination's up to rounding.
namespace {

// v of lane - h (lane + h), zero where that lane is outside the wave; every lane must call these
__device__ __forceinline__ double2 shfl_up2(double2 v, int h, int lane) {
    const double2 r = make_double2(__shfl_up(v.x, h, 64), __shfl_up(v.y, h, 64));
    return lane >= h ? r : make_double2(0.0, 0.0);
}
__device__ __forceinline__ double2 shfl_down2(double2 v, int h, int lane) {
    const double2 r = make_double2(__shfl_down(v.x, h, 64), __shfl_down(v.y, h, 64));
    return lane + h < 64 ? r : make_double2(0.0, 0.0);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) { return cmul(a, cinv(b)); }

struct Row {
    double2 D, r, bphi;       // diagonal, right-hand side, beta_Phi (delta positions)
    double lo, up;            // sub- and super-diagonal
};

template <int L>
__device__ void solve_chain_wave(const LcArgs& a, int m, int c, int i, int b, double alpha, int lane) {
    const int T = a.T;
    const size_t fs = (size_t)a.ncoef * 2;
    const int idx0 = coef_offset(T, m);
    const int J = T + 1 - m;
    const double two_omega = a.two_omega;
    const int ostate = a.mode == 0 ? (a.last_only ? b : b * a.M + i) : b;
    const double* __restrict__ be = (a.mode == 0 ? a.beta_ws + (size_t)ostate * 3 * fs
                                                 : a.beta + (size_t)b * 3 * fs);
    // the equations of this lane's positions j = lane L + q (identity rows past the chain)
    Row e[L];
#pragma unroll
    for (int q = 0; q < L; ++q) {
        const int j = lane * L + q;
        Row w;
        if (j < J) {
            const int k = m + j, idx = idx0 + j;
            const double2 ee = a.lc[idx];
            const double cn = k * (k + 1.0) * a.inv_a2;
            const double bk = k > 0 ? two_omega * m / (k * (k + 1.0)) : 0.0;
            if ((j & 1) == c) {
                w.D = make_double2(1.0, -alpha * bk);
                w.lo = two_omega * alpha * ee.x;
                w.up = two_omega * alpha * ee.y;
                w.r = ld(be + fs + 2 * (size_t)idx);
                w.bphi = make_double2(0.0, 0.0);
            } else {
                w.D = make_double2(1.0 + alpha * alpha * a.phibar * cn, -alpha * bk);
                w.lo = -two_omega * alpha * ee.x;
                w.up = -two_omega * alpha * ee.y;
                w.bphi = ld(be + 2 * (size_t)idx);
                w.r = cadd(ld(be + 2 * fs + 2 * (size_t)idx), rmul(alpha * cn, w.bphi));
            }
            if (j == 0) w.lo = 0.0;                       // degree m - 1 does not exist
            if (j == J - 1) w.up = 0.0;                   // degree T + 1 is truncated
        } else {
            w.D = make_double2(1.0, 0.0);
            w.lo = 0.0;
            w.up = 0.0;
            w.r = make_double2(0.0, 0.0);
            w.bphi = w.r;
        }
        e[q] = w;
    }
    // 1. interior q = 0 .. L-2: x_q = g_q + hl_q X_{p-1} + hr_q X_p
    double2 g[L], hl[L], hr[L];
    if constexpr (L > 1) {
        double2 cp[L];
        double2 dg[L], dl[L], dr[L];
#pragma unroll
        for (int q = 0; q < L - 1; ++q) {
            const double2 rl = q == 0 ? make_double2(-e[0].lo, 0.0) : make_double2(0.0, 0.0);
            const double2 rrr = q == L - 2 ? make_double2(-e[L - 2].up, 0.0) : make_double2(0.0, 0.0);
            const double2 den = q == 0 ? e[0].D : csub(e[q].D, rmul(e[q].lo, cp[q - 1]));
            const double2 inv = cinv(den);
            cp[q] = q < L - 2 ? rmul(e[q].up, inv) : make_double2(0.0, 0.0);
            dg[q] = cmul(q == 0 ? e[0].r : csub(e[q].r, rmul(e[q].lo, dg[q - 1])), inv);
            dl[q] = cmul(q == 0 ? rl : csub(rl, rmul(e[q].lo, dl[q - 1])), inv);
            dr[q] = cmul(q == 0 ? rrr : csub(rrr, rmul(e[q].lo, dr[q - 1])), inv);
        }
        g[L - 2] = dg[L - 2];
        hl[L - 2] = dl[L - 2];
        hr[L - 2] = dr[L - 2];
#pragma unroll
        for (int q = L - 3; q >= 0; --q) {
            g[q] = csub(dg[q], cmul(cp[q], g[q + 1]));
            hl[q] = csub(dl[q], cmul(cp[q], hl[q + 1]));
            hr[q] = csub(dr[q], cmul(cp[q], hr[q + 1]));
        }
    }
    // 2. the reduced equation of X_p: A X_{p-1} + B X_p + C X_{p+1} = R
    const Row& last = e[L - 1];
    double2 A, B, C, R;
    if constexpr (L > 1) {
        A = rmul(last.lo, hl[L - 2]);
        B = cadd(last.D, rmul(last.lo, hr[L - 2]));
        R = csub(last.r, rmul(last.lo, g[L - 2]));
    } else {
        A = make_double2(last.lo, 0.0);
        B = last.D;
        R = last.r;
    }
    {
        // x at the next segment's first position: its interior representation (L > 1) or X_{p+1}
        double2 ng, nl, nr;
        if constexpr (L > 1) {
            ng = shfl_down2(g[0], 1, lane);
            nl = shfl_down2(hl[0], 1, lane);
            nr = shfl_down2(hr[0], 1, lane);
        } else {
            ng = make_double2(0.0, 0.0);
            nl = ng;
            nr = make_double2(1.0, 0.0);
        }
        B = cadd(B, rmul(last.up, nl));
        C = rmul(last.up, nr);
        R = csub(R, rmul(last.up, ng));
    }
#pragma unroll
    for (int h = 1; h < 64; h *= 2) {
        // every lane shuffles (a lane reading an inactive lane's register gets no defined value);
        // equations past either end of the chain act as identity rows
        const double2 Am = shfl_up2(A, h, lane), Cm = shfl_up2(C, h, lane), Rm = shfl_up2(R, h, lane);
        const double2 Ap = shfl_down2(A, h, lane), Cp = shfl_down2(C, h, lane), Rp = shfl_down2(R, h, lane);
        const double2 Bm0 = shfl_up2(B, h, lane), Bp0 = shfl_down2(B, h, lane);
        const double2 Bm = lane >= h ? Bm0 : make_double2(1.0, 0.0);
        const double2 Bp = lane + h < 64 ? Bp0 : make_double2(1.0, 0.0);
        const double2 k1 = cdiv(A, Bm), k2 = cdiv(C, Bp);
        A = make_double2(0.0, 0.0);
        A = csub(A, cmul(Am, k1));
        C = csub(make_double2(0.0, 0.0), cmul(Cp, k2));
        B = csub(csub(B, cmul(Cm, k1)), cmul(Ap, k2));
        R = csub(csub(R, cmul(Rm, k1)), cmul(Rp, k2));
    }
    const double2 X = cdiv(R, B);
    const double2 Xm = shfl_up2(X, 1, lane);             // X_{p-1} (0 for lane 0: its lo is 0)
    // 3. values and outputs
    double* __restrict__ out =
        a.uout + (size_t)b * a.out_member + (size_t)(a.mode == 0 && !a.last_only ? i : 0) * a.out_node;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < L; ++q) {
        const int j = lane * L + q;
        if (j >= J) continue;
        double2 xv;
        if constexpr (L > 1) {
            xv = q == L - 1 ? X : cadd(g[q], cadd(cmul(hl[q], Xm), cmul(hr[q], X)));
        } else {
            xv = X;
        }
        const int idx = idx0 + j;
        if ((j & 1) == c) {
            *(double2*)(out + fs + 2 * (size_t)idx) = xv;
            bad = bad || !(isfinite(xv.x) && isfinite(xv.y));
        } else {
            const double2 phi = csub(e[q].bphi, rmul(alpha * a.phibar, xv));
            *(double2*)(out + 2 * fs + 2 * (size_t)idx) = xv;
            *(double2*)(out + 2 * (size_t)idx) = phi;
            bad = bad || !(isfinite(xv.x) && isfinite(xv.y) && isfinite(phi.x) && isfinite(phi.y));
        }
    }
    if (a.last_only && bad) a.flag[0] = 1;
}

}  // namespace

constexpr int kLcWaves = 4;                       // chains (waves) per workgroup

// LMAX: the segment length the longest chain (m = 0) needs; shorter chains use shorter segments.
template <int LMAX>
__global__ __launch_bounds__(64 * kLcWaves) void k_solve_lc_wave(LcArgs a) {
    const int nodes = a.mode == 0 ? (a.last_only ? 1 : a.M) : 1;
    const int t = blockIdx.x * kLcWaves + (threadIdx.x >> 6);          // chain of this wave
    const int lane = threadIdx.x & 63;
    const int per_m = 2 * nodes * a.batch;
    if (t >= (a.T + 1) * per_m) return;                                // uniform per wave
    const int m = t / per_m;
    int r = t - m * per_m;
    const int c = r / (nodes * a.batch);
    r -= c * nodes * a.batch;
    const int i = a.mode == 0 ? (a.last_only ? a.M - 1 : r / a.batch) : 0;
    const int b = r % a.batch;
    const int sdiv = a.sweep < a.M ? a.sweep : a.M;
    const double alpha = a.mode == 0 ? a.dt * a.tau[i] / sdiv : a.alpha;
    const int J = a.T + 1 - m;
    if (J <= 64 || LMAX == 1) solve_chain_wave<1>(a, m, c, i, b, alpha, lane);
    else if (J <= 128 || LMAX == 2) solve_chain_wave<LMAX >= 2 ? 2 : 1>(a, m, c, i, b, alpha, lane);
    else if (J <= 256 || LMAX == 4) solve_chain_wave<LMAX >= 4 ? 4 : 1>(a, m, c, i, b, alpha, lane);
    else solve_chain_wave<LMAX>(a, m, c, i, b, alpha, lane);
}

void launch_solve_lc(const LcArgs& a, hipStream_t st) {
    const int nodes = a.mode == 0 ? (a.last_only ? 1 : a.M) : 1;
    if (a.mode == 0) {
        dim3 grid((a.ncoef + kBlock - 1) / kBlock, a.batch);
        switch (a.M) {
        case 1: k_lc_rhs<1><<<grid, kBlock, 0, st>>>(a); break;
        case 2: k_lc_rhs<2><<<grid, kBlock, 0, st>>>(a); break;
        case 3: k_lc_rhs<3><<<grid, kBlock, 0, st>>>(a); break;
        case 4: k_lc_rhs<4><<<grid, kBlock, 0, st>>>(a); break;
        case 5: k_lc_rhs<5><<<grid, kBlock, 0, st>>>(a); break;
        case 6: k_lc_rhs<6><<<grid, kBlock, 0, st>>>(a); break;
        case 7: k_lc_rhs<7><<<grid, kBlock, 0, st>>>(a); break;
        default: k_lc_rhs<8><<<grid, kBlock, 0, st>>>(a); break;
        }
    }
    const int n = (a.T + 1) * 2 * nodes * a.batch;
    const int wgs = (n + kLcWaves - 1) / kLcWaves;
    if (a.T + 1 <= 64) k_solve_lc_wave<1><<<wgs, 64 * kLcWaves, 0, st>>>(a);
    else if (a.T + 1 <= 128) k_solve_lc_wave<2><<<wgs, 64 * kLcWaves, 0, st>>>(a);
    else if (a.T + 1 <= 256) k_solve_lc_wave<4><<<wgs, 64 * kLcWaves, 0, st>>>(a);
    else if (a.T + 1 <= 512) k_solve_lc_wave<8><<<wgs, 64 * kLcWaves, 0, st>>>(a);
    else k_solve_lc<<<(n + 63) / 64, 64, 0, st>>>(a);
}

// f_I = L_g + L_c of `batch` states; fI must not alias u (the neighbours are read).
__global__ __launch_bounds__(kBlock) void k_implicit_lc(const double* __restrict__ u, double* __restrict__ fI,
                                                        const int* __restrict__ n_of,
                                                        const int* __restrict__ m_of,
                                                        const double2* __restrict__ lc, double phibar,
                                                        double inv_a2, double two_omega, int T, int ncoef) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (idx >= ncoef) return;
    const size_t fs = (size_t)ncoef * 2;
    const int k = n_of[idx], m = m_of[idx];
    const double cn = k * (k + 1.0) * inv_a2;
    const double* us = u + (size_t)b * 3 * fs;
    const FI r = f_implicit_at(us, fs, idx, k, m, T, lc[idx], two_omega, phibar, cn);
    double* o = fI + (size_t)b * 3 * fs + 2 * (size_t)idx;
    *(double2*)o = r.phi;
    *(double2*)(o + fs) = r.zeta;
    *(double2*)(o + 2 * fs) = r.div;
}

void launch_implicit_lc(const double* u, double* fI, const int* n_of, const int* m_of, const double2* lc,
                        double phibar, double inv_a2, double two_omega, int T, int batch, int ncoef,
                        hipStream_t st) {
    dim3 grid((ncoef + kBlock - 1) / kBlock, batch);
    k_implicit_lc<<<grid, kBlock, 0, st>>>(u, fI, n_of, m_of, lc, phibar, inv_a2, two_omega, T, ncoef);
}
