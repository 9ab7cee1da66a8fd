// Coefficient-wise kernels of the step: the Q-matrix node integral fused with the per-degree
// implicit solve (node update of Section 4.2), f_I = L_g, and the solver of u - alpha f_I(u) = beta.
// All are HBM-bound streams over the coefficients; one thread per (member, coefficient).
//
// Gravity-wave operator per coefficient (c_n = n(n+1)/a^2, Phi_bar = g H):
//   L_g(Phi', zeta, delta) = (-Phi_bar delta, 0, c_n Phi')
// Solve of u - alpha L_g(u) = beta:
//   Phi' = (beta_Phi - alpha Phi_bar beta_delta) / (1 + alpha^2 Phi_bar c_n),
//   zeta = beta_zeta, delta = beta_delta + alpha c_n Phi'.
#include "node_update.h"

struct C3 {
    double2 phi, zeta, div;
};

__device__ __forceinline__ double2 ld2(const double* p) { return *(const double2*)p; }
__device__ __forceinline__ void st2(double* p, double2 v) { *(double2*)p = v; }

// One thread per (coefficient, part): every coefficient of the update is real, so the Re and Im
// parts are independent (twice the waves of a thread per coefficient for the same bytes).  The node
// count is a template parameter so that the per-node arrays live in registers.
template <int M>
__device__ __forceinline__ void update_body(const UpdateArgs& a, int bx, int by) {
    const int t = bx * blockDim.x + threadIdx.x;
    const int b = by;
    if (t >= 2 * a.ncoef) return;
    const size_t fs = (size_t)a.ncoef * 2;
    const double* e = a.E + (size_t)b * a.E_member + (size_t)t;
    node_update_part<M>(a, t >> 1, t & 1, b,
                        [&](int j, int f) { return e[(size_t)j * a.E_node + f * fs]; });
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_update(UpdateArgs a) {
    update_body<M>(a, blockIdx.x, blockIdx.y);
}

// One update launch over several handles (workgroup ranges as the multi-handle Legendre kernels).
template <int M>
__global__ __launch_bounds__(kBlock) void k_update_multi(const UpdArgsM* __restrict__ list, int n) {
    const int b = blockIdx.x;
    int h = 0;
    while (h + 1 < n && b >= list[h + 1].first) ++h;
    const UpdArgsM& u = list[h];
    const int local = b - u.first;
    if (local >= u.blocks) return;                           // padding to the next range (uniform)
    update_body<M>(u.a, local % u.gx, local / u.gx);
}

constexpr int kUpd = 64;           // small workgroups: the (coefficient, part) threads over all CUs

void launch_update_multi(int M, const UpdArgsM* list, int n, int blocks, hipStream_t st) {
    switch (M) {
    case 1: k_update_multi<1><<<blocks, kUpd, 0, st>>>(list, n); break;
    case 2: k_update_multi<2><<<blocks, kUpd, 0, st>>>(list, n); break;
    case 3: k_update_multi<3><<<blocks, kUpd, 0, st>>>(list, n); break;
    case 4: k_update_multi<4><<<blocks, kUpd, 0, st>>>(list, n); break;
    case 5: k_update_multi<5><<<blocks, kUpd, 0, st>>>(list, n); break;
    case 6: k_update_multi<6><<<blocks, kUpd, 0, st>>>(list, n); break;
    case 7: k_update_multi<7><<<blocks, kUpd, 0, st>>>(list, n); break;
    default: k_update_multi<8><<<blocks, kUpd, 0, st>>>(list, n); break;
    }
}

void launch_update(const UpdateArgs& a, hipStream_t st) {
    dim3 grid((2 * a.ncoef + kUpd - 1) / kUpd, a.batch);
    switch (a.M) {
    case 1: k_update<1><<<grid, kUpd, 0, st>>>(a); break;
    case 2: k_update<2><<<grid, kUpd, 0, st>>>(a); break;
    case 3: k_update<3><<<grid, kUpd, 0, st>>>(a); break;
    case 4: k_update<4><<<grid, kUpd, 0, st>>>(a); break;
    case 5: k_update<5><<<grid, kUpd, 0, st>>>(a); break;
    case 6: k_update<6><<<grid, kUpd, 0, st>>>(a); break;
    case 7: k_update<7><<<grid, kUpd, 0, st>>>(a); break;
    default: k_update<8><<<grid, kUpd, 0, st>>>(a); break;
    }
}

__global__ __launch_bounds__(kBlock) void k_implicit(const double* __restrict__ u, double* __restrict__ fI,
                                                     const int* __restrict__ n_of, double phibar,
                                                     double inv_a2, int ncoef) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (idx >= ncoef) return;
    const double cn = n_of[idx] * (n_of[idx] + 1.0) * inv_a2;
    const size_t fs = (size_t)ncoef * 2;
    const double* ub = u + (size_t)b * 3 * fs + (size_t)idx * 2;
    double* ob = fI + (size_t)b * 3 * fs + (size_t)idx * 2;
    const double2 p = ld2(ub), d = ld2(ub + 2 * fs);
    st2(ob, make_double2(-phibar * d.x, -phibar * d.y));
    st2(ob + fs, make_double2(0.0, 0.0));
    st2(ob + 2 * fs, make_double2(cn * p.x, cn * p.y));
}

void launch_implicit(const double* u, double* fI, const int* n_of, double phibar, double inv_a2,
                     int batch, int ncoef, hipStream_t st) {
    dim3 grid((ncoef + kBlock - 1) / kBlock, batch);
    k_implicit<<<grid, kBlock, 0, st>>>(u, fI, n_of, phibar, inv_a2, ncoef);
}

__global__ __launch_bounds__(kBlock) void k_solve(double alpha, const double* beta, double* u,
                                                  const int* __restrict__ n_of, double phibar,
                                                  double inv_a2, int ncoef) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (idx >= ncoef) return;
    const double cn = n_of[idx] * (n_of[idx] + 1.0) * inv_a2;
    const size_t fs = (size_t)ncoef * 2;
    const double* bb = beta + (size_t)b * 3 * fs + (size_t)idx * 2;
    double* ub = u + (size_t)b * 3 * fs + (size_t)idx * 2;
    const double2 bp = ld2(bb), bz = ld2(bb + fs), bd = ld2(bb + 2 * fs);
    const double den = 1.0 / (1.0 + alpha * alpha * phibar * cn);
    const double2 p = make_double2((bp.x - alpha * phibar * bd.x) * den, (bp.y - alpha * phibar * bd.y) * den);
    st2(ub, p);
    st2(ub + fs, bz);
    st2(ub + 2 * fs, make_double2(bd.x + alpha * cn * p.x, bd.y + alpha * cn * p.y));
}

void launch_solve(double alpha, const double* beta, double* u, const int* n_of, double phibar,
                  double inv_a2, int batch, int ncoef, hipStream_t st) {
    dim3 grid((ncoef + kBlock - 1) / kBlock, batch);
    k_solve<<<grid, kBlock, 0, st>>>(alpha, beta, u, n_of, phibar, inv_a2, ncoef);
}

// Node update of the sequential IMEX SDC of Algorithm 1 (Section 4.1) for node m of a sweep, one
// thread per (coefficient, Re/Im part, member):
//   beta = u_n + dt sum_j q_mj (L_g(u_j^k) + E_j^k)
//        + dt sum_{j<m} [dtau_{j+1} (E_j^{k+1} - E_j^k) + dtau_j (L_g(u_j^{k+1}) - L_g(u_j^k))]
//        - dt dtau_m L_g(u_m^k),
//   u_m^{k+1} = solve(dt dtau_m, beta),  dtau_1 = tau_1, dtau_j = tau_j - tau_{j-1}.
// Node arrays are node-major [node][member][3][ncoef] so that the f_E launch of one node reads
// and writes its members contiguously.
template <int M>
__global__ __launch_bounds__(kBlock) void k_update_seq(SeqArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= 2 * a.ncoef) return;
    const int idx = t >> 1, c = t & 1;
    const int n = a.n_of[idx];
    const double cn = n * (n + 1.0) * a.inv_a2;
    const size_t fs = (size_t)a.ncoef * 2;
    const size_t o = (size_t)b * 3 * fs + (size_t)t;           // member b, field 0 of a state
    const size_t nsn = (size_t)a.batch * 3 * fs;                // node stride of the new sweep
    const int m = a.m;
    double sp = 0.0, sz = 0.0, sd = 0.0;                          // the beta terms, per field
    double Lp_m = 0.0, Ld_m = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double* uo = a.uold + (size_t)j * a.uold_node + o;
        const double* eo = a.eold + (size_t)j * a.eold_node + o;
        const double Lp = -a.phibar * uo[2 * fs], Ld = cn * uo[0];   // L_g(u_j^k)
        const double Ep = eo[0], Ez = eo[fs], Ed = eo[2 * fs];
        const double q = a.Q[m * kMaxNodes + j];
        sp += q * (Lp + Ep);
        sz += q * Ez;
        sd += q * (Ld + Ed);
        if (j < m) {
            const double dj = a.tau[j] - (j > 0 ? a.tau[j - 1] : 0.0);
            const double dj1 = a.tau[j + 1] - a.tau[j];
            const double* un = a.unew + (size_t)j * nsn + o;
            const double* en = a.enew + (size_t)j * nsn + o;
            sp += dj1 * (en[0] - Ep) + dj * (-a.phibar * un[2 * fs] - Lp);
            sz += dj1 * (en[fs] - Ez);
            sd += dj1 * (en[2 * fs] - Ed) + dj * (cn * un[0] - Ld);
        }
        if (j == m) {
            Lp_m = Lp;
            Ld_m = Ld;
        }
    }
    const double dm = a.tau[m] - (m > 0 ? a.tau[m - 1] : 0.0);
    const double alpha = a.dt * dm;
    const double* un0 = a.un + o;
    const double bphi = un0[0] + a.dt * sp - alpha * Lp_m;
    const double bzeta = un0[fs] + a.dt * sz;
    const double bdiv = un0[2 * fs] + a.dt * sd - alpha * Ld_m;
    const double phi = (bphi - alpha * a.phibar * bdiv) / (1.0 + alpha * alpha * a.phibar * cn);
    const double dv = bdiv + alpha * cn * phi;
    double* out = a.out + o;
    out[0] = phi;
    out[fs] = bzeta;
    out[2 * fs] = dv;
    if (a.cml) {
        const int mo = a.m_of[idx], par = (n - mo) & 1, kk = (n - mo) >> 1;
        const double il = a.inv_lap[n];
        const size_t ci = (((size_t)a.rowoff[2 * mo + par] + kk) * a.batch + b) * kCmlVals + c;
        cml_put(a.cml, a.cml32, ci, bzeta);
        cml_put(a.cml, a.cml32, ci + 2, phi);
        cml_put(a.cml, a.cml32, ci + 4, il * bzeta);
        cml_put(a.cml, a.cml32, ci + 6, il * dv);
        if (c == 0)
            cml_clear_pad(a.cml, a.cml32, a.rowoff[2 * mo + par], kk, npk_of(a.T, mo, par), a.batch, b);
    } else if (!(isfinite(phi) && isfinite(bzeta) && isfinite(dv))) {
        a.flag[0] = 1;
    }
}

void launch_update_seq(const SeqArgs& a, hipStream_t st) {
    dim3 grid((2 * a.ncoef + kBlock - 1) / kBlock, a.batch);
    switch (a.M) {
    case 1: k_update_seq<1><<<grid, kBlock, 0, st>>>(a); break;
    case 2: k_update_seq<2><<<grid, kBlock, 0, st>>>(a); break;
    case 3: k_update_seq<3><<<grid, kBlock, 0, st>>>(a); break;
    case 4: k_update_seq<4><<<grid, kBlock, 0, st>>>(a); break;
    case 5: k_update_seq<5><<<grid, kBlock, 0, st>>>(a); break;
    case 6: k_update_seq<6><<<grid, kBlock, 0, st>>>(a); break;
    case 7: k_update_seq<7><<<grid, kBlock, 0, st>>>(a); break;
    default: k_update_seq<8><<<grid, kBlock, 0, st>>>(a); break;
    }
}

// NaN fill (all bits set: NaN in FP64 and FP32) of n 32-bit words, for read-before-write checks.
__global__ __launch_bounds__(kBlock) void k_poison(unsigned* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        p[i] = 0xFFFFFFFFu;
}

void launch_poison(void* p, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 4;
    if (n == 0) return;
    const unsigned blocks = (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
    k_poison<<<blocks, kBlock, 0, st>>>(static_cast<unsigned*>(p), n);
}
