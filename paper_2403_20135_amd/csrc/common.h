// Internal definitions shared by the HIP sources of the dSDC library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/sdc.h"

// ---------------------------------------------------------------------------------------------
// Limits of this implementation
// ---------------------------------------------------------------------------------------------
constexpr int kMaxNodes = 8;        // collocation nodes per step
constexpr int kMaxSweeps = 16;
constexpr int kMaxFFTStages = 16;
constexpr int kBlock = 256;         // threads per workgroup for all kernels (4 wave64)

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------------------------
// FFT plan: nlon = 2^p or 3 * 2^p, factored into radices 3, 16, 8, 4, 2.
// ---------------------------------------------------------------------------------------------
struct FFTPlan {
    int n;
    int nst;
    int fchunk;                 // signals advanced together per pass (register budget)
    int radix[kMaxFFTStages];
};
// tasks (butterflies) a thread may stage per radix: bounds the registers of an FFT stage to about
// 24 complex values
__host__ __device__ constexpr int fft_task_cap(int R) { return R >= 16 ? 1 : 24 / R; }

// ---------------------------------------------------------------------------------------------
// Geometry of one truncation as the kernels see it.
//   nh  = nlat/2 northern latitudes; nhp = nh rounded up to a multiple of 16 (zero padded).
//   ms  = T+1 Fourier wavenumbers stored per latitude row.
//   Legendre tables (Pbar and H, same layout): for order m and parity p of n-m, rows
//   kk = 0..npk4(m,p)-1 (n = m + p + 2 kk, zero rows beyond npk), each row nhp latitudes,
//   block offset toff[2m+p] elements.
// ---------------------------------------------------------------------------------------------
struct Geom {
    int T, nlat, nlon, nh, nhp, ms, ncoef;
    int nrows;          // table rows summed over (m, parity): sum of npk4
    double radius;
};

__host__ __device__ inline int coef_offset(int T, int m) { return m * (2 * T + 3 - m) / 2; }
__host__ __device__ inline int npk_of(int T, int m, int p) { return (T - m + 2 - p) / 2; }
// Legendre table layout.  Per (m, parity) block: np4 = npk rounded up to 4 rows, nhp northern
// latitudes, stored tile-major (16-latitude tiles of np4 x 16 values, rows contiguous within a
// tile), so that a wave streaming one tile, or 16 rows of one tile, reads contiguous memory:
//   P[toff[2m + p] + tab_index(np4, kk, jh)].
__host__ __device__ inline size_t tab_index(int np4, int kk, int jh) {
    return (size_t)(jh >> 4) * np4 * 16 + (size_t)kk * 16 + (jh & 15);
}

// Workgroups of a launch are dealt to the 8 XCDs round-robin by their linear index, and each
// XCD starts its share in order.  A Legendre analysis launch over G state groups uses a 1-D grid
// of xcd_grid(ntasks, G) workgroups.  Task t always runs on XCD t % 8.  Interleaved, the G groups
// of a task run back to back on that XCD (the table tile they share comes from HBM once and from
// the XCD's L2 for the other groups); otherwise group-major (group g starts after every task of
// group g - 1 has been issued).  Tasks >= ntasks are padding (the kernel returns).
__host__ inline unsigned xcd_grid(int ntasks, int ngroups) {
    return (unsigned)((ntasks + 7) / 8) * 8u * (unsigned)ngroups;
}
__device__ inline int2 xcd_task_group(int w, int ntasks, int ngroups, int interleave) {
    if (!interleave) {
        const int npad = (ntasks + 7) / 8 * 8;
        return make_int2(w % npad, w / npad);
    }
    const int x = w & 7, l = w >> 3;
    return make_int2((l / ngroups) * 8 + x, l % ngroups);
}

// Launch variants of the Legendre kernels, chosen per handle (defaults or timed at run time):
// synthesis latitude tiles per workgroup and operand stages in flight per wave ((1, 8), (1, 4),
// (2, 4), (2, 2), (3, 2), (4, 2), (4, 1), (6, 1)), analysis table stages per wave (4 or 2) and
// state-group order.  The
// defaults are the variants measured fastest for one T255 member.
struct LegPlan {
    int syn_tiles = 2, syn_depth = 2, ana_depth = 2, ana_interleave = 1;
    int fuse_update = 1;       // node updates inside the analysis (M in {1, 2, 4})
    int syn_recur = 0;         // synthesis regenerates Pbar, H in registers instead of reading them
    int ana_recur = 0;         // analysis regenerates them from a quarter of the stored entries
    int node_launch = 0;       // 1: the f_E of the nodes of a sweep one node per launch (batch 1)
};

// Upward recurrence of the orthonormal associated Legendre functions in n at fixed m and mu (the
// three-term relation with eps_n = sqrt((n^2 - m^2) / (4 n^2 - 1))):
//   Pbar_{n+1} = a_n mu Pbar_n - b_n Pbar_{n-1},   a_n = 1 / eps_{n+1},  b_n = eps_n / eps_{n+1},
//   H_n = c_n Pbar_{n-1} - d_n Pbar_{n+1},          c_n = (n + 1) eps_n,  d_n = n eps_{n+1},
// started from Pbar_{m-1} = 0 and the sectoral Pbar_m^m.  The table generator and the synthesis
// that regenerates the tables evaluate it with these two functions and the same stored
// coefficients, so both produce the same values bit for bit.
// Coefficients: rc[4 rec_index(T, m, n) + {0, 1, 2, 3}] = (a_n, b_n, c_n, d_n) for
// n = m .. T + kRecPad - 1 (rows past T feed the padding rows of the last 4-row steps).
constexpr int kRecPad = 16;
__host__ __device__ inline size_t rec_index(int T, int m, int n) {
    return (size_t)m * (T + kRecPad) + (n - m);
}
__device__ __forceinline__ double leg_next(double mu, double p, double pm1, double a, double b) {
    return fma(a * mu, p, -(b * pm1));
}
__device__ __forceinline__ double leg_h(double pm1, double pp1, double c, double d) {
    return fma(c, pm1, -(d * pp1));
}

// Synthesis input ("coefficient-major", written by the update/prep kernels): for table row
// (m, p, kk) and state s, 8 doubles (zeta, Phi', psi, chi) x (Re, Im) with psi, chi the inverse
// Laplacians of zeta and delta:  cml[((rowoff[2m+p] + kk) * S + s) * 8 + v].
constexpr int kCmlVals = 8;
// Rows np..np4-1 of every (m, parity) block are padding; each producer of the layout zeroes them
// for the states it writes (the thread of the block's last real row does it), so that the
// synthesis contracts whole 4-row steps without masks.
__device__ inline void cml_clear_pad(double* cml, bool cml32, size_t row0, int kk, int np, size_t S,
                                     size_t s) {
    if (kk != np - 1) return;
    const int np4 = (np + 3) & ~3;
    for (int r = np; r < np4; ++r) {
        const size_t i = ((row0 + r) * S + s) * kCmlVals;
        if (cml32) {
            float4* c = reinterpret_cast<float4*>(reinterpret_cast<float*>(cml) + i);
            for (int k = 0; k < kCmlVals / 4; ++k) c[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            double2* c = reinterpret_cast<double2*>(cml + i);
            for (int k = 0; k < kCmlVals / 2; ++k) c[k] = make_double2(0.0, 0.0);
        }
    }
}
// In the FP32 precision mode the synthesis input is stored in FP32 (cml32): its MFMAs consume the
// values rounded to FP32 anyway, so storing them rounded changes no result and halves the bytes.
// Element i of the layout (in values):
__device__ inline void cml_put(double* cml, bool cml32, size_t i, double v) {
    if (cml32)
        reinterpret_cast<float*>(cml)[i] = (float)v;
    else
        cml[i] = v;
}
// Fourier fields produced by the synthesis for the grid kernel: zeta, Phi', U, V, layout
// four[s][field][lat][m].
constexpr int kSynFields = 4;
// Analysis input of the forward tendency, written by the grid kernel, per (northern latitude jh,
// m, state s): 10 complex values, the north + south ("s") and north - south ("a") sums of the
// Fourier coefficients of the five grid products, weighted as g A, g B, g C, g D
// (g = w / (a (1 - mu^2) nlon)) and w E / nlon, in the order
//   Es, Cs, Da, As, Bs, Aa, Ba, Ca, Ds, Ea
// so that the seven columns of each parity of n - m are one contiguous window: values 0..6 for
// even n - m (Pbar pairs with the symmetric sums, H with the antisymmetric ones), values 3..9 for
// odd.
// The factors -i m (A, C) and +i m (B) of the Pbar columns are applied to the contraction's
// results.  Stored rounded to FP32 in the FP32 and BF16x3 modes (what their MFMAs consume).  The
// latitude is outermost and the states of a latitude are adjacent, so the grid workgroups of one
// latitude pair write one contiguous slab:
//   G[fwd_index(T, S, jh, m, s) + 2 v + part]
constexpr int kFwdVals = 10;
enum FwdVal { kEs = 0, kCs, kDa, kAs, kBs, kAa, kBa, kCa, kDs, kEa };
__host__ __device__ inline size_t fwd_index(int T, int S, int jh, int m, int s) {
    return (((size_t)jh * (T + 1) + m) * S + s) * (2 * kFwdVals);
}
// Transposed synthesis of the adjoint, written by the adjoint grid kernel, per (northern latitude
// jh, m, parity p, state s):
// 14 values = 7 complex columns (Pbar parts then H parts), already combined into the north +-
// south sums of parity p and weighted,
// padded to kAnaStride values (written whole with zeros in the pad: one 128-byte line in FP64; in
// the FP32 precision mode the values are stored rounded to FP32, 64 bytes, since that mode's
// analysis MFMAs consume them rounded anyway).  The latitude is outermost, so a grid workgroup
// (one latitude pair, one state) writes whole rows into one contiguous slab and the states of a
// latitude complete each other's rows:
//   G[ana_index(T, S, jh, m, p, s) + c]
constexpr int kAnaVals = 14;
constexpr int kAnaStride = 16;
__host__ __device__ inline size_t ana_index(int T, int S, int jh, int m, int p, int s) {
    return ((((size_t)jh * (T + 1) + m) * 2 + p) * S + s) * kAnaStride;
}

// ---------------------------------------------------------------------------------------------
// Launchers (defined in the .hip files; all enqueue on `st`)
// ---------------------------------------------------------------------------------------------
// setup.hip
void launch_gauss(double* mu, double* w, int nlat, hipStream_t st);
// Recurrence coefficients (rec_index layout), then the tables and the sectoral values
// sect[m * nhp + jh] = Pbar_m^m(mu_jh) (zero on the padding latitudes jh >= nh).
void launch_rec_coefs(double* rc, const Geom& g, hipStream_t st);
void launch_legendre_tables(const double* mu, const double* rc, double* P, double* H, double* sect,
                            const long long* toff, const Geom& g, hipStream_t st);
void launch_collocation(double* tau, double* Q, int Mmax, hipStream_t st);
void launch_degree_tables(int* n_of, int* m_of, double* inv_lap, double* neg_lap, int T,
                          double radius, hipStream_t st);

// legendre.hip
// The Legendre tables of the SWE kernels: FP64, and FP32 copies when the handle computes its
// Legendre contractions in FP32 or in BF16x3 (P32 != nullptr selects them; bf3 the BF16x3
// products on the FP32 values).
enum TableType { kTabF64 = 0, kTabF32 = 1, kTabBf3 = 2 };
struct Tables {
    const double* P;
    const double* H;
    const float* P32;
    const float* H32;
    int bf3;
    const double* rc;        // recurrence coefficients and sectoral values for the synthesis
    const double* sect;      // that regenerates the tables (LegPlan::syn_recur)
    const double* mu;
    const double* inv_lap;   // -a^2 / (n (n + 1)) per degree (state-input synthesis)
};
// Synthesis tasks: (m, latitude tile) per workgroup, XCD-ordered; x < 0 = pad.
// state_in != null: the input columns are read from nstates states in the state layout (the
// forward synthesis of a step's first f_E) instead of cml.
void launch_synthesis_swe(const Tables& tb, const LegPlan& plan, const long long* toff,
                          const int* rowoff, const int2* tasks, int ntasks, const double* cml,
                          int nstates, double2* four, const Geom& g, hipStream_t st,
                          const double* state_in = nullptr);
// Analysis tasks: (m, p, first row, valid) per workgroup, XCD-ordered.
// With fuse != null the tendencies are not written: the kernel applies the node update `*fuse`
// to them (fuse_mode 1: the states are members, as in the step's first f_E; 2: the states are
// (member, node) pairs of M in {1, 2, 4} nodes per member).
struct UpdateArgs;
void launch_analysis_swe(const Tables& tb, const LegPlan& plan, const long long* toff,
                         const int4* tasks, int nwg, const double* G, int nstates,
                         const double* neg_lap, double* out, const Geom& g, hipStream_t st,
                         const UpdateArgs* fuse = nullptr, int fuse_mode = 0);
void launch_synthesis_scalar(const double* P, const long long* toff, const int2* tasks, int ntasks,
                             const double* spec, int nfields, double2* four, const Geom& g,
                             hipStream_t st);
// With fuse != null the accumulated adjoints are not stored: the kernel's epilogue applies
// *fuse (the adjoint node update of the group's members, or the final copy to lam_out).
struct AdjFuse;
void launch_analysis_adjoint(const Tables& tb, const LegPlan& plan, const long long* toff,
                             const int4* tasks, int nwg, const double* G, int nstates,
                             const double* inv_lap, double* out_acc, const Geom& g, hipStream_t st,
                             const AdjFuse* fuse = nullptr);
void launch_round_tables(const double* P, const double* H, float* P32, float* H32, long long n,
                         hipStream_t st);
void launch_analysis_scalar(const double* P, const long long* toff, const int4* tasks, int ntasks,
                            const double2* ana, int nfields, double* spec, const Geom& g,
                            hipStream_t st);

// grid.hip
// save (optional): grid values of zeta, Phi', U, V per [state][field][northern latitude][lon]
// as (north, south) pairs, kept for the adjoint.
void launch_grid_swe(const double2* four, double* G, bool g32, const double* mu, const double* w,
                     const double2* tw, const FFTPlan& plan, int nstates, double two_omega,
                     double2* save, const Geom& g, hipStream_t st);
void launch_grid_adj(const double2* four5, const double2* save, double* G, bool g32, const double* mu,
                     const double* w, const double2* tw, const FFTPlan& plan, int nstates,
                     double two_omega, const Geom& g, hipStream_t st);
hipError_t grid_set_lds_limit(int nlon, size_t bytes);
bool fft_length_supported(int nlon);
void launch_fft_inverse_scalar(const double2* four, double* grid, const double2* tw,
                               const FFTPlan& plan, int nfields, const Geom& g, hipStream_t st);
void launch_fft_forward_scalar(const double* grid, double2* ana, const double* w,
                               const double2* tw, const FFTPlan& plan, int nfields,
                               int transpose_synthesis, const Geom& g, hipStream_t st);

// update.hip
struct UpdateArgs {
    const double* un;          // [B][3][ncoef][2]
    const double* uprev;       // node iterates of the previous sweep
    long long uprev_node, uprev_member;   // strides in doubles (node stride 0 = all equal u_n)
    const double* E;           // explicit tendencies of the previous sweep
    long long E_node, E_member;
    double* uout;              // [B][M][3][ncoef][2], or the state itself when last_only
    long long out_node, out_member;
    const int* m_of;           // order m of every coefficient
    const int* rowoff;         // table row offset of (m, parity)
    const double* inv_lap;     // -a^2/(n(n+1)), 0 at n = 0
    const double* tau;         // [M] Radau-right nodes (device, FP64)
    const double* Q;           // [M][M] collocation matrix (device, FP64)
    const int* n_of;           // degree of every coefficient
    int* flag;                 // set to 1 on a non-finite output (last_only only)
    double dt, phibar, inv_a2;
    int M, sweep, last_only, batch, ncoef, T;
};
void launch_update(const UpdateArgs& a, hipStream_t st);
// Fills bytes (a multiple of 4) with all-ones words: NaN in FP64 and FP32 (read-before-write checks).
void launch_poison(void* p, size_t bytes, hipStream_t st);
// Sequential IMEX SDC (Algorithm 1): update of node m of a sweep.  Node arrays [node][B][3][ncoef].
struct SeqArgs {
    const double* un;          // u_n [B][3][ncoef][2]
    const double* uold;        // nodes of the previous sweep; node stride uold_node (0: all u_n)
    const double* eold;        // their explicit tendencies; node stride eold_node (0: all E_0)
    long long uold_node, eold_node;
    const double* unew;        // nodes j < m of this sweep (node stride B * 3 * ncoef * 2)
    const double* enew;
    double* out;               // u_m of this sweep, or the state on the step's last update
    double* cml;               // synthesis layout of out (S = B), or null on the last update
    int cml32;
    const int* n_of;
    const int* m_of;
    const int* rowoff;
    const double* inv_lap;
    const double* tau;         // [M] nodes
    const double* Q;           // [M][kMaxNodes] collocation matrix rows
    int* flag;                 // non-finite output of the last update
    double dt, phibar, inv_a2;
    int M, m, batch, ncoef, T;
};
void launch_update_seq(const SeqArgs& a, hipStream_t st);
// imex2.hip: the coefficient-wise phases of an IMEX-o2 step for `batch` states [b][3][ncoef]
//   kImex2First:   out = C(dt/2) in (u*), and its synthesis layout in cml
//   kImex2Predict: synthesis layout of in + dt k1 (in = u*)
//   kImex2Last:    out = C(dt/2)(in + dt/2 (k1 + k2)), flag set on a non-finite value
constexpr int kImex2First = 0, kImex2Predict = 1, kImex2Last = 2;
struct Imex2Args {
    const double* in;
    const double* k1;
    const double* k2;
    double* out;
    double* cml;
    int cml32;
    const int* n_of;
    const int* m_of;
    const int* rowoff;
    const double* inv_lap;
    int* flag;
    double dt, phibar, inv_a2;
    int phase, batch, ncoef, T;
};
void launch_imex2(const Imex2Args& a, hipStream_t st);
void launch_implicit(const double* u, double* fI, const int* n_of, double phibar, double inv_a2,
                     int batch, int ncoef, hipStream_t st);
void launch_solve(double alpha, const double* beta, double* u, const int* n_of, double phibar,
                  double inv_a2, int batch, int ncoef, hipStream_t st);

// coriolis.hip: the split with the linear Coriolis term implicit (f_I = L_g + L_c)
struct LcArgs {
    int mode;                    // 0: node update of a sweep, 1: u = solve(alpha, beta)
    const double* un;            // mode 0: [B][3][ncoef]
    const double* uprev;         // mode 0: node iterates of the previous sweep (strides as UpdateArgs)
    long long uprev_node, uprev_member;
    const double* E;             // mode 0: f_E = N_a + N_r of the previous sweep's nodes
    long long E_node, E_member;
    double* uout;                // output states (mode 0: nodes, or the state when last_only)
    long long out_node, out_member;
    const double* beta;          // mode 1: [B][3][ncoef] (u may alias it)
    double alpha;                // mode 1
    double* beta_ws;             // mode 0: right-hand sides [output state][3][ncoef] (workspace)
    const int* n_of;             // mode 0: degree and order of every coefficient
    const int* m_of;
    const double* tau;
    const double* Q;
    const int* rowoff;
    const double* inv_lap;
    const double2* lc;           // (e-_k, e+_k) per coefficient
    double2* scratch;            // 3 complex per (output state, chain, coefficient)
    int* flag;
    double dt, phibar, inv_a2, two_omega;
    int M, batch, ncoef, T, sweep, last_only;
};
void launch_lc_coefs(double2* lc, const int* n_of, const int* m_of, int ncoef, hipStream_t st);
void launch_solve_lc(const LcArgs& a, hipStream_t st);
void launch_implicit_lc(const double* u, double* fI, const int* n_of, const int* m_of, const double2* lc,
                        double phibar, double inv_a2, double two_omega, int T, int batch, int ncoef,
                        hipStream_t st);

// Launches over several handles (members of different truncations) at once, one workgroup range
// per handle: the arguments of each handle's launch, the first workgroup of its range (a multiple
// of 8: XCD order kept) and its workgroup count.
struct SynArgs {
    const void* P;
    const void* H;
    const long long* toff;
    const int* rowoff;
    const int2* tasks;
    const void* cml;             // in the table type
    int nstates;
    double* four;
    Geom g;
    const double* rc;
    const double* sect;
    const double* mu;
    const double* sin_state;
    const double* inv_lap;
    int gx;                      // workgroups per state group (the task list's length)
    int first, blocks;
};
SynArgs make_syn_args(const Tables& tb, const long long* toff, const int* rowoff, const int2* tasks,
                      int ntasks, const double* cml, int nstates, double* four, const Geom& g,
                      const double* state_in);
void launch_synthesis_multi(const LegPlan& plan, int tt, bool state_in, const SynArgs* list, int n,
                            int blocks, hipStream_t st);
struct AnaArgs {
    const void* P;
    const void* H;
    const long long* toff;
    const int4* tasks;
    int ntasks, interleave;
    const void* G;               // in the table type
    int nstates;
    const double* nscale;
    double* out;
    Geom g;
    UpdateArgs fu;
    int fuse;
    const double* P64;
    const double* rc;
    const double* mu;
    int first, blocks;
};
AnaArgs make_ana_args(const Tables& tb, const LegPlan& plan, const long long* toff, const int4* tasks,
                      int nwg, const double* G, int nstates, const double* neg_lap, double* out,
                      const Geom& g, const UpdateArgs* fuse, int fuse_mode);
void launch_analysis_multi(const LegPlan& plan, int tt, const AnaArgs* list, int n, int blocks,
                           hipStream_t st);
struct GridArgs {
    const double2* four;
    double* G;                   // in the table type
    const double* mu;
    const double* w;
    const double2* tw;
    double two_omega;
    int nstates;
    double2* save;
    Geom g;
    int first, blocks;
};
GridArgs make_grid_args(const double2* four, double* G, const double* mu, const double* w, const double2* tw,
                        int nstates, double two_omega, double2* save, const Geom& g);
bool grid_multi_supported(int nlon);
void launch_grid_multi(bool g32, int nlon_max, const GridArgs* list, int n, int blocks, hipStream_t st);
struct UpdArgsM {
    UpdateArgs a;
    int gx, first, blocks;
};
void launch_update_multi(int M, const UpdArgsM* list, int n, int blocks, hipStream_t st);

// adjoint.hip
void launch_prep_cml_adj(const double* ebar, int nstates, double* cml, bool cml32, const int* n_of,
                         const int* m_of,
                         const int* rowoff, const double* neg_lap, int ncoef, int T, hipStream_t st);
void launch_synthesis_adj(const Tables& tb, const LegPlan& plan, const long long* toff,
                          const int* rowoff, const int2* tasks, int ntasks, const double* cml,
                          int nstates, double2* four5, const Geom& g, hipStream_t st);
struct AdjUpdateArgs {
    const double* ubar;          // [B][M][3][ncoef] adjoint of this sweep's nodes (or lam: [B][3][ncoef])
    long long ubar_node, ubar_member;
    double* ubar_prev;           // [B][M][3][ncoef] (written unless first_stage)
    double* ebar_prev;           // [B][M][3][ncoef] or E_0 adjoint [B][3][ncoef] when first_stage
    double* ubar_n;              // [B][3][ncoef]
    const double* tau;
    const double* Q;
    const int* n_of;
    double dt, phibar, inv_a2;
    int M, sweep, last, first_stage, init_un, batch, ncoef;
    // when cml is set the E adjoints are written in the synthesis-adjoint input layout instead
    // of ebar_prev (the transposed analysis' fused epilogue)
    double* cml;
    int cml32, T;
    const int* m_of;
    const int* rowoff;
    const double* neg_lap;
};
// Fused epilogue of the transposed analysis: mode 1 applies the adjoint node update `a` to the
// accumulated adjoints of the group's members (states b M + j); mode 2 (the step's first stage,
// states = members) writes the finished u_n adjoint to lam_out with the m = 0 imaginary parts
// set to zero.
struct AdjFuse {
    AdjUpdateArgs a;
    double* lam_out;
    const int* m_of;
    int mode;
};

void launch_update_adj(const AdjUpdateArgs& a, hipStream_t st);
void launch_finish_adj(const double* src, double* dst, const int* m_of, int ncoef, int nstates,
                       hipStream_t st);
