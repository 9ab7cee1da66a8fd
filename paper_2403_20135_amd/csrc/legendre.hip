// Legendre transforms as FP64 MFMA contractions (gfx950, v_mfma_f64_16x16x4).
//
// For every zonal wavenumber m the Legendre part of the spherical-harmonic transform is a
// small dense product between a table (latitudes x degrees n) and a few coefficient columns.
// Equatorial symmetry, Pbar_n^m(-mu) = (-1)^{n+m} Pbar_n^m(mu) and H_n^m(-mu) = -(-1)^{n+m}
// H_n^m(mu), halves both the table and the flops: the tables hold the northern latitudes only,
// split by the parity of n-m, and the southern values follow from even +- odd sums.
//
// MFMA operand layout (64 lanes, lane l, i = l % 16, q = l / 16):
//   A[i][q] (16x4), B[q][i] (4x16); the FP64 accumulator of lane l holds D[4r + q][i], r = 0..3
//   (rows interleaved across the four lane groups).
#include "common.h"

constexpr int kAnaForward = 0, kAnaAdjoint = 1;

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------------------------
// Synthesis for the shallow-water explicit tendency.  Per state the inputs are the spectral
// fields in the coefficient-major layout (zeta, Phi', psi, chi), psi = -a^2 zeta/(n(n+1)),
// chi = -a^2 delta/(n(n+1)); the outputs are the Fourier coefficients, at every latitude, of
//   zeta, Phi', U = (1/a) sum_n [i m chi Pbar - psi H], V = (1/a) sum_n [i m psi Pbar + chi H].
// Columns of one 16-wide Pbar tile: 2 states x (zeta, Phi', psi, chi) x (Re, Im); of the H tile:
// 4 states x (psi, chi) x (Re, Im).  A workgroup owns (m, one 16-latitude tile, 4 states); its 4
// waves take every fourth 4-row step of the degree loop (both parities), so the longest chain
// (m = 0) is a quarter of the degrees, and the partial tiles are summed in LDS in a fixed order.
// ---------------------------------------------------------------------------------------------
constexpr int kSynAcc = 24;      // doubles per lane: Pbar 2 parities x 2 tiles x 4, H 2 parities x 4

__global__ __launch_bounds__(kBlock) void k_synthesis_swe(
    const double* __restrict__ P, const double* __restrict__ H, const long long* __restrict__ toff,
    const int* __restrict__ rowoff, const int2* __restrict__ tasks, const double* __restrict__ cml,
    int nstates, double2* __restrict__ four, Geom g) {
    // partial accumulators [wave][value][lane]; then (aliased) the parity-combined tile
    // red[state][north/south][value][latitude]
    __shared__ double lds[4 * kSynAcc * 64];
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0) return;                          // padding workgroup (uniform)
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m = task.x, jt = task.y;
    const int S = nstates;
    const int s0 = blockIdx.y * 4;
    const int i = lane & 15, q = lane >> 4;
    const int vP = i & 7, vH = i & 3;

    v4d acc[6];                                       // [p*3 + {Pbar tile 0, Pbar tile 1, H}]
    for (int k = 0; k < 6; ++k) acc[k] = (v4d){0.0, 0.0, 0.0, 0.0};
    {
        // column -> state; out-of-range states read a valid address and are zeroed by a select
        const int sP0 = s0 + (i >> 3), sP1 = s0 + 2 + (i >> 3), sH = s0 + (i >> 2);
        const bool ok0 = sP0 < S, ok1 = sP1 < S, okh = sH < S;
        const int c0off = (ok0 ? sP0 : 0) * kCmlVals + vP;
        const int c1off = (ok1 ? sP1 : 0) * kCmlVals + vP;
        const int choff = (okh ? sH : 0) * kCmlVals + 4 + vH;
        for (int p = 0; p < 2; ++p) {
            const int np = npk_of(g.T, m, p);
            const int np4 = (np + 3) & ~3;
            // this wave takes the 4-row steps 4*wave, 4*wave + 16, ... of parity p
            const int steps = np4 > 4 * wave ? (np4 - 4 * wave + 15) / 16 : 0;   // uniform
            const double* Pp = P + toff[2 * m + p] + jt * 16 + i + (size_t)(4 * wave + q) * g.nhp;
            const double* Hp = H + toff[2 * m + p] + jt * 16 + i + (size_t)(4 * wave + q) * g.nhp;
            const double* Bp = cml + ((size_t)rowoff[2 * m + p] + 4 * wave + q) * S * kCmlVals;
            const size_t tstep = (size_t)16 * g.nhp, bstep = (size_t)16 * S * kCmlVals;
            v4d c0 = acc[p * 3], c1 = acc[p * 3 + 1], ch = acc[p * 3 + 2];
            int kk = 4 * wave + q;
#pragma unroll 2
            for (int it = 0; it < steps; ++it) {
                const bool vn = kk < np;
                const double ap = Pp[0], ah = Hp[0];
                const double b0 = Bp[c0off], b1 = Bp[c1off], bh = Bp[choff];
                c0 = mfma_f64(ap, (vn && ok0) ? b0 : 0.0, c0);
                c1 = mfma_f64(ap, (vn && ok1) ? b1 : 0.0, c1);
                ch = mfma_f64(ah, (vn && okh) ? bh : 0.0, ch);
                Pp += tstep;
                Hp += tstep;
                Bp += bstep;
                kk += 16;
            }
            acc[p * 3] = c0;
            acc[p * 3 + 1] = c1;
            acc[p * 3 + 2] = ch;
        }
    }
    for (int k = 0; k < 6; ++k)
        for (int r = 0; r < 4; ++r) lds[(wave * kSynAcc + k * 4 + r) * 64 + lane] = acc[k][r];
    __syncthreads();
    double* red = lds;                                // [sl][ns][12][16], written by wave 0 only
    if (wave == 0) {
        double tot[kSynAcc];
        for (int v = 0; v < kSynAcc; ++v) {
            double sum = lds[v * 64 + lane];
            for (int w = 1; w < 4; ++w) sum += lds[(w * kSynAcc + v) * 64 + lane];
            tot[v] = sum;
        }
        // north = even + odd; south = even - odd (Pbar) and odd - even (H)
        for (int r = 0; r < 4; ++r) {
            const int latl = 4 * r + q;
            for (int t = 0; t < 2; ++t) {
                const double e = tot[t * 4 + r], o = tot[12 + t * 4 + r];
                const int sl = 2 * t + (i >> 3);
                red[((sl * 2 + 0) * 12 + vP) * 16 + latl] = e + o;
                red[((sl * 2 + 1) * 12 + vP) * 16 + latl] = e - o;
            }
            const double e = tot[8 + r], o = tot[20 + r];
            red[(((i >> 2) * 2 + 0) * 12 + 8 + vH) * 16 + latl] = e + o;
            red[(((i >> 2) * 2 + 1) * 12 + 8 + vH) * 16 + latl] = o - e;
        }
    }
    __syncthreads();
    const int it = threadIdx.x;                       // (state, north/south, latitude): 128 items
    if (it >= 128) return;
    const int sl = it >> 5, ns = (it >> 4) & 1, latl = it & 15;
    const int s = s0 + sl, jh = jt * 16 + latl;
    if (s >= S || jh >= g.nh) return;
    const double inva = 1.0 / g.radius;
    const double mm = (double)m;
    const double* v = red + ((sl * 2 + ns) * 12) * 16 + latl;
    const double ppr = v[4 * 16], ppi = v[5 * 16];    // Pbar psi
    const double pcr = v[6 * 16], pci = v[7 * 16];    // Pbar chi
    const double hpr = v[8 * 16], hpi = v[9 * 16];    // H psi
    const double hcr = v[10 * 16], hci = v[11 * 16];  // H chi
    const int j = ns ? g.nlat - 1 - jh : jh;
    const size_t fstride = (size_t)g.nlat * g.ms;
    double2* base = four + (size_t)s * kSynFields * fstride + (size_t)j * g.ms + m;
    base[0] = make_double2(v[0 * 16], v[1 * 16]);
    base[fstride] = make_double2(v[2 * 16], v[3 * 16]);
    base[2 * fstride] = make_double2((-mm * pci - hpr) * inva, (mm * pcr - hpi) * inva);
    base[3 * fstride] = make_double2((-mm * ppi + hcr) * inva, (mm * ppr + hci) * inva);
}

void launch_synthesis_swe(const double* P, const double* H, const long long* toff,
                          const int* rowoff, const int2* tasks, int ntasks, const double* cml,
                          int nstates, double2* four, const Geom& g, hipStream_t st) {
    dim3 grid(ntasks, (nstates + 3) / 4);
    k_synthesis_swe<<<grid, kBlock, 0, st>>>(P, H, toff, rowoff, tasks, cml, nstates, four, g);
}

// ---------------------------------------------------------------------------------------------
// Analysis for the shallow-water explicit tendency (MODE = kAnaForward).  Input: per (m, parity
// p, latitude, state) the seven weighted Fourier columns of the grid kernel.  Output per state:
//   d zeta/dt = Pbar.col0 + H.col4, d delta/dt = Pbar.col1 + H.col5 + n(n+1)/a^2 Pbar.col2,
//   d Phi'/dt = Pbar.col3 + H.col6.
// Transposed synthesis of the adjoint (MODE = kAnaAdjoint), accumulated into the output:
//   zeta_adj += Pbar.col0 + (-a^2/(n(n+1))) (Pbar.col1 + H.col4'),
//   delta_adj += (-a^2/(n(n+1))) (Pbar.col2 + H.col5'),  Phi'_adj += Pbar.col3
// (col4', col5' stored in the H slots of kinds 1 and 2).
// A workgroup owns (m, parity, 16 consecutive rows n, 4 states); its 4 waves take every fourth
// 16-latitude block of the contraction and the partial tiles are summed in LDS in a fixed order.
// Tile columns: 2 states x (zeta, delta, KE, Phi') x (Re, Im).
// ---------------------------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_analysis_swe(
    const double* __restrict__ P, const double* __restrict__ H, const long long* __restrict__ toff,
    const int4* __restrict__ tasks, const double* __restrict__ G, int nstates,
    const double* __restrict__ nscale, double* __restrict__ out, Geom g) {
    __shared__ double lds[3 * 8 * 64];
    const int4 task = tasks[blockIdx.x];
    if (task.w == 0) return;                             // padding workgroup (uniform)
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m = task.x, p = task.y, kk0 = task.z;
    const int S = nstates;
    const int np = npk_of(g.T, m, p);
    const int np4 = (np + 3) & ~3;
    const int s0 = blockIdx.y * 4;
    const int i = lane & 15, q = lane >> 4;
    const int kr = kk0 + i;
    const bool rowok = kr < np4;
    const double* Pr = P + toff[2 * m + p] + (size_t)(rowok ? kr : 0) * g.nhp + 4 * q;
    const double* Hr = H + toff[2 * m + p] + (size_t)(rowok ? kr : 0) * g.nhp + 4 * q;

    // forward kinds: 0 zeta 1 delta 2 KE 3 Phi'; adjoint kinds: 0 zeta 1 zeta (via psi)
    // 2 delta (via chi) 3 Phi'
    const int v = i & 7, re = v & 1, kind = v >> 1;
    const bool has_h = MODE == kAnaForward ? kind != 2 : (kind == 1 || kind == 2);
    const int cH = (MODE == kAnaForward ? (kind == 0 ? 8 : (kind == 1 ? 10 : 12))
                                        : (kind == 1 ? 8 : 10)) + re;
    const size_t jstride = (size_t)S * kAnaVals;
    const double* gb = G + (size_t)(m * 2 + p) * g.nhp * jstride + 4 * q * jstride;
    bool okP[2], okH[2];
    int offP[2], offH[2];
    for (int t = 0; t < 2; ++t) {
        const int s = s0 + 2 * t + (i >> 3);
        okP[t] = s < S;
        okH[t] = okP[t] && has_h;
        offP[t] = (okP[t] ? s : 0) * kAnaVals + v;
        offH[t] = (okP[t] ? s : 0) * kAnaVals + cH;
    }
    v4d acc0 = (v4d){0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    // this wave takes latitude blocks 16*wave, 16*wave + 64, ...; the next block's operands are
    // loaded into the alternate register set while the current one is contracted
    const int steps = g.nhp > 16 * wave ? (g.nhp - 16 * wave + 63) / 64 : 0;   // uniform
    v4d A_ap, A_ah, B_ap, B_ah;
    double A_b[16], B_b[16];
#define ANA_LOAD(X, it)                                                                \
    {                                                                                  \
        int it_ = (it) < steps ? (it) : steps - 1;  /* clamp: valid, result unused */ \
        const int jh0_ = 16 * wave + 64 * it_;                                         \
        X##_ap = *(const v4d*)(Pr + jh0_);                                             \
        X##_ah = *(const v4d*)(Hr + jh0_);                                             \
        const double* go_ = gb + (size_t)jh0_ * jstride;                               \
        _Pragma("unroll") for (int qq = 0; qq < 4; ++qq) {                             \
            const double* gq_ = go_ + qq * jstride;                                    \
            X##_b[4 * qq + 0] = gq_[offP[0]];                                          \
            X##_b[4 * qq + 1] = gq_[offH[0]];                                          \
            X##_b[4 * qq + 2] = gq_[offP[1]];                                          \
            X##_b[4 * qq + 3] = gq_[offH[1]];                                          \
        }                                                                              \
    }
#define ANA_COMPUTE(X, it)                                                             \
    { /* a step past the end (odd step count) runs on zeroed operands: no branch */     \
        const bool live_ = (it) < steps;                                               \
        const int jh0_ = 16 * wave + 64 * (it);                                        \
        _Pragma("unroll") for (int qq = 0; qq < 4; ++qq) {                             \
            const bool jok = live_ && jh0_ + 4 * q + qq < g.nh;  /* padded rows unused */ \
            const double a_ = rowok ? X##_ap[qq] : 0.0, h_ = rowok ? X##_ah[qq] : 0.0;  \
            acc0 = mfma_f64(a_, (jok && okP[0]) ? X##_b[4 * qq + 0] : 0.0, acc0);        \
            acc0 = mfma_f64(h_, (jok && okH[0]) ? X##_b[4 * qq + 1] : 0.0, acc0);        \
            acc1 = mfma_f64(a_, (jok && okP[1]) ? X##_b[4 * qq + 2] : 0.0, acc1);        \
            acc1 = mfma_f64(h_, (jok && okH[1]) ? X##_b[4 * qq + 3] : 0.0, acc1);        \
        }                                                                              \
    }
    if (steps > 0) {
        ANA_LOAD(A, 0)
        for (int it = 0; it < steps; it += 2) {
            ANA_LOAD(B, it + 1)
            ANA_COMPUTE(A, it)
            ANA_LOAD(A, it + 2)
            ANA_COMPUTE(B, it + 1)
        }
    }
#undef ANA_LOAD
#undef ANA_COMPUTE
    if (wave > 0)
        for (int r = 0; r < 4; ++r) {
            lds[((wave - 1) * 8 + r) * 64 + lane] = acc0[r];
            lds[((wave - 1) * 8 + 4 + r) * 64 + lane] = acc1[r];
        }
    __syncthreads();
    if (wave != 0) return;
    for (int w = 0; w < 3; ++w)
        for (int r = 0; r < 4; ++r) {
            acc0[r] += lds[(w * 8 + r) * 64 + lane];
            acc1[r] += lds[(w * 8 + 4 + r) * 64 + lane];
        }
    const int cb = coef_offset(g.T, m) - m;
    for (int t = 0; t < 2; ++t) {
        const int s = s0 + 2 * t + (i >> 3);
        for (int r = 0; r < 4; ++r) {
            const double val = t == 0 ? acc0[r] : acc1[r];
            const double right = __shfl_down(val, 2, 64);   // the kind one to the right
            const int kk = kk0 + 4 * r + q;
            if (kk >= np || s >= S) continue;
            const int n = m + p + 2 * kk;
            if constexpr (MODE == kAnaForward) {
                if (kind == 2) continue;
                const int field = kind == 0 ? 1 : (kind == 1 ? 2 : 0);
                const double res = kind == 1 ? val + nscale[n] * right : val;
                out[((size_t)(s * 3 + field) * g.ncoef + cb + n) * 2 + re] = res;
            } else {
                if (kind == 1) continue;
                const int field = kind == 0 ? 1 : (kind == 2 ? 2 : 0);
                const double res = kind == 0 ? val + nscale[n] * right : (kind == 2 ? nscale[n] * val : val);
                out[((size_t)(s * 3 + field) * g.ncoef + cb + n) * 2 + re] += res;
            }
        }
    }
}

void launch_analysis_swe(const double* P, const double* H, const long long* toff,
                         const int4* tasks, int nwg, const double* G, int nstates,
                         const double* neg_lap, double* out, const Geom& g, hipStream_t st) {
    dim3 grid(nwg, (nstates + 3) / 4);
    k_analysis_swe<kAnaForward><<<grid, kBlock, 0, st>>>(P, H, toff, tasks, G, nstates, neg_lap, out, g);
}

void launch_analysis_adjoint(const double* P, const double* H, const long long* toff,
                             const int4* tasks, int nwg, const double* G, int nstates,
                             const double* inv_lap, double* out_acc, const Geom& g, hipStream_t st) {
    dim3 grid(nwg, (nstates + 3) / 4);
    k_analysis_swe<kAnaAdjoint><<<grid, kBlock, 0, st>>>(P, H, toff, tasks, G, nstates, inv_lap, out_acc, g);
}

// ---------------------------------------------------------------------------------------------
// Scalar transforms (sht_inverse / sht_forward): Pbar only, 8 fields x (Re, Im) per tile.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_synthesis_scalar(
    const double* __restrict__ P, const long long* __restrict__ toff, const int2* __restrict__ tasks,
    const double* __restrict__ spec, int nfields, double2* __restrict__ four, Geom g) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int2 task = tasks[blockIdx.x];
    const int m = task.x;
    const int jt = task.y * 4 + wave;
    if (jt >= (g.nhp >> 4)) return;
    const int f0 = blockIdx.y * 8;
    const int i = lane & 15, q = lane >> 4;
    const int f = f0 + (i >> 1), re = i & 1;
    const bool okf = f < nfields;
    const int cb = coef_offset(g.T, m) - m;
    const double* bp = spec + ((size_t)f * g.ncoef + cb) * 2 + re;
    v4d acc[2];
    for (int p = 0; p < 2; ++p) {
        const int np = npk_of(g.T, m, p);
        const int np4 = (np + 3) & ~3;
        const double* Pp = P + toff[2 * m + p] + jt * 16 + i;
        v4d c = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int kk0 = 0; kk0 < np4; kk0 += 4) {
            const int kk = kk0 + q;
            const int n = m + p + 2 * kk;
            const double ap = Pp[(size_t)kk * g.nhp];
            const double b = (kk < np && okf) ? bp[2 * n] : 0.0;
            c = mfma_f64(ap, b, c);
        }
        acc[p] = c;
    }
    for (int r = 0; r < 4; ++r) {
        const double nv = acc[0][r] + acc[1][r];
        const double sv = acc[0][r] - acc[1][r];
        const double nv_im = __shfl_xor(nv, 1, 64);
        const double sv_im = __shfl_xor(sv, 1, 64);
        const int jh = jt * 16 + 4 * r + q;
        if (re != 0 || !okf || jh >= g.nh) continue;
        // the imaginary part of m = 0 does not enter a real field
        const double ni = m == 0 ? 0.0 : nv_im, si = m == 0 ? 0.0 : sv_im;
        four[((size_t)f * g.nlat + jh) * g.ms + m] = make_double2(nv, ni);
        four[((size_t)f * g.nlat + (g.nlat - 1 - jh)) * g.ms + m] = make_double2(sv, si);
    }
}

void launch_synthesis_scalar(const double* P, const long long* toff, const int2* tasks, int ntasks,
                             const double* spec, int nfields, double2* four, const Geom& g,
                             hipStream_t st) {
    dim3 grid(ntasks, (nfields + 7) / 8);
    k_synthesis_scalar<<<grid, kBlock, 0, st>>>(P, toff, tasks, spec, nfields, four, g);
}

// Input ana[f][p][jh][m]: Gauss-weighted north +- south Fourier coefficients.
__global__ __launch_bounds__(kBlock) void k_analysis_scalar(
    const double* __restrict__ P, const long long* __restrict__ toff, const int4* __restrict__ tasks,
    int ntasks, const double2* __restrict__ ana, int nfields, double* __restrict__ spec, Geom g) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tid = blockIdx.x * 4 + wave;
    if (tid >= ntasks) return;
    const int4 task = tasks[tid];
    const int m = task.x, p = task.y, kk0 = task.z;
    const int np = npk_of(g.T, m, p);
    const int np4 = (np + 3) & ~3;
    const int i = lane & 15, q = lane >> 4;
    const int kr = kk0 + i;
    const bool rowok = kr < np4;
    const double* Pr = P + toff[2 * m + p] + (size_t)(rowok ? kr : 0) * g.nhp + 4 * q;
    const int f = blockIdx.y * 8 + (i >> 1), re = i & 1;
    const bool okf = f < nfields;
    const size_t jstride = (size_t)2 * g.ms;
    const double* bp = (const double*)(ana + (size_t)(f * 2 + p) * g.nhp * g.ms + m) + re + 4 * q * jstride;
    v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
    const v4d zero4 = acc;
    for (int jh0 = 0; jh0 < g.nhp; jh0 += 16) {
        const v4d ap = rowok ? *(const v4d*)(Pr + jh0) : zero4;
        const size_t o = (size_t)jh0 * jstride;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const bool jok = jh0 + 4 * q + qq < g.nh;
            const double b = (jok && okf) ? bp[o + qq * jstride] : 0.0;
            acc = mfma_f64(ap[qq], b, acc);
        }
    }
    const int cb = coef_offset(g.T, m) - m;
    for (int r = 0; r < 4; ++r) {
        const int kk = kk0 + 4 * r + q;
        if (kk >= np || !okf) continue;
        const int n = m + p + 2 * kk;
        const double val = (m == 0 && re == 1) ? 0.0 : acc[r];
        spec[((size_t)f * g.ncoef + cb + n) * 2 + re] = val;
    }
}

void launch_analysis_scalar(const double* P, const long long* toff, const int4* tasks, int ntasks,
                            const double2* ana, int nfields, double* spec, const Geom& g,
                            hipStream_t st) {
    dim3 grid((ntasks + 3) / 4, (nfields + 7) / 8);
    k_analysis_scalar<<<grid, kBlock, 0, st>>>(P, toff, tasks, ntasks, ana, nfields, spec, g);
}
