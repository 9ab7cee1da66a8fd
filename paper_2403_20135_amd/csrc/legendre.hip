// Legendre transforms as FP64 MFMA contractions (gfx950, v_mfma_f64_16x16x4f64).
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
//
// Both SWE kernels give every wave one whole contraction (no partial sums across waves, no LDS),
// keep several 4-row (synthesis) or 16-latitude (analysis) operand stages in flight in registers,
// and place the columns of their tiles so that every output is formed from values the lane
// already holds.
#include "adj_update.h"
#include "node_update.h"

#include <type_traits>

constexpr int kAnaForward = 0, kAnaAdjoint = 1;
constexpr int kSynForward = 0, kSynAdjoint = 1;

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d zero4() { return (v4d){0.0, 0.0, 0.0, 0.0}; }

// Table precision of the SWE kernels: FP64 (v_mfma_f64_16x16x4f64; the accumulator of lane l
// holds rows 4r + q) or FP32 (v_mfma_f32_16x16x4f32 with FP32 accumulation; rows 4q + r).  Both
// take A[i][q] and B[q][i] from lane i + 16 q.  The coefficient columns of both transforms are
// stored in the table precision by their producers (in the FP32 mode: rounded once, as the MFMA
// would round them); the analysis copies its columns to LDS as FP64 and rounds them at the MFMA.
typedef float v4f __attribute__((ext_vector_type(4)));
template <typename TT> struct Mma;
template <> struct Mma<double> {
    typedef v4d vec;
    __device__ static vec zero() { return (v4d){0.0, 0.0, 0.0, 0.0}; }
    __device__ static vec mma(double a, double b, vec c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static constexpr int row(int r, int q) { return 4 * r + q; }
};
template <> struct Mma<float> {
    typedef v4f vec;
    __device__ static vec zero() { return (v4f){0.0f, 0.0f, 0.0f, 0.0f}; }
    __device__ static vec mma(float a, float b, vec c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static constexpr int row(int r, int q) { return 4 * q + r; }
};

// BF16x3 mode: the tables and columns are the FP32 values of the FP32 mode (same storage), and
// each MFMA product a b is formed on the BF16 matrix cores from an exact three-term split
// x = x0 + x1 + x2 of both operands into BF16 values (x0 = x truncated to 8 significant bits,
// x1 = the remainder truncated likewise, x2 = what is left, at most 8 significant bits, so the
// sum is exact).  One v_mfma_f32_16x16x32_bf16 replaces one 16x16x4 FP32 step: the 8 BF16 slots
// of lane (i, q) hold the split terms of the lane's single operand A[i][q] (resp. B[q][i]),
// paired slot by slot so that the slot products are the 8 cross terms a_r b_s with r + s <= 3
// (every one but a2 b2, below 2^-32 |a b|); both operands map (lane group, slot) to the same
// k, so the instruction's sum over its 32 k is the 4-term contraction of the FP32 step with
// the compensated products, accumulated in FP32.
struct Bf3 {
    float v;
    Bf3() = default;
    __device__ Bf3(double x) : v((float)x) {}
    __device__ operator float() const { return v; }
};
static_assert(sizeof(Bf3) == sizeof(float), "BF16x3 operands are stored as FP32");
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
// high halves (the BF16 values) of x, of r1 = x - x0 and of r2 = r1 - x1
__device__ __forceinline__ void split3(float x, unsigned& h0, unsigned& h1, unsigned& h2) {
    const unsigned u0 = __float_as_uint(x);
    const float r1 = x - __uint_as_float(u0 & 0xffff0000u);          // exact
    const unsigned u1 = __float_as_uint(r1);
    const float r2 = r1 - __uint_as_float(u1 & 0xffff0000u);         // exact, <= 8 bits
    h0 = u0 >> 16;
    h1 = u1 >> 16;
    h2 = __float_as_uint(r2) >> 16;
}
// slots (low half first): A a0 a0 a1 a0 a1 a2 a1 a2, B b0 b1 b0 b2 b1 b0 b2 b1
__device__ __forceinline__ v4u bf3_a(float a) {
    unsigned a0, a1, a2;
    split3(a, a0, a1, a2);
    return (v4u){a0 | (a0 << 16), a1 | (a0 << 16), a1 | (a2 << 16), a1 | (a2 << 16)};
}
__device__ __forceinline__ v4u bf3_b(float b) {
    unsigned b0, b1, b2;
    split3(b, b0, b1, b2);
    return (v4u){b0 | (b1 << 16), b0 | (b2 << 16), b1 | (b0 << 16), b2 | (b1 << 16)};
}
template <> struct Mma<Bf3> {
    typedef v4f vec;
    __device__ static vec zero() { return (v4f){0.0f, 0.0f, 0.0f, 0.0f}; }
    __device__ static vec mma(float a, float b, vec c) { return mma_pre(a, bf3_b(b), c); }
    // with the B operand's slots already formed (the analysis stages them once per workgroup)
    __device__ static vec mma_pre(float a, v4u B, vec c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, bf3_a(a)),
                                                        __builtin_bit_cast(v8bf, B), c, 0, 0, 0);
    }
    __device__ static constexpr int row(int r, int q) { return 4 * q + r; }
};

// ---------------------------------------------------------------------------------------------
// Synthesis (forward SWE and the transposed analysis of the adjoint).
//
// A workgroup of two waves owns (m, one 16-latitude tile, 4 states); wave p contracts the degrees
// of parity p (4-row steps, D operand stages in flight in registers).  The two partial tiles meet
// in LDS once at the end: wave 0 writes the northern latitudes (even + odd), wave 1 the southern
// ones (even - odd for Pbar tiles, odd - even for H tiles).
//
// Column tiles: 16 columns = 4 states x 4 values (lane column i: state i >> 2, value v = i & 3).
// Forward, Fourier fields (zeta, Phi', U, V), cml values (zeta, Phi', psi, chi) x (Re, Im):
//   tile 0 (Pbar): zeta re, zeta im, Phi' re, Phi' im        -> cml value v
//   tile 1 (Pbar): chi im, chi re, psi im, psi re            -> cml value 7 - v
//   tile 2 (H):    psi re, psi im, chi re, chi im            -> cml value 4 + v
// so that U = (1/a)(i m chi Pbar - psi H) and V = (1/a)(i m psi Pbar + chi H) are lane-local:
//   (U re, U im, V re, V im)[v] = ((v odd ? m : -m) tile1 + (v < 2 ? -1 : 1) tile2) / a.
// Adjoint, fields (A^, B^, C^, D^, E^), cml values (zeta, delta, Phi, c_n delta)_adj x (Re, Im):
//   A^ = i m Pbar.zeta + H.delta,  B^ = H.zeta - i m Pbar.delta,  C^ = i m Pbar.Phi,
//   D^ = H.Phi,  E^ = Pbar.(c delta), all halved for m > 0;
//   tile 0 (Pbar): zeta im, zeta re, delta im, delta re      -> v ^ 1
//   tile 1 (H):    delta re, delta im, zeta re, zeta im      -> v ^ 2
//   tile 2 (Pbar): Phi im, Phi re, c delta re, c delta im    -> v < 2 ? 5 - v : 4 + v
//   tile 3 (H):    Phi re, Phi im, (unused), (unused)        -> 4 + (v & 1)
// Rows of the table past n = T are zero, and so are the matching rows of the cml input (written
// by its producers), so no row needs masking; columns of absent states read state S-1 and are
// dropped.
// ---------------------------------------------------------------------------------------------
template <int MODE> struct SynTiles;
// With one or two states a tile's columns are half empty: tile t then also carries the values of
// tile partner(t) (same table operand) in lane groups 2 and 3, and the partner (rider) is neither
// loaded nor contracted.
template <> struct SynTiles<kSynForward> {
    static constexpr int NT = 3, NF = kSynFields;
    __device__ static constexpr bool is_h(int t) { return t == 2; }
    __device__ static int col(int t, int v) { return t == 0 ? v : (t == 1 ? 7 - v : 4 + v); }
    __device__ static constexpr int partner(int t) { return t == 0 ? 1 : -1; }
    __device__ static constexpr bool rider(int t) { return t == 1; }
};
template <> struct SynTiles<kSynAdjoint> {
    static constexpr int NT = 4, NF = 5;
    __device__ static constexpr bool is_h(int t) { return t == 1 || t == 3; }
    __device__ static int col(int t, int v) {
        return t == 0 ? (v ^ 1) : (t == 1 ? (v ^ 2) : (t == 2 ? (v < 2 ? 5 - v : 4 + v) : 4 + (v & 1)));
    }
    __device__ static constexpr int partner(int t) { return t < 2 ? t + 2 : -1; }
    __device__ static constexpr bool rider(int t) { return t >= 2; }
};

template <typename TT, int NT, int JT> struct SynStage {
    TT a[JT][2];             // Pbar, H of each latitude tile
    TT b[NT];                // coefficient columns (stored in the table type)
};

constexpr int kSynBlock = 128;                   // two waves: the two parities

// JT latitude tiles per workgroup share every coefficient column they load; D operand stages are
// in flight per wave.  Task (m, jt0) covers tiles jt0 .. jt0 + JT - 1 (tiles past the last one
// re-read it and store nothing).
//
// REC (JT = 1, 2 or 4 latitude tiles per wave): the table operands are not read but regenerated
// in registers by the upward recurrence in n (leg_next / leg_h with the stored coefficients, the
// same evaluation as the table generator, hence the same values bit for bit), so only the
// coefficient columns stream from HBM.  Lane (i, q) of wave p runs the recurrence for latitude i
// of tile q % JT through all degrees (both parities: each value needs the two before it; the
// coefficients are wave-uniform scalar loads, issued a step ahead) and forms Pbar_n, H_n of the
// step's four rows n = m + p + 2 (4 j + k) in registers k = 0..3.  The MFMA slot of lane (i, q)
// for tile u takes row q of tile u, i.e. register q of lane (i, u): a 4 x 4 transpose between
// registers and lane groups, done by one row-pair swap (v_permlane32_swap) and one row swap
// (v_permlane16_swap); with JT < 4 the lane groups past JT repeat the first ones.
__device__ __forceinline__ void swap_rows32(unsigned& a, unsigned& b) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);   // rows 2,3 of a <-> rows 0,1 of b
    a = r[0];
    b = r[1];
}
__device__ __forceinline__ void swap_rows16(unsigned& a, unsigned& b) {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);   // odd rows of a <-> even rows of b
    a = r[0];
    b = r[1];
}
// v[u] at lane group q becomes v[q] at lane group u (rows are 16-lane groups)
__device__ __forceinline__ void transpose_rows4(double (&v)[4]) {
    unsigned lo[4], hi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        lo[k] = (unsigned)__double_as_longlong(v[k]);
        hi[k] = (unsigned)((unsigned long long)__double_as_longlong(v[k]) >> 32);
    }
    swap_rows32(lo[0], lo[2]);
    swap_rows32(lo[1], lo[3]);
    swap_rows32(hi[0], hi[2]);
    swap_rows32(hi[1], hi[3]);
    swap_rows16(lo[0], lo[1]);
    swap_rows16(lo[2], lo[3]);
    swap_rows16(hi[0], hi[1]);
    swap_rows16(hi[2], hi[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        v[k] = __longlong_as_double((long long)(((unsigned long long)hi[k] << 32) | lo[k]));
}

//
// SIN (forward): the input columns are read from the state layout itself
// ([state][Phi', zeta, delta][ncoef] complex) instead of the synthesis layout: value v is zeta
// (v < 2), Phi' (v < 4) or inv_lap[n] times zeta or delta (v >= 4), part v & 1, formed with the
// same products and roundings as the conversion kernel, so a step's first f_E needs no
// conversion launch and gives the same results bit for bit.
// The body of one workgroup (task bx of the task list, state group by); the kernels below run it
// for one handle's launch or for one workgroup of a launch over several handles.
template <int MODE, typename TT, int JT, int D, bool REC, bool SIN>
__device__ __forceinline__ void synthesis_body(
    const TT* __restrict__ P, const TT* __restrict__ H, const long long* __restrict__ toff,
    const int* __restrict__ rowoff, const int2* __restrict__ tasks, const TT* __restrict__ cml,
    int nstates, double* __restrict__ four, const Geom& g, const double* __restrict__ rc,
    const double* __restrict__ sect, const double* __restrict__ mu,
    const double* __restrict__ sin_state, const double* __restrict__ inv_lap, int bx, int by) {
    using TL = SynTiles<MODE>;
    using MM = Mma<TT>;
    constexpr int NT = TL::NT;
    constexpr unsigned tsz = sizeof(TT);
    __shared__ double part[2][NT][4][64];
    // state groups on by (the second grid dimension): the groups of one task run far apart in
    // time (sharing a table tile between co-scheduled groups through L2 measured slower)
    const int2 task = tasks[bx];
    if (task.x < 0) return;                                  // padding workgroup (uniform)
    const int p = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // parity of this wave
    const int m = task.x, jt0 = task.y, ntj = g.nhp >> 4;
    const int lane = threadIdx.x & 63, i = lane & 15, q = lane >> 4, v = i & 3;
    // REC state of this lane's latitude (tile q): mu, Pbar_{n-1}, Pbar_n at the step's first row
    // n = m + p + 8 j, and the coefficients of that row
    static_assert(!REC || JT == 1 || JT == 2 || JT == 4, "regenerating synthesis: 1, 2 or 4 tiles");
    double rx = 0.0, rpm1 = 0.0, rp0 = 0.0;
    const double* rcrow = rc + 4 * rec_index(g.T, m, m + p);
    double rcs[24];                                          // the next step's coefficients
    auto load_coefs = [&]() {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int e = 0; e < 6; ++e) rcs[6 * k + e] = rcrow[8 * k + e];   // wave-uniform
        rcrow += 32;
    };
    if constexpr (REC) {
        load_coefs();
        const int tq = jt0 + q % JT;
        const int jh = (tq < ntj ? tq : ntj - 1) * 16 + i;
        rx = jh < g.nh ? mu[jh] : 0.0;
        const double pmm = sect[(size_t)m * g.nhp + jh];
        if (p == 0) {
            rp0 = pmm;
        } else {                                             // one degree up: Pbar_m, Pbar_{m+1}
            const double* c0 = rc + 4 * rec_index(g.T, m, m);
            rpm1 = pmm;
            rp0 = leg_next(rx, pmm, 0.0, c0[0], c0[1]);
        }
    }
    const int S = nstates;
    const int s = by * 4 + (i >> 2);
    const int sc = s < S ? s : S - 1;
    // One or two states (a step's first f_E of one or two members): a tile and its partner (the
    // same table operand) share one MFMA, lane group i >> 2 = 2 h + s holding state s's values of
    // the tile (h = 0) or of the partner (h = 1), and the partner's products move back to lane
    // groups 0 and 1 (the states' own lanes) after the contraction.  Every product is formed from
    // the same operands as with separate tiles.
    const bool fold = S <= 2;                                       // uniform
    const int gs = (i >> 2) & 1, fs = gs < S ? gs : S - 1;          // fold: state of lane group
    auto colv = [&](int t) {
        return fold && TL::partner(t) >= 0 && (i >> 3) ? TL::col(TL::partner(t), v) : TL::col(t, v);
    };
    const int scol = fold ? fs : sc;                                // state of this lane's columns
    // 32-bit byte offsets from per-block (uniform) base addresses: one VGPR per address
    unsigned boff[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) boff[t] = (unsigned)(scol * kCmlVals + colv(t)) * tsz;
    static_assert(!SIN || MODE == kSynForward, "state input: forward synthesis");
    size_t soff[NT];
    bool sscale[NT];
    const int npk = npk_of(g.T, m, p);
    if constexpr (SIN) {
        const size_t fsd = (size_t)g.ncoef * 2;
        const size_t c0 = (size_t)coef_offset(g.T, m) * 2;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int vv = colv(t);
            const int field = vv < 2 ? 1 : (vv < 4 ? 0 : (vv < 6 ? 1 : 2));
            soff[t] = ((size_t)scol * 3 + field) * fsd + c0 + (vv & 1);
            sscale[t] = vv >= 4;
        }
    }
    const unsigned rstride = (unsigned)S * kCmlVals * tsz;          // bytes per cml row
    const int nst = (npk_of(g.T, m, p) + 3) >> 2;                   // 4-row steps of this parity
    const unsigned tstep = 4u * 16u * tsz, cstep = 4u * rstride;    // bytes per 4-row step
    unsigned tlane[JT];
#pragma unroll
    for (int u = 0; u < JT; ++u) {
        const int jt = jt0 + u < ntj ? jt0 + u : ntj - 1;
        tlane[u] = ((unsigned)(jt * 4 * nst + q) * 16 + i) * tsz;
    }
    const unsigned clane = (unsigned)q * rstride;
    const char* tP = (const char*)(P + toff[2 * m + p]);
    const char* tH = (const char*)(H + toff[2 * m + p]);
    const char* cb = (const char*)(cml + (size_t)rowoff[2 * m + p] * S * kCmlVals);
    auto ldt = [](const char* base, unsigned off) { return *(const TT*)(base + off); };

    typename MM::vec acc[JT][NT];
#pragma unroll
    for (int u = 0; u < JT; ++u)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[u][t] = MM::zero();
    // fold: a rider tile is neither loaded nor contracted (its values ride in its partner's columns)
    auto skip = [](auto fd, int t) { return decltype(fd)::value && TL::rider(t); };
    auto load = [&](auto fd, SynStage<TT, NT, JT>& x, int j) {
        const unsigned oc = clane + (unsigned)j * cstep;
        if constexpr (!REC) {
#pragma unroll
            for (int u = 0; u < JT; ++u) {
                const unsigned ot = tlane[u] + (unsigned)j * tstep;
                x.a[u][0] = ldt(tP, ot);
                x.a[u][1] = ldt(tH, ot);
            }
        }
        if constexpr (SIN) {
            // rows past the order's end read its last row and contribute zero
            const int kk = 4 * j + q;
            const int dn = p + 2 * (kk < npk ? kk : npk - 1);          // n - m
            const double il = inv_lap[m + dn];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (skip(fd, t)) continue;
                const double val = sin_state[soff[t] + 2 * (size_t)dn];
                const double w = sscale[t] ? il * val : val;
                x.b[t] = kk < npk ? (TT)w : (TT)0;
            }
        } else {
#pragma unroll
            for (int t = 0; t < NT; ++t)
                if (!skip(fd, t)) x.b[t] = ldt(cb, oc + boff[t]);
        }
    };
    auto mma_all = [&](auto fd, const TT (&a)[JT][2], const TT (&b)[NT]) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (skip(fd, t)) continue;
#pragma unroll
            for (int u = 0; u < JT; ++u) acc[u][t] = MM::mma(a[u][TL::is_h(t) ? 1 : 0], b[t], acc[u][t]);
        }
    };
    // REC: the eight degrees of the next step (row k of the step is degree 2k), then the transpose
    // (the following step's coefficients are requested as soon as these are used)
    auto generate = [&](TT (&a)[JT][2]) {
        double vp[4], vh[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double* ck = rcs + 6 * k;
            const double p1 = leg_next(rx, rp0, rpm1, ck[0], ck[1]);
            vp[k] = rp0;
            vh[k] = leg_h(rpm1, p1, ck[2], ck[3]);
            rpm1 = p1;
            rp0 = leg_next(rx, p1, vp[k], ck[4], ck[5]);
        }
        load_coefs();
        transpose_rows4(vp);
        transpose_rows4(vh);
#pragma unroll
        for (int u = 0; u < JT; ++u) {
            a[u][0] = (TT)vp[u];
            a[u][1] = (TT)vh[u];
        }
    };
    auto compute = [&](auto fd, const SynStage<TT, NT, JT>& x) {
        if constexpr (REC) {
            TT ga[JT][2];
            generate(ga);
            mma_all(fd, ga, x.b);
        } else {
            mma_all(fd, x.a, x.b);
        }
    };
    // Loads past the chain's end re-read its last step (cache hits, results unused): a
    // branch-free loop body lets every stage wait for its own loads only.
    auto pipeline = [&](auto fd) {
        SynStage<TT, NT, JT> st[D];
#pragma unroll
        for (int u = 0; u < D; ++u) load(fd, st[u], u < nst ? u : nst - 1);
        int j0 = 0;
        for (; j0 + D <= nst; j0 += D) {
#pragma unroll
            for (int u = 0; u < D; ++u) {
                compute(fd, st[u]);
                const int jn = j0 + u + D;
                load(fd, st[u], jn < nst ? jn : nst - 1);
            }
        }
#pragma unroll
        for (int u = 0; u < D; ++u)
            if (u < nst - j0) compute(fd, st[u]);
    };
    if (nst > 0) {
        if (fold) pipeline(std::true_type{});
        else pipeline(std::false_type{});
    }
    if (fold) {
        // the riders' products from lane groups 2, 3 to lane groups 0, 1 (the lanes of the states)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (TL::partner(t) < 0) continue;
#pragma unroll
            for (int u = 0; u < JT; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[u][TL::partner(t)][r] = __shfl_down(acc[u][t][r], 8, 64);
        }
    }

    // wave 0: north = even + odd; wave 1: south = even - odd (Pbar tiles), odd - even (H tiles);
    // one latitude tile at a time through the same LDS exchange buffer
    const int ns = p;
    const double mm = (double)m;
    const size_t fstride = (size_t)2 * g.nlat * g.ms;               // doubles per Fourier field
    const double inva = 1.0 / g.radius;
#pragma unroll
    for (int u = 0; u < JT; ++u) {
        if (u > 0) __syncthreads();
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[p][t][r][lane] = (double)acc[u][t][r];
        __syncthreads();
        if (jt0 + u >= ntj) continue;                        // uniform
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int jh = (jt0 + u) * 16 + MM::row(r, q);
            if (s >= S || jh >= g.nh) continue;
            const int j = ns ? g.nlat - 1 - jh : jh;
            double val[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double e = ns == 0 ? (double)acc[u][t][r] : part[0][t][r][lane];
                const double o = ns == 0 ? part[1][t][r][lane] : (double)acc[u][t][r];
                val[t] = ns == 0 ? e + o : (TL::is_h(t) ? o - e : e - o);
            }
            double* base = four + (((size_t)s * TL::NF * g.nlat + j) * g.ms + m) * 2 + (v & 1);
            if constexpr (MODE == kSynForward) {
                base[(size_t)(v >> 1) * fstride] = val[0];
                const double sx = (v & 1) ? mm : -mm, sh = v < 2 ? -1.0 : 1.0;
                base[(size_t)(2 + (v >> 1)) * fstride] = (sx * val[1] + sh * val[2]) * inva;
            } else {
                const double hf = m > 0 ? 0.5 : 1.0;
                const double sx = (v == 0 || v == 3) ? -mm : mm;
                base[(size_t)(v >> 1) * fstride] = hf * (sx * val[0] + val[1]);
                if (v < 2) {
                    base[2 * fstride] = hf * ((v ? mm : -mm) * val[2]);
                    base[3 * fstride] = hf * val[3];
                } else {
                    base[4 * fstride] = hf * val[2];
                }
            }
        }
    }
}

template <int MODE, typename TT, int JT, int D, bool REC, bool SIN = false>
__global__ __launch_bounds__(kSynBlock) void k_synthesis(
    const TT* __restrict__ P, const TT* __restrict__ H, const long long* __restrict__ toff,
    const int* __restrict__ rowoff, const int2* __restrict__ tasks, const TT* __restrict__ cml,
    int nstates, double* __restrict__ four, Geom g, const double* __restrict__ rc,
    const double* __restrict__ sect, const double* __restrict__ mu,
    const double* __restrict__ sin_state, const double* __restrict__ inv_lap) {
    synthesis_body<MODE, TT, JT, D, REC, SIN>(P, H, toff, rowoff, tasks, cml, nstates, four, g, rc, sect, mu,
                                             sin_state, inv_lap, blockIdx.x, blockIdx.y);
}

// One launch over the synthesis of several handles (members of different truncations): workgroup
// b belongs to the handle h with first[h] <= b < first[h + 1] (first[h] a multiple of 8, so every
// handle keeps its XCD-ordered task list) and runs that handle's task (b - first[h]) mod gx.
template <int MODE, typename TT, int JT, int D, bool REC, bool SIN = false>
__global__ __launch_bounds__(kSynBlock) void k_synthesis_multi(const SynArgs* __restrict__ list, int n) {
    const int b = blockIdx.x;
    int h = 0;
    while (h + 1 < n && b >= list[h + 1].first) ++h;
    const SynArgs& a = list[h];
    const int local = b - a.first;
    if (local >= a.blocks) return;                           // padding to the next range (uniform)
    synthesis_body<MODE, TT, JT, D, REC, SIN>(
        static_cast<const TT*>(a.P), static_cast<const TT*>(a.H), a.toff, a.rowoff, a.tasks,
        static_cast<const TT*>(a.cml), a.nstates, a.four, a.g, a.rc, a.sect, a.mu, a.sin_state, a.inv_lap,
        local % a.gx, local / a.gx);
}

// Synthesis variants (latitude tiles per workgroup, stages in flight): (1, 8), (1, 4), (2, 4),
// (2, 2), (3, 2), (4, 2), (4, 1), (6, 1) reading the tables; all but (3, 2) and (6, 1) also
// regenerating them.
template <int MODE, typename TT>
static void launch_synthesis_variant(const LegPlan& plan, dim3 grid, hipStream_t st,
                                     const Tables& tb, const TT* P, const TT* H,
                                     const long long* toff, const int* rowoff, const int2* tasks,
                                     const double* cml, int nstates, double* four, const Geom& g,
                                     const double* state_in) {
    const TT* cmlt = reinterpret_cast<const TT*>(cml);    // stored in the table type
#define SYN_ARGS P, H, toff, rowoff, tasks, cmlt, nstates, four, g, tb.rc, tb.sect, tb.mu, state_in, tb.inv_lap
#define SYN(JT, D) k_synthesis<MODE, TT, JT, D, false><<<grid, kSynBlock, 0, st>>>(SYN_ARGS)
#define SYN_REC(JT, D) k_synthesis<MODE, TT, JT, D, true><<<grid, kSynBlock, 0, st>>>(SYN_ARGS)
#define SYN_SIN(JT, D) k_synthesis<MODE, TT, JT, D, false, true><<<grid, kSynBlock, 0, st>>>(SYN_ARGS)
#define SYN_SIN_REC(JT, D) k_synthesis<MODE, TT, JT, D, true, true><<<grid, kSynBlock, 0, st>>>(SYN_ARGS)
    if constexpr (MODE == kSynForward) {
        if (state_in) {
            // the state-input variants, at the plan's shape (the task list follows the shape)
            const int jt = plan.syn_tiles, d = plan.syn_depth;
            if (plan.syn_recur) {
                if (jt == 4 && d == 1) SYN_SIN_REC(4, 1);
                else if (jt == 4) SYN_SIN_REC(4, 2);
                else if (jt == 2 && d == 2) SYN_SIN_REC(2, 2);
                else if (jt == 2) SYN_SIN_REC(2, 4);
                else if (d == 4) SYN_SIN_REC(1, 4);
                else SYN_SIN_REC(1, 8);
                return;
            }
            if (jt == 6) SYN_SIN(6, 1);
            else if (jt == 4 && d == 1) SYN_SIN(4, 1);
            else if (jt == 4) SYN_SIN(4, 2);
            else if (jt == 3) SYN_SIN(3, 2);
            else if (jt == 2 && d == 2) SYN_SIN(2, 2);
            else if (jt == 2) SYN_SIN(2, 4);
            else if (d == 4) SYN_SIN(1, 4);
            else SYN_SIN(1, 8);
            return;
        }
    }
    if (plan.syn_recur) {
        if (plan.syn_tiles == 4 && plan.syn_depth == 1) SYN_REC(4, 1);
        else if (plan.syn_tiles == 4) SYN_REC(4, 2);
        else if (plan.syn_tiles == 2 && plan.syn_depth == 2) SYN_REC(2, 2);
        else if (plan.syn_tiles == 2) SYN_REC(2, 4);
        else if (plan.syn_depth == 4) SYN_REC(1, 4);
        else SYN_REC(1, 8);
    } else if (plan.syn_tiles == 6) SYN(6, 1);
    else if (plan.syn_tiles == 4 && plan.syn_depth == 1) SYN(4, 1);
    else if (plan.syn_tiles == 4) SYN(4, 2);
    else if (plan.syn_tiles == 3) SYN(3, 2);
    else if (plan.syn_tiles == 2 && plan.syn_depth == 2) SYN(2, 2);
    else if (plan.syn_tiles == 2) SYN(2, 4);
    else if (plan.syn_depth == 4) SYN(1, 4);
    else SYN(1, 8);
#undef SYN
#undef SYN_REC
#undef SYN_SIN
#undef SYN_SIN_REC
#undef SYN_ARGS
}

void launch_synthesis_swe(const Tables& tb, const LegPlan& plan, const long long* toff,
                          const int* rowoff, const int2* tasks, int ntasks, const double* cml,
                          int nstates, double2* four, const Geom& g, hipStream_t st,
                          const double* state_in) {
    const dim3 grid(ntasks, (nstates + 3) / 4);
    if (tb.P32 && tb.bf3)
        launch_synthesis_variant<kSynForward, Bf3>(plan, grid, st, tb, reinterpret_cast<const Bf3*>(tb.P32),
                                                   reinterpret_cast<const Bf3*>(tb.H32), toff, rowoff,
                                                   tasks, cml, nstates, (double*)four, g, state_in);
    else if (tb.P32)
        launch_synthesis_variant<kSynForward, float>(plan, grid, st, tb, tb.P32, tb.H32, toff, rowoff,
                                                     tasks, cml, nstates, (double*)four, g, state_in);
    else
        launch_synthesis_variant<kSynForward, double>(plan, grid, st, tb, tb.P, tb.H, toff, rowoff,
                                                      tasks, cml, nstates, (double*)four, g, state_in);
}

SynArgs make_syn_args(const Tables& tb, const long long* toff, const int* rowoff, const int2* tasks,
                      int ntasks, const double* cml, int nstates, double* four, const Geom& g,
                      const double* state_in) {
    SynArgs a{};
    a.P = tb.P32 ? (const void*)tb.P32 : (const void*)tb.P;
    a.H = tb.P32 ? (const void*)tb.H32 : (const void*)tb.H;
    a.toff = toff;
    a.rowoff = rowoff;
    a.tasks = tasks;
    a.cml = cml;
    a.nstates = nstates;
    a.four = four;
    a.g = g;
    a.rc = tb.rc;
    a.sect = tb.sect;
    a.mu = tb.mu;
    a.sin_state = state_in;
    a.inv_lap = tb.inv_lap;
    a.gx = ntasks;
    a.blocks = ntasks * ((nstates + 3) / 4);
    return a;
}

void launch_synthesis_multi(const LegPlan& plan, int tt, bool state_in, const SynArgs* list, int n,
                            int blocks, hipStream_t st) {
#define SYNM(TT, JT, D, REC, SIN) k_synthesis_multi<kSynForward, TT, JT, D, REC, SIN><<<blocks, kSynBlock, 0, st>>>(list, n)
#define SYNM_PLAN(TT, SIN)                                                                        \
    do {                                                                                          \
        const int jt = plan.syn_tiles, d = plan.syn_depth;                                        \
        if (plan.syn_recur) {                                                                     \
            if (jt == 4 && d == 1) SYNM(TT, 4, 1, true, SIN);                                     \
            else if (jt == 4) SYNM(TT, 4, 2, true, SIN);                                          \
            else if (jt == 2 && d == 2) SYNM(TT, 2, 2, true, SIN);                                \
            else if (jt == 2) SYNM(TT, 2, 4, true, SIN);                                          \
            else if (d == 4) SYNM(TT, 1, 4, true, SIN);                                           \
            else SYNM(TT, 1, 8, true, SIN);                                                       \
        } else if (jt == 6) SYNM(TT, 6, 1, false, SIN);                                           \
        else if (jt == 4 && d == 1) SYNM(TT, 4, 1, false, SIN);                                   \
        else if (jt == 4) SYNM(TT, 4, 2, false, SIN);                                             \
        else if (jt == 3) SYNM(TT, 3, 2, false, SIN);                                             \
        else if (jt == 2 && d == 2) SYNM(TT, 2, 2, false, SIN);                                   \
        else if (jt == 2) SYNM(TT, 2, 4, false, SIN);                                             \
        else if (d == 4) SYNM(TT, 1, 4, false, SIN);                                              \
        else SYNM(TT, 1, 8, false, SIN);                                                          \
    } while (0)
    if (tt == kTabBf3) {
        if (state_in) SYNM_PLAN(Bf3, true);
        else SYNM_PLAN(Bf3, false);
    } else if (tt == kTabF32) {
        if (state_in) SYNM_PLAN(float, true);
        else SYNM_PLAN(float, false);
    } else {
        if (state_in) SYNM_PLAN(double, true);
        else SYNM_PLAN(double, false);
    }
#undef SYNM_PLAN
#undef SYNM
}

void launch_synthesis_adj(const Tables& tb, const LegPlan& plan, const long long* toff,
                          const int* rowoff, const int2* tasks, int ntasks, const double* cml,
                          int nstates, double2* four5, const Geom& g, hipStream_t st) {
    const dim3 grid(ntasks, (nstates + 3) / 4);
    if (tb.P32 && tb.bf3)
        launch_synthesis_variant<kSynAdjoint, Bf3>(plan, grid, st, tb, reinterpret_cast<const Bf3*>(tb.P32),
                                                   reinterpret_cast<const Bf3*>(tb.H32), toff, rowoff,
                                                   tasks, cml, nstates, (double*)four5, g, nullptr);
    else if (tb.P32)
        launch_synthesis_variant<kSynAdjoint, float>(plan, grid, st, tb, tb.P32, tb.H32, toff, rowoff,
                                                     tasks, cml, nstates, (double*)four5, g, nullptr);
    else
        launch_synthesis_variant<kSynAdjoint, double>(plan, grid, st, tb, tb.P, tb.H, toff, rowoff,
                                                      tasks, cml, nstates, (double*)four5, g, nullptr);
}

// ---------------------------------------------------------------------------------------------
// Analysis for the shallow-water explicit tendency (MODE = kAnaForward).  Input: per (latitude,
// m, state) the weighted north +- south sums of the products A..E (fwd_index); the workgroup of
// parity p reads its window of seven (col0..col6 = g A, g B, w E, g C with the sums Pbar pairs
// with, then g B, g A, g D with the others).  Output per state:
//   d zeta/dt = -i m Pbar.col0 + H.col4,
//   d delta/dt = i m Pbar.col1 + H.col5 + n(n+1)/a^2 Pbar.col2,
//   d Phi'/dt = -i m Pbar.col3 + H.col6.
// Transposed synthesis of the adjoint (MODE = kAnaAdjoint), accumulated into the output:
//   zeta_adj += Pbar.col0 + (-a^2/(n(n+1))) (Pbar.col1 + H.col4'),
//   delta_adj += (-a^2/(n(n+1))) (Pbar.col2 + H.col5'),  Phi'_adj += Pbar.col3
// (col4', col5' stored in the H slots of kinds 1 and 2).
//
// A workgroup owns (m, parity, 64 consecutive rows n, 4 states); wave w takes the 16-row tile w
// and all 4 states (two 16-column tiles: 2 states x (zeta, delta, KE, Phi') x (Re, Im)), and
// contracts over all latitudes in 16-latitude blocks.  The columns of a block (16 latitudes x 4
// states x 14 values) are loaded once per workgroup into LDS (double-buffered, one barrier per
// block) and read by all four waves; the table rows stream through D register stages per wave.
// The Pbar and H products of one column accumulate in the same lane (the H product of a kind
// without an H part is formed from another column and dropped), so every output except the KE
// term of delta (one lane to the right) is lane-local.
// ---------------------------------------------------------------------------------------------
constexpr int kAnaLat = 4 * kAnaVals + 2;       // LDS doubles per latitude (padded: no conflicts)
constexpr int kAnaBuf = 16 * kAnaLat;           // doubles per LDS block buffer
constexpr int kAnaChunks = 16 * 2 * kAnaVals;   // double2 chunks per block (16 lat x 4 states x 7)

template <typename TT, bool REC> struct AnaStage {
    typename Mma<TT>::vec aP, aH;   // table rows, 4 consecutive latitudes per lane group
};
// REC: the table entries of a block are regenerated from two stored values per lane
template <typename TT> struct AnaStage<TT, true> {
    double pm1, p0, mu;             // Pbar_{n0-1}, Pbar_{n0} and mu of the lane's latitude
};

// REC (restarting recurrence): instead of streaming a wave's 16 table rows for each block, lane
// (i, q) reads Pbar_{n0-1} and Pbar_{n0} of latitude i of the block at the first of its four rows
// kt + 4q (n0 = m + p + 2 (kt + 4 q)), continues the upward recurrence over the next eight
// degrees with leg_next / leg_h (the table generator's own evaluation, so the values are the
// table entries bit for bit) and so forms Pbar, H of rows kt + 4q .. kt + 4q + 3; a wave-private
// LDS transpose then hands lane (i, q) row i at the four latitudes 4q .. 4q + 3 its MFMA steps
// take.  A quarter of the table bytes is read; the coefficients of the lane's eight degrees stay
// in registers for the whole contraction.
constexpr int kAnaTrRow = 18;                   // LDS doubles per transpose row (16 + pad)
constexpr int kAnaTr = 2 * 16 * kAnaTrRow;      // doubles per wave: (Pbar, H) x 16 rows

// The body of workgroup w of one handle's analysis launch (the kernels below run it for one
// handle's launch or for one workgroup of a launch over several handles).
template <int MODE, typename TT, int D, bool REC>
__device__ __forceinline__ void analysis_body(
    const TT* __restrict__ P, const TT* __restrict__ H, const long long* __restrict__ toff,
    const int4* __restrict__ tasks, int ntasks, int interleave, const TT* __restrict__ G,
    int nstates, const double* __restrict__ nscale, double* __restrict__ out, const Geom& g,
    const UpdateArgs& fu, int fuse, const double* __restrict__ P64, const double* __restrict__ rc,
    const double* __restrict__ mu, const AdjFuse& af, int w) {
    using MM = Mma<TT>;
    using vec = typename MM::vec;
    // BF16x3: each column value is staged as its 8 BF16 B-operand slots (16 bytes), formed once
    // per workgroup instead of once per wave and k-step
    constexpr bool bf3 = std::is_same<TT, Bf3>::value;
    __shared__ __align__(16) double gl[2][(kAnaBuf + 4) * (bf3 ? 2 : 1)];   // + a dummy slot for idle threads
    __shared__ __align__(16) double tr[REC ? 4 * kAnaTr : 2];  // REC transposes, one area per wave
    const int2 tg = xcd_task_group(w, ntasks, (nstates + 3) >> 2, interleave);
    if (tg.x >= ntasks) return;
    const int4 task = tasks[tg.x];
    if (task.w == 0) return;                                 // padding workgroup (uniform)
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m = task.x, p = task.y;
    const int kt = task.z + 16 * wave;
    const int S = nstates, s0 = tg.y * 4;
    const int nsg = S - s0 < 4 ? S - s0 : 4;                 // states in this group
    const int np = npk_of(g.T, m, p);
    const bool active = kt < np;                             // wave-uniform
    const int lane = tid & 63, i = lane & 15, q = lane >> 4;
    const int np4 = (np + 3) & ~3;
    // rows past the block's end read its last row; their outputs are dropped
    const int kr = kt + i < np4 ? kt + i : np4 - 1;
    const TT* Pr = P + toff[2 * m + p] + tab_index(np4, kr, 4 * q);
    const TT* Hr = H + toff[2 * m + p] + tab_index(np4, kr, 4 * q);
    const size_t bstride = (size_t)np4 * 16;                 // doubles per 16-latitude tile
    const int nb = g.nhp >> 4;

    // forward kinds: 0 zeta 1 delta 2 KE 3 Phi'; adjoint kinds: 0 zeta 1 zeta (via psi)
    // 2 delta (via chi) 3 Phi'
    const int v = i & 7, re = v & 1, kind = v >> 1;
    const bool has_h = MODE == kAnaForward ? kind != 2 : (kind == 1 || kind == 2);
    const int cH = (MODE == kAnaForward ? (kind == 0 ? 8 : (kind == 1 ? 10 : 12))
                                        : (kind == 1 ? 8 : 10)) + re;
    int offP[2], offH[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        int sl = 2 * t + (i >> 3);
        sl = sl < nsg ? sl : nsg - 1;                        // absent states: column dropped
        offP[t] = sl * kAnaVals + v;
        offH[t] = sl * kAnaVals + (has_h ? cH : v);
    }

    // Cooperative copy of each 16-latitude block of G (16 latitudes x 4 states x 14 values) into
    // LDS as FP64, all loads of a block issued before the previous block is consumed.  FP64 input:
    // 448 chunks of two values, thread tid moving chunks tid and tid + 256.  FP32 input (the FP32
    // mode stores the columns already rounded, which is what its MFMAs consume): 256 chunks of
    // four values, one per thread (a state's fourth chunk holds values 12, 13 and the row's two
    // pad zeros, which go to the dummy slot).  Idle threads write the dummy slot.
    // Forward input (fwd_index lines of 10 complex values, FP64 or FP32): 448 chunks of one complex
    // value, the seven of this parity's window per (latitude, state), two per thread, each stored
    // into its column's LDS slot.
    constexpr bool g64 = sizeof(TT) == 8;
    constexpr bool fwd = MODE == kAnaForward;
    constexpr int NC = (g64 || fwd) ? 2 : 1;                         // chunks per thread
    const size_t jstride = fwd ? fwd_index(g.T, S, 1, 0, 0) : ana_index(g.T, S, 1, 0, 0, 0);
    const TT* gsrc = G + (fwd ? fwd_index(g.T, S, 0, m, s0) : ana_index(g.T, S, 0, m, p, s0));
    int clat[NC], csrc[NC], cdst[NC], cdst2[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        if constexpr (fwd) {
            // chunk c: latitude c / 28 of the block, state cw / 7, window value cw % 7; the window
            // of parity p starts at value 3 p, and value v of it is column fwd_col[p][v]
            constexpr int fwd_col[2][7] = {{2, 3, 6, 0, 1, 5, 4}, {5, 4, 0, 1, 3, 6, 2}};
            const int c = tid + kBlock * k;
            int lat = c / (2 * kAnaVals), cw = c % (2 * kAnaVals);
            const bool ok = c < kAnaChunks && cw < nsg * (kAnaVals / 2);
            if (!ok) { lat = 0; cw = 0; }
            const int st = cw / (kAnaVals / 2), kv = cw % (kAnaVals / 2);
            clat[k] = lat;
            csrc[k] = st * 2 * kFwdVals + 2 * (3 * p + kv);
            cdst[k] = ok ? lat * kAnaLat + st * kAnaVals + 2 * fwd_col[p][kv] : kAnaBuf;
            cdst2[k] = 0;
        } else if constexpr (g64) {
            // chunk c: latitude c / 14 of the block, state cw / 7, values 2 (cw % 7), 2 (cw % 7) + 1
            const int c = tid + kBlock * k;
            int lat = c / (2 * kAnaVals), cw = c % (2 * kAnaVals);
            const bool ok = c < kAnaChunks && cw < nsg * (kAnaVals / 2);
            if (!ok) { lat = 0; cw = 0; }
            clat[k] = lat;
            csrc[k] = (cw / (kAnaVals / 2)) * kAnaStride + 2 * (cw % (kAnaVals / 2));
            cdst[k] = ok ? lat * kAnaLat + 2 * cw : kAnaBuf;
            cdst2[k] = 0;
        } else {
            // chunk tid: latitude tid / 16, state (tid / 4) % 4, values 4 (tid % 4) .. + 3
            const int st = (tid >> 2) & 3, kq = tid & 3;
            const bool ok = st < nsg;
            clat[k] = ok ? tid >> 4 : 0;
            csrc[k] = (ok ? st : 0) * kAnaStride + 4 * kq;
            cdst[k] = ok ? clat[k] * kAnaLat + st * kAnaVals + 4 * kq : kAnaBuf;
            cdst2[k] = ok && kq < 3 ? cdst[k] + 2 : kAnaBuf + 2;
        }
    }
    typedef typename std::conditional<g64, double2,
                                      typename std::conditional<fwd, float2, float4>::type>::type GV;
    auto gload = [&](GV (&r)[NC], int b) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            int jh = 16 * b + clat[k];
            jh = jh < g.nh ? jh : g.nh - 1;
            r[k] = *(const GV*)(gsrc + (size_t)jh * jstride + csrc[k]);
        }
    };
    // latitudes past nh are stored as zeros (their table entries are zero as well)
    // (no branches: a load sunk into a branch would wait for every load in flight)
    auto gstore = [&](const GV (&r)[NC], int b, int buf) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const bool live = 16 * b + clat[k] < g.nh;
            if constexpr (bf3) {
                v4u* gv = reinterpret_cast<v4u*>(gl[buf]);
                const v4u z = (v4u){0u, 0u, 0u, 0u};
                if constexpr (fwd) {
                    gv[cdst[k]] = live ? bf3_b(r[k].x) : z;
                    gv[cdst[k] + 1] = live ? bf3_b(r[k].y) : z;
                } else {
                    gv[cdst[k]] = live ? bf3_b(r[k].x) : z;
                    gv[cdst[k] + 1] = live ? bf3_b(r[k].y) : z;
                    gv[cdst2[k]] = live ? bf3_b(r[k].z) : z;
                    gv[cdst2[k] + 1] = live ? bf3_b(r[k].w) : z;
                }
            } else if constexpr (g64) {
                *(double2*)&gl[buf][cdst[k]] = live ? r[k] : make_double2(0.0, 0.0);
            } else if constexpr (fwd) {
                const double2 v2 = make_double2((double)r[k].x, (double)r[k].y);
                *(double2*)&gl[buf][cdst[k]] = live ? v2 : make_double2(0.0, 0.0);
            } else {
                const double2 lo = make_double2((double)r[k].x, (double)r[k].y);
                const double2 hi = make_double2((double)r[k].z, (double)r[k].w);
                *(double2*)&gl[buf][cdst[k]] = live ? lo : make_double2(0.0, 0.0);
                *(double2*)&gl[buf][cdst2[k]] = live ? hi : make_double2(0.0, 0.0);
            }
        }
    };

    vec accP[2] = {MM::zero(), MM::zero()}, accH[2] = {MM::zero(), MM::zero()};
    // REC: restart rows and recurrence coefficients of this lane group's four rows (rows past the
    // order's end restart at a stored row; their outputs are dropped)
    const double* rP0 = P64;
    const double* rPm = P64;
    size_t rPm_tile = 0;                                     // doubles per latitude tile
    bool rzero = false;
    double ca[8], cbb[8], cc[4], cd[4];
    if constexpr (REC) {
        const int kq = kt + 4 * q < np4 ? kt + 4 * q : np4 - 1;
        const int n0 = m + p + 2 * kq;
        rP0 = P64 + toff[2 * m + p] + tab_index(np4, kq, i);
        // Pbar_{n0-1}: parity 1, row kq - 1 (p = 0) or parity 0, row kq (p = 1); zero at n0 = m
        const int po = 1 - p;
        const int npo4 = (npk_of(g.T, m, po) + 3) & ~3;
        int ko = p == 0 ? kq - 1 : kq;
        rzero = ko < 0 || npo4 == 0;
        ko = ko < 0 ? 0 : (ko < npo4 ? ko : npo4 - 1);
        rPm = npo4 > 0 ? P64 + toff[2 * m + po] + tab_index(npo4, ko, i) : rP0;
        rPm_tile = (size_t)npo4 * 16;
        const double* c0 = rc + 4 * rec_index(g.T, m, n0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            ca[k] = c0[4 * k];
            cbb[k] = c0[4 * k + 1];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            cc[k] = c0[8 * k + 2];
            cd[k] = c0[8 * k + 3];
        }
    }
    double* trw = tr + (REC ? wave * kAnaTr : 0);
    auto load = [&](AnaStage<TT, REC>& x, int b) {
        if constexpr (REC) {
            const int jh = 16 * b + i;
            x.p0 = rP0[(size_t)b * bstride];
            x.pm1 = rzero ? 0.0 : rPm[(size_t)b * rPm_tile];
            x.mu = jh < g.nh ? mu[jh] : 0.0;
        } else {
            x.aP = *(const vec*)(Pr + b * bstride);
            x.aH = *(const vec*)(Hr + b * bstride);
        }
    };
    // k-step qq of a block contracts latitude 4 q + qq of the block (lane group q).  A group of
    // at most two states (a step's first f_E of one member) leaves the second column tile empty:
    // its products are skipped (NTL = 1), the first tile's are formed exactly as with four states.
    auto contract = [&](auto ntl, const vec& aP, const vec& aH, const double* lb) {
        constexpr int NTL = decltype(ntl)::value;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            if constexpr (bf3) {
                const v4u* lq = reinterpret_cast<const v4u*>(lb) + (4 * q + qq) * kAnaLat;
#pragma unroll
                for (int t = 0; t < NTL; ++t) {
                    accP[t] = MM::mma_pre(aP[qq], lq[offP[t]], accP[t]);
                    accH[t] = MM::mma_pre(aH[qq], lq[offH[t]], accH[t]);
                }
            } else {
                const double* lq = lb + (4 * q + qq) * kAnaLat;
#pragma unroll
                for (int t = 0; t < NTL; ++t) {
                    accP[t] = MM::mma(aP[qq], (TT)lq[offP[t]], accP[t]);
                    accH[t] = MM::mma(aH[qq], (TT)lq[offH[t]], accH[t]);   // dropped for kinds without H
                }
            }
        }
    };
    auto compute = [&](auto ntl, const AnaStage<TT, REC>& x, const double* lb) {
        if constexpr (REC) {
            double pm1 = x.pm1, p0 = x.p0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double p1 = leg_next(x.mu, p0, pm1, ca[2 * k], cbb[2 * k]);
                trw[(4 * q + k) * kAnaTrRow + i] = p0;
                trw[(16 + 4 * q + k) * kAnaTrRow + i] = leg_h(pm1, p1, cc[k], cd[k]);
                pm1 = p1;
                p0 = leg_next(x.mu, p1, p0, ca[2 * k + 1], cbb[2 * k + 1]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const double2* rp = reinterpret_cast<const double2*>(trw + i * kAnaTrRow + 4 * q);
            const double2* rh = reinterpret_cast<const double2*>(trw + (16 + i) * kAnaTrRow + 4 * q);
            const double2 p01 = rp[0], p23 = rp[1], h01 = rh[0], h23 = rh[1];
            vec aP, aH;
            aP[0] = (TT)p01.x; aP[1] = (TT)p01.y; aP[2] = (TT)p23.x; aP[3] = (TT)p23.y;
            aH[0] = (TT)h01.x; aH[1] = (TT)h01.y; aH[2] = (TT)h23.x; aH[3] = (TT)h23.y;
            contract(ntl, aP, aH, lb);
        } else {
            contract(ntl, x.aP, x.aH, lb);
        }
    };

    // The columns of block b + 2 are requested while block b is contracted, into the register set
    // that held block b (staged already); block b + 1, requested an iteration earlier, is staged
    // into LDS after the contraction.  Two register sets alternate with the block's parity (D is
    // even, so the set of block b0 + u is u & 1).
    GV gr[2][NC];
    gload(gr[0], 0);
    gload(gr[1], nb > 1 ? 1 : 0);
    gstore(gr[0], 0, 0);
    __syncthreads();
    static_assert(D % 2 == 0, "the column register sets alternate with the block parity");
    // NTL column tiles contracted: 2, or 1 for a group of at most two states (see contract)
    auto contract_blocks = [&](auto ntl) {
        AnaStage<TT, REC> st[D];
#pragma unroll
        for (int u = 0; u < D; ++u) load(st[u], u < nb ? u : nb - 1);
        int b0 = 0;
        for (; b0 + D <= nb; b0 += D) {
#pragma unroll
            for (int u = 0; u < D; ++u) {
                const int b = b0 + u;
                gload(gr[u & 1], b + 2 < nb ? b + 2 : nb - 1);
                compute(ntl, st[u], gl[b & 1]);
                const int bn = b + D;
                load(st[u], bn < nb ? bn : nb - 1);          // past the end: re-read, unused
                gstore(gr[(u + 1) & 1], b + 1, (b + 1) & 1);
                __syncthreads();
            }
        }
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int b = b0 + u;
            if (b < nb) {                                    // uniform
                gload(gr[u & 1], b + 2 < nb ? b + 2 : nb - 1);
                compute(ntl, st[u], gl[b & 1]);
                gstore(gr[(u + 1) & 1], b + 1, (b + 1) & 1);
                __syncthreads();
            }
        }
    };
    if (active) {
        if (nsg > 2) contract_blocks(std::integral_constant<int, 2>{});
        else contract_blocks(std::integral_constant<int, 1>{});
    } else {
        // rows past the order's end: this wave only helps move the columns
        for (int b = 0; b < nb; b += 2) {
            gload(gr[0], b + 2 < nb ? b + 2 : nb - 1);
            gstore(gr[1], b + 1, (b + 1) & 1);
            __syncthreads();
            if (b + 1 < nb) {                                // uniform
                gload(gr[1], b + 3 < nb ? b + 3 : nb - 1);
                gstore(gr[0], b + 2, (b + 2) & 1);
                __syncthreads();
            }
        }
        if (!fuse && !(MODE == kAnaAdjoint && af.mode)) return;   // uniform
    }

    // The Pbar columns of the forward input carry no factor i m: the Pbar parts of zeta_t
    // (-i m A), Phi'_t (-i m C) and delta_t (+i m B) are rotated here, each lane taking the other
    // part of its complex value from its partner lane i ^ 1.
    double pv[2][4];
    {
        const double rot = (re == 0 ? 1.0 : -1.0) * (kind == 1 ? -1.0 : 1.0) * (double)m;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double x = (double)accP[t][r];
                if constexpr (MODE == kAnaForward) {
                    const double y = __shfl_xor(x, 1, 64);
                    pv[t][r] = kind == 2 ? x : rot * y;
                } else {
                    pv[t][r] = x;
                }
            }
    }
    const int cb = coef_offset(g.T, m) - m;
    if constexpr (MODE == kAnaAdjoint) {
        if (af.mode) {
            // Fused epilogue of the transposed tendency: the accumulated adjoints of this block's
            // rows (earlier contributions + this one, the sum the unfused kernel stores) go to LDS
            // as [row][state][field][part]; then mode 1 applies the adjoint node update to every
            // (row, part, member) of the block (adj_update_part, the same arithmetic as the
            // adjoint update kernel; a group of four states holds 4 / M whole members), and mode
            // 2 writes the finished u_n adjoint of every member to lam_out.
            double* eb = reinterpret_cast<double*>(gl);          // 64 x 4 x 3 x 2 doubles
            const int kk0 = task.z;
            if (active) {
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int sl = 2 * t + (i >> 3);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double val = has_h ? (double)accP[t][r] + (double)accH[t][r] : (double)accP[t][r];
                        const double right = __shfl_down(val, 2, 64);
                        const int kk = kt + MM::row(r, q);
                        if (kk >= np || sl >= nsg || kind == 1) continue;
                        const int n = m + p + 2 * kk;
                        const int field = kind == 0 ? 1 : (kind == 2 ? 2 : 0);
                        const double res = kind == 0 ? val + nscale[n] * right : (kind == 2 ? nscale[n] * val : val);
                        const double tot = out[((size_t)((s0 + sl) * 3 + field) * g.ncoef + cb + n) * 2 + re] + res;
                        eb[(((kk - kk0) * 4 + sl) * 3 + field) * 2 + re] = tot;
                    }
                }
            }
            __syncthreads();
            if (af.mode == 1) {
                const int Mn = af.a.M;
                const int nmem = nsg / Mn, bfirst = s0 / Mn;
                for (int it = tid; it < 128 * nmem; it += kBlock) {
                    const int row = (it >> 1) & 63, c = it & 1, k = it >> 7;
                    const int kk = kk0 + row;
                    if (kk >= np) continue;
                    const int t2 = 2 * (cb + m + p + 2 * kk) + c;
                    auto ub = [&](int j, int f) { return eb[((row * 4 + k * Mn + j) * 3 + f) * 2 + c]; };
                    if (Mn == 1) adj_update_part<1>(af.a, t2, bfirst + k, ub);
                    else if (Mn == 2) adj_update_part<2>(af.a, t2, bfirst + k, ub);
                    else adj_update_part<4>(af.a, t2, bfirst + k, ub);
                }
            } else {
                for (int it = tid; it < 128 * nsg; it += kBlock) {
                    const int row = (it >> 1) & 63, c = it & 1, k = it >> 7;
                    const int kk = kk0 + row;
                    if (kk >= np) continue;
                    const int idx = cb + m + p + 2 * kk;
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        const double v = eb[((row * 4 + k) * 3 + f) * 2 + c];
                        af.lam_out[((size_t)((s0 + k) * 3 + f) * g.ncoef + idx) * 2 + c] = (m == 0 && c == 1) ? 0.0 : v;
                    }
                }
            }
            return;
        }
    }
    if constexpr (MODE == kAnaForward) {
        if (fuse) {
            // Fused node update of the next sweep (the tendencies never leave the workgroup): the
            // tendencies of this block's rows go to LDS as [row][state][field][part], then every
            // (row, part, member) of the block is updated from them (node_update_part, the same
            // arithmetic as the update kernel).  fuse = 1: the states are members (the step's
            // first f_E, E_j = E_0 for every node); fuse = 2: state b M + j is node j of member b
            // and a group of four states holds 4 / M whole members.
            double* eb = reinterpret_cast<double*>(gl);          // 64 x 4 x 3 x 2 doubles
            const int kk0 = task.z;
            if (active) {
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int sl = 2 * t + (i >> 3);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double val = has_h ? pv[t][r] + (double)accH[t][r] : pv[t][r];
                        const double right = __shfl_down(val, 2, 64);
                        const int kk = kt + MM::row(r, q);
                        if (kk >= np || sl >= nsg || kind == 2) continue;
                        const int n = m + p + 2 * kk;
                        const int field = kind == 0 ? 1 : (kind == 1 ? 2 : 0);
                        const double res = kind == 1 ? val + nscale[n] * right : val;
                        eb[(((kk - kk0) * 4 + sl) * 3 + field) * 2 + re] = res;
                    }
                }
            }
            __syncthreads();
            const int Mn = fu.M;
            const int nmem = fuse == 1 ? nsg : nsg / Mn;
            const int bfirst = fuse == 1 ? s0 : s0 / Mn;
            for (int it = tid; it < 128 * nmem; it += kBlock) {
                const int row = (it >> 1) & 63, c = it & 1, k = it >> 7;
                const int kk = kk0 + row;
                if (kk >= np) continue;
                const int idx = cb + m + p + 2 * kk;
                auto ep = [&](int j, int f) {
                    const int sl = fuse == 1 ? k : k * Mn + j;
                    return eb[((row * 4 + sl) * 3 + f) * 2 + c];
                };
                if (Mn == 1) node_update_part<1>(fu, idx, c, bfirst + k, ep);
                else if (Mn == 2) node_update_part<2>(fu, idx, c, bfirst + k, ep);
                else node_update_part<4>(fu, idx, c, bfirst + k, ep);
            }
            return;
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int s = s0 + 2 * t + (i >> 3);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double val = has_h ? pv[t][r] + (double)accH[t][r] : pv[t][r];
            const double right = __shfl_down(val, 2, 64);    // the kind one to the right
            const int kk = kt + MM::row(r, q);
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

template <int MODE, typename TT, int D, bool REC>
__global__ __launch_bounds__(kBlock) void k_analysis_swe(
    const TT* __restrict__ P, const TT* __restrict__ H, const long long* __restrict__ toff,
    const int4* __restrict__ tasks, int ntasks, int interleave, const TT* __restrict__ G,
    int nstates, const double* __restrict__ nscale, double* __restrict__ out, Geom g,
    UpdateArgs fu, int fuse, const double* __restrict__ P64, const double* __restrict__ rc,
    const double* __restrict__ mu, AdjFuse af) {
    analysis_body<MODE, TT, D, REC>(P, H, toff, tasks, ntasks, interleave, G, nstates, nscale, out, g, fu,
                                    fuse, P64, rc, mu, af, blockIdx.x);
}

// One forward analysis launch over several handles (workgroup ranges as k_synthesis_multi).
template <typename TT, int D, bool REC>
__global__ __launch_bounds__(kBlock) void k_analysis_multi(const AnaArgs* __restrict__ list, int n) {
    const int b = blockIdx.x;
    int h = 0;
    while (h + 1 < n && b >= list[h + 1].first) ++h;
    const AnaArgs& a = list[h];
    if (b - a.first >= a.blocks) return;                     // padding to the next range (uniform)
    const AdjFuse none{};
    analysis_body<kAnaForward, TT, D, REC>(
        static_cast<const TT*>(a.P), static_cast<const TT*>(a.H), a.toff, a.tasks, a.ntasks, a.interleave,
        static_cast<const TT*>(a.G), a.nstates, a.nscale, a.out, a.g, a.fu, a.fuse, a.P64, a.rc, a.mu, none,
        b - a.first);
}

AnaArgs make_ana_args(const Tables& tb, const LegPlan& plan, const long long* toff, const int4* tasks,
                      int nwg, const double* G, int nstates, const double* neg_lap, double* out,
                      const Geom& g, const UpdateArgs* fuse, int fuse_mode) {
    AnaArgs a{};
    a.P = tb.P32 ? (const void*)tb.P32 : (const void*)tb.P;
    a.H = tb.P32 ? (const void*)tb.H32 : (const void*)tb.H;
    a.toff = toff;
    a.tasks = tasks;
    a.ntasks = nwg;
    a.interleave = plan.ana_interleave;
    a.G = G;
    a.nstates = nstates;
    a.nscale = neg_lap;
    a.out = out;
    a.g = g;
    if (fuse) a.fu = *fuse;
    a.fuse = fuse ? fuse_mode : 0;
    a.P64 = tb.P;
    a.rc = tb.rc;
    a.mu = tb.mu;
    a.blocks = (int)xcd_grid(nwg, (nstates + 3) / 4);
    return a;
}

void launch_analysis_multi(const LegPlan& plan, int tt, const AnaArgs* list, int n, int blocks,
                           hipStream_t st) {
#define ANAM(TT, D, REC) k_analysis_multi<TT, D, REC><<<blocks, kBlock, 0, st>>>(list, n)
#define ANAM_PLAN(TT)                                                                             \
    do {                                                                                          \
        if (plan.ana_recur) {                                                                     \
            if (plan.ana_depth == 2) ANAM(TT, 2, true);                                           \
            else ANAM(TT, 4, true);                                                               \
        } else if (plan.ana_depth == 2) {                                                         \
            ANAM(TT, 2, false);                                                                   \
        } else {                                                                                  \
            ANAM(TT, 4, false);                                                                   \
        }                                                                                         \
    } while (0)
    if (tt == kTabBf3) ANAM_PLAN(Bf3);
    else if (tt == kTabF32) ANAM_PLAN(float);
    else ANAM_PLAN(double);
#undef ANAM_PLAN
#undef ANAM
}

// Analysis variants: D = 4 or 2 table stages in flight per wave; state groups interleaved per
// XCD or group-major.
template <int MODE, typename TT>
static void launch_analysis_variant(const LegPlan& plan, unsigned grid, hipStream_t st,
                                    const Tables& tb, const TT* P, const TT* H,
                                    const long long* toff, const int4* tasks, int nwg,
                                    const void* Gv, int nstates, const double* nscale, double* out,
                                    const Geom& g, const UpdateArgs& fu, int fuse, const AdjFuse& af) {
    const TT* G = static_cast<const TT*>(Gv);      // the analysis input is stored in the table type
#define ANA(D, REC)                                                                                 \
    k_analysis_swe<MODE, TT, D, REC><<<grid, kBlock, 0, st>>>(P, H, toff, tasks, nwg,               \
                                                              plan.ana_interleave, G, nstates,      \
                                                              nscale, out, g, fu, fuse, tb.P,       \
                                                              tb.rc, tb.mu, af)
    if (plan.ana_recur) {
        if (plan.ana_depth == 2) ANA(2, true);
        else ANA(4, true);
    } else if (plan.ana_depth == 2) {
        ANA(2, false);
    } else {
        ANA(4, false);
    }
#undef ANA
}

void launch_analysis_swe(const Tables& tb, const LegPlan& plan, const long long* toff,
                         const int4* tasks, int nwg, const double* G, int nstates,
                         const double* neg_lap, double* out, const Geom& g, hipStream_t st,
                         const UpdateArgs* fuse, int fuse_mode) {
    const unsigned grid = xcd_grid(nwg, (nstates + 3) / 4);
    const UpdateArgs none{};
    const UpdateArgs& fu = fuse ? *fuse : none;
    const int mode = fuse ? fuse_mode : 0;
    const AdjFuse noadj{};
    if (tb.P32 && tb.bf3)
        launch_analysis_variant<kAnaForward, Bf3>(plan, grid, st, tb, reinterpret_cast<const Bf3*>(tb.P32),
                                                  reinterpret_cast<const Bf3*>(tb.H32), toff, tasks, nwg, G,
                                                  nstates, neg_lap, out, g, fu, mode, noadj);
    else if (tb.P32)
        launch_analysis_variant<kAnaForward, float>(plan, grid, st, tb, tb.P32, tb.H32, toff, tasks, nwg, G,
                                                    nstates, neg_lap, out, g, fu, mode, noadj);
    else
        launch_analysis_variant<kAnaForward, double>(plan, grid, st, tb, tb.P, tb.H, toff, tasks, nwg, G,
                                                     nstates, neg_lap, out, g, fu, mode, noadj);
}

void launch_analysis_adjoint(const Tables& tb, const LegPlan& plan, const long long* toff,
                             const int4* tasks, int nwg, const double* G, int nstates,
                             const double* inv_lap, double* out_acc, const Geom& g, hipStream_t st,
                             const AdjFuse* fuse) {
    const unsigned grid = xcd_grid(nwg, (nstates + 3) / 4);
    const AdjFuse none{};
    const AdjFuse& af = fuse ? *fuse : none;
    if (tb.P32 && tb.bf3)
        launch_analysis_variant<kAnaAdjoint, Bf3>(plan, grid, st, tb, reinterpret_cast<const Bf3*>(tb.P32),
                                                  reinterpret_cast<const Bf3*>(tb.H32), toff, tasks, nwg, G,
                                                  nstates, inv_lap, out_acc, g, UpdateArgs{}, 0, af);
    else if (tb.P32)
        launch_analysis_variant<kAnaAdjoint, float>(plan, grid, st, tb, tb.P32, tb.H32, toff, tasks, nwg, G,
                                                    nstates, inv_lap, out_acc, g, UpdateArgs{}, 0, af);
    else
        launch_analysis_variant<kAnaAdjoint, double>(plan, grid, st, tb, tb.P, tb.H, toff, tasks, nwg, G,
                                                     nstates, inv_lap, out_acc, g, UpdateArgs{}, 0, af);
}

// FP32 copies of the FP64 tables (same layout), for the FP32 precision mode.
__global__ __launch_bounds__(kBlock) void k_round_tables(const double* __restrict__ P,
                                                          const double* __restrict__ H,
                                                          float* __restrict__ P32,
                                                          float* __restrict__ H32, long long n) {
    const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    P32[k] = (float)P[k];
    H32[k] = (float)H[k];
}

void launch_round_tables(const double* P, const double* H, float* P32, float* H32, long long n,
                         hipStream_t st) {
    k_round_tables<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(P, H, P32, H32, n);
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
        const double* Pp = P + toff[2 * m + p] + tab_index(np4, 0, jt * 16 + i);
        v4d c = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int kk0 = 0; kk0 < np4; kk0 += 4) {
            const int kk = kk0 + q;
            const int n = m + p + 2 * kk;
            const double ap = Pp[(size_t)kk * 16];
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
    const double* Pr = P + toff[2 * m + p] + tab_index(np4, rowok ? kr : 0, 4 * q);
    const int f = blockIdx.y * 8 + (i >> 1), re = i & 1;
    const bool okf = f < nfields;
    const size_t jstride = (size_t)2 * g.ms;
    const double* bp = (const double*)(ana + (size_t)(f * 2 + p) * g.nhp * g.ms + m) + re + 4 * q * jstride;
    v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
    const v4d zero4 = acc;
    for (int jh0 = 0; jh0 < g.nhp; jh0 += 16) {
        const v4d ap = rowok ? *(const v4d*)(Pr + (size_t)(jh0 >> 4) * np4 * 16) : zero4;
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
