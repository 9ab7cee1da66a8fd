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

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------------------------
// Synthesis for the shallow-water explicit tendency.  Per state the inputs are the spectral
// fields (Phi', zeta, delta); the outputs are the Fourier coefficients, at every latitude, of
//   zeta, Phi', U = (1/a) sum_n [i m chi Pbar - psi H], V = (1/a) sum_n [i m psi Pbar + chi H]
// with psi = -a^2 zeta/(n(n+1)) and chi = -a^2 delta/(n(n+1)) (zero at n = 0).
// Columns of one 16-wide Pbar tile: 2 states x (zeta, Phi', psi, chi) x (Re, Im);
// of the H tile: 4 states x (psi, chi) x (Re, Im).  A wave owns (m, one 16-latitude tile,
// 4 states) and runs over all degrees n of both parities.
// Task (m, latitude group of 4 tiles) per workgroup; blockIdx.y selects 4 states.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_synthesis_swe(
    const double* __restrict__ P, const double* __restrict__ H, const long long* __restrict__ toff,
    const int2* __restrict__ tasks, const double* __restrict__ state, int nstates,
    const double* __restrict__ inv_lap, double2* __restrict__ four, Geom g) {
    __shared__ double red[4][4][2][12][16];   // [wave][state][north/south][value][latitude]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int2 task = tasks[blockIdx.x];
    const int m = task.x;
    const int jt = task.y * 4 + wave;
    const int ntj = g.nhp >> 4;
    const int s0 = blockIdx.y * 4;
    const int i = lane & 15, q = lane >> 4;
    const bool active = jt < ntj;

    const int vP = i & 7, reP = vP & 1, kindP = vP >> 1;     // kind: 0 zeta 1 Phi' 2 psi 3 chi
    const int vH = i & 3, reH = vH & 1, kindH = vH >> 1;     // kind: 0 psi 1 chi
    v4d accP[2][2], accH[2];
    for (int p = 0; p < 2; ++p) {
        accP[p][0] = accP[p][1] = accH[p] = (v4d){0.0, 0.0, 0.0, 0.0};
    }
    if (active) {
        const int fieldP = (kindP == 1) ? 0 : ((kindP == 3) ? 2 : 1);
        const bool scaleP = kindP >= 2;
        const int fieldH = kindH == 0 ? 1 : 2;
        const int cb = coef_offset(g.T, m) - m;
        const int sP0 = s0 + (i >> 3), sP1 = s0 + 2 + (i >> 3), sH = s0 + (i >> 2);
        const double* bp0 = state + ((size_t)(sP0 * 3 + fieldP) * g.ncoef + cb) * 2 + reP;
        const double* bp1 = state + ((size_t)(sP1 * 3 + fieldP) * g.ncoef + cb) * 2 + reP;
        const double* bph = state + ((size_t)(sH * 3 + fieldH) * g.ncoef + cb) * 2 + reH;
        const bool ok0 = sP0 < nstates, ok1 = sP1 < nstates, okh = sH < nstates;
        for (int p = 0; p < 2; ++p) {
            const int np = npk_of(g.T, m, p);
            const int np4 = (np + 3) & ~3;
            const double* Pp = P + toff[2 * m + p] + jt * 16 + i;
            const double* Hp = H + toff[2 * m + p] + jt * 16 + i;
            v4d c0 = accP[p][0], c1 = accP[p][1], ch = accH[p];
#pragma unroll 4
            for (int kk0 = 0; kk0 < np4; kk0 += 4) {
                const int kk = kk0 + q;
                const int n = m + p + 2 * kk;
                const bool vn = kk < np;
                const double ap = Pp[(size_t)kk * g.nhp];
                const double ah = Hp[(size_t)kk * g.nhp];
                const double il = vn ? inv_lap[n] : 0.0;
                double b0 = (vn && ok0) ? bp0[2 * n] : 0.0;
                double b1 = (vn && ok1) ? bp1[2 * n] : 0.0;
                const double bh = (vn && okh) ? bph[2 * n] * il : 0.0;
                if (scaleP) { b0 *= il; b1 *= il; }
                c0 = mfma_f64(ap, b0, c0);
                c1 = mfma_f64(ap, b1, c1);
                ch = mfma_f64(ah, bh, ch);
            }
            accP[p][0] = c0;
            accP[p][1] = c1;
            accH[p] = ch;
        }
        // north = even + odd; south = even - odd (Pbar) and odd - even (H)
        for (int r = 0; r < 4; ++r) {
            const int latl = 4 * r + q;
            for (int t = 0; t < 2; ++t) {
                const double e = accP[0][t][r], o = accP[1][t][r];
                const int sl = 2 * t + (i >> 3);
                red[wave][sl][0][vP][latl] = e + o;
                red[wave][sl][1][vP][latl] = e - o;
            }
            const double e = accH[0][r], o = accH[1][r];
            red[wave][i >> 2][0][8 + vH][latl] = e + o;
            red[wave][i >> 2][1][8 + vH][latl] = o - e;
        }
    }
    __syncthreads();
    if (!active) return;
    const double inva = 1.0 / g.radius;
    const double mm = (double)m;
    const size_t fstride = (size_t)g.nlat * g.ms;
    for (int it = lane; it < 128; it += 64) {
        const int sl = it >> 5, ns = (it >> 4) & 1, latl = it & 15;
        const int s = s0 + sl, jh = jt * 16 + latl;
        if (s >= nstates || jh >= g.nh) continue;
        const double* v = &red[wave][sl][ns][0][latl];
        const double2 zeta = make_double2(v[0 * 16], v[1 * 16]);
        const double2 phi = make_double2(v[2 * 16], v[3 * 16]);
        const double ppr = v[4 * 16], ppi = v[5 * 16];       // Pbar psi
        const double pcr = v[6 * 16], pci = v[7 * 16];       // Pbar chi
        const double hpr = v[8 * 16], hpi = v[9 * 16];       // H psi
        const double hcr = v[10 * 16], hci = v[11 * 16];     // H chi
        const double2 U = make_double2((-mm * pci - hpr) * inva, (mm * pcr - hpi) * inva);
        const double2 V = make_double2((-mm * ppi + hcr) * inva, (mm * ppr + hci) * inva);
        const int j = ns ? g.nlat - 1 - jh : jh;
        double2* base = four + ((size_t)s * kSynFields * g.nlat + j) * g.ms + m;
        base[0] = zeta;
        base[fstride] = phi;
        base[2 * fstride] = U;
        base[3 * fstride] = V;
    }
}

void launch_synthesis_swe(const double* P, const double* H, const long long* toff,
                          const int2* tasks, int ntasks, const double* state, int nstates,
                          const double* inv_lap, double2* four, const Geom& g, hipStream_t st) {
    dim3 grid(ntasks, (nstates + 3) / 4);
    k_synthesis_swe<<<grid, kBlock, 0, st>>>(P, H, toff, tasks, state, nstates, inv_lap, four, g);
}

// ---------------------------------------------------------------------------------------------
// Analysis for the shallow-water explicit tendency.  Input: per state and parity p the seven
// weighted Fourier columns produced by the grid kernel (already combined into the north +- south
// sums that pair with Pbar and H of that parity).  Output per state:
//   d zeta/dt = Pbar.col0 + H.col4, d delta/dt = Pbar.col1 + H.col5 + n(n+1)/a^2 Pbar.col2,
//   d Phi'/dt = Pbar.col3 + H.col6.
// A wave owns (m, parity, 16 consecutive rows n, 4 states) and contracts over all latitudes
// (uniform work per wave).  Tile columns: 2 states x (zeta, delta, KE, Phi') x (Re, Im).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_analysis_swe(
    const double* __restrict__ P, const double* __restrict__ H, const long long* __restrict__ toff,
    const int4* __restrict__ tasks, int ntasks, const double2* __restrict__ ana, int nstates,
    const double* __restrict__ neg_lap, double* __restrict__ out, Geom g) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tid = blockIdx.x * 4 + wave;
    if (tid >= ntasks) return;
    const int4 task = tasks[tid];
    const int m = task.x, p = task.y, kk0 = task.z;
    const int np = npk_of(g.T, m, p);
    const int np4 = (np + 3) & ~3;
    const int s0 = blockIdx.y * 4;
    const int i = lane & 15, q = lane >> 4;
    const int kr = kk0 + i;
    const bool rowok = kr < np4;
    const double* Pr = P + toff[2 * m + p] + (size_t)(rowok ? kr : 0) * g.nhp + 4 * q;
    const double* Hr = H + toff[2 * m + p] + (size_t)(rowok ? kr : 0) * g.nhp + 4 * q;

    const int v = i & 7, re = v & 1, kind = v >> 1;           // kind: 0 zeta 1 delta 2 KE 3 Phi'
    const int cH = kind == 0 ? 4 : (kind == 1 ? 5 : 6);
    const size_t jstride = (size_t)2 * g.ms;                   // doubles per latitude row
    const double* bP[2];
    const double* bH[2];
    bool okP[2], okH[2];
    for (int t = 0; t < 2; ++t) {
        const int s = s0 + 2 * t + (i >> 3);
        okP[t] = s < nstates;
        okH[t] = okP[t] && kind != 2;
        const size_t colbase = (size_t)(s * 2 + p) * kAnaCols;
        bP[t] = (const double*)(ana + (colbase + kind) * g.nhp * g.ms + m) + re + 4 * q * jstride;
        bH[t] = (const double*)(ana + (colbase + cH) * g.nhp * g.ms + m) + re + 4 * q * jstride;
    }
    v4d acc0 = (v4d){0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    const v4d zero4 = acc0;
    for (int jh0 = 0; jh0 < g.nhp; jh0 += 16) {
        const v4d ap = rowok ? *(const v4d*)(Pr + jh0) : zero4;
        const v4d ah = rowok ? *(const v4d*)(Hr + jh0) : zero4;
        const size_t o = (size_t)jh0 * jstride;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const size_t oo = o + qq * jstride;
            const bool jok = jh0 + 4 * q + qq < g.nh;      // padded latitude rows are never read
            const double p0 = (jok && okP[0]) ? bP[0][oo] : 0.0;
            const double h0 = (jok && okH[0]) ? bH[0][oo] : 0.0;
            const double p1 = (jok && okP[1]) ? bP[1][oo] : 0.0;
            const double h1 = (jok && okH[1]) ? bH[1][oo] : 0.0;
            acc0 = mfma_f64(ap[qq], p0, acc0);
            acc0 = mfma_f64(ah[qq], h0, acc0);
            acc1 = mfma_f64(ap[qq], p1, acc1);
            acc1 = mfma_f64(ah[qq], h1, acc1);
        }
    }
    const int cb = coef_offset(g.T, m) - m;
    for (int t = 0; t < 2; ++t) {
        const int s = s0 + 2 * t + (i >> 3);
        for (int r = 0; r < 4; ++r) {
            const double val = t == 0 ? acc0[r] : acc1[r];
            const double ke = __shfl_down(val, 2, 64);      // KE column sits two lanes to the right
            const int kk = kk0 + 4 * r + q;
            if (kk >= np || s >= nstates || kind == 2) continue;
            const int n = m + p + 2 * kk;
            const int field = kind == 0 ? 1 : (kind == 1 ? 2 : 0);
            const double res = kind == 1 ? val + neg_lap[n] * ke : val;
            out[((size_t)(s * 3 + field) * g.ncoef + cb + n) * 2 + re] = res;
        }
    }
}

void launch_analysis_swe(const double* P, const double* H, const long long* toff,
                         const int4* tasks, int ntasks, const double2* ana, int nstates,
                         const double* neg_lap, double* out, const Geom& g, hipStream_t st) {
    dim3 grid((ntasks + 3) / 4, (nstates + 3) / 4);
    k_analysis_swe<<<grid, kBlock, 0, st>>>(P, H, toff, tasks, ntasks, ana, nstates, neg_lap, out, g);
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
