// Longitude FFTs in LDS and the fused grid-space step of the explicit tendency.
//
// Each workgroup owns one pair of mirror latitudes (north j, south nlat-1-j).  A real field on
// the two rows is carried as one complex signal z = north + i south, so one complex FFT of
// length nlon serves both rows.  The FFT is a Stockham autosort transform with radices 3, 16, 8,
// 4 and 2 (nlon = 2^p or 3*2^p), one LDS buffer per signal (values staged in registers between
// the read and write halves of a stage).  In the shallow-water grid kernels each signal is carried
// through all stages by one wave without workgroup barriers; the scalar transforms advance all
// signals of a workgroup together.  Radix 16 and 8 stages keep the number of LDS passes low
// (nlon = 768 = 3 x 16 x 16).
#include "common.h"

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// multiply by -i (forward) or +i (inverse)
__device__ __forceinline__ double2 cmul_mi(double2 a, bool inv) {
    return inv ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

template <int R>
__device__ __forceinline__ void dft_small(double2 (&v)[R], bool inv) {
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        // X1,2 = v0 - (v1+v2)/2 +- s i (sqrt3/2)(v1 - v2), s = -1 forward, +1 inverse
        const double c = 0.86602540378443864676;
        const double2 t1 = cadd(v[1], v[2]);
        const double2 t2 = make_double2(v[0].x - 0.5 * t1.x, v[0].y - 0.5 * t1.y);
        const double2 d = csub(v[1], v[2]);
        const double2 t3 = inv ? make_double2(-c * d.y, c * d.x) : make_double2(c * d.y, -c * d.x);
        v[0] = cadd(v[0], t1);
        v[1] = cadd(t2, t3);
        v[2] = csub(t2, t3);
    } else if constexpr (R == 4) {
        const double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        const double2 a2 = cadd(v[1], v[3]), a3 = cmul_mi(csub(v[1], v[3]), inv);
        v[0] = cadd(a0, a2);
        v[2] = csub(a0, a2);
        v[1] = cadd(a1, a3);
        v[3] = csub(a1, a3);
    } else if constexpr (R == 16) {
        // 16 = 4 x 4: DFT4 over n1 of v[4 n1 + n2], twiddles W16^{n2 k1}, DFT4 over n2
        constexpr double C[10] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                                  0.38268343236508977173, 0.0, -0.38268343236508977173,
                                  -0.70710678118654752440, -0.92387953251128675613, -1.0,
                                  -0.92387953251128675613};
        constexpr double Sn[10] = {0.0, 0.38268343236508977173, 0.70710678118654752440,
                                   0.92387953251128675613, 1.0, 0.92387953251128675613,
                                   0.70710678118654752440, 0.38268343236508977173, 0.0,
                                   -0.38268343236508977173};
        const double sg = inv ? 1.0 : -1.0;
        double2 y[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            double2 t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
            dft_small<4>(t, inv);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) {
                const int j = n2 * k1;
                y[n2][k1] = j == 0 ? t[k1] : cmul(t[k1], make_double2(C[j], sg * Sn[j]));
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            double2 t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
            dft_small<4>(t, inv);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
        }
    } else if constexpr (R == 8) {
        // two radix-4 DFTs on even and odd inputs, combined with the eighth roots of unity
        double2 e[4] = {v[0], v[2], v[4], v[6]};
        double2 o[4] = {v[1], v[3], v[5], v[7]};
        dft_small<4>(e, inv);
        dft_small<4>(o, inv);
        const double r = 0.70710678118654752440;
        const double sg = inv ? 1.0 : -1.0;
        const double2 w1 = make_double2(r, sg * r), w3 = make_double2(-r, sg * r);
        const double2 o1 = cmul(o[1], w1), o2 = cmul_mi(o[2], inv), o3 = cmul(o[3], w3);
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
}

// Compile-time FFT plans for the supported lengths (radix-3 stage first, then radices 16/8/4/2;
// a pass advances up to fft_fchunk(N) of a workgroup's signals so that every stage stages at
// most fft_task_cap(R) butterflies per thread).  The host accepts exactly these lengths.
constexpr int fft_nst(int n) {
    switch (n) {
        case 16: return 1;
        case 24: case 48: case 32: case 64: case 128: case 256: return 2;
        case 96: case 192: case 384: case 768: case 512: return 3;
        case 1536: case 1024: case 2048: return 4;
        default: return 0;
    }
}
constexpr int fft_fchunk(int n) { return n == 1536 ? 4 : (n == 2048 ? 3 : 5); }
constexpr int fft_radix(int n, int s) {
    switch (n) {
        case 24: return s == 0 ? 3 : 8;
        case 48: return s == 0 ? 3 : 16;
        case 96: return s == 0 ? 3 : (s == 1 ? 16 : 2);
        case 192: return s == 0 ? 3 : (s == 1 ? 16 : 4);
        case 384: return s == 0 ? 3 : (s == 1 ? 16 : 8);
        case 768: return s == 0 ? 3 : 16;
        case 1536: return s == 0 ? 3 : 8;
        case 16: return 16;
        case 32: return s == 0 ? 16 : 2;
        case 64: return s == 0 ? 16 : 4;
        case 128: return s == 0 ? 16 : 8;
        case 256: return 16;
        case 512: return s < 2 ? 16 : 2;
        case 1024: return s < 3 ? 8 : 2;
        case 2048: return s < 3 ? 8 : 4;
        default: return 0;
    }
}

// One Stockham stage of radix R on F <= fft_fchunk(N) signals of length N at buf + f*N.  Task t
// of the workgroup is butterfly j = t mod (N/R) of signal f = t div (N/R); it reads x[j + r N/R],
// applies twiddles w^(r k), k = j mod NS, w = e^{-+2 pi i/(NS R)}, and writes
// y[(j/NS) NS R + k + r NS].  Up to MAXT tasks per thread are held in registers between the read
// and the write half (one LDS buffer per signal).
template <int R, int N, int NS, int MAXT, bool INV>
__device__ __forceinline__ void fft_stage(double2* buf, int F, const double2* tw) {
    constexpr int nb = N / R;
    constexpr int tstep = N / (NS * R);
    const int ntask = F * nb;
    double2 v[MAXT][R];
#pragma unroll
    for (int tt = 0; tt < MAXT; ++tt) {
        const int t = threadIdx.x + tt * kBlock;
        if (t < ntask) {
            const int f = t / nb, j = t - f * nb, k = j % NS;
            const double2* src = buf + f * N + j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[tt][r] = src[r * nb];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                double2 w = tw[r * k * tstep];
                if (INV) w.y = -w.y;
                v[tt][r] = cmul(v[tt][r], w);
            }
            dft_small<R>(v[tt], INV);
        }
    }
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < MAXT; ++tt) {
        const int t = threadIdx.x + tt * kBlock;
        if (t < ntask) {
            const int f = t / nb, j = t - f * nb, k = j % NS;
            double2* dst = buf + f * N + (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[r * NS] = v[tt][r];
        }
    }
    __syncthreads();
}

template <int N, int S, int NS, bool INV>
__device__ __forceinline__ void fft_stages(double2* buf, int F, const double2* tw) {
    if constexpr (S < fft_nst(N)) {
        constexpr int R = fft_radix(N, S);
        constexpr int MAXT = (fft_fchunk(N) * (N / R) + kBlock - 1) / kBlock;
        static_assert(MAXT <= fft_task_cap(R), "FFT stage exceeds the per-thread task budget");
        fft_stage<R, N, NS, MAXT, INV>(buf, F, tw);
        fft_stages<N, S + 1, NS * R, INV>(buf, F, tw);
    }
}

// Unnormalised DFT of F signals of length N in LDS: forward X_k = sum x_n e^{-2 pi i nk/N},
// inverse with +.
template <int N, bool INV>
__device__ __forceinline__ void fft_lds(double2* buf, int F, const double2* tw) {
    constexpr int FC = fft_fchunk(N);
    for (int f0 = 0; f0 < F; f0 += FC) fft_stages<N, 0, 1, INV>(buf + f0 * N, F - f0 < FC ? F - f0 : FC, tw);
}

// Wave-level transforms: one wave (64 lanes) carries one signal through every stage with no
// workgroup barrier.  The LDS operations of a wave execute in issue order, so all reads of a stage
// are done before its writes; the fences keep the compiler from moving LDS accesses across the
// read/write boundary (other lanes' data is involved).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Twiddle powers w^r, r = 1..R-1, from w^1 by a product tree (w^r = w^h w^(r-h), h the largest
// power of two <= r): log2(R) dependent products instead of R - 2.  The products add a few ulps,
// far below the transform's own rounding.
constexpr int pow2_floor(int r) { return r >= 8 ? 8 : (r >= 4 ? 4 : (r >= 2 ? 2 : 1)); }
template <int R>
__device__ __forceinline__ void twiddle_powers(double2 (&wr)[R], double2 w1) {
    wr[1] = w1;
#pragma unroll
    for (int r = 2; r < R; ++r) {
        const int h = pow2_floor(r);
        wr[r] = h == r ? cmul(wr[r / 2], wr[r / 2]) : cmul(wr[h], wr[r - h]);
    }
}

// Per-lane first twiddles of the wave transforms: for stage S and the lane's butterfly tt,
// w^k = tw[k tstep] with k = j mod NS (stage 0, NS = 1, needs none).  Loaded once per kernel so
// that no stage waits on a memory load; the inverse transforms conjugate them.
constexpr int kWaveMaxT = 8;
template <int N> using WaveTw = double2[fft_nst(N) > 0 ? fft_nst(N) : 1][kWaveMaxT];

template <int N, int S, int NS>
__device__ __forceinline__ void wave_tw_load(WaveTw<N>& w, const double2* __restrict__ tw, int lane) {
    if constexpr (S < fft_nst(N)) {
        constexpr int R = fft_radix(N, S), nb = N / R, MAXT = (nb + 63) / 64;
        constexpr int tstep = N / (NS * R);
        if constexpr (NS > 1) {
            static_assert(MAXT <= kWaveMaxT, "wave FFT stage exceeds the per-lane butterfly budget");
#pragma unroll
            for (int tt = 0; tt < MAXT; ++tt) {
                const int j = lane + 64 * tt;
                w[S][tt] = tw[(j < nb ? j % NS : 0) * tstep];
            }
        }
        wave_tw_load<N, S + 1, NS * R>(w, tw, lane);
    }
}

template <int R, int N, int NS, bool INV>
__device__ __forceinline__ void fft_wave_stage(double2* buf, const double2 (&w1s)[kWaveMaxT], int lane) {
    constexpr int nb = N / R;
    constexpr int MAXT = (nb + 63) / 64;
    double2 v[MAXT][R];
#pragma unroll
    for (int tt = 0; tt < MAXT; ++tt) {
        const int j = lane + 64 * tt;
        if (j < nb) {
            const double2* src = buf + j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[tt][r] = src[r * nb];
            if constexpr (NS > 1) {                       // first stage: all twiddles are 1
                double2 w1 = w1s[tt];
                if (INV) w1.y = -w1.y;
                double2 wr[R];
                twiddle_powers<R>(wr, w1);
#pragma unroll
                for (int r = 1; r < R; ++r) v[tt][r] = cmul(v[tt][r], wr[r]);
            }
            dft_small<R>(v[tt], INV);
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int tt = 0; tt < MAXT; ++tt) {
        const int j = lane + 64 * tt, k = j % NS;
        if (j < nb) {
            double2* dst = buf + (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[r * NS] = v[tt][r];
        }
    }
    wave_lds_sync();
}

template <int N, int S, int NS, bool INV>
__device__ __forceinline__ void fft_wave_stages(double2* buf, const WaveTw<N>& w, int lane) {
    if constexpr (S < fft_nst(N)) {
        constexpr int R = fft_radix(N, S);
        fft_wave_stage<R, N, NS, INV>(buf, w[S], lane);
        fft_wave_stages<N, S + 1, NS * R, INV>(buf, w, lane);
    }
}

// Unnormalised DFT of the signal of length N at buf by the calling wave alone (twiddles from
// wave_tw_load).
template <int N, bool INV>
__device__ __forceinline__ void fft_wave(double2* buf, const WaveTw<N>& w, int lane) {
    fft_wave_stages<N, 0, 1, INV>(buf, w, lane);
}

constexpr int kGridBlock = 256;               // four waves: one per LDS signal
constexpr int kGridSignals = 4;                 // LDS signal buffers of the grid kernels

// Workgroup-wide transform of ONE signal by all kGridBlock threads (barriers between stages), for
// the signal the grid kernels cannot give a wave of its own.  Plan: radix 3 when 3 | N, then
// radix 4 stages and a last radix 2 when needed, so that most stages give every thread a
// butterfly (768 = 3 x 4^4: 256 then 192 butterflies per stage).
constexpr int fftb_nst(int n) {
    int s = 0;
    if (n % 3 == 0) { n /= 3; ++s; }
    while (n % 4 == 0) { n /= 4; ++s; }
    return s + (n == 2 ? 1 : 0);
}
constexpr int fftb_radix(int n, int s) {
    return (n % 3 == 0) ? (s == 0 ? 3 : fftb_radix(n / 3, s - 1))
                        : (n % 4 == 0 ? (s == 0 ? 4 : fftb_radix(n / 4, s - 1)) : 2);
}
constexpr int kBlockMaxT = 4;
template <int N> using BlockTw = double2[fftb_nst(N)][kBlockMaxT];

template <int N, int S, int NS>
__device__ __forceinline__ void block_tw_load(BlockTw<N>& w, const double2* __restrict__ tw) {
    if constexpr (S < fftb_nst(N)) {
        constexpr int R = fftb_radix(N, S), nb = N / R;
        constexpr int MAXT = (nb + kGridBlock - 1) / kGridBlock, tstep = N / (NS * R);
        if constexpr (NS > 1) {
            static_assert(MAXT <= kBlockMaxT, "block FFT stage exceeds the per-thread budget");
#pragma unroll
            for (int tt = 0; tt < MAXT; ++tt) {
                const int j = threadIdx.x + kGridBlock * tt;
                w[S][tt] = tw[(j < nb ? j % NS : 0) * tstep];
            }
        }
        block_tw_load<N, S + 1, NS * R>(w, tw);
    }
}

template <int R, int N, int NS, bool INV>
__device__ __forceinline__ void fft_block_stage(double2* buf, const double2 (&w1s)[kBlockMaxT]) {
    constexpr int nb = N / R;
    constexpr int MAXT = (nb + kGridBlock - 1) / kGridBlock;
    double2 v[MAXT][R];
#pragma unroll
    for (int tt = 0; tt < MAXT; ++tt) {
        const int j = threadIdx.x + kGridBlock * tt;
        if (j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[tt][r] = buf[j + r * nb];
            if constexpr (NS > 1) {
                double2 w1 = w1s[tt];
                if (INV) w1.y = -w1.y;
                double2 wr[R];
                twiddle_powers<R>(wr, w1);
#pragma unroll
                for (int r = 1; r < R; ++r) v[tt][r] = cmul(v[tt][r], wr[r]);
            }
            dft_small<R>(v[tt], INV);
        }
    }
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < MAXT; ++tt) {
        const int j = threadIdx.x + kGridBlock * tt, k = j % NS;
        if (j < nb) {
            double2* dst = buf + (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[r * NS] = v[tt][r];
        }
    }
    __syncthreads();
}

template <int N, int S, int NS, bool INV>
__device__ __forceinline__ void fft_block_stages(double2* buf, const BlockTw<N>& w) {
    if constexpr (S < fftb_nst(N)) {
        constexpr int R = fftb_radix(N, S);
        fft_block_stage<R, N, NS, INV>(buf, w[S]);
        fft_block_stages<N, S + 1, NS * R, INV>(buf, w);
    }
}

// Unnormalised DFT of the signal at buf by the whole workgroup (every thread must call it; the
// caller synchronises before, the last stage ends with a barrier).
template <int N, bool INV>
__device__ __forceinline__ void fft_block(double2* buf, const BlockTw<N>& w) {
    fft_block_stages<N, 0, 1, INV>(buf, w);
}

bool fft_length_supported(int n) { return fft_nst(n) > 0; }

// calls BODY(N) with N the compile-time FFT length equal to the runtime value n
#define FFT_DISPATCH(n, BODY)                                                       \
    switch (n) {                                                                    \
        case 16: BODY(16); break;     case 24: BODY(24); break;                     \
        case 32: BODY(32); break;     case 48: BODY(48); break;                     \
        case 64: BODY(64); break;     case 96: BODY(96); break;                     \
        case 128: BODY(128); break;   case 192: BODY(192); break;                   \
        case 256: BODY(256); break;   case 384: BODY(384); break;                   \
        case 512: BODY(512); break;   case 768: BODY(768); break;                   \
        case 1024: BODY(1024); break; case 1536: BODY(1536); break;                 \
        case 2048: BODY(2048); break; default: break;                               \
    }

// Hermitian spectrum of the pair (north X, south Y) for the inverse transform of z = x + i y:
// W_0 = Re X_0 + i Re Y_0, W_m = X_m + i Y_m and W_{N-m} = conj(X_m) + i conj(Y_m) for 1<=m<=T.
__device__ __forceinline__ double2 pack_pair(const double2* __restrict__ xn, const double2* __restrict__ ys,
                                             int k, int N, int T) {
    if (k == 0) return make_double2(xn[0].x, ys[0].x);
    if (k <= T) {
        const double2 X = xn[k], Y = ys[k];
        return make_double2(X.x - Y.y, X.y + Y.x);
    }
    if (k >= N - T) {
        const double2 X = xn[N - k], Y = ys[N - k];
        return make_double2(X.x + Y.y, -X.y + Y.x);
    }
    return make_double2(0.0, 0.0);
}

// Split the forward transform W of z = a + i b: A_m = (W_m + conj W_{N-m})/2, B_m = (W_m - conj W_{N-m})/(2i)
__device__ __forceinline__ void unpack_pair(const double2* buf, int m, int N, double2& A, double2& B) {
    const double2 w = buf[m], c = buf[m == 0 ? 0 : N - m];
    A = make_double2(0.5 * (w.x + c.x), 0.5 * (w.y - c.y));
    B = make_double2(0.5 * (w.y + c.y), -0.5 * (w.x - c.x));
}

// The packed spectra (pack_pair) of F Fourier fields of one latitude pair, staged into LDS with
// all global loads of a chunk issued before its LDS stores (one memory round trip per chunk of
// 3 x kGridBlock points instead of one per field and point).

template <int N, int F>
__device__ __forceinline__ void stage_inputs(double2* buf, const double2* __restrict__ fs,
                                             size_t fstride, int jN, int jS, int T, int ms) {
    constexpr int KP = 3;
    for (int k0 = 0; k0 < N; k0 += KP * kGridBlock) {
        double2 xv[F][KP], yv[F][KP];
        int src[KP];
#pragma unroll
        for (int kk = 0; kk < KP; ++kk) {
            const int k = k0 + threadIdx.x + kk * kGridBlock;
            const int kc = k < N ? k : 0;
            src[kk] = kc <= T ? kc : (kc >= N - T ? N - kc : 0);
        }
#pragma unroll
        for (int f = 0; f < F; ++f)
#pragma unroll
            for (int kk = 0; kk < KP; ++kk) {
                xv[f][kk] = fs[f * fstride + (size_t)jN * ms + src[kk]];
                yv[f][kk] = fs[f * fstride + (size_t)jS * ms + src[kk]];
            }
#pragma unroll
        for (int kk = 0; kk < KP; ++kk) {
            const int k = k0 + threadIdx.x + kk * kGridBlock;
            if (k >= N) continue;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const double2 X = xv[f][kk], Y = yv[f][kk];
                double2 z;
                if (k == 0) z = make_double2(X.x, Y.x);
                else if (k <= T) z = make_double2(X.x - Y.y, X.y + Y.x);
                else if (k >= N - T) z = make_double2(X.x + Y.y, -X.y + Y.x);
                else z = make_double2(0.0, 0.0);
                buf[f * N + k] = z;
            }
        }
    }
}

// One row (16 values) of the analysis input, written as complex pairs: FP64, or FP32 in the FP32
// mode, whose analysis MFMAs consume the values rounded to FP32 anyway (storing them rounded
// changes no result and halves the bytes).
template <typename GT> struct Row;
template <> struct Row<double> {
    double2* p;
    __device__ Row(double* G, size_t off) : p(reinterpret_cast<double2*>(G + off)) {}
    __device__ void put(int k, double2 v) const { p[k] = v; }
};
template <> struct Row<float> {
    float2* p;
    __device__ Row(float* G, size_t off) : p(reinterpret_cast<float2*>(G + off)) {}
    __device__ void put(int k, double2 v) const { p[k] = make_float2((float)v.x, (float)v.y); }
};

// ---------------------------------------------------------------------------------------------
// Fused grid step of f_E for one latitude pair of one state:
//   inverse FFT of zeta, Phi', U, V -> grid products
//   A = (zeta+f) U, B = (zeta+f) V, C = Phi' U, D = Phi' V, E = (U^2+V^2)/(2(1-mu^2))
//   -> forward FFT -> analysis input: the north + south and north - south sums of g A, g B,
//   g C, g D and w E (g = w / (a (1-mu^2)), Fourier coefficients normalised by 1/nlon), one line
//   of 10 complex values per (latitude pair, m, state) (fwd_index).
// Workgroup b runs on XCD b % 8; each XCD takes a contiguous range of (latitude, state) tasks,
// states fastest, so the rows of the analysis input meet in one L2.  Each of the first eight
// signals is transformed by one wave; only the hand-offs between phases are workgroup barriers.
// LDS holds four signals (three workgroups fit a CU), and every thread loads the first twiddles
// of its butterflies once, ahead of their use: the fifth product E waits in registers while A..D are
// transformed, then reuses buffer 0 (A's contributions to the lines wait in registers) and is
// transformed by the whole workgroup; each analysis-input line (10 complex values) is then
// written whole by one thread.
// ---------------------------------------------------------------------------------------------
template <int N, typename GT>
__device__ __forceinline__ void grid_swe_body(
    const double2* __restrict__ four, GT* __restrict__ G, const double* __restrict__ mu,
    const double* __restrict__ w, const double2* __restrict__ tw, double two_omega,
    int nstates, double2* __restrict__ save, const Geom& g, int bx) {
    extern __shared__ double2 buf[];      // kGridSignals signals x N
    constexpr int KP = (N + kGridBlock - 1) / kGridBlock;
    const int ntask = g.nh * nstates;
    const int per = (ntask + 7) / 8;
    const int t = (bx & 7) * per + (bx >> 3);
    if (t >= ntask) return;                // uniform per workgroup, before any barrier
    const int jh = t / nstates, s = t % nstates;
    const int T = g.T;
    const int jN = jh, jS = g.nlat - 1 - jh;
    const size_t fstride = (size_t)g.nlat * g.ms;
    const double2* fs = four + (size_t)s * kSynFields * fstride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WaveTw<N> twl;
    wave_tw_load<N, 0, 1>(twl, tw, lane);
    stage_inputs<N, kSynFields>(buf, fs, fstride, jN, jS, T, g.ms);
    __syncthreads();
    if (wave < kSynFields) fft_wave<N, true>(buf + wave * N, twl, lane);
    __syncthreads();
    if (save) {      // grid values of zeta, Phi', U, V (north, south) for the adjoint
        for (int f = 0; f < kSynFields; ++f)
            for (int k = threadIdx.x; k < N; k += kGridBlock)
                save[((size_t)(s * kSynFields + f) * g.nh + jh) * N + k] = buf[f * N + k];
    }
    const double x = mu[jN];
    const double fN = two_omega * x, fS = -fN;
    const double ke = 0.5 / ((1.0 - x) * (1.0 + x));
    double2 ereg[KP];                      // E at this thread's points until buffer 0 is free
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
        const int k = threadIdx.x + kk * kGridBlock;
        if (k >= N) continue;
        const double2 zeta = buf[k], phi = buf[N + k], U = buf[2 * N + k], V = buf[3 * N + k];
        const double qn = zeta.x + fN, qs = zeta.y + fS;
        buf[k] = make_double2(qn * U.x, qs * U.y);
        buf[N + k] = make_double2(qn * V.x, qs * V.y);
        buf[2 * N + k] = make_double2(phi.x * U.x, phi.y * U.y);
        buf[3 * N + k] = make_double2(phi.x * V.x, phi.y * V.y);
        ereg[kk] = make_double2((U.x * U.x + V.x * V.x) * ke, (U.y * U.y + V.y * V.y) * ke);
    }
    __syncthreads();
    if (wave < 4) fft_wave<N, false>(buf + wave * N, twl, lane);
    __syncthreads();
    BlockTw<N> twb;                        // loaded here: in flight during the unpack of A..D
    block_tw_load<N, 0, 1>(twb, tw);
    const double invN = 1.0 / N;
    const double wt = w[jN];
    const double gg = wt / (g.radius * (1.0 - x) * (1.0 + x)) * invN;
    const double we = wt * invN;
    // Analysis input lines (fwd_index): the weighted north +- south sums of A..E, each line
    // written whole by one thread in its value order once E is transformed (a line left half
    // written while E is transformed can leave L2 partial and cost a read-back).  Buffer 0 (A) is
    // needed for E, so A's two values of this thread's first MP orders wait in registers; lines of
    // higher orders (grids with T + 1 > nlon / 3) are written in two parts.
    constexpr int MP = (N + 3 * kGridBlock - 1) / (3 * kGridBlock);
    double2 areg[MP][2];
#pragma unroll
    for (int mp = 0; mp < MP; ++mp) {
        const int m = threadIdx.x + mp * kGridBlock;
        if (m > T) continue;
        double2 AN, AS;
        unpack_pair(buf, m, N, AN, AS);
        areg[mp][0] = cscale(gg, cadd(AN, AS));
        areg[mp][1] = cscale(gg, csub(AN, AS));
    }
    for (int m = threadIdx.x + MP * kGridBlock; m <= T; m += kGridBlock) {
        double2 AN, AS, BN, BS, CN, CS, DN, DS;
        unpack_pair(buf, m, N, AN, AS);
        unpack_pair(buf + N, m, N, BN, BS);
        unpack_pair(buf + 2 * N, m, N, CN, CS);
        unpack_pair(buf + 3 * N, m, N, DN, DS);
        const Row<GT> o(G, fwd_index(T, nstates, jh, m, s));
        o.put(kCs, cscale(gg, cadd(CN, CS)));
        o.put(kDa, cscale(gg, csub(DN, DS)));
        o.put(kAs, cscale(gg, cadd(AN, AS)));
        o.put(kBs, cscale(gg, cadd(BN, BS)));
        o.put(kAa, cscale(gg, csub(AN, AS)));
        o.put(kBa, cscale(gg, csub(BN, BS)));
        o.put(kCa, cscale(gg, csub(CN, CS)));
        o.put(kDs, cscale(gg, cadd(DN, DS)));
    }
    __syncthreads();
    // E: into buffer 0 and transformed by the whole workgroup
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
        const int k = threadIdx.x + kk * kGridBlock;
        if (k < N) buf[k] = ereg[kk];
    }
    __syncthreads();
    fft_block<N, false>(buf, twb);
#pragma unroll
    for (int mp = 0; mp < MP; ++mp) {
        const int m = threadIdx.x + mp * kGridBlock;
        if (m > T) continue;
        double2 BN, BS, CN, CS, DN, DS, EN, ES;
        unpack_pair(buf + N, m, N, BN, BS);
        unpack_pair(buf + 2 * N, m, N, CN, CS);
        unpack_pair(buf + 3 * N, m, N, DN, DS);
        unpack_pair(buf, m, N, EN, ES);
        const Row<GT> o(G, fwd_index(T, nstates, jh, m, s));
        o.put(kEs, cscale(we, cadd(EN, ES)));
        o.put(kCs, cscale(gg, cadd(CN, CS)));
        o.put(kDa, cscale(gg, csub(DN, DS)));
        o.put(kAs, areg[mp][0]);
        o.put(kBs, cscale(gg, cadd(BN, BS)));
        o.put(kAa, areg[mp][1]);
        o.put(kBa, cscale(gg, csub(BN, BS)));
        o.put(kCa, cscale(gg, csub(CN, CS)));
        o.put(kDs, cscale(gg, cadd(DN, DS)));
        o.put(kEa, cscale(we, csub(EN, ES)));
    }
    for (int m = threadIdx.x + MP * kGridBlock; m <= T; m += kGridBlock) {
        double2 EN, ES;
        unpack_pair(buf, m, N, EN, ES);
        const Row<GT> o(G, fwd_index(T, nstates, jh, m, s));
        o.put(kEs, cscale(we, cadd(EN, ES)));
        o.put(kEa, cscale(we, csub(EN, ES)));
    }
}

template <int N, typename GT>
__global__ __launch_bounds__(kGridBlock) void k_grid_swe(
    const double2* __restrict__ four, GT* __restrict__ G, const double* __restrict__ mu,
    const double* __restrict__ w, const double2* __restrict__ tw, double two_omega,
    int nstates, double2* __restrict__ save, Geom g) {
    grid_swe_body<N, GT>(four, G, mu, w, tw, two_omega, nstates, save, g, blockIdx.x);
}

// One grid launch over several handles (workgroup ranges as k_synthesis_multi); each workgroup
// runs the FFT length of its handle, one of the lengths 3 * 2^p up to 768 (the dynamic LDS of
// the launch is the largest handle's).
template <typename GT>
__global__ __launch_bounds__(kGridBlock) void k_grid_multi(const GridArgs* __restrict__ list, int n) {
    const int b = blockIdx.x;
    int h = 0;
    while (h + 1 < n && b >= list[h + 1].first) ++h;
    const GridArgs& a = list[h];
    const int bx = b - a.first;
    if (bx >= a.blocks) return;                              // padding to the next range (uniform)
    GT* G = reinterpret_cast<GT*>(a.G);
    switch (a.g.nlon) {
    case 96: grid_swe_body<96, GT>(a.four, G, a.mu, a.w, a.tw, a.two_omega, a.nstates, a.save, a.g, bx); break;
    case 192: grid_swe_body<192, GT>(a.four, G, a.mu, a.w, a.tw, a.two_omega, a.nstates, a.save, a.g, bx); break;
    case 384: grid_swe_body<384, GT>(a.four, G, a.mu, a.w, a.tw, a.two_omega, a.nstates, a.save, a.g, bx); break;
    default: grid_swe_body<768, GT>(a.four, G, a.mu, a.w, a.tw, a.two_omega, a.nstates, a.save, a.g, bx); break;
    }
}

bool grid_multi_supported(int nlon) { return nlon == 96 || nlon == 192 || nlon == 384 || nlon == 768; }

GridArgs make_grid_args(const double2* four, double* G, const double* mu, const double* w, const double2* tw,
                        int nstates, double two_omega, double2* save, const Geom& g) {
    GridArgs a{};
    a.four = four;
    a.G = G;
    a.mu = mu;
    a.w = w;
    a.tw = tw;
    a.two_omega = two_omega;
    a.nstates = nstates;
    a.save = save;
    a.g = g;
    a.blocks = (g.nh * nstates + 7) / 8 * 8;
    return a;
}

void launch_grid_multi(bool g32, int nlon_max, const GridArgs* list, int n, int blocks, hipStream_t st) {
    const size_t lds = (size_t)kGridSignals * nlon_max * sizeof(double2);
    if (g32) k_grid_multi<float><<<blocks, kGridBlock, lds, st>>>(list, n);
    else k_grid_multi<double><<<blocks, kGridBlock, lds, st>>>(list, n);
}

void launch_grid_swe(const double2* four, double* G, bool g32, const double* mu, const double* w,
                     const double2* tw, const FFTPlan& plan, int nstates, double two_omega,
                     double2* save, const Geom& g, hipStream_t st) {
    const int ntask = g.nh * nstates;
    const int nblk = (ntask + 7) / 8 * 8;
    const size_t lds = (size_t)kGridSignals * plan.n * sizeof(double2);
#define LAUNCH(NN)                                                                                    \
    if (g32)                                                                                          \
        k_grid_swe<NN, float><<<nblk, kGridBlock, lds, st>>>(four, reinterpret_cast<float*>(G), mu, w, \
                                                             tw, two_omega, nstates, save, g);        \
    else                                                                                              \
        k_grid_swe<NN, double><<<nblk, kGridBlock, lds, st>>>(four, G, mu, w, tw, two_omega, nstates, save, g)
    FFT_DISPATCH(plan.n, LAUNCH)
#undef LAUNCH
}

// ---------------------------------------------------------------------------------------------
// Adjoint grid step for one latitude pair of one state: inverse FFT of the adjoint Fourier fields
// A^, B^, C^, D^, E^ (already halved for m > 0), latitude weights w/((1-mu^2) a nlon) and w/nlon,
// transposed products at the saved stage fields, forward FFT (unnormalised) of the adjoints of
// zeta, Phi', U, V, and the columns of the transposed synthesis (s_m = 1, 2 for m = 0, > 0):
//   Pbar: s_m Z, (s_m/a)(-i m V), (s_m/a)(-i m U), s_m Phi;   H: -(s_m/a) U, (s_m/a) V
// combined into north +- south sums per parity (Pbar: + for even n-m; H: - for even n-m).
// With four LDS signals, E^ is transformed first (by the whole workgroup) and held in registers
// during the products.
// ---------------------------------------------------------------------------------------------
template <int N, typename GT>
__global__ __launch_bounds__(kGridBlock) void k_grid_adj(
    const double2* __restrict__ four5, const double2* __restrict__ save, GT* __restrict__ G,
    const double* __restrict__ mu, const double* __restrict__ w, const double2* __restrict__ tw,
    double two_omega, int nstates, Geom g) {
    extern __shared__ double2 buf[];      // kGridSignals signals x N
    constexpr int KP = (N + kGridBlock - 1) / kGridBlock;
    const int ntask = g.nh * nstates;
    const int per = (ntask + 7) / 8;
    const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (t >= ntask) return;
    const int jh = t / nstates, s = t % nstates;
    const int T = g.T;
    const int jN = jh, jS = g.nlat - 1 - jh;
    const size_t fstride = (size_t)g.nlat * g.ms;
    const double2* fs = four5 + (size_t)s * 5 * fstride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WaveTw<N> twl;
    wave_tw_load<N, 0, 1>(twl, tw, lane);
    BlockTw<N> twb;
    block_tw_load<N, 0, 1>(twb, tw);
    // E^ first (whole workgroup), kept in registers at this thread's points, then A^..D^ (one
    // wave each)
    stage_inputs<N, 1>(buf, fs + 4 * fstride, fstride, jN, jS, T, g.ms);
    __syncthreads();
    fft_block<N, true>(buf, twb);
    double2 ereg[KP];
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
        const int k = threadIdx.x + kk * kGridBlock;
        ereg[kk] = buf[k < N ? k : 0];
    }
    __syncthreads();
    stage_inputs<N, 4>(buf, fs, fstride, jN, jS, T, g.ms);
    __syncthreads();
    if (wave < 4) fft_wave<N, true>(buf + wave * N, twl, lane);
    __syncthreads();
    const double x = mu[jN];
    const double fN = two_omega * x, fS = -fN;
    const double om2 = (1.0 - x) * (1.0 + x);
    const double inv = 1.0 / om2;
    const double gA = w[jN] / (om2 * g.radius * N), gE = w[jN] / N;
    const double2* sv = save + ((size_t)(s * kSynFields) * g.nh + jh) * N;
    const size_t sstride = (size_t)g.nh * N;
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
        const int k = threadIdx.x + kk * kGridBlock;
        if (k >= N) continue;
        const double2 a = buf[k], b = buf[N + k], c = buf[2 * N + k], d = buf[3 * N + k], e = ereg[kk];
        const double2 zeta = sv[k], phi = sv[sstride + k], U = sv[2 * sstride + k], V = sv[3 * sstride + k];
        const double An = gA * a.x, As = gA * a.y, Bn = gA * b.x, Bs = gA * b.y;
        const double Cn = gA * c.x, Cs = gA * c.y, Dn = gA * d.x, Ds = gA * d.y;
        const double En = gE * e.x * inv, Es = gE * e.y * inv;
        const double qn = zeta.x + fN, qs = zeta.y + fS;
        buf[k] = make_double2(An * U.x + Bn * V.x, As * U.y + Bs * V.y);
        buf[N + k] = make_double2(Cn * U.x + Dn * V.x, Cs * U.y + Ds * V.y);
        buf[2 * N + k] = make_double2(An * qn + Cn * phi.x + En * U.x, As * qs + Cs * phi.y + Es * U.y);
        buf[3 * N + k] = make_double2(Bn * qn + Dn * phi.x + En * V.x, Bs * qs + Ds * phi.y + Es * V.y);
    }
    __syncthreads();
    if (wave < kSynFields) fft_wave<N, false>(buf + wave * N, twl, lane);
    __syncthreads();
    const double inva = 1.0 / g.radius;
    const double2 z2 = make_double2(0.0, 0.0);
    for (int m = threadIdx.x; m <= T; m += kGridBlock) {
        double2 ZN, ZS, PN, PS, UN, US, VN, VS;
        unpack_pair(buf, m, N, ZN, ZS);
        unpack_pair(buf + N, m, N, PN, PS);
        unpack_pair(buf + 2 * N, m, N, UN, US);
        unpack_pair(buf + 3 * N, m, N, VN, VS);
        const double sm = m == 0 ? 1.0 : 2.0, sa = sm * inva, ms = (double)m * sa;
        const double2 Zs = cadd(ZN, ZS), Za = csub(ZN, ZS), Ps = cadd(PN, PS), Pa = csub(PN, PS);
        const double2 Us = cadd(UN, US), Ua = csub(UN, US), Vs = cadd(VN, VS), Va = csub(VN, VS);
        const Row<GT> o0(G, ana_index(T, nstates, jh, m, 0, s));
        const Row<GT> o1(G, ana_index(T, nstates, jh, m, 1, s));
        // -i m X (s_m/a) = (m sa X.y, -m sa X.x)
        o0.put(0, make_double2(sm * Zs.x, sm * Zs.y));
        o0.put(1, make_double2(ms * Vs.y, -ms * Vs.x));
        o0.put(2, make_double2(ms * Us.y, -ms * Us.x));
        o0.put(3, make_double2(sm * Ps.x, sm * Ps.y));
        o0.put(4, make_double2(-sa * Ua.x, -sa * Ua.y));
        o0.put(5, make_double2(sa * Va.x, sa * Va.y));
        o0.put(6, z2);
        o0.put(7, z2);
        o1.put(0, make_double2(sm * Za.x, sm * Za.y));
        o1.put(1, make_double2(ms * Va.y, -ms * Va.x));
        o1.put(2, make_double2(ms * Ua.y, -ms * Ua.x));
        o1.put(3, make_double2(sm * Pa.x, sm * Pa.y));
        o1.put(4, make_double2(-sa * Us.x, -sa * Us.y));
        o1.put(5, make_double2(sa * Vs.x, sa * Vs.y));
        o1.put(6, z2);
        o1.put(7, z2);
    }
}

void launch_grid_adj(const double2* four5, const double2* save, double* G, bool g32, const double* mu,
                     const double* w, const double2* tw, const FFTPlan& plan, int nstates,
                     double two_omega, const Geom& g, hipStream_t st) {
    const int ntask = g.nh * nstates;
    const int nblk = (ntask + 7) / 8 * 8;
    const size_t lds = (size_t)kGridSignals * plan.n * sizeof(double2);
#define LAUNCH(NN)                                                                                     \
    if (g32)                                                                                           \
        k_grid_adj<NN, float><<<nblk, kGridBlock, lds, st>>>(four5, save, reinterpret_cast<float*>(G), \
                                                             mu, w, tw, two_omega, nstates, g);        \
    else                                                                                               \
        k_grid_adj<NN, double><<<nblk, kGridBlock, lds, st>>>(four5, save, G, mu, w, tw, two_omega, nstates, g)
    FFT_DISPATCH(plan.n, LAUNCH)
#undef LAUNCH
}

// ---------------------------------------------------------------------------------------------
// Scalar longitude transforms for sht_inverse / sht_forward (one latitude pair per workgroup).
// ---------------------------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kBlock) void k_fft_inverse_scalar(
    const double2* __restrict__ four, double* __restrict__ grid, const double2* __restrict__ tw,
    Geom g) {
    extern __shared__ double2 buf[];
    const int jh = blockIdx.x, f = blockIdx.y;
    const int jN = jh, jS = g.nlat - 1 - jh;
    const double2* xn = four + ((size_t)f * g.nlat + jN) * g.ms;
    const double2* ys = four + ((size_t)f * g.nlat + jS) * g.ms;
    double2* twl = buf + N;
    for (int k = threadIdx.x; k < N; k += kBlock) {
        buf[k] = pack_pair(xn, ys, k, N, g.T);
        twl[k] = tw[k];
    }
    __syncthreads();
    fft_lds<N, true>(buf, 1, twl);
    double* rn = grid + ((size_t)f * g.nlat + jN) * g.nlon;
    double* rs = grid + ((size_t)f * g.nlat + jS) * g.nlon;
    for (int k = threadIdx.x; k < N; k += kBlock) {
        const double2 z = buf[k];
        rn[k] = z.x;
        rs[k] = z.y;
    }
}

void launch_fft_inverse_scalar(const double2* four, double* grid, const double2* tw,
                               const FFTPlan& plan, int nfields, const Geom& g, hipStream_t st) {
    dim3 gr(g.nh, nfields);
    const size_t lds = 2 * plan.n * sizeof(double2);
#define LAUNCH(NN) k_fft_inverse_scalar<NN><<<gr, kBlock, lds, st>>>(four, grid, tw, g)
    FFT_DISPATCH(plan.n, LAUNCH)
#undef LAUNCH
}

// Output ana[f][p][jh][m] = scale * (F_N +- F_S), + for parity 0, - for parity 1, with F the
// unnormalised DFT and scale = w_j/nlon (analysis) or s_m (transpose of the synthesis).
template <int N>
__global__ __launch_bounds__(kBlock) void k_fft_forward_scalar(
    const double* __restrict__ grid, double2* __restrict__ ana, const double* __restrict__ w,
    const double2* __restrict__ tw, int transpose_synthesis, Geom g) {
    extern __shared__ double2 buf[];
    const int jh = blockIdx.x, f = blockIdx.y;
    const int jN = jh, jS = g.nlat - 1 - jh;
    const double* rn = grid + ((size_t)f * g.nlat + jN) * g.nlon;
    const double* rs = grid + ((size_t)f * g.nlat + jS) * g.nlon;
    double2* twl = buf + N;
    for (int k = threadIdx.x; k < N; k += kBlock) {
        buf[k] = make_double2(rn[k], rs[k]);
        twl[k] = tw[k];
    }
    __syncthreads();
    fft_lds<N, false>(buf, 1, twl);
    const double wsc = w[jN] / N;
    double2* o0 = ana + ((size_t)(f * 2 + 0) * g.nhp + jh) * g.ms;
    double2* o1 = ana + ((size_t)(f * 2 + 1) * g.nhp + jh) * g.ms;
    for (int m = threadIdx.x; m <= g.T; m += kBlock) {
        double2 XN, XS;
        unpack_pair(buf, m, N, XN, XS);
        const double sc = transpose_synthesis ? (m == 0 ? 1.0 : 2.0) : wsc;
        o0[m] = make_double2(sc * (XN.x + XS.x), sc * (XN.y + XS.y));
        o1[m] = make_double2(sc * (XN.x - XS.x), sc * (XN.y - XS.y));
    }
}

void launch_fft_forward_scalar(const double* grid, double2* ana, const double* w,
                               const double2* tw, const FFTPlan& plan, int nfields,
                               int transpose_synthesis, const Geom& g, hipStream_t st) {
    dim3 gr(g.nh, nfields);
    const size_t lds = 2 * plan.n * sizeof(double2);
#define LAUNCH(NN) k_fft_forward_scalar<NN><<<gr, kBlock, lds, st>>>(grid, ana, w, tw, transpose_synthesis, g)
    FFT_DISPATCH(plan.n, LAUNCH)
#undef LAUNCH
}

hipError_t grid_set_lds_limit(int n, size_t bytes) {
    hipError_t e = hipSuccess;
#define SETLDS1(F)                                                                                   \
    if (e == hipSuccess)                                                                             \
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&F), hipFuncAttributeMaxDynamicSharedMemorySize, \
                                (int)bytes)
#define SETLDS(NN)                                                                                   \
    SETLDS1((k_grid_swe<NN, double>));                                                               \
    SETLDS1((k_grid_swe<NN, float>));                                                                \
    SETLDS1((k_grid_adj<NN, double>));                                                               \
    SETLDS1((k_grid_adj<NN, float>))
    FFT_DISPATCH(n, SETLDS)
#undef SETLDS
#undef SETLDS1
    return e;
}
