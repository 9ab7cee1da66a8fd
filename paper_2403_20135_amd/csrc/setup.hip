// FP64 setup on the GPU: Gauss-Legendre latitudes and weights, orthonormal associated Legendre
// functions Pbar_n^m and H_n^m = (1-mu^2) dPbar_n^m/dmu on the northern latitudes, and the
// Radau-right collocation nodes with their collocation matrices (Sections 4.1-4.2).
#include "common.h"

// P_n(x) and P_n'(x) by the three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}.
__device__ inline void legendre_pd(int n, double x, double& p, double& dp) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    dp = n * (x * p1 - p0) / (x * x - 1.0);
}

// One thread per northern root; the southern root is its mirror image.
__global__ void k_gauss(double* __restrict__ mu, double* __restrict__ w, int nlat) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int nh = nlat / 2;
    if (j >= nh) return;
    double x = cos(M_PI * (j + 0.75) / (nlat + 0.5));
    double p, dp;
    for (int it = 0; it < 100; ++it) {
        legendre_pd(nlat, x, p, dp);
        const double dx = p / dp;
        x -= dx;
        if (fabs(dx) < 1e-16) break;
    }
    legendre_pd(nlat, x, p, dp);
    x -= p / dp;
    legendre_pd(nlat, x, p, dp);
    const double wt = 2.0 / ((1.0 - x) * (1.0 + x) * dp * dp);
    mu[j] = x;
    w[j] = wt;
    mu[nlat - 1 - j] = -x;
    w[nlat - 1 - j] = wt;
}

void launch_gauss(double* mu, double* w, int nlat, hipStream_t st) {
    const int nh = nlat / 2;
    k_gauss<<<(nh + 127) / 128, 128, 0, st>>>(mu, w, nlat);
}

__device__ inline double eps_nm(int n, int m) {
    if (n <= m) return 0.0;
    const double nn = (double)n, mm = (double)m;
    return sqrt((nn * nn - mm * mm) / (4.0 * nn * nn - 1.0));
}

// One thread per (m, n): the recurrence coefficients of Pbar_n^m and H_n^m (rec_index layout).
__global__ void k_rec_coefs(double* __restrict__ rc, Geom g) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    const int n = m + k;
    if (m > g.T || n >= g.T + kRecPad) return;
    const double e_n = eps_nm(n, m), e_n1 = eps_nm(n + 1, m);
    double* c = rc + 4 * rec_index(g.T, m, n);
    c[0] = 1.0 / e_n1;
    c[1] = e_n / e_n1;
    c[2] = (n + 1) * e_n;
    c[3] = n * e_n1;
}

void launch_rec_coefs(double* rc, const Geom& g, hipStream_t st) {
    dim3 grid((g.T + kRecPad + 63) / 64, g.T + 1);
    k_rec_coefs<<<grid, 64, 0, st>>>(rc, g);
}

// One thread per (m, northern latitude): Pbar_m^m by its product formula, then the upward
// recurrence in n (leg_next / leg_h), writing Pbar and H for n = m..T into the parity-split
// packed layout (row n goes to parity (n-m)&1, row (n-m)>>1; tile-major, tab_index).
__global__ void k_legendre(const double* __restrict__ mu, const double* __restrict__ rc,
                           double* __restrict__ P, double* __restrict__ H,
                           double* __restrict__ sect, const long long* __restrict__ toff, Geom g) {
    const int jh = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (jh >= g.nh || m > g.T) return;
    const double x = mu[jh];
    const double s = sqrt((1.0 - x) * (1.0 + x));
    double pmm = 0.70710678118654752440;   // Pbar_0^0 = 1/sqrt(2)
    for (int k = 1; k <= m; ++k) pmm *= sqrt((2.0 * k + 1.0) / (2.0 * k)) * s;
    sect[(size_t)m * g.nhp + jh] = pmm;
    double pm1 = 0.0, p0 = pmm;            // Pbar_{n-1}, Pbar_n
    for (int n = m; n <= g.T; ++n) {
        const double* c = rc + 4 * rec_index(g.T, m, n);
        const double p1 = leg_next(x, p0, pm1, c[0], c[1]);
        const int par = (n - m) & 1, kk = (n - m) >> 1;
        const long long idx = toff[2 * m + par] + tab_index((npk_of(g.T, m, par) + 3) & ~3, kk, jh);
        P[idx] = p0;
        H[idx] = leg_h(pm1, p1, c[2], c[3]);
        pm1 = p0;
        p0 = p1;
    }
}

void launch_legendre_tables(const double* mu, const double* rc, double* P, double* H, double* sect,
                            const long long* toff, const Geom& g, hipStream_t st) {
    dim3 grid((g.nh + 63) / 64, g.T + 1);
    k_legendre<<<grid, 64, 0, st>>>(mu, rc, P, H, sect, toff, g);
}

// Radau-right nodes for every node count Mc = 1..Mmax: the roots of P_Mc(x) - P_{Mc-1}(x) on
// [-1, 1] mapped to t = (x+1)/2 (x = 1 is always a root), located by sign changes on a fine
// sampling and refined by bisection to full FP64 precision.  Q[m][j] = integral from 0
// to tau_m of the Lagrange polynomial l_j, by an 8-point Gauss-Legendre rule on [0, tau_m]
// (exact: l_j has degree Mc-1 <= 7).  Layout: tau[Mc*8 + m], Q[(Mc*8 + m)*8 + j].
__device__ inline double radau_poly(int M, double x) {
    double p, dp, q, dq;
    legendre_pd(M, x, p, dp);
    legendre_pd(M - 1, x, q, dq);
    return p - q;
}

__global__ void k_collocation(double* __restrict__ tau, double* __restrict__ Q, int Mmax) {
    const int Mc = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (Mc > Mmax) return;
    double t[kMaxNodes];
    int found = 0;
    const int NS = 4096;
    double xa = -1.0, fa = radau_poly(Mc, xa);
    for (int i = 1; i < NS && found < Mc - 1; ++i) {
        const double xb = -1.0 + 2.0 * i / NS;
        const double fb = radau_poly(Mc, xb);
        if (fa == 0.0 || fa * fb < 0.0) {
            double lo = xa, hi = xb, flo = fa;
            if (fa != 0.0) {
                for (int it = 0; it < 200; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    const double fm = radau_poly(Mc, mid);
                    if (fm == 0.0) { lo = hi = mid; break; }
                    if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
                }
            }
            t[found++] = 0.5 * (0.5 * (lo + hi) + 1.0);
        }
        xa = xb;
        fa = fb;
    }
    t[Mc - 1] = 1.0;
    // 8-point Gauss-Legendre rule on [-1, 1]
    double gx[8], gw[8];
    for (int k = 0; k < 8; ++k) {
        double x = cos(M_PI * (k + 0.75) / 8.5), p, dp;
        for (int it = 0; it < 60; ++it) {
            legendre_pd(8, x, p, dp);
            const double dx = p / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        legendre_pd(8, x, p, dp);
        gx[k] = x;
        gw[k] = 2.0 / ((1.0 - x) * (1.0 + x) * dp * dp);
    }
    for (int m = 0; m < Mc; ++m) {
        tau[Mc * kMaxNodes + m] = t[m];
        for (int j = 0; j < Mc; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 8; ++k) {
                const double sx = 0.5 * t[m] * (gx[k] + 1.0);
                double l = 1.0;
                for (int i = 0; i < Mc; ++i)
                    if (i != j) l *= (sx - t[i]) / (t[j] - t[i]);
                acc += gw[k] * l;
            }
            Q[(Mc * kMaxNodes + m) * kMaxNodes + j] = 0.5 * t[m] * acc;
        }
    }
}

void launch_collocation(double* tau, double* Q, int Mmax, hipStream_t st) {
    k_collocation<<<1, 64, 0, st>>>(tau, Q, Mmax);
}

// Degree tables: n and m of every stored coefficient, -a^2/(n(n+1)) (inverse Laplacian, 0 at n = 0)
// and n(n+1)/a^2 (minus the Laplacian) for n = 0..T.
__global__ void k_degree_tables(int* __restrict__ n_of, int* __restrict__ m_of,
                                double* __restrict__ inv_lap, double* __restrict__ neg_lap, int T,
                                double radius) {
    const int m = blockIdx.x;
    const int base = coef_offset(T, m);
    for (int n = m + threadIdx.x; n <= T; n += blockDim.x) {
        n_of[base + n - m] = n;
        m_of[base + n - m] = m;
    }
    if (m == 0) {
        for (int n = threadIdx.x; n <= T; n += blockDim.x) {
            const double nn = n * (n + 1.0);
            inv_lap[n] = n == 0 ? 0.0 : -radius * radius / nn;
            neg_lap[n] = nn / (radius * radius);
        }
    }
}

void launch_degree_tables(int* n_of, int* m_of, double* inv_lap, double* neg_lap, int T,
                          double radius, hipStream_t st) {
    k_degree_tables<<<T + 1, 64, 0, st>>>(n_of, m_of, inv_lap, neg_lap, T, radius);
}
