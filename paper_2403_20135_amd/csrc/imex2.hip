// IMEX-o2, the reference integrator of the spectral shallow-water model (Section 3.2): a Strang
// splitting with Crank-Nicolson half steps for the gravity part f_I = L_g around one Heun step
// for f_E = L_c + N_a + N_r:
//   u* = C(dt/2) u_n,  k1 = f_E(u*),  k2 = f_E(u* + dt k1),  u_{n+1} = C(dt/2)(u* + dt/2 (k1 + k2)),
// with C(h) u = solve(h/2, u + h/2 L_g(u)) per coefficient (the closed-form 2x2 solve of
// u - a L_g(u) = beta).  The coefficient-wise phases below run between the f_E evaluations; like
// the dSDC update they stream over the coefficients, one thread per (coefficient, Re/Im part),
// and write the synthesis layout of the state the next f_E evaluates.
#include "common.h"

// one Crank-Nicolson half step (a = dt/4) of the gravity-wave pair of one coefficient part
__device__ __forceinline__ void cn_half(double& phi, double& dv, double a, double phibar, double cn) {
    const double bphi = phi - a * phibar * dv;
    const double bdiv = dv + a * cn * phi;
    const double p = (bphi - a * phibar * bdiv) / (1.0 + a * a * phibar * cn);
    phi = p;
    dv = bdiv + a * cn * p;
}

__global__ __launch_bounds__(kBlock) void k_imex2(Imex2Args a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= 2 * a.ncoef) return;
    const int idx = t >> 1, c = t & 1;
    const int n = a.n_of[idx];
    const double cn = n * (n + 1.0) * a.inv_a2;
    const size_t fs = (size_t)a.ncoef * 2;              // field stride in doubles
    const size_t o = (size_t)b * 3 * fs + (size_t)t;    // (member, field 0, coefficient, part)
    const double q = 0.25 * a.dt;
    double phi = a.in[o], zeta = a.in[o + fs], dv = a.in[o + 2 * fs];
    if (a.phase == kImex2First) {
        cn_half(phi, dv, q, a.phibar, cn);
        a.out[o] = phi;
        a.out[o + fs] = zeta;
        a.out[o + 2 * fs] = dv;
    } else {
        const double* k1 = a.k1 + o;
        const double w = a.phase == kImex2Predict ? a.dt : 0.5 * a.dt;
        double e0 = k1[0], e1 = k1[fs], e2 = k1[2 * fs];
        if (a.phase == kImex2Last) {
            const double* k2 = a.k2 + o;
            e0 += k2[0];
            e1 += k2[fs];
            e2 += k2[2 * fs];
        }
        phi += w * e0;
        zeta += w * e1;
        dv += w * e2;
        if (a.phase == kImex2Last) {
            cn_half(phi, dv, q, a.phibar, cn);
            a.out[o] = phi;
            a.out[o + fs] = zeta;
            a.out[o + 2 * fs] = dv;
            if (!(isfinite(phi) && isfinite(zeta) && isfinite(dv))) a.flag[0] = 1;
            return;
        }
    }
    // synthesis layout of member b's next f_E input: (zeta, Phi', psi, chi) x (Re, Im)
    const int mo = a.m_of[idx], par = (n - mo) & 1, kk = (n - mo) >> 1;
    const double il = a.inv_lap[n];
    const size_t ci = (((size_t)a.rowoff[2 * mo + par] + kk) * a.batch + b) * kCmlVals + c;
    cml_put(a.cml, a.cml32, ci, zeta);
    cml_put(a.cml, a.cml32, ci + 2, phi);
    cml_put(a.cml, a.cml32, ci + 4, il * zeta);
    cml_put(a.cml, a.cml32, ci + 6, il * dv);
    if (c == 0) cml_clear_pad(a.cml, a.cml32, a.rowoff[2 * mo + par], kk, npk_of(a.T, mo, par), a.batch, b);
}

void launch_imex2(const Imex2Args& a, hipStream_t st) {
    dim3 grid((2 * a.ncoef + kBlock - 1) / kBlock, a.batch);
    k_imex2<<<grid, kBlock, 0, st>>>(a);
}
