// Kernels specific to the adjoint solve: per-cell Jacobian coefficients at
// the linearisation point and the final gradient with respect to delta.
#pragma once
#include "mg_kernels.h"

namespace mgk {

struct CoefsW {
    double *c[9][2];
};

// For every cell m: dK_m/dphi at its 6 face neighbours (x+ x- y+ y- z+ z-)
// and the 3 edge coefficients, K being the model term of L = lap - K.
// Derivatives of the forms used in model_term:
//   nDGP:  dF/dSigma = sign(alpha)/sqrt(D) (0 on the clamped branch),
//          dSigma/dphi(x+-) = 2(2A_x - A_y - A_z)/(3h^4),
//          dSigma/dphi(x+1,y+1) = N_xy/(4h^4) (sign pattern of N_xy).
//   Kmouflage: K = num/(c~ Sigma_1), num = src delta + Sigma_2, through
//          dg/dphi(x+-) = +-G_x/h and
//          dQ/dphi(x+-) = (2G_x^2 - G_y^2 - G_z^2)/(3h^2) +- (hH_xx G_x + D_xy G_y + D_xz G_z)/h,
//          dQ/dphi(x+1,y+1) = G_x G_y/(2h^2).
template <int MODEL>
__global__ __launch_bounds__(TPB) void k_adj_coefs(Mod M, Lvl L, CoefsW W, double h) {
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    const size_t half = (size_t)1 << (3 * L.logn - 1);
    if (t >= 2 * half) return;
    const int c = t >= half;
    const size_t tt = t - (c ? half : 0);
    const int m = (int)(tt & ((1u << L.lognh) - 1));
    const int j = (int)((tt >> L.lognh) & (L.n - 1));
    const int k = (int)(tt >> (L.lognh + L.logn));
    const double *A = c ? L.u1 : L.u0;
    const double *B = c ? L.u0 : L.u1;
    const Nb s = load_nb<double, double>(A, B, c, m, j, k, L.n, L.logn, L.lognh);
    const double delta = (c ? L.d1 : L.d0)[tt];
    const double ax = s.xp + s.xm, ay = s.yp + s.ym, az = s.zp + s.zm;
    double f[6], e[3];
    if (MODEL == MODEL_POISSON) {
        for (int q = 0; q < 6; ++q) f[q] = 0.0;
        e[0] = e[1] = e[2] = 0.0;
    } else if (MODEL == MODEL_DGP) {
        const double dxy = ax - ay, dxz = ax - az, dyz = ay - az;
        const double sig = (dxy * dxy + dxz * dxz + dyz * dyz) * L.c3h4
                         + (s.nxy * s.nxy + s.nxz * s.nxz + s.nyz * s.nyz) * L.c8h4 + M.s * delta;
        const double disc = M.alpha * M.alpha + (8.0 / 3.0) * sig;
        const double fp = disc > 0.0 ? M.sgn / sqrt(disc) : 0.0;
        const double w = 2.0 * fp * L.c3h4;
        f[0] = f[1] = w * (2.0 * ax - ay - az);
        f[2] = f[3] = w * (2.0 * ay - ax - az);
        f[4] = f[5] = w * (2.0 * az - ax - ay);
        e[0] = 2.0 * fp * L.c8h4 * s.nxy;
        e[1] = 2.0 * fp * L.c8h4 * s.nxz;
        e[2] = 2.0 * fp * L.c8h4 * s.nyz;
    } else {
        const double h2 = L.h2;
        const double gx = (s.xp - s.xm) / (2.0 * h), gy = (s.yp - s.ym) / (2.0 * h),
                     gz = (s.zp - s.zm) / (2.0 * h);
        const double g = gx * gx + gy * gy + gz * gz;
        const double hxx = (2.0 * ax - ay - az) / (3.0 * h2);
        const double hyy = (2.0 * ay - ax - az) / (3.0 * h2);
        const double hzz = (2.0 * az - ax - ay) / (3.0 * h2);
        const double dxy = s.nxy / (4.0 * h2), dxz = s.nxz / (4.0 * h2), dyz = s.nyz / (4.0 * h2);
        const double q = hxx * gx * gx + hyy * gy * gy + hzz * gz * gz
                       + 2.0 * (dxy * gx * gy + dxz * gx * gz + dyz * gy * gz);
        double gn2 = 1.0, gn3 = 1.0;
        for (int r = 0; r < M.nk - 2; ++r) gn2 *= g;
        for (int r = 0; r < M.nk - 3; ++r) gn3 *= g;
        const double sig1 = M.c0 + M.a1 * gn2 * g;
        const double num = M.src * delta + M.b2 * gn2 * q;
        const double ds1_dg = M.a1 * (M.nk - 1) * gn2;
        const double ds2_dg = (M.nk >= 3) ? M.b2 * (M.nk - 2) * gn3 * q : 0.0;
        const double ds2_dq = M.b2 * gn2;
        const double G[3] = {gx, gy, gz};
        const double dg2[3] = {(2.0 * gx * gx - gy * gy - gz * gz) / (3.0 * h2),
                               (2.0 * gy * gy - gx * gx - gz * gz) / (3.0 * h2),
                               (2.0 * gz * gz - gx * gx - gy * gy) / (3.0 * h2)};
        const double lin[3] = {(hxx * gx + dxy * gy + dxz * gz) / h,
                               (dxy * gx + hyy * gy + dyz * gz) / h,
                               (dxz * gx + dyz * gy + hzz * gz) / h};
        const double den = 1.0 / (M.ctil * sig1 * sig1);
#pragma unroll
        for (int ax3 = 0; ax3 < 3; ++ax3) {
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                const double sgn = sg ? -1.0 : 1.0;
                const double dg = sgn * G[ax3] / h;
                const double dq = dg2[ax3] + sgn * lin[ax3];
                const double d1 = ds1_dg * dg;
                const double d2 = ds2_dg * dg + ds2_dq * dq;
                f[2 * ax3 + sg] = (d2 * sig1 - num * d1) * den;
            }
        }
        const double ec = ds2_dq / (2.0 * h2 * M.ctil * sig1);
        e[0] = ec * gx * gy;
        e[1] = ec * gx * gz;
        e[2] = ec * gy * gz;
    }
    // nDGP and Poisson: the x+ and x- (y, z) coefficients are equal and the
    // minus arrays alias the plus ones, so only the plus arrays are written
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (MODEL == MODEL_KMO || !(q & 1)) W.c[q][c][tt] = f[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) W.c[6 + q][c][tt] = e[q];
}

// F' = dK/dSigma of the nDGP term at every cell of a level (sign(alpha)/sqrt(D),
// 0 on the clamped branch), the one per-cell array the tiled adjoint kernels
// keep: they rebuild the coefficients of k_adj_coefs from it and the staged
// linearisation point.
__global__ __launch_bounds__(TPB) void k_adj_kprime(Mod M, Lvl L, double *kp0, double *kp1) {
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    const size_t half = (size_t)1 << (3 * L.logn - 1);
    if (t >= 2 * half) return;
    const int c = t >= half;
    const size_t tt = t - (c ? half : 0);
    const int m = (int)(tt & ((1u << L.lognh) - 1));
    const int j = (int)((tt >> L.lognh) & (L.n - 1));
    const int k = (int)(tt >> (L.lognh + L.logn));
    const double *A = c ? L.u1 : L.u0;
    const double *B = c ? L.u0 : L.u1;
    const Nb s = load_nb<double, double>(A, B, c, m, j, k, L.n, L.logn, L.lognh);
    const double delta = (c ? L.d1 : L.d0)[tt];
    const double ax = s.xp + s.xm, ay = s.yp + s.ym, az = s.zp + s.zm;
    const double dxy = ax - ay, dxz = ax - az, dyz = ay - az;
    const double sig = (dxy * dxy + dxz * dxz + dyz * dyz) * L.c3h4
                     + (s.nxy * s.nxy + s.nxz * s.nxz + s.nyz * s.nyz) * L.c8h4 + M.s * delta;
    const double disc = M.alpha * M.alpha + (8.0 / 3.0) * sig;
    (c ? kp1 : kp0)[tt] = disc > 0.0 ? M.sgn / sqrt(disc) : 0.0;
}

// grad_delta = (dK/ddelta) mu on the finest level, written in natural layout.
template <int MODEL>
__global__ __launch_bounds__(TPB) void k_adj_grad(Mod M, Lvl L, const double *mu0,
                                                  const double *mu1, double *grad) {
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    const size_t half = (size_t)1 << (3 * L.logn - 1);
    if (t >= 2 * half) return;
    const int c = t >= half;
    const size_t tt = t - (c ? half : 0);
    const int m = (int)(tt & ((1u << L.lognh) - 1));
    const int j = (int)((tt >> L.lognh) & (L.n - 1));
    const int k = (int)(tt >> (L.lognh + L.logn));
    const double *A = c ? L.u1 : L.u0;
    const double *B = c ? L.u0 : L.u1;
    const Nb s = load_nb<double, double>(A, B, c, m, j, k, L.n, L.logn, L.lognh);
    const double delta = (c ? L.d1 : L.d0)[tt];
    double dk;
    if (MODEL == MODEL_POISSON) {
        dk = M.s;
    } else if (MODEL == MODEL_DGP) {
        const double ax = s.xp + s.xm, ay = s.yp + s.ym, az = s.zp + s.zm;
        const double dxy = ax - ay, dxz = ax - az, dyz = ay - az;
        const double sig = (dxy * dxy + dxz * dxz + dyz * dyz) * L.c3h4
                         + (s.nxy * s.nxy + s.nxz * s.nxz + s.nyz * s.nyz) * L.c8h4 + M.s * delta;
        const double disc = M.alpha * M.alpha + (8.0 / 3.0) * sig;
        dk = disc > 0.0 ? M.sgn / sqrt(disc) * M.s : 0.0;
    } else {
        const double ex = s.xp - s.xm, ey = s.yp - s.ym, ez = s.zp - s.zm;
        const double g = (ex * ex + ey * ey + ez * ez) * L.c4h2;
        double gn2 = 1.0;
        for (int r = 0; r < M.nk - 2; ++r) gn2 *= g;
        dk = M.src / (M.ctil * (M.c0 + M.a1 * gn2 * g));
    }
    const int p = (j + k + c) & 1;
    const size_t nat = ((size_t)k << (2 * L.logn)) + ((size_t)j << L.logn) + (size_t)(2 * m + p);
    grad[nat] = dk * (c ? mu1 : mu0)[tt];
}

}  // namespace mgk
