// Kernels of the FAS multigrid solve.  See mg_device.h for the storage
// layout.  Every kernel is one thread per cell (or per coarse cell), 256
// threads per block, with the block index remapped so that each of the 8
// XCDs works on a contiguous z-slab (its halo rows stay in its own L2).
// R is the storage type (double, or float for the FP32 phase of the mixed
// solve); the adjoint operator exists for double only.
#pragma once
#include "mg_device.h"

namespace mgk {

constexpr int TPB = 256;

// device scalar slots (one small array in the workspace)
enum {
    S_MU = 0,      // finest right-hand side mu = mean L(phi), lagged
    S_SHIFT = 1,   // mean change of the finest residual since mu was last set
    S_EPS2 = 2,    // squared RMS of the last reduced residual
    S_MEAN = 3,    // mean of the last summed field
    S_CSUM0 = 4,   // adjoint, tiled finest level: sum of mu over colour 0
    S_CSUM1 = 5,   // ... over colour 1 (each refreshed by the last kernel that wrote the colour)
    S_MU64 = 6,    // defect correction: the FP64 field's bordering scalar (S_MU is the inner one)
    S_EPS64 = 7,   // defect correction: squared RMS of the FP64 finest residual
    S_NSCAL = 16
};

enum { OP_DGP = MODEL_DGP, OP_KMO = MODEL_KMO, OP_POISSON = MODEL_POISSON, OP_ADJ = 3,
       OP_NEWTON = 4 };

// OP_NEWTON: the nDGP equation in its quadratic form eq:dgp_quadratic_eom,
// divided by alpha, L_N = D + 2 D^2 / (3 alpha) - Sigma / alpha with D the
// 7-point Laplacian (centre included), relaxed by the generic Newton-Gauss-
// Seidel step of eq:relaxation_iteration,
//   u <- u - (L_N - f) / (dL_N/du),  dL_N/du = -(6/h^2)(1 + 4 D / (3 alpha)).
// A comparator for the closed-form update: same fixed point on the physical
// branch.  cell_term returns Sigma / alpha; newton_term adds the D part.
template <typename T>
__device__ __forceinline__ T newton_term(const Mod &M, T sigma_over_alpha, T D) {
    return sigma_over_alpha - (T)(2.0 / (3.0 * M.alpha)) * D * D;
}
template <typename T>
__device__ __forceinline__ T newton_update(const Mod &M, T u, T faces, T sig, T f, T h2) {
    const T D = (faces - (T)6 * u) / h2;
    const T r = D - newton_term<T>(M, sig, D) - f;
    const T dL = -((T)6 / h2) * ((T)1 + (T)(4.0 / (3.0 * M.alpha)) * D);
    return u - r / dL;
}

// Blocks are dispatched round-robin over the 8 XCDs; hand XCD x the x-th
// contiguous eighth of the logical tiles.
__device__ __forceinline__ size_t xcd_block(unsigned b, unsigned nb) {
    if (nb & 7u) return b;
    return (size_t)(b & 7u) * (nb >> 3) + (b >> 3);
}

// Adjoint coefficient arrays of one level: for every cell m the derivative of
// its model term K_m with respect to the 6 face neighbours (x+ x- y+ y- z+ z-)
// and the 3 edge pairs (the (+,+)/(-,-) corners carry +e, the (+,-)/(-,+)
// corners -e).
struct Coefs {
    const double *c[9][2];
};

// Sum of the six face values and the non-Laplacian term at the cell of
// colour c, packed (m, j, k), in arithmetic type T.
template <int OP, typename T, typename R>
__device__ __forceinline__ T cell_term(const Mod &M, const LvlT<R> &L, const Coefs &Cf, int c,
                                       int m, int j, int k, T &faces, unsigned long long *clamp) {
    const R *A = c ? L.u1 : L.u0;
    const R *B = c ? L.u0 : L.u1;
    if (OP == OP_NEWTON) {
        const NbT<T> s = load_nb<T, R>(A, B, c, m, j, k, L.n, L.logn, L.lognh);
        faces = (s.xp + s.xm) + (s.yp + s.ym) + (s.zp + s.zm);
        const R *D = c ? L.d1 : L.d0;
        const T delta = (T)D[prow(j, k, L.logn, L.lognh) + m];
        (void)clamp;
        return dgp_sigma_over_alpha<T>(M, L, s, delta);
    } else if (OP != OP_ADJ) {
        const NbT<T> s = load_nb<T, R>(A, B, c, m, j, k, L.n, L.logn, L.lognh);
        faces = (s.xp + s.xm) + (s.yp + s.ym) + (s.zp + s.zm);
        const R *D = c ? L.d1 : L.d0;
        const T delta = (T)D[prow(j, k, L.logn, L.lognh) + m];
        return model_term<OP == OP_ADJ ? OP_DGP : OP, T>(M, L, s, delta, clamp);
    } else {
        // (J^T mu)_p = lap(mu)_p - sum over the neighbours q of p of
        // dK_q/dphi_p mu_q.  The face neighbour at p - x carries its x+
        // coefficient, the one at p + x its x- coefficient; edge corners carry
        // +e_xy at p-x-y and p+x+y, -e_xy at p-x+y and p+x-y.
        const int nm1 = L.n - 1, hm1 = (L.n >> 1) - 1;
        const int p = (j + k + c) & 1;
        const int mp = (m + p) & hm1, mm = (m + p - 1) & hm1;
        const int jp = (j + 1) & nm1, jm = (j - 1) & nm1;
        const int kp = (k + 1) & nm1, km = (k - 1) & nm1;
        const int ln = L.logn, lh = L.lognh;
        const size_t r00 = prow(j, k, ln, lh);
        const size_t rp0 = prow(jp, k, ln, lh), rm0 = prow(jm, k, ln, lh);
        const size_t r0p = prow(j, kp, ln, lh), r0m = prow(j, km, ln, lh);
        const size_t rpp = prow(jp, kp, ln, lh), rmm = prow(jm, km, ln, lh);
        const size_t rpm = prow(jp, km, ln, lh), rmp = prow(jm, kp, ln, lh);
        const int o = c ^ 1;
        const size_t ixp = r00 + mp, ixm = r00 + mm, iyp = rp0 + m, iym = rm0 + m,
                     izp = r0p + m, izm = r0m + m;
        const T vxp = B[ixp], vxm = B[ixm], vyp = B[iyp], vym = B[iym], vzp = B[izp],
                vzm = B[izm];
        faces = (vxp + vxm) + (vyp + vym) + (vzp + vzm);
        T g = Cf.c[0][o][ixm] * vxm + Cf.c[1][o][ixp] * vxp + Cf.c[2][o][iym] * vym
            + Cf.c[3][o][iyp] * vyp + Cf.c[4][o][izm] * vzm + Cf.c[5][o][izp] * vzp;
        const double *exy = Cf.c[6][c], *exz = Cf.c[7][c], *eyz = Cf.c[8][c];
        g += (exy[rm0 + mm] * A[rm0 + mm] + exy[rp0 + mp] * A[rp0 + mp])
           - (exy[rp0 + mm] * A[rp0 + mm] + exy[rm0 + mp] * A[rm0 + mp]);
        g += (exz[r0m + mm] * A[r0m + mm] + exz[r0p + mp] * A[r0p + mp])
           - (exz[r0p + mm] * A[r0p + mm] + exz[r0m + mp] * A[r0m + mp]);
        g += (eyz[rmm + m] * A[rmm + m] + eyz[rpp + m] * A[rpp + m])
           - (eyz[rmp + m] * A[rmp + m] + eyz[rpm + m] * A[rpm + m]);
        (void)clamp;
        return g;
    }
}

template <typename T, typename R>
__device__ __forceinline__ T rhs_at(const LvlT<R> &L, int c, size_t idx, const double *fptr,
                                    double fscale) {
    const R *fa = c ? L.f1 : L.f0;
    T f = fa ? (T)fa[idx] : (T)0;
    if (fptr) f += (T)(fscale * (*fptr));
    return f;
}

// One colour pass: every cell of colour c gets the exact solution of its own
// equation (faces - 6 u)/h^2 - K = f given its neighbours.
template <int OP, typename R>
__global__ __launch_bounds__(TPB) void k_pass(Mod M, LvlT<R> L, Coefs Cf, int c,
                                              R *__restrict__ out, const double *fptr,
                                              double fscale, unsigned long long *clamp) {
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    const size_t half = (size_t)1 << (3 * L.logn - 1);
    if (t >= half) return;
    const int m = (int)(t & ((1u << L.lognh) - 1));
    const int j = (int)((t >> L.lognh) & (L.n - 1));
    const int k = (int)(t >> (L.lognh + L.logn));
    R faces;
    const R K = cell_term<OP, R, R>(M, L, Cf, c, m, j, k, faces, clamp);
    const R f = rhs_at<R, R>(L, c, t, fptr, fscale);
    if constexpr (OP == OP_NEWTON)
        out[t] = newton_update<R>(M, (c ? L.u1 : L.u0)[t], faces, K, f, (R)L.h2);
    else
        out[t] = (faces - (R)L.h2 * (K + f)) * (R)(1.0 / 6.0);
}

// Deterministic block sum of two values into partials[2*blk .. 2*blk+1].
__device__ __forceinline__ void block_sum2(double a, double b, double *partials, size_t blk) {
    __shared__ double sa[TPB / 64], sb[TPB / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int q = 0; q < TPB / 64; ++q) {
            x += sa[q];
            y += sb[q];
        }
        partials[2 * blk] = x;
        partials[2 * blk + 1] = y;
    }
}

// Residual d = (faces - 6u)/h^2 - K - f (double arithmetic) at the 8 children
// of coarse cell t, restricted (8-cell mean) together with u.  With REDUCE
// the sums of d and d^2 accumulate into s1, s2 (finest level: norm and mean).
// The loop over the 8 children stays rolled (UNR = 1): unrolled, the adjoint
// and Kmouflage terms need 450-512 registers per lane (one wave per SIMD,
// with spills; the adjoint residual took 11.8 ms at 512^3, 3.8 ms rolled) and
// the single-workgroup tail spills at its 128-register cap.
template <int OP, bool REDUCE, typename R, int UNR = 1>
__device__ __forceinline__ void dev_resid_restrict(const Mod &M, const LvlT<R> &L, const Coefs &Cf,
                                                   const double *fptr, double fscale, R *ru0,
                                                   R *ru1, R *rd0, R *rd1,
                                                   unsigned long long *clamp, size_t t, double &s1,
                                                   double &s2) {
    const int lnc = L.logn - 1, nc = 1 << lnc;
    const size_t ncoarse = (size_t)1 << (3 * lnc);
    if (t < ncoarse) {
        const int I = (int)(t & (nc - 1));
        const int J = (int)((t >> lnc) & (nc - 1));
        const int K = (int)(t >> (2 * lnc));
        double sd = 0.0, su = 0.0;
        const double inv_h2 = 1.0 / L.h2;
#pragma unroll UNR
        for (int q = 0; q < 8; ++q) {
            const int a = q & 1, b = (q >> 1) & 1, cc = q >> 2;
            const int j = 2 * J + b, k = 2 * K + cc;
            const int col = (a + b + cc) & 1;
            double faces;
            double term = cell_term<OP, double, R>(M, L, Cf, col, I, j, k, faces, clamp);
            const size_t idx = prow(j, k, L.logn, L.lognh) + I;
            const double u = (double)(col ? L.u1 : L.u0)[idx];
            if constexpr (OP == OP_NEWTON) term = newton_term(M, term, (faces - 6.0 * u) * inv_h2);
            const double d = (faces - 6.0 * u) * inv_h2 - term
                           - rhs_at<double, R>(L, col, idx, fptr, fscale);
            sd += d;
            su += u;
            if (REDUCE) {
                s1 += d;
                s2 += d * d;
            }
        }
        const int ccol = (I + J + K) & 1;
        const size_t cidx = ((size_t)K << (2 * lnc - 1)) + ((size_t)J << (lnc - 1)) + (I >> 1);
        (ccol ? ru1 : ru0)[cidx] = (R)(0.125 * su);
        (ccol ? rd1 : rd0)[cidx] = (R)(0.125 * sd);
    }
}

template <int OP, bool REDUCE, typename R>
__global__ __launch_bounds__(TPB) void k_resid_restrict(Mod M, LvlT<R> L, Coefs Cf,
                                                        const double *fptr, double fscale, R *ru0,
                                                        R *ru1, R *rd0, R *rd1, double *partials,
                                                        unsigned long long *clamp) {
    const size_t blk = xcd_block(blockIdx.x, gridDim.x);
    const size_t t = blk * TPB + threadIdx.x;
    double s1 = 0.0, s2 = 0.0;
    dev_resid_restrict<OP, REDUCE, R>(M, L, Cf, fptr, fscale, ru0, ru1, rd0, rd1, clamp, t, s1, s2);
    if (REDUCE) block_sum2(s1, s2, partials, blk);
}

// Starting value of the finest level's bordering scalar mu: the mean of
// L(phi) - f over 64 cells spread over the mesh (one wave).  The finest
// residual is reduced in one pass, eps^2 = <d^2> - <d>^2, which cancels when
// |<d>| is many orders above eps.  A call's first residual evaluation would
// otherwise see mu = 0 and <d> = the whole mean of L(phi); started from this
// estimate, its <d> is of the order of the residual's spread, and its update
// mu += <d> gives the mean over all cells as before.
template <int OP, typename R>
__global__ __launch_bounds__(64) void k_mu_estimate(Mod M, LvlT<R> L, Coefs Cf, double *mu) {
    const int t = threadIdx.x;
    const int c = t & 1;
    const int m = (t * 5) & ((L.n >> 1) - 1);
    const int j = (t * 7 + 1) & (L.n - 1);
    const int k = (t * 11 + 2) & (L.n - 1);
    double faces;
    double term = cell_term<OP, double, R>(M, L, Cf, c, m, j, k, faces, nullptr);
    const size_t idx = prow(j, k, L.logn, L.lognh) + m;
    const double D = (faces - 6.0 * (double)(c ? L.u1 : L.u0)[idx]) / L.h2;
    if constexpr (OP == OP_NEWTON) term = newton_term(M, term, D);
    double d = D - term - rhs_at<double, R>(L, c, idx, nullptr, 0.0);
    for (int off = 32; off > 0; off >>= 1) d += __shfl_down(d, off, 64);
    if (t == 0) *mu = d * (1.0 / 64.0);
}

// FAS source on the coarse level: S = L^H(R u) - (R d - shift), written over
// the restricted residual; the coarse unknown starts from R u.
template <int OP, typename R>
__device__ __forceinline__ void dev_coarse_source(const Mod &M, const LvlT<R> &Lc, const Coefs &Cf,
                                                  R *s0, R *s1, R *u0, R *u1, const double *shift,
                                                  size_t t) {
    const size_t half = (size_t)1 << (3 * Lc.logn - 1);
    if (t >= 2 * half) return;
    const int c = t >= half;
    const size_t tt = t - (c ? half : 0);
    const int m = (int)(tt & ((1u << Lc.lognh) - 1));
    const int j = (int)((tt >> Lc.lognh) & (Lc.n - 1));
    const int k = (int)(tt >> (Lc.lognh + Lc.logn));
    double faces;
    double term = cell_term<OP, double, R>(M, Lc, Cf, c, m, j, k, faces, nullptr);
    const R ru = (c ? Lc.u1 : Lc.u0)[tt];
    if constexpr (OP == OP_NEWTON) term = newton_term(M, term, (faces - 6.0 * (double)ru) / Lc.h2);
    R *S = c ? s1 : s0;
    const double rd = (double)S[tt] - (shift ? *shift : 0.0);
    S[tt] = (R)((faces - 6.0 * (double)ru) / Lc.h2 - term - rd);
    (c ? u1 : u0)[tt] = ru;
}

template <int OP, typename R>
__global__ __launch_bounds__(TPB) void k_coarse_source(Mod M, LvlT<R> Lc, Coefs Cf, R *s0, R *s1,
                                                       R *u0, R *u1, const double *shift) {
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    dev_coarse_source<OP, R>(M, Lc, Cf, s0, s1, u0, u1, shift, t);
}

// u_fine += P(uc - rc) with the cell-centred trilinear weights 27/9/3/1 (/64).
template <typename R>
__device__ __forceinline__ void dev_prolong(R *f0, R *f1, int logn, const R *uc0, const R *uc1,
                                            const R *rc0, const R *rc1, size_t t) {
    const int n = 1 << logn, lognh = logn - 1;
    const size_t half = (size_t)1 << (3 * logn - 1);
    if (t >= 2 * half) return;
    const int c = t >= half;
    const size_t tt = t - (c ? half : 0);
    const int m = (int)(tt & ((1u << lognh) - 1));
    const int j = (int)((tt >> lognh) & (n - 1));
    const int k = (int)(tt >> (lognh + logn));
    const int p = (j + k + c) & 1;   // i = 2m + p, parent I = m
    const int lnc = logn - 1, ncm1 = (1 << lnc) - 1;
    const int I = m, J = j >> 1, K = k >> 1;
    const int di = p ? 1 : -1, dj = (j & 1) ? 1 : -1, dk = (k & 1) ? 1 : -1;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int a = q & 1, b = (q >> 1) & 1, cc = q >> 2;
        const int I2 = (I + a * di) & ncm1, J2 = (J + b * dj) & ncm1, K2 = (K + cc * dk) & ncm1;
        const size_t idx = ((size_t)K2 << (2 * lnc - 1)) + ((size_t)J2 << (lnc - 1)) + (I2 >> 1);
        const double v = ((I2 + J2 + K2) & 1) ? ((double)uc1[idx] - (double)rc1[idx])
                                              : ((double)uc0[idx] - (double)rc0[idx]);
        const double w = (a ? 1.0 : 3.0) * (b ? 1.0 : 3.0) * (cc ? 1.0 : 3.0);
        acc += w * v;
    }
    R *f = c ? f1 : f0;
    f[tt] = (R)((double)f[tt] + acc * (1.0 / 64.0));
}

template <typename R>
__global__ __launch_bounds__(TPB) void k_prolong(R *f0, R *f1, int logn, const R *uc0,
                                                 const R *uc1, const R *rc0, const R *rc1) {
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    dev_prolong<R>(f0, f1, logn, uc0, uc1, rc0, rc1, t);
}

// 8-cell mean of a packed field (density hierarchy, linearisation points).
template <typename R>
__global__ __launch_bounds__(TPB) void k_restrict(const R *f0, const R *f1, int logn, R *c0,
                                                  R *c1) {
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    const int lnc = logn - 1, nc = 1 << lnc;
    if (t >= ((size_t)1 << (3 * lnc))) return;
    const int I = (int)(t & (nc - 1)), J = (int)((t >> lnc) & (nc - 1)), K = (int)(t >> (2 * lnc));
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int a = q & 1, b = (q >> 1) & 1, cc = q >> 2;
        const int j = 2 * J + b, k = 2 * K + cc;
        const size_t idx = ((size_t)k << (2 * logn - 1)) + ((size_t)j << (logn - 1)) + I;
        s += ((a + b + cc) & 1) ? (double)f1[idx] : (double)f0[idx];
    }
    const size_t cidx = ((size_t)K << (2 * lnc - 1)) + ((size_t)J << (lnc - 1)) + (I >> 1);
    (((I + J + K) & 1) ? c1 : c0)[cidx] = (R)(0.125 * s);
}

// natural [z][y][x] -> packed colours (optionally minus a device scalar),
// converting the element type
template <typename Rin, typename Rout>
__global__ __launch_bounds__(TPB) void k_pack(const Rin *nat, int logn, Rout *c0, Rout *c1,
                                              const double *shift) {
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    if (t >= ((size_t)1 << (3 * logn))) return;
    const int n = 1 << logn;
    const int i = (int)(t & (n - 1)), j = (int)((t >> logn) & (n - 1)), k = (int)(t >> (2 * logn));
    const size_t idx = ((size_t)k << (2 * logn - 1)) + ((size_t)j << (logn - 1)) + (i >> 1);
    const double v = (double)nat[t] - (shift ? *shift : 0.0);
    (((i + j + k) & 1) ? c1 : c0)[idx] = (Rout)v;
}

// packed colours -> natural (optionally minus a device scalar)
template <typename Rin, typename Rout>
__global__ __launch_bounds__(TPB) void k_unpack(const Rin *c0, const Rin *c1, int logn,
                                                Rout *nat, const double *shift) {
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    if (t >= ((size_t)1 << (3 * logn))) return;
    const int n = 1 << logn;
    const int i = (int)(t & (n - 1)), j = (int)((t >> logn) & (n - 1)), k = (int)(t >> (2 * logn));
    const size_t idx = ((size_t)k << (2 * logn - 1)) + ((size_t)j << (logn - 1)) + (i >> 1);
    const double v = (double)(((i + j + k) & 1) ? c1 : c0)[idx];
    nat[t] = (Rout)(v - (shift ? *shift : 0.0));
}

// element-wise conversion between precisions (same packed layout)
template <typename Rin, typename Rout>
__global__ __launch_bounds__(TPB) void k_convert(const Rin *a, Rout *b, size_t n) {
    const size_t t = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (t < n) b[t] = (Rout)a[t];
}

// Block sums of a (and a^2) over up to two arrays laid end to end.
template <typename R>
__global__ __launch_bounds__(TPB) void k_sum(const R *a0, const R *a1, size_t nhalf,
                                             double *partials) {
    // grid-stride: a fixed grid for a given size keeps the order deterministic
    const size_t stride = (size_t)gridDim.x * TPB;
    double v = 0.0, v2 = 0.0;
    for (size_t t = (size_t)blockIdx.x * TPB + threadIdx.x; t < nhalf; t += stride) {
        const double x = (double)a0[t];
        v += x;
        v2 += x * x;
    }
    if (a1) {
        for (size_t t = (size_t)blockIdx.x * TPB + threadIdx.x; t < nhalf; t += stride) {
            const double x = (double)a1[t];
            v += x;
            v2 += x * x;
        }
    }
    block_sum2(v, v2, partials, blockIdx.x);
}

// Finalise a reduction.  mode 0: residual of the finest level with lagged mu
// (mu += mean, shift = mean, eps2 = variance); mode 1: plain mean into
// S_MEAN; mode 2: adjoint residual r = d - kappa*mean(mu) with mean(mu) in
// S_MEAN (shift = 0, eps2 = mean r^2); mode 3: the sum of one colour (colour)
// of the adjoint field into S_CSUM0 + colour, and S_MEAN = the mean of both
// colours' sums; mode 4: both colours' sums at once (first and second
// components); mode 5: mode 0 for the FP64 residual of the defect-correction
// solve (S_MU64 and S_EPS64).  Summation order is fixed.
__global__ __launch_bounds__(1024) void k_finalize(const double *partials, size_t nblocks,
                                                   double ncells, double *scal, int mode,
                                                   double kappa, int colour = 0) {
    __shared__ double sa[16], sb[16];
    double a = 0.0, b = 0.0;
    for (size_t q = threadIdx.x; q < nblocks; q += 1024) {
        a += partials[2 * q];
        b += partials[2 * q + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sa[threadIdx.x >> 6] = a;
        sb[threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int q = 0; q < 16; ++q) {
            x += sa[q];
            y += sb[q];
        }
        const double mean = x / ncells, msq = y / ncells;
        if (mode == 0) {
            scal[S_MU] += mean;
            scal[S_SHIFT] = mean;
            const double v = msq - mean * mean;
            scal[S_EPS2] = v < 0.0 ? 0.0 : v;   // keeps NaN
        } else if (mode == 1) {
            scal[S_MEAN] = mean;
        } else if (mode == 3) {
            scal[S_CSUM0 + colour] = x;
            scal[S_MEAN] = (scal[S_CSUM0] + scal[S_CSUM1]) / ncells;
        } else if (mode == 5) {
            scal[S_MU64] += mean;
            const double v = msq - mean * mean;
            scal[S_EPS64] = v < 0.0 ? 0.0 : v;   // keeps NaN
        } else if (mode == 4) {
            scal[S_CSUM0] = x;
            scal[S_CSUM1] = y;
            scal[S_MEAN] = (x + y) / ncells;
        } else {
            const double km = kappa * scal[S_MEAN];
            scal[S_SHIFT] = 0.0;
            const double v = msq - 2.0 * km * mean + km * km;
            scal[S_EPS2] = v < 0.0 ? 0.0 : v;   // keeps NaN
        }
    }
}

__global__ void k_fill(double *a, size_t n, double v) {
    const size_t t = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (t < n) a[t] = v;
}

__global__ void k_fill_u64(unsigned long long *a, size_t n) {
    const size_t t = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (t < n) a[t] = 0ull;
}

// Residual r = (faces - 6u)/h^2 - term - f at every cell, packed output (double).
template <int OP>
__global__ __launch_bounds__(TPB) void k_residual(Mod M, Lvl L, Coefs Cf, const double *fptr,
                                                  double fscale, double *r0, double *r1,
                                                  unsigned long long *clamp) {
    const size_t t = xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
    const size_t half = (size_t)1 << (3 * L.logn - 1);
    if (t >= 2 * half) return;
    const int c = t >= half;
    const size_t tt = t - (c ? half : 0);
    const int m = (int)(tt & ((1u << L.lognh) - 1));
    const int j = (int)((tt >> L.lognh) & (L.n - 1));
    const int k = (int)(tt >> (L.lognh + L.logn));
    double faces;
    double term = cell_term<OP, double, double>(M, L, Cf, c, m, j, k, faces, clamp);
    const double u = (c ? L.u1 : L.u0)[tt];
    if constexpr (OP == OP_NEWTON) term = newton_term(M, term, (faces - 6.0 * u) / L.h2);
    (c ? r1 : r0)[tt] = (faces - 6.0 * u) / L.h2 - term
                      - rhs_at<double, double>(L, c, tt, fptr, fscale);
}

// ---------------------------------------------------------------- coarse tail
// All levels from 16^3 down to 4^3 in one workgroup: the sub-cycle (smoothing,
// residual + restriction, coarse source, recursion, prolongation) runs with
// barriers between phases instead of one launch per phase.  A colour pass
// first computes every new value of the colour into registers, then writes
// them in place after a barrier, so all cells see the pre-pass state.
constexpr int TAIL_THREADS = 1024;
constexpr int TAIL_MAX_N = 16;   // <= 2048 cells per colour: 2 per thread
constexpr int TAIL_MAX_LEVELS = 3;

template <typename R>
struct TailLv {
    LvlT<R> L;      // u, d and f (the FAS source, workspace: written by the tail)
    R *ru0, *ru1;   // R u of the finer level (unused on the first tail level)
};

template <typename R>
struct TailArgs {
    int nlev, nu1, nu2, nuc;
    int cycle;   // 0 V, 1 F, 2 W
    TailLv<R> lv[TAIL_MAX_LEVELS];
    Coefs cf[TAIL_MAX_LEVELS];
};

template <int OP, typename R>
__device__ void tail_pass(const Mod &M, const TailLv<R> &T, const Coefs &Cf, int c) {
    const LvlT<R> &L = T.L;
    const int half = 1 << (3 * L.logn - 1);
    R nv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int t = threadIdx.x + q * TAIL_THREADS;
        if (t < half) {
            const int m = t & ((1 << L.lognh) - 1);
            const int j = (t >> L.lognh) & (L.n - 1);
            const int k = t >> (L.lognh + L.logn);
            R faces;
            const R K = cell_term<OP, R, R>(M, L, Cf, c, m, j, k, faces, nullptr);
            const R f = (c ? L.f1 : L.f0)[t];
            if constexpr (OP == OP_NEWTON)
                nv[q] = newton_update<R>(M, (c ? L.u1 : L.u0)[t], faces, K, f, (R)L.h2);
            else
                nv[q] = (faces - (R)L.h2 * (K + f)) * (R)(1.0 / 6.0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int t = threadIdx.x + q * TAIL_THREADS;
        if (t < half) (c ? L.u1 : L.u0)[t] = nv[q];
    }
    __syncthreads();
}

template <int OP, typename R>
__device__ void tail_sweeps(const Mod &M, const TailLv<R> &T, const Coefs &Cf, int count) {
    for (int s = 0; s < count; ++s) {
        tail_pass<OP, R>(M, T, Cf, 0);
        tail_pass<OP, R>(M, T, Cf, 1);
    }
}

// The sweeps of a level with at most 64 cells per colour (the 4^3 level) on
// the first wavefront alone: a lane per cell, and no workgroup barrier
// between passes.  A wavefront's LDS reads and writes take effect in program
// order, so every read of a pass precedes its writes and follows the previous
// pass's writes, as in tail_pass.
template <int OP, typename R>
__device__ void tail_sweeps_wave(const Mod &M, const TailLv<R> &T, const Coefs &Cf, int count) {
    const LvlT<R> &L = T.L;
    const int half = 1 << (3 * L.logn - 1);
    const int t = threadIdx.x;
    if (t < 64) {
        const int m = t & ((1 << L.lognh) - 1);
        const int j = (t >> L.lognh) & (L.n - 1);
        const int k = t >> (L.lognh + L.logn);
        for (int s = 0; s < count; ++s) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                R nv = (R)0;
                if (t < half) {
                    R faces;
                    const R K = cell_term<OP, R, R>(M, L, Cf, c, m, j, k, faces, nullptr);
                    const R f = (c ? L.f1 : L.f0)[t];
                    if constexpr (OP == OP_NEWTON)
                        nv = newton_update<R>(M, (c ? L.u1 : L.u0)[t], faces, K, f, (R)L.h2);
                    else
                        nv = (faces - (R)L.h2 * (K + f)) * (R)(1.0 / 6.0);
                }
                __builtin_amdgcn_wave_barrier();
                if (t < half) (c ? L.u1 : L.u0)[t] = nv;
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    __syncthreads();
}

// Elements of LDS the tail needs for levels l0 .. (u, d, f of every level,
// R u of every level below the first).
__host__ __device__ inline int tail_lds_elems(int logn0, int nl) {
    int tot = 0;
    for (int q = 0; q < nl; ++q) tot += (q ? 8 : 6) * (1 << (3 * (logn0 - q) - 1));
    return tot;
}

// FAS transfer from tail level l to l+1: residual, R u and R d, coarse source.
template <int OP, int NL, typename R>
__device__ __forceinline__ void tail_restrict(const Mod &M, TailLv<R> (&T)[NL],
                                              const Coefs (&Cf)[NL], int l) {
    TailLv<R> &Tc = T[l + 1];
    double s1 = 0.0, s2 = 0.0;
    const int ncoarse = 1 << (3 * Tc.L.logn);
    for (int t = threadIdx.x; t < ncoarse; t += TAIL_THREADS)
        dev_resid_restrict<OP, false, R>(M, T[l].L, Cf[l], nullptr, 0.0, Tc.ru0, Tc.ru1,
                                         const_cast<R *>(Tc.L.f0), const_cast<R *>(Tc.L.f1),
                                         nullptr, (size_t)t, s1, s2);
    __syncthreads();
    LvlT<R> Lr = Tc.L;
    Lr.u0 = Tc.ru0;
    Lr.u1 = Tc.ru1;
    for (int t = threadIdx.x; t < ncoarse; t += TAIL_THREADS)
        dev_coarse_source<OP, R>(M, Lr, Cf[l + 1], const_cast<R *>(Tc.L.f0),
                                 const_cast<R *>(Tc.L.f1), Tc.L.u0, Tc.L.u1, nullptr, (size_t)t);
    __syncthreads();
}

// One cycle (0 V, 1 F, 2 W) on tail level LV, recursing at compile time.
template <int OP, int NL, int LV, typename R>
__device__ __forceinline__ void tail_cycle(const Mod &M, TailLv<R> (&T)[NL], const Coefs (&Cf)[NL],
                           const TailArgs<R> &A, int type) {
    if constexpr (LV == NL - 1) {
        if (T[LV].L.n == 4)
            tail_sweeps_wave<OP, R>(M, T[LV], Cf[LV], A.nuc);
        else
            tail_sweeps<OP, R>(M, T[LV], Cf[LV], A.nuc);
    } else {
        tail_sweeps<OP, R>(M, T[LV], Cf[LV], A.nu1);
        tail_restrict<OP, NL, R>(M, T, Cf, LV);
        if (type == 2) {
            tail_cycle<OP, NL, LV + 1, R>(M, T, Cf, A, 2);
            tail_cycle<OP, NL, LV + 1, R>(M, T, Cf, A, 2);
        } else if (type == 1) {
            tail_cycle<OP, NL, LV + 1, R>(M, T, Cf, A, 1);
            tail_cycle<OP, NL, LV + 1, R>(M, T, Cf, A, 0);
        } else {
            tail_cycle<OP, NL, LV + 1, R>(M, T, Cf, A, 0);
        }
        const TailLv<R> &Tf = T[LV], &Tc = T[LV + 1];
        const int nfine = 1 << (3 * Tf.L.logn);
        for (int t = threadIdx.x; t < nfine; t += TAIL_THREADS)
            dev_prolong<R>(Tf.L.u0, Tf.L.u1, Tf.L.logn, Tc.L.u0, Tc.L.u1, Tc.ru0, Tc.ru1,
                           (size_t)t);
        __syncthreads();
        tail_sweeps<OP, R>(M, Tf, Cf[LV], A.nu2);
    }
}

template <typename R>
__device__ __forceinline__ void lds_copy(R *dst, const R *src, int n) {
    for (int t = threadIdx.x; t < n; t += TAIL_THREADS) dst[t] = src[t];
}

// The tail levels live in LDS for the whole sub-cycle: their fields are
// copied in, the sub-cycle runs on LDS, and the first level's u goes back.
template <int OP, int NL, typename R>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail(Mod M, TailArgs<R> A) {
    extern __shared__ double lds_raw[];
    R *lds = reinterpret_cast<R *>(lds_raw);
    TailLv<R> T[NL];
    Coefs Cf[NL];
    R *p = lds;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const TailLv<R> &G = A.lv[q];
        const int half = 1 << (3 * G.L.logn - 1);
        T[q] = G;
        Cf[q] = A.cf[q];
        R *u0 = p, *u1 = p + half, *d0 = p + 2 * half, *d1 = p + 3 * half;
        R *f0 = p + 4 * half, *f1 = p + 5 * half;
        p += 6 * half;
        T[q].L.u0 = u0;
        T[q].L.u1 = u1;
        T[q].L.d0 = d0;
        T[q].L.d1 = d1;
        T[q].L.f0 = f0;
        T[q].L.f1 = f1;
        lds_copy<R>(d0, G.L.d0, half);
        lds_copy<R>(d1, G.L.d1, half);
        if (q == 0) {
            lds_copy<R>(u0, G.L.u0, half);
            lds_copy<R>(u1, G.L.u1, half);
            lds_copy<R>(f0, G.L.f0, half);
            lds_copy<R>(f1, G.L.f1, half);
        } else {
            T[q].ru0 = p;
            T[q].ru1 = p + half;
            p += 2 * half;
        }
    }
    __syncthreads();
    tail_cycle<OP, NL, 0, R>(M, T, Cf, A, A.cycle);
    const int half0 = 1 << (3 * A.lv[0].L.logn - 1);
    lds_copy<R>(A.lv[0].L.u0, T[0].L.u0, half0);
    lds_copy<R>(A.lv[0].L.u1, T[0].L.u1, half0);
}

}  // namespace mgk
