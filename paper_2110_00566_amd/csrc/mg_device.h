// Device-side building blocks of the multigrid solve (gfx950, wave64).
//
// Storage: every mesh level keeps each red-black colour in its own packed
// half-array.  Cell (i, j, k) of an n^3 level has colour c = (i+j+k) & 1 and
// lives at  a_c[(k*n + j)*(n/2) + (i >> 1)].  A colour pass therefore reads
// the opposite colour (6 face neighbours) and its own colour (12 edge
// neighbours of the 19-point stencil) and writes a fresh array for its
// colour, so every cell of the colour is updated from the pre-pass state
// (the edge neighbours share the centre's colour).  Consecutive threads own
// consecutive packed x positions, so every load and store is coalesced.
//
// Precision: the storage type R is double (FP64 solve) or float (the FP32
// phase of the mixed solve).  With float storage the nDGP colour pass runs in
// float, with the closed-form root in its cancellation-free form (the
// Kmouflage term keeps its sums and division in double); the residual
// evaluates the Laplacian in double from the float values and the nDGP term
// in float; restriction sums and reductions are always evaluated in double.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgk {

enum { MODEL_DGP = 0, MODEL_KMO = 1, MODEL_POISSON = 2 };

// Level-independent model coefficients (host-computed).
struct Mod {
    double alpha, sgn, s;     // nDGP: alpha = 3 beta a^2 / R_c^2, s = alpha Omega_m/(beta a)
    double ctil, src;         // Kmouflage: c~, 3 beta A(phibar) Omega_m / a
    double c0;                // 1 + gamma (phibar'/H0)^(2(n-1))
    double a1;                // (2n+1) gamma / 3
    double b2;                // -2 c~ (n-1) gamma
    int nk;
};

// One level as seen by a kernel (storage type R).
template <typename R>
struct LvlT {
    R *u0, *u1;                   // current field, colour 0 / colour 1
    const R *d0, *d1;             // density contrast
    const R *f0, *f1;             // FAS right-hand side (null: scalar mu)
    int n, logn, lognh;
    double h2;                    // h^2
    double c3h4, c8h4;            // 1/(3 h^4), 1/(8 h^4)
    double c12h4, c4h2;           // 1/(12 h^4), 1/(4 h^2)
};
using Lvl = LvlT<double>;

__device__ __forceinline__ size_t prow(int j, int k, int logn, int lognh) {
    return ((size_t)k << (logn + lognh)) + ((size_t)j << lognh);
}

// The 19-point neighbourhood of one cell in the form the operators need.
template <typename T>
struct NbT {
    T xp, xm, yp, ym, zp, zm;   // face neighbours
    T nxy, nxz, nyz;            // 4-point cross differences (x 4h^2 D_ij)
};
using Nb = NbT<double>;

// Neighbourhood of the cell of colour c at packed (m, j, k).  A holds colour
// c (edge neighbours), B colour 1-c (face neighbours).
template <typename T, typename R>
__device__ __forceinline__ NbT<T> load_nb(const R *__restrict__ A, const R *__restrict__ B, int c,
                                          int m, int j, int k, int n, int logn, int lognh) {
    const int nm1 = n - 1, hm1 = (n >> 1) - 1;
    const int p = (j + k + c) & 1;              // i = 2m + p
    const int mp = (m + p) & hm1;               // packed index of i+1
    const int mm = (m + p - 1) & hm1;           // packed index of i-1
    const int jp = (j + 1) & nm1, jm = (j - 1) & nm1;
    const int kp = (k + 1) & nm1, km = (k - 1) & nm1;
    const size_t r00 = prow(j, k, logn, lognh);
    const size_t rp0 = prow(jp, k, logn, lognh), rm0 = prow(jm, k, logn, lognh);
    const size_t r0p = prow(j, kp, logn, lognh), r0m = prow(j, km, logn, lognh);
    const size_t rpp = prow(jp, kp, logn, lognh), rmm = prow(jm, km, logn, lognh);
    const size_t rpm = prow(jp, km, logn, lognh), rmp = prow(jm, kp, logn, lognh);
    NbT<T> s;
    s.xp = (T)B[r00 + mp];
    s.xm = (T)B[r00 + mm];
    s.yp = (T)B[rp0 + m];
    s.ym = (T)B[rm0 + m];
    s.zp = (T)B[r0p + m];
    s.zm = (T)B[r0m + m];
    s.nxy = ((T)A[rp0 + mp] + (T)A[rm0 + mm]) - ((T)A[rm0 + mp] + (T)A[rp0 + mm]);
    s.nxz = ((T)A[r0p + mp] + (T)A[r0m + mm]) - ((T)A[r0m + mp] + (T)A[r0p + mm]);
    s.nyz = ((T)A[rpp + m] + (T)A[rmm + m]) - ((T)A[rpm + m] + (T)A[rmp + m]);
    return s;
}

// Model term K of L = lap(phi) - K at one cell, arithmetic type T for the
// stencil combinations, double for the root.  K never involves the centre
// value, so a colour pass solves each cell's equation exactly.
//
// nDGP (Sec. 3.2.3): Sigma = hat(H):hat(H) + s delta where, with
// A_x = phi(i+1)+phi(i-1) etc. and the cross differences N_xy,
//   hat(H):hat(H) = [(A_x-A_y)^2 + (A_x-A_z)^2 + (A_y-A_z)^2]/(3h^4)
//                   + (N_xy^2 + N_xz^2 + N_yz^2)/(8h^4),
// and K is the root of eq:DGP, (3/4)[-alpha + sign(alpha) sqrt(D)] with
// D = alpha^2 + 8 Sigma/3, in that form.  Its cancellation for Sigma << alpha^2
// costs an absolute error of about one ulp of alpha (~1e-15 here), far below
// any residual tolerance, and saves the division of the cancellation-free
// 2 Sigma / (alpha + sign(alpha) sqrt(D)).  D < 0 is clamped to 0 (K = -3 alpha/4).
// Sigma / alpha of the nDGP operator at one cell (no centre dependence).
template <typename T, typename L_>
__device__ __forceinline__ T dgp_sigma_over_alpha(const Mod &M, const L_ &L, const NbT<T> &s,
                                                  T delta) {
    const T ax = s.xp + s.xm, ay = s.yp + s.ym, az = s.zp + s.zm;
    const T dxy = ax - ay, dxz = ax - az, dyz = ay - az;
    const T t3 = dxy * dxy + dxz * dxz + dyz * dyz;
    const T t8 = s.nxy * s.nxy + s.nxz * s.nxz + s.nyz * s.nyz;
    const double sig = (double)t3 * L.c3h4 + (double)t8 * L.c8h4 + M.s * (double)delta;
    return (T)(sig / M.alpha);
}

template <int MODEL, typename T, typename L_>
__device__ __forceinline__ T model_term(const Mod &M, const L_ &L, const NbT<T> &s, T delta,
                                        unsigned long long *clamp) {
    if (MODEL == MODEL_POISSON) return (T)M.s * delta;
    const T ax = s.xp + s.xm, ay = s.yp + s.ym, az = s.zp + s.zm;
    if (MODEL == MODEL_DGP) {
        const T dxy = ax - ay, dxz = ax - az, dyz = ay - az;
        const T t3 = dxy * dxy + dxz * dxz + dyz * dyz;
        const T t8 = s.nxy * s.nxy + s.nxz * s.nxz + s.nyz * s.nyz;
        if constexpr (sizeof(T) == 4) {
            // FP32 storage: the whole term in FP32, the root in the
            // cancellation-free form 2 Sigma / (alpha + sign(alpha) sqrt(D))
            // (equal to the printed one; accurate relative to K when
            // Sigma << alpha^2).  A clamped D gives -3 alpha / 4 as above.
            const float sig = t3 * (float)L.c3h4 + t8 * (float)L.c8h4 + (float)M.s * delta;
            const float disc = (float)(M.alpha * M.alpha) + (8.0f / 3.0f) * sig;
            if (disc < 0.0f) {
                if (clamp) atomicAdd(clamp, 1ull);
                return (T)(-0.75 * M.alpha);
            }
            return 2.0f * sig / ((float)M.alpha + (float)M.sgn * sqrtf(disc));
        }
        const double sig = (double)t3 * L.c3h4 + (double)t8 * L.c8h4 + M.s * (double)delta;
        double disc = M.alpha * M.alpha + (8.0 / 3.0) * sig;
        if (disc < 0.0) {
            disc = 0.0;
            if (clamp) atomicAdd(clamp, 1ull);
        }
        return (T)(0.75 * (M.sgn * sqrt(disc) - M.alpha));
    }
    // Kmouflage split form eq:kmf_eqn_codeunit_final: with e = 2h grad phi,
    //   g = |e|^2/(4h^2),  Q = hat(H)_ij G_i G_j
    //     = [e_x^2 (2A_x-A_y-A_z) + ...]/(12 h^4) + (N_xy e_x e_y + ...)/(8 h^4),
    //   K = (src delta + b2 g^(n-2) Q) / (c~ (c0 + a1 g^(n-1))).
    const T ex = s.xp - s.xm, ey = s.yp - s.ym, ez = s.zp - s.zm;
    if constexpr (sizeof(T) == 4) {
        // FP32 storage: the whole term in FP32 (its relative error stays far
        // below that of the FP32-stored field)
        const float g = (ex * ex + ey * ey + ez * ez) * (float)L.c4h2;
        const float q = (ex * ex * (2 * ax - ay - az) + ey * ey * (2 * ay - ax - az)
                         + ez * ez * (2 * az - ax - ay)) * (float)L.c12h4
                      + (s.nxy * ex * ey + s.nxz * ex * ez + s.nyz * ey * ez) * (float)L.c8h4;
        float gn2 = 1.0f;
        for (int t = 0; t < M.nk - 2; ++t) gn2 *= g;
        const float sig1 = (float)M.c0 + (float)M.a1 * gn2 * g;
        const float sig2 = (float)M.b2 * gn2 * q;
        return ((float)M.src * delta + sig2) / ((float)M.ctil * sig1);
    }
    const double g = (double)(ex * ex + ey * ey + ez * ez) * L.c4h2;
    const double q = (double)(ex * ex * (2 * ax - ay - az) + ey * ey * (2 * ay - ax - az)
                              + ez * ez * (2 * az - ax - ay)) * L.c12h4
                   + (double)(s.nxy * ex * ey + s.nxz * ex * ez + s.nyz * ey * ez) * L.c8h4;
    double gn2 = 1.0;
    for (int t = 0; t < M.nk - 2; ++t) gn2 *= g;
    const double sig1 = M.c0 + M.a1 * gn2 * g;
    const double sig2 = M.b2 * gn2 * q;
    return (T)((M.src * (double)delta + sig2) / (M.ctil * sig1));
}

// Correction form of the nDGP model term, used by the defect-correction
// cycles of the mixed-precision solve: the change of K between the field
// pb + e and the background pb, evaluated without cancellation so that it
// is accurate relative to itself when e is small.  With the stencil
// combinations a (of pb) and b (of e), T(pb + e) - T(pb) = sum (2a + b) b
// over the quadratic terms of T, and with D = alpha^2 + 8 Sigma / 3,
//   K(pb + e) - K(pb) = (3/4) sign(alpha) (sqrt(D1) - sqrt(D0))
//                     = 2 sign(alpha) dSigma / (sqrt(D1) + sqrt(D0)).
// The Poisson model term does not depend on the field (the change is 0).
template <int MODEL, typename T, typename L_>
__device__ __forceinline__ T corr_term(const Mod &M, const L_ &L, const NbT<T> &a,
                                       const NbT<T> &b, T delta) {
    if (MODEL == MODEL_POISSON) return (T)0;
    const T ax = a.xp + a.xm, ay = a.yp + a.ym, az = a.zp + a.zm;
    const T bx = b.xp + b.xm, by = b.yp + b.ym, bz = b.zp + b.zm;
    const T dxy = ax - ay, dxz = ax - az, dyz = ay - az;
    const T exy = bx - by, exz = bx - bz, eyz = by - bz;
    const T t3 = dxy * dxy + dxz * dxz + dyz * dyz;
    const T t8 = a.nxy * a.nxy + a.nxz * a.nxz + a.nyz * a.nyz;
    const T dt3 = ((T)2 * dxy + exy) * exy + ((T)2 * dxz + exz) * exz + ((T)2 * dyz + eyz) * eyz;
    const T dt8 = ((T)2 * a.nxy + b.nxy) * b.nxy + ((T)2 * a.nxz + b.nxz) * b.nxz
                + ((T)2 * a.nyz + b.nyz) * b.nyz;
    const T sig0 = t3 * (T)L.c3h4 + t8 * (T)L.c8h4 + (T)M.s * delta;
    const T dsig = dt3 * (T)L.c3h4 + dt8 * (T)L.c8h4;
    T d0 = (T)(M.alpha * M.alpha) + (T)(8.0 / 3.0) * sig0;
    T d1 = d0 + (T)(8.0 / 3.0) * dsig;
    d0 = d0 > (T)0 ? d0 : (T)0;
    d1 = d1 > (T)0 ? d1 : (T)0;
    const T den = sqrt(d1) + sqrt(d0);
    return den > (T)0 ? (T)(2.0 * M.sgn) * dsig / den : (T)0;
}

}  // namespace mgk
