// Kernels of the defect-correction form of the mixed-precision solve, on the
// finest level (>= 128^3, LDS-tiled like the FP32 kernels of mg_tiled.h).
//
// An outer step evaluates the FP64 residual r of the FP64 field phi64 and
// stores g = -r in FP32; the inner cycles then solve, in FP32, for a
// correction e of the frozen background pb = fl32(phi64):
//     A(e) = lap(e) - [K(pb + e) - K(pb)] = g + mu',
// with the model-term difference in the cancellation-free form of corr_term
// (so the FP32 arithmetic is accurate relative to e and r, not to |phi|),
// and mu' the inner bordering scalar (mean of the inner residual, lagged as
// on the finest level of the plain solve).  The coarse levels of an inner
// cycle are the FP64 FAS levels of the whole field: they receive
// R(pb + e) and R(inner residual) in FP64.  Then phi64 += e.
#pragma once
#include "mg_tiled.h"

namespace mgk {

// One FP32 colour pass of the correction equation: e of colour c from its
// neighbourhood, the background's, delta and g.  LDS: rings of 3 planes of
// both colours of e and pb (31.8 KB).
template <int MODEL>
__global__ __launch_bounds__(TPB) void k_corr_pass_tiled(Mod M, LvlT<float> L, const float *pb0,
                                                         const float *pb1, int c,
                                                         float *__restrict__ out,
                                                         const double *fptr, TileGeom G) {
    __shared__ __align__(16) float sA[3][TSLOT], sB[3][TSLOT], pA[3][TSLOT], pB[3][TSLOT];
    const size_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int bx = (int)(blk % G.ntx);
    const int by = (int)((blk / G.ntx) % G.nty);
    const int bz = (int)(blk / ((size_t)G.ntx * G.nty));
    const int m0 = bx * TX, j0 = by * TY, k0 = bz * G.kz;
    const float *A = c ? L.u1 : L.u0, *B = c ? L.u0 : L.u1;
    const float *PA = c ? pb1 : pb0, *PB = c ? pb0 : pb1;
    const float *D = c ? L.d1 : L.d0, *F = c ? L.f1 : L.f0;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const float fs = fptr ? (float)(*fptr) : 0.f;
    const float h2 = (float)L.h2;
    unsigned coff[2];
    Stage2<float> S, P;
    S.init(tid, j0, m0, L.logn, L.lognh);
    P.init(tid, j0, m0, L.logn, L.lognh);
#pragma unroll
    for (int h = 0; h < 2; ++h) coff[h] = cell_off<float>(j0 + ty + 4 * h, m0 + tx, L.lognh);
    auto fetch = [&](int k) {
        const size_t pl = plane_off<float>(k, L.logn, L.lognh);
        S.fetch(A, B, pl, tid);
        P.fetch(PA, PB, pl, tid);
    };
    auto store = [&](int slot) {
        S.store(sA[slot] + 1, sB[slot] + 1, tid);
        P.store(pA[slot] + 1, pB[slot] + 1, tid);
    };
    float dn[2], fn[2];
    auto fetch_cells = [&](int k) {
        const size_t pl = plane_off<float>(k, L.logn, L.lognh);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            dn[h] = ld_once(D, pl, coff[h]);
            fn[h] = ld_once(F, pl, coff[h]);
        }
    };
    fetch(k0 - 1);
    store(0);
    fetch(k0);
    store(1);
    fetch(k0 + 1);
    fetch_cells(k0);
    for (int k = k0; k < k0 + G.kz; ++k) {
        const int sm = (k - k0) % 3, s0 = (k - k0 + 1) % 3, sp = (k - k0 + 2) % 3;
        store(sp);
        const float d0 = dn[0], d1 = dn[1], f0 = fn[0], f1 = fn[1];
        __syncthreads();
        if (k + 2 <= k0 + G.kz) fetch(k + 2);
        if (k + 1 < k0 + G.kz) fetch_cells(k + 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = ty + 4 * h, j = j0 + row;
            const int p = (j + k + c) & 1;
            const NbT<float> s = lds_nb<float, float>(sA[sm] + 1, sA[s0] + 1, sA[sp] + 1, sB[s0] + 1,
                                                      sB[sm] + 1, sB[sp] + 1, row + 1, tx + 1, p);
            const NbT<float> a = lds_nb<float, float>(pA[sm] + 1, pA[s0] + 1, pA[sp] + 1, pB[s0] + 1,
                                                      pB[sm] + 1, pB[sp] + 1, row + 1, tx + 1, p);
            const float faces = (s.xp + s.xm) + (s.yp + s.ym) + (s.zp + s.zm);
            const float dK = corr_term<MODEL, float>(M, L, a, s, h ? d1 : d0);
            const float nv = (faces - h2 * (dK + (h ? f1 : f0) + fs)) * (1.0f / 6.0f);
            __builtin_nontemporal_store(nv, ptr(out, plane_off<float>(k, L.logn, L.lognh), coff[h]));
        }
        __syncthreads();
    }
}

// Inner residual d = A(e) - g - mu' at every cell of the tile (FP32
// arithmetic) and its restriction in FP64 into the first FP64 coarse level:
// R(pb + e) (the coarse initial guess of the whole field) and R d.  Block
// sums of d and d^2 (mu' and the inner norm).  Thread = coarse cell, as in
// k_resid_restrict_tiled.
template <int MODEL>
__global__ __launch_bounds__(TPB) void k_corr_resid_restrict_tiled(
    Mod M, LvlT<float> L, const float *pb0, const float *pb1, const double *fptr, double *ru0,
    double *ru1, double *rd0, double *rd1, double *partials, TileGeom G) {
    __shared__ __align__(16) float s0[3][TSLOT], s1[3][TSLOT], q0[3][TSLOT], q1[3][TSLOT];
    const size_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int bx = (int)(blk % G.ntx);
    const int by = (int)((blk / G.ntx) % G.nty);
    const int bz = (int)(blk / ((size_t)G.ntx * G.nty));
    const int m0 = bx * TX, j0 = by * TY, k0 = 2 * bz * G.kz, k1 = k0 + 2 * G.kz;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int lnc = L.logn - 1;
    unsigned coff[2];
    Stage2<float> S, P;
    S.init(tid, j0, m0, L.logn, L.lognh);
    P.init(tid, j0, m0, L.logn, L.lognh);
#pragma unroll
    for (int b = 0; b < 2; ++b) coff[b] = cell_off<float>(j0 + 2 * ty + b, m0 + tx, L.lognh);
    auto fetch = [&](int k) {
        const size_t pl = plane_off<float>(k, L.logn, L.lognh);
        S.fetch(L.u0, L.u1, pl, tid);
        P.fetch(pb0, pb1, pl, tid);
    };
    auto store = [&](int slot) {
        S.store(s0[slot] + 1, s1[slot] + 1, tid);
        P.store(q0[slot] + 1, q1[slot] + 1, tid);
    };
    float dn[4], fn[4];
    auto fetch_cells = [&](int k) {
        const size_t pl = plane_off<float>(k, L.logn, L.lognh);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            dn[2 * b] = ld_once(L.d0, pl, coff[b]);
            dn[2 * b + 1] = ld_once(L.d1, pl, coff[b]);
            fn[2 * b] = ld_once(L.f0, pl, coff[b]);
            fn[2 * b + 1] = ld_once(L.f1, pl, coff[b]);
        }
    };
    fetch(k0 - 1);
    store(0);
    fetch(k0);
    store(1);
    fetch(k0 + 1);
    fetch_cells(k0);
    double su = 0.0, sd = 0.0, acc1 = 0.0, acc2 = 0.0;
    const float fs = fptr ? (float)(*fptr) : 0.f;
    const float inv_h2 = (float)(1.0 / L.h2);
    for (int k = k0; k < k1; ++k) {
        const int sm = (k - k0) % 3, sz = (k - k0 + 1) % 3, sp = (k - k0 + 2) % 3;
        store(sp);
        float dc[4], fc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dc[q] = dn[q];
            fc[q] = fn[q];
        }
        __syncthreads();
        if (k + 2 <= k1) fetch(k + 2);
        if (k + 1 < k1) fetch_cells(k + 1);
#pragma unroll 1
        for (int b = 0; b < 2; ++b) {
#pragma unroll 1
            for (int c = 0; c < 2; ++c) {
                const int row = 2 * ty + b;
                const int p = (j0 + row + k + c) & 1;
                const float *Am = (c ? s1[sm] : s0[sm]) + 1, *A0 = (c ? s1[sz] : s0[sz]) + 1;
                const float *Ap = (c ? s1[sp] : s0[sp]) + 1, *Bm = (c ? s0[sm] : s1[sm]) + 1;
                const float *B0 = (c ? s0[sz] : s1[sz]) + 1, *Bp = (c ? s0[sp] : s1[sp]) + 1;
                const float *Qm = (c ? q1[sm] : q0[sm]) + 1, *Q0 = (c ? q1[sz] : q0[sz]) + 1;
                const float *Qp = (c ? q1[sp] : q0[sp]) + 1, *Rm = (c ? q0[sm] : q1[sm]) + 1;
                const float *R0 = (c ? q0[sz] : q1[sz]) + 1, *Rp = (c ? q0[sp] : q1[sp]) + 1;
                const int r = row + 1, q = tx + 1;
                const NbT<float> s = lds_nb<float, float>(Am, A0, Ap, B0, Bm, Bp, r, q, p);
                const NbT<float> a = lds_nb<float, float>(Qm, Q0, Qp, R0, Rm, Rp, r, q, p);
                const float e = A0[r * TXH + q];
                const float faces = (s.xp + s.xm) + (s.yp + s.ym) + (s.zp + s.zm);
                const float d = (faces - 6.0f * e) * inv_h2
                              - corr_term<MODEL, float>(M, L, a, s, dc[2 * b + c])
                              - fc[2 * b + c] - fs;
                sd += (double)d;
                su += (double)Q0[r * TXH + q] + (double)e;
                acc1 += (double)d;
                acc2 += (double)d * (double)d;
            }
        }
        if (k & 1) {
            const int K = k >> 1, I = m0 + tx, J = (j0 >> 1) + ty;
            const size_t cidx = ((size_t)K << (2 * lnc - 1)) + ((size_t)J << (lnc - 1)) + (I >> 1);
            const int ccol = (I + J + K) & 1;
            (ccol ? ru1 : ru0)[cidx] = 0.125 * su;
            (ccol ? rd1 : rd0)[cidx] = 0.125 * sd;
            su = 0.0;
            sd = 0.0;
        }
        __syncthreads();
    }
    block_sum2(acc1, acc2, partials, blk);
}

// phi64 += e, the background pb = fl32(phi64) and e = 0 (one colour's
// packed half-array of n values).
__global__ __launch_bounds__(TPB) void k_dc_accumulate(double *__restrict__ phi,
                                                       float *__restrict__ e,
                                                       float *__restrict__ pb, size_t n) {
    const size_t t = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (t >= n) return;
    const double v = phi[t] + (double)e[t];
    phi[t] = v;
    pb[t] = (float)v;
    e[t] = 0.f;
}

__global__ __launch_bounds__(TPB) void k_zero_f32(float *a, size_t n) {
    const size_t t = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (t < n) a[t] = 0.f;
}

}  // namespace mgk
