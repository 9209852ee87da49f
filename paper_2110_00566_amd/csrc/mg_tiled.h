// LDS-tiled versions of the three kernels that touch every finest-level cell
// (colour pass, residual + restriction, prolongation), for levels with at
// least 128 cells per side.
//
// A block owns a tile of TX = 64 packed x-columns (one wave wide) and TY = 8
// rows and marches through a z-chunk.  The planes it needs are staged once in
// LDS (tile plus a one-cell halo, periodic wrap) in a small ring, and the next
// plane is prefetched into registers while the current one is computed, so
// each global value is read about once per block instead of once per
// neighbouring thread.  Consecutive logical blocks are neighbours in y; the XCD
// remapping keeps a whole z-slab on one XCD so y-halos are L2 hits.
#pragma once
#include "mg_kernels.h"

namespace mgk {

constexpr int TX = 64, TY = 8, TXH = TX + 2, TYH = TY + 2;
constexpr int TPLANE = TXH * TYH;   // 660 values per staged plane
constexpr int TLOADS = (TPLANE + TPB - 1) / TPB;

struct TileGeom {
    int ntx, nty, kz;   // tiles in x, tiles in y, planes per block
};

// Byte offsets for the marching kernels: a thread's positions inside a z-plane
// are fixed for the whole march, so their offsets are computed once (32 bit)
// and each plane adds one uniform (scalar) base.
template <typename R>
__device__ __forceinline__ unsigned stage_off(int e, int j0, int m0, int logn, int lognh) {
    const int r = e / TXH, q = e - r * TXH;
    const unsigned j = (unsigned)(j0 - 1 + r) & ((1u << logn) - 1);
    const unsigned m = (unsigned)(m0 - 1 + q) & ((1u << lognh) - 1);
    return ((j << lognh) + m) * (unsigned)sizeof(R);
}
template <typename R>
__device__ __forceinline__ unsigned cell_off(int j, int m, int lognh) {
    return (((unsigned)j << lognh) + (unsigned)m) * (unsigned)sizeof(R);
}
template <typename R>
__device__ __forceinline__ size_t plane_off(int k, int logn, int lognh) {
    return ((size_t)((unsigned)k & ((1u << logn) - 1)) << (logn + lognh)) * sizeof(R);
}
template <typename R>
__device__ __forceinline__ R ld(const R *base, size_t plane, unsigned off) {
    return *reinterpret_cast<const R *>(reinterpret_cast<const char *>(base) + plane + off);
}
// A cell's own delta and f are read once per launch: non-temporal loads
// keep them from displacing the staged planes' halo rows in the caches.
template <typename R>
__device__ __forceinline__ R ld_once(const R *base, size_t plane, unsigned off) {
    return __builtin_nontemporal_load(
        reinterpret_cast<const R *>(reinterpret_cast<const char *>(base) + plane + off));
}
template <typename R>
__device__ __forceinline__ R *ptr(R *base, size_t plane, unsigned off) {
    return reinterpret_cast<R *>(reinterpret_cast<char *>(base) + plane + off);
}

// Staging of one z-plane (tile plus halo: TYH rows of TXH values) of two
// arrays of a level into LDS.  A staged plane starts one value into its LDS
// slot of TSLOT values.  FP64: each row's 64 interior values are read as 32
// 16-byte vectors (rows start on 512-byte boundaries of the level's arrays)
// and land on 16-byte LDS addresses (slot base + 8 + 528 r + 16 i); the two
// halo columns are single values.  320 vectors + 20 halo values: every thread
// takes one vector, then threads 0..63 one more and threads 64..83 a halo
// value.  FP32: one value per load.
constexpr int TSLOT = TPLANE + 2;

template <typename R>
struct Stage2 {
    unsigned soff[TLOADS];
    R ra[TLOADS], rb[TLOADS];
    __device__ __forceinline__ void init(int tid, int j0, int m0, int logn, int lognh) {
#pragma unroll
        for (int q = 0; q < TLOADS; ++q) soff[q] = stage_off<R>(tid + q * TPB, j0, m0, logn, lognh);
    }
    __device__ __forceinline__ void fetch(const R *A, const R *B, size_t pl, int tid) {
#pragma unroll
        for (int q = 0; q < TLOADS; ++q) {
            if (tid + q * TPB < TPLANE) {
                ra[q] = ld(A, pl, soff[q]);
                rb[q] = ld(B, pl, soff[q]);
            }
        }
    }
    // sa, sb: the slots' plane views (slot base + 1)
    __device__ __forceinline__ void store(R *sa, R *sb, int tid) const {
#pragma unroll
        for (int q = 0; q < TLOADS; ++q) {
            const int e = tid + q * TPB;
            if (e < TPLANE) {
                sa[e] = ra[q];
                sb[e] = rb[q];
            }
        }
    }
};

// FP32: 16 vectors of 4 values per row (160 per plane) and 20 halo values,
// one per thread; a vector lands in LDS as two 8-byte halves (a staged row
// starts 8 bytes off a 16-byte boundary in every other slot and row).
template <>
struct Stage2<float> {
    static constexpr int NV = TYH * (TX / 4);   // 160 vectors per plane
    static_assert(NV + 2 * TYH <= TPB, "staging split");
    unsigned g;   // byte offset inside a plane
    int l;        // value offset inside a plane view
    float4 a, b;
    __device__ __forceinline__ void init(int tid, int j0, int m0, int logn, int lognh) {
        const unsigned jm = (1u << logn) - 1, mm = (1u << lognh) - 1;
        if (tid < NV) {
            const int r = tid >> 4, i = tid & 15;
            g = ((((unsigned)(j0 - 1 + r) & jm) << lognh) + (unsigned)(m0 + 4 * i)) * 4u;
            l = r * TXH + 1 + 4 * i;
        } else {
            const int h = tid < NV + 2 * TYH ? tid - NV : 0, r = h >> 1, side = h & 1;
            const unsigned m = (unsigned)(side ? m0 + TX : m0 - 1) & mm;
            g = ((((unsigned)(j0 - 1 + r) & jm) << lognh) + m) * 4u;
            l = r * TXH + (side ? TXH - 1 : 0);
        }
    }
    __device__ __forceinline__ void fetch(const float *A, const float *B, size_t pl, int tid) {
        const char *pa = reinterpret_cast<const char *>(A) + pl + g;
        const char *pb = reinterpret_cast<const char *>(B) + pl + g;
        if (tid < NV) {
            a = *reinterpret_cast<const float4 *>(pa);
            b = *reinterpret_cast<const float4 *>(pb);
        } else if (tid < NV + 2 * TYH) {
            a.x = *reinterpret_cast<const float *>(pa);
            b.x = *reinterpret_cast<const float *>(pb);
        }
    }
    __device__ __forceinline__ void store(float *sa, float *sb, int tid) const {
        if (tid < NV) {
            *reinterpret_cast<float2 *>(sa + l) = make_float2(a.x, a.y);
            *reinterpret_cast<float2 *>(sa + l + 2) = make_float2(a.z, a.w);
            *reinterpret_cast<float2 *>(sb + l) = make_float2(b.x, b.y);
            *reinterpret_cast<float2 *>(sb + l + 2) = make_float2(b.z, b.w);
        } else if (tid < NV + 2 * TYH) {
            sa[l] = a.x;
            sb[l] = b.x;
        }
    }
};

template <>
struct Stage2<double> {
    static constexpr int NV = TYH * (TX / 2);   // 320 vectors per plane
    static_assert(TPB == 256 && NV - TPB == 64 && 2 * TYH <= TPB - 64, "staging split");
    unsigned g0, g1;   // byte offsets inside a plane
    int l0, l1;        // value offsets inside a plane view
    double2 a0, a1, b0, b1;
    double ha, hb;
    __device__ __forceinline__ void init(int tid, int j0, int m0, int logn, int lognh) {
        const unsigned jm = (1u << logn) - 1, mm = (1u << lognh) - 1;
        {
            const int r = tid >> 5, i = tid & 31;
            g0 = ((((unsigned)(j0 - 1 + r) & jm) << lognh) + (unsigned)(m0 + 2 * i)) * 8u;
            l0 = r * TXH + 1 + 2 * i;
        }
        if (tid < 64) {
            const int r = 8 + (tid >> 5), i = tid & 31;
            g1 = ((((unsigned)(j0 - 1 + r) & jm) << lognh) + (unsigned)(m0 + 2 * i)) * 8u;
            l1 = r * TXH + 1 + 2 * i;
        } else {
            const int h = tid < 64 + 2 * TYH ? tid - 64 : 0, r = h >> 1, side = h & 1;
            const unsigned m = (unsigned)(side ? m0 + TX : m0 - 1) & mm;
            g1 = ((((unsigned)(j0 - 1 + r) & jm) << lognh) + m) * 8u;
            l1 = r * TXH + (side ? TXH - 1 : 0);
        }
    }
    __device__ __forceinline__ void fetch(const double *A, const double *B, size_t pl, int tid) {
        const char *a = reinterpret_cast<const char *>(A) + pl;
        const char *b = reinterpret_cast<const char *>(B) + pl;
        a0 = *reinterpret_cast<const double2 *>(a + g0);
        b0 = *reinterpret_cast<const double2 *>(b + g0);
        if (tid < 64) {
            a1 = *reinterpret_cast<const double2 *>(a + g1);
            b1 = *reinterpret_cast<const double2 *>(b + g1);
        } else if (tid < 64 + 2 * TYH) {
            ha = *reinterpret_cast<const double *>(a + g1);
            hb = *reinterpret_cast<const double *>(b + g1);
        }
    }
    __device__ __forceinline__ void store(double *sa, double *sb, int tid) const {
        *reinterpret_cast<double2 *>(sa + l0) = a0;
        *reinterpret_cast<double2 *>(sb + l0) = b0;
        if (tid < 64) {
            *reinterpret_cast<double2 *>(sa + l1) = a1;
            *reinterpret_cast<double2 *>(sb + l1) = b1;
        } else if (tid < 64 + 2 * TYH) {
            sa[l1] = ha;
            sb[l1] = hb;
        }
    }
};

// Stencil of the cell at local (r, q) (halo-shifted tile coordinates) with
// packed-x parity p, from staged planes: B = opposite colour at plane k,
// A = own colour at k-1 / k / k+1, Bz = opposite colour at k-1 / k+1.
template <typename T, typename R>
__device__ __forceinline__ NbT<T> lds_nb(const R *Am, const R *A0, const R *Ap, const R *B0,
                                         const R *Bm, const R *Bp, int r, int q, int p) {
    const int qp = q + p, qm = q + p - 1;
    const int o = r * TXH, op = (r + 1) * TXH, om = (r - 1) * TXH;
    NbT<T> s;
    s.xp = (T)B0[o + qp];
    s.xm = (T)B0[o + qm];
    s.yp = (T)B0[op + q];
    s.ym = (T)B0[om + q];
    s.zp = (T)Bp[o + q];
    s.zm = (T)Bm[o + q];
    s.nxy = ((T)A0[op + qp] + (T)A0[om + qm]) - ((T)A0[om + qp] + (T)A0[op + qm]);
    s.nxz = ((T)Ap[o + qp] + (T)Am[o + qm]) - ((T)Am[o + qp] + (T)Ap[o + qm]);
    s.nyz = ((T)Ap[op + q] + (T)Am[om + q]) - ((T)Am[op + q] + (T)Ap[om + q]);
    return s;
}

// Non-Laplacian term of the tiled kernels at a cell with face sum faces and
// centre value u.  OP_NEWTON (the Newton-GS comparator) works on the
// quadratic form: Sigma/alpha - 2 D^2/(3 alpha), D = (faces - 6u)/h^2.
template <int OP, typename T, typename L_>
__device__ __forceinline__ T tiled_term(const Mod &M, const L_ &L, const NbT<T> &s, T delta,
                                        T faces, T u, unsigned long long *clamp) {
    if constexpr (OP == OP_NEWTON)
        return newton_term<T>(M, dgp_sigma_over_alpha<T>(M, L, s, delta),
                              (faces - (T)6 * u) / (T)L.h2);
    else
        return model_term<OP, T>(M, L, s, delta, clamp);
}

// New value of a cell in a colour pass: the closed-form update, or for
// OP_NEWTON the Newton-Gauss-Seidel step on the quadratic form.
template <int OP, typename R, typename L_>
__device__ __forceinline__ R tiled_update(const Mod &M, const L_ &L, const NbT<R> &s, R delta,
                                          R faces, R u, R f, unsigned long long *clamp) {
    if constexpr (OP == OP_NEWTON) {
        return newton_update<R>(M, u, faces, dgp_sigma_over_alpha<R>(M, L, s, delta), f,
                                (R)L.h2);
    } else {
        const R K = model_term<OP, R>(M, L, s, delta, clamp);
        return (faces - (R)L.h2 * (K + f)) * (R)(1.0 / 6.0);
    }
}

// One colour pass (see k_pass) on an LDS-staged tile.
template <int OP, typename R>
__global__ __launch_bounds__(TPB) void k_pass_tiled(Mod M, LvlT<R> L, int c, R *__restrict__ out,
                                                    const double *fptr, double fscale,
                                                    unsigned long long *clamp, TileGeom G) {
    __shared__ __align__(16) R sA[3][TSLOT], sB[3][TSLOT];
    const size_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int bx = (int)(blk % G.ntx);
    const int by = (int)((blk / G.ntx) % G.nty);
    const int bz = (int)(blk / ((size_t)G.ntx * G.nty));
    const int m0 = bx * TX, j0 = by * TY, k0 = bz * G.kz;
    const R *A = c ? L.u1 : L.u0;
    const R *B = c ? L.u0 : L.u1;
    const R *D = c ? L.d1 : L.d0;
    const R *F = c ? L.f1 : L.f0;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const R fs = (R)(fptr ? fscale * (*fptr) : 0.0);
    unsigned coff[2];
    Stage2<R> S;
    S.init(tid, j0, m0, L.logn, L.lognh);
#pragma unroll
    for (int h = 0; h < 2; ++h) coff[h] = cell_off<R>(j0 + ty + 4 * h, m0 + tx, L.lognh);
    auto fetch = [&](int k) { S.fetch(A, B, plane_off<R>(k, L.logn, L.lognh), tid); };
    auto store = [&](int slot) { S.store(sA[slot] + 1, sB[slot] + 1, tid); };
    // own cells' delta and f, one plane ahead
    R dn[2], fn[2];
    auto fetch_cells = [&](int k) {
        const size_t pl = plane_off<R>(k, L.logn, L.lognh);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            dn[h] = ld_once(D, pl, coff[h]);
            fn[h] = F ? ld_once(F, pl, coff[h]) : (R)0;
        }
    };
    // slot of plane k: (k - k0 + 1) mod 3
    fetch(k0 - 1);
    store(0);
    fetch(k0);
    store(1);
    fetch(k0 + 1);
    fetch_cells(k0);
    for (int k = k0; k < k0 + G.kz; ++k) {
        const int sm = (k - k0) % 3, s0 = (k - k0 + 1) % 3, sp = (k - k0 + 2) % 3;
        store(sp);
        const R d0 = dn[0], d1 = dn[1], f0 = fn[0], f1 = fn[1];
        __syncthreads();
        if (k + 2 <= k0 + G.kz) fetch(k + 2);
        if (k + 1 < k0 + G.kz) fetch_cells(k + 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = ty + 4 * h;
            const int j = j0 + row;
            const int p = (j + k + c) & 1;
            const NbT<R> s = lds_nb<R, R>(sA[sm] + 1, sA[s0] + 1, sA[sp] + 1, sB[s0] + 1,
                                          sB[sm] + 1, sB[sp] + 1, row + 1, tx + 1, p);
            const R faces = (s.xp + s.xm) + (s.yp + s.ym) + (s.zp + s.zm);
            const R f = (h ? f1 : f0) + fs;
            const R nv = tiled_update<OP, R>(M, L, s, h ? d1 : d0, faces,
                                             sA[s0][1 + (row + 1) * TXH + tx + 1], f, clamp);
            // streamed: the next reader is a later launch
            __builtin_nontemporal_store(nv, ptr(out, plane_off<R>(k, L.logn, L.lognh), coff[h]));
        }
        __syncthreads();
    }
}

// Residual + restriction (see k_resid_restrict) for a tile of 64 x 4 coarse
// cells.  The block marches over the fine planes of its coarse z-chunk with a
// ring of 3 staged planes of both colours, like the pass; a thread owns one
// coarse cell and computes its 4 children in each fine plane (rows 2ty,
// 2ty+1, both colours), summing over the two fine planes of the coarse
// plane.  kz counts coarse planes.  HASF: the level has a right-hand side f
// (every level but the finest).
// WG: also store g = -d of every fine cell in FP32 (g0/g1, the packed
// colours; the outer step of the defect-correction solve).
template <int OP, bool REDUCE, bool HASF, typename R, bool WG = false>
__global__ __launch_bounds__(TPB) void k_resid_restrict_tiled(Mod M, LvlT<R> L, const double *fptr,
                                                              double fscale, R *ru0, R *ru1,
                                                              R *rd0, R *rd1, double *partials,
                                                              unsigned long long *clamp,
                                                              TileGeom G, float *g0 = nullptr,
                                                              float *g1 = nullptr) {
    __shared__ __align__(16) R s0[3][TSLOT], s1[3][TSLOT];
    const size_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int bx = (int)(blk % G.ntx);
    const int by = (int)((blk / G.ntx) % G.nty);
    const int bz = (int)(blk / ((size_t)G.ntx * G.nty));
    // fine tile: packed columns m0.., fine rows j0 .. j0+7 (coarse rows j0/2 ..)
    const int m0 = bx * TX, j0 = by * TY, k0 = 2 * bz * G.kz, k1 = k0 + 2 * G.kz;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int lnc = L.logn - 1;
    unsigned coff[2];
    Stage2<R> S;
    S.init(tid, j0, m0, L.logn, L.lognh);
#pragma unroll
    for (int b = 0; b < 2; ++b) coff[b] = cell_off<R>(j0 + 2 * ty + b, m0 + tx, L.lognh);
    auto fetch = [&](int k) { S.fetch(L.u0, L.u1, plane_off<R>(k, L.logn, L.lognh), tid); };
    auto store = [&](int slot) { S.store(s0[slot] + 1, s1[slot] + 1, tid); };
    // delta (and f) of the 4 children in a fine plane, one plane ahead
    R dn[4], fn[4];
    auto fetch_cells = [&](int k) {
        const size_t pl = plane_off<R>(k, L.logn, L.lognh);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            dn[2 * b] = ld_once(L.d0, pl, coff[b]);
            dn[2 * b + 1] = ld_once(L.d1, pl, coff[b]);
            if (HASF) {
                fn[2 * b] = ld_once(L.f0, pl, coff[b]);
                fn[2 * b + 1] = ld_once(L.f1, pl, coff[b]);
            }
        }
    };
    // slot of fine plane k: (k - k0 + 1) mod 3
    fetch(k0 - 1);
    store(0);
    fetch(k0);
    store(1);
    fetch(k0 + 1);
    fetch_cells(k0);
    double su = 0.0, sd = 0.0, acc1 = 0.0, acc2 = 0.0;
    const double fs = fptr ? fscale * (*fptr) : 0.0;
    const double inv_h2 = 1.0 / L.h2;
    for (int k = k0; k < k1; ++k) {
        const int sm = (k - k0) % 3, sz = (k - k0 + 1) % 3, sp = (k - k0 + 2) % 3;
        store(sp);
        R dc[4], fc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dc[q] = dn[q];
            fc[q] = HASF ? fn[q] : R(0);
        }
        __syncthreads();
        if (k + 2 <= k1) fetch(k + 2);
        if (k + 1 < k1) fetch_cells(k + 1);
        // dv, fv: delta and f of child (b, c), passed by value so that the
        // rolled loop indexes no local array (that would put dc, fc in scratch)
        auto child = [&](int b, int c, R dv, R fv) {
            const int row = 2 * ty + b;
            const int p = (j0 + row + k + c) & 1;
            const R *Am = (c ? s1[sm] : s0[sm]) + 1;
            const R *A0 = (c ? s1[sz] : s0[sz]) + 1;
            const R *Ap = (c ? s1[sp] : s0[sp]) + 1;
            const R *Bm = (c ? s0[sm] : s1[sm]) + 1;
            const R *B0 = (c ? s0[sz] : s1[sz]) + 1;
            const R *Bp = (c ? s0[sp] : s1[sp]) + 1;
            const int r = row + 1, q = tx + 1;
            const double u = (double)A0[r * TXH + q];
            const double f = (HASF ? (double)fv : 0.0) + fs;
            double d;
            if constexpr (sizeof(R) == 4 && (OP == OP_DGP || OP == OP_KMO)) {
                // FP32 storage: the Laplacian in double, the model term in
                // float (nDGP) or from float stencil combinations (Kmouflage)
                const NbT<float> s = lds_nb<float, R>(Am, A0, Ap, B0, Bm, Bp, r, q, p);
                const double faces = ((double)s.xp + (double)s.xm) +
                                     ((double)s.yp + (double)s.ym) +
                                     ((double)s.zp + (double)s.zm);
                d = (faces - 6.0 * u) * inv_h2 -
                    (double)model_term<OP, float>(M, L, s, (float)dv, clamp) - f;
            } else {
                const Nb s = lds_nb<double, R>(Am, A0, Ap, B0, Bm, Bp, r, q, p);
                const double faces = (s.xp + s.xm) + (s.yp + s.ym) + (s.zp + s.zm);
                d = (faces - 6.0 * u) * inv_h2 -
                    tiled_term<OP, double>(M, L, s, (double)dv, faces, u, clamp) - f;
            }
            sd += d;
            su += u;
            if (REDUCE) {
                acc1 += d;
                acc2 += d * d;
            }
            if (WG)
                *ptr(c ? g1 : g0, plane_off<float>(k, L.logn, L.lognh),
                     cell_off<float>(j0 + row, m0 + tx, L.lognh)) = (float)(-d);
        };
        if constexpr (sizeof(R) == 4 && OP == OP_DGP) {
            // FP32 nDGP (70 registers rolled, 96 unrolled, 3% faster): the
            // four children unrolled
            child(0, 0, dc[0], fc[0]);
            child(0, 1, dc[1], fc[1]);
            child(1, 0, dc[2], fc[2]);
            child(1, 1, dc[3], fc[3]);
        } else {
            // the four children stay rolled (unrolled, the Kmouflage term
            // needs 200+ registers per lane; rolled the FP64 kernel is 4%
            // faster)
#pragma unroll 1
            for (int q = 0; q < 4; ++q) {
                const R dv = q == 0 ? dc[0] : q == 1 ? dc[1] : q == 2 ? dc[2] : dc[3];
                const R fv = q == 0 ? fc[0] : q == 1 ? fc[1] : q == 2 ? fc[2] : fc[3];
                child(q >> 1, q & 1, dv, fv);
            }
        }
        if (k & 1) {
            const int K = k >> 1, I = m0 + tx, J = (j0 >> 1) + ty;
            const size_t cidx = ((size_t)K << (2 * lnc - 1)) + ((size_t)J << (lnc - 1)) + (I >> 1);
            const int ccol = (I + J + K) & 1;
            (ccol ? ru1 : ru0)[cidx] = (R)(0.125 * su);
            (ccol ? rd1 : rd0)[cidx] = (R)(0.125 * sd);
            su = 0.0;
            sd = 0.0;
        }
        __syncthreads();
    }
    if (REDUCE) block_sum2(acc1, acc2, partials, blk);
}

// u_fine += P(uc - rc) (see k_prolong) with the coarse difference staged in
// LDS: 66 coarse columns x 6 coarse rows, ring of 3 coarse planes.  REDUCE:
// block sums of the corrected colour-0 and colour-1 values into partials.
// RC: storage type of the coarse level (the defect-correction cycles
// prolong an FP64 coarse correction into an FP32 finest level).
template <typename R, bool REDUCE = false, typename RC = R>
__global__ __launch_bounds__(TPB) void k_prolong_tiled(R *f0, R *f1, int logn, const RC *uc0,
                                                       const RC *uc1, const RC *rc0, const RC *rc1,
                                                       TileGeom G, double *partials = nullptr) {
    constexpr int CR = TY / 2 + 2;   // coarse rows staged
    constexpr int CPL = TXH * CR;    // 396 values per coarse plane
    __shared__ double sE[3][CPL];
    const size_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int bx = (int)(blk % G.ntx);
    const int by = (int)((blk / G.ntx) % G.nty);
    const int bz = (int)(blk / ((size_t)G.ntx * G.nty));
    const int m0 = bx * TX, j0 = by * TY, K0 = bz * G.kz;   // kz counts coarse planes
    const int lnc = logn - 1, ncm1 = (1 << lnc) - 1;
    const int lognh = logn - 1;
    const int tid = threadIdx.x;
    double re[2];
    auto fetch = [&](int K) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + q * TPB;
            if (e < CPL) {
                const int r = e / TXH, cI = e - r * TXH;
                const int I = (m0 - 1 + cI) & ncm1;
                const int J = ((j0 >> 1) - 1 + r) & ncm1;
                const int Kw = K & ncm1;
                const size_t idx = ((size_t)Kw << (2 * lnc - 1)) + ((size_t)J << (lnc - 1)) + (I >> 1);
                re[q] = ((I + J + Kw) & 1) ? ((double)uc1[idx] - (double)rc1[idx])
                                           : ((double)uc0[idx] - (double)rc0[idx]);
            }
        }
    };
    auto store = [&](int slot) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + q * TPB;
            if (e < CPL) sE[slot][e] = re[q];
        }
    };
    // slot of coarse plane K: (K - K0 + 1) mod 3
    fetch(K0 - 1);
    store(0);
    fetch(K0);
    store(1);
    fetch(K0 + 1);
    double bsum[2] = {0.0, 0.0};
    for (int K = K0; K < K0 + G.kz; ++K) {
        store((K - K0 + 2) % 3);
        __syncthreads();
        if (K + 2 <= K0 + G.kz) fetch(K + 2);
        // 2 fine planes x 8 rows x 64 columns x 2 colours = 2048 cells, 8 per thread
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int cell = tid + h * TPB;
            const int tx = cell & 63, row = (cell >> 6) & 7, c = (cell >> 9) & 1, kk = cell >> 10;
            const int k = 2 * K + kk, j = j0 + row, m = m0 + tx;
            const int p = (j + k + c) & 1;
            const int di = p ? 1 : -1, dj = (j & 1) ? 1 : -1, dk = kk ? 1 : -1;
            const int lc = tx + 1, lr = (j >> 1) - (j0 >> 1) + 1;
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int a = q & 1, b = (q >> 1) & 1, cc = q >> 2;
                const int slot = (K + cc * dk - K0 + 1 + 3) % 3;
                const double w = (a ? 1.0 : 3.0) * (b ? 1.0 : 3.0) * (cc ? 1.0 : 3.0);
                acc += w * sE[slot][(lr + b * dj) * TXH + lc + a * di];
            }
            const size_t idx = prow(j, k, logn, lognh) + m;
            R *f = c ? f1 : f0;
            const R nv = (R)((double)f[idx] + acc * (1.0 / 64.0));
            f[idx] = nv;
            if (REDUCE) bsum[c] += (double)nv;
        }
        __syncthreads();
    }
    if (REDUCE) block_sum2(bsum[0], bsum[1], partials, blk);
}

// Prolongation of the coarse correction fused with the first post-smoothing
// pass (colour 0).  Every staged fine value is corrected on the fly,
// u + P(uc - rc), colour-0 cells get the closed-form update from the corrected
// neighbourhood (out0) and colour-1 cells are written corrected (out1).  Both
// outputs are separate arrays: neighbouring tiles still read the old values.
//
// The 27/9/3/1 weights factor into a z part (3/4 own coarse plane, 1/4 the
// plane on the fine cell's side) times an x-y bilinear part (9, 3, 3, 1 over
// 16).  A thread keeps the x-y part of the two coarse planes the next staged
// fine planes need, at its staged positions and for both x parities, in
// registers; one coarse plane of 68 x 6 values around the tile passes through
// LDS every second fine plane.  kz (fine planes per block) is even.
// The Kmouflage instance is held to 3 waves per SIMD (167 registers, no
// spill; unconstrained it takes 171 and runs 2): its 512^3 solve is 4.5%
// faster.
template <int OP, typename R>
__global__ __launch_bounds__(TPB)
__attribute__((amdgpu_waves_per_eu(OP == OP_KMO ? 3 : 1))) void k_prolong_pass_tiled(Mod M, LvlT<R> L, R *__restrict__ out0,
                                                            R *__restrict__ out1, const R *uc0,
                                                            const R *uc1, const R *rc0,
                                                            const R *rc1, const double *fptr,
                                                            double fscale,
                                                            unsigned long long *clamp, TileGeom G) {
    constexpr int CW = TX + 4;           // coarse columns m0-2 .. m0+65
    constexpr int CH = TY / 2 + 2;       // coarse rows j0/2-1 .. j0/2+4
    constexpr int CPL = CW * CH;
    constexpr int CLOADS = (CPL + TPB - 1) / TPB;
    // arithmetic type of the coarse correction: that of the storage (in FP32
    // storage the correction, small beside phi, needs no FP64)
    using CT = R;
    __shared__ R sA[3][TPLANE], sB[3][TPLANE];
    __shared__ CT sC[CPL];
    const size_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int bx = (int)(blk % G.ntx);
    const int by = (int)((blk / G.ntx) % G.nty);
    const int bz = (int)(blk / ((size_t)G.ntx * G.nty));
    const int m0 = bx * TX, j0 = by * TY, k0 = bz * G.kz, K0 = k0 >> 1;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int lnc = L.logn - 1, ncm1 = (1 << lnc) - 1;
    const R fs = (R)(fptr ? fscale * (*fptr) : 0.0);

    // coarse difference uc - rc of one coarse plane, via registers into sC
    CT cu[CLOADS], cr[CLOADS];
    auto cfetch = [&](int Z) {
        const int Zw = Z & ncm1;
#pragma unroll
        for (int q = 0; q < CLOADS; ++q) {
            const int e = tid + q * TPB;
            if (e < CPL) {
                const int r = e / CW, cI = e - r * CW;
                const int X = (m0 - 2 + cI) & ncm1;
                const int Y = ((j0 >> 1) - 1 + r) & ncm1;
                const size_t idx =
                    ((size_t)Zw << (2 * lnc - 1)) + ((size_t)Y << (lnc - 1)) + (X >> 1);
                const bool odd = (X + Y + Zw) & 1;
                cu[q] = (odd ? uc1 : uc0)[idx];
                cr[q] = (odd ? rc1 : rc0)[idx];
            }
        }
    };
    auto cstore = [&]() {
#pragma unroll
        for (int q = 0; q < CLOADS; ++q) {
            const int e = tid + q * TPB;
            if (e < CPL) sC[e] = cu[q] - cr[q];
        }
    };
    // x-y bilinear part of the coarse plane in sC at the thread's staged
    // positions, for fine x = 2m (index 0, coarse neighbour m-1) and
    // x = 2m+1 (index 1, coarse neighbour m+1)
    CT xlo[TLOADS][2], xhi[TLOADS][2], xnx[TLOADS][2];
    auto interp = [&](CT (&x)[TLOADS][2]) {
#pragma unroll
        for (int q = 0; q < TLOADS; ++q) {
            const int e = tid + q * TPB;
            if (e < TPLANE) {
                const int r = e / TXH, cI = e - r * TXH;
                const int lr = (r + 1) >> 1, lc = cI + 1;
                const int ly = (r & 1) ? lr - 1 : lr + 1;   // fine row odd: coarse row above
                const CT c0 = sC[lr * CW + lc], cm = sC[lr * CW + lc - 1],
                         cp = sC[lr * CW + lc + 1];
                const CT d0 = sC[ly * CW + lc], dm = sC[ly * CW + lc - 1],
                         dp = sC[ly * CW + lc + 1];
                x[q][0] = (CT)(9.0 / 16.0) * c0 + (CT)(3.0 / 16.0) * cm +
                          (CT)(3.0 / 16.0) * d0 + (CT)(1.0 / 16.0) * dm;
                x[q][1] = (CT)(9.0 / 16.0) * c0 + (CT)(3.0 / 16.0) * cp +
                          (CT)(3.0 / 16.0) * d0 + (CT)(1.0 / 16.0) * dp;
            }
        }
    };

    // raw fine values of the next plane, and own cells' delta and f
    unsigned soff[TLOADS], coff[2];
#pragma unroll
    for (int q = 0; q < TLOADS; ++q) soff[q] = stage_off<R>(tid + q * TPB, j0, m0, L.logn, L.lognh);
#pragma unroll
    for (int h = 0; h < 2; ++h) coff[h] = cell_off<R>(j0 + ty + 4 * h, m0 + tx, L.lognh);
    R ra[TLOADS], rb[TLOADS];
    auto fetch = [&](int k) {
        const size_t pl = plane_off<R>(k, L.logn, L.lognh);
#pragma unroll
        for (int q = 0; q < TLOADS; ++q) {
            if (tid + q * TPB < TPLANE) {
                ra[q] = ld(L.u0, pl, soff[q]);
                rb[q] = ld(L.u1, pl, soff[q]);
            }
        }
    };
    // corrected plane k into ring slot; the coarse pair (lo, hi) holds the
    // plane's own coarse plane (hi for even k, lo for odd k) and its neighbour
    auto stage = [&](int slot, int k, bool kodd) {
        const CT wl = kodd ? (CT)0.75 : (CT)0.25, wh = kodd ? (CT)0.25 : (CT)0.75;
#pragma unroll
        for (int q = 0; q < TLOADS; ++q) {
            const int e = tid + q * TPB;
            if (e < TPLANE) {
                const int r = e / TXH;
                const bool p0 = (j0 - 1 + r + k) & 1;   // x parity of the colour-0 value
                const CT l0 = p0 ? xlo[q][1] : xlo[q][0], l1 = p0 ? xlo[q][0] : xlo[q][1];
                const CT h0 = p0 ? xhi[q][1] : xhi[q][0], h1 = p0 ? xhi[q][0] : xhi[q][1];
                sA[slot][e] = ra[q] + (wl * l0 + wh * h0);
                sB[slot][e] = rb[q] + (wl * l1 + wh * h1);
            }
        }
    };
    R dn[2], fn[2];
    auto fetch_cells = [&](int k) {
        const size_t pl = plane_off<R>(k, L.logn, L.lognh);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            dn[h] = ld_once(L.d0, pl, coff[h]);
            fn[h] = L.f0 ? ld_once(L.f0, pl, coff[h]) : (R)0;
        }
    };

    // coarse planes K0-1, K0 (pair for fine planes k0-1, k0) and K0+1
    cfetch(K0 - 1);
    cstore();
    __syncthreads();
    interp(xlo);
    __syncthreads();
    cfetch(K0);
    cstore();
    __syncthreads();
    interp(xhi);
    __syncthreads();
    cfetch(K0 + 1);
    cstore();
    __syncthreads();
    interp(xnx);
    // slot of fine plane k: (k - k0 + 1) mod 3
    fetch(k0 - 1);
    stage(0, k0 - 1, true);
    fetch(k0);
    stage(1, k0, false);
    fetch(k0 + 1);
    fetch_cells(k0);

    auto step = [&](int k, bool odd) {
        if (!odd) {
#pragma unroll
            for (int q = 0; q < TLOADS; ++q) {
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    xlo[q][b] = xhi[q][b];
                    xhi[q][b] = xnx[q][b];
                }
            }
        }
        const int sm = (k - k0) % 3, s0 = (k - k0 + 1) % 3, sp = (k - k0 + 2) % 3;
        stage(sp, k + 1, !odd);
        // a new coarse plane (k >> 1) + 2 is needed for fine planes beyond k + 2
        const bool cnew = odd && (k + 3 <= k0 + G.kz);
        if (cnew) cstore();
        const R d0 = dn[0], d1 = dn[1], f0 = fn[0], f1 = fn[1];
        __syncthreads();
        if (k + 2 <= k0 + G.kz) fetch(k + 2);
        if (k + 1 < k0 + G.kz) fetch_cells(k + 1);
        if (!odd && k + 4 <= k0 + G.kz) cfetch((k >> 1) + 2);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = ty + 4 * h;
            const int j = j0 + row;
            const int p = (j + k) & 1;
            const NbT<R> s = lds_nb<R, R>(sA[sm], sA[s0], sA[sp], sB[s0], sB[sm], sB[sp], row + 1,
                                          tx + 1, p);
            const size_t pl = plane_off<R>(k, L.logn, L.lognh);
            const R faces = (s.xp + s.xm) + (s.yp + s.ym) + (s.zp + s.zm);
            const R f = (h ? f1 : f0) + fs;
            const R nv = tiled_update<OP, R>(M, L, s, h ? d1 : d0, faces,
                                             sA[s0][(row + 1) * TXH + tx + 1], f, clamp);
            __builtin_nontemporal_store(nv, ptr(out0, pl, coff[h]));
            __builtin_nontemporal_store(sB[s0][(row + 1) * TXH + tx + 1], ptr(out1, pl, coff[h]));
        }
        if (cnew) interp(xnx);
        __syncthreads();
    };
    for (int k = k0; k < k0 + G.kz; k += 2) {
        step(k, false);
        step(k + 1, true);
    }
}

// FAS source on a coarse level (see k_coarse_source) on an LDS-staged tile:
// S = L(R u) - (R d - shift) at both colours, written over R d, and u = R u.
template <int OP, typename R>
__global__ __launch_bounds__(TPB) void k_coarse_source_tiled(Mod M, LvlT<R> Lc, R *s0, R *s1,
                                                             R *u0, R *u1, const double *shift,
                                                             TileGeom G) {
    __shared__ __align__(16) R sA[3][TSLOT], sB[3][TSLOT];   // colour 0 / colour 1 of R u
    const size_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int bx = (int)(blk % G.ntx);
    const int by = (int)((blk / G.ntx) % G.nty);
    const int bz = (int)(blk / ((size_t)G.ntx * G.nty));
    const int m0 = bx * TX, j0 = by * TY, k0 = bz * G.kz;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const double sh = shift ? *shift : 0.0;
    unsigned coff[2];
    Stage2<R> S2;
    S2.init(tid, j0, m0, Lc.logn, Lc.lognh);
#pragma unroll
    for (int h = 0; h < 2; ++h) coff[h] = cell_off<R>(j0 + ty + 4 * h, m0 + tx, Lc.lognh);
    auto fetch = [&](int k) { S2.fetch(Lc.u0, Lc.u1, plane_off<R>(k, Lc.logn, Lc.lognh), tid); };
    auto store = [&](int slot) { S2.store(sA[slot] + 1, sB[slot] + 1, tid); };
    fetch(k0 - 1);
    store(0);
    fetch(k0);
    store(1);
    fetch(k0 + 1);
    for (int k = k0; k < k0 + G.kz; ++k) {
        const int sm = (k - k0) % 3, sz = (k - k0 + 1) % 3, sp = (k - k0 + 2) % 3;
        store(sp);
        __syncthreads();
        if (k + 2 <= k0 + G.kz) fetch(k + 2);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int row = ty + 4 * (h & 1), c = h >> 1;
            const int j = j0 + row;
            const int p = (j + k + c) & 1;
            const R *Am = (c ? sB[sm] : sA[sm]) + 1;
            const R *A0 = (c ? sB[sz] : sA[sz]) + 1;
            const R *Ap = (c ? sB[sp] : sA[sp]) + 1;
            const R *Bm = (c ? sA[sm] : sB[sm]) + 1;
            const R *B0 = (c ? sA[sz] : sB[sz]) + 1;
            const R *Bp = (c ? sA[sp] : sB[sp]) + 1;
            const Nb s = lds_nb<double, R>(Am, A0, Ap, B0, Bm, Bp, row + 1, tx + 1, p);
            const size_t pl = plane_off<R>(k, Lc.logn, Lc.lognh);
            const unsigned o = coff[h & 1];
            const R ru = A0[(row + 1) * TXH + tx + 1];
            const double faces = (s.xp + s.xm) + (s.yp + s.ym) + (s.zp + s.zm);
            const double delta = (double)ld_once(c ? Lc.d1 : Lc.d0, pl, o);
            R *S = ptr(c ? s1 : s0, pl, o);
            const double rd = (double)ld_once(c ? s1 : s0, pl, o) - sh;
            *S = (R)((faces - 6.0 * (double)ru) / Lc.h2
                     - tiled_term<OP, double>(M, Lc, s, delta, faces, (double)ru, nullptr) - rd);
            *ptr(c ? u1 : u0, pl, o) = ru;
        }
        __syncthreads();
    }
}

}  // namespace mgk
