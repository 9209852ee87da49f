// LDS-tiled kernels of the adjoint solve (J^T mu = f by FAS-free linear
// multigrid with the Jacobian coefficients stored per level), for levels with
// at least 128 cells per side.
//
// (J^T mu)_p = lap(mu)_p - G_p with G_p = sum over the 18 neighbours q of p of
// dK_q/dphi_p mu_q (the diagonal of J^T is exactly -6/h^2: no model term
// depends on its own cell).  With the coefficient arrays of mg_adjoint.h:
//   faces (colour 1-c): cf0(p-x) mu(p-x) + cf1(p+x) mu(p+x) + same for y
//                       (cf2, cf3) and z (cf4, cf5),
//   edges (colour c):   cf6 over the xy corners with signs (+ + at p-x-y and
//                       p+x+y, - at p-x+y and p+x-y), cf7 (xz), cf8 (yz).
//
// A block owns a tile of 64 packed columns x 8 rows and marches through a
// z-chunk, as the forward tiled kernels do, but holds ONE staged plane in
// LDS at a time: mu of the face colour (for the Laplacian) and the products
// coefficient x mu that the cells of the target colour read (face products
// of the face colour, edge products of the target colour).  A plane k'
// contributes to the target cells of planes k'-1 (their +z terms), k' (the
// in-plane terms) and k'+1 (their -z terms); a thread keeps these partial
// sums for its own column in registers, so a cell is complete once the plane
// above it has been staged.  The z-face products of the thread's own column
// come from direct loads.  32 KB of LDS (nDGP, Poisson), 42 KB (Kmouflage,
// whose x+/x- face coefficients differ).
//
// One kernel, three modes, one colour c per launch:
//   PASS   mu_c <- (faces - h^2 (G + f_c + fs)) / 6 into a fresh array;
//          finest level: block sums of the new values (the colour's sum).
//   RESID  r = (faces - 6 mu)/h^2 - G - f at colour c, and its restriction:
//          the colour-0 launch writes the raw sums of its 4 children per
//          coarse cell, the colour-1 launch adds its 4 and scales by 1/8
//          (R mu and R r); finest level: block sums of r and r^2.
//   CSRC   coarse FAS source S = (faces - 6 Ru)/h^2 - G(Ru) - Rd written over
//          Rd, and u = Ru, at colour c (both launches: the whole level).
#pragma once
#include "mg_tiled.h"

namespace mgk {

enum { ADJ_PASS = 0, ADJ_RESID = 1, ADJ_CSRC = 2 };

struct AdjLevel {
    const double *u0, *u1;       // mu (CSRC: R mu of the finer level)
    const double *c[9][2];       // coefficient arrays (minus faces alias plus for nDGP/Poisson)
    const double *lin[2];        // RC: linearisation point phi of the level
    const double *kp[2];         // RC: dK/dSigma at every cell
    const double *f0, *f1;       // right-hand side, never null (CSRC: R r, overwritten by S)
    int n, logn, lognh;
    double h2;
    double c3h4, c8h4;           // 1/(3 h^4), 1/(8 h^4)
};

// Staging geometry of one FP64 plane (tile plus halo, 66 x 10 values): 320
// 16-byte vectors and 20 halo values.  NT = 256 threads: every thread takes
// one vector, threads 0..63 a second one and threads 64..83 a halo value;
// NT = 512: threads 0..319 one vector, 320..339 a halo value.
template <int NT>
struct SGeom {
    static constexpr int NV = TYH * (TX / 2);   // 320 vectors
    static_assert(NT == 256 || NT == 512, "staging split");
    static constexpr int V2 = NT == 256 ? NV - NT : 0;   // threads with a second vector
    static constexpr int H0 = NT == 256 ? V2 : NV;       // first halo thread
    unsigned g0, g1;   // byte offsets inside a plane
    int l0, l1;        // value offsets inside a plane view
    __device__ __forceinline__ void init(int tid, int j0, int m0, int logn, int lognh) {
        const unsigned jm = (1u << logn) - 1, mm = (1u << lognh) - 1;
        auto vec = [&](int v, unsigned &g, int &l) {
            const int r = v >> 5, i = v & 31;
            g = ((((unsigned)(j0 - 1 + r) & jm) << lognh) + (unsigned)(m0 + 2 * i)) * 8u;
            l = r * TXH + 1 + 2 * i;
        };
        auto halo = [&](int t, unsigned &g, int &l) {
            const int h = (t >= H0 && t < H0 + 2 * TYH) ? t - H0 : 0, r = h >> 1, side = h & 1;
            const unsigned m = (unsigned)(side ? m0 + TX : m0 - 1) & mm;
            g = ((((unsigned)(j0 - 1 + r) & jm) << lognh) + m) * 8u;
            l = r * TXH + (side ? TXH - 1 : 0);
        };
        if (NT == 256) {
            vec(tid, g0, l0);
            if (tid < V2)
                vec(NT + tid, g1, l1);
            else
                halo(tid, g1, l1);
        } else {
            if (tid < NV)
                vec(tid, g0, l0);
            else
                halo(tid, g0, l0);
            g1 = g0;
            l1 = l0;
        }
    }
};

// One staged plane of one array in registers.  NT = 256: a0 and a1 hold the
// thread's vectors and threads 64..83 keep their halo value in a1.x; NT =
// 512: a0 (a halo value in a0.x).  One register pair per use keeps the
// struct in registers.
template <int NT>
struct SReg {
    using G = SGeom<NT>;
    double2 a0, a1;
    __device__ __forceinline__ void load(const double *A, size_t pl, const G &g, int tid) {
        const char *a = reinterpret_cast<const char *>(A) + pl;
        if (NT == 256) {
            a0 = *reinterpret_cast<const double2 *>(a + g.g0);
            if (tid < G::V2)
                a1 = *reinterpret_cast<const double2 *>(a + g.g1);
            else if (tid < G::H0 + 2 * TYH)
                a1.x = *reinterpret_cast<const double *>(a + g.g1);
        } else {
            if (tid < G::NV)
                a0 = *reinterpret_cast<const double2 *>(a + g.g0);
            else if (tid < G::H0 + 2 * TYH)
                a0.x = *reinterpret_cast<const double *>(a + g.g0);
        }
    }
    __device__ __forceinline__ void store(double *s, const G &g, int tid) const {
        if (NT == 256) {
            *reinterpret_cast<double2 *>(s + g.l0) = a0;
            if (tid < G::V2)
                *reinterpret_cast<double2 *>(s + g.l1) = a1;
            else if (tid < G::H0 + 2 * TYH)
                s[g.l1] = a1.x;
        } else {
            if (tid < G::NV)
                *reinterpret_cast<double2 *>(s + g.l0) = a0;
            else if (tid < G::H0 + 2 * TYH)
                s[g.l0] = a0.x;
        }
    }
    // s = this * y (element-wise)
    __device__ __forceinline__ void store_prod(double *s, const SReg &y, const G &g,
                                               int tid) const {
        if (NT == 256) {
            *reinterpret_cast<double2 *>(s + g.l0) = make_double2(a0.x * y.a0.x, a0.y * y.a0.y);
            if (tid < G::V2)
                *reinterpret_cast<double2 *>(s + g.l1) =
                    make_double2(a1.x * y.a1.x, a1.y * y.a1.y);
            else if (tid < G::H0 + 2 * TYH)
                s[g.l1] = a1.x * y.a1.x;
        } else {
            if (tid < G::NV)
                *reinterpret_cast<double2 *>(s + g.l0) =
                    make_double2(a0.x * y.a0.x, a0.y * y.a0.y);
            else if (tid < G::H0 + 2 * TYH)
                s[g.l0] = a0.x * y.a0.x;
        }
    }
};

// Deterministic block sum of two values over NT threads into
// partials[2 blk .. 2 blk + 1].
template <int NT>
__device__ __forceinline__ void block_sum2_nt(double a, double b, double *partials, size_t blk) {
    __shared__ double sa[NT / 64], sb[NT / 64];
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
        for (int q = 0; q < NT / 64; ++q) {
            x += sa[q];
            y += sb[q];
        }
        partials[2 * blk] = x;
        partials[2 * blk + 1] = y;
    }
}

// SYM: the x+ and x- (y, z) face coefficients are one array (nDGP, Poisson);
// COEF: the model has a non-Laplacian term (not Poisson).  REDUCE: block sums
// into partials[2 blk ..] (PASS: the new values; RESID: r and r^2).
//
// RC (nDGP): the products are rebuilt from the linearisation point instead
// of read from coefficient arrays.  With F' = dK/dSigma of a cell (the one
// array kept per level), the face coefficient of a face-colour cell is
// 2 F' (2A_x - A_y - A_z)/(3h^4) and the edge coefficient of a target-colour
// cell 2 F' N_xy/(8h^4) (y, z alike, as in k_adj_coefs); both read only the
// target colour's phi (the face neighbours of a face-colour cell and the
// edge neighbours of a target-colour cell have the target colour).  phi_c is
// staged on the tile with a 2-cell halo (68 x 12 values per plane) in a ring
// of 4 planes, two planes ahead of the products, so a plane's products see
// phi at k - 1, k and k + 1.  Per cell and pass: mu of both colours, phi of
// the target colour, F' of both colours, f and the new value (28 B against
// 40 B with the stored coefficients).
template <int NT, bool SYM, bool COEF, int MODE, bool REDUCE, bool RC = false>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(RC ? 4 : 1))) void k_adj_tiled(AdjLevel L, int c, double *out, double *out2,
                                                   const double *fptr,
                                                   double fscale, double *ru0, double *ru1,
                                                   double *rd0, double *rd1, double *partials,
                                                   TileGeom G) {
    constexpr int NF = SYM ? 2 : 4;   // staged in-plane face product arrays
    constexpr int W = NT / 64;        // waves = rows per row group
    constexpr int RPT = TY / W;       // rows per thread
    __shared__ __align__(16) double sM[TSLOT];
    __shared__ __align__(16) double sF[COEF ? NF : 1][TSLOT];
    __shared__ __align__(16) double sE[COEF ? 3 : 1][TSLOT];
    __shared__ double sX[MODE == ADJ_RESID ? 2 * RPT : 1][MODE == ADJ_RESID ? NT : 1];
    constexpr int PW = TX + 4, PH = TY + 4;        // RC: phi_c plane with a 2-cell halo
    constexpr int PSLOT = PW * PH, PNV = PH * (PW / 2);
    static_assert(!RC || (SYM && COEF && NT >= PNV), "RC: nDGP, one phi vector per thread");
    __shared__ __align__(16) double sP[RC ? 4 : 1][RC ? PSLOT : 2];
    const size_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int bx = (int)(blk % G.ntx);
    const int by = (int)((blk / G.ntx) % G.nty);
    const int bz = (int)(blk / ((size_t)G.ntx * G.nty));
    const int m0 = bx * TX, j0 = by * TY, k0 = bz * G.kz, k1 = k0 + G.kz;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int o = c ^ 1;
    const double *Mo = o ? L.u1 : L.u0;   // face colour
    const double *Mc = c ? L.u1 : L.u0;   // target colour
    const double *F = c ? L.f1 : L.f0;
    const double fs = fptr ? fscale * (*fptr) : 0.0;
    const double inv_h2 = 1.0 / L.h2;

    SGeom<NT> g;
    g.init(tid, j0, m0, L.logn, L.lognh);
    unsigned coff[RPT];
#pragma unroll
    for (int h = 0; h < RPT; ++h) coff[h] = cell_off<double>(j0 + ty + W * h, m0 + tx, L.lognh);

    // staged raw values of the next plane
    SReg<NT> rMo, rFx, rFy, rFx2, rFy2, rMc, rE6, rE7, rE8, rKo, rKc;
    // RC: phi_c of a plane (vector tid of 408: row tid / 34, packed columns
    // m0 - 2 + 2 (tid % 34) and the next), two planes ahead of the products
    unsigned pg = 0;
    int plds = 0;
    if constexpr (RC) {
        const int v = tid < PNV ? tid : 0;
        const int r = v / (PW / 2), i = v - r * (PW / 2);
        const unsigned jm = (1u << L.logn) - 1, mm = (1u << L.lognh) - 1;
        pg = ((((unsigned)(j0 - 2 + r) & jm) << L.lognh) + ((unsigned)(m0 - 2 + 2 * i) & mm)) * 8u;
        plds = r * PW + 2 * i;
    }
    const double *Pc = L.lin[c];
    double2 rP = make_double2(0.0, 0.0);
    auto pfetch = [&](int k) {
        if (RC && tid < PNV)
            rP = *reinterpret_cast<const double2 *>(
                reinterpret_cast<const char *>(Pc) + plane_off<double>(k, L.logn, L.lognh) + pg);
    };
    auto pstore = [&](int k) {
        if (RC && tid < PNV) *reinterpret_cast<double2 *>(sP[(k + 4) & 3] + plds) = rP;
    };
    auto fetch = [&](int k) {
        const size_t pl = plane_off<double>(k, L.logn, L.lognh);
        rMo.load(Mo, pl, g, tid);
        if constexpr (RC) {
            rMc.load(Mc, pl, g, tid);
            rKo.load(L.kp[o], pl, g, tid);
            rKc.load(L.kp[c], pl, g, tid);
            pfetch(k + 2);
        } else if constexpr (COEF) {
            rFx.load(L.c[0][o], pl, g, tid);
            rFy.load(L.c[2][o], pl, g, tid);
            if constexpr (!SYM) {
                rFx2.load(L.c[1][o], pl, g, tid);
                rFy2.load(L.c[3][o], pl, g, tid);
            }
            rMc.load(Mc, pl, g, tid);
            rE6.load(L.c[6][c], pl, g, tid);
            rE7.load(L.c[7][c], pl, g, tid);
            rE8.load(L.c[8][c], pl, g, tid);
        }
    };
    // RC: face sums of the face-colour cell and cross differences of the
    // target-colour cell at staged position (r, ci) of plane kp (r: row
    // j0 - 1 + r, ci: packed column m0 - 1 + ci) from the phi_c ring
    auto faces_at = [&](int r, int ci, int kp, double &ax, double &ay, double &az) {
        const int po = (o + j0 - 1 + r + kp) & 1;
        const double *P0 = sP[(kp + 4) & 3], *Pm = sP[(kp + 3) & 3], *Pp = sP[(kp + 5) & 3];
        const int r0 = (r + 1) * PW, rp = (r + 2) * PW, rm = r * PW, x0 = ci + 1;
        ax = P0[r0 + x0 + po] + P0[r0 + ci + po];
        ay = P0[rp + x0] + P0[rm + x0];
        az = Pp[r0 + x0] + Pm[r0 + x0];
    };
    auto prod = [&](int r, int ci, int kp, int l, double mo, double ko, double mc, double kc) {
        if constexpr (!RC) return;
        double ax, ay, az;
        faces_at(r, ci, kp, ax, ay, az);
        const double w = 2.0 * ko * L.c3h4;
        sF[0][1 + l] = w * (2.0 * ax - ay - az) * mo;
        sF[COEF ? 1 : 0][1 + l] = w * (2.0 * ay - ax - az) * mo;
        const int pc = (c + j0 - 1 + r + kp) & 1;
        const double *P0 = sP[(kp + 4) & 3], *Pm = sP[(kp + 3) & 3], *Pp = sP[(kp + 5) & 3];
        const int r0 = (r + 1) * PW, rp = (r + 2) * PW, rm = r * PW, x0 = ci + 1;
        const int xp = x0 + pc, xm = ci + pc;
        const double nxy = (P0[rp + xp] + P0[rm + xm]) - (P0[rm + xp] + P0[rp + xm]);
        const double nxz = (Pp[r0 + xp] + Pm[r0 + xm]) - (Pm[r0 + xp] + Pp[r0 + xm]);
        const double nyz = (Pp[rp + x0] + Pm[rm + x0]) - (Pm[rp + x0] + Pp[rm + x0]);
        const double e = 2.0 * kc * L.c8h4;
        sE[0][1 + l] = e * nxy * mc;
        sE[COEF ? 1 : 0][1 + l] = e * nxz * mc;
        sE[COEF ? 2 : 0][1 + l] = e * nyz * mc;
    };
    auto store = [&](int kp) {
        rMo.store(sM + 1, g, tid);
        if constexpr (RC) {
            pstore(kp + 2);
            using SG = SGeom<NT>;
            if (tid < SG::NV) {
                const int r = tid >> 5, ci = 1 + 2 * (tid & 31);
                prod(r, ci, kp, g.l0, rMo.a0.x, rKo.a0.x, rMc.a0.x, rKc.a0.x);
                // residual and coarse source: one position at a time
                // (interleaved, they spill); the pass is faster interleaved
                if constexpr (MODE != ADJ_PASS) __builtin_amdgcn_sched_barrier(0);
                prod(r, ci + 1, kp, g.l0 + 1, rMo.a0.y, rKo.a0.y, rMc.a0.y, rKc.a0.y);
            } else if (tid < SG::H0 + 2 * TYH) {
                const int hh = tid - SG::H0, r = hh >> 1, ci = (hh & 1) ? TXH - 1 : 0;
                prod(r, ci, kp, g.l0, rMo.a0.x, rKo.a0.x, rMc.a0.x, rKc.a0.x);
            }
        } else if constexpr (COEF) {
            rFx.store_prod(sF[0] + 1, rMo, g, tid);
            rFy.store_prod(sF[1] + 1, rMo, g, tid);
            if constexpr (!SYM) {
                rFx2.store_prod(sF[NF - 2] + 1, rMo, g, tid);
                rFy2.store_prod(sF[NF - 1] + 1, rMo, g, tid);
            }
            rE6.store_prod(sE[0] + 1, rMc, g, tid);
            rE7.store_prod(sE[COEF ? 1 : 0] + 1, rMc, g, tid);
            rE8.store_prod(sE[COEF ? 2 : 0] + 1, rMc, g, tid);
        }
    };
    // own-column values one plane ahead: the z-face coefficients (x+ ... z-
    // order: 4 = z+, 5 = z-) of the face-colour cell, and f (and mu) of the
    // target cell
    double z4n[RPT] = {}, z5n[RPT] = {}, fn[RPT] = {}, un[RPT] = {};
    auto fetch_cells = [&](int k) {
        const size_t pl = plane_off<double>(k, L.logn, L.lognh);
#pragma unroll
        for (int h = 0; h < RPT; ++h) {
            if constexpr (RC) {
                z4n[h] = ld(L.kp[o], pl, coff[h]);   // F' of the face-colour cell
            } else if constexpr (COEF) {
                z4n[h] = ld(L.c[4][o], pl, coff[h]);
                z5n[h] = SYM ? z4n[h] : ld(L.c[5][o], pl, coff[h]);
            }
            // (also at the two planes outside the chunk, where they are unused:
            // plane_off wraps, so the loads stay inside the level)
            fn[h] = ld_once(F, pl, coff[h]);
            if constexpr (MODE != ADJ_PASS) un[h] = ld_once(Mc, pl, coff[h]);
        }
    };

    // partial sums (Laplacian neighbours, G) of the target cells in the
    // thread's column: pF/pG at plane kp - 1 (completed by plane kp), cF/cG at
    // plane kp (its -z terms so far)
    double pF[RPT] = {}, pG[RPT] = {}, cF[RPT] = {}, cG[RPT] = {};
    double fc[RPT] = {}, uc[RPT] = {};   // f, mu of the cells at plane kp
    double fp[RPT] = {}, up[RPT] = {};   // ... at plane kp - 1
    double bs1 = 0.0, bs2 = 0.0;         // block sums
    double rr[RPT] = {}, rm_[RPT] = {};  // restriction sums over a plane pair
    int pair_K = -1;                                 // pair waiting for its combine

    // combine a completed plane pair with the sibling row (ty ^ 1) and write
    // the coarse cells (even ty): rows j0 + ty + W h and j0 + ty + 1 + W h
    // form coarse row (j0 + ty + W h) / 2
    auto pair_combine = [&](int K) {
        if (ty & 1) return;
        const int lnc = L.logn - 1, I = m0 + tx;
#pragma unroll
        for (int h = 0; h < RPT; ++h) {
            const double sr = sX[2 * h][tid] + sX[2 * h][tid + 64];
            const double su = sX[2 * h + 1][tid] + sX[2 * h + 1][tid + 64];
            const int J = (j0 + ty + W * h) >> 1;
            const size_t cidx =
                ((size_t)K << (2 * lnc - 1)) + ((size_t)J << (lnc - 1)) + (size_t)(I >> 1);
            const bool odd = (I + J + K) & 1;
            double *pr = odd ? rd1 : rd0, *pu = odd ? ru1 : ru0;
            if (c == 0) {   // raw sums of the 4 colour-0 children
                pr[cidx] = sr;
                pu[cidx] = su;
            } else {        // add the 4 colour-1 children: the 8-cell mean
                pr[cidx] = 0.125 * (pr[cidx] + sr);
                pu[cidx] = 0.125 * (pu[cidx] + su);
            }
        }
    };

    if constexpr (RC) {   // phi_c planes k0 - 2 .. k0 (the products of k0 - 1 need them)
        for (int kk = k0 - 2; kk <= k0; ++kk) {
            pfetch(kk);
            pstore(kk);
        }
    }
    fetch(k0 - 1);
    fetch_cells(k0 - 1);
    if constexpr (RC) __syncthreads();
    for (int kp = k0 - 1; kp <= k1; ++kp) {
        store(kp);
        double z4[RPT], z5[RPT];
#pragma unroll
        for (int h = 0; h < RPT; ++h) {
            if constexpr (RC) {
                double ax, ay, az;
                faces_at(ty + W * h + 1, tx + 1, kp, ax, ay, az);
                z4[h] = 2.0 * z4n[h] * L.c3h4 * (2.0 * az - ax - ay);
            } else {
                z4[h] = z4n[h];
            }
            z5[h] = SYM ? z4[h] : z5n[h];
            fp[h] = fc[h];
            up[h] = uc[h];
            fc[h] = fn[h];
            uc[h] = un[h];
        }
        __syncthreads();
        if (kp + 1 <= k1) {
            fetch(kp + 1);
            fetch_cells(kp + 1);
        }
        if constexpr (MODE == ADJ_RESID) {
            if (pair_K >= 0) {
                pair_combine(pair_K);
                pair_K = -1;
            }
        }
        const bool mid = kp >= k0 && kp < k1;
        const bool fin = kp - 1 >= k0;
        const double *Mv = sM + 1;
#pragma unroll
        for (int h = 0; h < RPT; ++h) {
            const int row = ty + W * h, j = j0 + row;
            const int r = row + 1, q = tx + 1;
            const int ro = r * TXH, rp = (r + 1) * TXH, rm = (r - 1) * TXH;
            // x parity of the target cell of row j: p at plane kp, p ^ 1 at
            // planes kp - 1 and kp + 1
            const int p = (j + kp + c) & 1, pz = p ^ 1;
            // this plane's face-colour value under/over the target cells of
            // planes kp + 1 / kp - 1, and their xz, yz edge terms
            const double mz = Mv[ro + q];
            double gup = 0.0, gdn = 0.0;
            if constexpr (COEF) {
                const double *Exz = sE[1] + 1, *Eyz = sE[2] + 1;
                const double exm = Exz[ro + q + pz - 1], exq = Exz[ro + q + pz];
                const double eym = Eyz[rm + q], eyq = Eyz[rp + q];
                gup = z4[h] * mz + ((exm - exq) + (eym - eyq));   // to plane kp + 1
                gdn = z5[h] * mz + ((exq - exm) + (eyq - eym));   // to plane kp - 1
            }
            if (fin) {   // the cell of plane kp - 1 is complete
                const double Ft = pF[h] + mz, Gt = pG[h] + gdn;
                const size_t pl = plane_off<double>(kp - 1, L.logn, L.lognh);
                if constexpr (MODE == ADJ_PASS) {
                    const double nv = (Ft - L.h2 * (Gt + fp[h] + fs)) * (1.0 / 6.0);
                    __builtin_nontemporal_store(nv, ptr(out, pl, coff[h]));
                    if (REDUCE) bs1 += nv;
                } else if constexpr (MODE == ADJ_RESID) {
                    const double d = (Ft - 6.0 * up[h]) * inv_h2 - Gt - fp[h];
                    if (REDUCE) {
                        bs1 += d;
                        bs2 += d * d;
                    }
                    rr[h] += d;
                    rm_[h] += up[h];
                } else {
                    *ptr(out, pl, coff[h]) = (Ft - 6.0 * up[h]) * inv_h2 - Gt - fp[h];
                    *ptr(out2, pl, coff[h]) = up[h];
                }
            }
            double fin_f = 0.0, fin_g = 0.0;   // in-plane terms of the cell of plane kp
            if (mid) {
                const int qp = q + p, qm = q + p - 1;
                fin_f = (Mv[ro + qp] + Mv[ro + qm]) + (Mv[rp + q] + Mv[rm + q]);
                if constexpr (COEF) {
                    const double *Px = sF[0] + 1, *Py = sF[1] + 1;
                    const double *Px2 = sF[NF - 2] + 1, *Py2 = sF[NF - 1] + 1;   // x-, y- faces
                    const double *Exy = sE[0] + 1;
                    // p - x carries its x+ coefficient, p + x its x- one (y alike)
                    fin_g = (Px[ro + qm] + Px2[ro + qp]) + (Py[rm + q] + Py2[rp + q]);
                    fin_g += (Exy[rm + qm] + Exy[rp + qp]) - (Exy[rp + qm] + Exy[rm + qp]);
                }
            }
            pF[h] = cF[h] + fin_f;
            pG[h] = cG[h] + fin_g;
            cF[h] = mz;
            cG[h] = gup;
        }
        if constexpr (MODE == ADJ_RESID) {
            // plane kp - 1 closed a plane pair: publish the row sums
            if (fin && ((kp - 1) & 1)) {
#pragma unroll
                for (int h = 0; h < RPT; ++h) {
                    sX[2 * h][tid] = rr[h];
                    sX[2 * h + 1][tid] = rm_[h];
                    rr[h] = 0.0;
                    rm_[h] = 0.0;
                }
                pair_K = (kp - 1) >> 1;
            }
        }
        __syncthreads();
    }
    if constexpr (MODE == ADJ_RESID) {
        if (pair_K >= 0) pair_combine(pair_K);
    }
    if (REDUCE) block_sum2_nt<NT>(bs1, bs2, partials, blk);
}

}  // namespace mgk
