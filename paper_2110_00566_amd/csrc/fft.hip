// FFT Poisson solve of the particle-mesh step (Sec. 3.1 of the paper: the
// Newtonian potential from the density by FFT and the Green's function),
// FP64, periodic n^3 mesh, n a power of two.
//
// The Green's function of the 7-point Laplacian, G(k) = -1 / (4 sum_i
// sin^2(pi k_i / n)) with G(0) = 0, is real and even in every axis, so the
// convolution can use the separable discrete Hartley transform
// H(k) = sum_x f(x) cas(2 pi k x / n), cas = cos + sin, per axis: for a
// kernel even in each variable the transform of the convolution is the
// product of the transforms, and H is its own inverse up to 1/n.  Every
// array stays real and keeps its shape:
//   x pass (delta -> phi), y pass, z pass with the multiply by s G / n^3
//   and the inverse z transform in the same block, y pass, x pass.
// Each pass transforms B = 2 NP lines of one axis per block.  Two real lines
// a, b are transformed together as one complex FFT of z = a + i b, and the
// Hartley transforms follow from Z(k) and Z(n - k):
//   H_a(k) = [Re Z(k) + Re Z(n-k) - Im Z(k) + Im Z(n-k)] / 2,
//   H_b(k) = [Im Z(k) + Im Z(n-k) + Re Z(k) - Re Z(n-k)] / 2.
// The complex FFT is a self-sorting (Stockham) sequence of radix-16 stages
// (the last one radix 2, 4 or 8): a thread reads the R values x[j + m n/R],
// multiplies them by the stage's twiddles, takes their R-point DFT in
// registers and writes them to (j / Ns) Ns R + j mod Ns + r Ns, Ns being the
// product of the earlier radices.  The first stage reads its values straight
// from HBM (one 16-byte load of two neighbouring lines along y and z, so a
// row of the B lines is one 128-byte segment at B = 16), the later ones from
// the block's lines in LDS, padded by one value every 16 and one per line so
// that the strided accesses of a stage fall into distinct banks.  The
// Green multiply feeds the first stage of the inverse z transform directly.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/mgglam.h"

namespace mgglam_internal {
void set_error(const char *msg);   // mg_last_error() of the library
}

namespace {

mg_status fail(mg_status s, const char *msg) {
    mgglam_internal::set_error(msg);
    return s;
}

// Twiddle table: w[k] = exp(-2 pi i k / n), k < n / 2.
__global__ __launch_bounds__(256) void k_twiddles(double2 *w, int n) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n / 2) return;
    double s, c;
    sincospi(2.0 * k / n, &s, &c);
    w[k] = make_double2(c, -s);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
    return make_double2(a.x - b.x, a.y - b.y);
}

constexpr int brev(int i, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}
constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }

// R-point DFT (R = 2, 4, 8, 16) of v in registers, natural order in and out,
// forward sign: radix-2 decimation in time over the bit-reversed copy, with
// the twiddles exp(-2 pi i e / 16) as constants (e = 0 and e = 4, i.e. 1 and
// -i, need no multiply).
template <int R>
__device__ __forceinline__ void dft_reg(double2 (&v)[R]) {
    constexpr double C[8] = {1.0,
                             0.92387953251128675613,
                             0.70710678118654752440,
                             0.38268343236508977173,
                             0.0,
                             -0.38268343236508977173,
                             -0.70710678118654752440,
                             -0.92387953251128675613};
    constexpr int LR = ilog2c(R);
    double2 a[R];
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = v[brev(i, LR)];
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
        for (int g = 0; g < R; g += len) {
#pragma unroll
            for (int pos = 0; pos < len / 2; ++pos) {
                const int e = pos * (16 / len);
                double2 b = a[g + pos + len / 2];
                if (e == 4) {
                    b = make_double2(b.y, -b.x);
                } else if (e != 0) {
                    // exp(-2 pi i e / 16) = cos - i sin, sin(pi e / 8) = C[|4 - e|]
                    const double c = C[e], s = (e < 4) ? C[4 - e] : C[e - 4];
                    b = make_double2(b.x * c + b.y * s, b.y * c - b.x * s);
                }
                const double2 x = a[g + pos];
                a[g + pos] = cadd(x, b);
                a[g + pos + len / 2] = csub(x, b);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = a[i];
}

// padded LDS offset of element x of a line
__device__ __forceinline__ int phys(int x) { return x + (x >> 4); }

template <int LOGN>
struct Fft {
    static constexpr int n = 1 << LOGN;
    static constexpr int L0 = LOGN < 4 ? LOGN : 4;
    static constexpr int R0 = 1 << L0;           // radix of the first stage
    static constexpr int NR = n / R0;            // first-stage butterflies per line
    static constexpr int S = n + (n >> 4) + 1;   // padded line stride (complex values)
};

// The Stockham stages after the first: Ns = 2^NSL, radix 2^min(4, LOGN - NSL).
// Each of the T threads takes R0 / R butterflies; every value is read before
// the barrier and written after it, so the stage works in place.
template <int LOGN, int T, int NSL>
__device__ __forceinline__ void stages(double2 *Z, const double2 *__restrict__ wt) {
    if constexpr (NSL < LOGN) {
        using F = Fft<LOGN>;
        constexpr int LR = (LOGN - NSL) < 4 ? (LOGN - NSL) : 4;
        constexpr int R = 1 << LR, NS = 1 << NSL, NB = F::R0 / R, NRS = F::n / R;
        double2 v[NB][R];
        int off[NB], oout[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int u = threadIdx.x + b * T;
            const int p = u / NRS, jj = u % NRS, k = jj & (NS - 1);
            const double2 w1 = wt[k * (F::n / (NS * R))];
            off[b] = p * F::S;
            oout[b] = (jj / NS) * NS * R + k;
#pragma unroll
            for (int m = 0; m < R; ++m) v[b][m] = Z[off[b] + phys(jj + m * NRS)];
            double2 wp[R];
            wp[1] = w1;
#pragma unroll
            for (int m = 2; m < R; ++m) wp[m] = cmul(wp[m / 2], wp[m - m / 2]);
#pragma unroll
            for (int m = 1; m < R; ++m) v[b][m] = cmul(v[b][m], wp[m]);
            dft_reg<R>(v[b]);
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int r = 0; r < R; ++r) Z[off[b] + phys(oout[b] + r * NS)] = v[b][r];
        }
        __syncthreads();
        stages<LOGN, T, NSL + LR>(Z, wt);
    }
}

// cos(2 pi k / n) from the twiddle table (0 <= k < n)
__device__ __forceinline__ double cos_tab(const double2 *__restrict__ w, int k, int n) {
    if (k == n / 2) return -1.0;
    return w[k < n / 2 ? k : n - k].x;
}

// Hartley values of the two lines of a packed spectrum at k
__device__ __forceinline__ double2 hartley_pair(const double2 *Zl, int k, int n) {
    const double2 zk = Zl[phys(k)], zn = Zl[phys((n - k) & (n - 1))];
    return make_double2(0.5 * ((zk.x + zn.x) - (zk.y - zn.y)),
                        0.5 * ((zk.y + zn.y) + (zk.x - zn.x)));
}

// Geometry of a pass: block = line group g (B = 2 NP consecutive lines) of
// plane or row q; line b's element k at base + b sb + k sn,
// base = q qstride + g B sb.  XAXIS: lines along x (sn = 1, sb = n).
// rows_first (z pass): consecutive blocks take consecutive rows q of one
// line group, so the blocks in flight read rows that share address
// translations (every z-line block touches all n planes): 4% on that pass.
struct PassGeo {
    size_t qstride, sn, sb;
    int rows_first;
};

template <int LOGN, int NP, bool XAXIS, bool GREEN>
__global__ __launch_bounds__(NP * Fft<LOGN>::NR) void k_hartley(const double *src, double *dst,
                                                                PassGeo geo,
                                                                const double2 *__restrict__ wt,
                                                                double scale) {
    using F = Fft<LOGN>;
    constexpr int n = F::n, R0 = F::R0, NR = F::NR, T = NP * NR, B = 2 * NP;
    extern __shared__ double2 Z[];
    const int t = threadIdx.x;
    const int groups = n / B;
    const int g = geo.rows_first ? (int)(blockIdx.x / n) : (int)(blockIdx.x % groups);
    const int q = geo.rows_first ? (int)(blockIdx.x % n) : (int)(blockIdx.x / groups);
    const size_t base = (size_t)q * geo.qstride + (size_t)g * B * geo.sb;
    // first stage from HBM.  Along x consecutive threads take consecutive
    // elements of a line; along y and z consecutive line pairs.
    int p = XAXIS ? t / NR : t % NP;
    int j = XAXIS ? t % NR : t / NP;
    double2 v[R0];
#pragma unroll
    for (int m = 0; m < R0; ++m) {
        const size_t x = (size_t)(j + m * NR);
        if constexpr (XAXIS) {
            v[m] = make_double2(src[base + (size_t)(2 * p) * n + x],
                                src[base + (size_t)(2 * p + 1) * n + x]);
        } else {
            v[m] = *reinterpret_cast<const double2 *>(src + base + 2 * p + x * geo.sn);
        }
    }
    dft_reg<R0>(v);
#pragma unroll
    for (int r = 0; r < R0; ++r) Z[p * F::S + phys(j * R0 + r)] = v[r];
    __syncthreads();
    stages<LOGN, T, F::L0>(Z, wt);
    if constexpr (GREEN) {
        // Hartley values times scale G(kx, ky, kz) are the inverse
        // transform's input; its first stage takes them from here
        p = t / NR;
        j = t % NR;
        const int kx = g * B + 2 * p;
        const double sy = 0.5 * (1.0 - cos_tab(wt, q, n));
        const double sxa = 0.5 * (1.0 - cos_tab(wt, kx, n)) + sy;
        const double sxb = 0.5 * (1.0 - cos_tab(wt, kx + 1, n)) + sy;
#pragma unroll
        for (int m = 0; m < R0; ++m) {
            const int k = j + m * NR;
            const double2 h = hartley_pair(Z + p * F::S, k, n);
            const double sz = 0.5 * (1.0 - cos_tab(wt, k, n));
            const double da = 4.0 * (sxa + sz), db = 4.0 * (sxb + sz);
            v[m] = make_double2(da > 0.0 ? -scale / da * h.x : 0.0,
                                db > 0.0 ? -scale / db * h.y : 0.0);
        }
        __syncthreads();
        dft_reg<R0>(v);
#pragma unroll
        for (int r = 0; r < R0; ++r) Z[p * F::S + phys(j * R0 + r)] = v[r];
        __syncthreads();
        stages<LOGN, T, F::L0>(Z, wt);
    }
    // Hartley values of both lines, stored
    p = XAXIS ? t / NR : t % NP;
    j = XAXIS ? t % NR : t / NP;
#pragma unroll
    for (int m = 0; m < R0; ++m) {
        const int k = j + m * NR;
        const double2 h = hartley_pair(Z + p * F::S, k, n);
        if constexpr (XAXIS) {
            dst[base + (size_t)(2 * p) * n + k] = h.x;
            dst[base + (size_t)(2 * p + 1) * n + k] = h.y;
        } else {
            *reinterpret_cast<double2 *>(dst + base + 2 * p + (size_t)k * geo.sn) = h;
        }
    }
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// line pairs per block: about 256 threads (x) or 512 (y, z: 16 lines, a
// 128-byte row segment, at n = 1024), at most n / 2
#ifndef MG_FFT_THREADS_X
#define MG_FFT_THREADS_X 256
#endif
#ifndef MG_FFT_THREADS_YZ
#define MG_FFT_THREADS_YZ 512
#endif
#ifndef MG_FFT_THREADS_Z
#define MG_FFT_THREADS_Z MG_FFT_THREADS_YZ
#endif
constexpr int pairs_per_block(int logn, int threads) {
    const int n = 1 << logn, r0 = logn < 4 ? (1 << logn) : 16;
    const int np = threads * r0 / n;
    return np < 1 ? 1 : (np > n / 2 ? n / 2 : np);
}

template <int LOGN, int NP, bool XAXIS, bool GREEN>
mg_status launch_pass(const double *src, double *dst, PassGeo geo, const double2 *wt,
                      double scale, hipStream_t stream) {
    using F = Fft<LOGN>;
    constexpr size_t lds = sizeof(double2) * (size_t)NP * F::S;
    static_assert(lds <= 160 * 1024, "FFT block exceeds the LDS of a CU");
    if constexpr (lds > 64 * 1024) {
        static std::once_flag once;
        static hipError_t rc = hipSuccess;
        std::call_once(once, [&] {
            rc = hipFuncSetAttribute((const void *)k_hartley<LOGN, NP, XAXIS, GREEN>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        });
        if (rc != hipSuccess) {
            (void)hipGetLastError();
            const std::string m =
                std::string("HIP: cannot raise the FFT pass's LDS limit: ") + hipGetErrorString(rc);
            return fail(MG_ERR_HIP, m.c_str());
        }
    }
    const unsigned blocks = (unsigned)((size_t)(F::n / (2 * NP)) * F::n);
    k_hartley<LOGN, NP, XAXIS, GREEN><<<blocks, NP * F::NR, lds, stream>>>(src, dst, geo, wt, scale);
    return MG_OK;
}

template <int LOGN>
mg_status poisson_passes(const double *delta, double *phi, const double2 *w, double scale,
                         hipStream_t stream) {
    constexpr int n = 1 << LOGN;
    constexpr int NPX = pairs_per_block(LOGN, MG_FFT_THREADS_X);
    constexpr int NPYZ = pairs_per_block(LOGN, MG_FFT_THREADS_YZ);
    constexpr int NPZ = pairs_per_block(LOGN, MG_FFT_THREADS_Z);
    const size_t nn = (size_t)n * n;
    const PassGeo GX{nn, 1, (size_t)n, 0}, GY{nn, (size_t)n, 1, 0}, GZ{(size_t)n, nn, 1, 1};
    mg_status rc;
    if ((rc = launch_pass<LOGN, NPX, true, false>(delta, phi, GX, w, 0.0, stream)) != MG_OK) return rc;
    if ((rc = launch_pass<LOGN, NPYZ, false, false>(phi, phi, GY, w, 0.0, stream)) != MG_OK) return rc;
    if ((rc = launch_pass<LOGN, NPZ, false, true>(phi, phi, GZ, w, scale, stream)) != MG_OK) return rc;
    if ((rc = launch_pass<LOGN, NPYZ, false, false>(phi, phi, GY, w, 0.0, stream)) != MG_OK) return rc;
    return launch_pass<LOGN, NPX, true, false>(phi, phi, GX, w, 0.0, stream);
}

}  // namespace

namespace mgglam_internal {

size_t fft_poisson_ws_bytes(int n) { return pow2(n) ? (size_t)(n / 2) * 16 + 256 : 0; }

// phi = s * lap7^{-1} (delta - mean delta), zero mean (all device pointers;
// ws: n / 2 twiddles).  Enqueued on stream.
mg_status fft_poisson(int n, double s, const double *delta, double *phi, void *ws,
                      hipStream_t stream) {
    double2 *w = static_cast<double2 *>(ws);
    k_twiddles<<<(n / 2 + 255) / 256, 256, 0, stream>>>(w, n);
    const double scale = s / ((double)n * n * n);
    mg_status rc;
    switch (ilog2i(n)) {
        case 3: rc = poisson_passes<3>(delta, phi, w, scale, stream); break;
        case 4: rc = poisson_passes<4>(delta, phi, w, scale, stream); break;
        case 5: rc = poisson_passes<5>(delta, phi, w, scale, stream); break;
        case 6: rc = poisson_passes<6>(delta, phi, w, scale, stream); break;
        case 7: rc = poisson_passes<7>(delta, phi, w, scale, stream); break;
        case 8: rc = poisson_passes<8>(delta, phi, w, scale, stream); break;
        case 9: rc = poisson_passes<9>(delta, phi, w, scale, stream); break;
        case 10: rc = poisson_passes<10>(delta, phi, w, scale, stream); break;
        case 11: rc = poisson_passes<11>(delta, phi, w, scale, stream); break;
        default: return fail(MG_ERR_ARG, "n must be a power of two in [8, 2048]");
    }
    if (rc != MG_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        const std::string m = std::string("HIP: ") + hipGetErrorString(e);
        return fail(MG_ERR_HIP, m.c_str());
    }
    return MG_OK;
}

}  // namespace mgglam_internal

extern "C" {

size_t mg_fft_poisson_workspace_bytes(int n) {
    if (!pow2(n) || n < 8 || n > 2048) return 0;
    return mgglam_internal::fft_poisson_ws_bytes(n);
}

mg_status mg_fft_poisson(int n, double s, const double *delta, double *phi, void *ws,
                         size_t ws_bytes, hipStream_t stream) {
    mgglam_internal::set_error("");
    if (!pow2(n) || n < 8 || n > 2048)
        return fail(MG_ERR_ARG, "n must be a power of two in [8, 2048]");
    if (!std::isfinite(s)) return fail(MG_ERR_ARG, "s must be finite");
    if (!delta || !phi) return fail(MG_ERR_ARG, "delta and phi must be device pointers");
    if (delta == phi) return fail(MG_ERR_ARG, "delta and phi must not alias");
    if (((uintptr_t)delta | (uintptr_t)phi) & 15)
        return fail(MG_ERR_ARG, "delta and phi must be 16-byte aligned");
    if (!ws || ws_bytes < mg_fft_poisson_workspace_bytes(n) || ((uintptr_t)ws & 255))
        return fail(MG_ERR_WORKSPACE, "workspace is NULL, too small or not 256-byte aligned");
    const mg_status rc = mgglam_internal::fft_poisson(n, s, delta, phi, ws, stream);
    if (rc != MG_OK) return rc;
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        const std::string m = std::string("HIP: ") + hipGetErrorString(e);
        return fail(MG_ERR_HIP, m.c_str());
    }
    return MG_OK;
}

}  // extern "C"
