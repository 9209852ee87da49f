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
// Each pass transforms B lines of one axis per block in LDS.  Two real lines
// a, b are transformed together as one complex FFT of z = a + i b (radix-2,
// in place after a bit-reversed load), and the Hartley transforms follow
// from Z(k) and Z(n - k):
//   H_a(k) = [Re Z(k) + Re Z(n-k) - Im Z(k) + Im Z(n-k)] / 2,
//   H_b(k) = [Im Z(k) + Im Z(n-k) + Re Z(k) - Re Z(n-k)] / 2.
// Lines along y and z are batched over B consecutive x positions, so every
// global access moves B consecutive doubles.
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

constexpr int FT = 512;   // threads per block

// Twiddle table: w[k] = exp(-2 pi i k / n), k < n / 2.
__global__ __launch_bounds__(256) void k_twiddles(double2 *w, int n) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n / 2) return;
    double s, c;
    sincospi(2.0 * k / n, &s, &c);
    w[k] = make_double2(c, -s);
}

__device__ __forceinline__ int bitrev(int x, int logn) {
    return (int)(__builtin_bitreverse32((unsigned)x) >> (32 - logn));
}

// cos(2 pi k / n) from the twiddle table (any 0 <= k < n)
__device__ __forceinline__ double cos_tab(const double2 *w, int k, int n) {
    if (k == n / 2) return -1.0;
    return w[k < n / 2 ? k : n - k].x;
}

struct Lines {
    int n, logn, B;     // line length, lines per block
    size_t sn, sb;      // stride between elements of a line, between the block's lines
};

// Complex FFTs of length n of the block's NP = B / 2 packed line pairs in
// LDS (in place, input in bit-reversed order).
__device__ __forceinline__ void fft_lds(double2 *Z, const double2 *w, int n, int NP) {
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len >> 1, ts = n / len;
        const int nb = NP * (n >> 1);
        for (int q = threadIdx.x; q < nb; q += FT) {
            const int p = q / (n >> 1), j = q - p * (n >> 1);
            const int g = j / half, pos = j - g * half;
            double2 *z = Z + (size_t)p * n;
            const int i0 = g * len + pos, i1 = i0 + half;
            const double2 tw = w[pos * ts];
            const double2 a = z[i0], b = z[i1];
            const double2 bt = make_double2(b.x * tw.x - b.y * tw.y, b.x * tw.y + b.y * tw.x);
            z[i0] = make_double2(a.x + bt.x, a.y + bt.y);
            z[i1] = make_double2(a.x - bt.x, a.y - bt.y);
        }
        __syncthreads();
    }
}

// Hartley value of line b (0 .. B-1) at index k from the packed spectra.
__device__ __forceinline__ double hartley(const double2 *Z, int b, int k, int n) {
    const double2 *z = Z + (size_t)(b >> 1) * n;
    const double2 zk = z[k], zn = z[(n - k) & (n - 1)];
    return (b & 1) ? 0.5 * ((zk.y + zn.y) + (zk.x - zn.x))
                   : 0.5 * ((zk.x + zn.x) - (zk.y - zn.y));
}

// One pass: the Hartley transform of the block's B lines of one axis.
// GREEN (z pass): then the multiply by scale * G(kx, ky, kz) and the inverse
// transform along z before the store.  Block decomposition: block = line
// group g (B consecutive lines) of plane/row q; base offsets from the axis.
template <bool GREEN>
__global__ __launch_bounds__(FT) void k_dht_pass(const double *src, double *dst, Lines Ln,
                                                 int axis, const double2 *wg, double scale) {
    extern __shared__ double2 lds[];
    const int n = Ln.n, B = Ln.B, NP = B >> 1;
    double2 *Z = lds;                         // NP * n complex
    double2 *w = lds + (size_t)NP * n;        // n / 2 twiddles
    for (int k = threadIdx.x; k < n / 2; k += FT) w[k] = wg[k];
    const int groups = n / B;
    const int g = blockIdx.x % groups, q = blockIdx.x / groups;
    // first element of the block's first line; the lines follow at stride sb
    size_t base;
    int kx0 = 0, ky = 0;
    if (axis == 0) {   // lines along x: rows y = g B .. of plane z = q
        base = (size_t)q * n * n + (size_t)g * B * n;
    } else if (axis == 1) {   // lines along y: columns x = g B .. of plane z = q
        base = (size_t)q * n * n + (size_t)g * B;
    } else {   // lines along z: columns x = g B .. of row y = q
        base = (size_t)q * n + (size_t)g * B;
        kx0 = g * B;
        ky = q;
    }
    // load (bit-reversed within each line); coalesced along the contiguous
    // direction: the line itself (x pass) or the B lines (y, z passes)
    const int tot = B * n;
    for (int e = threadIdx.x; e < tot; e += FT) {
        int b, k;
        if (Ln.sn == 1) {
            b = e / n;
            k = e - b * n;
        } else {
            k = e / B;
            b = e - k * B;
        }
        const double v = src[base + (size_t)b * Ln.sb + (size_t)k * Ln.sn];
        double2 *z = Z + (size_t)(b >> 1) * n + bitrev(k, Ln.logn);
        if (b & 1)
            z->y = v;
        else
            z->x = v;
    }
    __syncthreads();
    fft_lds(Z, w, n, NP);
    if (GREEN) {
        // Hartley values times scale * G, repacked (bit-reversed) for the
        // inverse transform; the writes wait until every read is done.  At
        // most MAXV = 16384 / FT values per thread (B n <= 16384).
        constexpr int MAXV = 16384 / FT;
        double hv[MAXV];
        const double sy = 0.5 * (1.0 - cos_tab(w, ky, n));
#pragma unroll
        for (int it = 0; it < MAXV; ++it) {
            const int e = threadIdx.x + it * FT;
            if (e < tot) {
                const int k = e / B, b = e - k * B;   // k = kz
                const double sx = 0.5 * (1.0 - cos_tab(w, kx0 + b, n));
                const double sz = 0.5 * (1.0 - cos_tab(w, k, n));
                const double den = 4.0 * ((sx + sy) + sz);
                const double gk = den > 0.0 ? -scale / den : 0.0;
                hv[it] = gk * hartley(Z, b, k, n);
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < MAXV; ++it) {
            const int e = threadIdx.x + it * FT;
            if (e < tot) {
                const int k = e / B, b = e - k * B;
                double2 *z = Z + (size_t)(b >> 1) * n + bitrev(k, Ln.logn);
                if (b & 1)
                    z->y = hv[it];
                else
                    z->x = hv[it];
            }
        }
        __syncthreads();
        fft_lds(Z, w, n, NP);
    }
    for (int e = threadIdx.x; e < tot; e += FT) {
        int b, k;
        if (Ln.sn == 1) {
            b = e / n;
            k = e - b * n;
        } else {
            k = e / B;
            b = e - k * B;
        }
        dst[base + (size_t)b * Ln.sb + (size_t)k * Ln.sn] = hartley(Z, b, k, n);
    }
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// lines per block: 16 (a 128-byte segment per access) while the block's
// spectra and twiddles fit in 160 KB of LDS, else 8
int lines_per_block(int n) { return n >= 2048 ? 8 : (n >= 16 ? 16 : n); }

size_t lds_bytes(int n) {
    return sizeof(double2) * ((size_t)(lines_per_block(n) / 2) * n + n / 2);
}

}  // namespace

namespace mgglam_internal {

size_t fft_poisson_ws_bytes(int n) { return pow2(n) ? (size_t)(n / 2) * 16 + 256 : 0; }

// phi = s * lap7^{-1} (delta - mean delta), zero mean (all device pointers;
// ws: n / 2 twiddles).  Enqueued on stream.
mg_status fft_poisson(int n, double s, const double *delta, double *phi, void *ws,
                      hipStream_t stream) {
    const size_t lds = lds_bytes(n);
    if (lds > 64 * 1024) {   // allow the passes the CU's whole LDS
        static std::once_flag once;
        static hipError_t attr_rc = hipSuccess;
        std::call_once(once, [] {
            attr_rc = hipFuncSetAttribute((const void *)k_dht_pass<false>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (attr_rc == hipSuccess)
                attr_rc = hipFuncSetAttribute((const void *)k_dht_pass<true>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize,
                                              160 * 1024);
        });
        if (attr_rc != hipSuccess) {
            (void)hipGetLastError();
            const std::string m =
                std::string("HIP: cannot raise the FFT passes' LDS limit: ") + hipGetErrorString(attr_rc);
            return fail(MG_ERR_HIP, m.c_str());
        }
    }
    double2 *w = static_cast<double2 *>(ws);
    k_twiddles<<<(n / 2 + 255) / 256, 256, 0, stream>>>(w, n);
    const int B = lines_per_block(n), logn = ilog2i(n);
    const unsigned blocks = (unsigned)((size_t)(n / B) * n);
    const size_t nn = (size_t)n * n;
    const Lines LX{n, logn, B, 1, (size_t)n}, LY{n, logn, B, (size_t)n, 1},
        LZ{n, logn, B, nn, 1};
    const double scale = s / ((double)n * n * n);
    k_dht_pass<false><<<blocks, FT, lds, stream>>>(delta, phi, LX, 0, w, 0.0);
    k_dht_pass<false><<<blocks, FT, lds, stream>>>(phi, phi, LY, 1, w, 0.0);
    k_dht_pass<true><<<blocks, FT, lds, stream>>>(phi, phi, LZ, 2, w, scale);
    k_dht_pass<false><<<blocks, FT, lds, stream>>>(phi, phi, LY, 1, w, 0.0);
    k_dht_pass<false><<<blocks, FT, lds, stream>>>(phi, phi, LX, 0, w, 0.0);
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
