// Particle-mesh substrate around the scalar-field solve (Sec. 3.1 of the
// paper): cloud-in-cell density assignment, the Newtonian and scalar
// potentials, 3-point central-difference forces interpolated back to the
// particles with the same CIC weights, and a leapfrog kick-drift in a.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/mgglam.h"

namespace mgglam_internal {
void set_error(const char *msg);   // mg_last_error() of the library
// FFT Poisson solve (fft.hip): phi = s lap7^-1 (delta - mean), ws >= n/2 twiddles
mg_status fft_poisson(int n, double s, const double *delta, double *phi, void *ws,
                      hipStream_t stream);
}

namespace {

mg_status fail(mg_status s, const char *msg) {
    mgglam_internal::set_error(msg);
    return s;
}

// status of the launches enqueued so far (and, with sync, of their execution)
mg_status hip_status(hipStream_t stream, bool sync) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && sync) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        const std::string m = std::string("HIP: ") + hipGetErrorString(e);
        return fail(MG_ERR_HIP, m.c_str());
    }
    return MG_OK;
}

constexpr int PTPB = 256;

// Work-groups are dealt round-robin over the 8 XCDs, each with its own L2.
// The CIC gather, whose neighbouring tiles share lists and particles,
// renumbers block b so that each XCD takes one contiguous eighth of the
// blocks (a bijection when the block count is a multiple of 8, else the
// identity).
__device__ __forceinline__ size_t xcd_chunk(unsigned b, unsigned nblk) {
    if (nblk & 7u) return b;
    return (size_t)(b & 7u) * (nblk >> 3) + (b >> 3);
}
constexpr double FIX_SCALE = 4294967296.0;   // 2^32 fixed-point units per particle

__device__ __forceinline__ void cic_weights(const float *p, double f[3], int i0[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double x = (double)p[a] - 0.5;   // cell i has centre i + 1/2
        const double fl = floor(x);
        i0[a] = (int)fl;
        f[a] = x - fl;
    }
}

// Deposit: the eight weights of every particle, rounded to 64-bit fixed
// point, are added with integer atomics, so the sum is independent of order.
__global__ __launch_bounds__(PTPB) void k_cic(const float *__restrict__ pos, size_t np, int logn,
                                               unsigned long long *__restrict__ counts) {
    const size_t t = (size_t)blockIdx.x * PTPB + threadIdx.x;
    if (t >= np) return;
    const int nm1 = (1 << logn) - 1;
    double f[3];
    int i0[3];
    cic_weights(pos + 3 * t, f, i0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
        const double w = ((a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1])) * (c ? f[2] : 1.0 - f[2]);
        const int i = (i0[0] + a) & nm1, j = (i0[1] + b) & nm1, k = (i0[2] + c) & nm1;
        const size_t idx = ((size_t)k << (2 * logn)) + ((size_t)j << logn) + i;
        atomicAdd(counts + idx, __double2ull_rn(w * FIX_SCALE));
    }
}

// Gather form of the same deposit (for n_part^3 <= n_mesh^3): every particle
// is linked into the list of its lower CIC corner cell (one 32-bit atomic
// exchange per particle instead of eight 64-bit adds), then every cell sums
// the fixed-point weights of the particles in the 8 lists whose clouds reach
// it.  Integer sums are exact in any order, so delta is bit-identical to the
// scatter form whatever order the lists are built in.
__global__ __launch_bounds__(PTPB) void k_cic_link(const float *__restrict__ pos, int np, int logn,
                                                    int *__restrict__ head, int *__restrict__ next) {
    const int t = blockIdx.x * PTPB + threadIdx.x;
    if (t >= np) return;
    const int nm1 = (1 << logn) - 1;
    double f[3];
    int i0[3];
    cic_weights(pos + 3 * (size_t)t, f, i0);
    const size_t c = ((size_t)(i0[2] & nm1) << (2 * logn)) + ((size_t)(i0[1] & nm1) << logn) +
                     (size_t)(i0[0] & nm1);
    next[t] = atomicExch(head + c, t);
}

// Block-wide exclusive prefix sum of v over the PTPB threads (every thread
// calls it); *total receives the sum.
__device__ __forceinline__ int block_scan(int v, int *total) {
    __shared__ int wsum[PTPB / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < PTPB / 64; ++k) {
        if (k < w) base += wsum[k];
        tot += wsum[k];
    }
    *total = tot;
    __syncthreads();
    return base + x - v;
}

// Every particle in the NL lists of a block (list l starts at head[cell(l)]),
// handed to body(p, l) with all lanes busy: the lists are walked once to
// count them, the counts are scanned, and the (particle, list) pairs go into
// an LDS queue of KQ entries that all threads then drain; a tile with more
// than KQ particles takes several rounds (each walks the lists again).  The
// list, not the particle's position, says where it lies relative to the
// tile: on a mesh one tile wide the halo list below x = 0 is the tile's own
// last column.  With about
// one particle per eight cells, walking the lists directly would run the
// particle work once per list with most lanes idle.
constexpr int KQ = 1024;

template <int NL, class Cell, class Body>
__device__ __forceinline__ void tile_particles(const int *__restrict__ head,
                                               const int *__restrict__ next, Cell cell,
                                               int2 *queue, Body body) {
    constexpr int NR = (NL + PTPB - 1) / PTPB;
    int hd[NR], cnt = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int l = threadIdx.x + r * PTPB;
        hd[r] = l < NL ? head[cell(l)] : -1;
    }
#pragma unroll 1
    for (int r = 0; r < NR; ++r)
        for (int p = hd[r]; p >= 0; p = next[p]) ++cnt;
    int total;
    const int off = block_scan(cnt, &total);
    for (int base = 0; base < total; base += KQ) {
        int v = off;
#pragma unroll 1
        for (int r = 0; r < NR && v < base + KQ; ++r)
            for (int p = hd[r]; p >= 0 && v < base + KQ; p = next[p], ++v)
                if (v >= base) queue[v - base] = make_int2(p, threadIdx.x + r * PTPB);
        __syncthreads();
        const int m = total - base < KQ ? total - base : KQ;
        for (int e = threadIdx.x; e < m; e += PTPB) body(queue[e].x, queue[e].y);
        __syncthreads();
    }
}

// A block owns a tile of CGX x CGY x CGZ cells and walks, once, the lists
// of every corner cell whose particles reach the tile (the tile and one cell
// below it in each axis), adding the fixed-point weights that land inside
// the tile into LDS; then it writes the tile's delta.
// 32 x 8 x 8 walks 1.31 lists per cell (32 x 4 x 4: 1.61) and ran 16% faster
// on 256^3 particles over 512^3 cells than 32 x 4 x 4; taller or wider tiles
// were slower (fewer blocks per CU).
constexpr int CGX = 32, CGY = 8, CGZ = 8;
constexpr int CG_CELLS = CGX * CGY * CGZ;                      // 2048
constexpr int CG_LISTS = (CGX + 1) * (CGY + 1) * (CGZ + 1);    // 2673

template <typename T>
__global__ __launch_bounds__(PTPB) void k_cic_gather(const float *__restrict__ pos, int logn,
                                                      const int *__restrict__ head,
                                                      const int *__restrict__ next, double scale,
                                                      T *__restrict__ delta) {
    __shared__ unsigned long long acc[CG_CELLS];
    __shared__ int2 queue[KQ];
    const int nm1 = (1 << logn) - 1;
    const int ntx = (1 << logn) / CGX, nty = (1 << logn) / CGY;
    const int blk = (int)xcd_chunk(blockIdx.x, gridDim.x);
    const int bx = blk % ntx, by = (blk / ntx) % nty, bz = blk / (ntx * nty);
    const int x0 = bx * CGX, y0 = by * CGY, z0 = bz * CGZ;
    for (int q = threadIdx.x; q < CG_CELLS; q += PTPB) acc[q] = 0ull;
    // lists of the corner cells whose clouds reach the tile: the tile and
    // one cell below it in each axis
    auto cell = [&](int q) {
        const int lx = q % (CGX + 1) - 1, ly = (q / (CGX + 1)) % (CGY + 1) - 1,
                  lz = q / ((CGX + 1) * (CGY + 1)) - 1;
        return ((size_t)((z0 + lz) & nm1) << (2 * logn)) + ((size_t)((y0 + ly) & nm1) << logn) +
               (size_t)((x0 + lx) & nm1);
    };
    auto deposit = [&](int p, int q) {
        double f[3];
        int i0[3];
        cic_weights(pos + 3 * (size_t)p, f, i0);
        // the list's corner cell in tile coordinates (-1 .. CG-1)
        const int lx = q % (CGX + 1) - 1, ly = (q / (CGX + 1)) % (CGY + 1) - 1,
                  lz = q / ((CGX + 1) * (CGY + 1)) - 1;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int a = o & 1, b = (o >> 1) & 1, c = o >> 2;
            const int tx = lx + a, ty = ly + b, tz = lz + c;
            if (tx < 0 || tx >= CGX || ty < 0 || ty >= CGY || tz < 0 || tz >= CGZ) continue;
            const double w =
                ((a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1])) * (c ? f[2] : 1.0 - f[2]);
            atomicAdd(acc + (tz * CGY + ty) * CGX + tx, __double2ull_rn(w * FIX_SCALE));
        }
    };
    tile_particles<CG_LISTS>(head, next, cell, queue, deposit);
    for (int q = threadIdx.x; q < CG_CELLS; q += PTPB) {
        const int tx = q % CGX, ty = (q / CGX) % CGY, tz = q / (CGX * CGY);
        const size_t t = ((size_t)(z0 + tz) << (2 * logn)) + ((size_t)(y0 + ty) << logn) + (x0 + tx);
        delta[t] = (T)((double)acc[q] * scale - 1.0);
    }
}

__global__ void k_fill_i32(int *a, size_t n, int v) {
    const size_t t = (size_t)blockIdx.x * PTPB + threadIdx.x;
    if (t < n) a[t] = v;
}

template <typename T>
__global__ __launch_bounds__(PTPB) void k_counts_to_delta(const unsigned long long *counts,
                                                           size_t ncell, double scale, T *delta) {
    const size_t t = (size_t)blockIdx.x * PTPB + threadIdx.x;
    if (t >= ncell) return;
    delta[t] = (T)((double)counts[t] * scale - 1.0);
}

__global__ void k_zero_u64(unsigned long long *a, size_t n) {
    const size_t t = (size_t)blockIdx.x * PTPB + threadIdx.x;
    if (t < n) a[t] = 0ull;
}

// Force on the mesh, g = -grad(psi) by 3-point differences of the total
// potential psi = Phi_N + cphi phi (nDGP: cphi = 1/2; Kmouflage: cphi =
// beta c~), in FP64 and stored once rounded to FP32 as (gx, gy, gz, 0): the
// particle kernel then reads one 16-byte value per CIC cell instead of the
// potential at the six neighbours of each of its eight cells.  A thread owns
// one (x, y) column and marches fz planes of it, keeping psi of its own cell
// at k - 1, k and k + 1 in registers; the x and y neighbours at plane k are
// cells the adjacent threads loaded a step earlier and come from the caches.
// A block takes PTPB consecutive columns (x fastest) of one z-chunk, and each
// XCD a contiguous share of the blocks, so that the rows around a block's
// columns are loaded through the same L2.
__global__ __launch_bounds__(PTPB) void k_force(const double *__restrict__ phin,
                                                 const double *__restrict__ phi, double cphi,
                                                 float4 *__restrict__ force, int logn, int fz) {
    const int nm1 = (1 << logn) - 1;
    const size_t ncol = (size_t)1 << (2 * logn);
    const size_t ncb = (ncol + PTPB - 1) / PTPB;   // column blocks per z-chunk
    const size_t b = xcd_chunk(blockIdx.x, gridDim.x);
    const size_t col = (b % ncb) * PTPB + threadIdx.x;
    const int k0 = (int)(b / ncb) * fz;
    if (col >= ncol) return;
    const int i = (int)(col & nm1), j = (int)(col >> logn);
    auto psi = [&](int a, int bb, int k) {
        const size_t idx = ((size_t)(k & nm1) << (2 * logn)) + ((size_t)((j + bb) & nm1) << logn) +
                           ((i + a) & nm1);
        return phin[idx] + cphi * phi[idx];
    };
    double pm = psi(0, 0, k0 - 1), p0 = psi(0, 0, k0);
    for (int k = k0; k < k0 + fz; ++k) {
        const double pp = psi(0, 0, k + 1);
        const double gx = -0.5 * (psi(1, 0, k) - psi(-1, 0, k));
        const double gy = -0.5 * (psi(0, 1, k) - psi(0, -1, k));
        const double gz = -0.5 * (pp - pm);
        force[((size_t)k << (2 * logn)) + col] =
            make_float4((float)gx, (float)gy, (float)gz, 0.0f);
        pm = p0;
        p0 = pp;
    }
}

// The mesh force interpolated with the CIC weights of the particle's eight
// cells; p = damp p + g kick; x += p drift (periodic).  nDGP: damp = 1;
// Kmouflage: damp = 1 - beta (d phibar/da) da (the velocity term of
// eq:force_Kmo2).  One thread per particle, blocks in launch order.  (For
// 512^3 particles on a 1024^3 mesh, gathering the potential at the 3-point
// stencils of the eight cells -- 48 scattered loads per particle -- took
// 20 ms, bound by the cache requests.)
__global__ __launch_bounds__(PTPB) void k_kick_drift(float *__restrict__ pos,
                                                      float *__restrict__ mom, size_t np, int logn,
                                                      const float4 *__restrict__ force,
                                                      double damp, double kick, double drift) {
    const size_t t = (size_t)blockIdx.x * PTPB + threadIdx.x;
    if (t >= np) return;
    const int n = 1 << logn, nm1 = n - 1;
    double f[3];
    int i0[3];
    cic_weights(pos + 3 * t, f, i0);
    double g[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
        const double w = ((a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1])) * (c ? f[2] : 1.0 - f[2]);
        const size_t idx = ((size_t)((i0[2] + c) & nm1) << (2 * logn)) +
                           ((size_t)((i0[1] + b) & nm1) << logn) + ((i0[0] + a) & nm1);
        const float4 v = force[idx];
        g[0] += w * (double)v.x;
        g[1] += w * (double)v.y;
        g[2] += w * (double)v.z;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double pn = damp * (double)mom[3 * t + a] + g[a] * kick;
        double xn = fmod((double)pos[3 * t + a] + pn * drift, (double)n);
        if (xn < 0.0) xn += n;
        float xf = (float)xn;
        if (xf >= (float)n) xf = 0.0f;
        mom[3 * t + a] = (float)pn;
        pos[3 * t + a] = xf;
    }
}

unsigned nb(size_t threads) { return (unsigned)((threads + PTPB - 1) / PTPB); }

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// The deposit's gather form (particle lists in the CIC workspace) applies:
// no more particles than cells, 32-bit particle indices, tiles that fit.
bool cic_lists(int n_mesh, size_t np) {
    const size_t ncell = (size_t)n_mesh * n_mesh * n_mesh;
    return np <= ncell && np < ((size_t)1 << 31) && n_mesh >= CGX;
}

// counts: workspace of ncell 64-bit words (the gather form keeps its lists
// there: heads of the ncell cells, then the np links).  T: FP64 or FP32
// delta (the FP64 value rounded once).
template <typename T>
mg_status cic(int n_mesh, int n_part, const float *pos, T *delta, unsigned long long *counts,
              hipStream_t s) {
    const size_t ncell = (size_t)n_mesh * n_mesh * n_mesh;
    const size_t np = (size_t)n_part * n_part * n_part;
    const int logn = ilog2(n_mesh);
    const double scale = (1.0 / FIX_SCALE) * ((double)ncell / (double)np);
    if (cic_lists(n_mesh, np)) {
        // gather form: heads and links fit in the ncell 64-bit words
        int *head = reinterpret_cast<int *>(counts);
        int *next = head + ncell;
        k_fill_i32<<<nb(ncell), PTPB, 0, s>>>(head, ncell, -1);
        k_cic_link<<<nb(np), PTPB, 0, s>>>(pos, (int)np, logn, head, next);
        k_cic_gather<T><<<(unsigned)(ncell / CG_CELLS), PTPB, 0, s>>>(pos, logn, head, next,
                                                                     scale, delta);
        return hip_status(s, false);
    }
    k_zero_u64<<<nb(ncell), PTPB, 0, s>>>(counts, ncell);
    k_cic<<<nb(np), PTPB, 0, s>>>(pos, np, logn, counts);
    k_counts_to_delta<T><<<nb(ncell), PTPB, 0, s>>>(counts, ncell, scale, delta);
    return hip_status(s, false);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Mesh force (FP32, 16 bytes per cell, written from the start of the step's
// workspace: the CIC area and the solver workspace behind it are free once
// both potentials are solved), then kick and drift of every particle.
void potential_kick_drift(int n, int n_part, float *pos, float *mom, const double *phi_newton,
                          const double *phi, double cphi, void *ws, double damp, double kick,
                          double drift, hipStream_t stream) {
    const size_t np = (size_t)n_part * n_part * n_part;
    float4 *force = static_cast<float4 *>(ws);
    const int fz = n < 32 ? n : 32;   // planes per block
    const size_t ncb = ((size_t)n * n + PTPB - 1) / PTPB;
    k_force<<<(unsigned)(ncb * (size_t)(n / fz)), PTPB, 0, stream>>>(phi_newton, phi, cphi, force,
                                                                     ilog2(n), fz);
    k_kick_drift<<<nb(np), PTPB, 0, stream>>>(pos, mom, np, ilog2(n), force, damp, kick, drift);
}

// GPU time of the phases of a PM step (CIC, Newtonian potential, scalar
// field, total potential + kick-drift): HIP events on the step's stream at
// the phase boundaries, read after the step's final synchronisation.
struct PhaseTimer {
    static constexpr int NP = 4;
    hipEvent_t ev[NP + 1] = {};
    bool ok = true;
    hipStream_t st;
    explicit PhaseTimer(hipStream_t s) : st(s) {
        for (auto &e : ev)
            if (ok && hipEventCreate(&e) != hipSuccess) ok = false;
        if (!ok) (void)hipGetLastError();
    }
    void mark(int q) {
        if (ok && hipEventRecord(ev[q], st) != hipSuccess) ok = false;
    }
    void read(mg_stats *s) {
        for (int q = 0; q < NP; ++q) {
            float ms = 0.f;
            if (ok && hipEventElapsedTime(&ms, ev[q], ev[q + 1]) == hipSuccess)
                s->pm_ms[q] = ms;
        }
        (void)hipGetLastError();
    }
    ~PhaseTimer() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Background values of a Kmouflage step at a: lambda, phibar, d phibar/d tau
// and E = H/H0 at a and at a_h = a + da/2, from the caller's table or from
// the background solver.
struct KmoStepBg {
    double lambda, phibar, dphibar_dtau, e_a, e_half;
};

// index of x in the increasing host array t (relative match 1e-12), or -1
int table_index(const double *t, int n, double x) {
    for (int k = 0; k < n; ++k)
        if (std::fabs(t[k] - x) <= 1e-12 * std::fabs(x)) return k;
    return -1;
}

mg_status kmo_step_background(const mg_pm_kmo_params *par, KmoStepBg &b) {
    const double a = par->a, ah = a + 0.5 * par->da;
    const mg_kmo_bg_table *T = par->table;
    if (T) {
        if (T->n < 1 || !T->a || !T->hubble || !T->phibar || !T->dphibar_dtau ||
            !(T->lambda > 0.0))
            return fail(MG_ERR_ARG, "background table: n >= 1 host arrays and lambda > 0 needed");
        const int ia = table_index(T->a, T->n, a), ih = table_index(T->a, T->n, ah);
        if (ia < 0 || ih < 0)
            return fail(MG_ERR_ARG, "background table must hold a and a + da/2");
        b = {T->lambda, T->phibar[ia], T->dphibar_dtau[ia], T->hubble[ia], T->hubble[ih]};
    } else {
        // the background solver tabulates at a and a_h (one point when da = 0)
        const double at[2] = {a, ah};
        const int nt = ah > a ? 2 : 1;
        double hub[2], hdot[2], pb[2], pd[2];
        mg_kmo_bg_info info;
        const mg_status rc = mg_kmo_background(&par->bg, nt, at, hub, hdot, pb, pd, &info);
        if (rc != MG_OK) return rc;
        b = {info.lambda, pb[0], pd[0], hub[0], hub[nt - 1]};
    }
    if (!(b.e_a > 0.0) || !(b.e_half > 0.0) || !std::isfinite(b.phibar) ||
        !std::isfinite(b.dphibar_dtau))
        return fail(MG_ERR_ARG, "background values are not finite and positive");
    return MG_OK;
}

}  // namespace

extern "C" {

size_t mg_pm_workspace_bytes(int n_mesh) {
    if (!pow2(n_mesh) || n_mesh < 8 || n_mesh > 2048) return 0;
    const size_t ncell = (size_t)n_mesh * n_mesh * n_mesh;
    return align256(ncell * sizeof(unsigned long long)) +
           mg_workspace_bytes(n_mesh, MG_FP64, MG_MODEL_DGP, 0) + 256;
}

}  // extern "C"

namespace {
template <typename T>
mg_status cic_entry(int n_mesh, int n_part, const float *pos, T *delta, void *ws, size_t ws_bytes,
                    hipStream_t stream) {
    mgglam_internal::set_error("");
    if (!pow2(n_mesh) || n_mesh < 8 || n_mesh > 2048)
        return fail(MG_ERR_ARG, "n_mesh must be a power of two in [8, 2048]");
    if (n_part < 1 || n_part > 2048) return fail(MG_ERR_ARG, "n_part must be in [1, 2048]");
    if (!pos || !delta) return fail(MG_ERR_ARG, "pos and delta must be device pointers");
    const size_t need = (size_t)n_mesh * n_mesh * n_mesh * sizeof(unsigned long long);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255))
        return fail(MG_ERR_WORKSPACE, "workspace is NULL, too small or not 256-byte aligned");
    mg_status rc = cic(n_mesh, n_part, pos, delta, (unsigned long long *)ws, stream);
    if (rc != MG_OK) return rc;
    return hip_status(stream, true);
}
}  // namespace

extern "C" {

mg_status mg_cic_delta(int n_mesh, int n_part, const float *pos, double *delta, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
    return cic_entry(n_mesh, n_part, pos, delta, ws, ws_bytes, stream);
}

mg_status mg_cic_delta_f32(int n_mesh, int n_part, const float *pos, float *delta, void *ws,
                           size_t ws_bytes, hipStream_t stream) {
    return cic_entry(n_mesh, n_part, pos, delta, ws, ws_bytes, stream);
}

mg_status mg_pm_step(const mg_pm_params *par, float *pos, float *mom, double *phi,
                     double *phi_newton, double *delta_out, void *ws, size_t ws_bytes,
                     hipStream_t stream, mg_stats *stats) {
    mgglam_internal::set_error("");
    if (!par || !pos || !mom || !phi || !phi_newton || !delta_out || !stats)
        return fail(MG_ERR_ARG, "a parameter, array or stats pointer is NULL");
    const int n = par->n_mesh;
    if (!pow2(n) || n < 8 || n > 2048 || par->mg.n != n)
        return fail(MG_ERR_ARG, "n_mesh must be a power of two in [8, 2048] equal to mg.n");
    if (par->mg.no_sync)
        return fail(MG_ERR_ARG, "the PM steps wait for their phases: mg.no_sync must be 0");
    if (par->n_part < 1 || par->n_part > 2048 || !(par->a > 0.0) || !std::isfinite(par->da) ||
        !(par->omega_m > 0.0) || !(par->omega_m < 1.0))
        return fail(MG_ERR_ARG, "invalid n_part, a, da or omega_m");
    if (((uintptr_t)phi_newton | (uintptr_t)delta_out) & 15)
        return fail(MG_ERR_ARG, "phi_newton and delta_out must be 16-byte aligned");
    const size_t need = mg_pm_workspace_bytes(n);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255))
        return fail(MG_ERR_WORKSPACE, "workspace is NULL, too small or not 256-byte aligned");
    const size_t ncell = (size_t)n * n * n;
    unsigned long long *counts = (unsigned long long *)ws;
    char *solver_ws = (char *)ws + align256(ncell * sizeof(unsigned long long));
    const size_t solver_bytes = ws_bytes - align256(ncell * sizeof(unsigned long long));

    PhaseTimer T(stream);
    T.mark(0);
    mg_status rc = cic(n, par->n_part, pos, delta_out, counts, stream);
    if (rc != MG_OK) return rc;
    T.mark(1);
    // Newtonian potential, eq:GR_poisson_codeunit, by FFT with the Green's
    // function of the 7-point Laplacian (Sec. 3.1)
    rc = mgglam_internal::fft_poisson(n, 1.5 * par->omega_m / par->a, delta_out, phi_newton,
                                      solver_ws, stream);
    if (rc != MG_OK) return rc;
    T.mark(2);
    // scalar field, eq:dgp_eom_code
    mg_dgp_params dp{par->a, par->omega_m, par->h0rc};
    mg_opts so = par->mg;
    so.delta_fp32 = 0;   // the step's own FP64 density
    rc = mg_solve_dgp(&so, &dp, delta_out, phi, solver_ws, solver_bytes, stream, stats);
    if (rc < 0) return rc;
    T.mark(3);
    // leapfrog: kick with H0/adot = 1/(a E(a)) at a, drift with
    // H0/(a^2 adot) at a + da/2 (E^2 = Omega_m a^-3 + 1 - Omega_m)
    const double om = par->omega_m;
    const double a = par->a, ah = a + 0.5 * par->da;
    const double E = std::sqrt(om / (a * a * a) + 1.0 - om);
    const double Eh = std::sqrt(om / (ah * ah * ah) + 1.0 - om);
    const double kick = par->da / (a * E);
    const double drift = par->da / (ah * ah * ah * Eh);
    potential_kick_drift(n, par->n_part, pos, mom, phi_newton, phi, 0.5, counts, 1.0, kick,
                         drift, stream);
    T.mark(4);
    const mg_status hs = hip_status(stream, true);
    if (hs != MG_OK) return hs;
    T.read(stats);
    stats->pm_newton_cycles = 0;
    return rc;
}

mg_status mg_pm_step_kmouflage(const mg_pm_kmo_params *par, float *pos, float *mom, double *phi,
                               double *phi_newton, double *delta_out, void *ws, size_t ws_bytes,
                               hipStream_t stream, mg_stats *stats) {
    mgglam_internal::set_error("");
    if (!par || !pos || !mom || !phi || !phi_newton || !delta_out || !stats)
        return fail(MG_ERR_ARG, "a parameter, array or stats pointer is NULL");
    const int n = par->n_mesh;
    if (!pow2(n) || n < 8 || n > 2048 || par->mg.n != n)
        return fail(MG_ERR_ARG, "n_mesh must be a power of two in [8, 2048] equal to mg.n");
    if (par->mg.no_sync)
        return fail(MG_ERR_ARG, "the PM steps wait for their phases: mg.no_sync must be 0");
    if (par->n_part < 1 || par->n_part > 2048 || !(par->a > 0.0) || !(par->da >= 0.0) ||
        !std::isfinite(par->da) || !(par->a + 0.5 * par->da <= 1.0) || !(par->box_mpch > 0.0) ||
        !std::isfinite(par->box_mpch))
        return fail(MG_ERR_ARG, "invalid n_part, a, da (need a + da/2 <= 1) or box_mpch");
    if (((uintptr_t)phi_newton | (uintptr_t)delta_out) & 15)
        return fail(MG_ERR_ARG, "phi_newton and delta_out must be 16-byte aligned");
    const size_t need = mg_pm_workspace_bytes(n);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255))
        return fail(MG_ERR_WORKSPACE, "workspace is NULL, too small or not 256-byte aligned");
    KmoStepBg bg;
    mg_status rc = kmo_step_background(par, bg);
    if (rc != MG_OK) return rc;
    const double a = par->a, ah = a + 0.5 * par->da;
    const mg_kmo_params K{par->bg.n_k,     par->bg.k0, par->bg.beta, bg.lambda,     a,
                          par->bg.omega_m, par->box_mpch, bg.phibar, bg.dphibar_dtau};
    const size_t ncell = (size_t)n * n * n;
    unsigned long long *counts = (unsigned long long *)ws;
    char *solver_ws = (char *)ws + align256(ncell * sizeof(unsigned long long));
    const size_t solver_bytes = ws_bytes - align256(ncell * sizeof(unsigned long long));

    PhaseTimer T(stream);
    T.mark(0);
    rc = cic(n, par->n_part, pos, delta_out, counts, stream);
    if (rc != MG_OK) return rc;
    T.mark(1);
    // Newtonian potential with the rescaled particle mass,
    // eq:kmf_Poission_eqn_codeunit, by FFT
    const double A = std::exp(K.beta * K.phibar);
    rc = mgglam_internal::fft_poisson(n, 1.5 * A * K.omega_m / a, delta_out, phi_newton,
                                      solver_ws, stream);
    if (rc != MG_OK) return rc;
    T.mark(2);
    // scalar field, eq:kmf_eqn_codeunit_final
    mg_opts so = par->mg;
    so.delta_fp32 = 0;   // the step's own FP64 density
    rc = mg_solve_kmouflage(&so, &K, delta_out, phi, solver_ws, solver_bytes, stream, stats);
    if (rc < 0) return rc;
    T.mark(3);
    // eq:force_Kmo1/2: kick with H0/adot = 1/(a E(a)) and the velocity term
    // at a, drift with H0/(a^2 adot) at a + da/2.  d phibar/da follows from
    // the conformal-time derivative: da/dtau = a^2 E in units of H0.
    const double ctil = (double)n / K.box_mpch * 2997.92458;
    const double dphibar_da = bg.dphibar_dtau / (a * a * bg.e_a);
    const double kick = par->da / (a * bg.e_a);
    const double drift = par->da / (ah * ah * ah * bg.e_half);
    const double damp = 1.0 - K.beta * dphibar_da * par->da;
    potential_kick_drift(n, par->n_part, pos, mom, phi_newton, phi, K.beta * ctil, counts, damp,
                         kick, drift, stream);
    T.mark(4);
    const mg_status hs = hip_status(stream, true);
    if (hs != MG_OK) return hs;
    T.read(stats);
    stats->pm_newton_cycles = 0;
    return rc;
}

}  // extern "C"
