// Host driver and C ABI of the multigrid solver (see include/mgglam.h).
//
// The solve follows the FAS scheme of Sec. 3.2.1 of the paper: V-cycles of
// nonlinear red-black Gauss-Seidel smoothing (eq:relaxation_iteration with
// the exact per-cell solve of eq:nonlinear_GS_DGP), residual and 8-cell mean
// restriction, the coarse equation eq:general_pde_numerical_coarse with
// R(u) as initial guess, 27/9/3/1 prolongation of the correction
// (eq:solution_correction), down to a 4^3 level.  The periodic discrete
// problem is solved in bordered form: the finest right-hand side is the mean
// of L(phi), refreshed at the residual step of every cycle, and the returned
// field has zero mean.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mgglam.h"
#include "mg_adj_tiled.h"
#include "mg_adjoint.h"
#include "mg_dc.h"

using namespace mgk;

namespace {

thread_local std::string g_err;

mg_status fail(mg_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(x)                                                                  \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            g_err = std::string(#x) + ": " + hipGetErrorString(e_);                \
            return MG_ERR_HIP;                                                     \
        }                                                                          \
    } while (0)

int ilog2(long n) {
    int l = 0;
    while ((1L << l) < n) ++l;
    return l;
}
bool is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }

constexpr int MAX_LEVELS = 12;

struct Carve {
    char *base;
    size_t off;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// One level of a hierarchy with storage type R.  lin and cf (adjoint
// linearisation point and Jacobian coefficients) exist in FP64 only.
template <typename R>
struct HLevel {
    int n = 0, logn = 0;
    double h = 1.0;
    size_t half = 0;
    R *u[2] = {nullptr, nullptr};
    R *spare = nullptr;
    R *spare2 = nullptr;   // second output of the fused prolongation + pass (tiled levels)
    R *d[2] = {nullptr, nullptr};
    R *f[2] = {nullptr, nullptr};
    R *ru[2] = {nullptr, nullptr};
    double *lin[2] = {nullptr, nullptr};
    double *cf[9][2] = {};
    double *kp[2] = {nullptr, nullptr};   // nDGP adjoint on tiled levels: dK/dSigma (no cf)
    R *pb[2] = {nullptr, nullptr};   // defect correction (FP32 finest level): background
};

template <typename R>
struct Hier {
    int nlev = 0;
    HLevel<R> lv[MAX_LEVELS];
};

struct Ctx {
    Hier<double> h64;
    Hier<float> h32;
    double *partials = nullptr;
    size_t npartials = 0;
    double *scal = nullptr;
    unsigned long long *clamp = nullptr;
    hipStream_t st = nullptr;
    Mod M{};
    int nu1 = 1, nu2 = 1, nuc = 32;
    int cycle = 0;   // 0 V, 1 F, 2 W
    double kappa = 6.0;
    int adj_model = MODEL_DGP;   // model of the adjoint's Jacobian (tiled kernel dispatch)
    bool profile = false;
    // enqueue only (mg_opts.no_sync): no scalar is read back, nothing waits
    bool no_sync = false;
    std::vector<hipEvent_t> ev;
    int ev_used = 0;
    double pass_ms = 0.0;
    int pass_count = 0;
    // per-level timing (profile): events bracketing each level's segments
    struct Segment {
        int level, e0, e1;
    };
    std::vector<hipEvent_t> lev_ev;
    std::vector<Segment> segs;
    int lev_used = 0;
    double level_ms[MG_LEVELS] = {};
    // Early read of the cycle's stopping scalars: they are final once the
    // finest in-cycle residual has been reduced, so they are copied to pinned
    // host memory at that point and the host decides on the next cycle while
    // the coarse levels and the post-smoothing still run.
    double *pin = nullptr;
    hipEvent_t pin_ev = nullptr;
    bool pin_pending = false;
    Ctx() = default;
    Ctx(const Ctx &) = delete;
    Ctx &operator=(const Ctx &) = delete;
    ~Ctx() {
        // an early copy still in flight (a call that ended on an error) must
        // land before the next call on this thread reuses the pinned buffer
        if (pin_pending) (void)hipEventSynchronize(pin_ev);
        if (pin_ev) (void)hipEventDestroy(pin_ev);
    }
};

// Pinned host buffer for the per-cycle scalars, one per host thread (calls on
// one thread never overlap), allocated on first use and kept until the
// process ends.  nullptr if the allocation fails: the solver then reads the
// scalars after the whole cycle.
double *pinned_scalars() {
    thread_local double *p = nullptr;
    if (!p) {
        void *q = nullptr;
        if (hipHostMalloc(&q, sizeof(double) * S_NSCAL, hipHostMallocDefault) == hipSuccess)
            p = static_cast<double *>(q);
        else
            (void)hipGetLastError();
    }
    return p;
}

void arm_early_read(Ctx &C) {
    C.pin = pinned_scalars();
    if (C.pin && hipEventCreateWithFlags(&C.pin_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        C.pin_ev = nullptr;
    }
}

template <typename R>
Hier<R> &hier(Ctx &C);
template <>
Hier<double> &hier<double>(Ctx &C) { return C.h64; }
template <>
Hier<float> &hier<float>(Ctx &C) { return C.h32; }

// dc_fine: the finest level also holds the right-hand side array and the
// frozen background of the defect-correction cycles.  rc (nDGP adjoint):
// levels >= 128^3 keep dK/dSigma instead of the coefficient arrays (the
// tiled adjoint kernels rebuild the coefficients from it).
template <typename R>
void layout_hier(Hier<R> &Hh, Carve &cv, int n, bool adjoint, bool sym_coefs,
                 bool dc_fine = false, bool rc = false) {
    int L = 0;
    for (int m = n; m >= 4; m >>= 1) {
        HLevel<R> &H = Hh.lv[L];
        H.n = m;
        H.logn = ilog2(m);
        H.h = (double)n / m;
        H.half = (size_t)m * m * m / 2;
        H.u[0] = cv.take<R>(H.half);
        H.u[1] = cv.take<R>(H.half);
        H.spare = cv.take<R>(H.half);
        if (!adjoint && m >= 128) H.spare2 = cv.take<R>(H.half);
        H.d[0] = cv.take<R>(H.half);
        H.d[1] = cv.take<R>(H.half);
        if (L > 0 || adjoint || dc_fine) {
            H.f[0] = cv.take<R>(H.half);
            H.f[1] = cv.take<R>(H.half);
        }
        if (L == 0 && dc_fine) {
            H.pb[0] = cv.take<R>(H.half);
            H.pb[1] = cv.take<R>(H.half);
        }
        if (L > 0) {
            H.ru[0] = cv.take<R>(H.half);
            H.ru[1] = cv.take<R>(H.half);
        }
        if (adjoint && rc && m >= 128) {
            H.lin[0] = cv.take<double>(H.half);
            H.lin[1] = cv.take<double>(H.half);
            H.kp[0] = cv.take<double>(H.half);
            H.kp[1] = cv.take<double>(H.half);
        } else if (adjoint) {
            H.lin[0] = cv.take<double>(H.half);
            H.lin[1] = cv.take<double>(H.half);
            // nDGP and Poisson: the minus face arrays alias the plus ones
            for (int q = 0; q < 9; ++q)
                for (int c = 0; c < 2; ++c)
                    H.cf[q][c] = (sym_coefs && q < 6 && (q & 1)) ? H.cf[q - 1][c]
                                                                 : cv.take<double>(H.half);
        }
        ++L;
    }
    Hh.nlev = L;
}

// Lay the workspace out (base == nullptr: only measure): the FP64 hierarchy
// unless precision is MG_FP32, the FP32 one unless it is MG_FP64.
void layout(Ctx &C, Carve &cv, int n, bool adjoint, int precision, bool sym_coefs = false,
            bool rc = false) {
    if (precision != MG_FP32) layout_hier(C.h64, cv, n, adjoint, sym_coefs, false, rc);
    if (precision != MG_FP64)
        layout_hier(C.h32, cv, n, false, false, precision == MG_MIXED_DC);
    C.npartials = std::max<size_t>((size_t)n * n * n / TPB + 1, 1024);
    C.partials = cv.take<double>(2 * C.npartials);
    C.scal = cv.take<double>(S_NSCAL);
    C.clamp = cv.take<unsigned long long>(4);
}

template <typename R>
LvlT<R> view(const HLevel<R> &H, bool with_f) {
    LvlT<R> L;
    L.u0 = H.u[0];
    L.u1 = H.u[1];
    L.d0 = H.d[0];
    L.d1 = H.d[1];
    L.f0 = with_f ? H.f[0] : nullptr;
    L.f1 = with_f ? H.f[1] : nullptr;
    L.n = H.n;
    L.logn = H.logn;
    L.lognh = H.logn - 1;
    const double h2 = H.h * H.h, h4 = h2 * h2;
    L.h2 = h2;
    L.c3h4 = 1.0 / (3.0 * h4);
    L.c8h4 = 1.0 / (8.0 * h4);
    L.c12h4 = 1.0 / (12.0 * h4);
    L.c4h2 = 1.0 / (4.0 * h2);
    return L;
}

// The adjoint's face coefficients dK/dphi at x+ and x- (y, z) are equal for
// the nDGP and Poisson terms (both depend on phi through second differences
// only): point the minus arrays at the plus ones, so k_adj_coefs writes 6
// arrays instead of 9 and an adjoint pass reads 3 face arrays instead of 6.
template <typename R>
void alias_face_coefs(HLevel<R> &H, bool symmetric) {
    if (!symmetric || H.kp[0]) return;
    for (int q = 1; q < 6; q += 2)
        for (int c = 0; c < 2; ++c) H.cf[q][c] = H.cf[q - 1][c];
}

template <typename R>
Coefs coefs(const HLevel<R> &H) {
    Coefs C;
    for (int q = 0; q < 9; ++q)
        for (int c = 0; c < 2; ++c) C.c[q][c] = H.cf[q][c];
    return C;
}

unsigned nblocks(size_t threads) { return (unsigned)((threads + TPB - 1) / TPB); }

// ------------------------------------------------------------ kernel launchers
// Levels with >= 128 cells per side use the LDS-tiled kernels (64 packed
// columns x 8 rows per tile); smaller levels and the adjoint use the
// one-thread-per-cell kernels.

bool tiled_level(int n) { return n >= 128; }

// The tiled kernels implement the closed-form update only.
constexpr bool tiled_op(int OP) { return OP != OP_ADJ; }

// z-planes per block: the deepest chunk (4 .. kzmax planes) that still gives
// a launch at least 4096 blocks.  Deeper chunks re-read fewer z-halo planes;
// at 1024^3 (128 planes, 8192 blocks per pass) the V-cycle is 1% faster than
// with 64.  Kernels whose chunks count coarse planes (two fine planes each)
// keep at most 64: the 1024^3 residual + restriction took 4.43 ms with 128
// (4096 blocks) against 4.31 ms with 64.
TileGeom tile_geom(int n, int planes, int kzmax = 128) {
    TileGeom G;
    G.ntx = (n / 2) / TX;
    G.nty = n / TY;
    const long per = (long)G.ntx * G.nty;
    int kz = kzmax;
    while (kz > 4 && (long)planes * per / kz < 4096) kz >>= 1;
    while (planes % kz) kz >>= 1;
    G.kz = kz;
    return G;
}

unsigned tile_blocks(const TileGeom &G, int planes) {
    return (unsigned)((long)G.ntx * G.nty * (planes / G.kz));
}

constexpr int fwd_op(int OP) { return OP == OP_ADJ ? OP_DGP : OP; }

template <int OP, typename R>
void launch_pass(const Mod &M, const LvlT<R> &L, const Coefs &Cf, int c, R *out, const double *fptr,
                 double fs, unsigned long long *clamp, hipStream_t st) {
    if (tiled_op(OP) && tiled_level(L.n)) {
        const TileGeom G = tile_geom(L.n, L.n);
        k_pass_tiled<fwd_op(OP), R><<<tile_blocks(G, L.n), TPB, 0, st>>>(M, L, c, out, fptr, fs,
                                                                         clamp, G);
    } else {
        const size_t half = (size_t)L.n * L.n * L.n / 2;
        k_pass<OP, R><<<nblocks(half), TPB, 0, st>>>(M, L, Cf, c, out, fptr, fs, clamp);
    }
}

template <int OP, bool REDUCE, typename R>
unsigned launch_resid_restrict(const Mod &M, const LvlT<R> &L, const Coefs &Cf, const double *fptr,
                               double fs, R *ru0, R *ru1, R *rd0, R *rd1, double *partials,
                               unsigned long long *clamp, hipStream_t st) {
    if (tiled_op(OP) && tiled_level(L.n)) {
        const TileGeom G = tile_geom(L.n, L.n / 2, 64);
        const unsigned nb = tile_blocks(G, L.n / 2);
        if (L.f0)
            k_resid_restrict_tiled<fwd_op(OP), REDUCE, true, R><<<nb, TPB, 0, st>>>(
                M, L, fptr, fs, ru0, ru1, rd0, rd1, partials, clamp, G);
        else
            k_resid_restrict_tiled<fwd_op(OP), REDUCE, false, R><<<nb, TPB, 0, st>>>(
                M, L, fptr, fs, ru0, ru1, rd0, rd1, partials, clamp, G);
        return nb;
    }
    const size_t ncoarse = (size_t)L.n * L.n * L.n / 8;
    const unsigned nb = nblocks(ncoarse);
    k_resid_restrict<OP, REDUCE, R><<<nb, TPB, 0, st>>>(M, L, Cf, fptr, fs, ru0, ru1, rd0, rd1,
                                                        partials, clamp);
    return nb;
}

template <typename R>
void launch_prolong(R *f0, R *f1, int logn, const R *uc0, const R *uc1, const R *rc0,
                    const R *rc1, hipStream_t st) {
    const int n = 1 << logn;
    if (tiled_level(n)) {
        const TileGeom G = tile_geom(n, n / 2, 64);
        k_prolong_tiled<R><<<tile_blocks(G, n / 2), TPB, 0, st>>>(f0, f1, logn, uc0, uc1, rc0, rc1,
                                                                 G);
    } else {
        const size_t cells = (size_t)n * n * n;
        k_prolong<R><<<nblocks(cells), TPB, 0, st>>>(f0, f1, logn, uc0, uc1, rc0, rc1);
    }
}

AdjLevel adj_level(const HLevel<double> &H, const double *u0, const double *u1) {
    AdjLevel A;
    A.u0 = u0;
    A.u1 = u1;
    for (int q = 0; q < 9; ++q)
        for (int c = 0; c < 2; ++c) A.c[q][c] = H.cf[q][c];
    for (int c = 0; c < 2; ++c) {
        A.lin[c] = H.lin[c];
        A.kp[c] = H.kp[c];
    }
    A.f0 = H.f[0];
    A.f1 = H.f[1];
    A.n = H.n;
    A.logn = H.logn;
    A.lognh = H.logn - 1;
    A.h2 = H.h * H.h;
    const double h4 = A.h2 * A.h2;
    A.c3h4 = 1.0 / (3.0 * h4);
    A.c8h4 = 1.0 / (8.0 * h4);
    return A;
}

// Threads per block of the tiled adjoint kernels (256: two rows per thread).
#ifndef MG_ADJ_NT
#define MG_ADJ_NT 512
#endif
constexpr int ADJ_NT = MG_ADJ_NT;

// One colour launch of the tiled adjoint kernel (levels >= 128^3); returns
// the number of blocks (block sums land in partials[0 .. 2 nb)).
template <int MODE, bool REDUCE>
unsigned launch_adj_tiled(int model, const AdjLevel &A, int c, double *out, double *out2,
                          const double *fptr, double fscale, double *ru0, double *ru1,
                          double *rd0, double *rd1, double *partials, hipStream_t st) {
    const TileGeom G = tile_geom(A.n, A.n, 64);
    const unsigned nb = tile_blocks(G, A.n);
    switch (model) {
        case MODEL_KMO:
            k_adj_tiled<ADJ_NT, false, true, MODE, REDUCE><<<nb, ADJ_NT, 0, st>>>(
                A, c, out, out2, fptr, fscale, ru0, ru1, rd0, rd1, partials, G);
            break;
        case MODEL_POISSON:
            k_adj_tiled<ADJ_NT, true, false, MODE, REDUCE><<<nb, ADJ_NT, 0, st>>>(
                A, c, out, out2, fptr, fscale, ru0, ru1, rd0, rd1, partials, G);
            break;
        default:   // nDGP: coefficients rebuilt from dK/dSigma and phi
            k_adj_tiled<ADJ_NT, true, true, MODE, REDUCE, true><<<nb, ADJ_NT, 0, st>>>(
                A, c, out, out2, fptr, fscale, ru0, ru1, rd0, rd1, partials, G);
            break;
    }
    return nb;
}

// ---------------------------------------------------------------- model set-up

bool setup_dgp(const mg_dgp_params *p, Mod &M) {
    if (!(p->a > 0.0) || !(p->omega_m > 0.0) || !(p->omega_m < 1.0) || !(p->h0rc > 0.0) ||
        !std::isfinite(p->a) || !std::isfinite(p->h0rc))
        return false;
    // eq:beta_dgp with the LCDM H(a) of eq:H_lcdm; Omega_rc = 1/(4 R_c^2)
    const double a3 = p->a * p->a * p->a;
    const double om = p->omega_m, ol = 1.0 - om;
    const double orc = 1.0 / (4.0 * p->h0rc * p->h0rc);
    const double beta = 1.0 + (om / a3 + 2.0 * ol) / (2.0 * std::sqrt(orc * (om / a3 + ol)));
    M = Mod{};
    M.alpha = 3.0 * beta * p->a * p->a / (p->h0rc * p->h0rc);
    M.sgn = M.alpha >= 0.0 ? 1.0 : -1.0;
    M.s = M.alpha / beta * om / p->a;
    return true;
}

bool setup_kmo(const mg_kmo_params *p, int n, Mod &M) {
    if (p->n_k < 2 || p->n_k > 8 || !(p->k0 >= 0.0) || !(p->lambda > 0.0) || !(p->a > 0.0) ||
        !(p->omega_m > 0.0) || !(p->box_mpch > 0.0) || !std::isfinite(p->beta) ||
        !std::isfinite(p->phibar) || !std::isfinite(p->dphibar_dtau_over_h0))
        return false;
    const double x0 = 1.0 / (2.0 * p->a * p->a * p->lambda * p->lambda);
    const double b = p->dphibar_dtau_over_h0 * p->dphibar_dtau_over_h0;
    double xp = 1.0, bp = 1.0;
    for (int q = 0; q < p->n_k - 1; ++q) {
        xp *= x0;
        bp *= b;
    }
    const double gamma = p->n_k * p->k0 * xp;
    M = Mod{};
    M.ctil = (double)n / p->box_mpch * 2997.92458;
    M.c0 = 1.0 + gamma * bp;
    M.a1 = (2.0 * p->n_k + 1.0) * gamma / 3.0;
    M.b2 = -2.0 * M.ctil * (p->n_k - 1) * gamma;
    M.src = 3.0 * p->beta * std::exp(p->beta * p->phibar) * p->omega_m / p->a;
    M.nk = p->n_k;
    return true;
}

mg_status check_opts(const mg_opts *o) {
    if (!o) return fail(MG_ERR_ARG, "opts is NULL");
    if (!is_pow2(o->n) || o->n < 8 || o->n > 2048)
        return fail(MG_ERR_ARG, "opts.n must be a power of two in [8, 2048]");
    if (o->max_cycles < 0 || o->max_cycles > 100000)
        return fail(MG_ERR_ARG, "opts.max_cycles must be in [0, 100000]");
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(MG_ERR_ARG, "opts.tol must be >= 0");
    if (o->nu_pre < 0 || o->nu_post < 0 || o->nu_coarse < 1 || o->nu_pre > 64 || o->nu_post > 64 ||
        o->nu_coarse > 4096)
        return fail(MG_ERR_ARG, "sweep counts out of range");
    if (o->precision != MG_FP64 && o->precision != MG_MIXED && o->precision != MG_FP32 &&
        o->precision != MG_MIXED_DC)
        return fail(MG_ERR_ARG,
                    "opts.precision must be MG_FP64, MG_MIXED, MG_FP32 or MG_MIXED_DC");
    if (o->precision == MG_MIXED_DC && o->n < 128)
        return fail(MG_ERR_ARG, "MG_MIXED_DC needs opts.n >= 128");
    if (o->cycle < MG_CYCLE_V || o->cycle > MG_CYCLE_W)
        return fail(MG_ERR_ARG, "opts.cycle must be MG_CYCLE_V, MG_CYCLE_F or MG_CYCLE_W");
    if (o->delta_fp32 != 0 && o->delta_fp32 != 1)
        return fail(MG_ERR_ARG, "opts.delta_fp32 must be 0 (FP64 delta) or 1 (FP32 delta)");
    if (o->no_sync != 0 && o->no_sync != 1) return fail(MG_ERR_ARG, "opts.no_sync must be 0 or 1");
    if (o->no_sync && (o->tol != 0.0 || o->profile || o->precision != MG_FP64))
        return fail(MG_ERR_ARG, "opts.no_sync = 1 needs tol = 0, profile = 0 and MG_FP64");
    return MG_OK;
}

// ---------------------------------------------------------------- V-cycle

struct PhaseResult {
    int status = MG_NOT_CONVERGED;
    int cycles = 0;
    double eps0 = 0.0, eps = 0.0;
};

template <int OP, typename R>
struct Solver {
    Ctx &C;
    Hier<R> &Hh;
    explicit Solver(Ctx &c) : C(c), Hh(hier<R>(c)) {}

    void mean_of(R *a0, R *a1, size_t half) {
        const unsigned nb = (unsigned)std::min<size_t>(nblocks(half), 2048);
        k_sum<R><<<nb, TPB, 0, C.st>>>(a0, a1, half, C.partials);
        k_finalize<<<1, 1024, 0, C.st>>>(C.partials, nb, (double)(2 * half), C.scal, 1, 0.0);
    }

    // The adjoint on levels >= 128^3 runs the tiled adjoint kernels; on a
    // tiled finest level the mean of mu that the bordered equation needs is
    // kept from the colour sums that every kernel writing mu reports.
    static constexpr bool ADJ = OP == OP_ADJ;
    bool adj_tiled(int l) const { return ADJ && tiled_level(Hh.lv[l].n); }

    void pass(int l, int c) {
        HLevel<R> &H = Hh.lv[l];
        const double *fptr = nullptr;
        double fs = 0.0;
        if (l == 0) {
            if (OP == OP_ADJ) {
                if (!adj_tiled(0)) mean_of(H.u[0], H.u[1], H.half);
                fptr = C.scal + S_MEAN;
                fs = C.kappa;
            } else {
                fptr = C.scal + S_MU;
                fs = 1.0;
            }
        }
        const bool timed = C.profile && l == 0 && C.ev_used + 2 <= (int)C.ev.size();
        if (timed) (void)hipEventRecord(C.ev[C.ev_used], C.st);
        if constexpr (ADJ) {
            if (adj_tiled(l)) {
                const AdjLevel A = adj_level(H, H.u[0], H.u[1]);
                double *sp = reinterpret_cast<double *>(H.spare);
                if (l == 0) {
                    const unsigned nb = launch_adj_tiled<ADJ_PASS, true>(
                        C.adj_model, A, c, sp, nullptr, fptr, fs, nullptr, nullptr, nullptr,
                        nullptr, C.partials, C.st);
                    k_finalize<<<1, 1024, 0, C.st>>>(C.partials, nb, (double)H.n * H.n * H.n,
                                                     C.scal, 3, 0.0, c);
                } else {
                    launch_adj_tiled<ADJ_PASS, false>(C.adj_model, A, c, sp, nullptr, fptr, fs,
                                                      nullptr, nullptr, nullptr, nullptr, nullptr,
                                                      C.st);
                }
                if (timed) {
                    (void)hipEventRecord(C.ev[C.ev_used + 1], C.st);
                    C.ev_used += 2;
                }
                std::swap(H.u[c], H.spare);
                return;
            }
        }
        launch_pass<OP, R>(C.M, view(H, l > 0 || OP == OP_ADJ), coefs(H), c, H.spare, fptr, fs,
                           C.clamp, C.st);
        if (timed) {
            (void)hipEventRecord(C.ev[C.ev_used + 1], C.st);
            C.ev_used += 2;
        }
        std::swap(H.u[c], H.spare);
    }

    void sweep(int l) {
        pass(l, 0);
        pass(l, 1);
    }

    // residual (+ statistics on the finest level) and restriction into l+1
    void resid_restrict(int l) {
        HLevel<R> &H = Hh.lv[l], &Hc = Hh.lv[l + 1];
        const bool with_f = l > 0 || OP == OP_ADJ;
        const double *fptr = (l == 0 && OP != OP_ADJ) ? C.scal + S_MU : nullptr;
        if constexpr (ADJ) {
            if (adj_tiled(l)) {
                // colour 0 writes the raw sums of its children, colour 1
                // completes the 8-cell means; the finest level reduces r
                const AdjLevel A = adj_level(H, H.u[0], H.u[1]);
                double *q[4] = {(double *)Hc.ru[0], (double *)Hc.ru[1], (double *)Hc.f[0],
                                (double *)Hc.f[1]};
                if (l == 0) {
                    const unsigned nb = launch_adj_tiled<ADJ_RESID, true>(
                        C.adj_model, A, 0, nullptr, nullptr, nullptr, 0.0, q[0], q[1], q[2],
                        q[3], C.partials, C.st);
                    launch_adj_tiled<ADJ_RESID, true>(C.adj_model, A, 1, nullptr, nullptr,
                                                      nullptr, 0.0, q[0], q[1], q[2], q[3],
                                                      C.partials + 2 * nb, C.st);
                    k_finalize<<<1, 1024, 0, C.st>>>(C.partials, 2 * nb,
                                                     (double)H.n * H.n * H.n, C.scal, 2, C.kappa);
                } else {
                    for (int c = 0; c < 2; ++c)
                        launch_adj_tiled<ADJ_RESID, false>(C.adj_model, A, c, nullptr, nullptr,
                                                           nullptr, 0.0, q[0], q[1], q[2], q[3],
                                                           nullptr, C.st);
                }
                return;
            }
        }
        if (l == 0) {
            if (OP == OP_ADJ) mean_of(H.u[0], H.u[1], H.half);
            const unsigned nb = launch_resid_restrict<OP, true, R>(
                C.M, view(H, with_f), coefs(H), fptr, 1.0, Hc.ru[0], Hc.ru[1], Hc.f[0], Hc.f[1],
                C.partials, C.clamp, C.st);
            k_finalize<<<1, 1024, 0, C.st>>>(C.partials, nb, (double)H.n * H.n * H.n, C.scal,
                                             OP == OP_ADJ ? 2 : 0, C.kappa);
        } else {
            launch_resid_restrict<OP, false, R>(C.M, view(H, with_f), coefs(H), fptr, 1.0,
                                                Hc.ru[0], Hc.ru[1], Hc.f[0], Hc.f[1], C.partials,
                                                C.clamp, C.st);
        }
    }

    // mu from a sample of the finest residual before a call's first full
    // evaluation (k_mu_estimate); the adjoint's finest right-hand side is
    // an array and needs none
    void seed_mu() {
        if constexpr (!ADJ) {
            HLevel<R> &F = Hh.lv[0];
            k_mu_estimate<OP, R><<<1, 64, 0, C.st>>>(C.M, view(F, false), coefs(F),
                                                     C.scal + S_MU);
        }
    }

    void coarse_source(int lc) {
        HLevel<R> &Hc = Hh.lv[lc];
        LvlT<R> L = view(Hc, false);
        L.u0 = Hc.ru[0];
        L.u1 = Hc.ru[1];
        const double *shift = (lc == 1 && OP != OP_ADJ) ? C.scal + S_SHIFT : nullptr;
        if constexpr (ADJ) {
            if (adj_tiled(lc)) {
                const AdjLevel A = adj_level(Hc, Hc.ru[0], Hc.ru[1]);
                for (int c = 0; c < 2; ++c)
                    launch_adj_tiled<ADJ_CSRC, false>(C.adj_model, A, c, (double *)Hc.f[c],
                                                      (double *)Hc.u[c], nullptr, 0.0, nullptr,
                                                      nullptr, nullptr, nullptr, nullptr, C.st);
                return;
            }
        }
        if (tiled_op(OP) && tiled_level(Hc.n)) {
            const TileGeom G = tile_geom(Hc.n, Hc.n);
            k_coarse_source_tiled<fwd_op(OP), R><<<tile_blocks(G, Hc.n), TPB, 0, C.st>>>(
                C.M, L, Hc.f[0], Hc.f[1], Hc.u[0], Hc.u[1], shift, G);
        } else {
            k_coarse_source<OP, R><<<nblocks(2 * Hc.half), TPB, 0, C.st>>>(
                C.M, L, coefs(Hc), Hc.f[0], Hc.f[1], Hc.u[0], Hc.u[1], shift);
        }
    }

    void prolong(int l) {
        HLevel<R> &H = Hh.lv[l], &Hc = Hh.lv[l + 1];
        if (l == 0 && adj_tiled(0)) {
            // the colour sums of the corrected finest field
            const TileGeom G = tile_geom(H.n, H.n / 2, 64);
            const unsigned nb = tile_blocks(G, H.n / 2);
            k_prolong_tiled<R, true><<<nb, TPB, 0, C.st>>>(H.u[0], H.u[1], H.logn, Hc.u[0],
                                                          Hc.u[1], Hc.ru[0], Hc.ru[1], G,
                                                          C.partials);
            k_finalize<<<1, 1024, 0, C.st>>>(C.partials, nb, (double)H.n * H.n * H.n, C.scal, 4,
                                             0.0);
            return;
        }
        launch_prolong<R>(H.u[0], H.u[1], H.logn, Hc.u[0], Hc.u[1], Hc.ru[0], Hc.ru[1], C.st);
    }

    // prolongation fused with the colour-0 pass of the first post-sweep
    bool fused_prolong(int l) const {
        return tiled_op(OP) && C.nu2 >= 1 && Hh.lv[l].spare2 && tiled_level(Hh.lv[l].n);
    }
    void prolong_pass0(int l) {
        HLevel<R> &H = Hh.lv[l], &Hc = Hh.lv[l + 1];
        const TileGeom G = tile_geom(H.n, H.n);
        k_prolong_pass_tiled<fwd_op(OP), R><<<tile_blocks(G, H.n), TPB, 0, C.st>>>(
            C.M, view(H, l > 0), H.spare, H.spare2, Hc.u[0], Hc.u[1], Hc.ru[0], Hc.ru[1],
            l == 0 ? C.scal + S_MU : nullptr, 1.0, C.clamp, G);
        std::swap(H.u[0], H.spare);
        std::swap(H.u[1], H.spare2);
    }

    template <int NL>
    void launch_tail(const TailArgs<R> &A, size_t lds) {
        // once per instantiation and process (thread-safe); a failure stays
        // in the HIP error state and is reported with the solve's launches
        static std::once_flag once;
        std::call_once(once, [] {
            (void)hipFuncSetAttribute((const void *)k_tail<OP, NL, R>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        });
        k_tail<OP, NL, R><<<1, TAIL_THREADS, lds, C.st>>>(C.M, A);
    }

    // Levels l.. (all <= 16^3, l >= 1) in one single-workgroup launch that
    // runs a cycle of the given type on them.
    void tail(int l, int type) {
        TailArgs<R> A;
        A.nlev = Hh.nlev - l;
        A.nu1 = C.nu1;
        A.nu2 = C.nu2;
        A.nuc = C.nuc;
        A.cycle = type;
        for (int q = 0; q < A.nlev; ++q) {
            HLevel<R> &H = Hh.lv[l + q];
            A.lv[q].L = view(H, true);
            A.lv[q].ru0 = H.ru[0];
            A.lv[q].ru1 = H.ru[1];
            A.cf[q] = coefs(H);
        }
        const size_t lds = sizeof(R) * tail_lds_elems(Hh.lv[l].logn, A.nlev);
        switch (A.nlev) {
            case 1: launch_tail<1>(A, lds); break;
            case 2: launch_tail<2>(A, lds); break;
            default: launch_tail<3>(A, lds); break;
        }
    }

    int tail_start() const {
        for (int l = 1; l < Hh.nlev; ++l)
            if (Hh.lv[l].n <= TAIL_MAX_N && Hh.nlev - l <= TAIL_MAX_LEVELS) return l;
        return Hh.nlev;
    }

    // Profile mode: record an event on the stream (index, or -1), and a
    // segment of level l's work between two of them.
    int mark() {
        if (!C.profile) return -1;
        if (C.lev_used == (int)C.lev_ev.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            C.lev_ev.push_back(e);
        }
        (void)hipEventRecord(C.lev_ev[C.lev_used], C.st);
        return C.lev_used++;
    }
    void segment(int l, int e0, int e1) {
        if (e0 >= 0 && e1 >= 0) C.segs.push_back({std::min(l, MG_LEVELS - 1), e0, e1});
    }

    // One cycle of type 0 (V), 1 (F: a coarse F-cycle then a coarse V-cycle)
    // or 2 (W: two coarse W-cycles) on level l (Sec. 3.2.1).
    void cycle(int l, int type) {
        const int e0 = mark();
        if (l > 0 && l == tail_start()) {
            tail(l, type);
            segment(l, e0, mark());
            return;
        }
        if (l == Hh.nlev - 1) {
            for (int s = 0; s < C.nuc; ++s) sweep(l);
            segment(l, e0, mark());
            return;
        }
        for (int s = 0; s < C.nu1; ++s) sweep(l);
        resid_restrict(l);
        if (l == 0) copy_scal_early();
        coarse_source(l + 1);
        segment(l, e0, mark());
        if (type == 2) {
            cycle(l + 1, 2);
            cycle(l + 1, 2);
        } else if (type == 1) {
            cycle(l + 1, 1);
            cycle(l + 1, 0);
        } else {
            cycle(l + 1, 0);
        }
        const int e2 = mark();
        if (fused_prolong(l)) {
            prolong_pass0(l);
            pass(l, 1);
            for (int s = 1; s < C.nu2; ++s) sweep(l);
        } else {
            prolong(l);
            for (int s = 0; s < C.nu2; ++s) sweep(l);
        }
        segment(l, e2, mark());
    }

    // Scalars of the finest in-cycle residual into pinned memory (not in
    // profile mode, whose event timings need the whole cycle).  No kernel
    // later in the cycle writes mu or eps^2.
    void copy_scal_early() {
        if (C.profile || !C.pin || !C.pin_ev) return;
        if (hipMemcpyAsync(C.pin, C.scal, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost,
                           C.st) == hipSuccess &&
            hipEventRecord(C.pin_ev, C.st) == hipSuccess)
            C.pin_pending = true;
    }

    mg_status read_scal(double *hs) {
        HIPCHK(hipGetLastError());
        if (C.pin_pending) {
            C.pin_pending = false;
            HIPCHK(hipEventSynchronize(C.pin_ev));
            std::memcpy(hs, C.pin, sizeof(double) * S_NSCAL);
            return MG_OK;
        }
        HIPCHK(hipMemcpyAsync(hs, C.scal, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, C.st));
        HIPCHK(hipStreamSynchronize(C.st));
        if (C.profile) {
            for (int q = 0; q + 1 < C.ev_used; q += 2) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, C.ev[q], C.ev[q + 1]));
                C.pass_ms += ms;
                ++C.pass_count;
            }
            C.ev_used = 0;
            for (const auto &g : C.segs) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, C.lev_ev[g.e0], C.lev_ev[g.e1]));
                C.level_ms[g.level] += ms;
            }
            C.segs.clear();
            C.lev_used = 0;
        }
        return MG_OK;
    }

    // Cycle loop.  The finest field and right-hand side are set up.  Runs
    // until the residual is <= tol (confirmed by a residual evaluation of the
    // post-smoothed field), max_cycles, or -- with stall > 0 -- until a cycle
    // reduces the in-cycle residual by less than the factor stall.  Cycle
    // residuals go to hist[hist0 ...].  With eps_in >= 0 the initial residual
    // evaluation is skipped (eps_in stands for it and mu keeps its value);
    // with confirm_stall false a stall ends the phase without a final
    // residual evaluation (eps is then the last in-cycle residual).
    mg_status run(double tol, int max_cycles, double stall, mg_stats *st, int hist0,
                  PhaseResult &pr, double eps_in = -1.0, bool confirm_stall = true) {
        if (C.no_sync) {
            // enqueue only (tol = 0): the launches of the synchronous solve
            // below for tol = 0 -- initial residual, max_cycles cycles, final
            // residual -- in the same order, with no scalar read back
            if (eps_in < 0.0) {
                seed_mu();
                resid_restrict(0);
            }
            for (int c = 0; c < max_cycles; ++c) cycle(0, C.cycle);
            if (max_cycles > 0) resid_restrict(0);
            pr.status = MG_NOT_CONVERGED;
            pr.cycles = max_cycles;
            pr.eps0 = pr.eps = NAN;
            st->lambda = NAN;
            return MG_OK;
        }
        double hs[S_NSCAL] = {};
        mg_status rc;
        double eps = eps_in;
        if (eps_in < 0.0) {
            seed_mu();
            resid_restrict(0);
            if ((rc = read_scal(hs)) != MG_OK) return rc;
            eps = std::sqrt(hs[S_EPS2]);
        }
        pr.eps0 = eps;
        pr.eps = eps;
        if (!std::isfinite(eps)) {
            pr.status = MG_ERR_NONFINITE;
            fail(MG_ERR_NONFINITE, "initial residual is not finite");
            return MG_OK;
        }
        int status = (eps <= tol) ? MG_OK : MG_NOT_CONVERGED;
        double best = eps, prev = INFINITY;   // stall test compares consecutive cycles
        int cyc = 0;
        if (status != MG_OK) {
            for (cyc = 1; cyc <= max_cycles; ++cyc) {
                cycle(0, C.cycle);
                if ((rc = read_scal(hs)) != MG_OK) return rc;
                const double em = std::sqrt(hs[S_EPS2]);
                if (hist0 + cyc - 1 < MG_HIST) st->eps_hist[hist0 + cyc - 1] = em;
                if (!std::isfinite(em)) {
                    status = MG_ERR_NONFINITE;
                    break;
                }
                if (em > 1e3 * best) {
                    status = MG_ERR_DIVERGED;
                    break;
                }
                if (em < best) best = em;
                const bool stalled = stall > 0.0 && em > stall * prev;
                prev = em;
                if (stalled && !confirm_stall && em > tol) {
                    eps = em;
                    break;
                }
                if (em <= tol || cyc == max_cycles || stalled) {
                    resid_restrict(0);
                    if ((rc = read_scal(hs)) != MG_OK) return rc;
                    eps = std::sqrt(hs[S_EPS2]);
                    if (eps <= tol) {
                        status = MG_OK;
                        break;
                    }
                    if (stalled) break;
                }
            }
            if (cyc > max_cycles) cyc = max_cycles;
        }
        pr.status = status;
        pr.cycles = cyc;
        pr.eps = eps;
        st->lambda = -hs[S_MU];
        return MG_OK;
    }
};

// The caller's density: n^3 values in natural order, FP64 or FP32
// (mg_opts.delta_fp32).
struct DeltaIn {
    const void *p;
    bool f32;
};

// Pack delta into the finest level of hierarchy R and restrict it down.
template <typename R>
void density_hierarchy(Ctx &C, DeltaIn delta) {
    Hier<R> &Hh = hier<R>(C);
    HLevel<R> &F = Hh.lv[0];
    if (delta.f32)
        k_pack<float, R><<<nblocks(2 * F.half), TPB, 0, C.st>>>(
            static_cast<const float *>(delta.p), F.logn, F.d[0], F.d[1], nullptr);
    else
        k_pack<double, R><<<nblocks(2 * F.half), TPB, 0, C.st>>>(
            static_cast<const double *>(delta.p), F.logn, F.d[0], F.d[1], nullptr);
    for (int l = 0; l + 1 < Hh.nlev; ++l) {
        HLevel<R> &H = Hh.lv[l], &Hc = Hh.lv[l + 1];
        k_restrict<R><<<nblocks(2 * Hc.half), TPB, 0, C.st>>>(H.d[0], H.d[1], H.logn, Hc.d[0],
                                                             Hc.d[1]);
    }
}

void reset_scalars(Ctx &C) {
    k_fill<<<1, TPB, 0, C.st>>>(C.scal, S_NSCAL, 0.0);
    k_fill_u64<<<1, TPB, 0, C.st>>>(C.clamp, 4);
}

struct Profiler {
    Ctx &C;
    Profiler(Ctx &c, bool on, int per_cycle) : C(c) {
        C.profile = on;
        if (on) {
            C.ev.resize(2 * per_cycle);
            for (auto &e : C.ev) (void)hipEventCreate(&e);
        }
    }
    ~Profiler() {
        for (auto &e : C.ev) (void)hipEventDestroy(e);
        for (auto &e : C.lev_ev) (void)hipEventDestroy(e);
        C.ev.clear();
        C.lev_ev.clear();
    }
};

// Clamp count, timing and status of a finished forward solve.
mg_status finish(Ctx &C, mg_status status, mg_stats *st,
                 std::chrono::steady_clock::time_point t0) {
    unsigned long long ncl = 0;
    HIPCHK(hipGetLastError());
    if (C.no_sync) {   // everything is enqueued; the clamp count is not read
        st->n_clamped = -1;
        st->status = status;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return status;
    }
    HIPCHK(hipMemcpyAsync(&ncl, C.clamp, sizeof(ncl), hipMemcpyDeviceToHost, C.st));
    HIPCHK(hipStreamSynchronize(C.st));
    st->n_clamped = (long long)ncl;
    if (status == MG_OK && ncl > 0) status = MG_WARN_CLAMPED;
    st->status = status;
    st->pass_ms_avg = C.pass_count ? C.pass_ms / C.pass_count : 0.0;
    st->pass_count = C.pass_count;
    for (int l = 0; l < MG_LEVELS; ++l) st->level_ms[l] = C.level_ms[l];
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

// All-FP32 variant (the single-precision arrays of Sec. 3.2.2): every
// multigrid array in FP32 (the discriminant, residual norms and reductions
// stay FP64); delta and phi cross the boundary in FP64.  Cycles stop at tol,
// at max_cycles, or when a cycle no longer halves the residual (the FP32
// floor), which returns MG_NOT_CONVERGED with a valid phi.
template <int OP>
mg_status fp32_solve(const mg_opts *o, Ctx &C, DeltaIn delta, double *phi, mg_stats *st,
                     std::chrono::steady_clock::time_point t0) {
    density_hierarchy<float>(C, delta);
    HLevel<float> &G = C.h32.lv[0];
    k_pack<double, float><<<nblocks(2 * G.half), TPB, 0, C.st>>>(phi, G.logn, G.u[0], G.u[1],
                                                                 nullptr);
    Solver<OP, float> S(C);
    PhaseResult p;
    mg_status rc = S.run(o->tol, o->max_cycles, 0.5, st, 0, p);
    if (rc != MG_OK) return rc;
    st->cycles = p.cycles;
    st->cycles_fp32 = p.cycles;
    st->eps0 = p.eps0;
    st->eps = p.eps;
    st->eps_fp32 = p.eps;
    st->cell_updates = (long long)o->n * o->n * o->n * (o->nu_pre + o->nu_post) * st->cycles;
    if (p.status < 0) {
        st->status = p.status;
        return (mg_status)p.status;
    }
    S.mean_of(G.u[0], G.u[1], G.half);
    k_unpack<float, double><<<nblocks(2 * G.half), TPB, 0, C.st>>>(G.u[0], G.u[1], G.logn, phi,
                                                                   C.scal + S_MEAN);
    return finish(C, (mg_status)p.status, st, t0);
}

// Defect-correction finish of MG_MIXED_DC (kernels and scheme: mg_dc.h).
// The FP32 phase left its field in the FP32 finest level; that field becomes
// the first background pb and the FP64 field phi64.  Each outer step: the
// FP64 residual of phi64 (stored as g = -r in FP32; the stopping test), one
// inner cycle for the correction e (FP32 finest sweeps on the correction
// form, FP64 FAS on the coarse levels), then phi64 += e, pb = fl32(phi64).
template <int OP>
mg_status dc_finish(const mg_opts *o, Ctx &C, DeltaIn delta, double *phi, mg_stats *st,
                    const PhaseResult &p32, int cycles32,
                    std::chrono::steady_clock::time_point t0) {
    constexpr int MODEL = OP == OP_POISSON ? MODEL_POISSON : MODEL_DGP;
    HLevel<double> &F = C.h64.lv[0], &Hc = C.h64.lv[1];
    HLevel<float> &G = C.h32.lv[0];
    const double ncell = (double)F.n * F.n * F.n;
    density_hierarchy<double>(C, delta);
    for (int c = 0; c < 2; ++c) {
        k_convert<float, double><<<nblocks(G.half), TPB, 0, C.st>>>(G.u[c], F.u[c], G.half);
        std::swap(G.pb[c], G.u[c]);
        k_zero_f32<<<nblocks(G.half), TPB, 0, C.st>>>(G.u[c], G.half);
    }
    Solver<OP, double> S64(C);
    const TileGeom Gf = tile_geom(F.n, F.n), Gr = tile_geom(F.n, F.n / 2, 64);
    const unsigned nbf = tile_blocks(Gf, F.n), nbr = tile_blocks(Gr, F.n / 2);
    auto corr_pass = [&](int c) {
        k_corr_pass_tiled<MODEL><<<nbf, TPB, 0, C.st>>>(C.M, view(G, true), G.pb[0], G.pb[1], c,
                                                        G.spare, C.scal + S_MU, Gf);
        std::swap(G.u[c], G.spare);
    };
    double hs[S_NSCAL] = {};
    double best = INFINITY, eps = INFINITY;
    int status = MG_NOT_CONVERGED, cyc = 0;
    mg_status rc;
    for (;;) {
        // FP64 residual of phi64, g = -r in FP32 (its restriction is unused)
        k_resid_restrict_tiled<OP, true, false, double, true><<<nbr, TPB, 0, C.st>>>(
            C.M, view(F, false), C.scal + S_MU64, 1.0, Hc.ru[0], Hc.ru[1], Hc.f[0], Hc.f[1],
            C.partials, C.clamp, Gr, G.f[0], G.f[1]);
        k_finalize<<<1, 1024, 0, C.st>>>(C.partials, nbr, ncell, C.scal, 5, 0.0);
        if ((rc = S64.read_scal(hs)) != MG_OK) return rc;
        eps = std::sqrt(hs[S_EPS64]);
        if (cycles32 + cyc < MG_HIST) st->eps_hist[cycles32 + cyc] = eps;
        if (!std::isfinite(eps)) {
            status = MG_ERR_NONFINITE;
            break;
        }
        if (eps <= o->tol) {
            status = MG_OK;
            break;
        }
        if (eps > 1e3 * best) {
            status = MG_ERR_DIVERGED;
            break;
        }
        best = std::min(best, eps);
        if (cycles32 + cyc >= o->max_cycles) break;
        // one inner cycle for the correction, its bordering scalar from zero
        k_fill<<<1, TPB, 0, C.st>>>(C.scal + S_MU, 1, 0.0);
        for (int s = 0; s < C.nu1; ++s) {
            corr_pass(0);
            corr_pass(1);
        }
        k_corr_resid_restrict_tiled<MODEL><<<nbr, TPB, 0, C.st>>>(
            C.M, view(G, true), G.pb[0], G.pb[1], C.scal + S_MU, Hc.ru[0], Hc.ru[1], Hc.f[0],
            Hc.f[1], C.partials, Gr);
        k_finalize<<<1, 1024, 0, C.st>>>(C.partials, nbr, ncell, C.scal, 0, 0.0);
        S64.coarse_source(1);
        S64.cycle(1, C.cycle);
        k_prolong_tiled<float, false, double><<<nbr, TPB, 0, C.st>>>(
            G.u[0], G.u[1], G.logn, Hc.u[0], Hc.u[1], Hc.ru[0], Hc.ru[1], Gr);
        for (int s = 0; s < C.nu2; ++s) {
            corr_pass(0);
            corr_pass(1);
        }
        for (int c = 0; c < 2; ++c)
            k_dc_accumulate<<<nblocks(G.half), TPB, 0, C.st>>>(F.u[c], G.u[c], G.pb[c], G.half);
        ++cyc;
    }
    st->cycles = cycles32 + cyc;
    st->eps0 = p32.eps0;
    st->eps = eps;
    st->lambda = -hs[S_MU64];
    st->cell_updates = (long long)o->n * o->n * o->n * (o->nu_pre + o->nu_post) * st->cycles;
    if (status < 0) {
        st->status = status;
        return (mg_status)status;
    }
    // zero-mean gauge
    S64.mean_of(F.u[0], F.u[1], F.half);
    k_unpack<double, double><<<nblocks(2 * F.half), TPB, 0, C.st>>>(F.u[0], F.u[1], F.logn, phi,
                                                                    C.scal + S_MEAN);
    return finish(C, (mg_status)status, st, t0);
}

// noalloc: the caller cannot allocate (mg_solve_dgp_noalloc), so the solve
// creates no events and reads the per-cycle scalars with a plain copy into
// host stack memory instead of the pinned buffer.
template <int OP>
mg_status forward_solve(const mg_opts *o, const Mod &M, const void *delta_p, double *phi,
                        void *ws, size_t ws_bytes, hipStream_t stream, mg_stats *st,
                        bool noalloc = false) {
    auto t0 = std::chrono::steady_clock::now();
    const DeltaIn delta{delta_p, o->delta_fp32 != 0};
    const bool dc = o->precision == MG_MIXED_DC;
    const bool mixed = o->precision == MG_MIXED || dc;
    if (dc && OP != OP_DGP && OP != OP_POISSON)
        return fail(MG_ERR_ARG, "MG_MIXED_DC is available for the nDGP and Poisson solves");
    Ctx C;
    Carve cv{static_cast<char *>(ws), 0};
    layout(C, cv, o->n, false, o->precision);
    if (!ws || ws_bytes < cv.off || ((uintptr_t)ws & 255))
        return fail(MG_ERR_WORKSPACE, "workspace too small (need " + std::to_string(cv.off) +
                                          " bytes) or not 256-byte aligned");
    C.st = stream;
    C.M = M;
    C.nu1 = o->nu_pre;
    C.nu2 = o->nu_post;
    C.nuc = o->nu_coarse;
    C.cycle = o->cycle;
    C.no_sync = o->no_sync != 0;
    Profiler prof(C, o->profile != 0 && !noalloc, 2 * (o->nu_pre + o->nu_post) + 2);
    if (!noalloc && !C.no_sync) arm_early_read(C);
    reset_scalars(C);
    if (o->precision == MG_FP32) return fp32_solve<OP>(o, C, delta, phi, st, t0);
    HLevel<double> &F = C.h64.lv[0];
    PhaseResult p32, p64;
    int cycles32 = 0;
    if (mixed) {
        // FP32-storage cycles until the residual stops falling (FP32 floor)
        density_hierarchy<float>(C, delta);
        HLevel<float> &G = C.h32.lv[0];
        k_pack<double, float><<<nblocks(2 * G.half), TPB, 0, C.st>>>(phi, G.logn, G.u[0], G.u[1],
                                                                     nullptr);
        Solver<OP, float> S32(C);
        // a stall hands over to FP64 without a confirming FP32 residual
        mg_status rc = S32.run(o->tol, o->max_cycles, 0.5, st, 0, p32, -1.0, false);
        if (rc != MG_OK) return rc;
        if (p32.status < 0) {
            st->status = p32.status;
            return (mg_status)p32.status;
        }
        cycles32 = p32.cycles;
        st->cycles_fp32 = cycles32;
        st->eps_fp32 = p32.eps;
        if (dc) return dc_finish<OP>(o, C, delta, phi, st, p32, cycles32, t0);
        k_convert<float, double><<<nblocks(G.half), TPB, 0, C.st>>>(G.u[0], F.u[0], G.half);
        k_convert<float, double><<<nblocks(G.half), TPB, 0, C.st>>>(G.u[1], F.u[1], G.half);
    } else {
        k_pack<double, double><<<nblocks(2 * F.half), TPB, 0, C.st>>>(phi, F.logn, F.u[0],
                                                                      F.u[1], nullptr);
    }
    // FP64 cycles (the whole solve, or the finish of the mixed one)
    density_hierarchy<double>(C, delta);
    Solver<OP, double> S(C);
    // after an FP32 stall the FP64 cycles start without a separate residual
    // evaluation (mu from the FP32 phase; the first FP64 cycle refreshes it)
    const double eps_in = (mixed && p32.status == MG_NOT_CONVERGED && p32.eps > o->tol &&
                           cycles32 < o->max_cycles) ? p32.eps : -1.0;
    mg_status rc = S.run(o->tol, o->max_cycles - cycles32, 0.0, st, cycles32, p64, eps_in);
    if (rc != MG_OK) return rc;
    st->cycles = cycles32 + p64.cycles;
    st->eps0 = mixed ? p32.eps0 : p64.eps0;
    st->eps = p64.eps;
    st->cell_updates = (long long)o->n * o->n * o->n * (o->nu_pre + o->nu_post) * st->cycles;
    mg_status status = (mg_status)p64.status;
    if (status < 0) {
        st->status = status;
        return status;
    }
    // zero-mean gauge
    S.mean_of(F.u[0], F.u[1], F.half);
    k_unpack<double, double><<<nblocks(2 * F.half), TPB, 0, C.st>>>(F.u[0], F.u[1], F.logn, phi,
                                                                    C.scal + S_MEAN);
    return finish(C, status, st, t0);
}

template <int MODEL>
void adj_coefficients(Ctx &C, const double *phi) {
    // linearisation points: packed phi on the finest level, restricted below
    Hier<double> &Hh = C.h64;
    HLevel<double> &F = Hh.lv[0];
    k_pack<double, double><<<nblocks(2 * F.half), TPB, 0, C.st>>>(phi, F.logn, F.lin[0],
                                                                  F.lin[1], nullptr);
    for (int l = 0; l < Hh.nlev; ++l) {
        HLevel<double> &H = Hh.lv[l];
        alias_face_coefs(H, MODEL != MODEL_KMO);
        if (l + 1 < Hh.nlev) {
            HLevel<double> &Hc = Hh.lv[l + 1];
            k_restrict<double><<<nblocks(2 * Hc.half), TPB, 0, C.st>>>(H.lin[0], H.lin[1], H.logn,
                                                                      Hc.lin[0], Hc.lin[1]);
        }
        Lvl L = view(H, false);
        L.u0 = H.lin[0];
        L.u1 = H.lin[1];
        if (H.kp[0]) {   // nDGP, tiled level: dK/dSigma only
            k_adj_kprime<<<nblocks(2 * H.half), TPB, 0, C.st>>>(C.M, L, H.kp[0], H.kp[1]);
            continue;
        }
        CoefsW W;
        for (int q = 0; q < 9; ++q)
            for (int c = 0; c < 2; ++c) W.c[q][c] = H.cf[q][c];
        k_adj_coefs<MODEL><<<nblocks(2 * H.half), TPB, 0, C.st>>>(C.M, L, W, H.h);
    }
}

template <int MODEL>
mg_status adjoint_solve(const mg_opts *o, const Mod &M, const void *delta_p, const double *phi,
                        const double *w, double *grad, double *mu, void *ws, size_t ws_bytes,
                        hipStream_t stream, mg_stats *st) {
    auto t0 = std::chrono::steady_clock::now();
    const DeltaIn delta{delta_p, o->delta_fp32 != 0};
    Ctx C;
    Carve cv{static_cast<char *>(ws), 0};
    layout(C, cv, o->n, true, MG_FP64, MODEL != MODEL_KMO, MODEL == MODEL_DGP);
    if (!ws || ws_bytes < cv.off || ((uintptr_t)ws & 255))
        return fail(MG_ERR_WORKSPACE, "workspace too small (need " + std::to_string(cv.off) +
                                          " bytes) or not 256-byte aligned");
    C.st = stream;
    C.M = M;
    C.nu1 = o->nu_pre;
    C.nu2 = o->nu_post;
    C.nuc = o->nu_coarse;
    C.kappa = 6.0;   // 6/h^2 on the finest level: removes the mean of mu in one pass
    C.adj_model = MODEL;
    Profiler prof(C, false, 0);
    arm_early_read(C);
    reset_scalars(C);
    density_hierarchy<double>(C, delta);
    adj_coefficients<MODEL>(C, phi);
    HLevel<double> &F = C.h64.lv[0];
    // right-hand side b = w - mean(w) on the finest level
    k_pack<double, double><<<nblocks(2 * F.half), TPB, 0, C.st>>>(w, F.logn, F.f[0], F.f[1],
                                                                  nullptr);
    Solver<OP_ADJ, double> S(C);
    S.mean_of(F.f[0], F.f[1], F.half);
    k_pack<double, double><<<nblocks(2 * F.half), TPB, 0, C.st>>>(w, F.logn, F.f[0], F.f[1],
                                                                  C.scal + S_MEAN);
    k_pack<double, double><<<nblocks(2 * F.half), TPB, 0, C.st>>>(mu, F.logn, F.u[0], F.u[1],
                                                                  nullptr);
    if (tiled_level(F.n)) {
        // colour sums of the starting field (later kept by the kernels that write mu)
        const unsigned nb = (unsigned)std::min<size_t>(nblocks(F.half), 2048);
        for (int c = 0; c < 2; ++c) {
            k_sum<double><<<nb, TPB, 0, C.st>>>(F.u[c], nullptr, F.half, C.partials);
            k_finalize<<<1, 1024, 0, C.st>>>(C.partials, nb, (double)F.n * F.n * F.n, C.scal, 3,
                                             0.0, c);
        }
    }
    PhaseResult pr;
    mg_status rc = S.run(o->tol, o->max_cycles, 0.0, st, 0, pr);
    if (rc != MG_OK) return rc;
    st->cycles = pr.cycles;
    st->eps0 = pr.eps0;
    st->eps = pr.eps;
    st->cell_updates = (long long)o->n * o->n * o->n * (o->nu_pre + o->nu_post) * pr.cycles;
    if (pr.status < 0) {
        st->status = pr.status;
        return (mg_status)pr.status;
    }
    k_unpack<double, double><<<nblocks(2 * F.half), TPB, 0, C.st>>>(F.u[0], F.u[1], F.logn, mu,
                                                                    nullptr);
    Lvl L = view(F, false);
    L.u0 = F.lin[0];
    L.u1 = F.lin[1];
    k_adj_grad<MODEL><<<nblocks(2 * F.half), TPB, 0, C.st>>>(C.M, L, F.u[0], F.u[1], grad);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(C.st));
    st->status = pr.status;
    st->lambda = 0.0;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return (mg_status)pr.status;
}

// ------------------------------------------------------- single operations

size_t op_workspace_bytes(int n) {
    if (!is_pow2(n) || n < 4 || n > 2048) return 0;
    const size_t half = (size_t)n * n * n / 2;
    // u(2) + spare + d(2) + f(2) + out(2) + coefficients(18) + coarse (2+2)
    return (half * (2 + 1 + 2 + 2 + 2 + 18 + 2 + 2) + 64) * sizeof(double) + 256 * 40;
}

struct OpWs {
    HLevel<double> H;
    double *out[2];
    double *coarse[2];
};

mg_status op_layout(int n, double h, void *ws, size_t ws_bytes, OpWs &W) {
    if (!is_pow2(n) || n < 4 || n > 2048) return fail(MG_ERR_ARG, "n must be a power of two in [4, 2048]");
    if (!(h > 0.0)) return fail(MG_ERR_ARG, "h must be > 0");
    if (!ws || ws_bytes < op_workspace_bytes(n) || ((uintptr_t)ws & 255))
        return fail(MG_ERR_WORKSPACE, "workspace too small or not 256-byte aligned");
    Carve cv{static_cast<char *>(ws), 0};
    HLevel<double> &H = W.H;
    H.n = n;
    H.logn = ilog2(n);
    H.h = h;
    H.half = (size_t)n * n * n / 2;
    for (int c = 0; c < 2; ++c) H.u[c] = cv.take<double>(H.half);
    H.spare = cv.take<double>(H.half);
    for (int c = 0; c < 2; ++c) H.d[c] = cv.take<double>(H.half);
    for (int c = 0; c < 2; ++c) H.f[c] = cv.take<double>(H.half);
    for (int c = 0; c < 2; ++c) W.out[c] = cv.take<double>(H.half);
    for (int q = 0; q < 9; ++q)
        for (int c = 0; c < 2; ++c) H.cf[q][c] = cv.take<double>(H.half);
    for (int c = 0; c < 2; ++c) W.coarse[c] = cv.take<double>(H.half / 4 + 1);
    return MG_OK;
}

template <int OP>
void op_residual_launch(const Mod &M, OpWs &W, hipStream_t s, bool with_f) {
    HLevel<double> &H = W.H;
    k_residual<OP><<<nblocks(2 * H.half), TPB, 0, s>>>(M, view(H, with_f), coefs(H), nullptr, 1.0,
                                                       W.out[0], W.out[1], nullptr);
}

template <int OP>
void op_pass_launch(const Mod &M, OpWs &W, int colour, hipStream_t s) {
    HLevel<double> &H = W.H;
    launch_pass<OP, double>(M, view(H, true), coefs(H), colour, colour ? W.out[1] : W.out[0],
                            nullptr, 0.0, nullptr, s);
}

void pack_f(OpWs &W, const double *f, double fs, hipStream_t s) {
    HLevel<double> &H = W.H;
    if (f)
        k_pack<double, double><<<nblocks(2 * H.half), TPB, 0, s>>>(f, H.logn, H.f[0], H.f[1],
                                                                   nullptr);
    else {
        k_fill<<<nblocks(H.half), TPB, 0, s>>>(H.f[0], H.half, fs);
        k_fill<<<nblocks(H.half), TPB, 0, s>>>(H.f[1], H.half, fs);
    }
}

bool model_mod(int model, const void *params, int n, Mod &M) {
    if (!params) return false;
    if (model == MG_MODEL_DGP || model == MG_MODEL_DGP_NEWTON)
        return setup_dgp((const mg_dgp_params *)params, M);
    if (model == MG_MODEL_KMOUFLAGE) return setup_kmo((const mg_kmo_params *)params, n, M);
    if (model == MG_MODEL_POISSON) {
        M = Mod{};
        M.s = ((const mg_poisson_params *)params)->s;
        return std::isfinite(M.s);
    }
    return false;
}

mg_status common_checks(const mg_opts *o, const void *delta, const void *phi, void *ws,
                        mg_stats *st) {
    mg_status rc = check_opts(o);
    if (rc != MG_OK) return rc;
    if (!delta || !phi) return fail(MG_ERR_ARG, "delta and phi must be device pointers");
    if (!st) return fail(MG_ERR_ARG, "stats is NULL");
    if (!ws) return fail(MG_ERR_WORKSPACE, "workspace is NULL");
    if ((uintptr_t)ws & 255) return fail(MG_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    std::memset(st, 0, sizeof(*st));
    g_err.clear();
    return MG_OK;
}

// Workspace of mg_solve_dgp_noalloc: enough for any precision at n <= 128
// (mg_workspace_bytes(128, MG_MIXED, MG_MODEL_DGP, 0) is 87.6 MiB).
constexpr int NOALLOC_MAX_N = 128;
constexpr size_t NOALLOC_BYTES = (size_t)88 << 20;

}  // namespace

// Device-resident workspace of mg_solve_dgp_noalloc, one copy per GPU (at its
// own address on each), held until the process ends.  Host code must never
// pass this name to a kernel or a copy: it stands for a host-side shadow.
// The device address comes from hipGetSymbolAddress (noalloc_scratch()).
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of scratch on the current device, looked up once per device
// (with that device current) and kept.
mg_status noalloc_scratch(void **out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(MG_ERR_ARG, "mg_solve_dgp_noalloc supports device indices 0..63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255)) return fail(MG_ERR_HIP, "scratch symbol address invalid");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return MG_OK;
}

}  // namespace

namespace mgglam_internal {
void set_error(const char *msg) { g_err = msg; }
}  // namespace mgglam_internal

// ===================================================================== C ABI

extern "C" {

size_t mg_workspace_bytes(int n, int precision, int model, int adjoint) {
    if (!is_pow2(n) || n < 8 || n > 2048 || model < 0 || model > 3) return 0;
    if (model == MG_MODEL_DGP_NEWTON && (adjoint || precision != MG_FP64)) return 0;
    if (precision != MG_FP64 && precision != MG_MIXED && precision != MG_FP32 &&
        precision != MG_MIXED_DC)
        return 0;
    if (precision == MG_MIXED_DC && n < 128) return 0;
    if (adjoint && precision != MG_FP64) return 0;
    Ctx C;
    Carve cv{nullptr, 0};
    layout(C, cv, n, adjoint != 0, precision, model != MG_MODEL_KMOUFLAGE,
           adjoint != 0 && model == MG_MODEL_DGP);
    return cv.off + 256;
}

mg_status mg_linear_source(int model, const void *params, int n, double *s) {
    g_err.clear();
    if (!params || !s) return fail(MG_ERR_ARG, "params and s must not be NULL");
    if (model != MG_MODEL_DGP && model != MG_MODEL_KMOUFLAGE)
        return fail(MG_ERR_ARG, "model must be MG_MODEL_DGP or MG_MODEL_KMOUFLAGE");
    if (model == MG_MODEL_KMOUFLAGE && (n < 1 || n > 65536))
        return fail(MG_ERR_ARG, "n must be in [1, 65536]");
    Mod M;
    if (!model_mod(model, params, n, M)) return fail(MG_ERR_ARG, "invalid model parameters");
    // nDGP: F(Sigma) -> Sigma / alpha at small Sigma, T -> 0, so lap phi = (s / alpha) delta.
    // Kmouflage: Sigma_1 -> K_X = c0, Sigma_2 -> 0.
    *s = model == MG_MODEL_DGP ? M.s / M.alpha : M.src / (M.ctil * M.c0);
    return MG_OK;
}

mg_status mg_solve_dgp(const mg_opts *opts, const mg_dgp_params *par, const void *delta,
                       double *phi, void *ws, size_t ws_bytes, hipStream_t stream,
                       mg_stats *stats) {
    mg_status rc = common_checks(opts, delta, phi, ws, stats);
    if (rc != MG_OK) return rc;
    Mod M;
    if (!par || !setup_dgp(par, M)) return fail(MG_ERR_ARG, "invalid nDGP parameters");
    return forward_solve<OP_DGP>(opts, M, delta, phi, ws, ws_bytes, stream, stats);
}

mg_status mg_solve_dgp_noalloc(const mg_opts *opts, const mg_dgp_params *par,
                               const void *delta, double *phi, hipStream_t stream,
                               mg_stats *stats) {
    g_err.clear();
    mg_status rc = check_opts(opts);
    if (rc != MG_OK) return rc;
    if (opts->n > NOALLOC_MAX_N)
        return fail(MG_ERR_ARG, "mg_solve_dgp_noalloc: opts.n must be <= 128 (its static "
                                "workspace holds 88 MiB); use mg_solve_dgp for larger meshes");
    if (opts->profile) return fail(MG_ERR_ARG, "mg_solve_dgp_noalloc: profile must be 0");
    if (!delta || !phi) return fail(MG_ERR_ARG, "delta and phi must be device pointers");
    if (!stats) return fail(MG_ERR_ARG, "stats is NULL");
    Mod M;
    if (!par || !setup_dgp(par, M)) return fail(MG_ERR_ARG, "invalid nDGP parameters");
    std::memset(stats, 0, sizeof(*stats));
    void *ws = nullptr;
    if ((rc = noalloc_scratch(&ws)) != MG_OK) return rc;
    return forward_solve<OP_DGP>(opts, M, delta, phi, ws, NOALLOC_BYTES, stream, stats, true);
}

mg_status mg_solve_dgp_newton(const mg_opts *opts, const mg_dgp_params *par, const void *delta,
                              double *phi, void *ws, size_t ws_bytes, hipStream_t stream,
                              mg_stats *stats) {
    mg_status rc = common_checks(opts, delta, phi, ws, stats);
    if (rc != MG_OK) return rc;
    if (opts->precision != MG_FP64) return fail(MG_ERR_ARG, "the Newton-GS comparator is FP64 only");
    Mod M;
    if (!par || !setup_dgp(par, M)) return fail(MG_ERR_ARG, "invalid nDGP parameters");
    return forward_solve<OP_NEWTON>(opts, M, delta, phi, ws, ws_bytes, stream, stats);
}

mg_status mg_solve_kmouflage(const mg_opts *opts, const mg_kmo_params *par, const void *delta,
                             double *phi, void *ws, size_t ws_bytes, hipStream_t stream,
                             mg_stats *stats) {
    mg_status rc = common_checks(opts, delta, phi, ws, stats);
    if (rc != MG_OK) return rc;
    Mod M;
    if (!par || !setup_kmo(par, opts->n, M)) return fail(MG_ERR_ARG, "invalid Kmouflage parameters");
    return forward_solve<OP_KMO>(opts, M, delta, phi, ws, ws_bytes, stream, stats);
}

mg_status mg_solve_poisson(const mg_opts *opts, const mg_poisson_params *par, const void *delta,
                           double *phi, void *ws, size_t ws_bytes, hipStream_t stream,
                           mg_stats *stats) {
    mg_status rc = common_checks(opts, delta, phi, ws, stats);
    if (rc != MG_OK) return rc;
    if (!par || !std::isfinite(par->s)) return fail(MG_ERR_ARG, "invalid Poisson parameters");
    Mod M{};
    M.s = par->s;
    return forward_solve<OP_POISSON>(opts, M, delta, phi, ws, ws_bytes, stream, stats);
}

mg_status mg_solve_adjoint(const mg_opts *opts, int model, const void *params,
                           const void *delta, const double *phi, const double *w,
                           double *grad_delta, double *mu, void *ws, size_t ws_bytes,
                           hipStream_t stream, mg_stats *stats) {
    mg_status rc = common_checks(opts, delta, phi, ws, stats);
    if (rc != MG_OK) return rc;
    if (opts->precision != MG_FP64) return fail(MG_ERR_ARG, "the adjoint solve is FP64 only");
    if (opts->no_sync) return fail(MG_ERR_ARG, "the adjoint solve waits for its stream: opts.no_sync must be 0");
    if (opts->cycle != MG_CYCLE_V) return fail(MG_ERR_ARG, "the adjoint solve uses V-cycles only");
    if (model == MG_MODEL_DGP_NEWTON) return fail(MG_ERR_ARG, "no adjoint for the Newton-GS comparator");
    if (!w || !grad_delta || !mu) return fail(MG_ERR_ARG, "w, grad_delta and mu must be device pointers");
    Mod M;
    if (!model_mod(model, params, opts->n, M)) return fail(MG_ERR_ARG, "invalid model or parameters");
    switch (model) {
        case MG_MODEL_DGP:
            return adjoint_solve<MODEL_DGP>(opts, M, delta, phi, w, grad_delta, mu, ws, ws_bytes,
                                            stream, stats);
        case MG_MODEL_KMOUFLAGE:
            return adjoint_solve<MODEL_KMO>(opts, M, delta, phi, w, grad_delta, mu, ws, ws_bytes,
                                            stream, stats);
        default:
            return adjoint_solve<MODEL_POISSON>(opts, M, delta, phi, w, grad_delta, mu, ws,
                                                ws_bytes, stream, stats);
    }
}

size_t mg_op_workspace_bytes(int n) { return op_workspace_bytes(n); }

mg_status mg_op_residual(int model, const void *params, int n, double h, const double *phi,
                         const double *delta, const double *f, double fs, double *out, void *ws,
                         size_t ws_bytes, hipStream_t stream) {
    OpWs W;
    mg_status rc = op_layout(n, h, ws, ws_bytes, W);
    if (rc != MG_OK) return rc;
    if (!phi || !delta || !out) return fail(MG_ERR_ARG, "NULL array");
    Mod M;
    if (!model_mod(model, params, n, M)) return fail(MG_ERR_ARG, "invalid model or parameters");
    HLevel<double> &H = W.H;
    const unsigned nb = nblocks(2 * H.half);
    k_pack<double, double><<<nb, TPB, 0, stream>>>(phi, H.logn, H.u[0], H.u[1], nullptr);
    k_pack<double, double><<<nb, TPB, 0, stream>>>(delta, H.logn, H.d[0], H.d[1], nullptr);
    pack_f(W, f, fs, stream);
    switch (model) {
        case MG_MODEL_DGP: op_residual_launch<OP_DGP>(M, W, stream, true); break;
        case MG_MODEL_DGP_NEWTON: op_residual_launch<OP_NEWTON>(M, W, stream, true); break;
        case MG_MODEL_KMOUFLAGE: op_residual_launch<OP_KMO>(M, W, stream, true); break;
        default: op_residual_launch<OP_POISSON>(M, W, stream, true); break;
    }
    k_unpack<double, double><<<nb, TPB, 0, stream>>>(W.out[0], W.out[1], H.logn, out, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return MG_OK;
}

mg_status mg_op_colour_pass(int model, const void *params, int n, double h, int colour,
                            const double *phi_in, const double *delta, const double *f, double fs,
                            double *phi_out, void *ws, size_t ws_bytes, hipStream_t stream) {
    OpWs W;
    mg_status rc = op_layout(n, h, ws, ws_bytes, W);
    if (rc != MG_OK) return rc;
    if (!phi_in || !delta || !phi_out) return fail(MG_ERR_ARG, "NULL array");
    if (colour != 0 && colour != 1) return fail(MG_ERR_ARG, "colour must be 0 or 1");
    Mod M;
    if (!model_mod(model, params, n, M)) return fail(MG_ERR_ARG, "invalid model or parameters");
    HLevel<double> &H = W.H;
    const unsigned nb = nblocks(2 * H.half);
    k_pack<double, double><<<nb, TPB, 0, stream>>>(phi_in, H.logn, H.u[0], H.u[1], nullptr);
    k_pack<double, double><<<nb, TPB, 0, stream>>>(phi_in, H.logn, W.out[0], W.out[1], nullptr);
    k_pack<double, double><<<nb, TPB, 0, stream>>>(delta, H.logn, H.d[0], H.d[1], nullptr);
    pack_f(W, f, fs, stream);
    switch (model) {
        case MG_MODEL_DGP: op_pass_launch<OP_DGP>(M, W, colour, stream); break;
        case MG_MODEL_DGP_NEWTON: op_pass_launch<OP_NEWTON>(M, W, colour, stream); break;
        case MG_MODEL_KMOUFLAGE: op_pass_launch<OP_KMO>(M, W, colour, stream); break;
        default: op_pass_launch<OP_POISSON>(M, W, colour, stream); break;
    }
    k_unpack<double, double><<<nb, TPB, 0, stream>>>(W.out[0], W.out[1], H.logn, phi_out, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return MG_OK;
}

mg_status mg_op_restrict(int n, const double *fine, double *coarse, void *ws, size_t ws_bytes,
                         hipStream_t stream) {
    OpWs W;
    mg_status rc = op_layout(n, 1.0, ws, ws_bytes, W);
    if (rc != MG_OK) return rc;
    if (n < 8) return fail(MG_ERR_ARG, "n must be >= 8");
    if (!fine || !coarse) return fail(MG_ERR_ARG, "NULL array");
    HLevel<double> &H = W.H;
    k_pack<double, double><<<nblocks(2 * H.half), TPB, 0, stream>>>(fine, H.logn, H.u[0], H.u[1],
                                                                    nullptr);
    k_restrict<double><<<nblocks(H.half / 4), TPB, 0, stream>>>(H.u[0], H.u[1], H.logn,
                                                                W.coarse[0], W.coarse[1]);
    k_unpack<double, double><<<nblocks(H.half / 4), TPB, 0, stream>>>(W.coarse[0], W.coarse[1],
                                                                      H.logn - 1, coarse, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return MG_OK;
}

mg_status mg_op_prolong_add(int n, double *fine, const double *uc, const double *rc_,
                            void *ws, size_t ws_bytes, hipStream_t stream) {
    OpWs W;
    mg_status rc = op_layout(n, 1.0, ws, ws_bytes, W);
    if (rc != MG_OK) return rc;
    if (n < 8) return fail(MG_ERR_ARG, "n must be >= 8");
    if (!fine || !uc || !rc_) return fail(MG_ERR_ARG, "NULL array");
    HLevel<double> &H = W.H;
    const unsigned nbc = nblocks(H.half / 4);
    k_pack<double, double><<<nblocks(2 * H.half), TPB, 0, stream>>>(fine, H.logn, H.u[0], H.u[1],
                                                                    nullptr);
    k_pack<double, double><<<nbc, TPB, 0, stream>>>(uc, H.logn - 1, W.coarse[0], W.coarse[1],
                                                    nullptr);
    k_pack<double, double><<<nbc, TPB, 0, stream>>>(rc_, H.logn - 1, W.out[0], W.out[1], nullptr);
    launch_prolong<double>(H.u[0], H.u[1], H.logn, W.coarse[0], W.coarse[1], W.out[0], W.out[1],
                           stream);
    k_unpack<double, double><<<nblocks(2 * H.half), TPB, 0, stream>>>(H.u[0], H.u[1], H.logn,
                                                                      fine, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return MG_OK;
}

mg_status mg_op_jt_apply(int model, const void *params, int n, double h, const double *phi,
                         const double *delta, const double *v, double *out, void *ws,
                         size_t ws_bytes, hipStream_t stream) {
    OpWs W;
    mg_status rc = op_layout(n, h, ws, ws_bytes, W);
    if (rc != MG_OK) return rc;
    if (!phi || !delta || !v || !out) return fail(MG_ERR_ARG, "NULL array");
    Mod M;
    if (!model_mod(model, params, n, M)) return fail(MG_ERR_ARG, "invalid model or parameters");
    HLevel<double> &H = W.H;
    const unsigned nb = nblocks(2 * H.half);
    k_pack<double, double><<<nb, TPB, 0, stream>>>(phi, H.logn, H.u[0], H.u[1], nullptr);
    k_pack<double, double><<<nb, TPB, 0, stream>>>(delta, H.logn, H.d[0], H.d[1], nullptr);
    alias_face_coefs(H, model != MG_MODEL_KMOUFLAGE);
    CoefsW Wc;
    for (int q = 0; q < 9; ++q)
        for (int c = 0; c < 2; ++c) Wc.c[q][c] = H.cf[q][c];
    switch (model) {
        case MG_MODEL_DGP: k_adj_coefs<MODEL_DGP><<<nb, TPB, 0, stream>>>(M, view(H, false), Wc, h); break;
        case MG_MODEL_KMOUFLAGE: k_adj_coefs<MODEL_KMO><<<nb, TPB, 0, stream>>>(M, view(H, false), Wc, h); break;
        default: k_adj_coefs<MODEL_POISSON><<<nb, TPB, 0, stream>>>(M, view(H, false), Wc, h); break;
    }
    k_pack<double, double><<<nb, TPB, 0, stream>>>(v, H.logn, H.u[0], H.u[1], nullptr);
    op_residual_launch<OP_ADJ>(M, W, stream, false);
    k_unpack<double, double><<<nb, TPB, 0, stream>>>(W.out[0], W.out[1], H.logn, out, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return MG_OK;
}

const char *mg_status_string(mg_status s) {
    switch (s) {
        case MG_OK: return "MG_OK";
        case MG_NOT_CONVERGED: return "MG_NOT_CONVERGED: cycle cap reached before the tolerance";
        case MG_WARN_CLAMPED: return "MG_WARN_CLAMPED: converged; negative discriminants were clamped";
        case MG_ERR_ARG: return "MG_ERR_ARG: invalid argument";
        case MG_ERR_HIP: return "MG_ERR_HIP: HIP runtime error";
        case MG_ERR_NONFINITE: return "MG_ERR_NONFINITE: residual is not finite";
        case MG_ERR_DIVERGED: return "MG_ERR_DIVERGED: residual grew 1e3 above its minimum";
        case MG_ERR_WORKSPACE: return "MG_ERR_WORKSPACE: workspace missing or too small";
    }
    return "unknown mg_status";
}

const char *mg_last_error(void) { return g_err.c_str(); }

}  // extern "C"
