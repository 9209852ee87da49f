// Host-side checks of libmgglam's ABI code, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host part only (tests/test_sanitizers.py).
// No GPU is touched: every call below either computes on the host
// (workspace layouts, the Kmouflage background solver, linear-source
// coefficients, status strings) or is rejected by argument validation before
// the first HIP call.  Exits non-zero on the first unexpected result; the
// sanitizers abort on any memory or UB error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mgglam.h"

static int failures = 0;
#define CHECK(cond)                                                             \
    do {                                                                        \
        if (!(cond)) {                                                          \
            std::fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #cond);     \
            ++failures;                                                         \
        }                                                                       \
    } while (0)

static mg_opts opts(int n) {
    mg_opts o{};
    o.n = n;
    o.max_cycles = 10;
    o.tol = 1e-8;
    o.nu_pre = o.nu_post = 1;
    o.nu_coarse = 32;
    return o;
}

int main() {
    // workspace layouts: every size, precision, model and the adjoint carve
    // the same way they are measured (null base), and grow with n
    for (int model = 0; model < 4; ++model)
        for (int prec = 0; prec < 3; ++prec)
            for (int adj = 0; adj < 2; ++adj) {
                size_t prev = 0;
                for (int n = 8; n <= 2048; n *= 2) {
                    const size_t b = mg_workspace_bytes(n, prec, model, adj);
                    const bool valid = !(model == MG_MODEL_DGP_NEWTON && (adj || prec != MG_FP64)) &&
                                       !(adj && prec != MG_FP64);
                    if (valid) {
                        CHECK(b > prev);
                        prev = b;
                    } else {
                        CHECK(b == 0);
                    }
                }
                CHECK(mg_workspace_bytes(24, prec, model, adj) == 0);
                CHECK(mg_workspace_bytes(4096, prec, model, adj) == 0);
            }
    CHECK(mg_workspace_bytes(64, 7, 0, 0) == 0);
    CHECK(mg_workspace_bytes(64, 0, 9, 0) == 0);
    for (int n = 8; n <= 2048; n *= 2) {
        CHECK(mg_op_workspace_bytes(n) > 0);
        CHECK(mg_pm_workspace_bytes(n) > mg_workspace_bytes(n, MG_FP64, MG_MODEL_DGP, 0));
    }
    CHECK(mg_op_workspace_bytes(3) == 0);
    CHECK(mg_pm_workspace_bytes(12) == 0);

    // argument validation of the solver entry points (no GPU call is reached)
    std::vector<double> host(64);
    double *fake = host.data();   // never dereferenced: every call fails validation
    void *ws_aligned = reinterpret_cast<void *>((uintptr_t)0x100000);
    mg_stats st;
    mg_dgp_params dp{1.0, 0.3089, 1.0};
    mg_opts o = opts(64);
    CHECK(mg_solve_dgp(nullptr, &dp, fake, fake, ws_aligned, 1, nullptr, &st) == MG_ERR_ARG);
    CHECK(std::strlen(mg_last_error()) > 0);
    mg_opts bad = o;
    bad.n = 48;
    CHECK(mg_solve_dgp(&bad, &dp, fake, fake, ws_aligned, 1, nullptr, &st) == MG_ERR_ARG);
    bad = o;
    bad.tol = NAN;
    CHECK(mg_solve_dgp(&bad, &dp, fake, fake, ws_aligned, 1, nullptr, &st) == MG_ERR_ARG);
    bad = o;
    bad.precision = 5;
    CHECK(mg_solve_kmouflage(&bad, nullptr, fake, fake, ws_aligned, 1, nullptr, &st) == MG_ERR_ARG);
    CHECK(mg_solve_dgp(&o, nullptr, fake, fake, ws_aligned, 1, nullptr, &st) == MG_ERR_ARG);
    mg_dgp_params dbad{-1.0, 0.3089, 1.0};
    CHECK(mg_solve_dgp(&o, &dbad, fake, fake, ws_aligned, 1, nullptr, &st) == MG_ERR_ARG);
    CHECK(mg_solve_dgp(&o, &dp, nullptr, fake, ws_aligned, 1, nullptr, &st) == MG_ERR_ARG);
    CHECK(mg_solve_dgp(&o, &dp, fake, fake, nullptr, 1, nullptr, &st) == MG_ERR_WORKSPACE);
    CHECK(mg_solve_dgp(&o, &dp, fake, fake, reinterpret_cast<void *>((uintptr_t)0x100008), 1 << 30,
                       nullptr, &st) == MG_ERR_WORKSPACE);
    // too small by one byte: the layout is carved over the caller's pointer
    // and rejected before any GPU work
    for (int prec = 0; prec < 3; ++prec) {
        mg_opts op = o;
        op.precision = prec;
        const size_t need = mg_workspace_bytes(64, prec, MG_MODEL_DGP, 0);
        CHECK(mg_solve_dgp(&op, &dp, fake, fake, ws_aligned, need - 257, nullptr, &st) ==
              MG_ERR_WORKSPACE);
    }
    mg_kmo_params kp{3, 1.0, 0.1, std::sqrt(3 * (1 - 0.3089)), 1.0, 0.3089, 512.0, 0.0, 0.0};
    const size_t kneed = mg_workspace_bytes(64, MG_FP64, MG_MODEL_KMOUFLAGE, 1);
    CHECK(mg_solve_adjoint(&o, MG_MODEL_KMOUFLAGE, &kp, fake, fake, fake, fake, fake, ws_aligned,
                           kneed - 300, nullptr, &st) == MG_ERR_WORKSPACE);
    mg_opts ow = o;
    ow.cycle = MG_CYCLE_W;
    CHECK(mg_solve_adjoint(&ow, MG_MODEL_DGP, &dp, fake, fake, fake, fake, fake, ws_aligned,
                           kneed, nullptr, &st) == MG_ERR_ARG);
    CHECK(mg_solve_adjoint(&o, MG_MODEL_DGP_NEWTON, &dp, fake, fake, fake, fake, fake, ws_aligned,
                           kneed, nullptr, &st) == MG_ERR_ARG);
    mg_poisson_params pp{NAN};
    CHECK(mg_solve_poisson(&o, &pp, fake, fake, ws_aligned, 1 << 30, nullptr, &st) == MG_ERR_ARG);
    // enqueue-only solves: tol = 0, no profiling, FP64; not for the adjoint
    mg_opts ons = o;
    ons.no_sync = 1;   // with tol > 0
    CHECK(mg_solve_dgp(&ons, &dp, fake, fake, ws_aligned, 1 << 30, nullptr, &st) == MG_ERR_ARG);
    ons.tol = 0.0;
    ons.precision = MG_MIXED;
    CHECK(mg_solve_dgp(&ons, &dp, fake, fake, ws_aligned, 1 << 30, nullptr, &st) == MG_ERR_ARG);
    ons.precision = MG_FP64;
    ons.no_sync = 3;
    CHECK(mg_solve_dgp(&ons, &dp, fake, fake, ws_aligned, 1 << 30, nullptr, &st) == MG_ERR_ARG);
    ons.no_sync = 1;
    CHECK(mg_solve_adjoint(&ons, MG_MODEL_DGP, &dp, fake, fake, fake, fake, fake, ws_aligned,
                           kneed, nullptr, &st) == MG_ERR_ARG);

    // single operations
    CHECK(mg_op_residual(MG_MODEL_DGP, &dp, 6, 1.0, fake, fake, nullptr, 0.0, fake, ws_aligned,
                         1 << 30, nullptr) == MG_ERR_ARG);
    CHECK(mg_op_colour_pass(MG_MODEL_DGP, &dp, 16, 1.0, 2, fake, fake, nullptr, 0.0, fake,
                            ws_aligned, mg_op_workspace_bytes(16), nullptr) == MG_ERR_ARG);
    CHECK(mg_op_restrict(4, fake, fake, ws_aligned, mg_op_workspace_bytes(4), nullptr) ==
          MG_ERR_ARG);
    CHECK(mg_op_prolong_add(16, fake, fake, fake, ws_aligned, 10, nullptr) == MG_ERR_WORKSPACE);
    CHECK(mg_op_jt_apply(9, &dp, 16, 1.0, fake, fake, fake, fake, ws_aligned,
                         mg_op_workspace_bytes(16), nullptr) == MG_ERR_ARG);

    // host-only computations
    double s = 0.0;
    CHECK(mg_linear_source(MG_MODEL_DGP, &dp, 64, &s) == MG_OK && s > 0.0);
    CHECK(mg_linear_source(MG_MODEL_KMOUFLAGE, &kp, 64, &s) == MG_OK && s > 0.0);
    CHECK(mg_linear_source(MG_MODEL_POISSON, &dp, 64, &s) == MG_ERR_ARG);
    const double orad = mg_omega_radiation(0.6774, 2.7255, 3.046);
    CHECK(orad > 0.0 && orad < 1e-3);
    CHECK(mg_omega_radiation(-1.0, 2.7255, 3.046) < 0.0);
    mg_kmo_bg_params bp{2, 1.0, 0.2, 0.3089, orad, 1e5, 1e-10};
    std::vector<double> at{0.1, 0.25, 0.5, 0.75, 1.0}, hub(5), hd(5), pb(5), pd(5);
    mg_kmo_bg_info info;
    CHECK(mg_kmo_background(&bp, 5, at.data(), hub.data(), hd.data(), pb.data(), pd.data(),
                            &info) == MG_OK);
    CHECK(std::fabs(hub[4] - 1.0) < 1e-9 && pb[4] < 0.0 && info.lambda > 0.0);
    CHECK(mg_kmo_background(&bp, 0, nullptr, nullptr, nullptr, nullptr, nullptr, &info) == MG_OK);
    std::vector<double> unsorted{0.5, 0.4};
    CHECK(mg_kmo_background(&bp, 2, unsorted.data(), hub.data(), hd.data(), pb.data(), pd.data(),
                            &info) == MG_ERR_ARG);
    mg_kmo_bg_params bpb = bp;
    bpb.n_k = 1;
    CHECK(mg_kmo_background(&bpb, 5, at.data(), hub.data(), hd.data(), pb.data(), pd.data(),
                            &info) == MG_ERR_ARG);

    // particle-mesh entry points: rejected before the GPU, including the
    // Kmouflage background-table lookup
    mg_pm_params pm{32, 16, 0.3089, 1.0, 1.0, 0.01, opts(16)};
    float *fp = reinterpret_cast<float *>(host.data());
    CHECK(mg_pm_step(&pm, fp, fp, fake, fake, fake, ws_aligned, 1ull << 40, nullptr, &st) ==
          MG_ERR_ARG);
    CHECK(mg_cic_delta(24, 16, fp, fake, ws_aligned, 1ull << 40, nullptr) == MG_ERR_ARG);
    CHECK(mg_cic_delta(32, 16, fp, fake, ws_aligned, 8, nullptr) == MG_ERR_WORKSPACE);
    std::vector<double> ta{0.5, 0.6}, th{1.2, 1.1}, tp{0.0, 0.0}, tt{0.0, 0.0};
    mg_kmo_bg_table tab{2, ta.data(), th.data(), tp.data(), tt.data(), 1.4};
    mg_pm_kmo_params kpm{32, 16, 0.5, 0.01, 64.0, bp, &tab, opts(32)};
    CHECK(mg_pm_step_kmouflage(&kpm, fp, fp, fake, fake, fake, ws_aligned, 1ull << 40, nullptr,
                               &st) == MG_ERR_ARG);
    kpm.a = 0.99;
    kpm.da = 0.04;
    kpm.table = nullptr;
    CHECK(mg_pm_step_kmouflage(&kpm, fp, fp, fake, fake, fake, ws_aligned, 1ull << 40, nullptr,
                               &st) == MG_ERR_ARG);

    // FFT Poisson solve: size, aliasing, alignment and workspace checks
    double *fake2 = fake + 2;
    CHECK(mg_fft_poisson_workspace_bytes(48) == 0);
    CHECK(mg_fft_poisson_workspace_bytes(64) >= 32 * 16);
    CHECK(mg_fft_poisson(48, 1.0, fake, fake2, ws_aligned, 1 << 20, nullptr) == MG_ERR_ARG);
    CHECK(mg_fft_poisson(64, 1.0, fake, fake, ws_aligned, 1 << 20, nullptr) == MG_ERR_ARG);
    CHECK(mg_fft_poisson(64, 1.0, fake, fake + 1, ws_aligned, 1 << 20, nullptr) == MG_ERR_ARG);
    CHECK(mg_fft_poisson(64, 1.0, fake, fake2, ws_aligned, 16, nullptr) == MG_ERR_WORKSPACE);

    // the density-precision flag
    mg_opts of = opts(32);
    of.delta_fp32 = 3;
    CHECK(mg_solve_dgp(&of, &dp, fake, fake, ws_aligned, 1ull << 40, nullptr, &st) == MG_ERR_ARG);

    for (int c = -6; c <= 3; ++c) CHECK(mg_status_string((mg_status)c) != nullptr);
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host ABI checks passed\n");
    return 0;
}
