/*
 * mgglam.h -- C ABI of the MI355X (gfx950) multigrid solver for the scalar
 * fields of derivative-coupling modified gravity, after Hernandez-Aguayo et
 * al., "Fast full N-body simulations of generic modified gravity: derivative
 * coupling models" (arXiv:2110.00566).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Code units of Sec. 3.1.1: the finest mesh has cell size h = 1 and n
 *    cells per side; n is a power of two, 8 <= n <= 2048.
 *  - Mesh arrays are DEVICE pointers to contiguous C-order arrays
 *    a[z][y][x] (x fastest) of n^3 elements, periodic in every axis.
 *    Particle arrays are DEVICE pointers to [n_part^3][3] FP32 (x, y, z).
 *  - The caller owns every array and the workspace; the library never
 *    allocates, frees or keeps them.  Work is enqueued on the caller's
 *    stream.  Solver calls return after that stream has reached the end of
 *    the solve (the stopping test reads one residual per cycle), except
 *    FP64 forward solves with mg_opts.no_sync = 1, which only enqueue.
 *  - Arguments are validated before the first GPU call; invalid ones give
 *    MG_ERR_ARG and mg_last_error() says which.  Positive status codes mean
 *    the outputs are valid (see the stats); negative codes leave outputs
 *    unspecified.
 *  - Calls that share a workspace must not overlap in time.  Workspaces
 *    start on a 256-byte boundary (hipMalloc's and torch's allocations do).
 *  - Solver calls read the stopping residual through one 128-byte pinned
 *    host buffer per calling thread, allocated on first use and kept until
 *    the process ends.
 */
#ifndef MGGLAM_H
#define MGGLAM_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MG_OK = 0,
    MG_NOT_CONVERGED = 1,   /* cycle cap reached; phi valid, stats.eps > tol */
    MG_WARN_CLAMPED = 2,    /* converged, but a negative nDGP discriminant was clamped */
    MG_ERR_ARG = -1,
    MG_ERR_HIP = -2,
    MG_ERR_NONFINITE = -3,  /* residual became NaN/Inf (e.g. NaN in delta) */
    MG_ERR_DIVERGED = -4,   /* residual grew 1e3x above its minimum */
    MG_ERR_WORKSPACE = -5   /* workspace null, smaller than required or not 256-byte aligned */
} mg_status;

typedef enum { MG_FP64 = 0, MG_MIXED = 1, MG_FP32 = 2, MG_MIXED_DC = 3 } mg_precision;
typedef enum {
    MG_MODEL_DGP = 0,
    MG_MODEL_KMOUFLAGE = 1,
    MG_MODEL_POISSON = 2,
    MG_MODEL_DGP_NEWTON = 3   /* comparator: see mg_solve_dgp_newton (single ops and sizing) */
} mg_model;

/* Multigrid cycle arrangements of Sec. 3.2.1 (fig:multigrid_cycles), as the
 * textbook recursions: V = one coarse cycle per level, W = two coarse
 * W-cycles, F = a coarse F-cycle followed by a coarse V-cycle.  Every visit
 * of the 4^3 level runs nu_coarse sweeps. */
typedef enum { MG_CYCLE_V = 0, MG_CYCLE_F = 1, MG_CYCLE_W = 2 } mg_cycle;

/* Solver options.  Sec. 3.2.1: FAS cycles with nonlinear red-black
 * Gauss-Seidel smoothing, 8-cell mean restriction, 27/9/3/1 prolongation,
 * coarsest level 4^3. */
typedef struct {
    int n;            /* cells per side of the finest mesh (power of two, 8..2048).
                         Workspace plus the caller's FP64 delta and phi: 49 GB at
                         1024^3 (FP64); at 2048^3 393 GB (FP64), so only MG_FP32
                         (266 GB) fits in one MI355X's 288 GB.  Sizes above 1024
                         are untested. */
    int max_cycles;   /* cap on cycles (0..100000); default 50 */
    double tol;       /* stop when the RMS of the mean-projected finest residual
                         is <= tol (code units); 0 runs exactly max_cycles */
    int nu_pre;       /* smoothing sweeps before restriction (one sweep = colour 0
                         pass then colour 1 pass); default 1 */
    int nu_post;      /* sweeps after the coarse-grid correction; default 1 */
    int nu_coarse;    /* sweeps on the 4^3 level; default 32 */
    int precision;    /* mg_precision: MG_FP64, or MG_MIXED = FP32-storage FAS cycles
                         (FP64 discriminant, residuals and reductions) until the FP32
                         residual stops falling, then FP64 cycles from that field to
                         tol; the final residual is always the FP64 one; or MG_FP32 =
                         the FP32-storage cycles alone (every multigrid array in FP32,
                         as the single-precision arrays of Sec. 3.2.2), stopping at tol,
                         max_cycles or the FP32 floor (a cycle that no longer halves
                         the residual: MG_NOT_CONVERGED, phi valid); or MG_MIXED_DC =
                         the FP32-storage cycles to their floor, then defect correction:
                         each outer step evaluates the FP64 finest residual r of the
                         FP64 field, runs one FP32 cycle for a correction e of the
                         frozen background fl32(phi) -- finest-level sweeps in FP32 on
                         the correction form of the operator (model-term difference
                         without cancellation), coarse levels in FP64 -- and
                         accumulates phi += e in FP64; stats.eps_hist then holds the
                         FP64 residual before each outer step (nDGP and Poisson,
                         n >= 128).  Forward solves only; the adjoint and the Newton-GS
                         comparator are FP64 */
    int cycle;        /* mg_cycle: MG_CYCLE_V (default), MG_CYCLE_F or MG_CYCLE_W;
                         mg_solve_adjoint accepts MG_CYCLE_V only */
    int profile;      /* 1: time every finest-level colour pass with HIP events
                         on the caller's stream (stats.pass_ms_avg) */
    int delta_fp32;   /* 0: the solves' delta is FP64 (double *); 1: FP32 (float *),
                         any precision (it is widened or kept as the levels store
                         it; half the bytes of the caller's array).  phi and every
                         other array stay FP64.  The PM steps ignore it (their
                         density is their own FP64 delta_out). */
    int no_sync;      /* 0: the call waits for the stream (residual read per cycle).
                         1: enqueue only, for callers that capture the solve in a HIP
                         graph or pipeline it behind other work: needs tol = 0,
                         profile = 0 and MG_FP64 (mg_solve_dgp, _noalloc, _newton,
                         _kmouflage, _poisson; the adjoint and the PM steps reject it).
                         The call enqueues the same kernels as a tol = 0 solve of
                         max_cycles cycles (initial residual, the cycles, final
                         residual, zero-mean gauge, output) and returns
                         MG_NOT_CONVERGED without waiting; it runs every cycle even if
                         a residual reaches 0.  Nothing is read back: stats.cycles is
                         max_cycles, eps0, eps and lambda are NaN, eps_hist is unset,
                         n_clamped is -1, and non-finite or diverging residuals are
                         not detected.  The launches record no hipMemsetAsync, the
                         call allocates nothing and creates no HIP event (a solve of
                         the same instantiation should have run once before a
                         capture: the first tail launch sets a kernel attribute). */
} mg_opts;

#define MG_HIST 64
#define MG_LEVELS 16
typedef struct {
    int cycles;                 /* cycles run */
    int status;                 /* same as the return value */
    double eps0;                /* residual of the initial guess */
    double eps;                 /* residual of the returned field */
    double eps_hist[MG_HIST];   /* residual after the pre-smoothing of cycle c */
    double lambda;              /* Lagrange multiplier: L(phi) + lambda = 0 */
    long long cell_updates;     /* n^3 * (nu_pre + nu_post) * cycles */
    long long n_clamped;        /* clamped discriminants (nDGP) */
    double seconds;             /* host wall clock of the call */
    double pass_ms_avg;         /* mean finest colour-pass duration (profile=1) */
    int pass_count;             /* number of timed finest colour passes */
    int cycles_fp32;            /* MG_MIXED, MG_FP32: cycles in FP32 storage (included in cycles) */
    double eps_fp32;            /* MG_FP32: residual at the end of the FP32 cycles; MG_MIXED:
                                   the last in-cycle residual of the FP32 phase (a stall
                                   hands over to FP64 without a separate evaluation) */
    double level_ms[MG_LEVELS]; /* profile=1: GPU time of the cycles' work on each level
                                   (0 = finest), summed over all cycles and both precisions;
                                   the levels of the single-workgroup tail (<= 16^3) are
                                   reported together at the tail's first level; the residual
                                   evaluations outside the cycles are not included */
    double pm_ms[4];            /* mg_pm_step, mg_pm_step_kmouflage: GPU time (HIP events on
                                   the stream) of the step's phases: CIC deposit, Newtonian
                                   potential (FFT), scalar-field solve, total potential +
                                   force interpolation + kick-drift */
    int pm_newton_cycles;       /* mg_pm_step*: 0 (the Newtonian potential is solved by FFT) */
} mg_stats;

/* nDGP background (eq:beta_dgp with the LCDM expansion eq:H_lcdm, flat,
 * Omega_L = 1 - Omega_m); h0rc = H0 r_c / c = R_c. */
typedef struct { double a, omega_m, h0rc; } mg_dgp_params;

/* Kmouflage, K(X) = -1 + X + K0 X^n, A = exp(beta phi) (eq:kmf_model_K_function);
 * c~ = (n / box_mpch) * 2997.92458; gamma = n_k K0 (1/(2 a^2 lambda^2))^(n_k-1);
 * background part of Sigma_1 uses (phibar'/H0)^2 = dphibar_dtau_over_h0^2. */
typedef struct {
    int n_k;
    double k0, beta, lambda, a, omega_m, box_mpch, phibar, dphibar_dtau_over_h0;
} mg_kmo_params;

/* Kmouflage background cosmology (Sec. 3.2.5), computed on the host.
 * K(X) = -1 + X + K0 X^n, A = exp(beta phi); flat, matter + radiation.
 * The background field phibar(N), N = ln a, is integrated from z_init with
 * phibar = dphibar/dN = 1e-30, solving the modified Friedmann equation for
 * (aH)^2 at every step, and lambda is shot until H(a = 1) = H0 within
 * htol (relative).  Units H0 = 1. */
typedef struct {
    int n_k;          /* n >= 2 (2..8) */
    double k0;        /* K0 >= 0 */
    double beta;      /* beta_Kmo */
    double omega_m;   /* matter density today */
    double omega_r;   /* radiation density today (see mg_omega_radiation) */
    double z_init;    /* start of the integration, e.g. 1e5 */
    double htol;      /* relative tolerance on H(a=1)/H0, in (0, 1e-2) */
} mg_kmo_bg_params;

typedef struct {
    double lambda;    /* Lambda^4 / (M_Pl^2 H0^2) = lambda^2 of the model */
    double h_miss;    /* H(a=1)/H0 - 1 reached */
    int shots;        /* integrations run by the shooting */
    int steps;        /* Runge-Kutta steps of the tabulating integration */
} mg_kmo_bg_info;

/* Omega_r of photons at t_cmb (K) plus n_eff massless neutrinos for the
 * dimensionless Hubble constant h (Sec. 3.2.5: 2.7255 K, 3.046).  Returns a
 * negative value for invalid arguments. */
double mg_omega_radiation(double h, double t_cmb, double n_eff);

/* Solve the background and tabulate it at the n_table scale factors of
 * a_table (HOST array, strictly increasing within (1/(1+z_init), 1]): hubble
 * = H/H0, hubble_dot = (dH/dt)/H0^2, phibar, dphibar_dtau = (d phibar/d tau)/H0
 * (conformal time; the value mg_kmo_params.dphibar_dtau_over_h0 takes).
 * Outputs are caller-owned HOST arrays of n_table values (n_table may be 0
 * to get lambda only).  No GPU is used.  Errors: MG_ERR_ARG (invalid input,
 * no root of the Friedmann equation, or the shooting did not converge; see
 * mg_last_error). */
mg_status mg_kmo_background(const mg_kmo_bg_params *par, int n_table, const double *a_table,
                            double *hubble, double *hubble_dot, double *phibar,
                            double *dphibar_dtau, mg_kmo_bg_info *info);

/* Linear Poisson model lap(phi) = s * delta (the linearised comparators;
 * the PM steps take the Newtonian potential from mg_fft_poisson). */
typedef struct { double s; } mg_poisson_params;

/* Bytes of device workspace needed by a solve on an n^3 mesh.  precision is
 * an mg_precision, model an mg_model; adjoint != 0 sizes mg_solve_adjoint
 * (FP64 only): per level the linearisation point and the Jacobian's
 * coefficient arrays (9 for Kmouflage, 6 for Poisson), except that the nDGP
 * adjoint keeps only dK/dSigma on levels >= 128^3 (about 52 B per finest
 * cell in all, against 125 for Kmouflage).  Returns 0 for invalid
 * arguments. */
size_t mg_workspace_bytes(int n, int precision, int model, int adjoint);

/* Solve the nDGP scalar-field equation eq:dgp_eom_code in the form of
 * eq:DGP, i.e. L(phi) = lap(phi) - (3/4)[-alpha + sign(alpha) sqrt(alpha^2 +
 * 8 Sigma / 3)] = 0 with Sigma from the discrete operator of Sec. 3.2.3.
 * delta: density contrast (n^3), FP64 or, with opts->delta_fp32 = 1, FP32.
 * phi (FP64): in = initial guess, out = the zero-mean solution.  The periodic
 * discrete problem is solved in bordered form L(phi) + lambda = 0 (lambda in
 * stats). */
mg_status mg_solve_dgp(const mg_opts *opts, const mg_dgp_params *par, const void *delta,
                       double *phi, void *ws, size_t ws_bytes, hipStream_t stream,
                       mg_stats *stats);

/* mg_solve_dgp for callers that cannot allocate (serving loops, harnesses
 * that forbid allocation): same solve, same kernels, same arguments minus the
 * workspace.  The workspace is a static device array of 88 MiB inside the
 * library, one per GPU (the current device's), created when the library's
 * code is loaded on that GPU and held until the process ends.  Limit:
 * opts->n <= 128 in every precision (larger meshes: MG_ERR_ARG; use
 * mg_solve_dgp).  The call allocates nothing -- no device, pinned or managed
 * memory and no HIP events (opts->profile must be 0); it reads each cycle's
 * residual with a plain device-to-host copy.  The array keeps the previous
 * call's contents; every value the solve needs initialised it sets itself
 * with fill kernels on the stream.  Calls that overlap in time on one GPU
 * share the array and race: serialise them (one stream, or host order).
 * stream must belong to the current device. */
mg_status mg_solve_dgp_noalloc(const mg_opts *opts, const mg_dgp_params *par,
                               const void *delta, double *phi, hipStream_t stream,
                               mg_stats *stats);

/* Comparator for the closed-form relaxation: the same nDGP problem written in
 * its quadratic form eq:dgp_quadratic_eom (divided by alpha),
 *   L_N = D + 2 D^2 / (3 alpha) - Sigma / alpha = 0,  D = 7-point Laplacian
 * (centre included), smoothed by the generic Newton-Gauss-Seidel step of
 * eq:relaxation_iteration, u <- u - (L_N - f) / (dL_N/du), with
 * dL_N/du = -(6/h^2)(1 + 4 D / (3 alpha)) -- the iteration Sec. 3.2.3
 * replaces.  Same FAS cycles, transfers, bordering and gauge as mg_solve_dgp;
 * stats.eps is the RMS of the mean-projected L_N residual (equal to the
 * mg_solve_dgp residual to first order in Sigma/alpha^2).  FP64 only; the same
 * kernels as mg_solve_dgp (LDS-tiled on levels >= 128^3) with the Newton step
 * in place of the closed form; same arguments as mg_solve_dgp. */
mg_status mg_solve_dgp_newton(const mg_opts *opts, const mg_dgp_params *par, const void *delta,
                              double *phi, void *ws, size_t ws_bytes, hipStream_t stream,
                              mg_stats *stats);

/* Solve the Kmouflage equation in the split form eq:kmf_eqn_codeunit_final:
 * c~ lap(phi) = (3 beta A Omega_m delta / a + Sigma_2) / Sigma_1.
 * Same argument conventions as mg_solve_dgp. */
mg_status mg_solve_kmouflage(const mg_opts *opts, const mg_kmo_params *par,
                             const void *delta, double *phi, void *ws, size_t ws_bytes,
                             hipStream_t stream, mg_stats *stats);

/* Comparator: coefficient s of the linearised field equation lap(phi) = s
 * delta in code units, for mg_solve_poisson (the linear solves the full
 * equations are compared with).
 *   MG_MODEL_DGP (params mg_dgp_params): dropping the two nonlinear terms
 *     (eq:dgp_linear, phi/2 = Phi_N / (3 beta_DGP) with lap Phi_N =
 *     3/2 Omega_m delta / a) gives s = Omega_m / (a beta_DGP).
 *   MG_MODEL_KMOUFLAGE (params mg_kmo_params, n cells per side for c~):
 *     eq:linearised_Kmo, i.e. Sigma_1 -> K_X of the background and
 *     Sigma_2 -> 0, gives s = 3 beta A(phibar) Omega_m / (a c~ K_X).
 * Host only, no GPU.  Errors: MG_ERR_ARG (null pointer, other model,
 * invalid parameters). */
mg_status mg_linear_source(int model, const void *params, int n, double *s);

/* Solve the linear periodic Poisson equation lap(phi) = s (delta - mean
 * delta) with the same multigrid (zero-mean phi).  Equals the FFT solution
 * with the discrete Green's function of the 7-point Laplacian. */
mg_status mg_solve_poisson(const mg_opts *opts, const mg_poisson_params *par,
                           const void *delta, double *phi, void *ws, size_t ws_bytes,
                           hipStream_t stream, mg_stats *stats);

/* Gradient of loss = sum(phi * w) with respect to delta, phi being the
 * converged zero-mean solution of model (mg_model) with parameters params
 * (mg_dgp_params* or mg_kmo_params*).  Solves the bordered adjoint
 * J^T mu + nu 1 = w, sum(mu) = 0 (J = dL/dphi at phi) by multigrid with the
 * coarse-level linearisation points recomputed by restriction, then
 * grad_delta = -(dL/ddelta) mu.  opts->tol applies to the RMS of the adjoint
 * residual.  mu: in = warm start (zeros if unknown), out = adjoint field.
 * delta as in mg_solve_dgp (FP64, or FP32 with opts->delta_fp32); the other
 * arrays FP64. */
mg_status mg_solve_adjoint(const mg_opts *opts, int model, const void *params,
                           const void *delta, const double *phi, const double *w,
                           double *grad_delta, double *mu, void *ws, size_t ws_bytes,
                           hipStream_t stream, mg_stats *stats);

/* Newtonian potential of the particle-mesh step by FFT (Sec. 3.1): phi =
 * s lap7^{-1} (delta - mean delta), the exact solution of the 7-point
 * discrete Poisson equation lap(phi) = s (delta - mean delta) with zero mean
 * (the Green's function -1 / (4 sum_i sin^2(pi k_i / n)), 0 at k = 0).
 * n^3 FP64 device arrays (16-byte aligned; delta and phi must not alias), n a
 * power of two in [8, 2048]; ws: device workspace of mg_fft_poisson_workspace_bytes(n)
 * (twiddle factors).  Computed as separable Hartley transforms (the Green's
 * function is even in every axis), five passes over phi.  Returns after the
 * stream has finished; MG_ERR_ARG / MG_ERR_WORKSPACE (nothing launched) for
 * invalid arguments. */
size_t mg_fft_poisson_workspace_bytes(int n);
mg_status mg_fft_poisson(int n, double s, const double *delta, double *phi, void *ws,
                         size_t ws_bytes, hipStream_t stream);

/* One nDGP particle-mesh step (Sec. 3.1): CIC density from the particles,
 * Newtonian potential (eq:GR_poisson_codeunit, by mg_fft_poisson; phi_newton
 * is overwritten), scalar field (warm start from
 * phi), total potential Phi_N + phi/2 (eq:poisson_nDGP), 3-point force on
 * the mesh (computed in FP64, kept in FP32 in the workspace) interpolated
 * with CIC, kick dp/da = -(H0/adot) grad Phi at a, drift
 * dx/da = (H0/adot) p / a^2 at a + da/2.  pos in [0, n_mesh) is wrapped.
 * phi_newton and delta_out are 16-byte aligned (MG_ERR_ARG otherwise). */
typedef struct {
    int n_mesh, n_part;
    double omega_m, h0rc, a, da;
    mg_opts mg;   /* options of the scalar-field solve; mg.n must equal n_mesh */
} mg_pm_params;
size_t mg_pm_workspace_bytes(int n_mesh);
mg_status mg_pm_step(const mg_pm_params *par, float *pos, float *mom, double *phi,
                     double *phi_newton, double *delta_out, void *ws, size_t ws_bytes,
                     hipStream_t stream, mg_stats *stats);

/* Host table of a Kmouflage background, as mg_kmo_background returns it:
 * n strictly increasing scale factors a with hubble = H/H0, phibar and
 * dphibar_dtau there, and the model's lambda (mg_kmo_bg_info.lambda).  The
 * caller owns the arrays. */
typedef struct {
    int n;
    const double *a, *hubble, *phibar, *dphibar_dtau;
    double lambda;
} mg_kmo_bg_table;

/* One Kmouflage particle-mesh step (Sec. 3.2.4) from a to a + da: CIC
 * density, Newtonian potential with the rescaled mass,
 * lap Phi_N = 1.5 A(phibar) Omega_m delta / a (eq:kmf_Poission_eqn_codeunit),
 * the scalar field of eq:kmf_eqn_codeunit_final (warm start from phi), and
 * eq:force_Kmo1/2: kick
 * p <- (1 - beta (d phibar/da) da) p - (da / (a E(a))) grad(Phi_N + beta c~ phi)
 * at a, drift x += da / (a_h^3 E(a_h)) p at a_h = a + da/2 (a_h <= 1).  The
 * library derives every background value the step needs -- lambda, phibar
 * and its conformal-time derivative at a, E at a and a_h, and
 * d phibar/da = (d phibar/d tau) / (a^2 E(a)) -- from the background of bg:
 * looked up in table when given (it must hold a and a_h, relative match
 * 1e-12), otherwise solved by the library for this step (as
 * mg_kmo_background does, a few ms of host time).  c~ = (n_mesh / box_mpch)
 * c/H0.  Same arrays and workspace as mg_pm_step. */
typedef struct {
    int n_mesh, n_part;
    double a, da;
    double box_mpch;
    mg_kmo_bg_params bg;           /* model (n_k, K0, beta) and background cosmology */
    const mg_kmo_bg_table *table;  /* HOST, optional (NULL: solve the background here) */
    mg_opts mg;                    /* options of the scalar-field solve; mg.n must equal n_mesh */
} mg_pm_kmo_params;
mg_status mg_pm_step_kmouflage(const mg_pm_kmo_params *par, float *pos, float *mom, double *phi,
                               double *phi_newton, double *delta_out, void *ws, size_t ws_bytes,
                               hipStream_t stream, mg_stats *stats);

/* CIC density contrast of n_part^3 unit-mass particles on an n_mesh^3
 * mesh (cell i has centre i + 1/2): delta = rho / rho_bar - 1.  Deterministic:
 * weights accumulate as 64-bit fixed point (2^-32 per unit mass).  ws needs
 * mg_pm_workspace_bytes(n_mesh) bytes. */
mg_status mg_cic_delta(int n_mesh, int n_part, const float *pos, double *delta, void *ws,
                       size_t ws_bytes, hipStream_t stream);
/* The same deposit with an FP32 delta (each value the FP64 one rounded once),
 * for solves with opts.delta_fp32 = 1. */
mg_status mg_cic_delta_f32(int n_mesh, int n_part, const float *pos, float *delta, void *ws,
                           size_t ws_bytes, hipStream_t stream);

/* ---- single operations of the solve, for parity tests ------------------
 * Natural-layout device arrays of n^3 FP64; level spacing h; model/params
 * as in mg_solve_adjoint; f: device array or NULL for the scalar fs.
 * ws needs mg_op_workspace_bytes(n). */
size_t mg_op_workspace_bytes(int n);
/* out = L_h(phi) - f */
mg_status mg_op_residual(int model, const void *params, int n, double h, const double *phi,
                         const double *delta, const double *f, double fs, double *out,
                         void *ws, size_t ws_bytes, hipStream_t stream);
/* one colour pass (colour 0: (i+j+k) even) from phi_in to phi_out */
mg_status mg_op_colour_pass(int model, const void *params, int n, double h, int colour,
                            const double *phi_in, const double *delta, const double *f,
                            double fs, double *phi_out, void *ws, size_t ws_bytes,
                            hipStream_t stream);
/* coarse = 8-cell mean of fine (n = fine cells per side) */
mg_status mg_op_restrict(int n, const double *fine, double *coarse, void *ws, size_t ws_bytes,
                         hipStream_t stream);
/* fine += P(uc - rc) (n = fine cells per side) */
mg_status mg_op_prolong_add(int n, double *fine, const double *uc, const double *rc, void *ws,
                            size_t ws_bytes, hipStream_t stream);
/* out = J^T v, J = dL/dphi at (phi, delta) */
mg_status mg_op_jt_apply(int model, const void *params, int n, double h, const double *phi,
                         const double *delta, const double *v, double *out, void *ws,
                         size_t ws_bytes, hipStream_t stream);

const char *mg_status_string(mg_status s);
/* Detail of the last error on the calling thread ("" if none). */
const char *mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MGGLAM_H */
