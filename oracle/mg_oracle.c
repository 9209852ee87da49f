/*
 * FP64 CPU oracle for the MG-GLAM derivative-coupling multigrid solve
 * (Hernandez-Aguayo et al., arXiv:2110.00566).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code with
 * the HIP path and follows the paper's equations in their printed form:
 *
 *   - nDGP operator: eq. for L^h with the long-form Sigma_ijk (Sec. 3.2.3),
 *     closed-form root eq:DGP with sign(alpha), update eq:nonlinear_GS_DGP.
 *   - Kmouflage operator: eq:kmf_eqn_codeunit_final with Sigma_1, Sigma_2 and
 *     the discrete hat-Hessian contraction of Sec. 3.2.4 (cross-term
 *     coefficient read as 1/(8h^4), the continuum-consistent value).
 *   - Multigrid: relaxation eq:relaxation_iteration, FAS coarse equation
 *     eq:general_pde_numerical_coarse, 8-cell mean restriction, 27/9/3/1
 *     prolongation with eq:solution_correction, coarsest level 4^3 (Sec. 3.2.1).
 *   - Cycle arrangements of Sec. 3.2.1 and fig:multigrid_cycles, as the
 *     textbook recursions: V = one coarse cycle per level, W = two, F = an
 *     F-cycle followed by a V-cycle on the coarse problem; every visit of the
 *     coarsest level is nu_c sweeps.
 *
 * Readings where the paper is silent (all shared with the GPU path by
 * specification, never by code):
 *   - periodic solvability: the finest equation is L(phi) = mu with mu the
 *     mean of L(phi), refreshed once per cycle at the in-cycle residual; the
 *     returned phi has zero mean;
 *   - red-black ordering: colour 0 = (i+j+k) even first, and each colour pass
 *     updates all cells of the colour from the state at the start of the pass
 *     (the 19-point stencil couples same-colour edge neighbours);
 *   - a negative discriminant is clamped to 0 and counted.
 *
 * Layout: natural C order a[k][j][i] (x fastest), periodic in all axes.
 * Every function is plain loops; OpenMP only splits the outer z loop and all
 * reductions are summed per z-plane and then in plane order, so results do
 * not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_LEVELS 16
#define OR_HIST 256

typedef struct {
    int model;      /* 0 nDGP, 1 Kmouflage, 2 linear Poisson L = lap(phi) - s*delta */
    double alpha;   /* nDGP alpha = 3 beta a^2 / R_c^2 */
    double sgn;     /* sign(alpha), 1 for alpha >= 0 */
    double s;       /* nDGP: (alpha/beta) Omega_m / a ; linear: source factor */
    double ctil;    /* Kmouflage c~ = (N/L) c/H0 */
    double gamma;   /* n K0 (1/(2 a^2 lambda^2))^(n-1) */
    double C0;      /* 1 + gamma b^(n-1), b = (phibar'/H0)^2 */
    double src;     /* 3 beta A(phibar) Omega_m / a */
    int nk;         /* Kmouflage exponent n */
} or_model;

typedef struct {
    int cycles;
    double eps0, eps, mu;
    double hist[OR_HIST];
    long long nclamp;
    int status;     /* 0 converged, 1 cycle cap, -3 non-finite, -4 diverged */
} or_stats;

/* ------------------------------------------------------------------ */
/* model set-up                                                        */
/* ------------------------------------------------------------------ */

/* eq:beta_dgp with the LCDM expansion eq:H_lcdm, Omega_rc = 1/(4 R_c^2),
 * R_c = H0 r_c / c; alpha and the source factor from the definitions that
 * follow eq:dgp_quadratic_eom. */
void or_dgp_setup(double a, double omega_m, double h0rc, or_model *m, double *beta_out)
{
    double omega_l = 1.0 - omega_m;
    double omega_rc = 1.0 / (4.0 * h0rc * h0rc);
    double num = omega_m / (a * a * a) + 2.0 * omega_l;
    double den = 2.0 * sqrt(omega_rc * (omega_m / (a * a * a) + omega_l));
    double beta = 1.0 + num / den;
    memset(m, 0, sizeof(*m));
    m->model = 0;
    m->alpha = 3.0 * beta * a * a / (h0rc * h0rc);
    m->sgn = m->alpha >= 0.0 ? 1.0 : -1.0;
    m->s = m->alpha / beta * omega_m / a;
    if (beta_out) *beta_out = beta;
}

/* Sec. 3.2.4: c~ = c N_g / (H0 L) with c/H0 = 2997.92458 Mpc/h,
 * gamma = n K0 (1/(2 a^2 lambda^2))^(n-1), Sigma_1's background part
 * 1 + gamma (phibar'/H0)^(2(n-1)), source 3 dA/dphi(phibar) Omega_m / a with
 * A = exp(beta phi). */
void or_kmo_setup(int n_mesh, double box_mpch, int nk, double k0, double beta,
                  double lambda, double a, double omega_m, double phibar,
                  double dphibar_over_h0, or_model *m)
{
    double x0 = 1.0 / (2.0 * a * a * lambda * lambda);
    double b = dphibar_over_h0 * dphibar_over_h0;
    double gpow = 1.0, bpow = 1.0;
    for (int q = 0; q < nk - 1; ++q) { gpow *= x0; bpow *= b; }
    memset(m, 0, sizeof(*m));
    m->model = 1;
    m->nk = nk;
    m->ctil = (double)n_mesh / box_mpch * 2997.92458;
    m->gamma = nk * k0 * gpow;
    m->C0 = 1.0 + m->gamma * bpow;
    m->src = 3.0 * beta * exp(beta * phibar) * omega_m / a;
}

/* Comparator: the nDGP problem in the quadratic form eq:dgp_quadratic_eom,
 * divided by alpha, relaxed by the generic Newton-Gauss-Seidel step of
 * eq:relaxation_iteration (model 3): L = lap(phi) - K with
 * K = Sigma/alpha - 2 (lap phi)^2 / (3 alpha), which depends on the centre. */
void or_dgp_newton_setup(double a, double omega_m, double h0rc, or_model *m)
{
    or_dgp_setup(a, omega_m, h0rc, m, NULL);
    m->model = 3;
}

void or_linear_setup(double s, or_model *m)
{
    memset(m, 0, sizeof(*m));
    m->model = 2;
    m->s = s;
}

/* ------------------------------------------------------------------ */
/* the discrete operator                                               */
/* ------------------------------------------------------------------ */

static inline int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
static inline long IX(int n, int i, int j, int k)
{
    return ((long)wrap(k, n) * n + wrap(j, n)) * n + wrap(i, n);
}

static double ipow(double x, int p)
{
    double r = 1.0;
    for (int q = 0; q < p; ++q) r *= x;
    return r;
}

/* The non-Laplacian part of L^h at one cell, i.e. L^h = lap_h(phi) - K. */
static double model_term(const or_model *m, const double *phi, const double *delta,
                         int n, double h, int i, int j, int k, long long *nclamp)
{
    double c = phi[IX(n, i, j, k)];
    double xp = phi[IX(n, i + 1, j, k)], xm = phi[IX(n, i - 1, j, k)];
    double yp = phi[IX(n, i, j + 1, k)], ym = phi[IX(n, i, j - 1, k)];
    double zp = phi[IX(n, i, j, k + 1)], zm = phi[IX(n, i, j, k - 1)];
    double d = delta[IX(n, i, j, k)];
    double h4 = h * h * h * h;
    if (m->model == 2)
        return m->s * d;
    if (m->model == 0 || m->model == 3) {
        /* Sigma_ijk exactly as printed (Sec. 3.2.3) */
        double dxx = xp + xm - 2.0 * c;
        double dyy = yp + ym - 2.0 * c;
        double dzz = zp + zm - 2.0 * c;
        double nxy = phi[IX(n, i + 1, j + 1, k)] + phi[IX(n, i - 1, j - 1, k)]
                   - phi[IX(n, i + 1, j - 1, k)] - phi[IX(n, i - 1, j + 1, k)];
        double nxz = phi[IX(n, i + 1, j, k + 1)] + phi[IX(n, i - 1, j, k - 1)]
                   - phi[IX(n, i + 1, j, k - 1)] - phi[IX(n, i - 1, j, k + 1)];
        double nyz = phi[IX(n, i, j + 1, k + 1)] + phi[IX(n, i, j - 1, k - 1)]
                   - phi[IX(n, i, j + 1, k - 1)] - phi[IX(n, i, j - 1, k + 1)];
        double sigma = 2.0 / (3.0 * h4) * (dxx * dxx + dyy * dyy + dzz * dzz)
                     - 2.0 / (3.0 * h4) * dxx * dyy
                     - 2.0 / (3.0 * h4) * dxx * dzz
                     - 2.0 / (3.0 * h4) * dyy * dzz
                     + 1.0 / (8.0 * h4) * nxy * nxy
                     + 1.0 / (8.0 * h4) * nxz * nxz
                     + 1.0 / (8.0 * h4) * nyz * nyz
                     + m->s * d;
        if (m->model == 3) {
            double D = (xp + xm + yp + ym + zp + zm - 6.0 * c) / (h * h);
            return sigma / m->alpha - 2.0 * D * D / (3.0 * m->alpha);
        }
        double disc = m->alpha * m->alpha + 8.0 / 3.0 * sigma;
        if (disc < 0.0) {
            disc = 0.0;
            if (nclamp) ++*nclamp;
        }
        /* eq:DGP */
        return 0.75 * (-m->alpha + m->sgn * sqrt(disc));
    }
    /* Kmouflage, eq:kmf_eqn_codeunit_final */
    {
        double ex = xp - xm, ey = yp - ym, ez = zp - zm;   /* 2h * gradient */
        double gx = ex / (2.0 * h), gy = ey / (2.0 * h), gz = ez / (2.0 * h);
        double g = gx * gx + gy * gy + gz * gz;
        double nxy = phi[IX(n, i + 1, j + 1, k)] + phi[IX(n, i - 1, j - 1, k)]
                   - phi[IX(n, i + 1, j - 1, k)] - phi[IX(n, i - 1, j + 1, k)];
        double nxz = phi[IX(n, i + 1, j, k + 1)] + phi[IX(n, i - 1, j, k - 1)]
                   - phi[IX(n, i + 1, j, k - 1)] - phi[IX(n, i - 1, j, k + 1)];
        double nyz = phi[IX(n, i, j + 1, k + 1)] + phi[IX(n, i, j - 1, k - 1)]
                   - phi[IX(n, i, j + 1, k - 1)] - phi[IX(n, i, j - 1, k + 1)];
        /* discrete hat-Hessian contraction with the gradient */
        double q = 1.0 / (12.0 * h4) * ex * ex * (2.0 * xp + 2.0 * xm - yp - ym - zp - zm)
                 + 1.0 / (12.0 * h4) * ey * ey * (2.0 * yp + 2.0 * ym - xp - xm - zp - zm)
                 + 1.0 / (12.0 * h4) * ez * ez * (2.0 * zp + 2.0 * zm - xp - xm - yp - ym)
                 + 1.0 / (8.0 * h4) * nxy * ex * ey
                 + 1.0 / (8.0 * h4) * nxz * ex * ez
                 + 1.0 / (8.0 * h4) * nyz * ey * ez;
        int nk = m->nk;
        double sig1 = m->C0 + (2.0 * nk + 1.0) * m->gamma / 3.0 * ipow(g, nk - 1);
        double sig2 = -2.0 * m->ctil * (nk - 1) * m->gamma * ipow(g, nk - 2) * q;
        return (m->src * d + sig2) / (m->ctil * sig1);
    }
}

static double lap(const double *phi, int n, double h, int i, int j, int k)
{
    double sum = phi[IX(n, i + 1, j, k)] + phi[IX(n, i - 1, j, k)]
               + phi[IX(n, i, j + 1, k)] + phi[IX(n, i, j - 1, k)]
               + phi[IX(n, i, j, k + 1)] + phi[IX(n, i, j, k - 1)];
    return (sum - 6.0 * phi[IX(n, i, j, k)]) / (h * h);
}

double or_op_cell(const or_model *m, const double *phi, const double *delta, int n,
                  double h, int i, int j, int k)
{
    return lap(phi, n, h, i, j, k) - model_term(m, phi, delta, n, h, i, j, k, NULL);
}

/* L^h(phi) - f at every cell (f array, or the scalar fs when f is NULL). */
void or_residual(const or_model *m, const double *phi, const double *delta,
                 const double *f, double fs, int n, double h, double *out,
                 long long *nclamp)
{
    long long nc = 0;
#pragma omp parallel for reduction(+ : nc) schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long c = IX(n, i, j, k);
                double L = lap(phi, n, h, i, j, k)
                         - model_term(m, phi, delta, n, h, i, j, k, &nc);
                out[c] = L - (f ? f[c] : fs);
            }
    if (nclamp) *nclamp += nc;
}

/* One colour pass of the nonlinear Gauss-Seidel update
 * phi_new = phi_old - (L - f)/(dL/dphi), dL/dphi = -6/h^2, applied to the
 * cells with (i+j+k)%2 == colour, all from the state at the start of the pass. */
void or_colour_pass(const or_model *m, const double *phi_in, const double *delta,
                    const double *f, double fs, int n, double h, int colour,
                    double *phi_out, long long *nclamp)
{
    long long nc = 0;
    memcpy(phi_out, phi_in, sizeof(double) * (size_t)n * n * n);
#pragma omp parallel for reduction(+ : nc) schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                if (((i + j + k) & 1) != colour) continue;
                long c = IX(n, i, j, k);
                double D = lap(phi_in, n, h, i, j, k);
                double L = D - model_term(m, phi_in, delta, n, h, i, j, k, &nc);
                /* dL/dphi at the cell: the closed-form models do not depend on
                 * the centre through K; the quadratic form does through D */
                double dLdphi = -6.0 / (h * h);
                if (m->model == 3) dLdphi *= 1.0 + 4.0 * D / (3.0 * m->alpha);
                phi_out[c] = phi_in[c] - (L - (f ? f[c] : fs)) / dLdphi;
            }
    if (nclamp) *nclamp += nc;
}

/* Restriction: arithmetic mean of the 8 children (Sec. 3.2.1). */
void or_restrict(const double *fine, int nf, double *coarse)
{
    int nc = nf / 2;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < nc; ++K)
        for (int J = 0; J < nc; ++J)
            for (int I = 0; I < nc; ++I) {
                double s = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            s += fine[IX(nf, 2 * I + a, 2 * J + b, 2 * K + c)];
                coarse[IX(nc, I, J, K)] = s / 8.0;
            }
}

/* Prolongation of (uc - rc) with weights 27/64 (parent), 9/64 (3 face),
 * 3/64 (3 edge), 1/64 (vertex), added to the fine field
 * (eq:solution_correction).  The neighbours lie on the side of the parent
 * that the fine cell occupies. */
void or_prolong_add(double *fine, int nf, const double *uc, const double *rc)
{
    int nc = nf / 2;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nf; ++k)
        for (int j = 0; j < nf; ++j)
            for (int i = 0; i < nf; ++i) {
                int I = i / 2, J = j / 2, K = k / 2;
                int di = (i % 2) ? 1 : -1, dj = (j % 2) ? 1 : -1, dk = (k % 2) ? 1 : -1;
                double acc = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            double wx = a ? 1.0 : 3.0, wy = b ? 1.0 : 3.0, wz = c ? 1.0 : 3.0;
                            long q = IX(nc, I + a * di, J + b * dj, K + c * dk);
                            acc += wx * wy * wz / 64.0 * (uc[q] - rc[q]);
                        }
                fine[IX(nf, i, j, k)] += acc;
            }
}

/* Plane-ordered sums so the result does not depend on the thread count. */
static void sums(const double *a, long n3, int n, double *s1, double *s2)
{
    long plane = n3 / n;
    double *p1 = malloc(sizeof(double) * n), *p2 = malloc(sizeof(double) * n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        double x1 = 0.0, x2 = 0.0;
        for (long c = (long)k * plane; c < (long)(k + 1) * plane; ++c) {
            x1 += a[c];
            x2 += a[c] * a[c];
        }
        p1[k] = x1;
        p2[k] = x2;
    }
    double t1 = 0.0, t2 = 0.0;
    for (int k = 0; k < n; ++k) { t1 += p1[k]; t2 += p2[k]; }
    free(p1);
    free(p2);
    *s1 = t1;
    *s2 = t2;
}

double or_mean(const double *a, int n)
{
    double s1, s2;
    long n3 = (long)n * n * n;
    sums(a, n3, n, &s1, &s2);
    return s1 / (double)n3;
}

/* ------------------------------------------------------------------ */
/* FAS V-cycle and driver                                              */
/* ------------------------------------------------------------------ */

typedef struct {
    int nlev;
    int n[OR_MAX_LEVELS];
    double h[OR_MAX_LEVELS];
    double *delta[OR_MAX_LEVELS];   /* level 0 points at the caller's delta */
    double *u[OR_MAX_LEVELS];       /* level 0 points at the caller's phi */
    double *f[OR_MAX_LEVELS];       /* coarse FAS source S; unused on level 0 */
    double *ru[OR_MAX_LEVELS];      /* R u of the finer level */
    double *tmp[OR_MAX_LEVELS];
    double *res[OR_MAX_LEVELS];
    double mu;                      /* finest right-hand side (lagged mean L) */
    int nu1, nu2, nuc;
    long long nclamp;
    int *trace;                     /* optional: level of every smoothing visit */
    int ntrace, trace_cap;
} or_hier;

static int hier_init(or_hier *H, int n, double h0, const double *delta, double *phi)
{
    memset(H, 0, sizeof(*H));
    int L = 0;
    for (int m = n; m >= 4; m /= 2) {
        if (L >= OR_MAX_LEVELS) return -1;
        H->n[L] = m;
        H->h[L] = h0 * (double)n / m;
        ++L;
    }
    H->nlev = L;
    for (int l = 0; l < L; ++l) {
        size_t c = (size_t)H->n[l] * H->n[l] * H->n[l];
        if (l == 0) {
            H->delta[0] = (double *)delta;
            H->u[0] = phi;
        } else {
            H->delta[l] = malloc(sizeof(double) * c);
            H->u[l] = malloc(sizeof(double) * c);
            H->f[l] = malloc(sizeof(double) * c);
            H->ru[l] = malloc(sizeof(double) * c);
            or_restrict(H->delta[l - 1], H->n[l - 1], H->delta[l]);
        }
        H->tmp[l] = malloc(sizeof(double) * c);
        H->res[l] = malloc(sizeof(double) * c);
    }
    return 0;
}

static void hier_free(or_hier *H)
{
    for (int l = 0; l < H->nlev; ++l) {
        if (l > 0) {
            free(H->delta[l]);
            free(H->u[l]);
            free(H->f[l]);
            free(H->ru[l]);
        }
        free(H->tmp[l]);
        free(H->res[l]);
    }
}

static void sweep(const or_model *m, or_hier *H, int l)
{
    size_t c = (size_t)H->n[l] * H->n[l] * H->n[l];
    for (int colour = 0; colour < 2; ++colour) {
        or_colour_pass(m, H->u[l], H->delta[l], l ? H->f[l] : NULL, H->mu, H->n[l],
                       H->h[l], colour, H->tmp[l], &H->nclamp);
        memcpy(H->u[l], H->tmp[l], sizeof(double) * c);
    }
}

/* Finest-level residual statistics: mu = mean L(phi), eps = RMS(L - mu). */
static void finest_stats(const or_model *m, or_hier *H, double *mu, double *eps)
{
    int n = H->n[0];
    long n3 = (long)n * n * n;
    double s1, s2;
    or_residual(m, H->u[0], H->delta[0], NULL, 0.0, n, H->h[0], H->res[0], &H->nclamp);
    sums(H->res[0], n3, n, &s1, &s2);
    *mu = s1 / (double)n3;
    for (long c = 0; c < n3; ++c) H->res[0][c] -= *mu;
    sums(H->res[0], n3, n, &s1, &s2);
    *eps = sqrt(s2 / (double)n3);
}

static void visit(or_hier *H, int l)
{
    if (H->trace && H->ntrace < H->trace_cap) H->trace[H->ntrace] = l;
    if (H->trace) ++H->ntrace;
}

/* One cycle of type 0 (V), 1 (F) or 2 (W) on level l. */
static void mgcycle(const or_model *m, or_hier *H, int l, int type, double *eps_mid)
{
    int n = H->n[l];
    size_t c = (size_t)n * n * n;
    visit(H, l);
    if (l == H->nlev - 1) {
        for (int s = 0; s < H->nuc; ++s) sweep(m, H, l);
        return;
    }
    for (int s = 0; s < H->nu1; ++s) sweep(m, H, l);
    /* local residual d = L(u) - f; on the finest level f = mu is refreshed
     * to the mean of L(u) first */
    if (l == 0) {
        double mu, eps;
        finest_stats(m, H, &mu, &eps);   /* leaves res[0] = L - mu */
        H->mu = mu;
        if (eps_mid) *eps_mid = eps;
    } else {
        or_residual(m, H->u[l], H->delta[l], H->f[l], 0.0, n, H->h[l], H->res[l], &H->nclamp);
    }
    int lc = l + 1;
    int ncs = H->n[lc];
    size_t cc = (size_t)ncs * ncs * ncs;
    or_restrict(H->u[l], n, H->ru[lc]);
    or_restrict(H->res[l], n, H->tmp[lc]);              /* R d */
    /* S = L^H(R u) - R d */
    or_residual(m, H->ru[lc], H->delta[lc], NULL, 0.0, ncs, H->h[lc], H->f[lc], &H->nclamp);
    for (size_t q = 0; q < cc; ++q) H->f[lc][q] -= H->tmp[lc][q];
    memcpy(H->u[lc], H->ru[lc], sizeof(double) * cc);  /* initial guess R u */
    if (type == 2) {               /* W: two coarse W-cycles */
        mgcycle(m, H, lc, 2, NULL);
        mgcycle(m, H, lc, 2, NULL);
    } else if (type == 1) {        /* F: a coarse F-cycle, then a coarse V-cycle */
        mgcycle(m, H, lc, 1, NULL);
        mgcycle(m, H, lc, 0, NULL);
    } else {
        mgcycle(m, H, lc, 0, NULL);
    }
    or_prolong_add(H->u[l], n, H->u[lc], H->ru[lc]);
    visit(H, l);
    for (int s = 0; s < H->nu2; ++s) sweep(m, H, l);
    (void)c;
}

/* Solve the model equation for phi (in: initial guess, out: zero-mean
 * solution) on an n^3 mesh of spacing h0 (1 in code units).  tol is the absolute RMS of the mean-projected finest residual.
 * Returns the status code stored in st->status. */
/* Solve with cycles of the given type (0 V, 1 F, 2 W).  trace (may be NULL)
 * receives the level of every smoothing visit, at most trace_cap entries;
 * *ntrace the number of visits. */
int or_solve_cycle(const or_model *m, int n, double h0, const double *delta, double *phi,
                   int max_cycles, double tol, int nu1, int nu2, int nuc, int cycle,
                   int *trace, int trace_cap, int *ntrace, or_stats *st)
{
    or_hier H;
    memset(st, 0, sizeof(*st));
    if (cycle < 0 || cycle > 2) return -1;
    if (hier_init(&H, n, h0, delta, phi)) return -1;
    H.nu1 = nu1;
    H.nu2 = nu2;
    H.nuc = nuc;
    H.trace = trace;
    H.trace_cap = trace_cap;
    H.ntrace = 0;
    double mu, eps;
    finest_stats(m, &H, &mu, &eps);
    H.mu = mu;
    st->eps0 = eps;
    st->status = 1;
    double best = eps;
    int cyc = 0;
    if (eps <= tol) st->status = 0;
    else {
        for (cyc = 1; cyc <= max_cycles; ++cyc) {
            double eps_mid = 0.0;
            mgcycle(m, &H, 0, cycle, &eps_mid);
            if (cyc - 1 < OR_HIST) st->hist[cyc - 1] = eps_mid;
            if (!isfinite(eps_mid)) { st->status = -3; break; }
            if (eps_mid > 1e3 * best) { st->status = -4; break; }
            if (eps_mid < best) best = eps_mid;
            if (eps_mid <= tol || cyc == max_cycles) {
                finest_stats(m, &H, &mu, &eps);
                H.mu = mu;
                if (eps <= tol) { st->status = 0; break; }
            }
        }
        if (cyc > max_cycles) cyc = max_cycles;
    }
    st->cycles = cyc;
    st->eps = eps;
    st->mu = H.mu;
    double mean = or_mean(phi, n);
    long n3 = (long)n * n * n;
    for (long q = 0; q < n3; ++q) phi[q] -= mean;
    st->nclamp = H.nclamp;
    if (ntrace) *ntrace = H.ntrace;
    hier_free(&H);
    return st->status;
}

int or_solve(const or_model *m, int n, double h0, const double *delta, double *phi,
             int max_cycles, double tol, int nu1, int nu2, int nuc, or_stats *st)
{
    return or_solve_cycle(m, n, h0, delta, phi, max_cycles, tol, nu1, nu2, nuc, 0, NULL, 0, NULL,
                          st);
}

/* Exposed single V-cycle building blocks for tests: one sweep on one level
 * with a given f (array or scalar). */
void or_sweep(const or_model *m, double *phi, const double *delta, const double *f,
              double fs, int n, double h, double *work)
{
    size_t c = (size_t)n * n * n;
    for (int colour = 0; colour < 2; ++colour) {
        or_colour_pass(m, phi, delta, f, fs, n, h, colour, work, NULL);
        memcpy(phi, work, sizeof(double) * c);
    }
}

/* ------------------------------------------------------------------ */
/* adjoint                                                             */
/* ------------------------------------------------------------------ */
/*
 * J = dL/dphi at a linearisation point (phi*, delta).  The diagonal is
 * -6/h^2 for both models (the model term has no centre dependence).  The
 * transpose is applied by scattering every row of J: (J^T mu)_p =
 * sum_m J_mp mu_m.  Row m of J has entries on the 6 face and 12 edge
 * neighbours of m, obtained by differentiating the model term above.
 */

/* derivative of the model term K at cell m w.r.t. its 18 neighbours.
 * out[0..5]: faces x+ x- y+ y- z+ z-; out[6..17]: edges
 * xy: (+,+) (-,-) (+,-) (-,+), xz: same, yz: same. */
static void model_term_grad(const or_model *m, const double *phi, const double *delta,
                            int n, double h, int i, int j, int k, double out[18])
{
    double xp = phi[IX(n, i + 1, j, k)], xm = phi[IX(n, i - 1, j, k)];
    double yp = phi[IX(n, i, j + 1, k)], ym = phi[IX(n, i, j - 1, k)];
    double zp = phi[IX(n, i, j, k + 1)], zm = phi[IX(n, i, j, k - 1)];
    double c = phi[IX(n, i, j, k)];
    double d = delta[IX(n, i, j, k)];
    double h2 = h * h, h4 = h2 * h2;
    double nxy = phi[IX(n, i + 1, j + 1, k)] + phi[IX(n, i - 1, j - 1, k)]
               - phi[IX(n, i + 1, j - 1, k)] - phi[IX(n, i - 1, j + 1, k)];
    double nxz = phi[IX(n, i + 1, j, k + 1)] + phi[IX(n, i - 1, j, k - 1)]
               - phi[IX(n, i + 1, j, k - 1)] - phi[IX(n, i - 1, j, k + 1)];
    double nyz = phi[IX(n, i, j + 1, k + 1)] + phi[IX(n, i, j - 1, k - 1)]
               - phi[IX(n, i, j + 1, k - 1)] - phi[IX(n, i, j - 1, k + 1)];
    memset(out, 0, sizeof(double) * 18);
    if (m->model == 2) return;
    if (m->model == 0) {
        double dxx = xp + xm - 2.0 * c, dyy = yp + ym - 2.0 * c, dzz = zp + zm - 2.0 * c;
        double sigma = 2.0 / (3.0 * h4) * (dxx * dxx + dyy * dyy + dzz * dzz - dxx * dyy
                                           - dxx * dzz - dyy * dzz)
                     + 1.0 / (8.0 * h4) * (nxy * nxy + nxz * nxz + nyz * nyz) + m->s * d;
        double disc = m->alpha * m->alpha + 8.0 / 3.0 * sigma;
        /* dF/dSigma = sign(alpha)/sqrt(D); zero on the clamped branch */
        double fp = disc > 0.0 ? m->sgn / sqrt(disc) : 0.0;
        /* dSigma/dphi_(i+-1): 2/(3h^4) (2 dxx - dyy - dzz), etc. */
        double cx = fp * 2.0 / (3.0 * h4) * (2.0 * dxx - dyy - dzz);
        double cy = fp * 2.0 / (3.0 * h4) * (2.0 * dyy - dxx - dzz);
        double cz = fp * 2.0 / (3.0 * h4) * (2.0 * dzz - dxx - dyy);
        double exy = fp * nxy / (4.0 * h4), exz = fp * nxz / (4.0 * h4), eyz = fp * nyz / (4.0 * h4);
        out[0] = out[1] = cx;
        out[2] = out[3] = cy;
        out[4] = out[5] = cz;
        out[6] = exy; out[7] = exy; out[8] = -exy; out[9] = -exy;
        out[10] = exz; out[11] = exz; out[12] = -exz; out[13] = -exz;
        out[14] = eyz; out[15] = eyz; out[16] = -eyz; out[17] = -eyz;
        return;
    }
    {
        int nk = m->nk;
        double gx = (xp - xm) / (2.0 * h), gy = (yp - ym) / (2.0 * h), gz = (zp - zm) / (2.0 * h);
        double g = gx * gx + gy * gy + gz * gz;
        double hxx = (2.0 * xp + 2.0 * xm - yp - ym - zp - zm) / (3.0 * h2);
        double hyy = (2.0 * yp + 2.0 * ym - xp - xm - zp - zm) / (3.0 * h2);
        double hzz = (2.0 * zp + 2.0 * zm - xp - xm - yp - ym) / (3.0 * h2);
        double dxy = nxy / (4.0 * h2), dxz = nxz / (4.0 * h2), dyz = nyz / (4.0 * h2);
        double q = hxx * gx * gx + hyy * gy * gy + hzz * gz * gz
                 + 2.0 * (dxy * gx * gy + dxz * gx * gz + dyz * gy * gz);
        double a1 = (2.0 * nk + 1.0) * m->gamma / 3.0;
        double sig1 = m->C0 + a1 * ipow(g, nk - 1);
        double b2 = -2.0 * m->ctil * (nk - 1) * m->gamma;
        double sig2 = b2 * ipow(g, nk - 2) * q;
        double num = m->src * d + sig2;
        /* K = num / (ctil sig1) */
        double dsig1_dg = (nk >= 2) ? a1 * (nk - 1) * ipow(g, nk - 2) : 0.0;
        double dsig2_dg = (nk >= 3) ? b2 * (nk - 2) * ipow(g, nk - 3) * q : 0.0;
        double dsig2_dq = b2 * ipow(g, nk - 2);
        /* face derivatives: dg/dphi_(x+-) = +-gx/h,
         * dq/dphi_(x+-) = (2gx^2-gy^2-gz^2)/(3h^2) +- (hxx gx + dxy gy + dxz gz)/h */
        double gg[3] = {gx, gy, gz};
        double diag[3] = {(2 * gx * gx - gy * gy - gz * gz) / (3.0 * h2),
                          (2 * gy * gy - gx * gx - gz * gz) / (3.0 * h2),
                          (2 * gz * gz - gx * gx - gy * gy) / (3.0 * h2)};
        double lin[3] = {(hxx * gx + dxy * gy + dxz * gz) / h,
                         (dxy * gx + hyy * gy + dyz * gz) / h,
                         (dxz * gx + dyz * gy + hzz * gz) / h};
        for (int ax = 0; ax < 3; ++ax)
            for (int sgn = 0; sgn < 2; ++sgn) {
                double sg = sgn ? -1.0 : 1.0;
                double dg = sg * gg[ax] / h;
                double dq = diag[ax] + sg * lin[ax];
                double dsig1 = dsig1_dg * dg;
                double dsig2 = dsig2_dg * dg + dsig2_dq * dq;
                out[2 * ax + sgn] = (dsig2 * sig1 - num * dsig1) / (m->ctil * sig1 * sig1);
            }
        /* edges only enter q: dq/dphi_(+,+) = 2 gx gy /(4h^2) */
        double exy = dsig2_dq * (gx * gy / (2.0 * h2)) / (m->ctil * sig1);
        double exz = dsig2_dq * (gx * gz / (2.0 * h2)) / (m->ctil * sig1);
        double eyz = dsig2_dq * (gy * gz / (2.0 * h2)) / (m->ctil * sig1);
        out[6] = exy; out[7] = exy; out[8] = -exy; out[9] = -exy;
        out[10] = exz; out[11] = exz; out[12] = -exz; out[13] = -exz;
        out[14] = eyz; out[15] = eyz; out[16] = -eyz; out[17] = -eyz;
    }
}

static const int NB[18][3] = {
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* d K_m / d phi_p for the 18 neighbours of every cell (rows of J minus the
 * Laplacian), stored [cell][18]. */
void or_jac_rows(const or_model *m, const double *phi, const double *delta, int n,
                 double h, double *rows)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                model_term_grad(m, phi, delta, n, h, i, j, k, rows + 18 * IX(n, i, j, k));
}

/* y = J mu (forward directional derivative), for dot-product tests */
void or_jac_apply(const double *rows, const double *mu, int n, double h, double *y)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long c = IX(n, i, j, k);
                double acc = lap(mu, n, h, i, j, k);
                for (int q = 0; q < 18; ++q)
                    acc -= rows[18 * c + q] * mu[IX(n, i + NB[q][0], j + NB[q][1], k + NB[q][2])];
                y[c] = acc;
            }
}

/* y = J^T mu by scattering the rows; the Laplacian part is symmetric. */
void or_jac_t_apply(const double *rows, const double *mu, int n, double h, double *y)
{
    long n3 = (long)n * n * n;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                y[IX(n, i, j, k)] = lap(mu, n, h, i, j, k);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long c = IX(n, i, j, k);
                for (int q = 0; q < 18; ++q)
                    y[IX(n, i + NB[q][0], j + NB[q][1], k + NB[q][2])] -= rows[18 * c + q] * mu[c];
            }
    (void)n3;
}

typedef struct {
    int nlev;
    int n[OR_MAX_LEVELS];
    double h[OR_MAX_LEVELS];
    double *rows[OR_MAX_LEVELS];
    double *u[OR_MAX_LEVELS], *f[OR_MAX_LEVELS], *ru[OR_MAX_LEVELS];
    double *tmp[OR_MAX_LEVELS], *res[OR_MAX_LEVELS];
    int nu1, nu2, nuc;
    double kappa;
} or_adj;

/* residual J^T u - f (f array or scalar) */
static void adj_residual(or_adj *A, int l, const double *u, const double *f, double fs, double *out)
{
    int n = A->n[l];
    long n3 = (long)n * n * n;
    or_jac_t_apply(A->rows[l], u, n, A->h[l], out);
    for (long c = 0; c < n3; ++c) out[c] -= f ? f[c] : fs;
}

/* colour pass on J^T u = f (+ on the finest level kappa * mean(u), lagged
 * at the start of the pass); the diagonal of J^T is -6/h^2. */
static void adj_pass(or_adj *A, int l, const double *f, int colour)
{
    int n = A->n[l];
    long n3 = (long)n * n * n;
    double h = A->h[l];
    double shift = 0.0;
    if (l == 0) shift = A->kappa * or_mean(A->u[0], n);
    adj_residual(A, l, A->u[l], f, 0.0, A->res[l]);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                if (((i + j + k) & 1) != colour) continue;
                long c = IX(n, i, j, k);
                double r = A->res[l][c] - shift;
                A->tmp[l][c] = A->u[l][c] - r / (-6.0 / (h * h));
            }
    for (long c = 0; c < n3; ++c)
        if (((c % n + (c / n) % n + c / ((long)n * n)) & 1) == colour) A->u[l][c] = A->tmp[l][c];
}

static void adj_sweep(or_adj *A, int l, const double *f)
{
    adj_pass(A, l, f, 0);
    adj_pass(A, l, f, 1);
}

/* finest residual r = J^T u - kappa mean(u) - b, eps = RMS(r) */
static double adj_eps(or_adj *A, const double *b)
{
    int n = A->n[0];
    long n3 = (long)n * n * n;
    double m = or_mean(A->u[0], n);
    adj_residual(A, 0, A->u[0], b, 0.0, A->res[0]);
    for (long c = 0; c < n3; ++c) A->res[0][c] -= A->kappa * m;
    double s1, s2;
    sums(A->res[0], n3, n, &s1, &s2);
    return sqrt(s2 / (double)n3);
}

static void adj_vcycle(or_adj *A, int l, const double *b, double *eps_mid)
{
    int n = A->n[l];
    if (l == A->nlev - 1) {
        for (int s = 0; s < A->nuc; ++s) adj_sweep(A, l, l ? A->f[l] : b);
        return;
    }
    const double *f = l ? A->f[l] : b;
    for (int s = 0; s < A->nu1; ++s) adj_sweep(A, l, f);
    if (l == 0 && eps_mid) *eps_mid = adj_eps(A, b);
    /* residual restricted to the coarse level: J^T u - f (zero mean on the
     * finest level; the kappa term only fixes the gauge) */
    adj_residual(A, l, A->u[l], f, 0.0, A->res[l]);
    int lc = l + 1, ncs = A->n[lc];
    long cc = (long)ncs * ncs * ncs;
    or_restrict(A->u[l], n, A->ru[lc]);
    or_restrict(A->res[l], n, A->tmp[lc]);
    adj_residual(A, lc, A->ru[lc], NULL, 0.0, A->f[lc]);
    for (long q = 0; q < cc; ++q) A->f[lc][q] -= A->tmp[lc][q];
    memcpy(A->u[lc], A->ru[lc], sizeof(double) * cc);
    adj_vcycle(A, lc, NULL, NULL);
    or_prolong_add(A->u[l], n, A->u[lc], A->ru[lc]);
    for (int s = 0; s < A->nu2; ++s) adj_sweep(A, l, f);
}

/* Adjoint solve.  Given the converged forward phi (linearisation point) and
 * w = dLoss/dphi, solve J^T mu = w - mean(w) with mean(mu) = 0 (the bordered
 * adjoint of L(phi) + lambda = 0, sum(phi) = 0), then
 * grad_delta = -(dL/ddelta) mu = (dK/ddelta) mu.  mu is in/out (warm start). */
int or_adjoint(const or_model *m, int n, const double *delta, const double *phi,
               const double *w, double *grad, double *mu, int max_cycles, double tol,
               int nu1, int nu2, int nuc, or_stats *st)
{
    or_adj A;
    memset(&A, 0, sizeof(A));
    memset(st, 0, sizeof(*st));
    int L = 0;
    for (int q = n; q >= 4; q /= 2) { A.n[L] = q; A.h[L] = (double)n / q; ++L; }
    A.nlev = L;
    A.nu1 = nu1; A.nu2 = nu2; A.nuc = nuc;
    A.kappa = 6.0;
    long n3 = (long)n * n * n;
    double *lphi[OR_MAX_LEVELS] = {0}, *ldel[OR_MAX_LEVELS] = {0};
    for (int l = 0; l < L; ++l) {
        long c = (long)A.n[l] * A.n[l] * A.n[l];
        if (l > 0) {
            /* linearisation point on coarse levels: restricted phi and delta */
            lphi[l] = malloc(sizeof(double) * c);
            ldel[l] = malloc(sizeof(double) * c);
            or_restrict(l > 1 ? lphi[l - 1] : phi, A.n[l - 1], lphi[l]);
            or_restrict(l > 1 ? ldel[l - 1] : delta, A.n[l - 1], ldel[l]);
        }
        A.rows[l] = malloc(sizeof(double) * 18 * c);
        or_jac_rows(m, l ? lphi[l] : phi, l ? ldel[l] : delta, A.n[l], A.h[l], A.rows[l]);
        A.u[l] = l ? malloc(sizeof(double) * c) : mu;
        A.f[l] = l ? malloc(sizeof(double) * c) : NULL;
        A.ru[l] = l ? malloc(sizeof(double) * c) : NULL;
        A.tmp[l] = malloc(sizeof(double) * c);
        A.res[l] = malloc(sizeof(double) * c);
    }
    for (int l = 1; l < L; ++l) { free(lphi[l]); free(ldel[l]); }
    double *b = malloc(sizeof(double) * n3);
    double wm = or_mean(w, n);
    for (long c = 0; c < n3; ++c) b[c] = w[c] - wm;
    double eps = adj_eps(&A, b);
    st->eps0 = eps;
    st->status = 1;
    int cyc = 0;
    double best = eps;
    if (eps <= tol) st->status = 0;
    else {
        for (cyc = 1; cyc <= max_cycles; ++cyc) {
            double em = 0.0;
            adj_vcycle(&A, 0, b, &em);
            if (cyc - 1 < OR_HIST) st->hist[cyc - 1] = em;
            if (!isfinite(em)) { st->status = -3; break; }
            if (em > 1e3 * best) { st->status = -4; break; }
            if (em < best) best = em;
            if (em <= tol || cyc == max_cycles) {
                eps = adj_eps(&A, b);
                if (eps <= tol) { st->status = 0; break; }
            }
        }
        if (cyc > max_cycles) cyc = max_cycles;
    }
    st->cycles = cyc;
    st->eps = eps;
    st->mu = or_mean(mu, n);
    /* grad_delta_m = -(dL_m/ddelta_m) mu_m = (dK_m/ddelta_m) mu_m */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long c = IX(n, i, j, k);
                double dk;
                if (m->model == 2) dk = m->s;
                else if (m->model == 0) {
                    /* dK/ddelta = F'(Sigma) * s */
                    double xp = phi[IX(n, i + 1, j, k)], xm = phi[IX(n, i - 1, j, k)];
                    double yp = phi[IX(n, i, j + 1, k)], ym = phi[IX(n, i, j - 1, k)];
                    double zp = phi[IX(n, i, j, k + 1)], zm = phi[IX(n, i, j, k - 1)];
                    double cc0 = phi[c], h4 = 1.0;
                    double dxx = xp + xm - 2 * cc0, dyy = yp + ym - 2 * cc0, dzz = zp + zm - 2 * cc0;
                    double nxy = phi[IX(n, i + 1, j + 1, k)] + phi[IX(n, i - 1, j - 1, k)]
                               - phi[IX(n, i + 1, j - 1, k)] - phi[IX(n, i - 1, j + 1, k)];
                    double nxz = phi[IX(n, i + 1, j, k + 1)] + phi[IX(n, i - 1, j, k - 1)]
                               - phi[IX(n, i + 1, j, k - 1)] - phi[IX(n, i - 1, j, k + 1)];
                    double nyz = phi[IX(n, i, j + 1, k + 1)] + phi[IX(n, i, j - 1, k - 1)]
                               - phi[IX(n, i, j + 1, k - 1)] - phi[IX(n, i, j - 1, k + 1)];
                    double sigma = 2.0 / (3.0 * h4) * (dxx * dxx + dyy * dyy + dzz * dzz - dxx * dyy
                                                       - dxx * dzz - dyy * dzz)
                                 + 1.0 / (8.0 * h4) * (nxy * nxy + nxz * nxz + nyz * nyz)
                                 + m->s * delta[c];
                    double disc = m->alpha * m->alpha + 8.0 / 3.0 * sigma;
                    dk = disc > 0.0 ? m->sgn / sqrt(disc) * m->s : 0.0;
                } else {
                    double xp = phi[IX(n, i + 1, j, k)], xm = phi[IX(n, i - 1, j, k)];
                    double yp = phi[IX(n, i, j + 1, k)], ym = phi[IX(n, i, j - 1, k)];
                    double zp = phi[IX(n, i, j, k + 1)], zm = phi[IX(n, i, j, k - 1)];
                    double gx = (xp - xm) / 2, gy = (yp - ym) / 2, gz = (zp - zm) / 2;
                    double g = gx * gx + gy * gy + gz * gz;
                    double sig1 = m->C0 + (2.0 * m->nk + 1.0) * m->gamma / 3.0 * ipow(g, m->nk - 1);
                    dk = m->src / (m->ctil * sig1);
                }
                grad[c] = dk * mu[c];
            }
    for (int l = 0; l < L; ++l) {
        free(A.rows[l]);
        if (l) { free(A.u[l]); free(A.f[l]); free(A.ru[l]); }
        free(A.tmp[l]);
        free(A.res[l]);
    }
    free(b);
    return st->status;
}

/* ------------------------------------------------------------------ */
/* CIC deposit, forces, kick-drift (GLAM substrate, Sec. 3.1)          */
/* ------------------------------------------------------------------ */

/* Cloud-in-cell mass assignment of unit-mass particles; cell i has centre
 * i + 1/2.  rho[] (FP64, n^3) is overwritten with particle counts per cell.
 * Sequential, so the summation order is the particle order. */
void or_cic_deposit(int n, long npart, const float *pos, double *rho)
{
    memset(rho, 0, sizeof(double) * (size_t)n * n * n);
    for (long p = 0; p < npart; ++p) {
        double t[3], f[3];
        int i0[3];
        for (int a = 0; a < 3; ++a) {
            t[a] = (double)pos[3 * p + a] - 0.5;
            i0[a] = (int)floor(t[a]);
            f[a] = t[a] - i0[a];
        }
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    double wgt = (a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1])
                               * (c ? f[2] : 1.0 - f[2]);
                    rho[IX(n, i0[0] + a, i0[1] + b, i0[2] + c)] += wgt;
                }
    }
}

/* One leapfrog step of the particles given the total potential psi on the
 * mesh: g = -grad psi by 3-point central differences at cell centres,
 * interpolated with the CIC weights (the scheme of Sec. 3.1), then
 * p += g * kick, x += p * drift (wrapped to [0, n)). */
/* p <- damp p - kick grad(psi) (3-point differences at the 8 CIC cells,
 * CIC-weighted), then x <- x + drift p, periodic.  damp = 1 for nDGP;
 * 1 - beta (d phibar/da) da for the velocity term of eq:force_Kmo2. */
void or_kick_drift_damped(int n, long npart, const double *psi, float *pos, float *mom,
                          double damp, double kick, double drift)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < npart; ++p) {
        double t[3], f[3], g[3] = {0.0, 0.0, 0.0};
        int i0[3];
        for (int a = 0; a < 3; ++a) {
            t[a] = (double)pos[3 * p + a] - 0.5;
            i0[a] = (int)floor(t[a]);
            f[a] = t[a] - i0[a];
        }
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    double wgt = (a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1])
                               * (c ? f[2] : 1.0 - f[2]);
                    int i = i0[0] + a, j = i0[1] + b, k = i0[2] + c;
                    g[0] -= wgt * (psi[IX(n, i + 1, j, k)] - psi[IX(n, i - 1, j, k)]) / 2.0;
                    g[1] -= wgt * (psi[IX(n, i, j + 1, k)] - psi[IX(n, i, j - 1, k)]) / 2.0;
                    g[2] -= wgt * (psi[IX(n, i, j, k + 1)] - psi[IX(n, i, j, k - 1)]) / 2.0;
                }
        for (int a = 0; a < 3; ++a) {
            double pn = damp * (double)mom[3 * p + a] + g[a] * kick;
            double xn = (double)pos[3 * p + a] + pn * drift;
            xn = fmod(xn, (double)n);
            if (xn < 0.0) xn += n;
            mom[3 * p + a] = (float)pn;
            pos[3 * p + a] = (float)xn;
            if (pos[3 * p + a] >= (float)n) pos[3 * p + a] = 0.0f;
        }
    }
}

void or_kick_drift(int n, long npart, const double *psi, float *pos, float *mom,
                   double kick, double drift)
{
    or_kick_drift_damped(n, npart, psi, pos, mom, 1.0, kick, drift);
}
