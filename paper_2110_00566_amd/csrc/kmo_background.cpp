// Kmouflage background cosmology (Sec. 3.2.5), host code of the library.
//
// The background is a two-variable ODE (phibar and its N-derivative, N =
// ln a) solved once per model, so it runs on the host; the field solves
// read the tabulated values.  Units H0 = 1; calH = a H.
//
// With K(X) = -1 + X + K0 X^n, A = exp(beta phi), p = dphi/dN and
// X = calH^2 p^2 / (2 lambda^2 a^2):
//   Friedmann     calH^2 (1 - p^2/6) = Or/a^2 + A Om/a + lambda^2 a^2/3
//                                      + (2n-1)/3 lambda^2 a^2 K0 X^n,
//   Raychaudhuri  calH' = -(A Om/a + 2 Or/a^2)/2 + lambda^2 a^2/3 - calH^2 p^2/3
//                         - (n+1)/3 lambda^2 a^2 K0 X^n,
//   field         (K_X + 2X K_XX)(calH^2 p_N + calH' p) + 2(K_X - X K_XX) calH^2 p
//                   + 3 beta A Om exp(-N) = 0      (eq:kmf_background_eom2),
// the N-forms derived from eq:kmf_background_eom, eq:kmf_background_Friedmann
// and the scalar fluid's energy conservation (rho = 2XK_X - K, P = K in units
// of lambda^2 H0^2).  The Friedmann equation is solved for calH^2 by Newton's
// method from S/b, which converges monotonically to the physical root (the
// one that continues to S/b as K0 -> 0).  The integration is an adaptive
// Dormand-Prince 5(4) pair (Dormand & Prince 1980) from z = z_init with
// phi = p = 1e-30, and lambda is found by the secant method so that
// H(a = 1) = H0.
#include <array>
#include <cmath>
#include <vector>

#include "../../include/mgglam.h"

namespace mgglam_internal {
void set_error(const char *msg);   // mg_last_error() of the library
}

namespace {

struct Bg {
    int n;
    double k0, beta, om, orad, lam;
};

// calH^2 from the Friedmann equation; false if it has no physical root
bool calh2(const Bg &m, double N, double phi, double p, double &y) {
    const double a = std::exp(N), a2 = a * a, l2 = m.lam * m.lam;
    const double A = std::exp(m.beta * phi);
    const double S = m.orad / a2 + A * m.om / a + l2 * a2 / 3.0;
    const double b = 1.0 - p * p / 6.0;
    if (!(b > 0.0)) return false;
    // C y^n with C = (2n-1)/3 lambda^2 a^2 K0 (p^2 / (2 lambda^2 a^2))^n
    const double q = p * p / (2.0 * l2 * a2);
    const double C = (2.0 * m.n - 1.0) / 3.0 * l2 * a2 * m.k0 * std::pow(q, m.n);
    y = S / b;
    if (C == 0.0) return true;
    for (int it = 0; it < 200; ++it) {
        const double yn = std::pow(y, m.n);
        const double g = b * y - S - C * yn;              // increasing, concave on the branch
        const double dg = b - m.n * C * yn / y;
        if (!(dg > 0.0)) return false;                    // past the maximum: no root
        const double step = g / dg;
        y -= step;
        if (std::fabs(step) <= 1e-16 * y) return y > 0.0;
    }
    return false;
}

double raychaudhuri(const Bg &m, double N, double phi, double p, double y) {
    const double a = std::exp(N), a2 = a * a, l2 = m.lam * m.lam;
    const double A = std::exp(m.beta * phi);
    const double X = y * p * p / (2.0 * l2 * a2);
    return -(A * m.om / a + 2.0 * m.orad / a2) / 2.0 + l2 * a2 / 3.0 - y * p * p / 3.0 -
           (m.n + 1.0) / 3.0 * l2 * a2 * m.k0 * std::pow(X, m.n);
}

// d/dN (phi, p); false where the Friedmann equation has no root
bool deriv(const Bg &m, double N, const double s[2], double d[2]) {
    double y;
    if (!calh2(m, N, s[0], s[1], y)) return false;
    const double a = std::exp(N), l2 = m.lam * m.lam;
    const double A = std::exp(m.beta * s[0]);
    const double p = s[1];
    const double hp = raychaudhuri(m, N, s[0], p, y);
    const double X = y * p * p / (2.0 * l2 * a * a);
    const double kx = 1.0 + m.n * m.k0 * std::pow(X, m.n - 1);
    const double kxx = m.n * (m.n - 1.0) * m.k0 * std::pow(X, m.n - 2);
    const double c2 = kx + 2.0 * X * kxx;
    d[0] = p;
    d[1] = -(c2 * hp * p + 2.0 * (kx - X * kxx) * y * p + 3.0 * m.beta * A * m.om * std::exp(-N)) /
           (c2 * y);
    return std::isfinite(d[1]);
}

// Dormand-Prince 5(4) tableau
constexpr double C2 = 1.0 / 5, C3 = 3.0 / 10, C4 = 4.0 / 5, C5 = 8.0 / 9;
constexpr double A21 = 1.0 / 5;
constexpr double A31 = 3.0 / 40, A32 = 9.0 / 40;
constexpr double A41 = 44.0 / 45, A42 = -56.0 / 15, A43 = 32.0 / 9;
constexpr double A51 = 19372.0 / 6561, A52 = -25360.0 / 2187, A53 = 64448.0 / 6561,
                 A54 = -212.0 / 729;
constexpr double A61 = 9017.0 / 3168, A62 = -355.0 / 33, A63 = 46732.0 / 5247, A64 = 49.0 / 176,
                 A65 = -5103.0 / 18656;
constexpr double B1 = 35.0 / 384, B3 = 500.0 / 1113, B4 = 125.0 / 192, B5 = -2187.0 / 6784,
                 B6 = 11.0 / 84;
constexpr double E1 = B1 - 5179.0 / 57600, E3 = B3 - 7571.0 / 16695, E4 = B4 - 393.0 / 640,
                 E5 = B5 + 92097.0 / 339200, E6 = B6 - 187.0 / 2100, E7 = -1.0 / 40;

// Integrate from N0 to the increasing stops Ns (last one = 0), stepping
// exactly onto each; out[k] receives the state at Ns[k].  Returns the step
// count, or -1 on failure.
long integrate(const Bg &m, double N0, const std::vector<double> &Ns,
               std::vector<std::array<double, 2>> *out, double rtol) {
    double s[2] = {1e-30, 1e-30}, N = N0, h = 1e-3;
    long steps = 0;
    double k1[2], k2[2], k3[2], k4[2], k5[2], k6[2], k7[2], t[2], s5[2];
    if (!deriv(m, N, s, k1)) return -1;
    for (size_t stop = 0; stop < Ns.size(); ++stop) {
        const double Nend = Ns[stop];
        while (N < Nend) {
            if (++steps > 10000000) return -1;
            const bool last = N + h >= Nend;
            const double hh = last ? Nend - N : h;
            bool ok = true;
            for (int i = 0; i < 2; ++i) t[i] = s[i] + hh * A21 * k1[i];
            ok &= deriv(m, N + C2 * hh, t, k2);
            for (int i = 0; i < 2; ++i) t[i] = s[i] + hh * (A31 * k1[i] + A32 * k2[i]);
            ok &= deriv(m, N + C3 * hh, t, k3);
            for (int i = 0; i < 2; ++i) t[i] = s[i] + hh * (A41 * k1[i] + A42 * k2[i] + A43 * k3[i]);
            ok &= deriv(m, N + C4 * hh, t, k4);
            for (int i = 0; i < 2; ++i)
                t[i] = s[i] + hh * (A51 * k1[i] + A52 * k2[i] + A53 * k3[i] + A54 * k4[i]);
            ok &= deriv(m, N + C5 * hh, t, k5);
            for (int i = 0; i < 2; ++i)
                t[i] = s[i] + hh * (A61 * k1[i] + A62 * k2[i] + A63 * k3[i] + A64 * k4[i] +
                                    A65 * k5[i]);
            ok &= deriv(m, N + hh, t, k6);
            for (int i = 0; i < 2; ++i)
                s5[i] = s[i] + hh * (B1 * k1[i] + B3 * k3[i] + B4 * k4[i] + B5 * k5[i] + B6 * k6[i]);
            ok &= deriv(m, N + hh, s5, k7);
            double err = 0.0;
            if (ok) {
                for (int i = 0; i < 2; ++i) {
                    const double e = hh * (E1 * k1[i] + E3 * k3[i] + E4 * k4[i] + E5 * k5[i] +
                                           E6 * k6[i] + E7 * k7[i]);
                    const double sc = rtol * std::fmax(std::fabs(s[i]), std::fabs(s5[i])) + 1e-300;
                    err = std::fmax(err, std::fabs(e) / sc);
                }
            }
            if (!ok || !(err <= 1.0)) {
                h = hh * (ok && std::isfinite(err) ? std::fmax(0.2, 0.9 * std::pow(err, -0.2)) : 0.25);
                if (h < 1e-14) return -1;
                continue;
            }
            N = last ? Nend : N + hh;
            s[0] = s5[0];
            s[1] = s5[1];
            k1[0] = k7[0];
            k1[1] = k7[1];
            const double grow = err > 0.0 ? std::fmin(5.0, 0.9 * std::pow(err, -0.2)) : 5.0;
            if (!last) h = hh * grow;
        }
        if (out) (*out)[stop] = {s[0], s[1]};
    }
    return steps;
}

mg_status bg_fail(const char *m) {
    mgglam_internal::set_error(m);
    return MG_ERR_ARG;
}

}  // namespace

extern "C" {

double mg_omega_radiation(double h, double t_cmb, double n_eff) {
    if (!(h > 0.0) || !(t_cmb > 0.0) || !(n_eff >= 0.0)) return -1.0;
    const double og = 2.4728e-5 * std::pow(t_cmb / 2.7255, 4) / (h * h);
    return og * (1.0 + n_eff * (7.0 / 8.0) * std::pow(4.0 / 11.0, 4.0 / 3.0));
}

mg_status mg_kmo_background(const mg_kmo_bg_params *par, int n_table, const double *a_table,
                            double *hubble, double *hubble_dot, double *phibar,
                            double *dphibar_dtau, mg_kmo_bg_info *info) {
    if (!par || !info) return bg_fail("params and info must not be NULL");
    if (par->n_k < 2 || par->n_k > 8 || !(par->k0 >= 0.0) || !std::isfinite(par->k0) ||
        !std::isfinite(par->beta) || !(par->omega_m > 0.0) || !(par->omega_m < 1.0) ||
        !(par->omega_r >= 0.0) || !(par->omega_m + par->omega_r < 1.0) ||
        !(par->z_init > 0.0) || !(par->htol > 0.0) || !(par->htol < 1e-2))
        return bg_fail("invalid background parameters");
    if (n_table < 0 || (n_table > 0 && (!a_table || !hubble || !hubble_dot || !phibar ||
                                         !dphibar_dtau)))
        return bg_fail("table pointers must be host arrays of n_table values");
    const double N0 = -std::log1p(par->z_init);
    for (int k = 0; k < n_table; ++k)
        if (!(a_table[k] > 0.0) || !(std::log(a_table[k]) > N0) || a_table[k] > 1.0 ||
            (k > 0 && !(a_table[k] > a_table[k - 1])))
            return bg_fail("a_table must increase within (1/(1+z_init), 1]");
    Bg m{par->n_k, par->k0, par->beta, par->omega_m, par->omega_r, 0.0};
    const double rtol = 1e-12;
    std::vector<double> last{0.0};
    std::vector<std::array<double, 2>> end(1);
    int shots = 0;
    // miss(lambda) = H(a=1)/H0 - 1, increasing in lambda
    auto miss = [&](double lam, double &f) {
        m.lam = lam;
        ++shots;
        if (integrate(m, N0, last, &end, rtol) < 0) return false;
        double y;
        if (!calh2(m, 0.0, end[0][0], end[0][1], y)) return false;
        f = std::sqrt(y) - 1.0;
        return true;
    };
    // secant from the LCDM value, bisection when a step leaves the bracket
    double l0 = std::sqrt(3.0 * (1.0 - par->omega_m - par->omega_r)), l1 = 1.02 * l0, f0, f1;
    if (!miss(l0, f0) || !miss(l1, f1)) return bg_fail("background integration failed");
    double lo = 0.0, hi = 0.0, flo = 0.0, fhi = 0.0;
    bool have_lo = false, have_hi = false;
    auto note = [&](double l, double f) {
        if (f < 0 && (!have_lo || l > lo)) { lo = l; flo = f; have_lo = true; }
        if (f > 0 && (!have_hi || l < hi)) { hi = l; fhi = f; have_hi = true; }
    };
    note(l0, f0);
    note(l1, f1);
    for (int it = 0; it < 100 && std::fabs(f1) > par->htol; ++it) {
        double l2 = (f1 != f0) ? l1 - f1 * (l1 - l0) / (f1 - f0) : 1.05 * l1;
        if (have_lo && have_hi && !(l2 > lo && l2 < hi)) l2 = 0.5 * (lo + hi);
        if (!(l2 > 0.0)) l2 = 0.5 * l1;
        double f2;
        if (!miss(l2, f2)) return bg_fail("background integration failed");
        note(l2, f2);
        l0 = l1;
        f0 = f1;
        l1 = l2;
        f1 = f2;
    }
    if (!(std::fabs(f1) <= par->htol)) return bg_fail("lambda shooting did not converge");
    m.lam = l1;
    info->lambda = l1;
    info->shots = shots;
    info->h_miss = f1;
    if (n_table > 0) {
        std::vector<double> Ns(n_table);
        for (int k = 0; k < n_table; ++k) Ns[k] = std::log(a_table[k]);
        std::vector<std::array<double, 2>> st(n_table);
        const long steps = integrate(m, N0, Ns, &st, rtol);
        if (steps < 0) return bg_fail("background integration failed");
        info->steps = (int)steps;
        for (int k = 0; k < n_table; ++k) {
            const double N = Ns[k], a = a_table[k];
            double y;
            if (!calh2(m, N, st[k][0], st[k][1], y)) return bg_fail("no Friedmann root");
            const double hp = raychaudhuri(m, N, st[k][0], st[k][1], y);
            hubble[k] = std::sqrt(y) / a;
            hubble_dot[k] = (hp - y) / (a * a);
            phibar[k] = st[k][0];
            dphibar_dtau[k] = std::sqrt(y) * st[k][1];
        }
    }
    return MG_OK;
}

}  // extern "C"
