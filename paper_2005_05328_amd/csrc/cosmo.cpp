// Host-side cosmology for the step: kick and drift factors, comoving distance and the
// Chebyshev series the lightcone crossing solve evaluates on the GPU.  Flat LCDM without
// radiation, H(a) = H0 sqrt(Om a^-3 + 1 - Om), H0 = 100 km/s/(Mpc/h).
//
//   K(a0,a1) = int da / (a^2 H)   (p = a^2 dx/dt, dp/dt = g/a)
//   D(a0,a1) = int da / (a^3 H)   (dx/dt = p/a^2)
//   chi(a)   = c int_a^1 da / (a^2 H)
//
// Integrals: composite 16-point Gauss-Legendre on panels [a, a(1+1/4)] (capped at width
// 0.05), whose Bernstein-ellipse margin to the a = 0 singularity makes each panel exact to
// well below double rounding.
#include <math.h>
#include <string.h>

#include "../../include/dzs.h"

namespace {

const double kH0 = 100.0;
const double kC = 299792.458;

struct GaussLegendre16 {
    double x[16], w[16];
    GaussLegendre16() {
        const int n = 16;
        for (int i = 0; i < n; ++i) {
            long double z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
            for (int it = 0; it < 100; ++it) {
                long double p0 = 1.0L, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                long double dp = n * (z * p1 - p0) / (z * z - 1.0L);
                long double dz = p1 / dp;
                z -= dz;
                if (fabsl(dz) < 1e-19L)
                    break;
            }
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            long double dp = n * (z * p1 - p0) / (z * z - 1.0L);
            x[i] = (double)z;
            w[i] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
        }
    }
};

const GaussLegendre16 &gl16() {
    static GaussLegendre16 g;
    return g;
}

inline long double E(long double a, double om) {
    return sqrtl((long double)om / (a * a * a) + (1.0L - om));
}

// int_{lo}^{hi} a^-pow / E(a) da
long double integrate(double lo, double hi, int pw, double om) {
    if (hi <= lo)
        return 0.0L;
    const GaussLegendre16 &g = gl16();
    long double sum = 0.0L;
    double a = lo;
    while (a < hi) {
        double w = 0.25 * a;
        if (w > 0.05)
            w = 0.05;
        double b = a + w;
        if (b > hi || hi - b < 1e-3 * w)
            b = hi;
        long double c = 0.5L * ((long double)a + b), h = 0.5L * ((long double)b - a);
        long double s = 0.0L;
        for (int i = 0; i < 16; ++i) {
            long double t = c + h * g.x[i];
            long double ap = powl(t, (long double)pw);
            s += g.w[i] / (ap * E(t, om));
        }
        sum += s * h;
        a = b;
    }
    return sum;
}

double kick(double a0, double a1, double om) { return (double)(integrate(a0, a1, 2, om) / kH0); }
double drift(double a0, double a1, double om) { return (double)(integrate(a0, a1, 3, om) / kH0); }
double chi(double a, double om) { return (double)(kC * integrate(a, 1.0, 2, om) / kH0); }

// Chebyshev coefficients of f on [a0, a1] from n samples at the Chebyshev nodes.
template <typename F>
void cheb_fit(F f, double a0, double a1, int n, double *c) {
    const long double pi = 3.14159265358979323846264338327950288L;
    long double fv[DZS_CHEB_MAX];
    for (int j = 0; j < n; ++j) {
        long double th = pi * (j + 0.5L) / n;
        long double t = cosl(th);
        double a = (double)(0.5L * (a0 + a1) + 0.5L * (a1 - a0) * t);
        fv[j] = f(a);
    }
    for (int k = 0; k < n; ++k) {
        long double s = 0.0L;
        for (int j = 0; j < n; ++j)
            s += fv[j] * cosl(pi * k * (j + 0.5L) / n);
        c[k] = (double)(s * (k == 0 ? 1.0L : 2.0L) / n);
    }
}

}  // namespace

double dzs_kick_factor(double a0, double a1, double omega_m) { return kick(a0, a1, omega_m); }

void dzs_merge_thresholds(double L, double R_lc, double b, double theta, double *T2) {
    for (int k = 0; k <= 21; ++k) {
        double lk = ldexp(L, -k);
        double T = (R_lc + b) + lk / theta;
        T2[k] = T * T;
    }
}

#ifndef DZS_SOURCE_HASH
#error "build with -DDZS_SOURCE_HASH (the build script passes the hash of the sources)"
#endif
extern "C" const char *dzs_source_hash(void) { return DZS_SOURCE_HASH; }

extern "C" dzs_status dzs_step_factors(double a0, double a1, double omega_m,
                                       dzs_step_params *out) {
    if (!out || !(a0 > 0.0) || !(a1 > a0) || !(a1 <= 1.0) || !(omega_m > 0.0) ||
        !(omega_m <= 1.0))
        return DZS_EINVAL;
    const double ah = sqrt(a0 * a1);
    out->K1 = kick(a0, ah, omega_m);
    out->K2 = kick(ah, a1, omega_m);
    out->lc.a0 = a0;
    out->lc.a1 = a1;
    out->lc.D = drift(a0, a1, omega_m);
    const double c0 = chi(a0, omega_m), c1 = a1 < 1.0 ? chi(a1, omega_m) : 0.0;
    out->lc.chi2_0 = c0 * c0;
    out->lc.chi2_1 = c1 * c1;
    const int n = 20;
    out->lc.n_cheb = n;
    memset(out->lc.cheb_chi, 0, sizeof(out->lc.cheb_chi));
    memset(out->lc.cheb_drift, 0, sizeof(out->lc.cheb_drift));
    cheb_fit([&](double a) { return a < 1.0 ? chi(a, omega_m) : 0.0; }, a0, a1, n, out->lc.cheb_chi);
    cheb_fit([&](double a) { return drift(a0, a, omega_m); }, a0, a1, n, out->lc.cheb_drift);
    return DZS_OK;
}

// ---------------------------------------------------------------------------------------
// Run control (Sec. 4.1.1) and the speed-up forecast (Sec. 4.2, eqs. 4-7): host logic only.
// ---------------------------------------------------------------------------------------

extern "C" uint32_t dzs_halt_check(const dzs_halt_params *prm, const dzs_halt_state *st) {
    if (!prm || !st)
        return 0u;
    uint32_t why = 0u;
    if (prm->max_balance > 0.0 && st->balance > prm->max_balance)
        why |= DZS_HALT_BALANCE;
    if (st->ratio < prm->min_ratio)
        why |= DZS_HALT_RATIO;
    if (prm->runtime_limit_s > 0.0 && st->t >= prm->runtime_limit_s && st->t > st->t_prev) {
        // R(t) extrapolated linearly from the last two samples to the end of the window
        // that follows the restart
        const double slope = (st->ratio - st->ratio_prev) / (st->t - st->t_prev);
        if (st->ratio + slope * prm->restart_window_s < prm->min_ratio)
            why |= DZS_HALT_PREDICTED;
    }
    return why;
}

extern "C" dzs_status dzs_forecast_speedup(double L, double n_part, double omega_m,
                                           dzs_forecast *out) {
    if (!out || !(L > 0.0) || !(n_part >= 1.0) || !(omega_m > 0.0) || !(omega_m <= 1.0))
        return DZS_EINVAL;
    // particle mass (1e10 Msun/h) from the critical density 2.775e11 h^2 Msun / Mpc^3
    const double rho_crit = 27.75366;
    auto mass = [&](double Lb, double n) { return omega_m * rho_crit * Lb * Lb * Lb / n; };
    const double m = mass(L, n_part);
    const double m_small = mass(512.0, 512.0 * 512.0 * 512.0);
    const double m_large = mass(8192.0, 512.0 * 512.0 * 512.0);
    const double r_lin = 0.4 + (1.0 - 0.4) / (m_small - m_large) * (m - m_large);
    const double r = r_lin > 0.4 ? r_lin : 0.4;
    // a_DZS: the lightcone sphere holds half the box volume, 4/3 pi chi^3 = L^3 / 2
    const double R = cbrt(3.0 / (8.0 * 3.14159265358979323846)) * L;
    double lo = 1e-4, hi = 1.0;
    if (!(chi(lo, omega_m) > R))
        return DZS_EINVAL;  // the sphere encloses half the box from the start
    for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (chi(mid, omega_m) > R)
            lo = mid;
        else
            hi = mid;
    }
    out->a_dzs = 0.5 * (lo + hi);
    out->r = r;
    out->speedup = pow(out->a_dzs, -r);
    out->particle_mass = m;
    return DZS_OK;
}
