// lbm_consts.cpp -- host FP64 constants of the semiclassical LBM (library side).
//
// Weight integrals I_2N of eq. (i2n-cont2) (Sec. 3) by composite Gauss-Legendre
// quadrature on panels finer than the width of the Fermi edge; polynomial coefficients
// of Sec. 3 (K <= 2); reference speed and weights of Sec. 8 / Table 1 and of D1V7
// (App. A); the reduced equilibrium of Sec. 9.1 collapsed to
// what_a [1 + A (xi.u) + Bc (xi.u)^2 + C_k u^2].
#include "lbm_internal.h"

#include <cmath>
#include <complex>
#include <vector>

namespace lbm {

namespace {

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n (long double).
void gauss_legendre(int n, std::vector<long double> &x, std::vector<long double> &w)
{
    x.assign(n, 0.0L);
    w.assign(n, 0.0L);
    for (int i = 0; i < n; ++i) {
        long double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        long double dp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_n(z), p0 = P_{n-1}(z)
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            const long double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-19L) break;
        }
        x[i] = z;
        w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
}

// Radial weight omega(xi), evaluated in long double.
long double omega(int stats, long double xi, long double theta, long double mu, int D)
{
    if (stats == LBM_HERMITE) return std::exp(-0.5L * xi * xi) / std::pow(2.0L * (long double)M_PI, 0.5L * D);
    if (stats == LBM_BOSE_EINSTEIN) return 1.0L / std::expm1((xi * xi - mu) / theta);  // mu < 0
    // 1/(exp((xi^2 - mu)/theta) + 1), written to stay finite for large arguments
    const long double a = (xi * xi - mu) / theta;
    if (a > 0) {
        const long double e = std::exp(-a);
        return e / (1.0L + e);
    }
    return 1.0L / (std::exp(a) + 1.0L);
}

}  // namespace

// I_2N for N = 0..3 (out[0..3] = I_0, I_2, I_4, I_6).
int weight_integrals(int stats, int D, double theta, double mu, double out[4])
{
    return weight_integrals_n(stats, D, theta, mu, 4, out);
}

// I_2N for N = 0..n-1 (n <= 5; out[N] = I_2N), D = 1, 2 or 3.
int weight_integrals_n(int stats, int D, double theta, double mu, int n, double *out)
{
    if (!(D >= 1 && D <= 3) || n < 1 || n > 5) return LBM_EINVAL;
    if (stats == LBM_HERMITE) {
        for (int i = 0; i < n; ++i) out[i] = 1.0;  // exact for the Hermite weight, Sec. 3
        // (kept analytic; the quadrature path is used for every other weight)
        return LBM_OK;
    }
    if (stats != LBM_FERMI_DIRAC && stats != LBM_BOSE_EINSTEIN) return LBM_EINVAL;
    if (!(theta > 0) || !std::isfinite(theta) || !std::isfinite(mu)) return LBM_EINVAL;
    if (stats == LBM_BOSE_EINSTEIN && !(mu < 0)) return LBM_EINVAL;
    // The integrand is negligible beyond xi^2 = mu + 80 theta (omega < e^-80). Panels
    // are narrower than the width of the Fermi edge (~theta/2 in xi near xi^2 = mu), or,
    // for the Bose-Einstein weight, than a quarter of its scales sqrt(theta) and
    // sqrt(|mu|); nodes, weights and sums are carried in long double and rounded once.
    const long double th = theta, m = mu;
    const long double xmax = std::sqrt(std::fmax(mu, 0.0) + 80.0 * theta);
    const long double h = stats == LBM_FERMI_DIRAC
                              ? std::fmin(1e-3L, 0.25L * th / std::fmax(1.0L, xmax))
                              : std::fmin(1e-3L, 0.25L * std::sqrt(std::fmin(th, std::fabs(m))));
    const int npan = (int)std::ceil(xmax / h);
    std::vector<long double> gx, gw;
    gauss_legendre(10, gx, gw);
    long double acc[5] = {0, 0, 0, 0, 0};
    for (int p = 0; p < npan; ++p) {
        const long double a = p * (xmax / npan), b = (p + 1) * (xmax / npan);
        const long double c = 0.5L * (a + b), r = 0.5L * (b - a);
        for (size_t k = 0; k < gx.size(); ++k) {
            const long double xi = c + r * gx[k];
            const long double wk = r * gw[k] * omega(stats, xi, th, m, D);
            long double pw = D == 1 ? 1.0L : std::pow(xi, (long double)(D - 1));
            for (int N = 0; N < n; ++N) {
                acc[N] += wk * pw;
                pw *= xi * xi;
            }
        }
    }
    for (int N = 0; N < n; ++N)
        out[N] = (double)(std::pow((long double)M_PI, 0.5L * D) /
                          (std::pow(2.0L, (long double)(N - 1)) * std::tgamma(N + 0.5L * D)) * acc[N]);
    return LBM_OK;
}

// D1V7 (App. A): c_s from the printed closed form of the root of
// 12 I_2 - 49 I_4 c^2 + 70 I_6 c^4 - 35 I_8 c^6 = 0 (principal square and cube roots, in
// complex arithmetic; the result is real up to rounding), then the printed solution
// w_0..w_3 of the quadrature equations (weights of |e| = 0..3).
int d1v7_constants(const double I[5], double *cs_out, double w[4])
{
    using C = std::complex<long double>;
    const long double I0 = I[0], I2 = I[1], I4 = I[2], I6 = I[3], I8 = I[4];
    const long double A = -4900.0L * I6 * I6 + 5145.0L * I4 * I8;
    const long double B = 686000.0L * I6 * I6 * I6 - 1080450.0L * I4 * I6 * I8 + 396900.0L * I2 * I8 * I8;
    const C R = std::pow(C(B) + std::sqrt(C(4.0L * A * A * A + B * B)), 1.0L / 3.0L);
    const long double c2r = std::cbrt(2.0L);
    const C c2 = C(2.0L * I6 / (3.0L * I8)) - 49.0L * c2r * I4 / R + 140.0L * c2r * I6 * I6 / (3.0L * I8 * R) +
                 R / (105.0L * c2r * I8);
    if (!(c2.real() > 0) || std::fabs(c2.imag()) > 1e-9L * c2.real()) return LBM_EUNSUPPORTED;
    const long double y = c2.real();
    const long double cubic = 12.0L * I2 - 49.0L * I4 * y + 70.0L * I6 * y * y - 35.0L * I8 * y * y * y;
    if (!(std::fabs(cubic) <= 1e-9L * 12.0L * I2)) return LBM_EUNSUPPORTED;
    w[0] = (double)((360.0L * I0 - 150.0L * I6 * y * y * y + 420.0L * I4 * y * y - 490.0L * I2 * y) / 360.0L);
    w[1] = (double)((-13.0L * I4 * y * y + 5.0L * I6 * y * y * y + 12.0L * I2 * y) / 16.0L);
    w[2] = (double)((30.0L * I4 * y * y - 15.0L * I6 * y * y * y - 9.0L * I2 * y) / 120.0L);
    w[3] = (double)((15.0L * I6 * y * y * y - 15.0L * I4 * y * y + 4.0L * I2 * y) / 720.0L);
    for (int i = 0; i < 4; ++i)
        if (!(w[i] > 0)) return LBM_EUNSUPPORTED;
    *cs_out = (double)std::sqrt(y);
    return LBM_OK;
}

int compute_constants(const lbm_params *p, lbm_constants *k)
{
    if (p->lattice == LBM_D1V7) {
        double I[5], w[4], cs;
        int rc = weight_integrals_n(p->stats, 1, p->theta, p->mu, 5, I);
        if (rc != LBM_OK) return rc;
        rc = d1v7_constants(I, &cs, w);
        if (rc != LBM_OK) return rc;
        *k = lbm_constants{};
        k->I0 = I[0];
        k->I2 = I[1];
        k->I4 = I[2];
        k->c0 = 1.0 / std::sqrt(I[0]);
        k->c1 = 1.0 / std::sqrt(I[1]);
        k->c2 = 1.0 / std::sqrt(I[2]);
        k->J2 = I[1] * I[1] / (I[2] * I[0]);
        k->theta_bar = I[1] / I[0];
        k->cs = cs;
        for (int s = 0; s < 4; ++s) {
            k->w[s] = w[s];
            k->what[s] = w[s] / I[0];
        }
        return LBM_OK;
    }
    int D;
    if (p->lattice == LBM_D2V9)
        D = 2;
    else if (p->lattice == LBM_D3V19 || p->lattice == LBM_D3V15)
        D = 3;
    else
        return LBM_EINVAL;
    double I[4];
    const int rc = weight_integrals(p->stats, D, p->theta, p->mu, I);
    if (rc != LBM_OK) return rc;
    *k = lbm_constants{};
    k->I0 = I[0];
    k->I2 = I[1];
    k->I4 = I[2];
    k->c0 = 1.0 / std::sqrt(I[0]);
    k->c1 = 1.0 / std::sqrt(I[1]);
    k->c2 = 1.0 / std::sqrt(I[2]);
    k->J2 = I[1] * I[1] / (I[2] * I[0]);
    const double den = (D + 2.0) - k->J2 * D;
    if (!(den > 0)) return LBM_EUNSUPPORTED;
    k->Delta2 = std::sqrt(2.0 / den);
    k->c2bar = k->c2 * (k->Delta2 - 1.0) / D;
    k->c2p = -k->c2 * (I[1] / I[0]) * k->Delta2;
    k->theta_bar = I[1] / I[0];
    k->cs = std::sqrt(I[1] / (3.0 * I[2]));
    const double J2 = k->J2, I0 = I[0];
    if (p->lattice == LBM_D2V9) {
        k->w[0] = I0 * (1.0 - 5.0 * J2 / 9.0);
        k->w[1] = I0 * J2 / 9.0;
        k->w[2] = I0 * J2 / 36.0;
    } else if (p->lattice == LBM_D3V19) {
        k->w[0] = I0 * (1.0 - 2.0 * J2 / 3.0);
        k->w[1] = I0 * J2 / 18.0;
        k->w[2] = I0 * J2 / 36.0;
    } else {  // D3V15, Sec. 8
        k->w[0] = I0 * (1.0 - 7.0 * J2 / 9.0);
        k->w[1] = I0 * J2 / 9.0;
        k->w[3] = I0 * J2 / 72.0;
    }
    const int shells[3] = {0, 1, p->lattice == LBM_D3V15 ? 3 : 2};
    for (int i = 0; i < 3; ++i)
        if (!(k->w[shells[i]] > 0)) return LBM_EUNSUPPORTED;  // Sec. 8: weights must be positive
    for (int s = 0; s < 4; ++s) k->what[s] = k->w[s] / I0;  // 0 for absent shells
    // Collapse the reduced EDF of Sec. 9.1 using c0^2 = 1/I_0:
    //   A = I_0 c1^2, Bc = I_0 c2^2 / 2,
    //   C_k = I_0 [c2 cbar2 xi_k^2 + (cbar2 xi_k^2 + c'2)(c2 + D cbar2)] / 2, xi_k^2 = k / c_s^2.
    k->A = I0 * k->c1 * k->c1;
    k->Bc = 0.5 * I0 * k->c2 * k->c2;
    for (int s = 0; s < 4; ++s) {
        if (!(k->w[s] > 0)) continue;  // shell not in this lattice
        const double xi2 = s / (k->cs * k->cs);
        k->C[s] = 0.5 * I0 * (k->c2 * k->c2bar * xi2 + (k->c2bar * xi2 + k->c2p) * (k->c2 + D * k->c2bar));
    }
    return LBM_OK;
}

}  // namespace lbm
