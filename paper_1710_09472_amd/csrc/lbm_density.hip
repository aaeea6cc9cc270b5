// lbm_density.hip -- density <-> chemical potential of the semiclassical weight
// (Sec. 9.1 and 9.2): rho = (pi theta)^(D/2) g_(D/2)(e^(mu/theta)), with the complete
// Fermi-Dirac (g_nu(z) = -Li_nu(-z)) or Bose-Einstein (g_nu(z) = Li_nu(z)) integrals
//   g_nu(e^eta) = 1/Gamma(nu) int_0^inf x^(nu-1) / (e^(x - eta) +- 1) dx.
// In 2D g_1 is elementary (ln(1 + z), -ln(1 - z)); in 3D g_3/2 is integrated in FP64 per
// element and inverted by Newton's method with g_3/2' = g_1/2. Used to set initial
// conditions in mu and to report mu; not part of the time step.
#include "lbm_internal.h"

#include <cmath>

namespace lbm {

namespace {

// 8-point Gauss-Legendre nodes and weights on [-1, 1].
__constant__ double kGLx[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290, -0.1834346424956498,
                               0.1834346424956498,  0.5255324099163290,  0.7966664774136267,  0.9602898564975363};
__constant__ double kGLw[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873, 0.3626837833783620,
                               0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};

// Occupation 1/(e^(t^2 - eta) + 1) (FD) or 1/(e^(t^2 - eta) - 1) (BE, eta < 0).
__device__ __forceinline__ double occupation(bool fd, double t, double eta)
{
    const double a = t * t - eta;
    if (!fd) return 1.0 / expm1(a);
    return a > 0 ? exp(-a) / (1.0 + exp(-a)) : 1.0 / (exp(a) + 1.0);
}

// Adds int_a^b of occupation * (t^2, 1) over [a, b] in `panels` equal panels.
__device__ void integrate(bool fd, double eta, double a, double b, int panels, double &s2, double &s0)
{
    const double h = (b - a) / panels;
    for (int p = 0; p < panels; ++p) {
        const double c = a + (p + 0.5) * h, r = 0.5 * h;
        for (int k = 0; k < 8; ++k) {
            const double t = c + r * kGLx[k];
            const double v = r * kGLw[k] * occupation(fd, t, eta);
            s2 += v * t * t;
            s0 += v;
        }
    }
}

// g_3/2(e^eta) and g_1/2(e^eta) with x = t^2: g_3/2 = (4/sqrt(pi)) int t^2 n dt,
// g_1/2 = (2/sqrt(pi)) int n dt. Panels: FD -- coarse where the occupation is 1 to
// within e^-40, fine (a quarter of the edge width 1/(2 sqrt(eta))) across the edge, cut
// where it is below e^-60; BE -- geometric panels from t = 0 on the scale sqrt(-eta) (the
// occupation behaves as 1/(t^2 - eta) there), then uniform up to e^-60.
__device__ void g_half_orders(bool fd, double eta, double &g32, double &g12)
{
    double s2 = 0.0, s0 = 0.0;
    if (fd) {
        const double t1 = sqrt(fmax(eta - 40.0, 0.0)), t2 = sqrt(fmax(eta, 0.0) + 60.0);
        if (t1 > 0) integrate(fd, eta, 0.0, t1, (int)ceil(t1 / 0.5), s2, s0);
        const double w = fmin(0.05, 0.125 / sqrt(fmax(eta, 1.0)));
        integrate(fd, eta, t1, t2, (int)ceil((t2 - t1) / w), s2, s0);
    } else {
        const double tmax = sqrt(60.0);
        double a = 0.0, b = 0.25 * fmax(sqrt(-eta), 1e-10);
        while (b < 1.0) {
            integrate(fd, eta, a, b, 1, s2, s0);
            a = b;
            b *= 2.0;
        }
        integrate(fd, eta, a, tmax, (int)ceil((tmax - a) / 0.125), s2, s0);
    }
    const double inv_sqrt_pi = 0.56418958354775628695;
    g32 = 4.0 * inv_sqrt_pi * s2;
    g12 = 2.0 * inv_sqrt_pi * s0;
}

__device__ double density_of(int D, bool fd, double theta, double mu)
{
    const double eta = mu / theta, pt = M_PI * theta;
    if (!fd && !(eta < 0)) return NAN;
    if (D == 2) {
        if (fd) return pt * (eta > 0 ? eta + log1p(exp(-eta)) : log1p(exp(eta)));  // ln(1 + z)
        return -pt * log(-expm1(eta));                                             // -ln(1 - z)
    }
    double g32, g12;
    g_half_orders(fd, eta, g32, g12);
    return pt * sqrt(pt) * g32;
}

__device__ double mu_of(int D, bool fd, double theta, double rho)
{
    const double pt = M_PI * theta;
    if (!(rho > 0)) return NAN;
    if (D == 2) {
        const double x = rho / pt;
        if (fd) return theta * (x + log(-expm1(-x)));  // ln(e^x - 1)
        return theta * log(-expm1(-x));                // ln(1 - e^-x)
    }
    const double y = rho / (pt * sqrt(pt));
    const double zeta32 = 2.6123753486854883433;  // g_3/2(1) of BE: no solution above it
    if (!fd && !(y < zeta32)) return NAN;
    // g_3/2(e^eta) is increasing and convex in eta, so Newton's iterates approach the
    // root monotonically from the right; these starts are right of it (FD: the degenerate
    // estimate under-counts g; BE: g >= e^eta) or one step from the right (FD, y <= 1).
    double eta = fd ? (y > 1.0 ? cbrt(1.3293403881791355 * y * 1.3293403881791355 * y) : log(y))
                    : fmin(log(y), -1e-12);
    // Stop when the step is at rounding level, or when it stops shrinking (the rounding
    // noise of the quadrature then sets it) with the residual at rounding level.
    double prev = INFINITY;
    for (int it = 0; it < 100; ++it) {
        double g32, g12;
        g_half_orders(fd, eta, g32, g12);
        const double res = g32 - y;
        double next = eta - res / g12;
        if (!fd) next = fmin(next, 0.5 * eta);  // stay below 0 (the step is leftward there)
        const double d = fabs(next - eta);
        if (d <= 4e-16 * fmax(1.0, fabs(eta)) || (d >= prev && fabs(res) <= 1e-13 * y)) return theta * next;
        prev = d;
        eta = next;
    }
    return NAN;
}

__global__ __launch_bounds__(256) void k_density(int D, int fd, double theta, const double *__restrict__ mu,
                                                 double *__restrict__ rho, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rho[i] = density_of(D, fd != 0, theta, mu[i]);
}

__global__ __launch_bounds__(256) void k_mu(int D, int fd, double theta, const double *__restrict__ rho,
                                            double *__restrict__ mu, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mu[i] = mu_of(D, fd != 0, theta, rho[i]);
}

}  // namespace

hipError_t launch_density(int D, int stats, double theta, const double *in, double *out, size_t n, bool to_mu,
                          hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const int fd = stats == LBM_FERMI_DIRAC ? 1 : 0;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (to_mu)
        hipLaunchKernelGGL(k_mu, grid, block, 0, st, D, fd, theta, in, out, n);
    else
        hipLaunchKernelGGL(k_density, grid, block, 0, st, D, fd, theta, in, out, n);
    return hipGetLastError();
}

}  // namespace lbm
