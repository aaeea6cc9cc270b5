// lbm_thermal.hip -- the fourth-order thermal model on D1V7 (App. A), one dimension,
// periodic. The state holds the post-collision deviations d_a = f_a - rho0 what_a of the
// previous step (structure of arrays, array a at offset a * stride, e in the order
// 0, +1, -1, +2, -2, +3, -3). A step pulls f_a(x) = g_a(x - e_a), takes
//   rho = rho0 + sum d, j = rho u = sum d e, second moment sum f e^2 = rho (thetabar + u^2),
// builds the moments of the local equilibrium to fourth order (eqs. rho-def-eq,
// vel-def-eq, theta-bar-def-eq, gz-def-eq, with g held at the weight's value),
//   M_3 = rho (u^3 + 3 u thetabar), M_4 = rho (u^4 + 6 u^2 thetabar + 3 thetabar^2 g0),
// matches them with what_a p(e_a), p of degree 4 (the weight-orthogonal projection of
// the expansion of Sec. 3-5, exact on D1V7's order-9 quadrature), relaxes (BGK) and
// stores at the node.
//
// Precision. Deviations are formed throughout, so that rounding is relative to the
// departure from the weight's state, not to the populations. Velocities are the
// integer e_a (u and thetabar in lattice units), so every power of e_a is exact; the
// FP32 constants (what, the Hankel inverses) are not exactly consistent with each other,
// and a fixed mismatch of the equilibrium's moments would act on every step in the same
// direction (a drift of the conserved totals, a shift of the sound speed through M_3,
// the energy flux). One residual step removes it: the moments 1..4 of the polynomial's
// populations are taken again and their differences from the targets are put back on
// e = +-1, +-2 (a 2x2 solve per parity, with exact integer matrices); the rest population
// closes the mass. The equilibrium then carries moments 0..4 up to the rounding of the
// sums, as the projection does in exact arithmetic.
#include "lbm_device.h"

namespace lbm {
namespace {

constexpr int kQ7 = 7;
__device__ constexpr int kE7[kQ7] = {0, 1, -1, 2, -2, 3, -3};
__device__ constexpr float kEf[kQ7] = {0.f, 1.f, -1.f, 2.f, -2.f, 3.f, -3.f};
__device__ constexpr float kE2[kQ7] = {0.f, 1.f, 1.f, 4.f, 4.f, 9.f, 9.f};
__device__ constexpr float kE3[kQ7] = {0.f, 1.f, -1.f, 8.f, -8.f, 27.f, -27.f};
__device__ constexpr float kE4[kQ7] = {0.f, 1.f, 1.f, 16.f, 16.f, 81.f, 81.f};

__device__ __forceinline__ unsigned wrap_shift(int x, int e, int n)
{
    int s = x - e;
    if (s < 0) s += n;
    if (s >= n) s -= n;
    return (unsigned)s;
}

// Macroscopic fields of a node, lattice units: rho, u_e, thetabar_e - T.
struct ThermalNode {
    float rho, u, dtb;
};

// Deviations feq_a - rho0 what_a of the equilibrium of a node with moment deviations
// drho = sum d, j = sum d e, dE = sum d e^2 (lattice units).
__device__ __forceinline__ ThermalNode thermal_equilibrium(const ThermalPhysics &p, float drho, float j, float dE,
                                                           float *feq)
{
    ThermalNode m;
    m.rho = p.rho0 + drho;
    const float inv = 1.0f / m.rho;
    m.u = j * inv;
    // thetabar - T = (dE - T drho) / rho - u^2   (sum rho0 what e^2 = rho0 T)
    const float dtb = (dE - __builtin_fmaf(p.tb_hi, drho, p.tb_lo * drho)) * inv - m.u * m.u;
    m.dtb = dtb;
    const float tb = p.tb_hi + dtb;
    const float u2 = m.u * m.u;
    const float dM3 = j * (u2 + 3.0f * tb);
    // rho tb^2 g0 - rho0 T^2 g0 = g0 [drho tb^2 + rho0 dtb (2 T + dtb)]
    const float dA = p.g0 * __builtin_fmaf(drho, tb * tb, p.rho0 * dtb * (2.0f * p.tb_hi + dtb));
    const float dM4 = __builtin_fmaf(j * m.u, u2 + 6.0f * tb, 3.0f * dA);
    const float c0 = p.He_inv[0] * drho + p.He_inv[1] * dE + p.He_inv[2] * dM4;
    const float c2 = p.He_inv[3] * drho + p.He_inv[4] * dE + p.He_inv[5] * dM4;
    const float c4 = p.He_inv[6] * drho + p.He_inv[7] * dE + p.He_inv[8] * dM4;
    const float c1 = p.Ho_inv[0] * j + p.Ho_inv[1] * dM3;
    const float c3 = p.Ho_inv[2] * j + p.Ho_inv[3] * dM3;
    float r1 = j, r2 = dE, r3 = dM3, r4 = dM4;
#pragma unroll
    for (int a = 1; a < kQ7; ++a) {
        const float x = kEf[a];
        const float poly = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(__builtin_fmaf(c4, x, c3), x, c2), x, c1), x, c0);
        feq[a] = p.what[a] * poly;
        r1 = __builtin_fmaf(-feq[a], kEf[a], r1);
        r2 = __builtin_fmaf(-feq[a], kE2[a], r2);
        r3 = __builtin_fmaf(-feq[a], kE3[a], r3);
        r4 = __builtin_fmaf(-feq[a], kE4[a], r4);
    }
    // odd: o1 + 2 o2 = r1, o1 + 8 o2 = r3; even: s1 + 4 s2 = r2, s1 + 16 s2 = r4, with
    // o_k, s_k the difference and the sum of the corrections on e = +k and e = -k
    const float o2 = (r3 - r1) * (1.0f / 6.0f), o1 = __builtin_fmaf(-2.0f, o2, r1);
    const float s2 = (r4 - r2) * (1.0f / 12.0f), s1 = __builtin_fmaf(-4.0f, s2, r2);
    feq[1] += 0.5f * (s1 + o1);
    feq[2] += 0.5f * (s1 - o1);
    feq[3] += 0.5f * (s2 + o2);
    feq[4] += 0.5f * (s2 - o2);
    float sum = 0.f;
#pragma unroll
    for (int a = 1; a < kQ7; ++a) sum += feq[a];
    feq[0] = drho - sum;  // mass closure: the equilibrium carries exactly the node's mass
    return m;
}

__device__ __forceinline__ void thermal_moments(const float *d, float &drho, float &j, float &dE)
{
    drho = d[0];
    j = 0.f;
    dE = 0.f;
#pragma unroll
    for (int a = 1; a < kQ7; ++a) {
        drho += d[a];
        j = __builtin_fmaf(d[a], kEf[a], j);
        dE = __builtin_fmaf(d[a], kE2[a], dE);
    }
}

__device__ __forceinline__ void thermal_pull(const ThermalArgs &a, int x, float *d)
{
#pragma unroll
    for (int q = 0; q < kQ7; ++q)
        d[q] = __builtin_nontemporal_load(at32(a.src + (size_t)q * a.stride, wrap_shift(x, kE7[q], a.n)));
}

__global__ __launch_bounds__(kBlock) void k_thermal_step(ThermalArgs a)
{
    const int x = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x >= a.n) return;
    float d[kQ7], feq[kQ7];
    if (x >= 3 && x + 3 < a.n) {
        // no wrap: the rest population is read once (non-temporal); the shifted ones stay
        // cached, since the lines at a tile's edges are shared with the neighbouring tiles
        // (measured 2 % faster than non-temporal loads throughout)
        d[0] = __builtin_nontemporal_load(at32(a.src, (unsigned)x));
#pragma unroll
        for (int q = 1; q < kQ7; ++q) d[q] = a.src[(size_t)q * a.stride + (unsigned)(x - kE7[q])];
    } else {
        thermal_pull(a, x, d);
    }
    float drho, j, dE;
    thermal_moments(d, drho, j, dE);
    thermal_equilibrium(a.ph, drho, j, dE, feq);
#pragma unroll
    for (int q = 0; q < kQ7; ++q)
        __builtin_nontemporal_store(__builtin_fmaf(a.ph.omega, feq[q] - d[q], d[q]),
                                    at32(a.dst + (size_t)q * a.stride, (unsigned)x));
}

// Initial state f = f^eq(rho, u, thetabar): the deviations of node x are stored where
// the first pull reads them (slot a of x - e_a... i.e. of the node the pull into x reads).
__global__ __launch_bounds__(kBlock) void k_thermal_init(ThermalArgs a)
{
    const int x = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x >= a.n) return;
    const ThermalPhysics &p = a.ph;
    const double rho = a.rho[x];
    const double u = a.u ? a.u[x] * p.cs : 0.0;                         // lattice units
    const double tb = a.tb ? a.tb[x] * p.cs * p.cs : p.T;
    // moment deviations from the weight's state (sum what e^2 = T)
    const float drho = (float)(rho - (double)p.rho0);
    const float j = (float)(rho * u);
    const float dE = (float)(rho * (tb + u * u) - (double)p.rho0 * p.T);
    float feq[kQ7];
    thermal_equilibrium(p, drho, j, dE, feq);
#pragma unroll
    for (int q = 0; q < kQ7; ++q) {
        // the pull of q into node y reads slot q of y - e_q: node x's value goes to x
        // itself only when e_q = 0; store f^eq_q(x) at slot q of x - e_q
        a.dst[(size_t)q * a.stride + wrap_shift(x, kE7[q], a.n)] = feq[q];
    }
}

__global__ __launch_bounds__(kBlock) void k_thermal_fields(ThermalArgs a)
{
    const int x = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x >= a.n) return;
    float d[kQ7], feq[kQ7];
    thermal_pull(a, x, d);
    if (a.f64) {
#pragma unroll
        for (int q = 0; q < kQ7; ++q) a.f64[(size_t)q * a.n + x] = a.ph.what_rho0[q] + (double)d[q];
        return;
    }
    float drho, j, dE;
    thermal_moments(d, drho, j, dE);
    const ThermalNode m = thermal_equilibrium(a.ph, drho, j, dE, feq);
    // xi units: u = u_e / c_s, thetabar = (T + dtb) / c_s^2, each rounded once to FP32
    const double inv_cs = 1.0 / a.ph.cs;
    if (a.out_rho) a.out_rho[x] = m.rho;
    if (a.out_u) a.out_u[x] = (float)((double)m.u * inv_cs);
    if (a.out_tb) a.out_tb[x] = (float)((a.ph.T + (double)m.dtb) * inv_cs * inv_cs);
}

// Per-block FP64 sums of (drho, j, dE), lattice units, over a grid-stride range of nodes.
__global__ __launch_bounds__(kBlock) void k_thermal_partials(ThermalArgs a)
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int x = (int)(blockIdx.x * kBlock + threadIdx.x); x < a.n; x += (int)(gridDim.x * kBlock)) {
        float d[kQ7];
        thermal_pull(a, x, d);
        float drho, j, dE;
        thermal_moments(d, drho, j, dE);
        acc[0] += drho;
        acc[1] += j;
        acc[2] += dE;
    }
    __shared__ double sh[kBlock / 64][3];
    for (int c = 0; c < 3; ++c)
        for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 64);
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < 3; ++c) sh[threadIdx.x >> 6][c] = acc[c];
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w][threadIdx.x];
        a.partials[(size_t)blockIdx.x * 3 + threadIdx.x] = t;
    }
}

}  // namespace

hipError_t launch_thermal(int mode, const ThermalArgs &a, int nblocks_reduce, hipStream_t st)
{
    const dim3 block(kBlock), grid((a.n + kBlock - 1) / kBlock);
    switch (mode) {
    case 0:
        if (!a.src || !a.dst || a.src == a.dst) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_thermal_step, grid, block, 0, st, a);
        break;
    case 1:
        if (!a.dst || !a.rho) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_thermal_init, grid, block, 0, st, a);
        break;
    case 2:
    case 3:
        if (!a.src) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_thermal_fields, grid, block, 0, st, a);
        break;
    case 4:
        if (!a.src || !a.partials || nblocks_reduce < 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_thermal_partials, dim3(nblocks_reduce), block, 0, st, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
