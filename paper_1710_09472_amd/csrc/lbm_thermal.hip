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
// stores at the node. With order 3 (the truncation that carries the momentum equation,
// Sec. 6) p has degree 3 and matches M_0..M_3; the host sets c4's constants to zero.
//
// Precision. Deviations are formed throughout, so that rounding is relative to the
// departure from the weight's state, not to the populations. Velocities are the
// integer e_a (u and thetabar in lattice units), so every power of e_a is exact. The
// polynomial's coefficients come from the moment deviations with the linear parts of
// M_3 and M_4 folded into constants computed in long double: only remainders of second
// order are combined at run time, so no coefficient is a small difference of large terms.
// Populations e = +-2, +-3 take the polynomial's values; e = +-1 then carry the node's
// momentum and second moment and e = 0 its mass (a closure on the conserved moments), so
// that no fixed mismatch of the FP32 constants can drift the conserved totals.
#include "lbm_device.h"

namespace lbm {
namespace {

constexpr int kQ7 = 7;
__device__ constexpr int kE7[kQ7] = {0, 1, -1, 2, -2, 3, -3};
__device__ constexpr float kEf[kQ7] = {0.f, 1.f, -1.f, 2.f, -2.f, 3.f, -3.f};
__device__ constexpr float kE2[kQ7] = {0.f, 1.f, 1.f, 4.f, 4.f, 9.f, 9.f};
__device__ constexpr int kOpp7[kQ7] = {0, 2, 1, 4, 3, 6, 5};

// (x - e) mod n for 0 <= x < n, |e| <= 3: one correction for n >= 3, up to three on the
// shortest grids (n = 1, 2)
__device__ __forceinline__ unsigned wrap_shift(int x, int e, int n)
{
    int s = x - e;
    while (s < 0) s += n;
    while (s >= n) s -= n;
    return (unsigned)s;
}

// Macroscopic fields of a node, lattice units: rho, u_e, thetabar_e - T.
struct ThermalNode {
    float rho, u, dtb;
};

// Deviations feq_a - rho0 what_a of the equilibrium of a node with moment deviations
// drho = sum d, j = sum d e, dE = sum d e^2 (lattice units). SC: the moments and feq are in
// stored units (deviations x p.scale, a power of two); the node's fields rho, u, thetabar
// are formed with p.inv_scale folded into 1/rho, and every other term keeps the stored
// units. Scaling by a power of two is exact, so both give the same bits (the FP16 step
// then decodes and encodes without a multiply per population).
template <bool SC = false>
__device__ __forceinline__ ThermalNode thermal_equilibrium(const ThermalPhysics &p, float drho, float j, float dE,
                                                           float *feq)
{
#pragma clang fp contract(off)  // every fused multiply-add is explicit: the same bits in every kernel
    ThermalNode m;
    m.rho = SC ? __builtin_fmaf(drho, p.inv_scale, p.rho0) : p.rho0 + drho;  // one rounding either way
    const float inv = __builtin_amdgcn_rcpf(m.rho);  // v_rcp_f32 (1 ulp), as in the isothermal step
    const float invs = SC ? inv * p.inv_scale : inv;
    m.u = j * invs;
    const float u2 = m.u * m.u;
    // D = dE - T drho = rho (thetabar - T) + rho u^2   (sum rho0 what e^2 = rho0 T)
    const float D = dE - __builtin_fmaf(p.tb_hi, drho, p.tb_lo * drho);
    const float dtb = __builtin_fmaf(D, invs, -u2);
    m.dtb = dtb;
    // second-order remainders of the targets dM_3, dM_4 (their linear parts are in pe, ko)
    const float r3 = j * __builtin_fmaf(3.0f, dtb, u2);
    const float rho_s = SC ? m.rho * p.scale : m.rho;
    const float r4 = rho_s * __builtin_fmaf(u2, __builtin_fmaf(6.0f, dtb, u2) + p.k6, 3.0f * p.g0 * dtb * dtb);
    const float c0 = __builtin_fmaf(p.he[0], r4, __builtin_fmaf(p.pe[0], D, drho));
    const float c2 = __builtin_fmaf(p.he[1], r4, p.pe[1] * D);
    const float c4 = __builtin_fmaf(p.he[2], r4, p.pe[2] * D);
    const float c1 = __builtin_fmaf(p.ho[0], r3, p.ko[0] * j);
    const float c3 = __builtin_fmaf(p.ho[1], r3, p.ko[1] * j);
#pragma unroll
    for (int a = 3; a < kQ7; ++a) {
        const float x = kEf[a];
        const float poly = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(__builtin_fmaf(c4, x, c3), x, c2), x, c1), x, c0);
        feq[a] = p.what[a] * poly;
    }
    // conservation closure: e = +-1 carry the node's momentum and second moment, e = 0 its
    // mass, so that the collision conserves all three up to the rounding of these sums
    float mj = j, mE = dE;
#pragma unroll
    for (int a = 3; a < kQ7; ++a) {
        mj = __builtin_fmaf(-feq[a], kEf[a], mj);
        mE = __builtin_fmaf(-feq[a], kE2[a], mE);
    }
    feq[1] = 0.5f * (mE + mj);
    feq[2] = 0.5f * (mE - mj);
    float sum = 0.f;
#pragma unroll
    for (int a = 1; a < kQ7; ++a) sum += feq[a];
    feq[0] = drho - sum;
    return m;
}

__device__ __forceinline__ void thermal_moments(const float *d, float &drho, float &j, float &dE)
{
#pragma clang fp contract(off)
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

// Stored value of a deviation: FP32, FP16 x 2^k or BF16 (Codec); ld/st decode and encode.
template <int ST>
using TT = typename Codec<ST>::T;

template <int ST>
__device__ __forceinline__ float tload_nt(const TT<ST> *p, float inv_scale)
{
    return Codec<ST>::dec(__builtin_nontemporal_load(p), inv_scale);
}

// The step kernels work in stored units where the format has a scale (FP16: no multiply
// in decoding and encoding); the other kernels decode to deviations.
template <int ST>
constexpr bool kStoredUnits = ST == LBM_F16;

// The pre-collision populations of node x: slot q of x - e_q (the layout the two-buffer
// step leaves, "even"), or, after the pull phase of the in-place step ("odd"), slot qbar
// of x itself; decoded with inv_scale.
template <int ST>
__device__ __forceinline__ void thermal_pull(const ThermalArgs &a, int x, float *d, float inv_scale)
{
    const TT<ST> *src = static_cast<const TT<ST> *>(a.src);
#pragma unroll
    for (int q = 0; q < kQ7; ++q)
        d[q] = a.odd ? tload_nt<ST>(at32(src + (size_t)kOpp7[q] * a.stride, (unsigned)x), inv_scale)
                     : tload_nt<ST>(at32(src + (size_t)q * a.stride, wrap_shift(x, kE7[q], a.n)), inv_scale);
}

// post-collision deviations of a node from its pre-collision ones (SC: stored units)
template <bool SC>
__device__ __forceinline__ void thermal_collide(const ThermalPhysics &p, const float *d, float *o)
{
    float feq[kQ7], drho, j, dE;
    thermal_moments(d, drho, j, dE);
    thermal_equilibrium<SC>(p, drho, j, dE, feq);
#pragma unroll
    for (int q = 0; q < kQ7; ++q) o[q] = __builtin_fmaf(p.omega, feq[q] - d[q], d[q]);
}

template <int ST>
__global__ __launch_bounds__(kBlock) void k_thermal_step(ThermalArgs a)
{
    const int x = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x >= a.n) return;
    const TT<ST> *src = static_cast<const TT<ST> *>(a.src);
    TT<ST> *dst = static_cast<TT<ST> *>(a.dst);
    constexpr bool SC = kStoredUnits<ST>;
    const float dsc = SC ? 1.f : a.ph.inv_scale, esc = SC ? 1.f : a.ph.scale;
    float d[kQ7], o[kQ7];
    if (x >= 3 && x + 3 < a.n) {
        // no wrap: the rest population is read once (non-temporal); the shifted ones stay
        // cached, since the lines at a tile's edges are shared with the neighbouring tiles
        // (measured 2 % faster than non-temporal loads throughout)
        d[0] = tload_nt<ST>(at32(src, (unsigned)x), dsc);
#pragma unroll
        for (int q = 1; q < kQ7; ++q) d[q] = Codec<ST>::dec(src[(size_t)q * a.stride + (unsigned)(x - kE7[q])], dsc);
    } else {
        thermal_pull<ST>(a, x, d, dsc);
    }
    thermal_collide<SC>(a.ph, d, o);
#pragma unroll
    for (int q = 0; q < kQ7; ++q)
        __builtin_nontemporal_store(Codec<ST>::enc(o[q], esc), at32(dst + (size_t)q * a.stride, (unsigned)x));
}

// The same step with 16-bit storage, two nodes per thread (x0 = 2 i and x0 + 1; n even):
// the two values a population pulls, from x0 - e and x0 + 1 - e, are adjacent, so one
// 4-byte load fetches them (2-byte aligned for odd e: gfx9 global loads allow it), and the
// stores are aligned 4-byte pairs. Threads whose pulls wrap around the ends load the
// values one by one. The node arithmetic is that of k_thermal_step (the same bits).
template <int ST>
__global__ __launch_bounds__(kBlock) void k_thermal_step2(ThermalArgs a)
{
    static_assert(sizeof(TT<ST>) == 2, "pairs of 16-bit values");
    using T = TT<ST>;
    typedef T T2 __attribute__((ext_vector_type(2)));
    typedef uint32_t u32a2 __attribute__((aligned(2)));
    const int x0 = 2 * (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x0 >= a.n) return;
    const T *src = static_cast<const T *>(a.src);
    T *dst = static_cast<T *>(a.dst);
    constexpr bool SC = kStoredUnits<ST>;
    const float dsc = SC ? 1.f : a.ph.inv_scale, esc = SC ? 1.f : a.ph.scale;
    float d0[kQ7], d1[kQ7], o0[kQ7], o1[kQ7];
    if (x0 >= 3 && x0 + 4 < a.n) {
#pragma unroll
        for (int q = 0; q < kQ7; ++q) {
            const T *p = at32(src + (size_t)q * a.stride, (unsigned)(x0 - kE7[q]));
            // the rest population is read once (non-temporal); the shifted pairs share their
            // lines with the neighbouring threads and tiles and stay cached
            const uint32_t w = q == 0 ? __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(p))
                                      : *reinterpret_cast<const u32a2 *>(p);
            d0[q] = Codec<ST>::dec(__builtin_bit_cast(T, (uint16_t)w), dsc);
            d1[q] = Codec<ST>::dec(__builtin_bit_cast(T, (uint16_t)(w >> 16)), dsc);
        }
    } else {
        const int x1 = x0 + 1 < a.n ? x0 + 1 : x0;  // n even: x0 + 1 < n always
#pragma unroll
        for (int q = 0; q < kQ7; ++q) {
            d0[q] = Codec<ST>::dec(*at32(src + (size_t)q * a.stride, wrap_shift(x0, kE7[q], a.n)), dsc);
            d1[q] = Codec<ST>::dec(*at32(src + (size_t)q * a.stride, wrap_shift(x1, kE7[q], a.n)), dsc);
        }
    }
    thermal_collide<SC>(a.ph, d0, o0);
    thermal_collide<SC>(a.ph, d1, o1);
#pragma unroll
    for (int q = 0; q < kQ7; ++q) {
        const T2 v = {Codec<ST>::enc(o0[q], esc), Codec<ST>::enc(o1[q], esc)};
        __builtin_nontemporal_store(v, reinterpret_cast<T2 *>(at32(dst + (size_t)q * a.stride, (unsigned)x0)));
    }
}

// In-place step (one buffer, the AA pattern), phase 0: pull as the two-buffer step does
// (slot q of x - e_q), collide, and store g_q(x) where the opposite population was pulled
// from, slot qbar of x + e_q; each node writes exactly the locations it read, which no
// other node touches. The buffer then holds the streamed ("odd") layout: f_q(x) in slot
// qbar of x.
template <int ST>
__global__ __launch_bounds__(kBlock) void k_thermal_aa_pull(ThermalArgs a)
{
    const int x = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x >= a.n) return;
    TT<ST> *f = static_cast<TT<ST> *>(a.dst);
    constexpr bool SC = kStoredUnits<ST>;
    const float dsc = SC ? 1.f : a.ph.inv_scale, esc = SC ? 1.f : a.ph.scale;
    float d[kQ7], o[kQ7];
    const bool interior = x >= 3 && x + 3 < a.n;
#pragma unroll
    for (int q = 0; q < kQ7; ++q)
        d[q] = Codec<ST>::dec(f[(size_t)q * a.stride + (interior ? (unsigned)(x - kE7[q]) : wrap_shift(x, kE7[q], a.n))],
                              dsc);
    thermal_collide<SC>(a.ph, d, o);
#pragma unroll
    for (int q = 0; q < kQ7; ++q)
        __builtin_nontemporal_store(Codec<ST>::enc(o[q], esc),
                                    at32(f + (size_t)kOpp7[q] * a.stride,
                                         interior ? (unsigned)(x + kE7[q]) : wrap_shift(x, -kE7[q], a.n)));
}

// Phase 1: f_q(x) from slot qbar of x, collide, store g_q(x) in slot q of x (the
// two-buffer layout again).
template <int ST>
__global__ __launch_bounds__(kBlock) void k_thermal_aa_local(ThermalArgs a)
{
    const int x = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x >= a.n) return;
    TT<ST> *f = static_cast<TT<ST> *>(a.dst);
    constexpr bool SC = kStoredUnits<ST>;
    const float dsc = SC ? 1.f : a.ph.inv_scale, esc = SC ? 1.f : a.ph.scale;
    float d[kQ7], o[kQ7];
#pragma unroll
    for (int q = 0; q < kQ7; ++q) d[q] = tload_nt<ST>(at32(f + (size_t)kOpp7[q] * a.stride, (unsigned)x), dsc);
    thermal_collide<SC>(a.ph, d, o);
#pragma unroll
    for (int q = 0; q < kQ7; ++q)
        __builtin_nontemporal_store(Codec<ST>::enc(o[q], esc), at32(f + (size_t)q * a.stride, (unsigned)x));
}

// The two in-place phases with 16-bit storage and two nodes per thread (n even), as
// k_thermal_step2: the pull phase loads and stores shifted pairs (x0 -+ e, x0 + 1 -+ e) with
// one 4-byte access each (2-byte aligned for odd e), the local phase aligned pairs;
// threads whose pairs wrap around the ends go value by value. A thread writes exactly the
// locations its two nodes read, as in the one-node kernels.
template <int ST>
__global__ __launch_bounds__(kBlock) void k_thermal_aa_pull2(ThermalArgs a)
{
    static_assert(sizeof(TT<ST>) == 2, "pairs of 16-bit values");
    using T = TT<ST>;
    typedef uint32_t u32a2 __attribute__((aligned(2)));
    const int x0 = 2 * (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x0 >= a.n) return;
    T *f = static_cast<T *>(a.dst);
    constexpr bool SC = kStoredUnits<ST>;
    const float dsc = SC ? 1.f : a.ph.inv_scale, esc = SC ? 1.f : a.ph.scale;
    float d0[kQ7], d1[kQ7], o0[kQ7], o1[kQ7];
    const bool interior = x0 >= 3 && x0 + 4 < a.n;
    if (interior) {
#pragma unroll
        for (int q = 0; q < kQ7; ++q) {
            const uint32_t w = *reinterpret_cast<const u32a2 *>(at32(f + (size_t)q * a.stride, (unsigned)(x0 - kE7[q])));
            d0[q] = Codec<ST>::dec(__builtin_bit_cast(T, (uint16_t)w), dsc);
            d1[q] = Codec<ST>::dec(__builtin_bit_cast(T, (uint16_t)(w >> 16)), dsc);
        }
    } else {
#pragma unroll
        for (int q = 0; q < kQ7; ++q) {
            d0[q] = Codec<ST>::dec(*at32(f + (size_t)q * a.stride, wrap_shift(x0, kE7[q], a.n)), dsc);
            d1[q] = Codec<ST>::dec(*at32(f + (size_t)q * a.stride, wrap_shift(x0 + 1, kE7[q], a.n)), dsc);
        }
    }
    thermal_collide<SC>(a.ph, d0, o0);
    thermal_collide<SC>(a.ph, d1, o1);
#pragma unroll
    for (int q = 0; q < kQ7; ++q) {
        const T c0 = Codec<ST>::enc(o0[q], esc), c1 = Codec<ST>::enc(o1[q], esc);
        T *row = f + (size_t)kOpp7[q] * a.stride;
        if (interior) {
            const uint32_t w = (uint32_t)__builtin_bit_cast(uint16_t, c0) | ((uint32_t)__builtin_bit_cast(uint16_t, c1) << 16);
            __builtin_nontemporal_store(w, reinterpret_cast<u32a2 *>(at32(row, (unsigned)(x0 + kE7[q]))));
        } else {
            __builtin_nontemporal_store(c0, at32(row, wrap_shift(x0, -kE7[q], a.n)));
            __builtin_nontemporal_store(c1, at32(row, wrap_shift(x0 + 1, -kE7[q], a.n)));
        }
    }
}

template <int ST>
__global__ __launch_bounds__(kBlock) void k_thermal_aa_local2(ThermalArgs a)
{
    static_assert(sizeof(TT<ST>) == 2, "pairs of 16-bit values");
    using T = TT<ST>;
    typedef T T2 __attribute__((ext_vector_type(2)));
    const int x0 = 2 * (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x0 >= a.n) return;
    T *f = static_cast<T *>(a.dst);
    constexpr bool SC = kStoredUnits<ST>;
    const float dsc = SC ? 1.f : a.ph.inv_scale, esc = SC ? 1.f : a.ph.scale;
    float d0[kQ7], d1[kQ7], o0[kQ7], o1[kQ7];
#pragma unroll
    for (int q = 0; q < kQ7; ++q) {
        const T2 v = __builtin_nontemporal_load(reinterpret_cast<const T2 *>(at32(f + (size_t)kOpp7[q] * a.stride, (unsigned)x0)));
        d0[q] = Codec<ST>::dec(v[0], dsc);
        d1[q] = Codec<ST>::dec(v[1], dsc);
    }
    thermal_collide<SC>(a.ph, d0, o0);
    thermal_collide<SC>(a.ph, d1, o1);
#pragma unroll
    for (int q = 0; q < kQ7; ++q) {
        const T2 v = {Codec<ST>::enc(o0[q], esc), Codec<ST>::enc(o1[q], esc)};
        __builtin_nontemporal_store(v, reinterpret_cast<T2 *>(at32(f + (size_t)q * a.stride, (unsigned)x0)));
    }
}

// Odd layout src -> even layout dst: g_q(y) = src slot qbar of y + e_q (stored values moved
// as they are).
template <int ST>
__global__ __launch_bounds__(kBlock) void k_thermal_canon(ThermalArgs a)
{
    const int y = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (y >= a.n) return;
    const TT<ST> *src = static_cast<const TT<ST> *>(a.src);
    TT<ST> *dst = static_cast<TT<ST> *>(a.dst);
#pragma unroll
    for (int q = 0; q < kQ7; ++q)
        dst[(size_t)q * a.stride + y] = src[(size_t)kOpp7[q] * a.stride + wrap_shift(y, -kE7[q], a.n)];
}

// Initial state f = f^eq(rho, u, thetabar): the deviations of node x are stored where
// the first pull into each node reads them, slot q of x - e_q.
template <int ST>
__global__ __launch_bounds__(kBlock) void k_thermal_init(ThermalArgs a)
{
    const int x = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x >= a.n) return;
    const ThermalPhysics &p = a.ph;
    TT<ST> *dst = static_cast<TT<ST> *>(a.dst);
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
    for (int q = 0; q < kQ7; ++q) dst[(size_t)q * a.stride + wrap_shift(x, kE7[q], a.n)] = Codec<ST>::enc(feq[q], p.scale);
}

template <int ST>
__global__ __launch_bounds__(kBlock) void k_thermal_fields(ThermalArgs a)
{
    const int x = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x >= a.n) return;
    float d[kQ7], feq[kQ7];
    thermal_pull<ST>(a, x, d, a.ph.inv_scale);
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
template <int ST>
__global__ __launch_bounds__(kBlock) void k_thermal_partials(ThermalArgs a)
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int x = (int)(blockIdx.x * kBlock + threadIdx.x); x < a.n; x += (int)(gridDim.x * kBlock)) {
        float d[kQ7];
        thermal_pull<ST>(a, x, d, a.ph.inv_scale);
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

template <int ST>
hipError_t launch_thermal_st(int mode, const ThermalArgs &a, int nblocks_reduce, hipStream_t st)
{
    const dim3 block(kBlock), grid((a.n + kBlock - 1) / kBlock);
    switch (mode) {
    case 0:
        if (!a.src || !a.dst || a.src == a.dst) return hipErrorInvalidValue;
        if constexpr (ST != LBM_F32) {
            if (a.n % 2 == 0) {  // two nodes per thread (measured on MI355X: see k_thermal_step2)
                const int pairs = a.n / 2;
                hipLaunchKernelGGL(k_thermal_step2<ST>, dim3((pairs + kBlock - 1) / kBlock), block, 0, st, a);
                break;
            }
        }
        hipLaunchKernelGGL(k_thermal_step<ST>, grid, block, 0, st, a);
        break;
    case 1:
        if (!a.dst || !a.rho) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_thermal_init<ST>, grid, block, 0, st, a);
        break;
    case 2:
    case 3:
        if (!a.src) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_thermal_fields<ST>, grid, block, 0, st, a);
        break;
    case 4:
        if (!a.src || !a.partials || nblocks_reduce < 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_thermal_partials<ST>, dim3(nblocks_reduce), block, 0, st, a);
        break;
    case 5:
    case 6:
        if (!a.dst || a.src != a.dst) return hipErrorInvalidValue;
        if constexpr (ST != LBM_F32) {
            if (a.n % 2 == 0) {  // two nodes per thread
                const dim3 g2((a.n / 2 + kBlock - 1) / kBlock);
                if (mode == 5)
                    hipLaunchKernelGGL(k_thermal_aa_pull2<ST>, g2, block, 0, st, a);
                else
                    hipLaunchKernelGGL(k_thermal_aa_local2<ST>, g2, block, 0, st, a);
                break;
            }
        }
        if (mode == 5)
            hipLaunchKernelGGL(k_thermal_aa_pull<ST>, grid, block, 0, st, a);
        else
            hipLaunchKernelGGL(k_thermal_aa_local<ST>, grid, block, 0, st, a);
        break;
    case 7:
        if (!a.src || !a.dst || a.src == a.dst) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_thermal_canon<ST>, grid, block, 0, st, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_thermal(int mode, int storage, const ThermalArgs &a, int nblocks_reduce, hipStream_t st)
{
    if (storage == LBM_F32) return launch_thermal_st<LBM_F32>(mode, a, nblocks_reduce, st);
    if (storage == LBM_F16) return launch_thermal_st<LBM_F16>(mode, a, nblocks_reduce, st);
    if (storage == LBM_BF16) return launch_thermal_st<LBM_BF16>(mode, a, nblocks_reduce, st);
    return hipErrorInvalidValue;
}

}  // namespace lbm
