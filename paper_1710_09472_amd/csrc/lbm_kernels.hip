// lbm_kernels.hip -- gfx950 kernels of the semiclassical lattice Boltzmann step.
//
// One thread per lattice node, 256 threads (4 wave64) per block along x. The state
// holds post-collision populations of the previous step as structure-of-arrays
// deviations d_a = f_a - what_a rho0 (FP32, FP16 x 2^k or BF16); a step pulls
// f_a(x) = g_a(x - e_a) from the neighbours (misaligned by at most one element in x,
// whole rows in y and z), or g_abar(x) when x - e_a is solid (halfway bounce-back),
// collides in FP32 registers and writes its own node's Q values to the other buffer:
// every population is read once and written once per step.
//
// The block index is remapped so that each of the 8 XCDs (which receive blocks
// round-robin) works on one contiguous slab of the grid; neighbouring tiles, whose
// x-halo cache lines overlap, then share an L2.
#include "lbm_internal.h"

namespace lbm {
namespace {

// ---------------------------------------------------------------------------------
// Storage codecs: deviation <-> stored value.
// ---------------------------------------------------------------------------------
template <int ST>
struct Codec;

template <>
struct Codec<LBM_F32> {
    using T = float;
    static __device__ __forceinline__ float dec(T v, float) { return v; }
    static __device__ __forceinline__ T enc(float f, float) { return f; }
};

template <>
struct Codec<LBM_F16> {
    using T = _Float16;
    // value = d * 2^k: the scale is a power of two, so scaling is exact
    static __device__ __forceinline__ float dec(T v, float inv_scale) { return (float)v * inv_scale; }
    static __device__ __forceinline__ T enc(float f, float scale) { return (T)(f * scale); }  // RNE
};

template <>
struct Codec<LBM_BF16> {
    using T = uint16_t;
    static __device__ __forceinline__ float dec(T v, float) { return __uint_as_float(((uint32_t)v) << 16); }
    static __device__ __forceinline__ T enc(float f, float)
    {
        uint32_t u = __float_as_uint(f);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (T)((u >> 16) | 0x0040u);  // keep NaN a NaN
        u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
        return (T)(u >> 16);
    }
};

// Block -> contiguous slab per XCD (blocks are dealt to the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = bid & 7, k = bid >> 3;
    return xcd * per + min(xcd, rem) + k;
}

struct Node {
    int x, y, z, n;
};

// Node of this thread, or n = -1 past the end of a row.
__device__ __forceinline__ Node node_of_thread(const Geometry &g, bool remap)
{
    const int bid = remap ? xcd_remap((int)blockIdx.x, g.nblocks) : (int)blockIdx.x;
    const int row = bid / g.ntx;
    Node nd;
    nd.x = (bid - row * g.ntx) * kBlock + (int)threadIdx.x;
    nd.y = row % g.ny;
    nd.z = row / g.ny;
    nd.n = nd.x < g.nx ? nd.x + g.nx * row : -1;
    return nd;
}

__device__ __forceinline__ int wrapm(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wrapp(int i, int n) { return i == n - 1 ? 0 : i + 1; }

// Pull the pre-collision deviations of node nd from the post-collision state.
template <int LAT, int ST, bool MASK>
__device__ __forceinline__ void gather(const Geometry &g, const typename Codec<ST>::T *__restrict__ src,
                                       float inv_scale, const Node &nd, float *d)
{
    using L = Lat<LAT>;
    const int xm = wrapm(nd.x, g.nx), xp = wrapp(nd.x, g.nx);
    const int ym = wrapm(nd.y, g.ny), yp = wrapp(nd.y, g.ny);
    const int zm = wrapm(nd.z, g.nz), zp = wrapp(nd.z, g.nz);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const int sx = L::ex[q] > 0 ? xm : (L::ex[q] < 0 ? xp : nd.x);
        const int sy = L::ey[q] > 0 ? ym : (L::ey[q] < 0 ? yp : nd.y);
        const int sz = L::ez[q] > 0 ? zm : (L::ez[q] < 0 ? zp : nd.z);
        const int sn = sx + g.nx * (sy + g.ny * sz);
        int idx = q * g.stride + sn;
        if (MASK && q != 0) {
            if (g.mask[sn]) idx = L::opp[q] * g.stride + nd.n;
        }
        d[q] = Codec<ST>::dec(src[idx], inv_scale);
    }
}

// Macroscopic quantities from pre-collision deviations:
// drho = sum d, rho = rho0 + drho, U = u / c_s = (sum d e) / (rho c_s^2).
template <int LAT>
struct Macro {
    float drho, rho, j[3], U[3], U2;  // j = sum d e (lattice units), U = j / (rho c_s^2)
};

template <int LAT>
__device__ __forceinline__ Macro<LAT> macro(const Physics &p, const float *d)
{
    using L = Lat<LAT>;
    Macro<LAT> m;
    float r = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        r += d[q];
        if (L::ex[q]) jx += L::ex[q] * d[q];
        if (L::ey[q]) jy += L::ey[q] * d[q];
        if (L::ez[q]) jz += L::ez[q] * d[q];
    }
    m.drho = r;
    m.rho = p.rho0 + r;
    m.j[0] = jx;
    m.j[1] = jy;
    m.j[2] = jz;
    const float k = p.inv_cs2 / m.rho;
    m.U[0] = jx * k;
    m.U[1] = jy * k;
    m.U[2] = jz * k;
    m.U2 = m.U[0] * m.U[0] + m.U[1] * m.U[1] + m.U[2] * m.U[2];
    return m;
}

template <int LAT, int q>
__device__ __forceinline__ float edot(const float *v)
{
    using L = Lat<LAT>;
    float r = 0.f;
    if (L::ex[q]) r += L::ex[q] * v[0];
    if (L::ey[q]) r += L::ey[q] * v[1];
    if (L::ez[q]) r += L::ez[q] * v[2];
    return r;
}

template <int LAT, int q>
__device__ __forceinline__ constexpr int shell()
{
    using L = Lat<LAT>;
    return L::ex[q] * L::ex[q] + L::ey[q] * L::ey[q] + L::ez[q] * L::ez[q];
}

// Unrolled compile-time loop over q.
template <int Q, int q = 0, typename F>
__device__ __forceinline__ void for_q(F &&f)
{
    if constexpr (q < Q) {
        f(std::integral_constant<int, q>{});
        for_q<Q, q + 1>(f);
    }
}

// Equilibrium deviation of a moving population q != 0 (reduced EDF of Sec. 9.1):
//   deq_q = what_k drho + lam_k (e.j) + what_k rho (Bc (e.U)^2 + C_k c_s^2 U^2),
// where lam_k (e.j) = what_k rho A (e.U). Written with e.j and weights lam_k whose
// second moment is exactly the identity, the equilibrium carries exactly the momentum
// j of the node: FP32 rounding of the constants then cannot bias momentum relaxation.
// The rest population is closed by mass conservation, deq_0 = drho - sum_(q != 0) deq_q.
template <int LAT, int q>
__device__ __forceinline__ float deq_moving(const Physics &p, float drho, float rho, const float *j,
                                            const float *U, float U2, float sign = 1.f)
{
    constexpr int k = shell<LAT, q>();
    const float eu = sign * edot<LAT, q>(U);
    const float ej = sign * edot<LAT, q>(j);
    return p.what[k] * drho + p.lam[k] * ej + p.what[k] * rho * (p.Bc * eu * eu + p.Cp[k] * U2);
}

// Post-collision values of one node (deviation form), before partial bounce-back:
//   d*_q = d_q + omega (deq_q - d_q) + rho what_q sigma_q,
//   sigma_q = (e.E / c_s)(A + 2 Bc e.U) + 2 C_k (c_s U.E + e.(B x U))   (source of Sec. 7).
// deq (optional) receives the equilibrium deviations.
template <int LAT, bool MAG>
__device__ __forceinline__ void collide_bgk(const Physics &p, const Macro<LAT> &m, const float *d, float *o,
                                            float *deq_out = nullptr)
{
    using L = Lat<LAT>;
    const float UE = p.cs * (m.U[0] * p.E[0] + m.U[1] * p.E[1] + m.U[2] * p.E[2]);
    float W[3] = {0.f, 0.f, 0.f};
    if (MAG) {
        W[0] = p.B[1] * m.U[2] - p.B[2] * m.U[1];
        W[1] = p.B[2] * m.U[0] - p.B[0] * m.U[2];
        W[2] = p.B[0] * m.U[1] - p.B[1] * m.U[0];
    }
    const float inv_cs = p.cs * p.inv_cs2;
    const float om = p.omega;
    float sum_eq = 0.f;
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (q != 0) {
            constexpr int k = shell<LAT, q>();
            const float eu = edot<LAT, q>(m.U);
            const float eE = edot<LAT, q>(p.E) * inv_cs;
            const float deq = deq_moving<LAT, q>(p, m.drho, m.rho, m.j, m.U, m.U2);
            sum_eq += deq;
            float sig = eE * (p.A + 2.f * p.Bc * eu) + 2.f * p.C[k] * UE;
            if (MAG) sig += 2.f * p.C[k] * edot<LAT, q>(W);
            o[q] = d[q] + om * (deq - d[q]) + m.rho * p.what[k] * sig;
            if (deq_out) deq_out[q] = deq;
        }
    });
    const float deq0 = m.drho - sum_eq;
    o[0] = d[0] + om * (deq0 - d[0]) + m.rho * p.what[0] * (2.f * p.C[0] * UE);
    if (deq_out) deq_out[0] = deq0;
}

// Collision of one node (discrete BGK of Sec. 9.1 with the source of Sec. 7), then the
// optional partial bounce-back g_q = (1 - s) d*_q + s d_qbar.
template <int LAT, bool SOFT, bool MAG>
__device__ __forceinline__ void collide(const Physics &p, const float *d, float s, float *o)
{
    using L = Lat<LAT>;
    const Macro<LAT> m = macro<LAT>(p, d);
    collide_bgk<LAT, MAG>(p, m, d, o);
    if (SOFT) {
        float t[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) t[q] = (1.f - s) * o[q] + s * d[L::opp[q]];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) o[q] = t[q];
    }
}

// ---------------------------------------------------------------------------------
// K1: fused pull-stream + collide + force + partial bounce-back.
// ---------------------------------------------------------------------------------
template <int LAT, int ST, bool MASK, bool SOFT, bool MAG>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs a)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    const Node nd = node_of_thread(a.g, true);
    if (nd.n < 0) return;
    if (MASK && a.g.mask[nd.n]) return;
    float d[L::Q], o[L::Q];
    gather<LAT, ST, MASK>(a.g, static_cast<const T *>(a.src), a.ph.inv_scale, nd, d);
    collide<LAT, SOFT, MAG>(a.ph, d, SOFT ? a.g.s[nd.n] : 0.f, o);
    T *__restrict__ dst = static_cast<T *>(a.dst);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) dst[q * a.g.stride + nd.n] = Codec<ST>::enc(o[q], a.ph.scale);
}

// ---------------------------------------------------------------------------------
// K2: initial state. The stored state is post-collision, so node y holds, for each q,
// the value that the next pull delivers: f^eq_q(x + e_q) when x + e_q is fluid, or
// f^eq_qbar(x) when it is solid (bounced back).
// ---------------------------------------------------------------------------------
template <int LAT, int ST>
__global__ __launch_bounds__(kBlock) void k_init(InitArgs a)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    const Node nd = node_of_thread(a.g, false);
    if (nd.n < 0) return;
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const Geometry &g = a.g;
    const Physics &p = a.ph;
    const int N = g.nx * g.ny * g.nz;
    if (g.mask && g.mask[nd.n]) {
#pragma unroll
        for (int q = 0; q < L::Q; ++q) dst[q * g.stride + nd.n] = Codec<ST>::enc(0.f, p.scale);
        return;
    }
    const int xm = wrapm(nd.x, g.nx), xp = wrapp(nd.x, g.nx);
    const int ym = wrapm(nd.y, g.ny), yp = wrapp(nd.y, g.ny);
    const int zm = wrapm(nd.z, g.nz), zp = wrapp(nd.z, g.nz);
    const float inv_cs = p.cs * p.inv_cs2;
    // rho, j, U of a node from the caller's FP64 fields (u in xi-units, j = rho c_s u)
    auto node_state = [&](int m, float &drho, float &rho, float *j, float *U, float &U2) {
        const double r = a.rho[m];
        drho = (float)(r - (double)p.rho0);
        rho = (float)r;
        for (int i = 0; i < 3; ++i) {
            const double ui = (a.u && i < L::D) ? a.u[(size_t)i * N + m] : 0.0;
            U[i] = (float)ui * inv_cs;
            j[i] = (float)(r * ui * (double)p.cs);
        }
        U2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    };
    float drho0, rho0, j0[3], U0[3], U20;
    node_state(nd.n, drho0, rho0, j0, U0, U20);
    float sum_eq = 0.f;
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (q != 0) sum_eq += deq_moving<LAT, q>(p, drho0, rho0, j0, U0, U20);
    });
    dst[nd.n] = Codec<ST>::enc(drho0 - sum_eq, p.scale);
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (q != 0) {
            const int tx = L::ex[q] > 0 ? xp : (L::ex[q] < 0 ? xm : nd.x);
            const int ty = L::ey[q] > 0 ? yp : (L::ey[q] < 0 ? ym : nd.y);
            const int tz = L::ez[q] > 0 ? zp : (L::ez[q] < 0 ? zm : nd.z);
            const int tn = tx + g.nx * (ty + g.ny * tz);
            float dev;
            if (g.mask && g.mask[tn]) {
                dev = deq_moving<LAT, q>(p, drho0, rho0, j0, U0, U20, -1.f);  // f^eq of the opposite direction
            } else {
                float dr, r, j[3], U[3], U2;
                node_state(tn, dr, r, j, U, U2);
                dev = deq_moving<LAT, q>(p, dr, r, j, U, U2);
            }
            dst[q * g.stride + nd.n] = Codec<ST>::enc(dev, p.scale);
        }
    });
}

// ---------------------------------------------------------------------------------
// K3/K4: gather kernels. MODE 0: rho and u fields; 1: FP64 export of the populations;
// 2: per-block FP64 partial sums (sum drho, sum d e_x, sum d e_y, sum d e_z, nodes).
// ---------------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void block_sum_store(double *v, double *out)
{
    __shared__ double sh[kBlock / 64][NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < NC; ++c) sh[wid][c] = v[c];
    __syncthreads();
    if (threadIdx.x < NC) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

template <int LAT, int ST, bool MASK, int MODE>
__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs a)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    const T *src = static_cast<const T *>(a.src);
    if constexpr (MODE == 2) {
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int b = blockIdx.x; b < a.g.nblocks; b += gridDim.x) {
            const int row = b / a.g.ntx;
            Node nd;
            nd.x = (b - row * a.g.ntx) * kBlock + (int)threadIdx.x;
            nd.y = row % a.g.ny;
            nd.z = row / a.g.ny;
            if (nd.x >= a.g.nx) continue;
            nd.n = nd.x + a.g.nx * row;
            if (MASK && a.g.mask[nd.n]) continue;
            float d[L::Q];
            gather<LAT, ST, MASK>(a.g, src, a.ph.inv_scale, nd, d);
            float r = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
            for (int q = 0; q < L::Q; ++q) {
                r += d[q];
                jx += L::ex[q] * d[q];
                jy += L::ey[q] * d[q];
                jz += L::ez[q] * d[q];
            }
            acc[0] += r;
            acc[1] += jx;
            acc[2] += jy;
            acc[3] += jz;
            acc[4] += 1.0;
        }
        block_sum_store<5>(acc, a.partials + (size_t)blockIdx.x * 5);
    } else {
        const Node nd = node_of_thread(a.g, false);
        if (nd.n < 0) return;
        const bool solid = MASK && a.g.mask[nd.n];
        float d[L::Q];
        if (!solid) gather<LAT, ST, MASK>(a.g, src, a.ph.inv_scale, nd, d);
        if constexpr (MODE == 0) {
            if (solid) {
                if (a.rho) a.rho[nd.n] = 0.f;
                if (a.u)
                    for (int i = 0; i < L::D; ++i) a.u[(size_t)i * a.N + nd.n] = 0.f;
                return;
            }
            const Macro<LAT> m = macro<LAT>(a.ph, d);
            if (a.rho) a.rho[nd.n] = m.rho;
            if (a.u)
                for (int i = 0; i < L::D; ++i) a.u[(size_t)i * a.N + nd.n] = m.U[i] * a.ph.cs;
        } else {
            for_q<L::Q>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int k = shell<LAT, q>();
                a.f64[(size_t)q * a.N + nd.n] = solid ? 0.0 : a.what_rho0[k] + (double)d[q];
            });
        }
    }
}

// Final reduction of per-block partials: out[c] (+)= sum_b partials[b*ncomp + c].
__global__ __launch_bounds__(kBlock) void k_reduce_final(const double *__restrict__ partials, int nparts,
                                                         int ncomp, double *out, int accumulate)
{
    __shared__ double sh[kBlock / 64];
    for (int c = 0; c < ncomp; ++c) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nparts; b += kBlock) v += partials[(size_t)b * ncomp + c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
            out[c] = accumulate ? out[c] + t : t;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------
// K5: one reverse step of the discrete adjoint. lam_out = dJ/df(t) from
// lam_in = dJ/df(t+1); f(t) is pulled from the stored state as in K1.
//   gbar_a = lam_in(x + e_a, a), or lam_in(x, abar) if x + e_a is solid;
//   hbar_a = (1 - s) gbar_a;
//   dJ/ds  += sum_a gbar_a (d_abar - d*_a);
//   dJ/dtau += omega^2 sum_a hbar_a (d_a - deq_a);
//   dJ/dE_i += sum_a hbar_a rho what_a [(A + 2 Bc e.U) e_i / c_s + 2 C_k c_s U_i];
//   rhobar = sum_a hbar_a what_a [omega (1 + P_a) + sigma_a];
//   V_i = sum_a hbar_a what_a [omega (A e_i + 2 Bc (e.U) e_i + 2 C_k c_s^2 U_i)
//                              + 2 Bc e_i (e.E)/c_s + 2 C_k (c_s E_i + (e x B)_i)];
//   lam_out_b = (1 - omega) hbar_b + s gbar_bbar + rhobar + V . (e_b / c_s^2 - U).
// ---------------------------------------------------------------------------------
template <int LAT, int ST, bool MASK, bool SOFT, bool MAG>
__global__ __launch_bounds__(kBlock) void k_adjoint(AdjointArgs a)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    const Geometry &g = a.g;
    const Physics &p = a.ph;
    const Node nd = node_of_thread(g, true);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (nd.n >= 0) {
        if (MASK && g.mask[nd.n]) {
#pragma unroll
            for (int q = 0; q < L::Q; ++q) a.lam_out[q * g.stride + nd.n] = 0.f;
        } else {
            float d[L::Q], gb[L::Q];
            gather<LAT, ST, MASK>(g, static_cast<const T *>(a.state), p.inv_scale, nd, d);
            {
                const int xm = wrapm(nd.x, g.nx), xp = wrapp(nd.x, g.nx);
                const int ym = wrapm(nd.y, g.ny), yp = wrapp(nd.y, g.ny);
                const int zm = wrapm(nd.z, g.nz), zp = wrapp(nd.z, g.nz);
#pragma unroll
                for (int q = 0; q < L::Q; ++q) {
                    const int tx = L::ex[q] > 0 ? xp : (L::ex[q] < 0 ? xm : nd.x);
                    const int ty = L::ey[q] > 0 ? yp : (L::ey[q] < 0 ? ym : nd.y);
                    const int tz = L::ez[q] > 0 ? zp : (L::ez[q] < 0 ? zm : nd.z);
                    const int tn = tx + g.nx * (ty + g.ny * tz);
                    int idx = q * g.stride + tn;
                    if (MASK && q != 0) {
                        if (g.mask[tn]) idx = L::opp[q] * g.stride + nd.n;
                    }
                    gb[q] = a.lam_in[idx];
                }
            }
            const float s = SOFT ? g.s[nd.n] : 0.f;
            const Macro<LAT> m = macro<LAT>(p, d);
            float dst[L::Q], deq[L::Q];
            collide_bgk<LAT, MAG>(p, m, d, dst, deq);
            const float UE = p.cs * (m.U[0] * p.E[0] + m.U[1] * p.E[1] + m.U[2] * p.E[2]);
            float W[3] = {0.f, 0.f, 0.f};
            if (MAG) {
                W[0] = p.B[1] * m.U[2] - p.B[2] * m.U[1];
                W[1] = p.B[2] * m.U[0] - p.B[0] * m.U[2];
                W[2] = p.B[0] * m.U[1] - p.B[1] * m.U[0];
            }
            const float inv_cs = p.cs * p.inv_cs2;
            const float om = p.omega;
            const float inv_rho = 1.f / m.rho;
            float ds = 0.f, dtau = 0.f, dE[3] = {0.f, 0.f, 0.f}, rbar = 0.f, V[3] = {0.f, 0.f, 0.f};
            float hb[L::Q];
            for_q<L::Q>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int k = shell<LAT, q>();
                constexpr int ex = L::ex[q], ey = L::ey[q], ez = L::ez[q];
                const float eu = edot<LAT, q>(m.U);
                const float eE = edot<LAT, q>(p.E) * inv_cs;
                float sig = eE * (p.A + 2.f * p.Bc * eu) + 2.f * p.C[k] * UE;
                if (MAG) sig += 2.f * p.C[k] * edot<LAT, q>(W);
                const float h = (1.f - s) * gb[q];
                hb[q] = h;
                if (SOFT) ds += gb[q] * (d[L::opp[q]] - dst[q]);
                dtau += h * (d[q] - deq[q]);
                const float hw = h * p.what[k];
                const float cE = (p.A + 2.f * p.Bc * eu) * inv_cs;
                const float c2 = 2.f * p.C[k];
                // dS/dE_i = rho what [cE e_i + 2 C_k c_s U_i]
                dE[0] += hw * (cE * ex + c2 * p.cs * m.U[0]);
                dE[1] += hw * (cE * ey + c2 * p.cs * m.U[1]);
                dE[2] += hw * (cE * ez + c2 * p.cs * m.U[2]);
                // Phi_q / rho = omega f^eq_q / rho + what_q sigma_q, f^eq_q = what_q rho0 + deq_q
                rbar += h * (om * (p.what[k] * p.rho0 + deq[q]) * inv_rho) + hw * sig;
                const float a1 = om * (p.A + 2.f * p.Bc * eu) + 2.f * p.Bc * eE;  // times e_i
                const float a2 = om * 2.f * p.Cp[k];                                // times U_i
                float eB[3] = {0.f, 0.f, 0.f};
                if (MAG) {
                    eB[0] = ey * p.B[2] - ez * p.B[1];
                    eB[1] = ez * p.B[0] - ex * p.B[2];
                    eB[2] = ex * p.B[1] - ey * p.B[0];
                }
                V[0] += hw * (a1 * ex + a2 * m.U[0] + c2 * (p.cs * p.E[0] + eB[0]));
                V[1] += hw * (a1 * ey + a2 * m.U[1] + c2 * (p.cs * p.E[1] + eB[1]));
                V[2] += hw * (a1 * ez + a2 * m.U[2] + c2 * (p.cs * p.E[2] + eB[2]));
            });
            const float VU = V[0] * m.U[0] + V[1] * m.U[1] + V[2] * m.U[2];
            const float base = rbar - VU;
            const float vi = p.inv_cs2;
            for_q<L::Q>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                const float ev = edot<LAT, q>(V) * vi;
                float out = (1.f - om) * hb[q] + base + ev;
                if (SOFT) out += s * gb[L::opp[q]];
                a.lam_out[q * g.stride + nd.n] = out;
            });
            if (SOFT && g.s && a.grad_s) a.grad_s[nd.n] += ds;
            acc[0] = (double)m.rho * (double)dE[0];
            acc[1] = (double)m.rho * (double)dE[1];
            acc[2] = (double)m.rho * (double)dE[2];
            acc[3] = (double)(om * om) * (double)dtau;
        }
    }
    if (a.partials) block_sum_store<4>(acc, a.partials + (size_t)blockIdx.x * 4);
}

// Adjoint seed: lam(a, n) = e_a[axis] * value at fluid nodes (value = 1/(c_s norm)).
template <int LAT>
__global__ __launch_bounds__(kBlock) void k_seed(Geometry g, float value, int axis, float *lam)
{
    using L = Lat<LAT>;
    const Node nd = node_of_thread(g, false);
    if (nd.n < 0) return;
    const bool solid = g.mask && g.mask[nd.n];
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const int e = axis == 0 ? L::ex[q] : (axis == 1 ? L::ey[q] : L::ez[q]);
        lam[q * g.stride + nd.n] = solid ? 0.f : (float)e * value;
    }
}

}  // namespace
}  // namespace lbm
// ---------------------------------------------------------------------------------
// Launchers: runtime flags -> template instances.
// ---------------------------------------------------------------------------------
namespace lbm {
namespace {

template <int LAT, int ST>
hipError_t step_lat_st(bool mag, const StepArgs &a, hipStream_t st)
{
    const bool mask = a.g.mask != nullptr, soft = a.g.s != nullptr;
    const dim3 grid(a.g.nblocks), block(kBlock);
#define LBM_STEP(M, S, B) hipLaunchKernelGGL((k_step<LAT, ST, M, S, B>), grid, block, 0, st, a)
    if (mask) {
        if (soft) {
            if (mag) LBM_STEP(true, true, true); else LBM_STEP(true, true, false);
        } else {
            if (mag) LBM_STEP(true, false, true); else LBM_STEP(true, false, false);
        }
    } else {
        if (soft) {
            if (mag) LBM_STEP(false, true, true); else LBM_STEP(false, true, false);
        } else {
            if (mag) LBM_STEP(false, false, true); else LBM_STEP(false, false, false);
        }
    }
#undef LBM_STEP
    return hipGetLastError();
}

template <int LAT, int ST>
hipError_t adjoint_lat_st(bool mag, const AdjointArgs &a, hipStream_t st)
{
    const bool mask = a.g.mask != nullptr, soft = a.g.s != nullptr;
    const dim3 grid(a.g.nblocks), block(kBlock);
#define LBM_ADJ(M, S, B) hipLaunchKernelGGL((k_adjoint<LAT, ST, M, S, B>), grid, block, 0, st, a)
    if (mask) {
        if (soft) {
            if (mag) LBM_ADJ(true, true, true); else LBM_ADJ(true, true, false);
        } else {
            if (mag) LBM_ADJ(true, false, true); else LBM_ADJ(true, false, false);
        }
    } else {
        if (soft) {
            if (mag) LBM_ADJ(false, true, true); else LBM_ADJ(false, true, false);
        } else {
            if (mag) LBM_ADJ(false, false, true); else LBM_ADJ(false, false, false);
        }
    }
#undef LBM_ADJ
    return hipGetLastError();
}

template <int LAT, int ST>
hipError_t gather_lat_st(const GatherArgs &a, int nred, hipStream_t st)
{
    const bool mask = a.g.mask != nullptr;
    const dim3 block(kBlock);
    const int mode = a.partials ? 2 : (a.f64 ? 1 : 0);
    const dim3 grid(mode == 2 ? nred : a.g.nblocks);
#define LBM_G(M, MODE) hipLaunchKernelGGL((k_gather<LAT, ST, M, MODE>), grid, block, 0, st, a)
    if (mask) {
        if (mode == 0) LBM_G(true, 0); else if (mode == 1) LBM_G(true, 1); else LBM_G(true, 2);
    } else {
        if (mode == 0) LBM_G(false, 0); else if (mode == 1) LBM_G(false, 1); else LBM_G(false, 2);
    }
#undef LBM_G
    return hipGetLastError();
}

}  // namespace

#define LBM_DISPATCH(FN, ...)                                                             \
    do {                                                                                  \
        if (lattice == LBM_D2V9) {                                                        \
            if (storage == LBM_F32) return FN<LBM_D2V9, LBM_F32>(__VA_ARGS__);            \
            if (storage == LBM_F16) return FN<LBM_D2V9, LBM_F16>(__VA_ARGS__);            \
            if (storage == LBM_BF16) return FN<LBM_D2V9, LBM_BF16>(__VA_ARGS__);          \
        } else if (lattice == LBM_D3V19) {                                                \
            if (storage == LBM_F32) return FN<LBM_D3V19, LBM_F32>(__VA_ARGS__);           \
            if (storage == LBM_F16) return FN<LBM_D3V19, LBM_F16>(__VA_ARGS__);           \
            if (storage == LBM_BF16) return FN<LBM_D3V19, LBM_BF16>(__VA_ARGS__);         \
        }                                                                                 \
        return hipErrorInvalidValue;                                                      \
    } while (0)

hipError_t launch_step(int lattice, int storage, bool mag, const StepArgs &a, hipStream_t st)
{
    LBM_DISPATCH(step_lat_st, mag, a, st);
}

hipError_t launch_adjoint(int lattice, int storage, bool mag, const AdjointArgs &a, hipStream_t st)
{
    LBM_DISPATCH(adjoint_lat_st, mag, a, st);
}

hipError_t launch_gather(int lattice, int storage, const GatherArgs &a, int nblocks_reduce, hipStream_t st)
{
    LBM_DISPATCH(gather_lat_st, a, nblocks_reduce, st);
}

namespace {
template <int LAT, int ST>
hipError_t init_lat_st(const InitArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_init<LAT, ST>), dim3(a.g.nblocks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_init(int lattice, int storage, const InitArgs &a, hipStream_t st)
{
    LBM_DISPATCH(init_lat_st, a, st);
}

hipError_t launch_reduce_final(const double *partials, int nparts, int ncomp, double *out, int accumulate,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, partials, nparts, ncomp, out, accumulate);
    return hipGetLastError();
}

hipError_t launch_seed(int lattice, const Geometry &g, float value, int axis, float *lam, hipStream_t st)
{
    if (lattice == LBM_D2V9)
        hipLaunchKernelGGL(k_seed<LBM_D2V9>, dim3(g.nblocks), dim3(kBlock), 0, st, g, value, axis, lam);
    else if (lattice == LBM_D3V19)
        hipLaunchKernelGGL(k_seed<LBM_D3V19>, dim3(g.nblocks), dim3(kBlock), 0, st, g, value, axis, lam);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace lbm
