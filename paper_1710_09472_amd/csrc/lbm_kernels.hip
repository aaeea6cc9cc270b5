// lbm_kernels.hip -- gfx950 kernels of the semiclassical lattice Boltzmann step.
//
// Layout: the state holds the post-collision populations of the previous step as
// structure-of-arrays deviations d_a = f_a - what_a rho0 (FP32, FP16 x 2^k or BF16),
// array a at offset a*stride, node n = x + nx*(y + ny*z). A step pulls
// f_a(x) = g_a(x - e_a) from the neighbours (halfway bounce-back where x - e_a is solid,
// specular reflection where it lies in a free-slip wall plane), collides in FP32
// registers and writes the node's Q values to the other buffer: every population is read
// once and written once per step.
//
// Launch: 256 threads (4 wave64) per block over part of one x row; each thread owns V
// consecutive nodes (V = 1 or 2), so the arrays are read and written with V-wide vector
// accesses; the one value of an x-shifted population that falls outside the thread's V
// nodes is fetched with a scalar load (it lies in a neighbouring lane's cache line). All
// loads of a thread are issued before any arithmetic. Where there are solids or soft
// fields, blocks are remapped so that each of the 8 XCDs (which receive blocks
// round-robin) works on one contiguous slab of the grid. Solid nodes are described by a
// per-node link mask built once: bit a set when the pull of a into x bounces back, top
// bit set when x itself is solid.
#include "lbm_step_kernels.h"

#include <cstdlib>
#include <mutex>

namespace lbm {

static int env_int(const char *name, int dflt)
{
    const char *e = std::getenv(name);
    return e ? std::atoi(e) : dflt;
}

// Nodes per thread of the step kernel (measured on MI355X): 1 for FP32 and for D3V19,
// 2 for 16-bit D2V9 except in the local phase of the in-place step with solids (FP16
// 2048^2 disks in place: pull phase 33.0 us with one node per thread, 30.8 us with two;
// local phase 46.4 us with one, 53.7 us with two); halved until it divides nx. The
// layout and the bits are the same for either width. LBM_STEP_VEC=1|2 overrides it.
int step_vector_width(int lattice, int storage, int nx, bool local_phase_solids)
{
    static const int forced = env_int("LBM_STEP_VEC", 0);
    int v = forced;
    if (v != 1 && v != 2) v = (storage != LBM_F32 && lattice == LBM_D2V9 && !local_phase_solids) ? 2 : 1;
    while (v > 1 && nx % v) v >>= 1;
    return v;
}

// XCD-contiguous block order (measured on MI355X): it pays off where the reads of a node
// span several rows of solids or planes (D3V19, masks, porosity fields) and costs ~8 %
// on the plain D2V9 grid, which keeps the hardware order. 2 asks for whole rows of tiles
// per XCD, dealt round-robin (block_order; remap_code turns it into the kernel's code).
// LBM_XCD_REMAP=0|1|2 overrides.
int use_xcd_remap(int lattice, bool mask, bool soft)
{
    static const int forced = env_int("LBM_XCD_REMAP", -1);
    if (forced == 0 || forced == 1 || forced == 2) return forced;
    return (lattice == LBM_D3V19 || mask || soft) ? 1 : 0;
}

// The block_order code of a launch with ntx tiles per row: 2 + log2(ntx) for whole rows
// per XCD where ntx is a power of two, the hardware order where it is not.
int remap_code(int remap, int ntx)
{
    if (remap != 2) return remap;
    if (ntx < 1 || (ntx & (ntx - 1))) return 0;
    int sh = 0;
    while ((1 << sh) < ntx) ++sh;
    return 2 + sh;
}

// One block per row where the row fits in a block: the row's waves only (tile_of then
// maps thread i to node i * V of the row for any block size). Measured on MI355X on the
// 128^3 grids, where a 256-thread block used to carry two idle waves.
int row_block_threads(int nx, int V)
{
    const int per = (nx + V - 1) / V;
    if (per > kBlock) return kBlock;
    return (per + 63) / 64 * 64;
}

namespace {

// ---------------------------------------------------------------------------------
// Link masks: the top bit when x is solid (an obstacle of the mask or a node of a
// free-slip wall plane), and then no other bit; for a fluid x, bit q when the pull of
// population q into x bounces back, i.e. its source x - e_q is an obstacle or, where
// x - e_q lies in a wall plane, the specular source (x - e_q with the wall-axis
// coordinates of x) is an obstacle. (A solid node's loads then never include the reloads
// of bounced links: the step kernels let solid lanes load and skip only their stores.)
// ---------------------------------------------------------------------------------
template <int LAT>
__global__ __launch_bounds__(kBlock) void k_links(Geometry g, typename LinkMask<LAT>::T *links)
{
    using L = Lat<LAT>;
    using LT = typename LinkMask<LAT>::T;
    const Tile t = tile_of(g, (int)blockIdx.x);
    if (!t.valid) return;
    const int xm = wrapm(t.x0, g.nx), xp = wrapp(t.x0, g.nx);
    const int ym = wrapm(t.y, g.ny), yp = wrapp(t.y, g.ny);
    const int zm = wrapm(t.z, g.nz), zp = wrapp(t.z, g.nz);
    auto obstacle = [&](int x, int y, int z) { return g.mask && g.mask[x + g.nx * (y + g.ny * z)]; };
    auto wall_y = [&](int y) { return (g.slip & LBM_SLIP_Y) && (y == 0 || y == g.ny - 1); };
    auto wall_z = [&](int z) { return (g.slip & LBM_SLIP_Z) && (z == 0 || z == g.nz - 1); };
    const bool own_solid = obstacle(t.x0, t.y, t.z) || wall_y(t.y) || wall_z(t.z);
    if (own_solid) {
        links[t.own] = LinkMask<LAT>::solid;
        return;
    }
    LT bits = 0;
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
        const int sx = L::ex[q] > 0 ? xm : (L::ex[q] < 0 ? xp : t.x0);
        int sy = L::ey[q] > 0 ? ym : (L::ey[q] < 0 ? yp : t.y);
        int sz = L::ez[q] > 0 ? zm : (L::ez[q] < 0 ? zp : t.z);
        if (L::ey[q] != 0 && wall_y(sy)) sy = t.y;
        if (L::ez[q] != 0 && wall_z(sz)) sz = t.z;
        if (obstacle(sx, sy, sz)) bits |= (LT)(1u << q);
    }
    links[t.own] = bits;
}

// ---------------------------------------------------------------------------------
// K2: initial state, written from the reader's side: every fluid node x stores its
// equilibrium deviations f^eq_q(rho(x), u(x)) at the addresses its first pull reads
// them from (the same pull_row as the step: slot q of x - e_q, or the specular source
// beside a free-slip wall; for a bounce-back link slot qbar of x itself (own slot) or
// slot q of the solid source (solid slot)). Every such address has exactly one reader,
// so the writes do not overlap. Slots that no pull reads are left as they were.
// ---------------------------------------------------------------------------------
template <int LAT, int q>
__device__ __forceinline__ float deq_moving(const Physics &p, float drho, float rho, const float *j,
                                            const float *U, float U2)
{
    constexpr int k = shell<LAT, q>();
    const float eu = edot<LAT, q>(U);
    const float ej = edot<LAT, q>(j);
    return p.what[k] * drho + p.lam[k] * ej + p.what[k] * rho * (p.Bc * eu * eu + p.Cp[k] * U2);
}

template <int LAT, int ST>
__global__ __launch_bounds__(kBlock) void k_init(InitArgs a)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    const Geometry &g = a.g;
    const Physics &p = a.ph;
    const Tile t = tile_of(g, (int)blockIdx.x);
    if (!t.valid) return;
    const LT lk = a.links ? static_cast<const LT *>(a.links)[t.own] : (LT)0;
    if (lk & LinkMask<LAT>::solid) return;
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const int N = g.nx * g.ny * g.nz;
    const float inv_cs = p.cs * p.inv_cs2;
    // rho, j, U of the node from the caller's FP64 fields (u in xi-units, j = rho c_s u)
    const double r = a.rho[t.own];
    const float drho = (float)(r - (double)p.rho0), rho = (float)r;
    float j[3], U[3];
    for (int i = 0; i < 3; ++i) {
        const double ui = (a.u && i < L::D) ? a.u[(size_t)i * N + t.own] : 0.0;
        U[i] = (float)ui * inv_cs;
        j[i] = (float)(r * ui * (double)p.cs);
    }
    const float U2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    // rest population by closure, so that the deviations of the node sum to drho
    float sum_eq = 0.f;
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (q != 0) sum_eq += deq_moving<LAT, q>(p, drho, rho, j, U, U2);
    });
    dst[t.own] = Codec<ST>::enc(drho - sum_eq, p.scale);
    const PullRows rows = pull_rows<1>(g, t);
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (q != 0) {
            const T v = Codec<ST>::enc(deq_moving<LAT, q>(p, drho, rho, j, U, U2), p.scale);
            if (!kSolidSlotBB<ST> && ((lk >> q) & 1u))
                dst[(size_t)L::opp[q] * g.stride + t.own] = v;  // bounced, own slot
            else
                *at32(dst + pull_row<LAT, q>(g, t, rows), pull_x<LAT, q, 1>(rows, 0)) = v;
        }
    });
}

// ---------------------------------------------------------------------------------
// Block reductions.
// ---------------------------------------------------------------------------------
// Sum of v over the 64 lanes of a wave, complete in lane 63, with DPP lane moves of the
// CDNA ISA (no LDS): quad permutes xor 1 and xor 2, half-row and row mirrors (every lane
// then holds its 16-lane row sum), then row broadcasts of lanes 15 and 31 into the rows
// above. Lanes of rows a move leaves out add 0. Needs all 64 lanes active.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_add(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xF, false);
    return v + __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double wave_sum_last_lane(double v)
{
    v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xF>(v);  // row_mirror
    v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// out[c] = sum over the block of v[c].
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
    if ((int)threadIdx.x < NC) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// The convergence measure of the Ohm's-law runs (Sec. 9.4): over the nodes whose new
// speed |u| is non-zero, the sum of | |u_new| - |u_old| | / |u_new| and their count, as
// FP64 per-block partials [block][2] (grid-stride, wave64 shuffles, LDS across waves);
// speed[n] <- |u_new| at every node. u is the (D, N) field of lbm_moments (zero at solids).
__global__ __launch_bounds__(kBlock) void k_speed_change(const float *__restrict__ u, int D, int N,
                                                         float *__restrict__ speed, int have_prev,
                                                         double *__restrict__ partials)
{
    double acc[2] = {0.0, 0.0};
    for (int n = (int)(blockIdx.x * kBlock + threadIdx.x); n < N; n += (int)(gridDim.x * kBlock)) {
        float s2 = 0.f;
        for (int d = 0; d < D; ++d) {
            const float v = u[(size_t)d * N + n];
            s2 = __builtin_fmaf(v, v, s2);
        }
        const float s = sqrtf(s2);
        if (have_prev && s > 0.f) {
            acc[0] += fabs((double)s - (double)speed[n]) / (double)s;
            acc[1] += 1.0;
        }
        speed[n] = s;
    }
    __shared__ double sh[kBlock / 64][2];
    for (int c = 0; c < 2; ++c)
        for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 64);
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < 2; ++c) sh[threadIdx.x >> 6][c] = acc[c];
    __syncthreads();
    if (threadIdx.x < 2) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w][threadIdx.x];
        partials[(size_t)blockIdx.x * 2 + threadIdx.x] = t;
    }
}

// First stage of a two-stage reduction of per-block partials laid out [part][ncomp]:
// block b sums a contiguous chunk of parts into out[b*ncomp + c] (coalesced reads).
__global__ __launch_bounds__(kBlock) void k_reduce_stage1(const double *__restrict__ partials, int nparts,
                                                          int ncomp, double *__restrict__ out)
{
    const int per = (nparts + gridDim.x - 1) / gridDim.x;
    const int p0 = blockIdx.x * per;
    const int p1 = min(nparts, p0 + per);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = p0 * ncomp + (int)threadIdx.x; i < p1 * ncomp; i += kBlock) acc[i % ncomp] += partials[i];
    __shared__ double sh[kBlock / 64][8];
    for (int c = 0; c < ncomp; ++c)
        for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 64);
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < ncomp; ++c) sh[threadIdx.x >> 6][c] = acc[c];
    __syncthreads();
    if ((int)threadIdx.x < ncomp) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w][threadIdx.x];
        out[(size_t)blockIdx.x * ncomp + threadIdx.x] = t;
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
// K3/K4: gather kernels over the current state. MODE 0: rho and u fields; 1: FP64
// export of the populations; 2: per-block FP64 partial sums
// (sum drho, sum d e_x, sum d e_y, sum d e_z, fluid nodes). ODD: the state is in the odd
// layout of the in-place step (populations already streamed).
// ---------------------------------------------------------------------------------
template <int LAT, int ST, bool MASK, int MODE, bool ODD>
__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs a)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    const T *src = static_cast<const T *>(a.src);
    const LT *links = static_cast<const LT *>(a.links);
    auto pull = [&](const Tile &t, const LT *lk, float (&d)[1][L::Q]) {
        if constexpr (ODD)
            gather_odd<LAT, ST, MASK, 1>(a.g, src, a.ph.inv_scale, t, lk, d);
        else
            gather_tile<LAT, ST, MASK, 1>(a.g, src, a.ph.inv_scale, t, lk, d);
    };
    if constexpr (MODE == 2) {
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int b = blockIdx.x; b < a.g.nblocks; b += gridDim.x) {
            const Tile t = tile_of(a.g, b);
            if (!t.valid) continue;
            LT lk[1] = {0};
            if (MASK) {
                lk[0] = links[t.own];
                if (lk[0] & LinkMask<LAT>::solid) continue;
            }
            float d[1][L::Q];
            pull(t, lk, d);
            const Macro<LAT> m = macro<LAT>(a.ph, d[0]);
            acc[0] += m.drho;
            acc[1] += m.j[0];
            acc[2] += m.j[1];
            if (L::D == 3) acc[3] += m.j[2];
            acc[4] += 1.0;
        }
        block_sum_store<5>(acc, a.partials + (size_t)blockIdx.x * 5);
    } else {
        const Tile t = tile_of(a.g, (int)blockIdx.x);
        if (!t.valid) return;
        LT lk[1] = {0};
        bool solid = false;
        if (MASK) {
            lk[0] = links[t.own];
            solid = (lk[0] & LinkMask<LAT>::solid) != 0;
        }
        float d[1][L::Q];
        if (!solid) pull(t, lk, d);
        if constexpr (MODE == 0) {
            if (solid) {
                if (a.rho) a.rho[t.own] = 0.f;
                if (a.u)
                    for (int i = 0; i < L::D; ++i) a.u[(size_t)i * a.N + t.own] = 0.f;
                return;
            }
            const Macro<LAT> m = macro<LAT>(a.ph, d[0]);
            if (a.rho) a.rho[t.own] = m.rho;
            if (a.u)
                for (int i = 0; i < L::D; ++i) a.u[(size_t)i * a.N + t.own] = m.U[i] * a.ph.cs;
        } else {
            for_q<L::Q>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int k = shell<LAT, q>();
                a.f64[(size_t)q * a.N + t.own] = solid ? 0.0 : a.what_rho0[k] + (double)d[0][q];
            });
        }
    }
}

// dJ/dg_q(x) for every q of the fluid node of tile t: lam_in at the node and slot that
// pull g_q(x) in the forward step (the transpose of pull_row): slot q of x + e_q; where
// x + e_q lies in a free-slip wall plane, slot reflected(q) of x + e_q with the wall-axis
// coordinates of x; where that destination is an obstacle (link bit qbar of x: the pull
// of qbar into x bounces), slot qbar of x itself.
template <int LAT, bool MASK>
__device__ __forceinline__ void adjoint_pull(const Geometry &g, const Tile &t, const float *__restrict__ lam_in,
                                             typename LinkMask<LAT>::T lk, float (&gb)[Lat<LAT>::Q])
{
    using L = Lat<LAT>;
    const int xm = wrapm(t.x0, g.nx), xp = wrapp(t.x0, g.nx);
    const int ym = wrapm(t.y, g.ny), yp = wrapp(t.y, g.ny);
    const int zm = wrapm(t.z, g.nz), zp = wrapp(t.z, g.nz);
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const unsigned tx = (unsigned)(L::ex[q] > 0 ? xp : (L::ex[q] < 0 ? xm : t.x0));
        int ty = L::ey[q] > 0 ? yp : (L::ey[q] < 0 ? ym : t.y);
        int tz = L::ez[q] > 0 ? zp : (L::ez[q] < 0 ? zm : t.z);
        int p = q;
        if (g.slip) {
            const bool fy = L::ey[q] != 0 && (g.slip & LBM_SLIP_Y) && (ty == 0 || ty == g.ny - 1);
            const bool fz = L::ez[q] != 0 && (g.slip & LBM_SLIP_Z) && (tz == 0 || tz == g.nz - 1);
            if (fy) ty = t.y;
            if (fz) tz = t.z;
            constexpr int py = reflected<LAT>(q, true, false), pz = reflected<LAT>(q, false, true);
            constexpr int pyz = reflected<LAT>(q, true, true);
            p = fy ? (fz ? pyz : py) : (fz ? pz : q);
        }
        const float *src = at32(lam_in + (size_t)((unsigned)p * (unsigned)g.stride +
                                                  (unsigned)g.nx * (unsigned)(ty + g.ny * tz)), tx);
        // as in the forward pull: unshifted in x, a wave's loads cover whole cache lines that
        // no other wave reads (streamed loads); x-shifted loads reach one element into the
        // neighbouring wave's lines, which the cache then serves
        float v = L::ex[q] == 0 ? __builtin_nontemporal_load(src) : *src;
        if constexpr (MASK && q != 0)
            if ((lk >> L::opp[q]) & 1u) v = *at32(lam_in + slot_off(L::opp[q], g.stride), (unsigned)t.own);
        gb[q] = v;
    });
}

// ---------------------------------------------------------------------------------
// K5: one reverse step of the discrete adjoint. lam_out = dJ/df(t) from
// lam_in = dJ/df(t+1); f(t) is pulled from the stored state as in K1.
//   gbar_a = lam_in(x + e_a, a), or lam_in(x, abar) if x + e_a is solid (beside a free-slip
//   wall plane: the specular destination, adjoint_pull);
//   hbar_a = (1 - s) gbar_a;
//   dJ/ds  += sum_a gbar_a (d_abar - d*_a);
//   dJ/dtau += omega^2 sum_a hbar_a (d_a - deq_a);
//   dJ/dE_i += sum_a hbar_a rho what_a [(A + 2 Bc e.U) e_i / c_s + 2 C_k c_s U_i];
//   rhobar = sum_a hbar_a [omega f^eq_a / rho + what_a sigma_a];
//   V_i = sum_a hbar_a what_a [omega (A e_i + 2 Bc (e.U) e_i + 2 C_k c_s^2 U_i)
//                              + 2 Bc e_i (e.E)/c_s + 2 C_k (c_s E_i + (e x B)_i)];
//   lam_out_b = (1 - omega) hbar_b + s gbar_bbar + rhobar + V . (e_b / c_s^2 - U).
// ---------------------------------------------------------------------------------
template <int LAT, int ST, bool MASK, bool SOFT, bool MAG>
__global__ __launch_bounds__(kBlock) void k_adjoint(AdjointArgs a)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    const Geometry &g = a.g;
    const Physics &p = a.ph;
    const int bid = block_order((int)blockIdx.x, g.nblocks, a.remap);
    const Tile t = tile_of(g, bid);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // One partial per wave, written by its last lane. The accumulated value is read first
    // (a wave-uniform address: scalar registers), so its latency overlaps the pulls below.
    const bool last_lane = (threadIdx.x & 63) == 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    double *part = a.partials + ((size_t)blockIdx.x * (blockDim.x >> 6) + wave) * 4;
    // whole waves beyond the row (rows shorter than a block) have no work beyond a zero
    // partial; partial waves go on with their extra lanes idle (the sums need 64 lanes)
    if ((bid - fast_div(bid, g.div_ntx) * g.ntx) * kBlock + wave * 64 >= g.nx) {
        if (!a.accumulate && last_lane)
            for (int c = 0; c < 4; ++c) part[c] = 0.0;
        return;
    }
    double prev[4] = {0.0, 0.0, 0.0, 0.0};
    if (a.accumulate)
        for (int c = 0; c < 4; ++c) prev[c] = part[c];
    const float gs_prev = (SOFT && a.grad_s && t.valid) ? *at32(a.grad_s, (unsigned)t.own) : 0.f;
    LT lk[1] = {0};
    bool solid = false;
    if (MASK && t.valid) {
        lk[0] = *at32(static_cast<const LT *>(a.links), (unsigned)t.own);
        solid = (lk[0] & LinkMask<LAT>::solid) != 0;
    }
    // Solid nodes compute like fluid ones (their reads stay in bounds, and a solid node's
    // link mask has no link bits) and then store zeros and contribute nothing: no lane waits
    // for its link mask before its state and lambda loads issue.
    if (t.valid) {
        float d[1][L::Q], gb[L::Q];
        gather_tile<LAT, ST, MASK, 1>(g, static_cast<const T *>(a.state), p.inv_scale, t, lk, d);
        adjoint_pull<LAT, MASK>(g, t, a.lam_in, lk[0], gb);
        const float s = SOFT ? *at32(g.s, (unsigned)t.own) : 0.f;
        const Macro<LAT> m = macro<LAT>(p, d[0]);
        const float inv_cs = p.cs * p.inv_cs2;
        const float om = p.omega;
        const float inv_rho = __builtin_amdgcn_rcpf(m.rho);
        const float one_s = 1.f - s;
        // Forward quantities of the node, per shell k: what_k drho, what_k rho, Cp_k U^2 and
        // the source's 2 C_k c_s (U.E); W = U x B.
        float wd[3], wr[3], cu[3], sk[3] = {0.f, 0.f, 0.f}, W[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            wd[k] = p.what[k] * m.drho;
            wr[k] = p.what[k] * m.rho;
            cu[k] = p.Cp[k] * m.U2;
        }
        {
            float UE = m.U[0] * p.E[0] + m.U[1] * p.E[1];
            if constexpr (L::D == 3) UE += m.U[2] * p.E[2];
            UE *= p.cs;
#pragma unroll
            for (int k = 0; k < 3; ++k) sk[k] = p.C2[k] * UE;
        }
        if (MAG) {
            W[0] = p.B[1] * m.U[2] - p.B[2] * m.U[1];
            W[1] = p.B[2] * m.U[0] - p.B[0] * m.U[2];
            W[2] = p.B[0] * m.U[1] - p.B[1] * m.U[0];
        }
        // Sums over q, with the q-independent factors applied once at the end:
        //   Ee = sum hw (A + 2 Bc e.U) e,  Ve = sum hw a1 e,  Wc = sum hw 2 C_k e,
        //   S1 = sum hw 2 C_k,  S2 = sum hw C_k c_s^2,  R1 = sum h (what rho0 + deq),
        //   R2 = sum hw sigma, with hw = h what_k, a1 = omega (A + 2 Bc e.U) + 2 Bc (e.E)/c_s.
        // deq, sigma and the post-collision d* of each q are formed inside the loop (as in
        // the forward step, rest population last by closure), so no per-q arrays stay live.
        float Ee[3] = {0.f, 0.f, 0.f}, Ve[3] = {0.f, 0.f, 0.f}, Wc[3] = {0.f, 0.f, 0.f};
        float S1 = 0.f, S2 = 0.f, R1 = 0.f, R2 = 0.f, ds = 0.f, dtau = 0.f, sum_eq = 0.f;
        auto acc_e = [](float *acc, float v, int ex, int ey, int ez) {
            if (ex) acc[0] += ex > 0 ? v : -v;
            if (ey) acc[1] += ey > 0 ? v : -v;
            if (ez) acc[2] += ez > 0 ? v : -v;
        };
        auto terms = [&](auto qc, float deq, float sig) {
            constexpr int q = decltype(qc)::value;
            constexpr int k = shell<LAT, q>();
            constexpr int ex = L::ex[q], ey = L::ey[q], ez = L::ez[q];
            const float h = one_s * gb[q];
            const float hw = h * p.what[k];
            if (SOFT) {
                const float dstq = __builtin_fmaf(wr[k], sig, __builtin_fmaf(om, deq - d[0][q], d[0][q]));
                ds = __builtin_fmaf(gb[q], d[0][L::opp[q]] - dstq, ds);
            }
            dtau = __builtin_fmaf(h, d[0][q] - deq, dtau);
            R1 = __builtin_fmaf(h, p.what[k] * p.rho0 + deq, R1);
            R2 = __builtin_fmaf(hw, sig, R2);
            S1 = __builtin_fmaf(hw, p.C2[k], S1);
            S2 = __builtin_fmaf(hw, p.Cp[k], S2);
            if constexpr (q != 0) {
                const float eu = edot<LAT, q>(m.U);
                const float t1 = __builtin_fmaf(2.f * p.Bc, eu, p.A);
                const float a1 = __builtin_fmaf(om, t1, p.c2q[q]);
                acc_e(Ee, hw * t1, ex, ey, ez);
                acc_e(Ve, hw * a1, ex, ey, ez);
                if (MAG) acc_e(Wc, hw * p.C2[k], ex, ey, ez);
            }
        };
        for_q<L::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (q != 0) {
                constexpr int k = shell<LAT, q>();
                const float eu = edot<LAT, q>(m.U);
                const float ej = edot<LAT, q>(m.j);
                const float quad = __builtin_fmaf(p.Bc * eu, eu, cu[k]);
                const float deq = __builtin_fmaf(wr[k], quad, __builtin_fmaf(p.lam[k], ej, wd[k]));
                sum_eq = (q == 1) ? deq : sum_eq + deq;
                float sig = __builtin_fmaf(p.c2q[q], eu, p.c1q[q] + sk[k]);
                if (MAG) sig = __builtin_fmaf(p.C2[k], edot<LAT, q>(W), sig);
                terms(qc, deq, sig);
            }
        });
        terms(std::integral_constant<int, 0>{}, m.drho - sum_eq, sk[0]);
        // dJ/dE_i = sum hw [(A + 2 Bc e.U) e_i / c_s + 2 C_k c_s U_i]  (times rho below)
        float dE[3], V[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            dE[i] = __builtin_fmaf(inv_cs, Ee[i], p.cs * m.U[i] * S1);
            V[i] = Ve[i] + 2.f * om * S2 * m.U[i] + p.cs * p.E[i] * S1;
        }
        if (MAG) {  // sum hw 2 C_k (e x B) = (sum hw 2 C_k e) x B
            V[0] += Wc[1] * p.B[2] - Wc[2] * p.B[1];
            V[1] += Wc[2] * p.B[0] - Wc[0] * p.B[2];
            V[2] += Wc[0] * p.B[1] - Wc[1] * p.B[0];
        }
        const float rbar = om * inv_rho * R1 + R2;
        const float VU = V[0] * m.U[0] + V[1] * m.U[1] + V[2] * m.U[2];
        const float base = rbar - VU;
        float Vs[3] = {V[0] * p.inv_cs2, V[1] * p.inv_cs2, V[2] * p.inv_cs2};
        const float one_om = 1.f - om;
        for_q<L::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            float out = __builtin_fmaf(one_om, one_s * gb[q], base + edot<LAT, q>(Vs));
            if (SOFT) out = __builtin_fmaf(s, gb[L::opp[q]], out);
            __builtin_nontemporal_store(solid ? 0.f : out, at32(a.lam_out + slot_off(q, g.stride), (unsigned)t.own));
        });
        if (SOFT && a.grad_s && !solid) *at32(a.grad_s, (unsigned)t.own) = gs_prev + ds;
        acc[0] = (double)m.rho * (double)dE[0];
        acc[1] = (double)m.rho * (double)dE[1];
        acc[2] = (double)m.rho * (double)dE[2];
        acc[3] = (double)(om * om) * (double)dtau;
        if (solid)
            for (int c = 0; c < 4; ++c) acc[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = wave_sum_last_lane(acc[c]);
    if (last_lane)
        for (int c = 0; c < 4; ++c) part[c] = prev[c] + acc[c];
}

// ---------------------------------------------------------------------------------
// K5 for the velocity shift (eq. u-update-force-term-eq: f^eq at u + tau (E + u x B), no
// source term). In lattice units with j = sum d e, the shifted momentum is
//   j' = j + rho tau c_s E + tau (j x B),   U' = j' / (c_s^2 rho),
// and f*_q = d_q + omega (deq_q(drho, j') - d_q) with deq_q = what_k drho + lam_k e.j'
// + what_k rho (Bc (e.U')^2 + Cp_k U'^2), the rest population by mass closure. With
// hbar = (1 - s) gbar and eta_q = hbar_q - hbar_0 (q != 0):
//   G = omega sum eta_q [lam_k e_q + 2 what_k (Bc (e.U') e_q + Cp_k U') / c_s^2]  (d/dj')
//   C = omega sum eta_q (what_k - Q_q / rho) + tau c_s G.E,  Q_q = what_k rho (Bc (e.U')^2
//       + Cp_k U'^2)
//   lam_out_b = (1 - omega) hbar_b + omega hbar_0 + C + e_b . (G + tau B x G) + s gbar_bbar
//   dJ/dE += rho tau c_s G;  dJ/dtau += omega^2 sum eta_q (d_q - deq_q) + G.(rho c_s E + j x B);
//   dJ/ds += sum_q gbar_q (d_qbar - f*_q).
// ---------------------------------------------------------------------------------
template <int LAT, int ST, bool MASK, bool SOFT, bool MAG>
__global__ __launch_bounds__(kBlock) void k_adjoint_shift(AdjointArgs a)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    const Geometry &g = a.g;
    const Physics &p = a.ph;
    const int bid = block_order((int)blockIdx.x, g.nblocks, a.remap);
    const Tile t = tile_of(g, bid);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const bool last_lane = (threadIdx.x & 63) == 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    double *part = a.partials + ((size_t)blockIdx.x * (blockDim.x >> 6) + wave) * 4;
    if ((bid - fast_div(bid, g.div_ntx) * g.ntx) * kBlock + wave * 64 >= g.nx) {
        if (!a.accumulate && last_lane)
            for (int c = 0; c < 4; ++c) part[c] = 0.0;
        return;
    }
    double prev[4] = {0.0, 0.0, 0.0, 0.0};
    if (a.accumulate)
        for (int c = 0; c < 4; ++c) prev[c] = part[c];
    const float gs_prev = (SOFT && a.grad_s && t.valid) ? *at32(a.grad_s, (unsigned)t.own) : 0.f;
    LT lk[1] = {0};
    bool solid = false;
    if (MASK && t.valid) {
        lk[0] = *at32(static_cast<const LT *>(a.links), (unsigned)t.own);
        solid = (lk[0] & LinkMask<LAT>::solid) != 0;
    }
    // Solid nodes compute like fluid ones (their reads stay in bounds, and a solid node's
    // link mask has no link bits) and then store zeros and contribute nothing: no lane waits
    // for its link mask before its state and lambda loads issue.
    if (t.valid) {
        float d[1][L::Q], gb[L::Q];
        gather_tile<LAT, ST, MASK, 1>(g, static_cast<const T *>(a.state), p.inv_scale, t, lk, d);
        adjoint_pull<LAT, MASK>(g, t, a.lam_in, lk[0], gb);
        const float s = SOFT ? *at32(g.s, (unsigned)t.own) : 0.f;
        const Macro<LAT> m = macro<LAT>(p, d[0]);
        const float om = p.omega;
        const float tau = 1.f / om;
        const float inv_rho = __builtin_amdgcn_rcpf(m.rho);
        const float one_s = 1.f - s;
        // shifted momentum j' and velocity U'
        float jxB[3] = {0.f, 0.f, 0.f}, jp[3], Up[3];
        if (MAG) {
            jxB[0] = m.j[1] * p.B[2] - m.j[2] * p.B[1];
            jxB[1] = m.j[2] * p.B[0] - m.j[0] * p.B[2];
            jxB[2] = m.j[0] * p.B[1] - m.j[1] * p.B[0];
        }
        const float kk = p.inv_cs2 * inv_rho;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            jp[i] = m.j[i] + tau * (m.rho * p.cs * p.E[i] + jxB[i]);
            Up[i] = jp[i] * kk;
        }
        if (L::D == 2) {
            jp[2] = 0.f;
            Up[2] = 0.f;
        }
        const float U2 = Up[0] * Up[0] + Up[1] * Up[1] + Up[2] * Up[2];
        const float h0 = one_s * gb[0];
        float Ge[3] = {0.f, 0.f, 0.f};
        float Sc = 0.f, Cs = 0.f, dtau = 0.f, ds = 0.f, sum_eq = 0.f;
        auto acc_e = [](float *acc3, float v, int ex, int ey, int ez) {
            if (ex) acc3[0] += ex > 0 ? v : -v;
            if (ey) acc3[1] += ey > 0 ? v : -v;
            if (ez) acc3[2] += ez > 0 ? v : -v;
        };
        for_q<L::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (q != 0) {
                constexpr int k = shell<LAT, q>();
                constexpr int ex = L::ex[q], ey = L::ey[q], ez = L::ez[q];
                const float eu = edot<LAT, q>(Up);
                const float ej = edot<LAT, q>(jp);
                const float quad = __builtin_fmaf(p.Bc * eu, eu, p.Cp[k] * U2);
                const float Qq = p.what[k] * m.rho * quad;
                const float deq = __builtin_fmaf(p.lam[k], ej, p.what[k] * m.drho) + Qq;
                sum_eq += deq;
                const float eta = one_s * gb[q] - h0;
                acc_e(Ge, eta * (p.lam[k] + 2.f * p.what[k] * p.inv_cs2 * p.Bc * eu), ex, ey, ez);
                Sc = __builtin_fmaf(eta, 2.f * p.what[k] * p.inv_cs2 * p.Cp[k], Sc);
                Cs = __builtin_fmaf(eta, p.what[k] - Qq * inv_rho, Cs);
                dtau = __builtin_fmaf(eta, d[0][q] - deq, dtau);
                if (SOFT) {
                    const float fst = __builtin_fmaf(om, deq - d[0][q], d[0][q]);
                    ds = __builtin_fmaf(gb[q], d[0][L::opp[q]] - fst, ds);
                }
            }
        });
        if (SOFT) {
            const float deq0 = m.drho - sum_eq;
            const float fst0 = __builtin_fmaf(om, deq0 - d[0][0], d[0][0]);
            ds = __builtin_fmaf(gb[0], d[0][0] - fst0, ds);
        }
        float G[3], H[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) G[i] = om * __builtin_fmaf(Sc, Up[i], Ge[i]);
        if (L::D == 2) G[2] = 0.f;
        const float GE = G[0] * p.E[0] + G[1] * p.E[1] + G[2] * p.E[2];
        const float C = __builtin_fmaf(om, Cs, tau * p.cs * GE);
        H[0] = G[0];
        H[1] = G[1];
        H[2] = G[2];
        if (MAG) {  // + tau B x G
            H[0] += tau * (p.B[1] * G[2] - p.B[2] * G[1]);
            H[1] += tau * (p.B[2] * G[0] - p.B[0] * G[2]);
            H[2] += tau * (p.B[0] * G[1] - p.B[1] * G[0]);
        }
        const float base = __builtin_fmaf(om, h0, C);
        const float one_om = 1.f - om;
        for_q<L::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            float out = __builtin_fmaf(one_om, one_s * gb[q], base + edot<LAT, q>(H));
            if (SOFT) out = __builtin_fmaf(s, gb[L::opp[q]], out);
            __builtin_nontemporal_store(solid ? 0.f : out, at32(a.lam_out + slot_off(q, g.stride), (unsigned)t.own));
        });
        if (SOFT && a.grad_s && !solid) *at32(a.grad_s, (unsigned)t.own) = gs_prev + ds;
        const float rtc = m.rho * tau * p.cs;
        acc[0] = (double)(rtc * G[0]);
        acc[1] = (double)(rtc * G[1]);
        acc[2] = (double)(rtc * G[2]);
        float Gt = 0.f;
#pragma unroll
        for (int i = 0; i < 3; ++i) Gt = __builtin_fmaf(G[i], m.rho * p.cs * p.E[i] + jxB[i], Gt);
        acc[3] = (double)(om * om) * (double)dtau + (double)Gt;
        if (solid)
            for (int c = 0; c < 4; ++c) acc[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = wave_sum_last_lane(acc[c]);
    if (last_lane)
        for (int c = 0; c < 4; ++c) part[c] = prev[c] + acc[c];
}

// Adjoint seed: lam(a, n) = e_a[axis] * value at fluid nodes (value = 1/(c_s norm)), 0 at
// obstacles and in free-slip wall planes.
template <int LAT>
__global__ __launch_bounds__(kBlock) void k_seed(Geometry g, float value, int axis, float *lam)
{
    using L = Lat<LAT>;
    const Tile t = tile_of(g, (int)blockIdx.x);
    if (!t.valid) return;
    const bool solid = (g.mask && g.mask[t.own]) || ((g.slip & LBM_SLIP_Y) && (t.y == 0 || t.y == g.ny - 1)) ||
                       ((g.slip & LBM_SLIP_Z) && (t.z == 0 || t.z == g.nz - 1));
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const int e = axis == 0 ? L::ex[q] : (axis == 1 ? L::ey[q] : L::ez[q]);
        lam[q * g.stride + t.own] = solid ? 0.f : (float)e * value;
    }
}

// ---------------------------------------------------------------------------------
// Launchers: runtime flags -> template instances.
// ---------------------------------------------------------------------------------
template <int LAT, int ST>
hipError_t step_nearest(int force, const StepArgs &a, hipStream_t st)
{
    return step_lat_st<LAT, ST, false>(force, a, st);
}

template <int LAT, int ST>
hipError_t adjoint_lat_st(bool mag, bool shift, const AdjointArgs &a, hipStream_t st)
{
    const bool mask = a.links != nullptr, soft = a.g.s != nullptr;
    const dim3 grid(a.g.nblocks), block(row_block_threads(a.g.nx, 1));
    AdjointArgs b = a;
    b.remap = remap_code(a.remap, a.g.ntx);
#define LBM_ADJ(M, S, B)                                                                  \
    do {                                                                                  \
        if (shift)                                                                        \
            hipLaunchKernelGGL((k_adjoint_shift<LAT, ST, M, S, B>), grid, block, 0, st, b); \
        else                                                                              \
            hipLaunchKernelGGL((k_adjoint<LAT, ST, M, S, B>), grid, block, 0, st, b);       \
    } while (0)
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
    const bool mask = a.links != nullptr;
    const dim3 block(kBlock);
    const int mode = a.partials ? 2 : (a.f64 ? 1 : 0);
    const dim3 grid(mode == 2 ? nred : a.g.nblocks);
#define LBM_G(M, MODE, O) hipLaunchKernelGGL((k_gather<LAT, ST, M, MODE, O>), grid, block, 0, st, a)
#define LBM_G_MODE(M, O) \
    if (mode == 0) LBM_G(M, 0, O); else if (mode == 1) LBM_G(M, 1, O); else LBM_G(M, 2, O)
    if (a.odd) {
        if (mask) LBM_G_MODE(true, true); else LBM_G_MODE(false, true);
    } else {
        if (mask) LBM_G_MODE(true, false); else LBM_G_MODE(false, false);
    }
#undef LBM_G_MODE
#undef LBM_G
    return hipGetLastError();
}

template <int LAT, int ST>
hipError_t init_lat_st(const InitArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_init<LAT, ST>), dim3(a.g.nblocks), dim3(kBlock), 0, st, a);
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

hipError_t launch_step(int lattice, int storage, int force, const StepArgs &a, hipStream_t st)
{
    if (a.sr) return launch_step_sr(lattice, storage, force, a, st);
    LBM_DISPATCH(step_nearest, force, a, st);
}

hipError_t launch_adjoint(int lattice, int storage, bool mag, bool shift, const AdjointArgs &a, hipStream_t st)
{
    LBM_DISPATCH(adjoint_lat_st, mag, shift, a, st);
}

hipError_t launch_gather(int lattice, int storage, const GatherArgs &a, int nblocks_reduce, hipStream_t st)
{
    LBM_DISPATCH(gather_lat_st, a, nblocks_reduce, st);
}

hipError_t launch_init(int lattice, int storage, const InitArgs &a, hipStream_t st)
{
    LBM_DISPATCH(init_lat_st, a, st);
}

hipError_t launch_links(int lattice, const Geometry &g, void *links, hipStream_t st)
{
    if (lattice == LBM_D2V9)
        hipLaunchKernelGGL(k_links<LBM_D2V9>, dim3(g.nblocks), dim3(kBlock), 0, st, g,
                           static_cast<LinkMask<LBM_D2V9>::T *>(links));
    else if (lattice == LBM_D3V19)
        hipLaunchKernelGGL(k_links<LBM_D3V19>, dim3(g.nblocks), dim3(kBlock), 0, st, g,
                           static_cast<LinkMask<LBM_D3V19>::T *>(links));
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

size_t link_mask_bytes(int lattice) { return lattice == LBM_D2V9 ? 2 : 4; }

hipError_t launch_reduce_final(const double *partials, int nparts, int ncomp, double *out, int accumulate,
                               hipStream_t st, double *stage)
{
    if (ncomp > 8) return hipErrorInvalidValue;
    if (stage && nparts > 2 * kReduceStage) {
        hipLaunchKernelGGL(k_reduce_stage1, dim3(kReduceStage), dim3(kBlock), 0, st, partials, nparts, ncomp, stage);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        partials = stage;
        nparts = kReduceStage;
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, partials, nparts, ncomp, out, accumulate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Totals without a workspace: the reduction partials of lbm_current_noalloc live in a
// fixed device-resident array of this file instead of the caller's workspace. Its host
// name is only a stand-in: host code uses the device address that hipGetSymbolAddress
// returns, looked up once per device with that device current.
// ---------------------------------------------------------------------------------
namespace {

// parts [kReduceBlocks][5] | stage [kReduceStage][8] | sums [8]
constexpr size_t kScratchParts = 0;
constexpr size_t kScratchStage = kScratchParts + (size_t)kReduceBlocks * 5;
constexpr size_t kScratchSums = kScratchStage + (size_t)kReduceStage * 8;
constexpr size_t kScratchUsed = kScratchSums + 8;
constexpr size_t kScratchDoubles = 8192;  // 64 KiB per device
static_assert(kScratchUsed <= kScratchDoubles, "static scratch too small for the totals reduction");

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

// out = (nfluid rho0 + sum drho, sum j / c_s) from the sums (sum drho, sum j_x, sum j_y,
// sum j_z, nfluid), the same FP64 operations as lbm_current performs on the host.
__global__ void k_totals_finish(const double *__restrict__ sums, double rho0, double cs, double *__restrict__ out)
{
#pragma clang fp contract(off)
    const int i = (int)threadIdx.x;
    if (i == 0) out[0] = sums[4] * rho0 + sums[0];
    if (i >= 1 && i < 4) out[i] = sums[i] / cs;
}

}  // namespace

hipError_t static_scratch(int device, double **ptr, size_t *bytes)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != device) {
            const hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    *ptr = g_scratch_ptr[device];
    *bytes = kScratchDoubles * sizeof(double);
    return hipSuccess;
}

size_t totals_scratch_bytes() { return kScratchUsed * sizeof(double); }

hipError_t launch_totals_noalloc(int lattice, int storage, const GatherArgs &a, double rho0, double cs, double *out,
                                 hipStream_t st, double *scratch_dev)
{
    if (!out || !scratch_dev) return hipErrorInvalidValue;
    GatherArgs b = a;
    b.rho = b.u = nullptr;
    b.f64 = nullptr;
    b.partials = scratch_dev + kScratchParts;
    hipError_t e = launch_gather(lattice, storage, b, kReduceBlocks, st);
    if (e != hipSuccess) return e;
    e = launch_reduce_final(scratch_dev + kScratchParts, kReduceBlocks, 5, scratch_dev + kScratchSums, 0, st,
                            scratch_dev + kScratchStage);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_totals_finish, dim3(1), dim3(64), 0, st, scratch_dev + kScratchSums, rho0, cs, out);
    return hipGetLastError();
}

hipError_t launch_speed_change(const float *u, int D, int N, float *speed, int have_prev, double *partials,
                               int nblocks, hipStream_t st)
{
    if (!u || !speed || !partials || D < 1 || D > 3 || N < 1 || nblocks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_speed_change, dim3(nblocks), dim3(kBlock), 0, st, u, D, N, speed, have_prev, partials);
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
