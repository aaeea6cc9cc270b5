// lbm_step_kernels.h -- the two-buffer step kernel and its launcher, as templates: the
// round-to-nearest instances are built in lbm_kernels.hip, the stochastic-rounding ones
// in lbm_step_sr.hip (two translation units, compiled in parallel).
#pragma once

#include "lbm_device.h"

namespace lbm {
namespace {

// ---------------------------------------------------------------------------------
// K1: fused pull-stream + collide + force + partial bounce-back. SR: stochastic
// rounding of the stored 16-bit values, with the random bits of (node, population,
// a.sr_key).
// ---------------------------------------------------------------------------------
template <int LAT, int ST, bool MASK, bool SOFT, int FORCE, int V, bool SLIP, bool SR>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs a, int ntx, FastDiv div_ntx, int nblocks)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    // without free-slip planes the reflection logic of every pull is compiled out where
    // there are solids (measured on MI355X: FP16 duct +10 %, FP16 disks +8 %, with the
    // loads issued before the link masks arrive); the kernels without solids keep the
    // runtime test, whose code measured 3 % faster on the 4096^2 FP32 grid
    if constexpr (MASK && !SLIP) a.g.slip = 0;
    const int bid = block_order((int)blockIdx.x, nblocks, a.remap);
    const Tile t = tile_of<V>(a.g, bid, ntx, div_ntx);
    if (!t.valid) return;  // beyond the row (rows shorter than a block): no work
    LT lk[V];
    // Solid nodes go through the loads and the collision like fluid ones; store_tile
    // decides which of their values are stored: leaving early would make every lane wait for
    // its link mask before the population loads could issue, one more memory round trip per
    // wave. Their pulls stay inside the state (the same row arithmetic as a fluid node's).
    if (MASK) load_links<LAT, V>(static_cast<const LT *>(a.links), t.own, lk);
    float d[V][L::Q];
    gather_tile<LAT, ST, MASK, V>(a.g, static_cast<const T *>(a.src), 1.f, t, lk, d);  // stored units throughout
    float sv[V];
    if (SOFT) vload<LBM_F32, V>(at32(a.g.s, (unsigned)t.own), 1.f, sv);
    float o[V][L::Q];
#pragma unroll
    for (int i = 0; i < V; ++i) collide<LAT, SOFT, FORCE>(a.ph, d[i], SOFT ? sv[i] : 0.f, o[i]);
    uint32_t h[V];
#pragma unroll
    for (int i = 0; i < V; ++i) h[i] = SR ? sr_node((uint32_t)t.own + (uint32_t)i, a.sr_key) : 0u;
    store_tile<LAT, ST, MASK, V, SR>(a.g, static_cast<typename Codec<ST>::T *>(a.dst), t, lk, o, h);
}

// Runtime flags -> template instances.
template <int LAT, int ST, int V, bool SR>
hipError_t step_v(int force, const StepArgs &a, hipStream_t st)
{
    const bool mask = a.links != nullptr, soft = a.g.s != nullptr;
    const int ntx = (a.g.nx + kBlock * V - 1) / (kBlock * V);
    const int nblocks = ntx * a.g.ny * a.g.nz;
    const FastDiv div_ntx = make_fastdiv(ntx);
    const dim3 grid(nblocks), block(row_block_threads(a.g.nx, V));
    StepArgs b = a;
    b.remap = remap_code(a.remap, ntx);
#define LBM_STEP_K(M, S, F, SL) \
    hipLaunchKernelGGL((k_step<LAT, ST, M, S, F, V, SL, SR>), grid, block, 0, st, b, ntx, div_ntx, nblocks)
#define LBM_STEP(M, S, F)               \
    do {                                \
        if (M && b.g.slip)              \
            LBM_STEP_K(M, S, F, M);     \
        else                            \
            LBM_STEP_K(M, S, F, false); \
    } while (0)
#define LBM_STEP_F(M, S)   \
    if (force == 0)        \
        LBM_STEP(M, S, 0); \
    else if (force == 1)   \
        LBM_STEP(M, S, 1); \
    else if (force == 2)   \
        LBM_STEP(M, S, 2); \
    else                   \
        LBM_STEP(M, S, 3)
    if (mask) {
        if (soft) LBM_STEP_F(true, true); else LBM_STEP_F(true, false);
    } else {
        if (soft) LBM_STEP_F(false, true); else LBM_STEP_F(false, false);
    }
#undef LBM_STEP_F
#undef LBM_STEP
#undef LBM_STEP_K
    return hipGetLastError();
}

template <int LAT, int ST, bool SR>
hipError_t step_lat_st(int force, const StepArgs &a, hipStream_t st)
{
    const int v = step_vector_width(LAT, ST, a.g.nx);
    if (v == 2) return step_v<LAT, ST, 2, SR>(force, a, st);
    return step_v<LAT, ST, 1, SR>(force, a, st);
}

}  // namespace
}  // namespace lbm
