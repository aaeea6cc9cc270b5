// lbm_aa_kernels.h -- the in-place time step on one state buffer: the AA access pattern
// (Bailey, Myre, Walsh, Lilja and Saar, ICPP 2009; not in the paper), built on the pull,
// collision, bounce-back and free-slip conventions of the two-buffer step.
//
// Let P(x, q) be the location (node, slot) from which the two-buffer step pulls f_q(x):
// slot q of x - e_q; beside a free-slip wall plane the specular source in the row of x;
// for a bounced link slot qbar of x (own-slot convention, FP32) or slot q of the solid
// node x - e_q (solid-slot convention, 16-bit). Over the fluid nodes P is one-to-one.
//
// Even layout (the two-buffer layout): the state holds the post-collision populations
// g of the previous step as the two-buffer step leaves them.
// Phase 0 (even -> odd): each fluid node x pulls f_q(x) from P(x, q) for every q,
//   collides and stores g_q(x) at P(x, qbar), where the pull of the opposite population
//   reads. Node x writes exactly the Q locations it read, and no other node touches
//   them, so the update is race-free in place. The populations are now streamed: f_q(x)
//   sits in slot qbar of x, or, for a bounced link under the solid-slot convention, at
//   P(x, q).
// Phase 1 (odd -> even): each fluid node reads those Q values of its own, collides and
//   stores g_q(x) in slot q of x (and bounced values in solid slots, as the two-buffer
//   step does), which is the even layout again.
// Each phase reads and writes every population once, as a two-buffer step does, with
// half the state memory. The arithmetic of a node is the same code as the two-buffer
// step, so both give the same bits.
//
// Templates: the round-to-nearest instances are built in lbm_aa.hip, the
// stochastic-rounding ones in lbm_aa_sr.hip (compiled in parallel).
#pragma once

#include "lbm_device.h"

namespace lbm {
namespace {

// Two values encoded in 16 bits each, a in the low half (16-bit storage only).
// Population q of two nodes with hashes ha, hb (stochastic rounding with SR).
template <int ST, bool SR>
__device__ __forceinline__ uint32_t pack_pair(float a, float b, uint32_t ha, uint32_t hb, int q)
{
    using T = typename Codec<ST>::T;
    if constexpr (sizeof(T) == 2 && SR)
        return __builtin_bit_cast(uint32_t, Codec<ST>::enc_sr2(a, sr_bits(ha, q), b, sr_bits(hb, q)));
    else if constexpr (sizeof(T) == 2)
        return (uint32_t)__builtin_bit_cast(uint16_t, enc_store<ST, SR>(a, ha, q)) |
               ((uint32_t)__builtin_bit_cast(uint16_t, enc_store<ST, SR>(b, hb, q)) << 16);
    else
        return 0u;  // no pair stores with FP32 storage
}

// Store of an x-shifted population, 16-bit storage with two nodes per thread: the lane's
// pair P = (g(x0), g(x0+1)) lands at x0 + 1, x0 + 2 (towards +x) or x0 - 1, x0 (towards
// -x), adjacent elements, so one 4-byte store at 2-byte alignment writes both (gfx9
// global stores allow it); only where the pair wraps around the row are its halves
// stored apart. Measured on MI355X: 2 % faster than joining neighbouring lanes' halves
// into aligned pairs by DPP, and every node's values go to the same locations.
template <int DIR>
__device__ __forceinline__ void store_pair_shifted(uint16_t *row, const PullRows &r, uint32_t P, unsigned nx)
{
    typedef uint32_t u32a2 __attribute__((aligned(2)));
    if constexpr (DIR > 0) {
        if (r.x0 + 2u < nx) {
            __builtin_nontemporal_store(P, reinterpret_cast<u32a2 *>(at32(row, r.x0 + 1u)));
        } else {  // x0 + 2 wraps to 0 (r.xr)
            __builtin_nontemporal_store((uint16_t)P, at32(row, r.x0 + 1u));
            __builtin_nontemporal_store((uint16_t)(P >> 16), at32(row, r.xr));
        }
    } else {
        if (r.x0 != 0u) {
            __builtin_nontemporal_store(P, reinterpret_cast<u32a2 *>(at32(row, r.x0 - 1u)));
        } else {  // x0 - 1 wraps to nx - 1 (r.xl)
            __builtin_nontemporal_store((uint16_t)P, at32(row, r.xl));
            __builtin_nontemporal_store((uint16_t)(P >> 16), at32(row, r.x0));
        }
    }
}

// Phase 0: pull, collide, store back where the opposite population was pulled from.
// V nodes per thread as in the two-buffer step (the local phase with solids takes one,
// step_vector_width); the node arithmetic is the same either way. The
// stores of x-shifted populations are shifted like their loads: one value at a time,
// or, with 16-bit storage and two nodes per thread, one 4-byte store per pair.
template <int LAT, int ST, bool MASK, bool SOFT, int FORCE, int V, bool SLIP, bool SR>
__global__ __launch_bounds__(kBlock) void k_step_aa_pull(StepArgs a, int ntx, FastDiv div_ntx, int nblocks)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    if constexpr (MASK && !SLIP) a.g.slip = 0;  // no free-slip planes: reflections compiled out
    const int bid = block_order((int)blockIdx.x, nblocks, a.remap);
    const Tile t = tile_of<V>(a.g, bid, ntx, div_ntx);
    if (!t.valid) return;
    // Rows of free-slip wall planes are solid as a whole: their blocks leave at once (a
    // wave-uniform test on the row, no memory access). Every other solid node takes part in
    // the loads and the collision, so that no lane waits for its link mask before its
    // population loads issue, and only fluid nodes store; except that with 16-bit storage
    // and two nodes per thread pairs are stored whole, obstacle nodes included: under the
    // solid-slot convention the locations an obstacle node pulls from (and so stores to)
    // are read and written by no fluid node (the index-map emulation of the host tests
    // checks this, for waves of obstacles only too). Wall-plane nodes are not like that,
    // which is why their rows leave.
    constexpr bool kPairs = ST != LBM_F32 && V == 2;
    static_assert(!kPairs || kSolidSlotBB<ST>, "pair stores rely on the solid-slot convention");
    if (MASK && a.g.slip &&
        (((a.g.slip & LBM_SLIP_Y) && (t.y == 0 || t.y == a.g.ny - 1)) ||
         ((a.g.slip & LBM_SLIP_Z) && (t.z == 0 || t.z == a.g.nz - 1))))
        return;
    LT lk[V];
    bool fluid[V];
    bool all_fluid = true;
    if (MASK) {
        load_links<LAT, V>(static_cast<const LT *>(a.links), t.own, lk);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            fluid[i] = !(lk[i] & LinkMask<LAT>::solid);
            all_fluid = all_fluid && fluid[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) fluid[i] = true;
    }
    T *f = static_cast<T *>(a.dst);
    float d[V][L::Q];
    gather_tile<LAT, ST, MASK, V>(a.g, f, 1.f, t, lk, d);  // stored units throughout
    float sv[V];
    if (SOFT) vload<LBM_F32, V>(at32(a.g.s, (unsigned)t.own), 1.f, sv);
    float o[V][L::Q];
#pragma unroll
    for (int i = 0; i < V; ++i) collide<LAT, SOFT, FORCE>(a.ph, d[i], SOFT ? sv[i] : 0.f, o[i]);
    uint32_t h[V];  // stochastic rounding: g_q(x) takes the bits of (x, q) wherever it goes
#pragma unroll
    for (int i = 0; i < V; ++i) h[i] = SR ? sr_node((uint32_t)t.own + (uint32_t)i, a.sr_key) : 0u;
    const PullRows r = pull_rows<V>(a.g, t);
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int qb = L::opp[q];
        T *row = f + pull_row<LAT, qb>(a.g, t, r);  // P(x, qbar) without bounce-back
        if constexpr (kPairs) {
            if constexpr (L::ex[q] != 0) {
                store_pair_shifted<L::ex[q]>(reinterpret_cast<uint16_t *>(row), r,
                                             pack_pair<ST, SR>(o[0][q], o[V - 1][q], h[0], h[V - 1], q),
                                             (unsigned)a.g.nx);
            } else {
                float v[V];
#pragma unroll
                for (int i = 0; i < V; ++i) v[i] = o[i][q];
                vstore_q<ST, V, SR>(at32(row, r.x0), v, h, q);
            }
            return;
        }
        if constexpr (L::ex[q] == 0 && (!MASK || kSolidSlotBB<ST>)) {
            if (all_fluid) {
                float v[V];
#pragma unroll
                for (int i = 0; i < V; ++i) v[i] = o[i][q];
                vstore_q<ST, V, SR>(at32(row, r.x0), v, h, q);
                return;
            }
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            if (!fluid[i]) continue;
            T *p;
            if (MASK && !kSolidSlotBB<ST> && ((lk[i] >> qb) & 1u))
                p = at32(f + slot_off(q, a.g.stride), (unsigned)t.own + i);  // bounced: slot q of x
            else
                p = at32(row, pull_x<LAT, qb, V>(r, i));
            vstore_q<ST, 1, SR>(p, &o[i][q], &h[i], q);
        }
    });
}

// Phase 0 without solids, 16-bit storage, two nodes per thread taken one node to the right
// (xa = x0 + 1, xb = x0 + 2 mod nx): the pairs a population pulls from and stores to start
// at x0 (towards +x pulls, towards -x stores), x0 + 2 mod nx (the other way) or x0 + 1
// (unshifted), so the x-shifted accesses, six of nine, are aligned 4-byte pairs and only
// the unshifted ones straddle; the last thread of a row (xb = 0) goes value by value for
// those. Same node arithmetic and same locations per node as k_step_aa_pull.
template <int LAT, int ST, bool SOFT, int FORCE, bool SR>
__global__ __launch_bounds__(kBlock) void k_step_aa_pull_odd(StepArgs a, int ntx, FastDiv div_ntx, int nblocks)
{
    static_assert(LAT == LBM_D2V9 && ST != LBM_F32, "16-bit D2V9 pairs");
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    typedef uint32_t u32a2 __attribute__((aligned(2)));
    const int bid = block_order((int)blockIdx.x, nblocks, a.remap);
    const Tile t = tile_of<2>(a.g, bid, ntx, div_ntx);
    if (!t.valid) return;
    const unsigned nx = (unsigned)a.g.nx;
    const unsigned x0 = (unsigned)t.x0, xa = x0 + 1u, xb = x0 + 2u == nx ? 0u : x0 + 2u;
    const bool last = xb == 0u;
    const unsigned rowbase = (unsigned)(t.own - t.x0);  // node index of x = 0 in this row
    T *f = static_cast<T *>(a.dst);
    const PullRows r = pull_rows<2>(a.g, t);
    auto pair_at = [&](int q) -> unsigned {  // first element of the pair node xa pulls q from
        return L::ex[q] > 0 ? x0 : (L::ex[q] < 0 ? xb : xa);
    };
    float d[2][L::Q];
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const T *row = f + pull_row<LAT, q>(a.g, t, r);
        uint32_t w;
        if constexpr (L::ex[q] == 0) {
            if (!last) {
                w = *reinterpret_cast<const u32a2 *>(at32(row, xa));
            } else {
                w = (uint32_t)__builtin_bit_cast(uint16_t, *at32(row, xa)) |
                    ((uint32_t)__builtin_bit_cast(uint16_t, *at32(row, 0u)) << 16);
            }
        } else {
            w = *reinterpret_cast<const uint32_t *>(at32(row, pair_at(q)));
        }
        d[0][q] = Codec<ST>::dec(__builtin_bit_cast(T, (uint16_t)w), 1.f);
        d[1][q] = Codec<ST>::dec(__builtin_bit_cast(T, (uint16_t)(w >> 16)), 1.f);
    });
    float sv[2] = {0.f, 0.f};
    if (SOFT) {
        sv[0] = *at32(a.g.s, rowbase + xa);
        sv[1] = *at32(a.g.s, rowbase + xb);
    }
    float o[2][L::Q];
    collide<LAT, SOFT, FORCE>(a.ph, d[0], sv[0], o[0]);
    collide<LAT, SOFT, FORCE>(a.ph, d[1], sv[1], o[1]);
    uint32_t h[2] = {0u, 0u};
    if (SR) {
        h[0] = sr_node(rowbase + xa, a.sr_key);
        h[1] = sr_node(rowbase + xb, a.sr_key);
    }
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int qb = L::opp[q];
        T *row = f + pull_row<LAT, qb>(a.g, t, r);  // P(x, qbar): slot qbar of x + e_q
        const uint32_t P = pack_pair<ST, SR>(o[0][q], o[1][q], h[0], h[1], q);
        if constexpr (L::ex[q] == 0) {
            if (!last) {
                __builtin_nontemporal_store(P, reinterpret_cast<u32a2 *>(at32(row, xa)));
            } else {
                __builtin_nontemporal_store((uint16_t)P, reinterpret_cast<uint16_t *>(at32(row, xa)));
                __builtin_nontemporal_store((uint16_t)(P >> 16), reinterpret_cast<uint16_t *>(at32(row, 0u)));
            }
        } else {
            // the pair node xa pulls qbar from is where g_q(xa), g_q(xb) go
            __builtin_nontemporal_store(P, reinterpret_cast<uint32_t *>(at32(row, pair_at(qb))));
        }
    });
}

// Phase 1: read the streamed populations of the node, collide, store in place.
template <int LAT, int ST, bool MASK, bool SOFT, int FORCE, int V, bool SLIP, bool SR>
__global__ __launch_bounds__(kBlock) void k_step_aa_local(StepArgs a, int ntx, FastDiv div_ntx, int nblocks)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    if constexpr (MASK && !SLIP) a.g.slip = 0;
    const int bid = block_order((int)blockIdx.x, nblocks, a.remap);
    const Tile t = tile_of<V>(a.g, bid, ntx, div_ntx);
    if (!t.valid) return;
    // solid nodes load and collide too (their own slots, in bounds), so that no lane waits
    // for its link mask before its loads issue; store_tile decides what they store
    LT lk[V];
    if (MASK) load_links<LAT, V>(static_cast<const LT *>(a.links), t.own, lk);
    T *f = static_cast<T *>(a.dst);
    float d[V][L::Q];
    gather_odd<LAT, ST, MASK, V>(a.g, f, 1.f, t, lk, d);
    float sv[V];
    if (SOFT) vload<LBM_F32, V>(at32(a.g.s, (unsigned)t.own), 1.f, sv);
    float o[V][L::Q];
#pragma unroll
    for (int i = 0; i < V; ++i) collide<LAT, SOFT, FORCE>(a.ph, d[i], SOFT ? sv[i] : 0.f, o[i]);
    uint32_t h[V];
#pragma unroll
    for (int i = 0; i < V; ++i) h[i] = SR ? sr_node((uint32_t)t.own + (uint32_t)i, a.sr_key) : 0u;
    store_tile<LAT, ST, MASK, V, SR, true>(a.g, f, t, lk, o, h);
}

// Runtime flags -> template instances.
template <int LAT, int ST, int V, bool SR>
hipError_t aa_v(int force, int phase, const StepArgs &a, hipStream_t st)
{
    const bool mask = a.links != nullptr, soft = a.g.s != nullptr;
    const int ntx = (a.g.nx + kBlock * V - 1) / (kBlock * V);
    const int nblocks = ntx * a.g.ny * a.g.nz;
    const FastDiv div_ntx = make_fastdiv(ntx);
    const dim3 grid(nblocks), block(row_block_threads(a.g.nx, V));
    StepArgs b = a;
    b.remap = remap_code(a.remap, ntx);
#define LBM_AA_SL(M, S, F, SL)                                                                                   \
    if constexpr (!M && LAT == LBM_D2V9 && ST != LBM_F32 && V == 2) {                                           \
        if (phase == 0) {                                                                                       \
            hipLaunchKernelGGL((k_step_aa_pull_odd<LAT, ST, S, F, SR>), grid, block, 0, st, b, ntx, div_ntx,     \
                               nblocks);                                                                        \
            break;                                                                                              \
        }                                                                                                       \
    }                                                                                                           \
    if (phase == 0)                                                                                             \
        hipLaunchKernelGGL((k_step_aa_pull<LAT, ST, M, S, F, V, SL, SR>), grid, block, 0, st, b, ntx, div_ntx,  \
                           nblocks);                                                                            \
    else                                                                                                        \
        hipLaunchKernelGGL((k_step_aa_local<LAT, ST, M, S, F, V, SL, SR>), grid, block, 0, st, b, ntx, div_ntx, \
                           nblocks)
#define LBM_AA(M, S, F)                \
    do {                               \
        if (M && a.g.slip) {           \
            LBM_AA_SL(M, S, F, M);     \
        } else {                       \
            LBM_AA_SL(M, S, F, false); \
        }                              \
    } while (0)
#define LBM_AA_F(M, S)     \
    if (force == 0)        \
        LBM_AA(M, S, 0);   \
    else if (force == 1)   \
        LBM_AA(M, S, 1);   \
    else if (force == 2)   \
        LBM_AA(M, S, 2);   \
    else                   \
        LBM_AA(M, S, 3)
    if (mask) {
        if (soft) LBM_AA_F(true, true); else LBM_AA_F(true, false);
    } else {
        if (soft) LBM_AA_F(false, true); else LBM_AA_F(false, false);
    }
#undef LBM_AA_F
#undef LBM_AA
#undef LBM_AA_SL
    return hipGetLastError();
}

template <int LAT, int ST, bool SR>
hipError_t aa_lat_st(int force, int phase, const StepArgs &a, hipStream_t st)
{
    if (step_vector_width(LAT, ST, a.g.nx, a.links != nullptr && phase == 1) == 2)
        return aa_v<LAT, ST, 2, SR>(force, phase, a, st);
    return aa_v<LAT, ST, 1, SR>(force, phase, a, st);
}

}  // namespace
}  // namespace lbm
