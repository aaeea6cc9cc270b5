// lbm_aa.hip -- the in-place time step on one state buffer: the AA access pattern
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
#include "lbm_device.h"

namespace lbm {
namespace {

// Two values encoded in 16 bits each, a in the low half (16-bit storage only).
template <int ST>
__device__ __forceinline__ uint32_t pack_pair(float a, float b)
{
    using T = typename Codec<ST>::T;
    if constexpr (sizeof(T) == 2)
        return (uint32_t)__builtin_bit_cast(uint16_t, Codec<ST>::enc(a, 1.f)) |
               ((uint32_t)__builtin_bit_cast(uint16_t, Codec<ST>::enc(b, 1.f)) << 16);
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
// V nodes per thread as in the two-buffer step (same node arithmetic, same bits). The
// stores of x-shifted populations are shifted like their loads: one value at a time,
// or, with 16-bit storage and two nodes per thread, one 4-byte store per pair.
template <int LAT, int ST, bool MASK, bool SOFT, int FORCE, int V, bool SLIP>
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
    const PullRows r = pull_rows<V>(a.g, t);
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int qb = L::opp[q];
        T *row = f + pull_row<LAT, qb>(a.g, t, r);  // P(x, qbar) without bounce-back
        if constexpr (kPairs) {
            if constexpr (L::ex[q] != 0) {
                store_pair_shifted<L::ex[q]>(reinterpret_cast<uint16_t *>(row), r,
                                             pack_pair<ST>(o[0][q], o[V - 1][q]), (unsigned)a.g.nx);
            } else {
                float v[V];
#pragma unroll
                for (int i = 0; i < V; ++i) v[i] = o[i][q];
                vstore<ST, V>(at32(row, r.x0), 1.f, v);
            }
            return;
        }
        if constexpr (L::ex[q] == 0 && (!MASK || kSolidSlotBB<ST>)) {
            if (all_fluid) {
                float v[V];
#pragma unroll
                for (int i = 0; i < V; ++i) v[i] = o[i][q];
                vstore<ST, V>(at32(row, r.x0), 1.f, v);
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
            vstore<ST, 1>(p, 1.f, &o[i][q]);
        }
    });
}

// Phase 1: read the streamed populations of the node, collide, store in place.
template <int LAT, int ST, bool MASK, bool SOFT, int FORCE, int V, bool SLIP>
__global__ __launch_bounds__(kBlock) void k_step_aa_local(StepArgs a, int ntx, FastDiv div_ntx, int nblocks)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    if constexpr (MASK && !SLIP) a.g.slip = 0;
    const int bid = block_order((int)blockIdx.x, nblocks, a.remap);
    const Tile t = tile_of<V>(a.g, bid, ntx, div_ntx);
    if (!t.valid) return;
    // solid nodes load and collide too (their own slots, in bounds) and store nothing:
    // no lane waits for its link mask before its loads issue
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
    store_tile<LAT, ST, MASK, V>(a.g, f, t, lk, o);
}

// Even layout of an odd-layout state, out of place: g_q(x) = src[P(x, qbar)] into slot q
// of x, and under the solid-slot convention the bounced values (already where the pull
// reads them) copied to the same solid slots of dst. Slots no pull reads are left as
// they were. Stored values are moved unchanged (decoding and re-encoding in stored units
// is exact).
template <int LAT, int ST, bool MASK>
__global__ __launch_bounds__(kBlock) void k_canon(StepArgs a)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    const Tile t = tile_of(a.g, (int)blockIdx.x);
    if (!t.valid) return;
    LT lk[1] = {0};
    if (MASK) {
        lk[0] = *at32(static_cast<const LT *>(a.links), (unsigned)t.own);
        if (lk[0] & LinkMask<LAT>::solid) return;
    }
    float d[1][L::Q];
    gather_tile<LAT, ST, MASK, 1>(a.g, static_cast<const T *>(a.src), 1.f, t, lk, d);  // d[q] = src[P(x, q)]
    T *dst = static_cast<T *>(a.dst);
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
        *at32(dst + slot_off(q, a.g.stride), (unsigned)t.own) = Codec<ST>::enc(d[0][L::opp[q]], 1.f);
    if constexpr (MASK && kSolidSlotBB<ST>) {
        if (lk[0]) {
            const PullRows r = pull_rows<1>(a.g, t);
            for_q<L::Q>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if constexpr (q != 0)
                    if ((lk[0] >> q) & 1u)
                        *at32(dst + pull_row<LAT, q>(a.g, t, r), pull_x<LAT, q, 1>(r, 0)) =
                            Codec<ST>::enc(d[0][q], 1.f);
            });
        }
    }
}

template <int LAT, int ST, int V>
hipError_t aa_v(int force, int phase, const StepArgs &a, hipStream_t st)
{
    const bool mask = a.links != nullptr, soft = a.g.s != nullptr;
    const int ntx = (a.g.nx + kBlock * V - 1) / (kBlock * V);
    const int nblocks = ntx * a.g.ny * a.g.nz;
    const FastDiv div_ntx = make_fastdiv(ntx);
    const dim3 grid(nblocks), block(row_block_threads(a.g.nx, V));
    StepArgs b = a;
    b.remap = remap_code(a.remap, ntx);
#define LBM_AA_SL(M, S, F, SL)                                                                                     \
    if (phase == 0)                                                                                               \
        hipLaunchKernelGGL((k_step_aa_pull<LAT, ST, M, S, F, V, SL>), grid, block, 0, st, b, ntx, div_ntx, nblocks); \
    else                                                                                                          \
        hipLaunchKernelGGL((k_step_aa_local<LAT, ST, M, S, F, V, SL>), grid, block, 0, st, b, ntx, div_ntx, nblocks)
#define LBM_AA(M, S, F)           \
    do {                          \
        if (M && a.g.slip) {      \
            LBM_AA_SL(M, S, F, M);     \
        } else {                  \
            LBM_AA_SL(M, S, F, false); \
        }                         \
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

template <int LAT, int ST>
hipError_t aa_lat_st(int force, int phase, const StepArgs &a, hipStream_t st)
{
    if (step_vector_width(LAT, ST, a.g.nx) == 2) return aa_v<LAT, ST, 2>(force, phase, a, st);
    return aa_v<LAT, ST, 1>(force, phase, a, st);
}

template <int LAT, int ST>
hipError_t canon_lat_st(const StepArgs &a, hipStream_t st)
{
    const dim3 grid(a.g.nblocks), block(kBlock);
    if (a.links)
        hipLaunchKernelGGL((k_canon<LAT, ST, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_canon<LAT, ST, false>), grid, block, 0, st, a);
    return hipGetLastError();
}

}  // namespace

#define LBM_AA_DISPATCH(FN, ...)                                                          \
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

hipError_t launch_step_aa(int lattice, int storage, int force, int phase, const StepArgs &a, hipStream_t st)
{
    if (a.src != a.dst || (phase != 0 && phase != 1)) return hipErrorInvalidValue;
    LBM_AA_DISPATCH(aa_lat_st, force, phase, a, st);
}

hipError_t launch_canon(int lattice, int storage, const StepArgs &a, hipStream_t st)
{
    if (a.src == a.dst) return hipErrorInvalidValue;
    LBM_AA_DISPATCH(canon_lat_st, a, st);
}

}  // namespace lbm
