// lbm_device.h -- device-side building blocks shared by the step kernels: storage codecs,
// vector loads and stores, lattice helpers, the thread -> node map, the pull of a tile
// (streaming with halfway bounce-back and free-slip walls) and the collision of one node.
#pragma once

#include "lbm_internal.h"

#include <type_traits>

#ifndef LBM_NT_STORE
#define LBM_NT_STORE 1
#endif

namespace lbm {

// ---------------------------------------------------------------------------------
// Storage codecs: deviation <-> stored value (round to nearest even; stochastic
// rounding for the 16-bit formats further down).
// ---------------------------------------------------------------------------------
template <int ST>
struct Codec;

template <>
struct Codec<LBM_F32> {
    using T = float;
    static __device__ __forceinline__ float dec(T v, float) { return v; }
    static __device__ __forceinline__ T enc(float f, float) { return f; }
    static __device__ __forceinline__ T enc_sr(float f, uint32_t) { return f; }
};

// Encoding rounds the FP32 value: the empty asm statement makes it opaque, so that the
// conversion is not folded into the fused multiply-add that produced the value (a mixed
// FMA that writes 16 bits, which the compiler chooses in some kernels and not in others,
// and which can round differently).
__device__ __forceinline__ float opaque(float f)
{
    asm("" : "+v"(f));
    return f;
}

template <>
struct Codec<LBM_F16> {
    using T = _Float16;
    // stored value = d * 2^k; the scale is a power of two, so scaling is exact
    static __device__ __forceinline__ float dec(T v, float inv_scale) { return (float)v * inv_scale; }
    static __device__ __forceinline__ T enc(float f, float scale) { return (T)opaque(f * scale); }
    // stochastic rounding of a value already in stored units, random bits r
    typedef _Float16 T2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ T enc_sr(float f, uint32_t r)
    {
        return __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(T2, r), opaque(f), r, false)[0];
    }
    // two values into one register (a low, b high): the second conversion writes the high
    // half in place, and the first one's register is that of its random word
    static __device__ __forceinline__ T2 enc_sr2(float a, uint32_t ra, float b, uint32_t rb)
    {
        const T2 lo = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(T2, ra), opaque(a), ra, false);
        return __builtin_amdgcn_cvt_sr_f16_f32(lo, opaque(b), rb, true);
    }
};

template <>
struct Codec<LBM_BF16> {
    using T = __bf16;
    static __device__ __forceinline__ float dec(T v, float) { return (float)v; }
    static __device__ __forceinline__ T enc(float f, float) { return (T)opaque(f); }
    typedef __bf16 T2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ T enc_sr(float f, uint32_t r)
    {
        return __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(T2, r), opaque(f), r, false)[0];
    }
    static __device__ __forceinline__ T2 enc_sr2(float a, uint32_t ra, float b, uint32_t rb)
    {
        const T2 lo = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(T2, ra), opaque(a), ra, false);
        return __builtin_amdgcn_cvt_sr_bf16_f32(lo, opaque(b), rb, true);
    }
};

// ---------------------------------------------------------------------------------
// Stochastic rounding of the stored 16-bit values (optional; not in the paper). The
// random bits for the value of population q that the step of key k writes for node n
// are sr_bits(sr_node(n, k), q): one integer hash per node -- Wellons's "lowbias32"
// mixer, a bijection of 32-bit words -- of the node index and the step's key, then a
// Weyl increment per population (any fixed set of bits of the result is uniform over
// the nodes). Each stored value carries the bits of its own (node, population), so the
// same value gets the same bits wherever a step stores it (own slot, solid slot, the
// layouts of the in-place step).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t sr_node(uint32_t n, uint32_t key)
{
    uint32_t x = (n * 0x9E3779B9u) ^ key;
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ uint32_t sr_bits(uint32_t h, int q) { return h + (uint32_t)q * 0x9E3779B9u; }

// The stored code of a value in stored units: round to nearest even, or stochastic with
// the bits of (node hash h, population q).
template <int ST, bool SR>
__device__ __forceinline__ typename Codec<ST>::T enc_store(float f, uint32_t h, int q)
{
    if constexpr (SR)
        return Codec<ST>::enc_sr(f, sr_bits(h, q));
    else
        return Codec<ST>::enc(f, 1.f);
}

// Where a bounced population is kept between steps (halfway bounce-back: the value
// pulled into fluid x as population q, when x - e_q is solid, is f*_qbar(x)):
// * own slot (FP32): it stays in slot qbar of x, where the step stores it anyway, and
//   the pull at x reloads it from there for the links of x;
// * solid slot (16-bit): the step also stores it in slot q of the solid node x - e_q,
//   so every pull is a plain read of x - e_q and waits on no link mask.
// Measured on MI355X: the solid slot wins where both state buffers stay in the 256 MB
// Infinity Cache (16-bit 2048^2 disks 1.3x); with FP32 buffers beyond it, its scattered
// partial-line stores cost more than the reloads (FP32 2048^2 disks 0.89x).
template <int ST>
constexpr bool kSolidSlotBB = ST != LBM_F32;

template <int ST, int V>
struct VecT {
    typedef typename Codec<ST>::T type __attribute__((ext_vector_type(V)));
};
template <int ST>
struct VecT<ST, 1> {
    using type = typename Codec<ST>::T;
};

// Non-temporal loads: each value is read once per step (measured on MI355X: +3 % on the
// 4096^2 FP32 step, +5 % on the FP32 duct and the 16-bit disk packing). The x-shifted
// populations of one-node tiles, the edge values of V-wide tiles and the shifted 16-bit
// pairs are loaded through the cache instead (gather_tile): their lines straddle the
// neighbouring tile's.
template <int ST, int V>
__device__ __forceinline__ void vload(const typename Codec<ST>::T *p, float inv_scale, float *f)
{
    if constexpr (V == 1) {
        f[0] = Codec<ST>::dec(__builtin_nontemporal_load(p), inv_scale);
    } else {
        using VT = typename VecT<ST, V>::type;
        const VT v = __builtin_nontemporal_load(reinterpret_cast<const VT *>(p));
#pragma unroll
        for (int i = 0; i < V; ++i) f[i] = Codec<ST>::dec(v[i], inv_scale);
    }
}

// V encoded values (V-wide store)
template <int ST, int V>
__device__ __forceinline__ void vstore_codes(typename Codec<ST>::T *p, const typename Codec<ST>::T *c)
{
    if constexpr (V == 1) {
#if LBM_NT_STORE
        __builtin_nontemporal_store(c[0], p);
#else
        *p = c[0];
#endif
    } else {
        using VT = typename VecT<ST, V>::type;
        VT v;
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = c[i];
#if LBM_NT_STORE
        __builtin_nontemporal_store(v, reinterpret_cast<VT *>(p));
#else
        *reinterpret_cast<VT *>(p) = v;
#endif
    }
}

template <int ST, int V>
__device__ __forceinline__ void vstore(typename Codec<ST>::T *p, float scale, const float *f)
{
    typename Codec<ST>::T c[V];
#pragma unroll
    for (int i = 0; i < V; ++i) c[i] = Codec<ST>::enc(f[i], scale);
    vstore_codes<ST, V>(p, c);
}

// Population q of V consecutive nodes with node hashes h (values in stored units).
template <int ST, int V, bool SR>
__device__ __forceinline__ void vstore_q(typename Codec<ST>::T *p, const float *f, const uint32_t *h, int q)
{
    if constexpr (SR && V == 2 && ST != LBM_F32) {
        using VT = typename VecT<ST, 2>::type;
        const VT v = Codec<ST>::enc_sr2(f[0], sr_bits(h[0], q), f[1], sr_bits(h[1], q));
#if LBM_NT_STORE
        __builtin_nontemporal_store(v, reinterpret_cast<VT *>(p));
#else
        *reinterpret_cast<VT *>(p) = v;
#endif
    } else {
        typename Codec<ST>::T c[V];
#pragma unroll
        for (int i = 0; i < V; ++i) c[i] = enc_store<ST, SR>(f[i], SR ? h[i] : 0u, q);
        vstore_codes<ST, V>(p, c);
    }
}

// Element offset of slot q (the start of population array q). Every element offset of a
// state or adjoint field fits in 32 bits (Q * stride < 2^31 is checked at create), so the
// products are formed in 32-bit arithmetic and only widened for the final address.
__device__ __forceinline__ size_t slot_off(int q, int stride) { return (size_t)((unsigned)q * (unsigned)stride); }

// base + idx elements with the byte offset formed in 32 bits, so that a load or store
// takes the uniform base in SGPRs and one VGPR offset instead of a 64-bit lane address.
// Every array indexed this way is below 4 GiB (Q * stride < 2^31 elements).
template <class T>
__device__ __forceinline__ T *at32(T *base, unsigned idx)
{
    using C = std::conditional_t<std::is_const_v<T>, const char, char>;
    return reinterpret_cast<T *>(reinterpret_cast<C *>(base) + idx * (unsigned)sizeof(T));
}

// ---------------------------------------------------------------------------------
// Lattice helpers (all indices compile-time after unrolling).
// ---------------------------------------------------------------------------------
template <int LAT, int q>
__device__ __forceinline__ constexpr int shell()
{
    using L = Lat<LAT>;
    return L::ex[q] * L::ex[q] + L::ey[q] * L::ey[q] + L::ez[q] * L::ez[q];
}

// e_q . v without adding zeros (0 + x cannot be folded in IEEE arithmetic).
template <int LAT, int q>
__device__ __forceinline__ float edot(const float *v)
{
#pragma clang fp contract(off)
    using L = Lat<LAT>;
    constexpr int a = L::ex[q], b = L::ey[q], c = L::ez[q];
    if constexpr (a == 0 && b == 0 && c == 0) {
        return 0.f;
    } else {
        float r = 0.f;
        bool first = true;
        if constexpr (a != 0) {
            r = a > 0 ? v[0] : -v[0];
            first = false;
        }
        if constexpr (b != 0) {
            const float t = b > 0 ? v[1] : -v[1];
            r = first ? t : r + t;
            first = false;
        }
        if constexpr (c != 0) {
            const float t = c > 0 ? v[2] : -v[2];
            r = first ? t : r + t;
        }
        return r;
    }
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

template <int LAT>
struct LinkMask;
template <>
struct LinkMask<LBM_D2V9> {
    using T = uint16_t;
    static constexpr T solid = (T)0x8000u;
};
template <>
struct LinkMask<LBM_D3V19> {
    using T = uint32_t;
    static constexpr T solid = 0x80000000u;
};

// ---------------------------------------------------------------------------------
// Thread -> nodes.
// ---------------------------------------------------------------------------------
// Block -> contiguous slab per XCD.
__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = bid & 7, k = bid >> 3;
    return xcd * per + min(xcd, rem) + k;
}

// Block order of the node kernels (the hardware deals blocks round-robin to the 8 XCDs):
//   remap 0: the hardware order;
//   remap 1: each XCD a contiguous slab of the grid (xcd_remap);
//   remap c >= 2: chunks of 2^(c - 2) consecutive tiles (a whole row of tiles) dealt
//   round-robin to the XCDs, so that the tiles of a row, which share the cache lines at
//   their x edges, run on one XCD (one L2) while the 8 XCDs still work on neighbouring
//   rows; a tail of fewer than 8 chunks keeps the hardware order.
__device__ __forceinline__ int block_order(int bid, int nb, int remap)
{
    if (remap == 1) return xcd_remap(bid, nb);
    if (remap >= 2) {
        const int sh = remap - 2, group = 8 << sh;
        if (bid >= nb - nb % group) return bid;
        const int xcd = bid & 7, k = bid >> 3;
        return ((((k >> sh) << 3) + xcd) << sh) + (k & ((1 << sh) - 1));
    }
    return bid;
}

__device__ __forceinline__ int wrapm(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wrapp(int i, int n) { return i == n - 1 ? 0 : i + 1; }

struct Tile {
    int x0, y, z;  // first node of this thread (clamped into the row)
    int own;       // node index of x0
    bool valid;    // the thread owns nodes
};

__device__ __forceinline__ int fast_div(int n, FastDiv f)
{
    return (int)(((uint64_t)(uint32_t)n * f.m) >> f.sh);
}

// Block bid covers kBlock * V nodes of one x row; ntx such blocks per row.
template <int V>
__device__ __forceinline__ Tile tile_of(const Geometry &g, int bid, int ntx, FastDiv div_ntx)
{
    const int row = fast_div(bid, div_ntx);
    Tile t;
    int x0 = ((bid - row * ntx) * kBlock + (int)threadIdx.x) * V;
    t.valid = x0 < g.nx;
    if (!t.valid) x0 = g.nx - V;
    t.x0 = x0;
    t.z = fast_div(row, g.div_ny);
    t.y = row - t.z * g.ny;
    t.own = x0 + g.nx * row;
    return t;
}

__device__ __forceinline__ Tile tile_of(const Geometry &g, int bid) { return tile_of<1>(g, bid, g.ntx, g.div_ntx); }

// Source of the pull of population q into node x0 + i of tile t: the row of x - e_q
// (element offset of its first node) and the x index within that row.
struct PullRows {
    int ym, yp, zm, zp;
    unsigned x0, xl, xr;
};

template <int V>
__device__ __forceinline__ PullRows pull_rows(const Geometry &g, const Tile &t)
{
    PullRows r;
    r.ym = wrapm(t.y, g.ny);
    r.yp = wrapp(t.y, g.ny);
    r.zm = wrapm(t.z, g.nz);
    r.zp = wrapp(t.z, g.nz);
    // lane offsets are unsigned 32-bit, so accesses use a scalar base and one VGPR offset
    r.x0 = (unsigned)t.x0;
    r.xl = t.x0 == 0 ? (unsigned)(g.nx - 1) : r.x0 - 1u;
    r.xr = t.x0 + V >= g.nx ? 0u : r.x0 + (unsigned)V;
    return r;
}

// Index of e_q with its y (fy) and/or z (fz) component reversed.
template <int LAT>
constexpr int reflected(int q, bool fy, bool fz)
{
    using L = Lat<LAT>;
    for (int b = 0; b < L::Q; ++b)
        if (L::ex[b] == L::ex[q] && L::ey[b] == (fy ? -L::ey[q] : L::ey[q]) &&
            L::ez[b] == (fz ? -L::ez[q] : L::ez[q]))
            return b;
    return -1;
}

// Element offset of the value pulled into the row of tile t as population q: slot q of
// the row of x - e_q; where that row is a free-slip wall plane, the specular source,
// i.e. slot qr (e_q with the wall-normal components reversed) of the row of x itself
// (the tile's row is uniform over the block, so this choice is a scalar one).
template <int LAT, int q>
__device__ __forceinline__ size_t pull_row(const Geometry &g, const Tile &t, const PullRows &r)
{
    using L = Lat<LAT>;
    int sy = L::ey[q] > 0 ? r.ym : (L::ey[q] < 0 ? r.yp : t.y);
    int sz = L::ez[q] > 0 ? r.zm : (L::ez[q] < 0 ? r.zp : t.z);
    int p = q;
    if (g.slip) {
        const bool fy = L::ey[q] != 0 && (g.slip & LBM_SLIP_Y) && (sy == 0 || sy == g.ny - 1);
        const bool fz = L::ez[q] != 0 && (g.slip & LBM_SLIP_Z) && (sz == 0 || sz == g.nz - 1);
        if (fy) sy = t.y;
        if (fz) sz = t.z;
        constexpr int py = reflected<LAT>(q, true, false), pz = reflected<LAT>(q, false, true);
        constexpr int pyz = reflected<LAT>(q, true, true);
        p = fy ? (fz ? pyz : py) : (fz ? pz : q);
    }
    return (size_t)((unsigned)p * (unsigned)g.stride + (unsigned)g.nx * (unsigned)(sy + g.ny * sz));
}

template <int LAT, int q, int V>
__device__ __forceinline__ unsigned pull_x(const PullRows &r, int i)
{
    using L = Lat<LAT>;
    if constexpr (L::ex[q] > 0) return i == 0 ? r.xl : r.x0 + (unsigned)(i - 1);
    else if constexpr (L::ex[q] < 0) return i == V - 1 ? r.xr : r.x0 + (unsigned)(i + 1);
    else return r.x0 + (unsigned)i;
}

// Pull the pre-collision deviations of the V nodes of tile t (link masks lk). With the
// solid-slot convention every pull is a plain read of x - e_q; with the own-slot one the
// populations whose source x - e_q is solid are then reloaded from slot qbar of x.
template <int LAT, int ST, bool MASK, int V>
__device__ __forceinline__ void gather_tile(const Geometry &g, const typename Codec<ST>::T *__restrict__ src,
                                            float inv_scale, const Tile &t,
                                            const typename LinkMask<LAT>::T *lk, float (&d)[V][Lat<LAT>::Q])
{
    using L = Lat<LAT>;
    const PullRows r = pull_rows<V>(g, t);
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const typename Codec<ST>::T *base = src + pull_row<LAT, q>(g, t, r);
        if constexpr (L::ex[q] == 0) {
            float f[V];
            vload<ST, V>(at32(base, r.x0), inv_scale, f);
#pragma unroll
            for (int i = 0; i < V; ++i) d[i][q] = f[i];
        } else if constexpr (V == 1) {
            d[0][q] = Codec<ST>::dec(*at32(base, L::ex[q] > 0 ? r.xl : r.xr), inv_scale);
        } else if constexpr (ST != LBM_F32 && V == 2) {
            // 16-bit pairs: the two pulled values (x0 - 1, x0) or (x0 + 1, x0 + 2) are adjacent,
            // so one 4-byte load at 2-byte alignment fetches them (gfx9 global loads allow
            // it); it stays cached, its lines being shared with the neighbouring lanes. Where
            // the pair wraps around the row, the address is clamped into the row and the
            // element from the row's other end comes from a wave-uniform load (a wave lies in
            // one row). Branch-free: a conditional load would make the wave wait for it.
            // Measured on MI355X: 4096^2 FP16 +9 %, in place +5 %, against an aligned pair
            // load plus a 2-byte load of the edge element.
            using T = typename Codec<ST>::T;
            typedef uint32_t u32a2 __attribute__((aligned(2)));
            const uint32_t *row32 = reinterpret_cast<const uint32_t *>(base);  // 4-byte aligned: stride, nx even
            uint16_t e0, e1;
            if constexpr (L::ex[q] > 0) {  // (x0 - 1, x0); at x0 = 0 the first is x = nx - 1
                const bool wrap = r.x0 == 0u;
                const uint32_t w = *reinterpret_cast<const u32a2 *>(at32(base, wrap ? 0u : r.x0 - 1u));
                const uint32_t last = row32[(unsigned)g.nx / 2u - 1u];  // (nx - 2, nx - 1)
                e0 = wrap ? (uint16_t)(last >> 16) : (uint16_t)w;
                e1 = wrap ? (uint16_t)w : (uint16_t)(w >> 16);
            } else {  // (x0 + 1, x0 + 2); at x0 = nx - 2 the second is x = 0
                const bool wrap = r.x0 + 2u >= (unsigned)g.nx;
                const uint32_t w = *reinterpret_cast<const u32a2 *>(at32(base, wrap ? r.x0 : r.x0 + 1u));
                const uint32_t first = row32[0];  // (0, 1)
                e0 = wrap ? (uint16_t)(w >> 16) : (uint16_t)w;
                e1 = wrap ? (uint16_t)first : (uint16_t)(w >> 16);
            }
            T t0, t1;
            __builtin_memcpy(&t0, &e0, 2);
            __builtin_memcpy(&t1, &e1, 2);
            d[0][q] = Codec<ST>::dec(t0, inv_scale);
            d[1][q] = Codec<ST>::dec(t1, inv_scale);
        } else if constexpr (L::ex[q] > 0) {  // from x - 1
            float f[V];
            vload<ST, V>(at32(base, r.x0), inv_scale, f);
            d[0][q] = Codec<ST>::dec(*at32(base, r.xl), inv_scale);
#pragma unroll
            for (int i = 1; i < V; ++i) d[i][q] = f[i - 1];
        } else {  // from x + 1
            float f[V];
            vload<ST, V>(at32(base, r.x0), inv_scale, f);
#pragma unroll
            for (int i = 0; i < V - 1; ++i) d[i][q] = f[i + 1];
            d[V - 1][q] = Codec<ST>::dec(*at32(base, r.xr), inv_scale);
        }
    });
    if constexpr (MASK && !kSolidSlotBB<ST>) {
        // one branch for the whole tile: most tiles have no solid neighbour at all
        typename LinkMask<LAT>::T any = 0;
#pragma unroll
        for (int i = 0; i < V; ++i) any |= lk[i] & (typename LinkMask<LAT>::T)~LinkMask<LAT>::solid;
        if (any) {
            const unsigned own = (unsigned)t.own;
#pragma unroll
            for (int i = 0; i < V; ++i) {
#pragma unroll
                for (int q = 1; q < L::Q; ++q)
                    if ((lk[i] >> q) & 1u)
                        d[i][q] = Codec<ST>::dec(*at32(src + slot_off(L::opp[q], g.stride), own + i), inv_scale);
            }
        }
    }
}

// Pre-collision deviations of the V nodes of tile t from a state in the odd layout of the
// in-place step, where the pulled population f_q(x) sits in slot qbar of x itself, except
// that with the solid-slot convention a bounced one stays where the pull reads it (slot q
// of the solid node x - e_q). There every value is loaded once from a per-lane address
// (own slot or solid slot), so that no load waits for another; 16-bit states are below
// 4 GiB, so one 32-bit byte offset from src reaches every slot. Waves without a bounced
// link load node pairs with vector loads. The per-lane loads go through the cache (not
// non-temporal): the local phase then stores the bounced copies into the same solid-slot
// lines, and the next pull phase finds them cached (measured on MI355X with the in-place
// local phase's non-temporal bounced stores: FP16 2048^2 disks -11 % per step, FP16 Hall
// duct -6 %, the paper's 3D Ohm sample in FP16 -6 %).
template <int LAT, int ST, bool MASK, int V>
__device__ __forceinline__ void gather_odd(const Geometry &g, const typename Codec<ST>::T *src, float inv_scale,
                                           const Tile &t, const typename LinkMask<LAT>::T *lk,
                                           float (&d)[V][Lat<LAT>::Q])
{
    using L = Lat<LAT>;
    using LT = typename LinkMask<LAT>::T;
    if constexpr (MASK && kSolidSlotBB<ST>) {
        LT any = 0;
#pragma unroll
        for (int i = 0; i < V; ++i) any |= lk[i] & (LT)~LinkMask<LAT>::solid;
        if (V == 1 || __builtin_amdgcn_ballot_w64(any != 0) != 0) {
            const PullRows r = pull_rows<V>(g, t);
            for_q<L::Q>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                const unsigned own = (unsigned)L::opp[q] * (unsigned)g.stride + (unsigned)t.own;
                const unsigned row = (unsigned)pull_row<LAT, q>(g, t, r);
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    const unsigned off = (q != 0 && ((lk[i] >> q) & 1u)) ? row + pull_x<LAT, q, V>(r, i) : own + i;
                    d[i][q] = Codec<ST>::dec(*at32(src, off), inv_scale);
                }
            });
            return;
        }
    }
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        float f[V];
        vload<ST, V>(at32(src + slot_off(L::opp[q], g.stride), (unsigned)t.own), inv_scale, f);
#pragma unroll
        for (int i = 0; i < V; ++i) d[i][q] = f[i];
    }
}

template <int LAT, int V>
__device__ __forceinline__ void load_links(const typename LinkMask<LAT>::T *links, int own,
                                           typename LinkMask<LAT>::T (&lk)[V])
{
    using LT = typename LinkMask<LAT>::T;
    if constexpr (V == 1) {
        lk[0] = *at32(links, (unsigned)own);
    } else {
        typedef LT VT __attribute__((ext_vector_type(V)));
        const VT v = *reinterpret_cast<const VT *>(at32(links, (unsigned)own));
#pragma unroll
        for (int i = 0; i < V; ++i) lk[i] = v[i];
    }
}

// ---------------------------------------------------------------------------------
// Collision of one node in deviation form: the discrete BGK update of Sec. 9.1 with the
// reduced second-order EDF and the Lorentz source of Sec. 7, then the optional partial
// bounce-back.
//   rho = rho0 + drho, drho = sum d, j = sum d e, U = u / c_s = j / (rho c_s^2);
//   deq_q = what_k drho + lam_k (e.j) + what_k rho (Bc (e.U)^2 + C_k c_s^2 U^2), q != 0,
//           lam_k (e.j) = what_k rho A (e.U) with lam weights whose second moment is
//           exactly the identity: the equilibrium carries exactly the node's momentum;
//   deq_0 = drho - sum_(q != 0) deq_q (mass closure);
//   sigma_q = (e.E / c_s)(A + 2 Bc e.U) + 2 C_k (c_s U.E + e.(B x U));
//   d*_q = d_q + omega (deq_q - d_q) + rho what_k sigma_q;
//   g_q = (1 - s) d*_q + s d_qbar.
// FORCE: 0 no field, 1 E only, 2 E and B (source term); 3 velocity shift (E and B): no
// sigma, and deq_q taken at j + rho tau c_s (E + u x B), i.e. at u + tau (E + u x B).
// ---------------------------------------------------------------------------------
// Products written with explicit fused multiply-adds: left to the compiler, a*b + c*d
// may be contracted either way round. The node arithmetic below (macro, relax_node,
// collide) states every fused multiply-add and turns implicit contraction off, so that
// every kernel built from it rounds the same way: the two-buffer and in-place steps
// give the same bits.
template <int D>
__device__ __forceinline__ float dot_fma(const float *a, const float *b)
{
#pragma clang fp contract(off)
    float r = __builtin_fmaf(a[1], b[1], a[0] * b[0]);
    if constexpr (D == 3) r = __builtin_fmaf(a[2], b[2], r);
    return r;
}

// w = a x b
__device__ __forceinline__ void cross_fma(const float *a, const float *b, float *w)
{
#pragma clang fp contract(off)
    w[0] = __builtin_fmaf(a[1], b[2], -(a[2] * b[1]));
    w[1] = __builtin_fmaf(a[2], b[0], -(a[0] * b[2]));
    w[2] = __builtin_fmaf(a[0], b[1], -(a[1] * b[0]));
}

template <int LAT>
struct Macro {
    float drho, rho, j[3], U[3], U2;
};

// Zeroth and first moments of the deviations: r = sum_q d_q, j = sum_q d_q e_q.
template <int LAT>
__device__ __forceinline__ void moment_sums(const float *d, float &r, float (&j)[3])
{
#pragma clang fp contract(off)
    using L = Lat<LAT>;
    r = d[0];
#pragma unroll
    for (int q = 1; q < L::Q; ++q) r += d[q];
    j[0] = j[1] = j[2] = 0.f;
    bool fx = true, fy = true, fz = true;
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
        if (L::ex[q]) {
            const float t = L::ex[q] > 0 ? d[q] : -d[q];
            j[0] = fx ? t : j[0] + t;
            fx = false;
        }
        if (L::ey[q]) {
            const float t = L::ey[q] > 0 ? d[q] : -d[q];
            j[1] = fy ? t : j[1] + t;
            fy = false;
        }
        if (L::ez[q]) {
            const float t = L::ez[q] > 0 ? d[q] : -d[q];
            j[2] = fz ? t : j[2] + t;
            fz = false;
        }
    }
}

template <int LAT>
__device__ __forceinline__ Macro<LAT> macro(const Physics &p, const float *d)
{
#pragma clang fp contract(off)
    using L = Lat<LAT>;
    Macro<LAT> m;
    float r, j[3];
    moment_sums<LAT>(d, r, j);
    m.drho = r;
    m.rho = p.rho0 + r;
    const float k = p.inv_cs2 * __builtin_amdgcn_rcpf(m.rho);
    m.j[0] = j[0];
    m.j[1] = j[1];
    m.j[2] = j[2];
    m.U[0] = j[0] * k;
    m.U[1] = j[1] * k;
    m.U[2] = L::D == 3 ? j[2] * k : 0.f;
    m.U2 = dot_fma<L::D>(m.U, m.U);
    return m;
}

// Forward collision of one node in stored units (deviations times the storage scale S):
// BGK relaxation toward the reduced equilibrium plus the Lorentz source, with omega and S
// folded into per-shell constants,
//   o_q = (1 - omega) D_q + omega S deq_q + S w_q rho sigma_q
//       = c0 D_q + ol_k (e_q.j) + owhat_k drho + whatS_k rho [omega Bc (e_q.U)^2
//         + omega Cp_k U^2 + sigma_q],
// sigma_q = (e_q.c1v) + c2q (e_q.U) + C2_k c_s (U.E) + C2_k e_q.(U x B). The rest population
// follows from mass closure (relaxation and source conserve mass), o_0 = sum_q D_q -
// sum_{q>0} o_q, which also keeps FP32 mass conservation exact up to one rounding per node.
template <int LAT, int FORCE>
__device__ __forceinline__ void relax_node(const Physics &p, const float *D, float *o)
{
#pragma clang fp contract(off)
    using L = Lat<LAT>;
    float drho, j[3];  // stored units
    moment_sums<LAT>(D, drho, j);
    const float rho = __builtin_fmaf(drho, p.inv_scale, p.rho0);
    const float kk = p.inv_cs2S * __builtin_amdgcn_rcpf(rho);
    float U[3] = {j[0] * kk, j[1] * kk, L::D == 3 ? j[2] * kk : 0.f};
    if constexpr (FORCE == 3) {
        // velocity shift: the equilibrium takes u + tau (E + u x B), i.e. j + rho (shE +
        // shB U x B); the relaxation then moves momentum by rho (E + u x B) per step
        float W[3];
        cross_fma(U, p.B, W);  // U x B
#pragma unroll
        for (int i = 0; i < L::D; ++i) {
            j[i] = __builtin_fmaf(rho, __builtin_fmaf(p.shB, W[i], p.shE[i]), j[i]);
            U[i] = j[i] * kk;
        }
    }
    const float U2 = dot_fma<L::D>(U, U);
    float wr[3], owd[3], P[3];
#pragma unroll
    for (int k = 1; k < 3; ++k) {
        wr[k] = p.whatS[k] * rho;
        owd[k] = p.owhat[k] * drho;
        P[k] = p.oCp[k] * U2;
    }
    float H[3][3];
    if constexpr (FORCE == 1 || FORCE == 2) {
        const float UE = dot_fma<L::D>(U, p.E) * p.cs;
#pragma unroll
        for (int k = 1; k < 3; ++k) P[k] = __builtin_fmaf(p.C2[k], UE, P[k]);
    }
    if constexpr (FORCE == 2) {
        float W[3];
        cross_fma(p.B, U, W);  // B x U
#pragma unroll
        for (int k = 1; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < 3; ++i) H[k][i] = __builtin_fmaf(p.C2[k], W[i], p.c1v[i]);
    }
    float sum = 0.f;
    for_q<L::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (q != 0) {
            constexpr int k = shell<LAT, q>();
            const float eu = edot<LAT, q>(U);
            const float ej = edot<LAT, q>(j);
            float inner;
            if constexpr (FORCE == 0 || FORCE == 3)
                inner = __builtin_fmaf(p.omBc * eu, eu, P[k]);
            else if constexpr (FORCE == 1)
                inner = __builtin_fmaf(__builtin_fmaf(p.omBc, eu, p.c2q[q]), eu, P[k] + p.c1q[q]);
            else
                inner = __builtin_fmaf(__builtin_fmaf(p.omBc, eu, p.c2q[q]), eu, P[k] + edot<LAT, q>(H[k]));
            const float v = __builtin_fmaf(wr[k], inner,
                                           __builtin_fmaf(p.ol[k], ej, __builtin_fmaf(p.c0, D[q], owd[k])));
            o[q] = v;
            sum = (q == 1) ? v : sum + v;
        }
    });
    o[0] = drho - sum;
}

template <int LAT, bool SOFT, int FORCE>
__device__ __forceinline__ void collide(const Physics &p, const float *D, float s, float *o)
{
#pragma clang fp contract(off)
    using L = Lat<LAT>;
    relax_node<LAT, FORCE>(p, D, o);
    if (SOFT) {
        float t[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) t[q] = __builtin_fmaf(s, D[L::opp[q]] - o[q], o[q]);
#pragma unroll
        for (int q = 0; q < L::Q; ++q) o[q] = t[q];
    }
}


// Store the post-collision deviations o of the fluid nodes of tile t at their own nodes
// (slot q of x), and with the solid-slot convention each bounced one where the next pull
// reads it: where x - e_q is solid, the value pulled into x as population q is
// f*_qbar(x), kept in slot q of that solid node. With the own-slot convention solid nodes
// beside fluid ones in the wave store their own slots too (read by no pull).
// With SR the codes are rounded stochastically with the node hashes h (sr_node).
// NT_BOUNCED: the bounced copies are non-temporal stores (the in-place local phase; in the
// two-buffer step they measured slower: 2048^2 disks +3 %, the paper's 3D Ohm sample +8 %).
template <int LAT, int ST, bool MASK, int V, bool SR = false, bool NT_BOUNCED = false>
__device__ __forceinline__ void store_tile(const Geometry &g, typename Codec<ST>::T *__restrict__ dst, const Tile &t,
                                           const typename LinkMask<LAT>::T (&lk)[V], const float (&o)[V][Lat<LAT>::Q],
                                           const uint32_t *h = nullptr)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    bool fluid[V];
    bool all_fluid = true;
    LT links = 0;  // union of the solid-neighbour bits of the fluid nodes
#pragma unroll
    for (int i = 0; i < V; ++i) {
        fluid[i] = !MASK || !(lk[i] & LinkMask<LAT>::solid);
        all_fluid = all_fluid && fluid[i];
        if (MASK && fluid[i]) links |= lk[i];
    }
    if constexpr (MASK && !kSolidSlotBB<ST>) {
        // Own-slot convention: no pull reads a solid node's slots, so in a wave that holds a
        // fluid node the solid lanes store their (unused) values too, and every store of the
        // wave covers whole lines instead of leaving gaps at the obstacles; a wave of solid
        // nodes only stores nothing. Measured on MI355X: FP32 2048^2 disks +5 %, in place
        // +19 %; the paper's 3D Ohm sample +3 % / +5 %; the duct's wall rows unchanged.
        bool any = false;
#pragma unroll
        for (int i = 0; i < V; ++i) any = any || fluid[i];
        if (__builtin_amdgcn_ballot_w64(any) == 0) return;
        all_fluid = true;
    }
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        T *p = at32(dst + slot_off(q, g.stride), (unsigned)t.own);
        if (!MASK || all_fluid) {
            float f[V];
#pragma unroll
            for (int i = 0; i < V; ++i) f[i] = o[i][q];
            vstore_q<ST, V, SR>(p, f, h, q);
        } else {
#pragma unroll
            for (int i = 0; i < V; ++i)
                if (fluid[i]) *at32(p, (unsigned)i) = enc_store<ST, SR>(o[i][q], SR ? h[i] : 0u, q);
        }
    }
    if (MASK && kSolidSlotBB<ST> && links) {
        const PullRows r = pull_rows<V>(g, t);
        for_q<L::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (q != 0) {
                T *row = dst + pull_row<LAT, q>(g, t, r);
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (fluid[i] && ((lk[i] >> q) & 1u)) {
                        const T c = enc_store<ST, SR>(o[i][L::opp[q]], SR ? h[i] : 0u, L::opp[q]);
                        if constexpr (NT_BOUNCED)
                            __builtin_nontemporal_store(c, at32(row, pull_x<LAT, q, V>(r, i)));
                        else
                            *at32(row, pull_x<LAT, q, V>(r, i)) = c;
                    }
            }
        });
    }
}

}  // namespace lbm
