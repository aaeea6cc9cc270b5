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
#include "lbm_internal.h"

#include <cstdlib>
#include <type_traits>

#ifndef LBM_NT_STORE
#define LBM_NT_STORE 1
#endif

namespace lbm {

static int env_int(const char *name, int dflt)
{
    const char *e = std::getenv(name);
    return e ? std::atoi(e) : dflt;
}

// Nodes per thread of the step kernel (measured on MI355X): 1 for FP32 and for D3V19,
// 2 for 16-bit D2V9; halved until it divides nx. LBM_STEP_VEC=1|2 overrides it.
int step_vector_width(int lattice, int storage, int nx)
{
    static const int forced = env_int("LBM_STEP_VEC", 0);
    int v = forced;
    if (v != 1 && v != 2) v = (storage != LBM_F32 && lattice == LBM_D2V9) ? 2 : 1;
    while (v > 1 && nx % v) v >>= 1;
    return v;
}

// XCD-contiguous block order (measured on MI355X): it pays off where the reads of a node
// span several rows of solids or planes (D3V19, masks, porosity fields) and costs ~8 %
// on the plain D2V9 grid, which keeps the hardware order. LBM_XCD_REMAP=0|1 overrides.
int use_xcd_remap(int lattice, bool mask, bool soft)
{
    static const int forced = env_int("LBM_XCD_REMAP", -1);
    if (forced == 0 || forced == 1) return forced;
    return (lattice == LBM_D3V19 || mask || soft) ? 1 : 0;
}

namespace {

// ---------------------------------------------------------------------------------
// Storage codecs: deviation <-> stored value (round to nearest even).
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
    // stored value = d * 2^k; the scale is a power of two, so scaling is exact
    static __device__ __forceinline__ float dec(T v, float inv_scale) { return (float)v * inv_scale; }
    static __device__ __forceinline__ T enc(float f, float scale) { return (T)(f * scale); }
};

template <>
struct Codec<LBM_BF16> {
    using T = __bf16;
    static __device__ __forceinline__ float dec(T v, float) { return (float)v; }
    static __device__ __forceinline__ T enc(float f, float) { return (T)f; }
};

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
// populations of one-node tiles and the edge values of V-wide tiles are loaded through
// the cache instead (gather_tile): their lines straddle the neighbouring tile's.
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

template <int ST, int V>
__device__ __forceinline__ void vstore(typename Codec<ST>::T *p, float scale, const float *f)
{
    if constexpr (V == 1) {
        const typename Codec<ST>::T v = Codec<ST>::enc(f[0], scale);
#if LBM_NT_STORE
        __builtin_nontemporal_store(v, p);
#else
        *p = v;
#endif
    } else {
        using VT = typename VecT<ST, V>::type;
        VT v;
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = Codec<ST>::enc(f[i], scale);
#if LBM_NT_STORE
        __builtin_nontemporal_store(v, reinterpret_cast<VT *>(p));
#else
        *reinterpret_cast<VT *>(p) = v;
#endif
    }
}

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
    return (size_t)p * g.stride + (size_t)g.nx * (sy + g.ny * sz);
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
                        d[i][q] = Codec<ST>::dec(*at32(src + (size_t)L::opp[q] * g.stride, own + i), inv_scale);
            }
        }
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
template <int LAT>
struct Macro {
    float drho, rho, j[3], U[3], U2;
};

// Zeroth and first moments of the deviations: r = sum_q d_q, j = sum_q d_q e_q.
template <int LAT>
__device__ __forceinline__ void moment_sums(const float *d, float &r, float (&j)[3])
{
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
    if constexpr (L::D == 3) {
        m.U[2] = j[2] * k;
        m.U2 = m.U[0] * m.U[0] + m.U[1] * m.U[1] + m.U[2] * m.U[2];
    } else {
        m.U[2] = 0.f;
        m.U2 = m.U[0] * m.U[0] + m.U[1] * m.U[1];
    }
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
    using L = Lat<LAT>;
    float drho, j[3];  // stored units
    moment_sums<LAT>(D, drho, j);
    const float rho = __builtin_fmaf(drho, p.inv_scale, p.rho0);
    const float kk = p.inv_cs2S * __builtin_amdgcn_rcpf(rho);
    float U[3] = {j[0] * kk, j[1] * kk, L::D == 3 ? j[2] * kk : 0.f};
    if constexpr (FORCE == 3) {
        // velocity shift: the equilibrium takes u + tau (E + u x B), i.e. j + rho (shE +
        // shB U x B); the relaxation then moves momentum by rho (E + u x B) per step
        const float W[3] = {U[1] * p.B[2] - U[2] * p.B[1], U[2] * p.B[0] - U[0] * p.B[2],
                            U[0] * p.B[1] - U[1] * p.B[0]};  // U x B
#pragma unroll
        for (int i = 0; i < L::D; ++i) {
            j[i] = __builtin_fmaf(rho, __builtin_fmaf(p.shB, W[i], p.shE[i]), j[i]);
            U[i] = j[i] * kk;
        }
    }
    float U2 = U[0] * U[0] + U[1] * U[1];
    if constexpr (L::D == 3) U2 = __builtin_fmaf(U[2], U[2], U2);
    float wr[3], owd[3], P[3];
#pragma unroll
    for (int k = 1; k < 3; ++k) {
        wr[k] = p.whatS[k] * rho;
        owd[k] = p.owhat[k] * drho;
        P[k] = p.oCp[k] * U2;
    }
    float H[3][3];
    if constexpr (FORCE == 1 || FORCE == 2) {
        float UE = U[0] * p.E[0] + U[1] * p.E[1];
        if constexpr (L::D == 3) UE = __builtin_fmaf(U[2], p.E[2], UE);
        UE *= p.cs;
#pragma unroll
        for (int k = 1; k < 3; ++k) P[k] = __builtin_fmaf(p.C2[k], UE, P[k]);
    }
    if constexpr (FORCE == 2) {
        const float W[3] = {p.B[1] * U[2] - p.B[2] * U[1], p.B[2] * U[0] - p.B[0] * U[2],
                            p.B[0] * U[1] - p.B[1] * U[0]};
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

// ---------------------------------------------------------------------------------
// K1: fused pull-stream + collide + force + partial bounce-back.
// ---------------------------------------------------------------------------------
template <int LAT, int ST, bool MASK, bool SOFT, int FORCE, int V>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs a, int ntx, FastDiv div_ntx, int nblocks)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    const int bid = a.remap ? xcd_remap((int)blockIdx.x, nblocks) : (int)blockIdx.x;
    const Tile t = tile_of<V>(a.g, bid, ntx, div_ntx);
    if (!t.valid) return;  // beyond the row (rows shorter than a block): no work
    LT lk[V];
    if (MASK) {
        load_links<LAT, V>(static_cast<const LT *>(a.links), t.own, lk);
        bool any_fluid = false;
#pragma unroll
        for (int i = 0; i < V; ++i) any_fluid = any_fluid || !(lk[i] & LinkMask<LAT>::solid);
        if (!any_fluid) return;
    }
    float d[V][L::Q];
    gather_tile<LAT, ST, MASK, V>(a.g, static_cast<const T *>(a.src), 1.f, t, lk, d);  // stored units throughout
    float sv[V];
    if (SOFT) vload<LBM_F32, V>(at32(a.g.s, (unsigned)t.own), 1.f, sv);
    float o[V][L::Q];
#pragma unroll
    for (int i = 0; i < V; ++i) collide<LAT, SOFT, FORCE>(a.ph, d[i], SOFT ? sv[i] : 0.f, o[i]);
    bool fluid[V];
    bool all_fluid = true;
    LT links = 0;  // union of the solid-neighbour bits of the fluid nodes
#pragma unroll
    for (int i = 0; i < V; ++i) {
        fluid[i] = !MASK || !(lk[i] & LinkMask<LAT>::solid);
        all_fluid = all_fluid && fluid[i];
        if (MASK && fluid[i]) links |= lk[i];
    }
    T *__restrict__ dst = static_cast<T *>(a.dst);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        T *p = at32(dst + (size_t)q * a.g.stride, (unsigned)t.own);
        if (!MASK || all_fluid) {
            float f[V];
#pragma unroll
            for (int i = 0; i < V; ++i) f[i] = o[i][q];
            vstore<ST, V>(p, 1.f, f);
        } else {
#pragma unroll
            for (int i = 0; i < V; ++i)
                if (fluid[i]) *at32(p, (unsigned)i) = Codec<ST>::enc(o[i][q], 1.f);
        }
    }
    if (MASK && kSolidSlotBB<ST> && links) {
        // solid-slot bounce-back: where x - e_q is solid, the value the next step pulls
        // into x as population q is f*_qbar(x); store it in slot q of that solid node
        const PullRows r = pull_rows<V>(a.g, t);
        for_q<L::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (q != 0) {
                T *row = dst + pull_row<LAT, q>(a.g, t, r);
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (fluid[i] && ((lk[i] >> q) & 1u))
                        *at32(row, pull_x<LAT, q, V>(r, i)) = Codec<ST>::enc(o[i][L::opp[q]], 1.f);
            }
        });
    }
}

// ---------------------------------------------------------------------------------
// Link masks: the top bit when x is solid (an obstacle of the mask or a node of a
// free-slip wall plane); bit q when the pull of population q into x bounces back, i.e.
// its source x - e_q is an obstacle or, where x - e_q lies in a wall plane, the
// specular source (x - e_q with the wall-axis coordinates of x) is an obstacle.
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
    LT bits = own_solid ? LinkMask<LAT>::solid : (LT)0;
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
// (sum drho, sum d e_x, sum d e_y, sum d e_z, fluid nodes).
// ---------------------------------------------------------------------------------
template <int LAT, int ST, bool MASK, int MODE>
__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs a)
{
    using L = Lat<LAT>;
    using T = typename Codec<ST>::T;
    using LT = typename LinkMask<LAT>::T;
    const T *src = static_cast<const T *>(a.src);
    const LT *links = static_cast<const LT *>(a.links);
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
            gather_tile<LAT, ST, MASK, 1>(a.g, src, a.ph.inv_scale, t, lk, d);
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
        if (!solid) gather_tile<LAT, ST, MASK, 1>(a.g, src, a.ph.inv_scale, t, lk, d);
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

// ---------------------------------------------------------------------------------
// K5: one reverse step of the discrete adjoint. lam_out = dJ/df(t) from
// lam_in = dJ/df(t+1); f(t) is pulled from the stored state as in K1.
//   gbar_a = lam_in(x + e_a, a), or lam_in(x, abar) if x + e_a is solid;
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
    const int bid = a.remap ? xcd_remap((int)blockIdx.x, g.nblocks) : (int)blockIdx.x;
    const Tile t = tile_of(g, bid);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // One partial per wave, written by its last lane. The accumulated value is read first
    // (a wave-uniform address: scalar registers), so its latency overlaps the pulls below.
    const bool last_lane = (threadIdx.x & 63) == 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    double *part = a.partials + ((size_t)blockIdx.x * (kBlock / 64) + wave) * 4;
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
    if (t.valid && solid) {
#pragma unroll
        for (int q = 0; q < L::Q; ++q) *at32(a.lam_out + (size_t)q * g.stride, (unsigned)t.own) = 0.f;
    } else if (t.valid) {
        float d[1][L::Q], gb[L::Q];
        gather_tile<LAT, ST, MASK, 1>(g, static_cast<const T *>(a.state), p.inv_scale, t, lk, d);
        {
            const int xm = wrapm(t.x0, g.nx), xp = wrapp(t.x0, g.nx);
            const int ym = wrapm(t.y, g.ny), yp = wrapp(t.y, g.ny);
            const int zm = wrapm(t.z, g.nz), zp = wrapp(t.z, g.nz);
#pragma unroll
            for (int q = 0; q < L::Q; ++q) {
                const unsigned tx = (unsigned)(L::ex[q] > 0 ? xp : (L::ex[q] < 0 ? xm : t.x0));
                const int ty = L::ey[q] > 0 ? yp : (L::ey[q] < 0 ? ym : t.y);
                const int tz = L::ez[q] > 0 ? zp : (L::ez[q] < 0 ? zm : t.z);
                const float *lq = a.lam_in + (size_t)q * g.stride;
                float v = *at32(lq + (size_t)g.nx * (ty + g.ny * tz), tx);
                // x + e_q solid <=> the pull of the opposite population at x bounces
                if (MASK && q != 0 && ((lk[0] >> L::opp[q]) & 1u))
                    v = *at32(a.lam_in + (size_t)L::opp[q] * g.stride, (unsigned)t.own);
                gb[q] = v;
            }
        }
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
            *at32(a.lam_out + (size_t)q * g.stride, (unsigned)t.own) = out;
        });
        if (SOFT && a.grad_s) *at32(a.grad_s, (unsigned)t.own) = gs_prev + ds;
        acc[0] = (double)m.rho * (double)dE[0];
        acc[1] = (double)m.rho * (double)dE[1];
        acc[2] = (double)m.rho * (double)dE[2];
        acc[3] = (double)(om * om) * (double)dtau;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = wave_sum_last_lane(acc[c]);
    if (last_lane)
        for (int c = 0; c < 4; ++c) part[c] = prev[c] + acc[c];
}

// Adjoint seed: lam(a, n) = e_a[axis] * value at fluid nodes (value = 1/(c_s norm)).
template <int LAT>
__global__ __launch_bounds__(kBlock) void k_seed(Geometry g, float value, int axis, float *lam)
{
    using L = Lat<LAT>;
    const Tile t = tile_of(g, (int)blockIdx.x);
    if (!t.valid) return;
    const bool solid = g.mask && g.mask[t.own];
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const int e = axis == 0 ? L::ex[q] : (axis == 1 ? L::ey[q] : L::ez[q]);
        lam[q * g.stride + t.own] = solid ? 0.f : (float)e * value;
    }
}

// ---------------------------------------------------------------------------------
// Launchers: runtime flags -> template instances.
// ---------------------------------------------------------------------------------
template <int LAT, int ST, int V>
hipError_t step_v(int force, const StepArgs &a, hipStream_t st)
{
    const bool mask = a.links != nullptr, soft = a.g.s != nullptr;
    const int ntx = (a.g.nx + kBlock * V - 1) / (kBlock * V);
    const int nblocks = ntx * a.g.ny * a.g.nz;
    const FastDiv div_ntx = make_fastdiv(ntx);
    const dim3 grid(nblocks), block(kBlock);
#define LBM_STEP(M, S, F) \
    hipLaunchKernelGGL((k_step<LAT, ST, M, S, F, V>), grid, block, 0, st, a, ntx, div_ntx, nblocks)
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
    return hipGetLastError();
}

template <int LAT, int ST>
hipError_t step_lat_st(int force, const StepArgs &a, hipStream_t st)
{
    const int v = step_vector_width(LAT, ST, a.g.nx);
    if (v == 2) return step_v<LAT, ST, 2>(force, a, st);
    return step_v<LAT, ST, 1>(force, a, st);
}

template <int LAT, int ST>
hipError_t adjoint_lat_st(bool mag, const AdjointArgs &a, hipStream_t st)
{
    const bool mask = a.links != nullptr, soft = a.g.s != nullptr;
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
    const bool mask = a.links != nullptr;
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
    LBM_DISPATCH(step_lat_st, force, a, st);
}

hipError_t launch_adjoint(int lattice, int storage, bool mag, const AdjointArgs &a, hipStream_t st)
{
    LBM_DISPATCH(adjoint_lat_st, mag, a, st);
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
