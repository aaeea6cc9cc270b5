// lbm_aa.hip -- the in-place time step (AA access pattern; the kernels and their
// description are in lbm_aa_kernels.h): round-to-nearest instances, the conversion of an
// odd-layout state to the two-buffer layout, and the launchers.
#include "lbm_aa_kernels.h"

namespace lbm {
namespace {

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

template <int LAT, int ST>
hipError_t aa_nearest(int force, int phase, const StepArgs &a, hipStream_t st)
{
    return aa_lat_st<LAT, ST, false>(force, phase, a, st);
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
    if (a.sr) return launch_step_aa_sr(lattice, storage, force, phase, a, st);
    LBM_AA_DISPATCH(aa_nearest, force, phase, a, st);
}

hipError_t launch_canon(int lattice, int storage, const StepArgs &a, hipStream_t st)
{
    if (a.src == a.dst) return hipErrorInvalidValue;
    LBM_AA_DISPATCH(canon_lat_st, a, st);
}

}  // namespace lbm
