// lbm_aa_sr.hip -- the in-place step with stochastic rounding of the stored 16-bit
// values (the kernels of lbm_aa_kernels.h, SR instances; FP16 and BF16 storage only).
#include "lbm_aa_kernels.h"

namespace lbm {

hipError_t launch_step_aa_sr(int lattice, int storage, int force, int phase, const StepArgs &a, hipStream_t st)
{
    if (!a.sr || a.src != a.dst || (phase != 0 && phase != 1)) return hipErrorInvalidValue;
    if (lattice == LBM_D2V9) {
        if (storage == LBM_F16) return aa_lat_st<LBM_D2V9, LBM_F16, true>(force, phase, a, st);
        if (storage == LBM_BF16) return aa_lat_st<LBM_D2V9, LBM_BF16, true>(force, phase, a, st);
    } else if (lattice == LBM_D3V19) {
        if (storage == LBM_F16) return aa_lat_st<LBM_D3V19, LBM_F16, true>(force, phase, a, st);
        if (storage == LBM_BF16) return aa_lat_st<LBM_D3V19, LBM_BF16, true>(force, phase, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
