// lbm_step_sr.hip -- the two-buffer step with stochastic rounding of the stored 16-bit
// values (the kernel of lbm_step_kernels.h, SR instances; FP16 and BF16 storage only).
#include "lbm_step_kernels.h"

namespace lbm {

hipError_t launch_step_sr(int lattice, int storage, int force, const StepArgs &a, hipStream_t st)
{
    if (!a.sr) return hipErrorInvalidValue;
    if (lattice == LBM_D2V9) {
        if (storage == LBM_F16) return step_lat_st<LBM_D2V9, LBM_F16, true>(force, a, st);
        if (storage == LBM_BF16) return step_lat_st<LBM_D2V9, LBM_BF16, true>(force, a, st);
    } else if (lattice == LBM_D3V19) {
        if (storage == LBM_F16) return step_lat_st<LBM_D3V19, LBM_F16, true>(force, a, st);
        if (storage == LBM_BF16) return step_lat_st<LBM_D3V19, LBM_BF16, true>(force, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
