// One (window, cost) variant of the fused plane-sweep kernel, chosen at
// compile time by FMVS_CW, FMVS_CH and FMVS_COST (0 census, 1 NCC).
#include "k_sweep.hpp"

#if !defined(FMVS_CW) || !defined(FMVS_CH) || !defined(FMVS_COST)
#error "k_sweep_inst.hip needs FMVS_CW, FMVS_CH and FMVS_COST"
#endif

namespace fmvs {
template hipError_t sweep_launch_cfg<FMVS_CW, FMVS_CH, FMVS_COST>(const SweepArgs &, dim3, int, hipStream_t);
template hipError_t sweep_launch_batch_cfg<FMVS_CW, FMVS_CH, FMVS_COST>(const SweepArgs *, const int *, int, int,
                                                                        int, hipStream_t);
}  // namespace fmvs
