// The two-label semi-global aggregation kernel for FMVS_KP label pairs per
// lane (all its variants), one translation unit per KP.
#include "k_sgm.hpp"

#if !defined(FMVS_KP)
#error "k_sgm_inst.hip needs FMVS_KP"
#endif

namespace fmvs {
template void sgm_launch_pk<FMVS_KP>(const SgmArgs &, bool, bool, dim3, hipStream_t);
template hipError_t sgm_launch_pk_jobs<FMVS_KP>(const SgmArgs *, const int *, int, unsigned *, bool, bool, int, int,
                                                hipStream_t);
}  // namespace fmvs
