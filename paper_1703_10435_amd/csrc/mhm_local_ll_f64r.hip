// FP64 instances of the left-looking kernel that carry the refinement step
// (panel width 2, 8 waves, one workgroup per CU, fused: from kappa): the
// FP64 pass after a launch, over the elements whose plain FP64 solve is not
// accurate enough (deferred by the other FP64 instances and the
// register-tile kernel) or whose FP32 refinement did not converge.
#include "mhm_local_ll.h"

namespace mhm {

template <bool FUSED>
static hipError_t launch_ref(int rpw, const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  switch (rpw) {
    case 2: return launch_ll_t<double, FUSED, 2, 2, 1, 8, false, true>(d, a, lds, grid, st);
    case 3: return launch_ll_t<double, FUSED, 2, 3, 1, 8, false, true>(d, a, lds, grid, st);
    case 5: return launch_ll_t<double, FUSED, 2, 5, 1, 8, false, true>(d, a, lds, grid, st);
    case 10: return launch_ll_t<double, FUSED, 2, 10, 1, 8, false, true>(d, a, lds, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_local_ll_f64_ref(bool fused, int pw, int occ, int nw, int rpw, const BatchDev& d, LocalArgs a,
                                   size_t lds, int grid, hipStream_t st) {
  if (!fused || pw != 2 || occ != 1 || nw != 8) return hipErrorInvalidValue;
  return launch_ref<true>(rpw, d, a, lds, grid, st);
}

}  // namespace mhm
