// FP32 instances of the left-looking kernel (panel widths 2 and 4; panel
// width 2 also with two resident workgroups per CU; 16 waves per element
// for the largest elements).
#include "mhm_local_ll.h"

namespace mhm {

template <bool FUSED, int PW, int OCC>
static hipError_t launch_rpw(int rpw, const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  switch (rpw) {
    case 2: return launch_ll_t<float, FUSED, PW, 2, OCC>(d, a, lds, grid, st);
    case 3: return launch_ll_t<float, FUSED, PW, 3, OCC>(d, a, lds, grid, st);
    case 5: return launch_ll_t<float, FUSED, PW, 5, OCC>(d, a, lds, grid, st);
    case 10: return launch_ll_t<float, FUSED, PW, 10, OCC>(d, a, lds, grid, st);
    default: return hipErrorInvalidValue;
  }
}

// More than 16 right-hand sides (chunked): panel width 2, 8 waves, one
// workgroup per CU.
template <bool FUSED>
static hipError_t launch_mc(int rpw, const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  switch (rpw) {
    case 2: return launch_ll_t<float, FUSED, 2, 2, 1, 8, true>(d, a, lds, grid, st);
    case 3: return launch_ll_t<float, FUSED, 2, 3, 1, 8, true>(d, a, lds, grid, st);
    case 5: return launch_ll_t<float, FUSED, 2, 5, 1, 8, true>(d, a, lds, grid, st);
    case 10: return launch_ll_t<float, FUSED, 2, 10, 1, 8, true>(d, a, lds, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_local_ll_f32(bool fused, int pw, int occ, int nw, int rpw, bool mc, const BatchDev& d,
                               LocalArgs a, size_t lds, int grid, hipStream_t st) {
  if (mc) {
    if (pw != 2 || occ != 1 || nw != 8) return hipErrorInvalidValue;
    return fused ? launch_mc<true>(rpw, d, a, lds, grid, st) : launch_mc<false>(rpw, d, a, lds, grid, st);
  }
  if (nw == 16) {
    if (rpw != 5 || occ != 1) return hipErrorInvalidValue;
    if (pw == 2) return fused ? launch_ll_t<float, true, 2, 5, 1, 16>(d, a, lds, grid, st)
                              : launch_ll_t<float, false, 2, 5, 1, 16>(d, a, lds, grid, st);
    if (pw == 4) return fused ? launch_ll_t<float, true, 4, 5, 1, 16>(d, a, lds, grid, st)
                              : launch_ll_t<float, false, 4, 5, 1, 16>(d, a, lds, grid, st);
    return hipErrorInvalidValue;
  }
  if (occ == 2) {
    if (pw != 2) return hipErrorInvalidValue;
    return fused ? launch_rpw<true, 2, 2>(rpw, d, a, lds, grid, st) : launch_rpw<false, 2, 2>(rpw, d, a, lds, grid, st);
  }
  if (pw == 4) return fused ? launch_rpw<true, 4, 1>(rpw, d, a, lds, grid, st) : launch_rpw<false, 4, 1>(rpw, d, a, lds, grid, st);
  if (pw == 2) return fused ? launch_rpw<true, 2, 1>(rpw, d, a, lds, grid, st) : launch_rpw<false, 2, 1>(rpw, d, a, lds, grid, st);
  return hipErrorInvalidValue;
}

}  // namespace mhm
