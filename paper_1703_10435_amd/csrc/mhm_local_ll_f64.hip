// FP64 instances of the left-looking kernel (panel width 2; width 4 for up to
// 24 tile rows, where the register panel still fits, and for the largest
// elements in row passes; width 2 with two resident workgroups per CU for up
// to 24 tile rows; width 1 and 16 waves per element for the largest
// elements).
#include "mhm_local_ll.h"

namespace mhm {

template <bool FUSED>
static hipError_t launch_rpw2(int rpw, const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  switch (rpw) {
    case 2: return launch_ll_t<double, FUSED, 2, 2, 1>(d, a, lds, grid, st);
    case 3: return launch_ll_t<double, FUSED, 2, 3, 1>(d, a, lds, grid, st);
    case 5: return launch_ll_t<double, FUSED, 2, 5, 1>(d, a, lds, grid, st);
    case 10: return launch_ll_t<double, FUSED, 2, 10, 1>(d, a, lds, grid, st);
    default: return hipErrorInvalidValue;
  }
}
template <bool FUSED>
static hipError_t launch_rpw4(int rpw, const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  switch (rpw) {
    case 2: return launch_ll_t<double, FUSED, 4, 2, 1>(d, a, lds, grid, st);
    case 3: return launch_ll_t<double, FUSED, 4, 3, 1>(d, a, lds, grid, st);
    case 10: return launch_ll_t<double, FUSED, 4, 10, 1>(d, a, lds, grid, st);
    default: return hipErrorInvalidValue;
  }
}
template <bool FUSED>
static hipError_t launch_occ2(int rpw, const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  switch (rpw) {
    case 2: return launch_ll_t<double, FUSED, 2, 2, 2>(d, a, lds, grid, st);
    case 3: return launch_ll_t<double, FUSED, 2, 3, 2>(d, a, lds, grid, st);
    default: return hipErrorInvalidValue;
  }
}

// More than 16 right-hand sides (chunked): panel width 2, 8 waves, one
// workgroup per CU.
template <bool FUSED>
static hipError_t launch_mc(int rpw, const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  switch (rpw) {
    case 2: return launch_ll_t<double, FUSED, 2, 2, 1, 8, true>(d, a, lds, grid, st);
    case 3: return launch_ll_t<double, FUSED, 2, 3, 1, 8, true>(d, a, lds, grid, st);
    case 5: return launch_ll_t<double, FUSED, 2, 5, 1, 8, true>(d, a, lds, grid, st);
    case 10: return launch_ll_t<double, FUSED, 2, 10, 1, 8, true>(d, a, lds, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_local_ll_f64(bool fused, int pw, int occ, int nw, int rpw, bool mc, const BatchDev& d,
                               LocalArgs a, size_t lds, int grid, hipStream_t st) {
  if (mc) {
    if (pw != 2 || occ != 1 || nw != 8) return hipErrorInvalidValue;
    return fused ? launch_mc<true>(rpw, d, a, lds, grid, st) : launch_mc<false>(rpw, d, a, lds, grid, st);
  }
  if (nw == 16) {
    if (rpw != 5 || occ != 1) return hipErrorInvalidValue;
    if (pw == 1) return fused ? launch_ll_t<double, true, 1, 5, 1, 16>(d, a, lds, grid, st)
                              : launch_ll_t<double, false, 1, 5, 1, 16>(d, a, lds, grid, st);
    if (pw != 2) return hipErrorInvalidValue;
    return fused ? launch_ll_t<double, true, 2, 5, 1, 16>(d, a, lds, grid, st)
                 : launch_ll_t<double, false, 2, 5, 1, 16>(d, a, lds, grid, st);
  }
  if (pw == 1) {   // one tile column per panel: half the accumulator registers (the largest elements)
    if (rpw != 10 || occ != 1) return hipErrorInvalidValue;
    return fused ? launch_ll_t<double, true, 1, 10, 1>(d, a, lds, grid, st)
                 : launch_ll_t<double, false, 1, 10, 1>(d, a, lds, grid, st);
  }
  if (occ == 2) {
    if (pw != 2) return hipErrorInvalidValue;
    return fused ? launch_occ2<true>(rpw, d, a, lds, grid, st) : launch_occ2<false>(rpw, d, a, lds, grid, st);
  }
  if (pw == 2) return fused ? launch_rpw2<true>(rpw, d, a, lds, grid, st) : launch_rpw2<false>(rpw, d, a, lds, grid, st);
  if (pw == 4) return fused ? launch_rpw4<true>(rpw, d, a, lds, grid, st) : launch_rpw4<false>(rpw, d, a, lds, grid, st);
  return hipErrorInvalidValue;
}

}  // namespace mhm
