// Left-looking local-problem kernel: launch geometry and precision dispatch
// (the kernel is in mhm_local_ll.h, its instances in mhm_local_ll_f32.hip and
// mhm_local_ll_f64.hip).
#include "mhm_local_ll.h"

namespace mhm {

hipError_t launch_local_ll_f32(bool fused, int pw, int occ, int nw, int rpw, bool mc, const BatchDev& d,
                               LocalArgs a, size_t lds, int grid, hipStream_t st);
hipError_t launch_local_ll_f64(bool fused, int pw, int occ, int nw, int rpw, bool mc, const BatchDev& d,
                               LocalArgs a, size_t lds, int grid, hipStream_t st);
hipError_t launch_local_ll_f64_ref(bool fused, int pw, int occ, int nw, int rpw, const BatchDev& d, LocalArgs a,
                                   size_t lds, int grid, hipStream_t st);

int local_ll_rows_per_wave(int nt, int nw) {
  const int rows = nt + 1;
  if (rows <= 2 * nw) return 2;
  if (rows <= 3 * nw) return 3;
  if (rows <= 5 * nw) return 5;
  if (rows <= 10 * nw && nw == 8) return 10;
  return -1;
}

// FP32: width 4.  FP64: width 2, and 4 for the elements of five or ten rows
// per wave (on the ten-row instance, in passes of two rows): every earlier
// tile column is then read once per four panel columns instead of two, which
// halves the factor traffic that bounds these elements (C4's s = 48 class,
// 2048 elements: 38 ms against 50 ms with two-tile panels; its s = 32 class
// 6.0 against 6.6 ms).
int local_ll_default_panel(bool fp32, int nt) {
  if (fp32) return 4;
  const int rpw = local_ll_rows_per_wave(nt, 8);
  return rpw == 10 || rpw == 5 ? 4 : 2;
}

// Rows per wave of the instance a launch takes: the fewest that hold the
// class's tile rows, except that FP64 four-tile panels for five rows per wave
// run on the ten-row instance (its row passes past the last row are skipped),
// since a five-row FP64 instance would hold all its rows' panel accumulators
// at once and spill.
static int local_ll_launch_rows(bool fp32, int pw, int occ, int nw, bool mc, bool ref, int nt) {
  const int rpw = local_ll_rows_per_wave(nt, nw);
  if (!fp32 && !mc && !ref && pw == 4 && occ == 1 && nw == 8 && rpw == 5) return 10;
  return rpw;
}

bool local_ll_has(bool fp32, int pw, int nt, int occ, int nw, bool mc) {
  if (mc)   // chunked right-hand sides: panel width 2, 8 waves, one workgroup per CU
    return pw == 2 && occ == 1 && nw == 8 && local_ll_rows_per_wave(nt, 8) > 0;
  if (nw == 16)   // built for the largest elements only (49 to 80 tile rows)
    return occ == 1 && nt + 1 > 48 && local_ll_rows_per_wave(nt, 16) == 5 &&
           (pw == 2 || (fp32 && pw == 4) || (!fp32 && pw == 1));
  if (nw != 8) return false;
  const int rpw = local_ll_rows_per_wave(nt, 8);
  if (rpw < 0) return false;
  if (occ == 2) return pw == 2 && (fp32 || rpw <= 3);
  if (occ != 1) return false;
  if (fp32) return pw == 2 || pw == 4;
  return pw == 2 || (pw == 4 && (rpw <= 3 || rpw >= 5)) || (pw == 1 && rpw == 10);
}

size_t local_ll_lds_bytes(bool fp32, int pw, int n_cap, int f_cap, int nw) {
  return sizeof(double) * (2 * (size_t)n_cap + (size_t)f_cap) +
         (size_t)(2 + pw + pw * pw + nw) * TILE * (fp32 ? sizeof(float) : sizeof(double));
}

hipError_t launch_local_ll(bool fp32, bool fused, int pw, int occ, int nw, bool mc, bool ref, int nt_max,
                           const mhm_batch* bt, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  if (!local_ll_has(fp32, pw, nt_max, occ, nw, mc)) return hipErrorInvalidValue;
  // an FP64 pass over deferred or recomputed elements must refine, never defer again
  if (!fp32 && !mc && a.only_fallback && !ref) return hipErrorInvalidValue;
  const int rpw = local_ll_launch_rows(fp32, pw, occ, nw, mc, ref, nt_max);
  const BatchDev d = to_dev(bt);
  if (fp32) return launch_local_ll_f32(fused, pw, occ, nw, rpw, mc, d, a, lds, grid, st);
  if (ref && !mc) return launch_local_ll_f64_ref(fused, pw, occ, nw, rpw, d, a, lds, grid, st);
  return launch_local_ll_f64(fused, pw, occ, nw, rpw, mc, d, a, lds, grid, st);   // chunked instances refine
}

}  // namespace mhm
