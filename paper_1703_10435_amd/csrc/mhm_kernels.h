// Internal interface between the C ABI (mhm_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mhm.h"

namespace mhm {

struct LocalArgs {
  const double* Ahat;   // load mode: assembled Ahat (column-major per element)
  const double* Btil;   // load mode: compatible right-hand sides
  double* Lout;         // factor output (may be null)
  double* X;            // solutions, n x r per element at rhs_off
  double* M;            // fused mode: contribution blocks (may be null)
  double* E;
  double* B;
  double* F;
  int32_t* info;
  int32_t* ir_iters;    // may be null
  int max_iters;
  int only_fallback;    // process only elements whose info is -1
  int fb_final;         // with only_fallback: a pass of an FP64 run (elements deferred by the
                        // register-tile kernel); a finished element's info becomes 0
  int refine64;         // FP64 refinement with a double-double residual: 0 where the element
                        // needs it (refine64_needed), 1 every element, -1 none
  double ir_tol;        // normwise backward-error target of the refinement
  void* ws;             // workspace mode: per-workgroup tile slots
  int64_t ws_slot;      // elements (of the tile type) per slot
  int tile_cap;         // tiles that fit in LDS or in one slot
  int n_cap;            // largest n (length of the LDS c and source-load arrays)
  int f_cap;            // LDS doubles of the face-load table, 3 (l_max+1)(s_max+1)
  int k_cap;            // LDS doubles reserved for kappa (fused, LDS mode)
  const int32_t* elist; // if set: process elements elist[0 .. *ecount) instead of 0 .. n_elem
  const int32_t* ecount;
  // factor store (left-looking kernel): element e's factor tiles at byte
  // offset fac_off[e] of fac; fac_state[e] 0 = factor and store, 1 = reuse
  void* fac;
  const int64_t* fac_off;
  const int8_t* fac_state;
};

// Time step on stored factors: the source column only.
struct SourceArgs {
  const void* fac;          // factor store (tiles as written by the left-looking kernel)
  const int64_t* fac_off;   // byte offset of element e's factor
  const int8_t* fac_state;  // 1 = a valid factor is stored
  double* X;                // only column N_I (the source) of each element is written
  double* E;
  double* F;
  int32_t* info;
  int32_t* ir_iters;        // may be null
  int max_iters;
  int refine64;             // as LocalArgs::refine64 (FP64 factors)
  double ir_tol;
  int n_cap;                // largest n of the launch
  int wave_words;           // LDS doubles per wave
};

// Element k of a launch (identity, or through the element list of a size class).
__device__ __forceinline__ int launch_count(const LocalArgs& a, int n_elem) { return a.ecount ? *a.ecount : n_elem; }
__device__ __forceinline__ int launch_elem(const LocalArgs& a, int k) { return a.elist ? a.elist[k] : k; }

constexpr int TILE_WORDS = 16 * 17;   // stored tile: 16 rows, padded stride 17
constexpr int RHS_CHUNK = 16;         // right-hand sides per tile row (the one-chunk kernels' limit)

// Size classes for ragged batches (upper s bound of each class, ascending).
constexpr int BIN_MAX_CLASSES = 8;
struct BinClasses {
  int n;
  int s_hi[BIN_MAX_CLASSES];
};
hipError_t launch_bin(const mhm_batch* bt, const BinClasses& cls, int32_t* elist, int32_t* counts, hipStream_t st);

size_t source_step_lds(bool fp32, int n_cap, int& wave_words);
int source_step_waves();
hipError_t launch_source_step(bool fp32, const mhm_batch* bt, const SourceArgs& a, size_t lds, int grid,
                              hipStream_t st);

size_t skeleton_solve_bytes(int n, int pb);
int skeleton_block_max();
hipError_t skeleton_csr_check(int n, const int32_t* rp, const int32_t* ci, void* work, int* host_bad,
                              hipStream_t st);
hipError_t skeleton_solve(int n, int n_lambda, int pb, const int32_t* rp, const int32_t* ci, const double* va,
                          const double* b, double* x, double tol, int max_iters, void* work, double* host_sc,
                          int* iters, double* relres, hipStream_t st);

hipError_t launch_reconstruct(const mhm_batch* bt, const double* X, const int32_t* gdof, const int32_t* erow,
                              const double* sol, int32_t n_rows, double* u, const int32_t* info, int grid,
                              hipStream_t st);
hipError_t launch_skeleton_scatter(const mhm_batch* bt, const double* M, const double* E, const double* B,
                                   const double* F, const int32_t* gdof, const int32_t* erow, const int32_t* row_ptr,
                                   const int32_t* col_idx, int32_t n_rows, double* vals, double* rhs,
                                   const int32_t* info, int32_t* missing, int grid, hipStream_t st);

hipError_t launch_assemble(const mhm_batch* bt, double* Ahat, double* Btil, double* c, double* area,
                           int32_t* info, int grid, hipStream_t st);
hipError_t launch_contrib(const mhm_batch* bt, const double* X, double* M, double* E, double* B, double* F,
                          const int32_t* info, int grid, hipStream_t st);
size_t local_lds_bytes(bool fp32, bool in_lds, int n_cap, int f_cap, int k_cap, int tile_cap);
int local_face_cap(const mhm_batch* bt);
// Register-resident FP64 kernel for elements with n <= 16 * local_rr_max_nt().
size_t local_rr_lds_bytes(int n_cap, int f_cap, int k_cap, int occ);
int local_rr_max_nt();
// occ: resident workgroups per CU the kernel is built for (2 or 3).
hipError_t launch_local_rr(bool fused, int occ, const mhm_batch* bt, LocalArgs a, size_t lds, int grid,
                           hipStream_t st);
// Left-looking kernel for large elements (tiles in a workspace slot), panel
// width pw (block columns of pw tiles); mc: the instance that takes more than
// RHS_CHUNK right-hand sides (in chunks); ref (FP64): an instance with the
// refinement step (pw 2, 8 waves, one workgroup per CU; the chunked ones
// always have it), required for a pass over deferred elements.
int local_ll_rows_per_wave(int nt, int nw);
int local_ll_default_panel(bool fp32, int nt);
bool local_ll_has(bool fp32, int pw, int nt, int occ, int nw, bool mc);
size_t local_ll_lds_bytes(bool fp32, int pw, int n_cap, int f_cap, int nw);
hipError_t launch_local_ll(bool fp32, bool fused, int pw, int occ, int nw, bool mc, bool ref, int nt_max,
                           const mhm_batch* bt, LocalArgs a, size_t lds, int grid, hipStream_t st);
hipError_t launch_local(bool fp32, bool in_lds, bool fused, const mhm_batch* bt, LocalArgs a, size_t lds, int grid,
                        hipStream_t st);

}  // namespace mhm
