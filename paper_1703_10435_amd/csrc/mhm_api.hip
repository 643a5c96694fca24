// C ABI of the MHM local-problem engine: argument checks, launch planning,
// workspace management.  All compute happens in the kernels of mhm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../include/mhm.h"
#include "mhm_kernels.h"

struct mhm_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  size_t lds_limit = 160 * 1024;
  bool no_rr = false;          // MHM_NO_RR=1: use the LDS-tile kernel for FP64 too
  bool no_ll = false;          // MHM_NO_LL=1: right-looking workspace kernel for large elements
  void* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
};

namespace {

constexpr int kGridCap = 1 << 20;
constexpr size_t kStaticLds = 4096;      // static __shared__ of k_local, rounded up
constexpr double kIrTol = 4.0e-15;

thread_local std::string g_err;   // errors of calls without a context

mhm_status fail(mhm_ctx c, mhm_status st, const std::string& msg) {
  if (c) c->err = msg;
  else g_err = msg;
  return st;
}

mhm_status hip_fail(mhm_ctx c, hipError_t e, const char* where) {
  return fail(c, MHM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

int n_of(int s) { return (s + 1) * (s + 2) / 2; }

mhm_status check_batch(mhm_ctx c, const mhm_batch* b, bool need_mat, bool need_node) {
  if (!c) return MHM_E_ARG;
  if (!b) return fail(c, MHM_E_ARG, "batch is NULL");
  if (b->n_elem < 0) return fail(c, MHM_E_ARG, "n_elem < 0");
  if (b->n_elem == 0) return MHM_OK;
  if (b->s_max < 1 || b->s_max > MHM_S_LIMIT) return fail(c, MHM_E_UNSUPPORTED, "s_max outside [1, MHM_S_LIMIT]");
  if (b->l_max < 0 || b->l_max > MHM_L_LIMIT) return fail(c, MHM_E_UNSUPPORTED, "l_max outside [0, MHM_L_LIMIT]");
  if (!b->s || !b->l || !b->vert || !b->sigma || !b->flip || !b->kappa || !b->f || !b->tri_off || !b->rhs_off)
    return fail(c, MHM_E_ARG, "a required batch array is NULL");
  if (need_mat && !b->mat_off) return fail(c, MHM_E_ARG, "mat_off is NULL");
  if (need_node && !b->node_off) return fail(c, MHM_E_ARG, "node_off is NULL");
  if (b->tri_total < 0 || b->rhs_total < 0 || b->mat_total < 0 || b->node_total < 0)
    return fail(c, MHM_E_ARG, "negative *_total");
  return MHM_OK;
}

int grid_for(const mhm_batch* b) { return std::min(b->n_elem, kGridCap); }

// Launch plan of k_local for a batch.
struct Plan {
  bool fp32, in_lds, rr, ll;
  int nt, tile_cap, n_cap, f_cap, k_cap, grid;
  size_t lds, ws_need;
  int64_t ws_slot;
};

Plan plan_local(mhm_ctx c, const mhm_batch* b, bool fp32, bool fused, bool force_ws) {
  Plan p;
  p.fp32 = fp32;
  p.n_cap = n_of(b->s_max);
  p.f_cap = mhm::local_face_cap(b);
  p.nt = (p.n_cap + 15) / 16;
  p.tile_cap = p.nt * (p.nt + 1) / 2 + p.nt;
  const size_t tsz = fp32 ? sizeof(float) : sizeof(double);
  const int k_lds = fused ? b->s_max * b->s_max : 0;
  const size_t lds_in = mhm::local_lds_bytes(fp32, true, p.n_cap, p.f_cap, k_lds, p.tile_cap);
  p.in_lds = !force_ws && lds_in + kStaticLds <= c->lds_limit;
  // FP64 elements of up to 16 * local_rr_max_nt() nodes: register-resident kernel
  p.ll = false;
  p.rr = !fp32 && !force_ws && !c->no_rr && p.nt <= mhm::local_rr_max_nt();
  if (p.rr) {
    p.in_lds = true;
    p.k_cap = k_lds;
    p.lds = mhm::local_rr_lds_bytes(p.n_cap, p.f_cap, k_lds);
    p.grid = grid_for(b);
    p.ws_slot = 0;
    p.ws_need = 0;
    return p;
  }
  if (p.in_lds) {
    p.k_cap = k_lds;
    p.lds = lds_in;
    p.grid = grid_for(b);
    p.ws_slot = 0;
    p.ws_need = 0;
  } else {
    p.k_cap = 0;
    p.ll = !c->no_ll && mhm::local_ll_rows_per_wave(p.nt) > 0;
    p.lds = p.ll ? mhm::local_ll_lds_bytes(fp32, p.n_cap, p.f_cap)
                 : mhm::local_lds_bytes(fp32, false, p.n_cap, p.f_cap, 0, p.tile_cap);
    p.grid = std::min(b->n_elem, 2 * c->n_cu);
    p.ws_slot = (int64_t)p.tile_cap * mhm::TILE_WORDS;
    p.ws_need = (size_t)p.grid * (size_t)p.ws_slot * tsz;
  }
  return p;
}

mhm_status ensure_ws(mhm_ctx c, size_t bytes) {
  if (bytes <= c->ws_bytes) return MHM_OK;
  if (c->ws) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    (void)hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  hipError_t e = hipMalloc(&c->ws, bytes);
  if (e != hipSuccess) {
    c->ws = nullptr;
    return fail(c, MHM_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " workspace bytes failed");
  }
  c->ws_bytes = bytes;
  return MHM_OK;
}

// One k_local pass (+ the FP64 fallback pass after an FP32 pass).
mhm_status run_local(mhm_ctx c, const mhm_batch* b, mhm_prec prec, bool fused, const double* Ahat,
                     const double* Btil, double* Lout, double* X, double* M, double* E, double* B, double* F,
                     int32_t* info, int32_t* ir_iters, int max_iters) {
  const bool fp32 = prec == MHM_FP32_IR;
  Plan p = plan_local(c, b, fp32, fused, false);
  Plan fb = plan_local(c, b, false, true, true);
  size_t need = p.ws_need;
  if (fp32) need = std::max(need, fb.ws_need);
  mhm_status st = ensure_ws(c, need);
  if (st != MHM_OK) return st;

  mhm::LocalArgs a;
  std::memset(&a, 0, sizeof(a));
  a.Ahat = Ahat;
  a.Btil = Btil;
  a.Lout = Lout;
  a.X = X;
  a.M = M;
  a.E = E;
  a.B = B;
  a.F = F;
  a.info = info;
  a.ir_iters = ir_iters;
  a.max_iters = std::max(0, max_iters);
  a.only_fallback = 0;
  a.ir_tol = kIrTol;
  a.ws = c->ws;
  a.ws_slot = p.ws_slot;
  a.tile_cap = p.tile_cap;
  a.n_cap = p.n_cap;
  a.f_cap = p.f_cap;
  a.k_cap = p.k_cap;
  hipError_t e = p.rr ? mhm::launch_local_rr(fused, b, a, p.lds, p.grid, c->stream)
               : p.ll ? mhm::launch_local_ll(fp32, fused, p.nt, b, a, p.lds, p.grid, c->stream)
                      : mhm::launch_local(fp32, p.in_lds, fused, b, a, p.lds, p.grid, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "k_local launch");
  if (fp32) {
    // FP64 recomputation of the elements whose refinement did not converge
    mhm::LocalArgs f = a;
    f.Ahat = nullptr;
    f.Btil = nullptr;
    f.only_fallback = 1;
    f.ws_slot = fb.ws_slot;
    f.tile_cap = fb.tile_cap;
    f.n_cap = fb.n_cap;
    f.f_cap = fb.f_cap;
    f.k_cap = 0;
    if (!fused) {
      f.M = f.E = f.B = f.F = nullptr;
    }
    e = fb.ll ? mhm::launch_local_ll(false, true, fb.nt, b, f, fb.lds, fb.grid, c->stream)
              : mhm::launch_local(false, false, true, b, f, fb.lds, fb.grid, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "k_local fallback launch");
  }
  return MHM_OK;
}

}  // namespace

extern "C" {

mhm_status mhm_create(mhm_ctx* out, int device, void* hip_stream) {
  if (!out) return fail(nullptr, MHM_E_ARG, "ctx is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev)
    return fail(nullptr, MHM_E_DEVICE, "device " + std::to_string(device) + " of " + std::to_string(ndev));
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  mhm_ctx c = new mhm_ctx_s();
  c->device = device;
  const char* nrr = std::getenv("MHM_NO_RR");
  c->no_rr = nrr && nrr[0] == '1';
  const char* nll = std::getenv("MHM_NO_LL");
  c->no_ll = nll && nll[0] == '1';
  c->stream = static_cast<hipStream_t>(hip_stream);
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0) c->n_cu = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
    c->lds_limit = (size_t)v;
  *out = c;
  return MHM_OK;
}

mhm_status mhm_destroy(mhm_ctx c) {
  if (!c) return MHM_E_ARG;
  if (c->ws) {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->ws);
  }
  delete c;
  return MHM_OK;
}

mhm_status mhm_set_stream(mhm_ctx c, void* hip_stream) {
  if (!c) return MHM_E_ARG;
  c->stream = static_cast<hipStream_t>(hip_stream);
  return MHM_OK;
}

const char* mhm_last_error(mhm_ctx c) { return c ? c->err.c_str() : g_err.c_str(); }

mhm_status mhm_sync(mhm_ctx c) {
  if (!c) return MHM_E_ARG;
  hipError_t e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? MHM_OK : hip_fail(c, e, "hipStreamSynchronize");
}

size_t mhm_workspace_bytes(mhm_ctx c, const mhm_batch* b, mhm_prec prec) {
  if (!c || !b || b->n_elem <= 0 || b->s_max < 1 || b->s_max > MHM_S_LIMIT) return 0;
  const bool fp32 = prec == MHM_FP32_IR;
  size_t need = plan_local(c, b, fp32, true, false).ws_need;
  need = std::max(need, plan_local(c, b, fp32, false, false).ws_need);
  if (fp32) need = std::max(need, plan_local(c, b, false, true, true).ws_need);
  return need;
}

mhm_status mhm_local_assemble(mhm_ctx c, const mhm_batch* b, double* Ahat, double* Btil, double* cvec,
                              double* area, int32_t* info) {
  mhm_status st = check_batch(c, b, true, true);
  if (st != MHM_OK || b->n_elem == 0) return st;
  if (!Ahat || !Btil || !cvec) return fail(c, MHM_E_ARG, "Ahat, Btilde and c are required");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  e = mhm::launch_assemble(b, Ahat, Btil, cvec, area, info, grid_for(b), c->stream);
  return e == hipSuccess ? MHM_OK : hip_fail(c, e, "k_assemble launch");
}

mhm_status mhm_local_factor_solve(mhm_ctx c, const mhm_batch* b, mhm_prec prec, double* Ahat_io,
                                  const double* Btil, double* X, int32_t* info, int32_t* ir_iters, int max_iters) {
  mhm_status st = check_batch(c, b, true, false);
  if (st != MHM_OK || b->n_elem == 0) return st;
  if (prec != MHM_FP64 && prec != MHM_FP32_IR) return fail(c, MHM_E_ARG, "unknown precision");
  if (!Ahat_io || !Btil || !X || !info) return fail(c, MHM_E_ARG, "Ahat_io, Btilde, X and info are required");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  return run_local(c, b, prec, false, Ahat_io, Btil, Ahat_io, X, nullptr, nullptr, nullptr, nullptr, info,
                   ir_iters, max_iters);
}

mhm_status mhm_skeleton_contrib(mhm_ctx c, const mhm_batch* b, const double* X, double* M, double* E, double* B,
                                double* F, const int32_t* info) {
  mhm_status st = check_batch(c, b, false, false);
  if (st != MHM_OK || b->n_elem == 0) return st;
  if (!X || !M || !E || !B || !F) return fail(c, MHM_E_ARG, "X, M, E, B and F are required");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  e = mhm::launch_contrib(b, X, M, E, B, F, info, grid_for(b), c->stream);
  return e == hipSuccess ? MHM_OK : hip_fail(c, e, "k_contrib launch");
}

mhm_status mhm_local_batch_run(mhm_ctx c, const mhm_batch* b, mhm_prec prec, double* X, double* M, double* E,
                               double* B, double* F, int32_t* info, int32_t* ir_iters, int max_iters) {
  mhm_status st = check_batch(c, b, false, false);
  if (st != MHM_OK || b->n_elem == 0) return st;
  if (prec != MHM_FP64 && prec != MHM_FP32_IR) return fail(c, MHM_E_ARG, "unknown precision");
  if (!X || !M || !E || !B || !F || !info) return fail(c, MHM_E_ARG, "X, M, E, B, F and info are required");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  return run_local(c, b, prec, true, nullptr, nullptr, nullptr, X, M, E, B, F, info, ir_iters, max_iters);
}

}  // extern "C"
