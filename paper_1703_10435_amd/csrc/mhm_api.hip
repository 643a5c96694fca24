// C ABI of the MHM local-problem engine: argument checks, launch planning
// (size classes, kernel families, autotuning), workspace management, graph
// capture.  All compute happens in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mhm.h"
#include "mhm_kernels.h"

namespace {

constexpr int kGridCap = 1 << 20;
constexpr size_t kStaticLds = 4096;      // static __shared__ of k_local, rounded up
constexpr double kIrTol = 4.0e-15;
constexpr size_t kAlign = 256;

// Size classes of ragged batches (upper s of each class).  A batch whose s
// range falls in one class runs as one launch; otherwise a binning kernel
// sorts the elements into per-class lists and every class gets its own
// persistent launch, on its own stream, sized for that class.
constexpr int kNumClasses = 5;
constexpr int kClassHi[kNumClasses] = {16, 25, 33, 48, 64};
static_assert(kNumClasses <= mhm::BIN_MAX_CLASSES, "class table");

int class_of(int s) {
  for (int c = 0; c < kNumClasses; ++c)
    if (s <= kClassHi[c]) return c;
  return kNumClasses - 1;
}

// Kernel family ("tile shape") of a launch.
enum Fam { FAM_RR = 0, FAM_LDS = 1, FAM_LL = 2, FAM_WS = 3 };
const char* fam_name(int f) {
  switch (f) {
    case FAM_RR: return "register-tiles";
    case FAM_LDS: return "lds-tiles";
    case FAM_LL: return "left-looking";
    default: return "workspace";
  }
}
struct Choice {
  int fam = -1;
  int pw = 0;    // panel width (left-looking)
  int occ = 1;   // resident workgroups per CU the kernel is built for (left-looking, register tiles)
  int nw = 8;    // waves per element (left-looking)
};

}  // namespace

// Device scratch of mhm_local_batch_run_noalloc (class lists and workspace
// slots), one copy per GPU for the life of the process.  In host code the
// name is a stand-in, not a device address: every use goes through the
// address hipGetSymbolAddress returned for the device (scratch_ptr below).
static __device__ __align__(256) char scratch[MHM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on `device` (which is current), looked up
// once per device; null on failure.
void* scratch_ptr(int device, hipError_t* err) {
  *err = hipSuccess;
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

}  // namespace

struct mhm_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  size_t lds_limit = 160 * 1024;
  // options (mhm_set_option)
  bool no_rr = false;          // never use the register-tile kernel
  bool no_ll = false;          // never use the left-looking kernel
  bool ll_occ2 = false;        // left-looking default with two workgroups per CU
  bool ll_nw16 = false;        // left-looking default with 16 waves where it applies
  int ll_pw = 0;               // left-looking default panel width (1, 2, 4), where built
  int rr_occ = 0;              // register-tile kernel default workgroups per CU (2, 3)
  int refine64 = 0;            // FP64 refinement: 0 where needed, 1 every element, -1 none
  void* scratch = nullptr;     // this device's scratch array (mhm_local_batch_run_noalloc)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t aux[kNumClasses] = {};   // class streams of ragged runs
  hipEvent_t fork = nullptr;
  hipEvent_t join[kNumClasses] = {};
  // MHM_OPT_CLASS_TIMING: events around each class's main launch
  bool class_timing = false;
  bool concurrent_classes = false;   // MHM_OPT_CONCURRENT_CLASSES: size classes on forked streams
  hipEvent_t t_beg[kNumClasses] = {}, t_end[kNumClasses] = {};
  int timed_n = -1;
  int timed_cap[kNumClasses] = {};
  Choice tuned[kNumClasses][2][2];     // [class][fp32][fused], from mhm_autotune
  std::string tune_log;
  std::string err;
};

struct mhm_graph_s {
  mhm_ctx ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* ws = nullptr;
};

namespace {

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
// Bound on the face DoFs per face, m (l + 1); the contribution blocks are 3x that wide.
int p_bound(const mhm_batch* b) { return b->p_max > 0 ? b->p_max : b->l_max + 1; }
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

mhm_status check_batch(mhm_ctx c, const mhm_batch* b, bool need_mat, bool need_node) {
  if (!c) return MHM_E_ARG;
  if (!b) return fail(c, MHM_E_ARG, "batch is NULL");
  if (b->n_elem < 0) return fail(c, MHM_E_ARG, "n_elem < 0");
  if (b->n_elem == 0) return MHM_OK;
  if (b->s_max < 1 || b->s_max > MHM_S_LIMIT) return fail(c, MHM_E_UNSUPPORTED, "s_max outside [1, MHM_S_LIMIT]");
  if (b->s_min < 0 || b->s_min > b->s_max) return fail(c, MHM_E_ARG, "s_min outside [0, s_max]");
  if (b->l_max < 0 || b->l_max > MHM_L_LIMIT) return fail(c, MHM_E_UNSUPPORTED, "l_max outside [0, MHM_L_LIMIT]");
  if (b->p_max < 0 || p_bound(b) > MHM_P_LIMIT)
    return fail(c, MHM_E_UNSUPPORTED, "p_max (bound on m(l+1)) outside [0, MHM_P_LIMIT]");
  if (!b->s || !b->l || !b->vert || !b->sigma || !b->flip || !b->kappa || !b->f || !b->tri_off || !b->rhs_off)
    return fail(c, MHM_E_ARG, "a required batch array is NULL");
  if (need_mat && !b->mat_off) return fail(c, MHM_E_ARG, "mat_off is NULL");
  if (need_node && !b->node_off) return fail(c, MHM_E_ARG, "node_off is NULL");
  if (b->tri_total < 0 || b->rhs_total < 0 || b->mat_total < 0 || b->node_total < 0)
    return fail(c, MHM_E_ARG, "negative *_total");
  return MHM_OK;
}

int grid_for(const mhm_batch* b) { return std::min(b->n_elem, kGridCap); }

// Launch plan of one local-problem kernel for elements with s <= s_cap.
struct Plan {
  bool ok = false, fp32 = false, fused = false;
  bool mc = false;   // more than RHS_CHUNK right-hand sides (left-looking kernel only)
  bool ref = false;  // FP64 left-looking instance with the refinement step (the FP64 pass)
  Choice ch;
  int nt = 0, tile_cap = 0, n_cap = 0, f_cap = 0, k_cap = 0, grid = 0;
  size_t lds = 0, ws_need = 0;
  int64_t ws_slot = 0;
};

Plan plan_for(const mhm_ctx c, const mhm_batch* b, bool fp32, bool fused, int s_cap, Choice ch, bool listed,
              bool cached = false) {
  Plan p;
  p.fp32 = fp32;
  p.fused = fused;
  p.ch = ch;
  p.n_cap = n_of(s_cap);
  p.f_cap = 3 * p_bound(b) * (s_cap + 1);
  p.nt = (p.n_cap + 15) / 16;
  p.tile_cap = p.nt * (p.nt + 1) / 2 + p.nt;
  // every right-hand side in one 16-wide chunk: the families other than the
  // left-looking one take only that
  const bool one_chunk = 3 * p_bound(b) + 1 <= mhm::RHS_CHUNK;
  p.mc = !one_chunk;
  const size_t tsz = fp32 ? sizeof(float) : sizeof(double);
  const int k_lds = fused ? s_cap * s_cap : 0;
  // one workgroup per element, or a persistent grid over a class list
  const int one_each = listed ? std::min(b->n_elem, 8 * c->n_cu) : grid_for(b);
  const int slots = std::min(b->n_elem, 2 * c->n_cu);
  switch (ch.fam) {
    case FAM_RR:
      // two or three resident workgroups per CU; by default two (the build
      // for three spills in its factorisation loop: at C2 it is 3% faster
      // but moves eight times the bytes, so only the tuner picks it)
      if (p.ch.occ != 2 && p.ch.occ != 3) p.ch.occ = c->rr_occ ? c->rr_occ : 2;
      p.ok = !fp32 && p.nt <= mhm::local_rr_max_nt() && one_chunk;
      p.k_cap = k_lds;
      p.lds = mhm::local_rr_lds_bytes(p.n_cap, p.f_cap, k_lds, p.ch.occ);
      p.grid = one_each;
      break;
    case FAM_LDS:
      p.k_cap = k_lds;
      p.lds = mhm::local_lds_bytes(fp32, true, p.n_cap, p.f_cap, k_lds, p.tile_cap);
      p.ok = p.lds + kStaticLds <= c->lds_limit && one_chunk;
      p.grid = one_each;
      break;
    case FAM_LL:
      p.ok = mhm::local_ll_has(fp32, ch.pw, p.nt, ch.occ, ch.nw, p.mc);
      p.lds = mhm::local_ll_lds_bytes(fp32, ch.pw, p.n_cap, p.f_cap, ch.nw);
      p.grid = slots;
      {
        // right-hand-side tile rows (one per 16 columns), then the diagonal
        // factor tiles kept for the factor output; with the factor in the
        // caller's store, the right-hand-side rows only
        const int nch = p.mc ? (3 * p_bound(b) + 1 + mhm::RHS_CHUNK - 1) / mhm::RHS_CHUNK : 1;
        p.tile_cap += nch * p.nt;
        if (cached) p.tile_cap = nch * p.nt;
      }
      p.ws_slot = (int64_t)p.tile_cap * mhm::TILE_WORDS;
      break;
    default:
      p.lds = mhm::local_lds_bytes(fp32, false, p.n_cap, p.f_cap, 0, p.tile_cap);
      p.ok = p.lds + kStaticLds <= c->lds_limit && one_chunk;
      p.grid = slots;
      p.ws_slot = (int64_t)p.tile_cap * mhm::TILE_WORDS;
      break;
  }
  p.ok = p.ok && p.lds + kStaticLds <= c->lds_limit && (!cached || ch.fam == FAM_LL);
  p.ws_need = align_up((size_t)p.grid * (size_t)p.ws_slot * tsz);
  return p;
}

// Default family when nothing was tuned.
Choice default_choice(const mhm_ctx c, const mhm_batch* b, bool fp32, bool fused, int s_cap, bool listed) {
  const int nt = (n_of(s_cap) + 15) / 16;
  const int pw = c->ll_pw > 0 ? c->ll_pw : mhm::local_ll_default_panel(fp32, nt);
  const Choice ll = c->ll_occ2 ? Choice{FAM_LL, 2, 2} : Choice{FAM_LL, pw, 1};
  const Choice ll16{FAM_LL, 2, 1, 16};
  const Choice cands[] = {{FAM_RR, 0}, {FAM_LDS, 0}, c->ll_nw16 ? ll16 : ll, ll, {FAM_LL, 2, 1}, {FAM_WS, 0}};
  for (const Choice& ch : cands) {
    if (ch.fam == FAM_RR && c->no_rr) continue;
    if (ch.fam == FAM_LL && c->no_ll) continue;
    if (plan_for(c, b, fp32, fused, s_cap, ch, listed).ok) return ch;
  }
  return Choice{FAM_WS, 0};
}

// The FP64 pass after a launch, always from kappa (fused): the
// recomputation of an FP32 launch's elements whose refinement did not
// converge, or the elements an FP64 launch deferred because they need the
// refinement step (after a three-call factor_solve it also writes their
// factor).  Left-looking where it applies, else the workspace kernel.
Plan fallback_plan(const mhm_ctx c, const mhm_batch* b, int s_cap, bool listed, bool cached = false) {
  // the left-looking instances with the refinement step: panel width 2, 8
  // waves (with stored factors: the deferred elements of a cached FP64 run)
  Plan p = plan_for(c, b, false, true, s_cap, Choice{FAM_LL, 2, 1, 8}, listed, cached);
  if (!cached && (c->no_ll || !p.ok)) p = plan_for(c, b, false, true, s_cap, Choice{FAM_WS, 0}, listed);
  p.ref = true;
  return p;
}

// Whether an FP64 pass follows a main launch: always after FP32 (the
// recomputation of elements whose refinement did not converge); after the
// FP64 register-tile kernel and the one-chunk FP64 left-looking instances
// when they may defer elements that need the refinement step.
bool has_fp64_pass(const mhm_ctx c, const Plan& m) {
  if (m.fp32) return true;
  if (c->refine64 < 0) return false;
  return (m.ch.fam == FAM_RR && m.fused) || (m.ch.fam == FAM_LL && !m.mc);
}

// Everything one run of the local problems enqueues.
struct ClassRun {
  int cls = 0, s_cap = 0;
  bool has_fb = false;   // an FP64 pass follows the main launch
  Plan main, fb;
  size_t ws_off = 0;   // this class's workspace (main and fallback pass share it)
};
struct RunPlan {
  bool listed = false;   // binned into class lists
  int n_runs = 0;
  ClassRun run[kNumClasses];
  size_t list_bytes = 0;  // class lists + counts at the start of the workspace
  size_t ws_total = 0;
};

// `over`: force this choice for every class (tuning); otherwise the tuned
// or default choice per class.
RunPlan make_run_plan(const mhm_ctx c, const mhm_batch* b, bool fp32, bool fused, const Choice* over,
                      bool cached = false) {
  RunPlan rp;
  const int s_lo = b->s_min > 0 ? b->s_min : 1;
  const int c_lo = class_of(s_lo), c_hi = class_of(b->s_max);
  rp.listed = c_lo != c_hi;
  if (rp.listed) rp.list_bytes = align_up(sizeof(int32_t) * ((size_t)kNumClasses * b->n_elem + kNumClasses));
  size_t off = rp.list_bytes;
  // largest class first: it goes on the caller's stream and starts first
  for (int k = c_hi; k >= c_lo; --k) {
    ClassRun& r = rp.run[rp.n_runs++];
    r.cls = k;
    r.s_cap = rp.listed ? std::min(kClassHi[k], b->s_max) : b->s_max;
    Choice ch = over ? *over : c->tuned[k][fp32][fused];
    if (cached) {
      // stored factors: the left-looking kernel (tuned panel width if any;
      // the chunked instance for more than RHS_CHUNK right-hand sides)
      if (ch.fam != FAM_LL) ch = Choice{FAM_LL, mhm::local_ll_default_panel(fp32, (n_of(r.s_cap) + 15) / 16)};
      if (3 * p_bound(b) + 1 > mhm::RHS_CHUNK) ch = Choice{FAM_LL, 2};
    } else if (ch.fam < 0 || !plan_for(c, b, fp32, fused, r.s_cap, ch, rp.listed).ok) {
      ch = default_choice(c, b, fp32, fused, r.s_cap, rp.listed);
    }
    r.main = plan_for(c, b, fp32, fused, r.s_cap, ch, rp.listed, cached);
    // the FP64 pass: FP32 recomputation, or the elements an FP64 launch
    // defers (those that need the refinement step)
    r.has_fb = has_fp64_pass(c, r.main);
    if (r.has_fb) r.fb = fallback_plan(c, b, r.s_cap, rp.listed, !fp32 && cached);
    r.ws_off = off;
    off += std::max(r.main.ws_need, r.has_fb ? r.fb.ws_need : 0);
  }
  rp.ws_total = off;
  return rp;
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

mhm_status ensure_streams(mhm_ctx c) {
  if (c->fork) return MHM_OK;
  hipError_t e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(c, e, "hipEventCreateWithFlags");
  for (int k = 0; k < kNumClasses; ++k) {
    e = hipStreamCreateWithFlags(&c->aux[k], hipStreamNonBlocking);   // default priority
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreateWithFlags");
    e = hipEventCreateWithFlags(&c->join[k], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventCreateWithFlags");
  }
  return MHM_OK;
}

// Pointers of one run.
struct RunIO {
  const double* Ahat = nullptr;
  const double* Btil = nullptr;
  double* Lout = nullptr;
  double *X = nullptr, *M = nullptr, *E = nullptr, *B = nullptr, *F = nullptr;
  int32_t* info = nullptr;
  int32_t* ir_iters = nullptr;
  int max_iters = 0;
  void* fac = nullptr;              // factor store (left-looking kernel only)
  const int64_t* fac_off = nullptr;
  const int8_t* fac_state = nullptr;
};

hipError_t launch_plan(const Plan& p, const mhm_batch* b, const mhm::LocalArgs& a, hipStream_t st) {
  switch (p.ch.fam) {
    case FAM_RR: return mhm::launch_local_rr(p.fused, p.ch.occ, b, a, p.lds, p.grid, st);
    case FAM_LDS: return mhm::launch_local(p.fp32, true, p.fused, b, a, p.lds, p.grid, st);
    case FAM_LL:
      return mhm::launch_local_ll(p.fp32, p.fused, p.ch.pw, p.ch.occ, p.ch.nw, p.mc, p.ref, p.nt, b, a, p.lds, p.grid,
                                  st);
    default: return mhm::launch_local(p.fp32, false, p.fused, b, a, p.lds, p.grid, st);
  }
}

mhm::LocalArgs local_args(const mhm_ctx c, const Plan& p, const RunIO& io, void* ws, const int32_t* elist,
                          const int32_t* ecount) {
  mhm::LocalArgs a;
  std::memset(&a, 0, sizeof(a));
  a.refine64 = c->refine64;
  a.Ahat = io.Ahat;
  a.Btil = io.Btil;
  a.Lout = io.Lout;
  a.X = io.X;
  a.M = io.M;
  a.E = io.E;
  a.B = io.B;
  a.F = io.F;
  a.info = io.info;
  a.ir_iters = io.ir_iters;
  a.max_iters = std::max(0, io.max_iters);
  a.ir_tol = kIrTol;
  a.ws = ws;
  a.ws_slot = p.ws_slot;
  a.tile_cap = p.tile_cap;
  a.n_cap = p.n_cap;
  a.f_cap = p.f_cap;
  a.k_cap = p.k_cap;
  a.elist = elist;
  a.ecount = ecount;
  a.fac = io.fac;
  a.fac_off = io.fac_off;
  a.fac_state = io.fac_state;
  return a;
}

// One class: the main pass, then the FP64 pass: of the elements whose FP32
// refinement did not converge, or of those an FP64 register-tile launch
// deferred to a kernel with the refinement step.
mhm_status enqueue_class(mhm_ctx c, const ClassRun& r, const mhm_batch* b, const RunIO& io, char* ws,
                         const int32_t* elist, const int32_t* ecount, hipStream_t st, bool fallback_only = false,
                         int timing_slot = -1) {
  hipError_t e = hipSuccess;
  if (!fallback_only) {
    mhm::LocalArgs a = local_args(c, r.main, io, ws + r.ws_off, elist, ecount);
    if (timing_slot >= 0) {
      e = hipEventRecord(c->t_beg[timing_slot], st);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventRecord");
    }
    e = launch_plan(r.main, b, a, st);
    if (e != hipSuccess) return hip_fail(c, e, "local kernel launch");
    if (timing_slot >= 0) {
      e = hipEventRecord(c->t_end[timing_slot], st);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventRecord");
      c->timed_cap[timing_slot] = r.s_cap;
    }
  }
  if (r.has_fb && r.main.fp32) {
    RunIO f = io;
    f.Ahat = nullptr;
    f.Btil = nullptr;
    f.Lout = nullptr;  // the FP32 factor stays in Ahat_io
    f.fac = nullptr;   // the FP64 recomputation does not store its factor
    f.fac_off = nullptr;
    f.fac_state = nullptr;
    if (!r.main.fused) f.M = f.E = f.B = f.F = nullptr;
    mhm::LocalArgs fa = local_args(c, r.fb, f, ws + r.ws_off, elist, ecount);
    fa.only_fallback = 1;
    e = launch_plan(r.fb, b, fa, st);
    if (e != hipSuccess) return hip_fail(c, e, "FP64 fallback launch");
  } else if (r.has_fb) {
    // deferred elements of an FP64 launch: recomputed from kappa, with the
    // same outputs (the three-call form's factor into Ahat_io, the contribution
    // blocks of the fused form), and their info ends 0
    RunIO f = io;
    f.Ahat = nullptr;
    f.Btil = nullptr;
    mhm::LocalArgs fa = local_args(c, r.fb, f, ws + r.ws_off, elist, ecount);
    fa.only_fallback = 1;
    fa.fb_final = 1;
    e = launch_plan(r.fb, b, fa, st);
    if (e != hipSuccess) return hip_fail(c, e, "FP64 refinement pass launch");
  }
  return MHM_OK;
}

mhm::BinClasses bin_classes() {
  mhm::BinClasses bc;
  std::memset(&bc, 0, sizeof(bc));
  bc.n = kNumClasses;
  for (int k = 0; k < kNumClasses; ++k) bc.s_hi[k] = kClassHi[k];
  return bc;
}

// Enqueue a whole run on stream `st` (also under stream capture): binning,
// then the classes, largest first, one after another on `st` (with
// MHM_OPT_CONCURRENT_CLASSES: the largest on `st` and the others forked onto
// the context's class streams and joined back).
mhm_status enqueue_run(mhm_ctx c, const RunPlan& rp, const mhm_batch* b, const RunIO& io, void* ws_v, hipStream_t st,
                       bool fallback_only = false, bool one_stream = false) {
  char* ws = static_cast<char*>(ws_v);
  int32_t* lists = reinterpret_cast<int32_t*>(ws);
  int32_t* counts = lists + (size_t)kNumClasses * b->n_elem;
  if (rp.listed) {
    hipError_t e = mhm::launch_bin(b, bin_classes(), lists, counts, st);
    if (e != hipSuccess) return hip_fail(c, e, "k_bin launch");
  }
  const bool fork = rp.n_runs > 1 && !one_stream && c->concurrent_classes;
  if (fork) {
    mhm_status s0 = ensure_streams(c);
    if (s0 != MHM_OK) return s0;
    hipError_t e = hipEventRecord(c->fork, st);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventRecord");
    for (int i = 1; i < rp.n_runs; ++i) {
      e = hipStreamWaitEvent(c->aux[i], c->fork, 0);
      if (e != hipSuccess) return hip_fail(c, e, "hipStreamWaitEvent");
    }
  }
  for (int i = 0; i < rp.n_runs; ++i) {
    const ClassRun& r = rp.run[i];
    const int32_t* el = rp.listed ? lists + (size_t)r.cls * b->n_elem : nullptr;
    const int32_t* ec = rp.listed ? counts + r.cls : nullptr;
    const int slot = c->class_timing && !fallback_only ? i : -1;
    mhm_status s1 = enqueue_class(c, r, b, io, ws, el, ec, i == 0 || !fork ? st : c->aux[i], fallback_only, slot);
    if (s1 != MHM_OK) return s1;
  }
  if (c->class_timing && !fallback_only) c->timed_n = rp.n_runs;
  if (fork) {
    for (int i = 1; i < rp.n_runs; ++i) {
      hipError_t e = hipEventRecord(c->join[i], c->aux[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, c->join[i], 0);
      if (e != hipSuccess) return hip_fail(c, e, "stream join");
    }
  }
  return MHM_OK;
}

mhm_status run_local(mhm_ctx c, const mhm_batch* b, mhm_prec prec, bool fused, const RunIO& io) {
  const bool cached = io.fac != nullptr;
  const RunPlan rp = make_run_plan(c, b, prec == MHM_FP32_IR, fused, nullptr, cached);
  if (cached)
    for (int i = 0; i < rp.n_runs; ++i)
      if (!rp.run[i].main.ok) return fail(c, MHM_E_UNSUPPORTED, "stored factors need s <= 48");
  mhm_status st = ensure_ws(c, rp.ws_total);
  if (st != MHM_OK) return st;
  return enqueue_run(c, rp, b, io, c->ws, c->stream);
}

RunIO fused_io(double* X, double* M, double* E, double* B, double* F, int32_t* info, int32_t* ir_iters,
               int max_iters) {
  RunIO io;
  io.X = X;
  io.M = M;
  io.E = E;
  io.B = B;
  io.F = F;
  io.info = info;
  io.ir_iters = ir_iters;
  io.max_iters = max_iters;
  return io;
}

mhm_status check_fused(mhm_ctx c, const mhm_batch* b, mhm_prec prec, double* X, double* M, double* E, double* B,
                       double* F, int32_t* info) {
  mhm_status st = check_batch(c, b, false, false);
  if (st != MHM_OK) return st;
  if (prec != MHM_FP64 && prec != MHM_FP32_IR) return fail(c, MHM_E_ARG, "unknown precision");
  if (b->n_elem > 0 && (!X || !M || !E || !B || !F || !info))
    return fail(c, MHM_E_ARG, "X, M, E, B, F and info are required");
  return MHM_OK;
}

// Autotuning of one class: every feasible family / panel width on up to
// `cap` of its elements, timed with events; returns the fastest.
Choice tune_class(mhm_ctx c, const mhm_batch* b, bool fp32, const RunPlan& base, int i, const RunIO& io,
                  int32_t* dcount, int cap, int count, std::string& log, mhm_status& st) {
  const ClassRun& r0 = base.run[i];
  std::vector<Choice> cands;
  const Choice all[] = {{FAM_RR, 0, 3},     {FAM_RR, 0, 2},     {FAM_LDS, 0, 1},    {FAM_LL, 2, 1},
                        {FAM_LL, 4, 1},     {FAM_LL, 2, 2},     {FAM_LL, 2, 1, 16}, {FAM_LL, 4, 1, 16},
                        {FAM_LL, 1, 1},     {FAM_LL, 1, 1, 16}, {FAM_WS, 0, 1}};
  bool have_ll = false;
  for (const Choice& ch : all) {
    if (ch.fam == FAM_RR && c->no_rr) continue;
    if (ch.fam == FAM_LL && c->no_ll) continue;
    if (ch.fam == FAM_WS && have_ll) continue;   // the right-looking workspace kernel only without a left-looking one
    if (plan_for(c, b, fp32, true, r0.s_cap, ch, base.listed).ok) {
      cands.push_back(ch);
      if (ch.fam == FAM_LL) have_ll = true;
    }
  }
  Choice best = r0.main.ch;
  if (cands.size() < 2) return best;
  const int sub = std::min(count, cap);
  hipError_t e = hipMemcpyAsync(dcount, &sub, sizeof(int), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) {
    st = hip_fail(c, e, "hipMemcpyAsync");
    return best;
  }
  const int32_t* el = nullptr;
  if (base.listed) el = reinterpret_cast<int32_t*>(c->ws) + (size_t)r0.cls * b->n_elem;
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  float best_ms = 0.0f;
  char buf[160];
  for (const Choice& ch : cands) {
    ClassRun r = r0;
    r.main = plan_for(c, b, fp32, true, r.s_cap, ch, base.listed);
    r.has_fb = has_fp64_pass(c, r.main);
    if (r.has_fb) r.fb = fallback_plan(c, b, r.s_cap, base.listed);
    r.ws_off = base.list_bytes;   // classes are tuned one after another
    float ms = 0.0f;
    for (int rep = 0; rep < 3 && st == MHM_OK; ++rep) {   // first repetition warms up
      (void)hipEventRecord(t0, c->stream);
      st = enqueue_class(c, r, b, io, static_cast<char*>(c->ws), el, dcount, c->stream);
      (void)hipEventRecord(t1, c->stream);
      if (hipEventSynchronize(t1) != hipSuccess) st = fail(c, MHM_E_DEVICE, "tuning run failed");
      float m = 0.0f;
      (void)hipEventElapsedTime(&m, t0, t1);
      if (rep > 0) ms += m / 2;
    }
    if (st != MHM_OK) break;
    std::snprintf(buf, sizeof(buf),
                  "%s{\"s_max\": %d, \"prec\": \"%s\", \"kernel\": \"%s\", \"pw\": %d, \"wg_per_cu\": %d, "
                  "\"waves\": %d, \"ms\": %.4f, \"elements\": %d}",
                  log.empty() ? "" : ", ", r.s_cap, fp32 ? "fp32_ir" : "fp64", fam_name(ch.fam), ch.pw, ch.occ,
                  ch.fam == FAM_LL ? ch.nw : 4, ms, sub);
    log += buf;
    if (best_ms == 0.0f || ms < best_ms) {
      best_ms = ms;
      best = ch;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  return best;
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
  c->stream = static_cast<hipStream_t>(hip_stream);
  // the no-allocation entry point's scratch array on this device (set-up
  // time: the lookup loads the code object on the device)
  c->scratch = scratch_ptr(device, &e);
  if (!c->scratch) {
    delete c;
    return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
  }
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0) c->n_cu = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
    c->lds_limit = (size_t)v;
  *out = c;
  return MHM_OK;
}

mhm_status mhm_destroy(mhm_ctx c) {
  if (!c) return MHM_E_ARG;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (int k = 0; k < kNumClasses; ++k) {
    if (c->aux[k]) {
      (void)hipStreamSynchronize(c->aux[k]);
      (void)hipStreamDestroy(c->aux[k]);
    }
    if (c->join[k]) (void)hipEventDestroy(c->join[k]);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  for (int k = 0; k < kNumClasses; ++k) {
    if (c->t_beg[k]) (void)hipEventDestroy(c->t_beg[k]);
    if (c->t_end[k]) (void)hipEventDestroy(c->t_end[k]);
  }
  if (c->ws) (void)hipFree(c->ws);
  delete c;
  return MHM_OK;
}

mhm_status mhm_set_option(mhm_ctx c, int option, int value) {
  if (!c) return MHM_E_ARG;
  auto flag = [&](bool& dst) {
    if (value != 0 && value != 1) return fail(c, MHM_E_ARG, "option value must be 0 or 1");
    dst = value != 0;
    return MHM_OK;
  };
  switch (option) {
    case MHM_OPT_REFINE64:
      if (value < -1 || value > 1) return fail(c, MHM_E_ARG, "MHM_OPT_REFINE64 takes -1, 0 or 1");
      c->refine64 = value;
      return MHM_OK;
    case MHM_OPT_NO_RR: return flag(c->no_rr);
    case MHM_OPT_NO_LL: return flag(c->no_ll);
    case MHM_OPT_LL_OCC2: return flag(c->ll_occ2);
    case MHM_OPT_LL_NW16: return flag(c->ll_nw16);
    case MHM_OPT_LL_PW:
      if (value != 0 && value != 1 && value != 2 && value != 4) return fail(c, MHM_E_ARG, "MHM_OPT_LL_PW takes 0, 1, 2 or 4");
      c->ll_pw = value;
      return MHM_OK;
    case MHM_OPT_RR_OCC:
      if (value != 0 && value != 2 && value != 3) return fail(c, MHM_E_ARG, "MHM_OPT_RR_OCC takes 0, 2 or 3");
      c->rr_occ = value;
      return MHM_OK;
    case MHM_OPT_CONCURRENT_CLASSES: {
      if (value != 0 && value != 1) return fail(c, MHM_E_ARG, "MHM_OPT_CONCURRENT_CLASSES takes 0 or 1");
      c->concurrent_classes = value != 0;
      return MHM_OK;
    }
    case MHM_OPT_CLASS_TIMING: {
      if (value != 0 && value != 1) return fail(c, MHM_E_ARG, "MHM_OPT_CLASS_TIMING takes 0 or 1");
      if (value && !c->t_beg[0]) {
        hipError_t e = hipSetDevice(c->device);
        for (int k = 0; k < kNumClasses && e == hipSuccess; ++k) {
          e = hipEventCreate(&c->t_beg[k]);
          if (e == hipSuccess) e = hipEventCreate(&c->t_end[k]);
        }
        if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
      }
      c->class_timing = value != 0;
      c->timed_n = -1;
      return MHM_OK;
    }
    default: return fail(c, MHM_E_ARG, "unknown option " + std::to_string(option));
  }
}

int mhm_class_times(mhm_ctx c, int32_t* s_cap, float* ms, int max) {
  if (!c || !c->class_timing || c->timed_n < 0 || max < 0) return -1;
  const int n = std::min(c->timed_n, max);
  for (int k = 0; k < n; ++k) {
    float t = 0.0f;
    if (hipEventSynchronize(c->t_end[k]) != hipSuccess || hipEventElapsedTime(&t, c->t_beg[k], c->t_end[k]) != hipSuccess)
      return -1;
    if (s_cap) s_cap[k] = c->timed_cap[k];
    if (ms) ms[k] = t;
  }
  return n;
}

mhm_status mhm_set_stream(mhm_ctx c, void* hip_stream) {
  if (!c) return MHM_E_ARG;
  c->stream = static_cast<hipStream_t>(hip_stream);
  return MHM_OK;
}

const char* mhm_last_error(mhm_ctx c) { return c ? c->err.c_str() : g_err.c_str(); }

// The build passes the SHA-256 of the sources it compiles; the tag makes the
// same text findable in the library file without loading it.
#ifndef MHM_SOURCE_HASH
#define MHM_SOURCE_HASH "unstamped"
#endif
__attribute__((used)) static const char kSourceStamp[] = "MHM_SOURCE_SHA256=" MHM_SOURCE_HASH;

const char* mhm_source_hash(void) { return kSourceStamp + sizeof("MHM_SOURCE_SHA256=") - 1; }

mhm_status mhm_sync(mhm_ctx c) {
  if (!c) return MHM_E_ARG;
  hipError_t e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? MHM_OK : hip_fail(c, e, "hipStreamSynchronize");
}

size_t mhm_workspace_bytes(mhm_ctx c, const mhm_batch* b, mhm_prec prec) {
  if (!c || !b || b->n_elem <= 0 || b->s_max < 1 || b->s_max > MHM_S_LIMIT || b->s_min < 0 || b->s_min > b->s_max)
    return 0;
  const bool fp32 = prec == MHM_FP32_IR;
  return std::max(make_run_plan(c, b, fp32, true, nullptr).ws_total, make_run_plan(c, b, fp32, false, nullptr).ws_total);
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
  RunIO io;
  io.Ahat = Ahat_io;
  io.Btil = Btil;
  io.Lout = Ahat_io;
  io.X = X;
  io.info = info;
  io.ir_iters = ir_iters;
  io.max_iters = max_iters;
  return run_local(c, b, prec, false, io);
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
  mhm_status st = check_fused(c, b, prec, X, M, E, B, F, info);
  if (st != MHM_OK || b->n_elem == 0) return st;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  return run_local(c, b, prec, true, fused_io(X, M, E, B, F, info, ir_iters, max_iters));
}

mhm_status mhm_local_batch_run_noalloc(mhm_ctx c, const mhm_batch* b, mhm_prec prec, double* X, double* M,
                                       double* E, double* B, double* F, int32_t* info, int32_t* ir_iters,
                                       int max_iters) {
  mhm_status st = check_fused(c, b, prec, X, M, E, B, F, info);
  if (st != MHM_OK || b->n_elem == 0) return st;
  if (!c->scratch) return fail(c, MHM_E_DEVICE, "the scratch array of this device was not found at mhm_create");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  // The plan of mhm_local_batch_run, fitted into the scratch array: the
  // classes run one after another on the context's stream (no forked
  // streams), each from the end of the class lists, and a launch whose
  // workgroups each need a workspace slot gets only as many workgroups as
  // slots fit (the kernels are persistent, so fewer workgroups only take
  // longer).
  const bool fp32 = prec == MHM_FP32_IR;
  RunPlan rp = make_run_plan(c, b, fp32, true, nullptr);
  const size_t cap = MHM_NOALLOC_SCRATCH_BYTES;
  if (rp.list_bytes >= cap)
    return fail(c, MHM_E_ARG, "batch too large for mhm_local_batch_run_noalloc: its class lists need " +
                                  std::to_string(rp.list_bytes) + " of the " + std::to_string(cap) +
                                  " scratch bytes");
  const size_t avail = cap - rp.list_bytes;
  auto fit = [&](Plan& p, size_t tsz) -> bool {
    if (p.ws_slot <= 0) return true;
    const size_t per = (size_t)p.ws_slot * tsz;
    const size_t g = avail / per;
    if (g < 1) return false;
    p.grid = (int)std::min<size_t>((size_t)p.grid, g);
    p.ws_need = align_up((size_t)p.grid * per);
    return true;
  };
  for (int i = 0; i < rp.n_runs; ++i) {
    ClassRun& r = rp.run[i];
    const bool ok = fit(r.main, fp32 ? sizeof(float) : sizeof(double)) && (!r.has_fb || fit(r.fb, sizeof(double)));
    if (!ok)
      return fail(c, MHM_E_ARG, "elements with s up to " + std::to_string(r.s_cap) +
                                    " need a workspace slot larger than the scratch array's " +
                                    std::to_string(avail) + " bytes after the class lists");
    r.ws_off = rp.list_bytes;
  }
  return enqueue_run(c, rp, b, fused_io(X, M, E, B, F, info, ir_iters, max_iters), c->scratch, c->stream, false,
                     true);
}

mhm_status mhm_reconstruct(mhm_ctx c, const mhm_batch* b, const double* X, const int32_t* gdof, const int32_t* erow,
                           const double* sol, int32_t n_rows, double* u, const int32_t* info) {
  mhm_status st = check_batch(c, b, false, true);
  if (st != MHM_OK || b->n_elem == 0) return st;
  if (!X || !gdof || !erow || !sol || !u) return fail(c, MHM_E_ARG, "X, gdof, erow, sol and u are required");
  if (n_rows < 1) return fail(c, MHM_E_ARG, "n_rows < 1");
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = mhm::launch_reconstruct(b, X, gdof, erow, sol, n_rows, u, info, grid_for(b), c->stream);
  return e == hipSuccess ? MHM_OK : hip_fail(c, e, "k_reconstruct launch");
}

mhm_status mhm_skeleton_scatter(mhm_ctx c, const mhm_batch* b, const double* M, const double* E, const double* B,
                                const double* F, const int32_t* gdof, const int32_t* erow, const int32_t* row_ptr,
                                const int32_t* col_idx, int32_t n_rows, double* vals, double* rhs,
                                const int32_t* info, int32_t* missing) {
  mhm_status st = check_batch(c, b, false, false);
  if (st != MHM_OK || b->n_elem == 0) return st;
  if (!M || !E || !B || !F || !gdof || !erow || !row_ptr || !col_idx || !vals || !rhs)
    return fail(c, MHM_E_ARG, "M, E, B, F, gdof, erow, row_ptr, col_idx, vals and rhs are required");
  if (n_rows < 1) return fail(c, MHM_E_ARG, "n_rows < 1");
  hipError_t e = hipSetDevice(c->device);
  const int grid = std::min<int64_t>(kGridCap, 4 * c->n_cu);
  if (e == hipSuccess)
    e = mhm::launch_skeleton_scatter(b, M, E, B, F, gdof, erow, row_ptr, col_idx, n_rows, vals, rhs, info, missing,
                                     grid, c->stream);
  return e == hipSuccess ? MHM_OK : hip_fail(c, e, "k_skeleton_scatter launch");
}

mhm_status mhm_skeleton_solve(mhm_ctx c, int32_t n_rows, int32_t n_lambda, int32_t lambda_block,
                              const int32_t* row_ptr, const int32_t* col_idx, const double* vals, const double* rhs,
                              double* sol, double tol, int32_t max_iters, int32_t* iters, double* relres) {
  if (!c) return MHM_E_ARG;
  if (n_rows < 0 || n_lambda < 0 || n_lambda > n_rows) return fail(c, MHM_E_ARG, "need 0 <= n_lambda <= n_rows");
  if (lambda_block < 1 || lambda_block > mhm::skeleton_block_max() || (n_lambda % lambda_block) != 0)
    return fail(c, MHM_E_ARG, "lambda_block must be in [1, 8] and divide n_lambda");
  if (!(tol > 0.0) || max_iters < 0) return fail(c, MHM_E_ARG, "need tol > 0 and max_iters >= 0");
  if (iters) *iters = 0;
  if (relres) *relres = 0.0;
  if (n_rows == 0) return MHM_OK;
  if (!row_ptr || !col_idx || !vals || !rhs || !sol)
    return fail(c, MHM_E_ARG, "row_ptr, col_idx, vals, rhs and sol are required");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  mhm_status st = ensure_ws(c, mhm::skeleton_solve_bytes(n_rows, lambda_block));
  if (st != MHM_OK) return st;
  int bad = 0;
  e = mhm::skeleton_csr_check(n_rows, row_ptr, col_idx, c->ws, &bad, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "CSR check");
  if (bad) return fail(c, MHM_E_ARG, std::to_string(bad) + " row pointers or column indices out of range");
  std::vector<double> host_sc(64, 0.0);
  int it = 0;
  double rr = 0.0;
  e = mhm::skeleton_solve(n_rows, n_lambda, lambda_block, row_ptr, col_idx, vals, rhs, sol, tol, max_iters, c->ws,
                          host_sc.data(), &it, &rr, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "skeleton solve");
  if (iters) *iters = it;
  if (relres) *relres = rr;
  return MHM_OK;
}

size_t mhm_factor_bytes(int s, mhm_prec prec) {
  if (s < 1 || s > MHM_S_LIMIT) return 0;
  const int nt = (n_of(s) + 15) / 16;
  const size_t tsz = prec == MHM_FP32_IR ? sizeof(float) : sizeof(double);
  return align_up((size_t)(nt * (nt + 1) / 2) * mhm::TILE_WORDS * tsz);
}

mhm_status mhm_local_batch_run_cached(mhm_ctx c, const mhm_batch* b, mhm_prec prec, void* factors,
                                      const int64_t* factor_off, const int8_t* factor_state, double* X, double* M,
                                      double* E, double* B, double* F, int32_t* info, int32_t* ir_iters,
                                      int max_iters) {
  mhm_status st = check_fused(c, b, prec, X, M, E, B, F, info);
  if (st != MHM_OK || b->n_elem == 0) return st;
  if (!factors || !factor_off || !factor_state) return fail(c, MHM_E_ARG, "factors, factor_off and factor_state are required");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  RunIO io = fused_io(X, M, E, B, F, info, ir_iters, max_iters);
  io.fac = factors;
  io.fac_off = factor_off;
  io.fac_state = factor_state;
  return run_local(c, b, prec, true, io);
}

mhm_status mhm_local_source_step(mhm_ctx c, const mhm_batch* b, mhm_prec prec, const void* factors,
                                 const int64_t* factor_off, const int8_t* factor_state, double* X, double* M,
                                 double* E, double* B, double* F, int32_t* info, int32_t* ir_iters, int max_iters) {
  mhm_status st = check_batch(c, b, false, false);
  if (st != MHM_OK || b->n_elem == 0) return st;
  if (prec != MHM_FP64 && prec != MHM_FP32_IR) return fail(c, MHM_E_ARG, "unknown precision");
  const bool fp32 = prec == MHM_FP32_IR;
  if (!factors || !factor_off || !factor_state || !X || !E || !F || !info)
    return fail(c, MHM_E_ARG, "factors, factor_off, factor_state, X, E, F and info are required");
  if (fp32 && (!M || !B)) return fail(c, MHM_E_ARG, "M and B are required with MHM_FP32_IR (FP64 fallback)");
  if (b->s_max > 48) return fail(c, MHM_E_UNSUPPORTED, "stored factors need s <= 48");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  mhm::SourceArgs a;
  std::memset(&a, 0, sizeof(a));
  a.fac = factors;
  a.fac_off = factor_off;
  a.fac_state = factor_state;
  a.X = X;
  a.E = E;
  a.F = F;
  a.info = info;
  a.ir_iters = ir_iters;
  a.max_iters = std::max(0, max_iters);
  a.refine64 = c->refine64;
  a.ir_tol = kIrTol;
  a.n_cap = n_of(b->s_max);
  const size_t lds = mhm::source_step_lds(fp32, a.n_cap, a.wave_words);
  const int waves = mhm::source_step_waves();
  const int grid = (int)std::min<int64_t>(((int64_t)b->n_elem + waves - 1) / waves, kGridCap);
  e = mhm::launch_source_step(fp32, b, a, lds, grid, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "k_source_step launch");
  if (!fp32) return MHM_OK;
  // elements whose refinement did not converge: full FP64 recomputation
  RunIO io = fused_io(X, M, E, B, F, info, ir_iters, max_iters);
  const RunPlan rp = make_run_plan(c, b, true, true, nullptr, false);
  st = ensure_ws(c, rp.ws_total);
  if (st != MHM_OK) return st;
  return enqueue_run(c, rp, b, io, c->ws, c->stream, true);
}

mhm_status mhm_autotune(mhm_ctx c, const mhm_batch* b, mhm_prec prec, double* X, double* M, double* E, double* B,
                        double* F, int32_t* info, int32_t* ir_iters, int max_iters) {
  mhm_status st = check_fused(c, b, prec, X, M, E, B, F, info);
  if (st != MHM_OK || b->n_elem == 0) return st;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const bool fp32 = prec == MHM_FP32_IR;
  const RunIO io = fused_io(X, M, E, B, F, info, ir_iters, max_iters);
  for (int k = 0; k < kNumClasses; ++k) c->tuned[k][fp32][1] = Choice();
  const RunPlan base = make_run_plan(c, b, fp32, true, nullptr);
  // workspace: class lists, a tuning count, and the largest candidate slot set
  size_t need = 0;
  for (int i = 0; i < base.n_runs; ++i) {
    for (const Choice ch : {Choice{FAM_RR, 0, 1}, Choice{FAM_LDS, 0, 1}, Choice{FAM_LL, 2, 1}, Choice{FAM_LL, 4, 1},
                            Choice{FAM_LL, 2, 2}, Choice{FAM_LL, 2, 1, 16}, Choice{FAM_LL, 4, 1, 16},
                            Choice{FAM_WS, 0, 1}}) {
      const Plan p = plan_for(c, b, fp32, true, base.run[i].s_cap, ch, base.listed);
      if (p.ok) need = std::max(need, p.ws_need);
    }
    // the FP64 pass (FP32 recomputation, or the register-tile kernel's deferred elements)
    need = std::max(need, fallback_plan(c, b, base.run[i].s_cap, base.listed).ws_need);
  }
  const size_t cnt_off = base.list_bytes + need;
  st = ensure_ws(c, std::max(base.ws_total, cnt_off + kAlign));
  if (st != MHM_OK) return st;
  int32_t* dcount = reinterpret_cast<int32_t*>(static_cast<char*>(c->ws) + cnt_off);
  int counts[kNumClasses] = {};
  if (base.listed) {
    int32_t* lists = static_cast<int32_t*>(c->ws);
    e = mhm::launch_bin(b, bin_classes(), lists, lists + (size_t)kNumClasses * b->n_elem, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(counts, lists + (size_t)kNumClasses * b->n_elem, sizeof(counts), hipMemcpyDeviceToHost,
                         c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "binning for tuning");
  } else {
    counts[base.run[0].cls] = b->n_elem;
  }
  std::string log;
  for (int i = 0; i < base.n_runs && st == MHM_OK; ++i) {
    const int k = base.run[i].cls;
    if (counts[k] == 0) continue;
    const Choice best = tune_class(c, b, fp32, base, i, io, dcount, 4 * c->n_cu, counts[k], log, st);
    c->tuned[k][fp32][1] = best;
  }
  c->tune_log = "[" + log + "]";
  if (st != MHM_OK) return st;
  return run_local(c, b, prec, true, io);   // leaves the outputs of the tuned run
}

size_t mhm_tune_report(mhm_ctx c, char* buf, size_t len) {
  if (!c) return 0;
  if (buf && len > 0) {
    const size_t k = std::min(len - 1, c->tune_log.size());
    std::memcpy(buf, c->tune_log.data(), k);
    buf[k] = '\0';
  }
  return c->tune_log.size() + 1;
}

mhm_status mhm_graph_create(mhm_ctx c, const mhm_batch* b, mhm_prec prec, double* X, double* M, double* E, double* B,
                            double* F, int32_t* info, int32_t* ir_iters, int max_iters, mhm_graph* out) {
  if (!out) return fail(c, MHM_E_ARG, "graph is NULL");
  *out = nullptr;
  mhm_status st = check_fused(c, b, prec, X, M, E, B, F, info);
  if (st != MHM_OK) return st;
  if (b->n_elem == 0) return fail(c, MHM_E_ARG, "empty batch");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const RunPlan rp = make_run_plan(c, b, prec == MHM_FP32_IR, true, nullptr);
  if (rp.n_runs > 1) {
    st = ensure_streams(c);
    if (st != MHM_OK) return st;
  }
  mhm_graph g = new mhm_graph_s();
  g->ctx = c;
  if (rp.ws_total > 0) {
    e = hipMalloc(&g->ws, rp.ws_total);
    if (e != hipSuccess) {
      delete g;
      return fail(c, MHM_E_NOMEM, "hipMalloc of the graph workspace failed");
    }
  }
  hipStream_t cs = nullptr;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    const bool timing = c->class_timing;   // no timing events inside a captured graph
    c->class_timing = false;
    st = enqueue_run(c, rp, b, fused_io(X, M, E, B, F, info, ir_iters, max_iters), g->ws, cs);
    c->class_timing = timing;
    const hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
    if (st == MHM_OK && e2 != hipSuccess) st = hip_fail(c, e2, "hipStreamEndCapture");
    if (st == MHM_OK) {
      e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) st = hip_fail(c, e, "hipGraphInstantiate");
    }
  } else {
    st = hip_fail(c, e, "hipStreamBeginCapture");
  }
  if (cs) (void)hipStreamDestroy(cs);
  if (st != MHM_OK) {
    mhm_graph_destroy(g);
    return st;
  }
  *out = g;
  return MHM_OK;
}

mhm_status mhm_graph_launch(mhm_graph g) {
  if (!g || !g->exec) return MHM_E_ARG;
  mhm_ctx c = g->ctx;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipGraphLaunch(g->exec, c->stream);
  return e == hipSuccess ? MHM_OK : hip_fail(c, e, "hipGraphLaunch");
}

mhm_status mhm_graph_destroy(mhm_graph g) {
  if (!g) return MHM_E_ARG;
  mhm_ctx c = g->ctx;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->ws) (void)hipFree(g->ws);
  delete g;
  return MHM_OK;
}

}  // extern "C"
