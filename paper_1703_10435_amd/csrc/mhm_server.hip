// Serving runtime for local problems that arrive one by one (host code).
//
// Requests are queued by mhm_server_submit*.  A worker thread keeps up to
// `in_flight` launches on the device, each on its own stream and context
// (own workspace): whenever a launch slot is free it takes the requests
// queued so far (continuous batching, arrival order), packs them into one
// ragged batch in pinned host memory, copies it to the device and runs
// mhm_local_batch_run_cached on it.  Factors stay on the device in an LRU
// cache keyed by the caller's content key, so a repeated (geometry, s,
// kappa) solves only its new right-hand sides (Section 3: one factorisation,
// many load vectors).  Everything the server allocates on the device -
// per-slot buffers, workspaces and the factor arena - stays within the
// configured HBM budget; when the arena has no room left after evicting
// every unpinned factor, requests wait in the queue until running launches
// finish (admission by memory).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/mhm.h"
#include "mhm_server_core.h"

namespace {

using mhm_srv::Key;
using mhm_srv::n_of;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
size_t up256(size_t x) { return (x + 255) / 256 * 256; }

struct Req {
  uint64_t ticket;
  Key key;
  bool keyed;
  int s, l;
  double vert[6];
  int8_t sigma[3], flip[3];
  std::vector<double> kappa, f;
  double t_arrival;
};

// Host (pinned) and device buffers of one launch slot, sized for the
// configured maximum batch.
struct Slot {
  mhm_ctx ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  char* h = nullptr;   // pinned staging of inputs and outputs
  char* d = nullptr;   // device copy
  size_t in_bytes = 0, out_bytes = 0;
  std::vector<Req> reqs;
  mhm_srv::Admitted adm;   // factor state, offset and entry of each request
  // layout (byte offsets into h / d)
  size_t o_s, o_l, o_vert, o_sig, o_flip, o_kap, o_f, o_tri, o_rhs, o_foff, o_fst;
  size_t o_X, o_M, o_E, o_B, o_F, o_info, o_it;
  int l_max = 0;
};

}  // namespace

struct mhm_server_s {
  mhm_server_config cfg;
  int device = 0;
  std::vector<Slot> slots;
  char* arena = nullptr;
  mhm_srv::Cache cache;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req> queue;
  std::vector<mhm_result> done;
  std::vector<std::vector<double>> done_data;   // storage of the results handed out
  std::vector<mhm_result> handed;
  std::vector<std::vector<double>> handed_data;
  std::atomic<bool> stop{false};
  std::thread worker;
  uint64_t next_ticket = 1;
  mhm_server_stats stats = {};
  std::string err;
  // per-slot capacities
  int64_t cap_tri = 0, cap_rhs = 0;
};

namespace {

mhm_status set_err(mhm_server srv, mhm_status st, const std::string& m) {
  srv->err = m;
  return st;
}

void layout(Slot& sl, int B, int64_t cap_tri, int64_t cap_rhs, int NI) {
  size_t o = 0;
  auto put = [&](size_t bytes) {
    const size_t at = o;
    o = up256(o + bytes);
    return at;
  };
  sl.o_s = put(4 * (size_t)B);
  sl.o_l = put(4 * (size_t)B);
  sl.o_vert = put(48 * (size_t)B);
  sl.o_sig = put(3 * (size_t)B);
  sl.o_flip = put(3 * (size_t)B);
  sl.o_kap = put(8 * (size_t)cap_tri);
  sl.o_f = put(8 * (size_t)cap_tri);
  sl.o_tri = put(8 * (size_t)(B + 1));
  sl.o_rhs = put(8 * (size_t)(B + 1));
  sl.o_foff = put(8 * (size_t)B);
  sl.o_fst = put((size_t)B);
  sl.in_bytes = o;
  sl.o_X = put(8 * (size_t)cap_rhs);
  sl.o_M = put(8 * (size_t)B * NI * NI);
  sl.o_E = put(8 * (size_t)B * NI);
  sl.o_B = put(8 * (size_t)B * NI);
  sl.o_F = put(8 * (size_t)B);
  sl.o_info = put(4 * (size_t)B);
  sl.o_it = put(4 * (size_t)B);
  sl.out_bytes = o - sl.in_bytes;
}

// Every request of a launch that could not run completes at once with info
// MHM_INFO_LAUNCH_FAILED and NaN outputs; the factors it created are
// dropped, never marked valid.  Caller holds the lock.
void fail_launch(mhm_server srv, Slot& sl) {
  (void)hipStreamSynchronize(sl.stream);   // the staging buffer may still be read by a copy
  (void)hipGetLastError();
  const double t = now_s();
  for (size_t k = 0; k < sl.reqs.size(); ++k) {
    const Req& q = sl.reqs[k];
    const int n = n_of(q.s), ni = 3 * (q.l + 1), r = ni + 1;
    mhm_result res;
    std::memset(&res, 0, sizeof(res));
    res.ticket = q.ticket;
    res.info = MHM_INFO_LAUNCH_FAILED;
    res.cache_hit = sl.adm.state[k] == 1;
    res.s = q.s;
    res.l = q.l;
    res.n = n;
    res.r = r;
    res.t_arrival = q.t_arrival;
    res.t_done = t;
    srv->done.push_back(res);
    srv->done_data.emplace_back((size_t)n * r + (size_t)ni * ni + 2 * ni + 1, __builtin_nan(""));
    mhm_srv::settle(srv->cache, sl.adm, k, false, res.info);
    srv->stats.completed++;
  }
  sl.reqs.clear();
  sl.busy = false;
}

// Launch the queued requests on a free slot.  Caller holds the lock.
bool launch(mhm_server srv, Slot& sl) {
  const mhm_server_config& c = srv->cfg;
  const mhm_srv::Limits lim{c.max_batch, srv->cap_tri, srv->cap_rhs, c.reuse != 0};
  mhm_srv::admit(srv->cache, srv->queue, lim, [&](int s) { return mhm_factor_bytes(s, (mhm_prec)c.prec); },
                 sl.reqs, sl.adm);
  srv->stats.cache_hits += sl.adm.hits;
  const int B = (int)sl.reqs.size();
  if (B == 0) return false;
  // pack
  char* h = sl.h;
  int32_t* hs = reinterpret_cast<int32_t*>(h + sl.o_s);
  int32_t* hl = reinterpret_cast<int32_t*>(h + sl.o_l);
  double* hv = reinterpret_cast<double*>(h + sl.o_vert);
  int8_t* hsg = reinterpret_cast<int8_t*>(h + sl.o_sig);
  int8_t* hfl = reinterpret_cast<int8_t*>(h + sl.o_flip);
  double* hk = reinterpret_cast<double*>(h + sl.o_kap);
  double* hf = reinterpret_cast<double*>(h + sl.o_f);
  int64_t* htri = reinterpret_cast<int64_t*>(h + sl.o_tri);
  int64_t* hrhs = reinterpret_cast<int64_t*>(h + sl.o_rhs);
  int64_t* hfo = reinterpret_cast<int64_t*>(h + sl.o_foff);
  int8_t* hst = reinterpret_cast<int8_t*>(h + sl.o_fst);
  int s_max = 1, s_min = 64, l_max = 0;
  htri[0] = 0;
  hrhs[0] = 0;
  for (int e = 0; e < B; ++e) {
    const Req& q = sl.reqs[e];
    hs[e] = q.s;
    hl[e] = q.l;
    std::memcpy(hv + 6 * e, q.vert, sizeof(q.vert));
    std::memcpy(hsg + 3 * e, q.sigma, 3);
    std::memcpy(hfl + 3 * e, q.flip, 3);
    std::memcpy(hk + htri[e], q.kappa.data(), sizeof(double) * q.s * q.s);
    std::memcpy(hf + htri[e], q.f.data(), sizeof(double) * q.s * q.s);
    htri[e + 1] = htri[e] + (int64_t)q.s * q.s;
    hrhs[e + 1] = hrhs[e] + (int64_t)n_of(q.s) * (3 * (q.l + 1) + 1);
    hfo[e] = (int64_t)sl.adm.foff[e];
    hst[e] = sl.adm.state[e];
    s_max = std::max(s_max, q.s);
    s_min = std::min(s_min, q.s);
    l_max = std::max(l_max, q.l);
  }
  sl.l_max = l_max;
  hipError_t e = hipMemcpyAsync(sl.d, sl.h, sl.in_bytes, hipMemcpyHostToDevice, sl.stream);
  mhm_batch b;
  std::memset(&b, 0, sizeof(b));
  b.n_elem = B;
  b.s_max = s_max;
  b.s_min = s_min;
  b.l_max = l_max;
  char* d = sl.d;
  b.s = reinterpret_cast<const int32_t*>(d + sl.o_s);
  b.l = reinterpret_cast<const int32_t*>(d + sl.o_l);
  b.vert = reinterpret_cast<const double*>(d + sl.o_vert);
  b.sigma = reinterpret_cast<const int8_t*>(d + sl.o_sig);
  b.flip = reinterpret_cast<const int8_t*>(d + sl.o_flip);
  b.kappa = reinterpret_cast<const double*>(d + sl.o_kap);
  b.f = reinterpret_cast<const double*>(d + sl.o_f);
  b.tri_off = reinterpret_cast<const int64_t*>(d + sl.o_tri);
  b.rhs_off = reinterpret_cast<const int64_t*>(d + sl.o_rhs);
  b.tri_total = htri[B];
  b.rhs_total = hrhs[B];
  mhm_status st = MHM_OK;
  if (e == hipSuccess) {
    st = mhm_local_batch_run_cached(
        sl.ctx, &b, (mhm_prec)c.prec, srv->arena, reinterpret_cast<const int64_t*>(d + sl.o_foff),
        reinterpret_cast<const int8_t*>(d + sl.o_fst), reinterpret_cast<double*>(d + sl.o_X),
        reinterpret_cast<double*>(d + sl.o_M), reinterpret_cast<double*>(d + sl.o_E),
        reinterpret_cast<double*>(d + sl.o_B), reinterpret_cast<double*>(d + sl.o_F),
        reinterpret_cast<int32_t*>(d + sl.o_info), reinterpret_cast<int32_t*>(d + sl.o_it), c.max_iters);
  }
  // results back: X up to this batch's size, then the fixed blocks
  if (e == hipSuccess && st == MHM_OK)
    e = hipMemcpyAsync(h + sl.o_X, d + sl.o_X, 8 * (size_t)hrhs[B], hipMemcpyDeviceToHost, sl.stream);
  if (e == hipSuccess && st == MHM_OK)
    e = hipMemcpyAsync(h + sl.o_M, d + sl.o_M, sl.in_bytes + sl.out_bytes - sl.o_M, hipMemcpyDeviceToHost,
                       sl.stream);
  if (e == hipSuccess && st == MHM_OK) e = hipEventRecord(sl.done, sl.stream);
  srv->stats.launches++;
  srv->stats.max_batch_seen = std::max<int64_t>(srv->stats.max_batch_seen, B);
  if (e != hipSuccess || st != MHM_OK) {
    srv->err = st != MHM_OK ? std::string(mhm_last_error(sl.ctx)) : std::string(hipGetErrorString(e));
    srv->stats.errors++;
    fail_launch(srv, sl);
    return true;
  }
  sl.busy = true;
  return true;
}

// Collect a finished slot's results.  Caller holds the lock.
void harvest(mhm_server srv, Slot& sl) {
  const double t = now_s();
  const char* h = sl.h;
  const int NI = 3 * (sl.l_max + 1);
  const int64_t* hrhs = reinterpret_cast<const int64_t*>(h + sl.o_rhs);
  const double* X = reinterpret_cast<const double*>(h + sl.o_X);
  const double* M = reinterpret_cast<const double*>(h + sl.o_M);
  const double* E = reinterpret_cast<const double*>(h + sl.o_E);
  const double* Bv = reinterpret_cast<const double*>(h + sl.o_B);
  const double* F = reinterpret_cast<const double*>(h + sl.o_F);
  const int32_t* info = reinterpret_cast<const int32_t*>(h + sl.o_info);
  const int32_t* its = reinterpret_cast<const int32_t*>(h + sl.o_it);
  for (size_t k = 0; k < sl.reqs.size(); ++k) {
    const Req& q = sl.reqs[k];
    const int n = n_of(q.s), ni = 3 * (q.l + 1), r = ni + 1;
    mhm_result res;
    std::memset(&res, 0, sizeof(res));
    res.ticket = q.ticket;
    res.info = info[k];
    res.ir_iters = its[k];
    res.cache_hit = sl.adm.state[k] == 1;
    res.s = q.s;
    res.l = q.l;
    res.n = n;
    res.r = r;
    res.t_arrival = q.t_arrival;
    res.t_done = t;
    std::vector<double> data((size_t)n * r + (size_t)ni * ni + 2 * ni + 1);
    std::memcpy(data.data(), X + hrhs[k], sizeof(double) * n * r);
    double* m = data.data() + (size_t)n * r;
    for (int j = 0; j < ni; ++j)
      for (int i = 0; i < ni; ++i) m[i + ni * j] = M[(size_t)k * NI * NI + i + (size_t)NI * j];
    for (int i = 0; i < ni; ++i) {
      m[ni * ni + i] = E[(size_t)k * NI + i];
      m[ni * ni + ni + i] = Bv[(size_t)k * NI + i];
    }
    m[ni * ni + 2 * ni] = F[k];
    srv->done.push_back(res);
    srv->done_data.push_back(std::move(data));
    mhm_srv::settle(srv->cache, sl.adm, k, true, res.info);
    srv->stats.completed++;
    if (res.info == -1) srv->stats.ir_fallbacks++;
  }
  sl.reqs.clear();
  sl.busy = false;
}

void worker_loop(mhm_server srv) {
  (void)hipSetDevice(srv->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  while (!srv->stop.load()) {
    bool progress = false;
    for (Slot& sl : srv->slots) {
      if (sl.busy && hipEventQuery(sl.done) == hipSuccess) {
        harvest(srv, sl);
        progress = true;
      }
    }
    for (Slot& sl : srv->slots) {
      if (!sl.busy && !srv->queue.empty()) {
        if (launch(srv, sl)) progress = true;
        else break;   // nothing admissible now
      }
    }
    if (!progress) {
      const bool any_busy = std::any_of(srv->slots.begin(), srv->slots.end(), [](const Slot& s) { return s.busy; });
      if (any_busy) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else {
        srv->cv.wait_for(lk, std::chrono::milliseconds(2));
      }
    }
  }
}

}  // namespace

extern "C" {

double mhm_server_now(void) { return now_s(); }

mhm_status mhm_server_create(int device, const mhm_server_config* cfg, mhm_server* out) {
  if (!out || !cfg) return MHM_E_ARG;
  *out = nullptr;
  if (cfg->prec != MHM_FP64 && cfg->prec != MHM_FP32_IR) return MHM_E_ARG;
  if (cfg->max_batch < 1 || cfg->max_batch > 65536 || cfg->in_flight < 1 || cfg->in_flight > 8) return MHM_E_ARG;
  if (cfg->s_max < 1 || cfg->s_max > 48 || cfg->l_max < 0 || cfg->l_max > MHM_L_LIMIT) return MHM_E_UNSUPPORTED;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return MHM_E_DEVICE;
  mhm_server srv = new mhm_server_s();
  srv->cfg = *cfg;
  srv->device = device;
  const int B = cfg->max_batch;
  const int NI = 3 * (cfg->l_max + 1);
  srv->cap_tri = (int64_t)B * cfg->s_max * cfg->s_max;
  srv->cap_rhs = (int64_t)B * n_of(cfg->s_max) * (NI + 1);
  size_t fixed = 0;
  srv->slots.resize(cfg->in_flight);
  mhm_status st = MHM_OK;
  for (Slot& sl : srv->slots) {
    layout(sl, B, srv->cap_tri, srv->cap_rhs, NI);
    const size_t bytes = sl.in_bytes + sl.out_bytes;
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.h), bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&sl.d), bytes) != hipSuccess) {
      st = MHM_E_NOMEM;
      break;
    }
    st = mhm_create(&sl.ctx, device, sl.stream);
    if (st != MHM_OK) break;
    // buffers plus an upper bound of the context's workspace (a full batch
    // of the largest elements, including the FP64 recomputation pass)
    mhm_batch wb;
    std::memset(&wb, 0, sizeof(wb));
    wb.n_elem = B;
    wb.s_max = cfg->s_max;
    wb.s_min = 1;
    wb.l_max = cfg->l_max;
    fixed += bytes + mhm_workspace_bytes(sl.ctx, &wb, (mhm_prec)cfg->prec);
  }
  if (st == MHM_OK) {
    if (cfg->hbm_budget <= fixed) {
      st = MHM_E_NOMEM;
    } else {
      const size_t arena = std::min<size_t>(cfg->hbm_budget - fixed, cfg->factor_cache_max ? cfg->factor_cache_max
                                                                                              : cfg->hbm_budget);
      if (hipMalloc(reinterpret_cast<void**>(&srv->arena), arena) != hipSuccess) st = MHM_E_NOMEM;
      else srv->cache.init(arena);
      srv->stats.arena_bytes = (int64_t)arena;
      srv->stats.fixed_bytes = (int64_t)fixed;
    }
  }
  if (st != MHM_OK) {
    mhm_server_destroy(srv);
    return st;
  }
  srv->worker = std::thread(worker_loop, srv);
  *out = srv;
  return MHM_OK;
}

mhm_status mhm_server_submit(mhm_server srv, const mhm_request* reqs, int n, uint64_t* tickets) {
  if (!srv || (n > 0 && !reqs)) return MHM_E_ARG;
  std::vector<Req> in;
  in.reserve(n);
  for (int k = 0; k < n; ++k) {
    const mhm_request& r = reqs[k];
    if (r.s < 1 || r.s > srv->cfg.s_max || r.l < 0 || r.l > srv->cfg.l_max || !r.kappa || !r.f)
      return set_err(srv, MHM_E_ARG, "request " + std::to_string(k) + " outside the server's s/l limits");
    Req q;
    q.key = Key{r.key_hi, r.key_lo};
    q.keyed = r.key_hi != 0 || r.key_lo != 0;
    q.s = r.s;
    q.l = r.l;
    std::memcpy(q.vert, r.vert, sizeof(q.vert));
    std::memcpy(q.sigma, r.sigma, 3);
    std::memcpy(q.flip, r.flip, 3);
    q.kappa.assign(r.kappa, r.kappa + (size_t)r.s * r.s);
    q.f.assign(r.f, r.f + (size_t)r.s * r.s);
    q.t_arrival = r.t_arrival;
    in.push_back(std::move(q));
  }
  {
    std::lock_guard<std::mutex> g(srv->mu);
    for (int k = 0; k < n; ++k) {
      in[k].ticket = srv->next_ticket++;
      if (tickets) tickets[k] = in[k].ticket;
      srv->queue.push_back(std::move(in[k]));
    }
    srv->stats.submitted += n;
  }
  srv->cv.notify_one();
  return MHM_OK;
}

int mhm_server_poll(mhm_server srv, mhm_result* out, int max) {
  if (!srv || max < 0) return -1;
  std::lock_guard<std::mutex> g(srv->mu);
  srv->handed.clear();
  srv->handed_data.clear();
  const int k = std::min<int>(max, (int)srv->done.size());
  for (int i = 0; i < k; ++i) {
    srv->handed.push_back(srv->done[i]);
    srv->handed_data.push_back(std::move(srv->done_data[i]));
  }
  srv->done.erase(srv->done.begin(), srv->done.begin() + k);
  srv->done_data.erase(srv->done_data.begin(), srv->done_data.begin() + k);
  for (int i = 0; i < k; ++i) {
    mhm_result r = srv->handed[i];
    const double* p = srv->handed_data[i].data();
    const int ni = r.r - 1;
    r.X = p;
    r.M = p + (size_t)r.n * r.r;
    r.E = r.M + (size_t)ni * ni;
    r.B = r.E + ni;
    r.F = r.B[ni];
    out[i] = r;
  }
  return k;
}

mhm_status mhm_server_stats_get(mhm_server srv, mhm_server_stats* st) {
  if (!srv || !st) return MHM_E_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  srv->stats.queued = (int64_t)srv->queue.size();
  srv->stats.cache_entries = (int64_t)srv->cache.map.size();
  srv->stats.cache_bytes = (int64_t)srv->cache.used;
  srv->stats.cache_evictions = (int64_t)srv->cache.evictions;
  *st = srv->stats;
  return MHM_OK;
}

const char* mhm_server_last_error(mhm_server srv) { return srv ? srv->err.c_str() : ""; }

mhm_status mhm_server_destroy(mhm_server srv) {
  if (!srv) return MHM_E_ARG;
  srv->stop.store(true);
  srv->cv.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  (void)hipSetDevice(srv->device);
  for (Slot& sl : srv->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.ctx) mhm_destroy(sl.ctx);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h) (void)hipHostFree(sl.h);
    if (sl.d) (void)hipFree(sl.d);
  }
  if (srv->arena) (void)hipFree(srv->arena);
  delete srv;
  return MHM_OK;
}

}  // extern "C"
