// Serving runtime: many live tuning sessions, BO step requests arriving at
// any time.  Each request appends one evaluation to its session (a rank-1
// extension of the device-resident factor, or a visited mark only for an
// evaluation that failed) and runs the posterior, acquisitions and selection.
//
//  - Memory admission: a session's device state (workspace, observation
//    arrays, visited mask) is allocated when it fits in the HBM budget; until
//    then the session waits, and so do its requests.  Closing a session
//    returns its memory and admits waiting sessions in arrival order.  A
//    setup thread allocates, uploads and fits admitted sessions and frees
//    closed ones, outside the scheduler's lock and on streams that do not
//    wait for the launches, so admissions never stall the launches.
//  - Continuous batching: a scheduler thread gathers the pending requests of
//    idle sessions (one in flight per session, oldest first) into a launch of
//    the batched step graph, on whichever of the server's launch
//    contexts (one stream each) is free.  Requests that arrive while launches
//    run join the next launch as soon as a context frees up, so launches
//    overlap on the device.
//  - Latency is measured from submission to the moment the scheduler has the
//    result.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "batch_ctx.h"
#include "bo_internal.h"
#include "session_impl.h"

using namespace bo;

namespace {

using Clock = std::chrono::steady_clock;

struct SrvSession {
  int32_t id = -1;
  bo_problem prob{};
  bo_gp_params gp{};
  std::vector<int32_t> levels;
  std::vector<int64_t> cand;
  std::vector<uint8_t> invalid;
  std::vector<int64_t> obs0;
  std::vector<double> y0;
  size_t bytes = 0;
  void* dev = nullptr;
  bo_session* s = nullptr;
  int64_t* obs_dev = nullptr;
  double* y_dev = nullptr;
  uint8_t* vis_dev = nullptr;
  int32_t n = 0;
  int state = 0;  // 0 waiting for memory, 1 resident, 2 closing, 3 setup failed, 4 being set up
  bool close_requested = false;  // closed while being set up
  bool reserved = false;         // its bytes are counted in the server's `used`
  bool busy = false;
  bool need_refit = false;
  int32_t setup_status = BO_OK;
};

struct Request {
  int32_t sid = -1;
  int64_t idx = 0;
  double y = 0.0;
  int32_t valid = 1;
  AcqArgs acq{};
  Clock::time_point t_submit, t_launch, t_done;
  bo_acq_result res{};
  bool done = false;
  int32_t n_new = 0;
};

struct Launch {
  BatchCtx ctx;
  bool busy = false;
  std::vector<uint64_t> tickets;
  std::vector<BatchItem> items;
  std::vector<bo_acq_result> out;
};

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

struct bo_server {
  struct Freed {
    void* dev;
    bo_session* s;
    size_t bytes;
  };
  bo_server_config cfg{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work;   // new requests / sessions / stop
  std::condition_variable cv_done;   // results / admissions
  std::condition_variable cv_setup;  // sessions to set up / memory to free / stop
  std::deque<int32_t> setup_q;       // admitted sessions (state 4) to set up
  std::vector<Freed> free_q;         // memory of closed sessions, still counted in `used`
  std::deque<uint64_t> completed;    // finished tickets, in order of completion
  std::vector<hipStream_t> launch_streams;
  void* staging = nullptr;           // setup thread's device staging buffer
  size_t staging_bytes = 0;
  std::map<int32_t, std::unique_ptr<SrvSession>> sessions;
  std::deque<int32_t> waiting;      // sessions waiting for memory, in arrival order
  std::map<uint64_t, Request> reqs;
  std::deque<uint64_t> pending;     // submitted, not launched, in arrival order
  std::vector<std::unique_ptr<Launch>> launches;
  void* ctx_mem = nullptr;
  hipStream_t setup_stream = nullptr;
  size_t used = 0;
  int32_t next_id = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  std::thread setup_worker;
  int64_t steps_done = 0, n_launches = 0, items_launched = 0;
  // latency decomposition: submission to launch call (summed over requests),
  // host time of the launch calls, device time of the launches
  double wait_s = 0.0, launch_s = 0.0, gpu_ms = 0.0;
  int64_t gpu_timed = 0;
};

namespace {

size_t session_bytes(const bo_problem& p, size_t* ws) {
  size_t w = 0;
  if (bo_workspace_query(&p, &w) != BO_OK) return 0;
  *ws = w;
  return a256(w) + a256(sizeof(int64_t) * p.n_max) + a256(sizeof(double) * p.n_max) + a256((size_t)p.N);
}

// Frees a session's device state at once (server teardown).
void free_session_memory(bo_server* srv, SrvSession* ss) {
  if (ss->s) bo_session_destroy(ss->s);
  ss->s = nullptr;
  if (ss->dev) (void)hipFree(ss->dev);
  ss->dev = nullptr;
  if (ss->reserved) srv->used -= ss->bytes;
  ss->reserved = false;
}

// Hands a session's device state and its reserved bytes to the setup thread,
// which frees the memory and then returns the bytes to the budget.  Lock held.
void defer_free(bo_server* srv, SrvSession* ss) {
  if (ss->s || ss->dev || ss->reserved) {
    srv->free_q.push_back(bo_server::Freed{ss->dev, ss->s, ss->reserved ? ss->bytes : 0});
    srv->cv_setup.notify_all();
  }
  ss->s = nullptr;
  ss->dev = nullptr;
  ss->reserved = false;
}

// Allocates and initializes a session's device state (the candidate set, the
// initial observations and their fit) on the setup stream.  Runs on the setup
// thread without the server lock: nothing else touches the session while it
// is being set up (state 4).
int32_t setup_session(bo_server* srv, SrvSession* ss) {
  size_t ws = 0;
  session_bytes(ss->prob, &ws);
  hipStream_t st = srv->setup_stream;
  hipError_t e = hipMalloc(&ss->dev, ss->bytes);
  if (e != hipSuccess) {
    ss->dev = nullptr;
    return set_error(BO_E_HIP, "session memory: %s", hipGetErrorString(e));
  }
  unsigned char* p = (unsigned char*)ss->dev;
  void* wsp = p;
  p += a256(ws);
  ss->obs_dev = (int64_t*)p;
  p += a256(sizeof(int64_t) * ss->prob.n_max);
  ss->y_dev = (double*)p;
  p += a256(sizeof(double) * ss->prob.n_max);
  ss->vis_dev = (uint8_t*)p;
  bo_status rc = bo_session_create(&ss->s, &ss->prob, &ss->gp, wsp, ws, st);
  if (rc != BO_OK) return rc;
  // candidate list through the setup thread's staging buffer, restriction
  // mask through the visited array's space; the visited mask is written after
  const int64_t N = ss->prob.N;
  const size_t cand_bytes = ss->cand.empty() ? 0 : sizeof(int64_t) * N;
  if (cand_bytes > srv->staging_bytes) {
    if (srv->staging) (void)hipFree(srv->staging);
    srv->staging = nullptr;
    srv->staging_bytes = 0;
    e = hipMalloc(&srv->staging, cand_bytes);
    if (e != hipSuccess) return set_error(BO_E_HIP, "staging: %s", hipGetErrorString(e));
    srv->staging_bytes = cand_bytes;
  }
  e = hipSuccess;
  if (cand_bytes) e = hipMemcpyAsync(srv->staging, ss->cand.data(), cand_bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !ss->invalid.empty())
    e = hipMemcpyAsync(ss->vis_dev, ss->invalid.data(), (size_t)N, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return set_error(BO_E_HIP, "staging copy: %s", hipGetErrorString(e));
  rc = bo_set_grid(ss->s, ss->levels.data(), cand_bytes ? (const int64_t*)srv->staging : nullptr,
                   ss->invalid.empty() ? nullptr : ss->vis_dev, nullptr);
  if (rc != BO_OK) return rc;
  std::vector<uint8_t> vis((size_t)N, 0);
  for (int64_t i : ss->obs0)
    if (i >= 0 && i < N) vis[(size_t)i] = 1;
  e = hipMemcpyAsync(ss->vis_dev, vis.data(), (size_t)N, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ss->obs_dev, ss->obs0.data(), sizeof(int64_t) * ss->obs0.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ss->y_dev, ss->y0.data(), sizeof(double) * ss->y0.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host vectors go out of scope below
  if (e != hipSuccess) return set_error(BO_E_HIP, "initial observations: %s", hipGetErrorString(e));
  ss->n = (int32_t)ss->obs0.size();
  rc = bo_gp_fit(ss->s, ss->obs_dev, ss->y_dev, ss->n);
  if (rc != BO_OK) return rc;
  bo_fit_info info;
  rc = bo_fit_read(ss->s, &info, nullptr, nullptr);
  if (rc != BO_OK) ss->need_refit = true;  // reported by the session's first step
  ss->levels.clear();
  ss->levels.shrink_to_fit();
  ss->cand.clear();
  ss->cand.shrink_to_fit();
  ss->invalid.clear();
  ss->invalid.shrink_to_fit();
  return BO_OK;
}

// Admits waiting sessions in arrival order while they fit: their memory is
// reserved and the setup thread sets them up.  Lock held.
void admit(bo_server* srv) {
  while (!srv->waiting.empty()) {
    auto it = srv->sessions.find(srv->waiting.front());
    if (it == srv->sessions.end()) {
      srv->waiting.pop_front();
      continue;
    }
    SrvSession* ss = it->second.get();
    if (srv->used + ss->bytes > srv->cfg.hbm_budget) break;
    srv->waiting.pop_front();
    srv->used += ss->bytes;
    ss->reserved = true;
    ss->state = 4;
    srv->setup_q.push_back(ss->id);
    srv->cv_setup.notify_all();
  }
}

void setup_main(bo_server* srv) {
  (void)hipSetDevice(srv->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    srv->cv_setup.wait(lk, [&] { return srv->stop || !srv->setup_q.empty() || !srv->free_q.empty(); });
    if (srv->stop) break;
    if (!srv->free_q.empty()) {
      std::vector<bo_server::Freed> f;
      f.swap(srv->free_q);
      lk.unlock();
      for (auto& x : f) {
        if (x.s) bo_session_destroy(x.s);
        if (x.dev) (void)hipFree(x.dev);
      }
      lk.lock();
      for (auto& x : f) srv->used -= x.bytes;
      admit(srv);
      srv->cv_work.notify_all();
      continue;
    }
    const int32_t id = srv->setup_q.front();
    srv->setup_q.pop_front();
    auto it = srv->sessions.find(id);
    if (it == srv->sessions.end()) continue;
    SrvSession* ss = it->second.get();
    lk.unlock();
    const int32_t rc = setup_session(srv, ss);
    lk.lock();
    if (rc != BO_OK) {
      defer_free(srv, ss);
      ss->state = 3;
      ss->setup_status = rc;
    } else {
      ss->state = 1;
    }
    if (ss->close_requested) ss->state = 2;
    srv->cv_work.notify_all();
    srv->cv_done.notify_all();
  }
}

void fail_request(bo_server* srv, uint64_t t, int32_t status) {
  Request& r = srv->reqs[t];
  bo_acq_result z{};
  for (int k = 0; k < 3; ++k) {
    z.idx[k] = -1;
    z.score[k] = __builtin_nan("");
  }
  z.status = status;
  r.res = z;
  r.done = true;
  r.t_done = Clock::now();
  srv->completed.push_back(t);
}

// Collects finished launches.  Lock held.
void retire(bo_server* srv) {
  for (auto& L : srv->launches) {
    if (!L->busy || !L->ctx.done()) continue;
    const int cnt = (int)L->tickets.size();
    L->out.resize(cnt);
    float ms = -1.f;
    const bo_status rc = L->ctx.finish(L->out.data(), &ms);
    if (ms >= 0.f) {
      srv->gpu_ms += ms;
      ++srv->gpu_timed;
    }
    const auto now = Clock::now();
    for (int i = 0; i < cnt; ++i) {
      Request& r = srv->reqs[L->tickets[i]];
      SrvSession* ss = srv->sessions[r.sid].get();
      r.res = L->out[i];
      if (rc != BO_OK) r.res.status = rc;
      r.done = true;
      r.t_done = now;
      srv->wait_s += std::chrono::duration<double>(r.t_launch - r.t_submit).count();
      srv->completed.push_back(L->tickets[i]);
      ss->busy = false;
      const int32_t st = r.res.status;
      if (r.valid) {
        if (st == BO_E_INVALID_ARG || rc != BO_OK) {
          ss->need_refit = true;  // the bad entry at position n is overwritten by the next step
        } else {
          ss->n = r.n_new;
          ss->need_refit = (st == BO_E_NOT_PD);
        }
      } else if (st != BO_OK && st != BO_E_NO_CANDIDATE && st != BO_E_NUMERIC) {
        ss->need_refit = true;
      }
      ++srv->steps_done;
    }
    L->busy = false;
    L->tickets.clear();
    srv->cv_done.notify_all();
  }
  // tickets taken by bo_server_wait stay in the completion queue until
  // bo_server_wait_any passes them; keep the queue bounded for callers that
  // never call it
  if (srv->completed.size() > 2 * srv->reqs.size() + 4096) {
    std::deque<uint64_t> keep;
    for (uint64_t t : srv->completed)
      if (srv->reqs.count(t)) keep.push_back(t);
    srv->completed.swap(keep);
  }
  // sessions being closed free their memory once idle
  for (auto it = srv->sessions.begin(); it != srv->sessions.end();) {
    SrvSession* ss = it->second.get();
    bool queued = false;
    if (ss->state == 2 && !ss->busy)
      for (uint64_t t : srv->pending)
        if (srv->reqs[t].sid == ss->id) {
          queued = true;
          break;
        }
    if (ss->state == 2 && !ss->busy && !queued) {
      defer_free(srv, ss);
      it = srv->sessions.erase(it);
    } else {
      ++it;
    }
  }
}

// Forms and starts launches from the pending requests.  Lock held.
void dispatch(bo_server* srv) {
  for (auto& L : srv->launches) {
    if (L->busy) continue;
    L->items.clear();
    L->tickets.clear();
    std::vector<int32_t> taken;
    for (auto it = srv->pending.begin(); it != srv->pending.end() && (int)L->items.size() < srv->cfg.max_batch;) {
      const uint64_t t = *it;
      Request& r = srv->reqs[t];
      SrvSession* ss = srv->sessions[r.sid].get();
      if (ss->state == 3) {
        fail_request(srv, t, ss->setup_status);
        it = srv->pending.erase(it);
        srv->cv_done.notify_all();
        continue;
      }
      const bool idle = (ss->state == 1 || ss->state == 2) && !ss->busy &&
                        std::find(taken.begin(), taken.end(), r.sid) == taken.end();
      if (!idle) {
        ++it;
        continue;
      }
      BatchItem b{};
      b.s = ss->s;
      b.obs_idx = ss->obs_dev;
      b.y = ss->y_dev;
      b.visited = ss->vis_dev;
      b.acq = r.acq;
      b.mark = ss->vis_dev;
      b.new_idx = r.idx;
      b.new_y = r.y;
      if (r.valid) {
        b.n = ss->n + 1;
        b.write_obs = 1;
        b.fit_kind = ss->need_refit ? 0 : 1;
      } else {
        b.n = ss->n;
        b.write_obs = 0;
        b.fit_kind = ss->need_refit ? 0 : 2;
      }
      if (b.n > ss->prob.n_max || b.n > kSmallFitMax || b.n < 1) {
        fail_request(srv, t, BO_E_INVALID_ARG);
        it = srv->pending.erase(it);
        srv->cv_done.notify_all();
        continue;
      }
      r.n_new = b.n;
      taken.push_back(r.sid);
      L->items.push_back(b);
      L->tickets.push_back(t);
      it = srv->pending.erase(it);
    }
    if (L->items.empty()) return;
    const auto t0 = Clock::now();
    for (uint64_t t : L->tickets) srv->reqs[t].t_launch = t0;
    const bo_status rc = L->ctx.launch(L->items.data(), (int)L->items.size(), srv->cfg.tiles);
    srv->launch_s += std::chrono::duration<double>(Clock::now() - t0).count();
    if (rc != BO_OK) {
      for (uint64_t t : L->tickets) fail_request(srv, t, rc);
      L->tickets.clear();
      srv->cv_done.notify_all();
      continue;
    }
    for (uint64_t t : L->tickets) srv->sessions[srv->reqs[t].sid]->busy = true;
    L->busy = true;
    ++srv->n_launches;
    srv->items_launched += (int64_t)L->items.size();
  }
}

void worker_main(bo_server* srv) {
  (void)hipSetDevice(srv->device);
  // the completion polls below are short timed waits: without this, the
  // kernel's default timer slack (50 us) would stretch each one to ~70 us
  (void)prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    retire(srv);
    admit(srv);
    if (srv->stop) {
      // requests not yet launched are refused; launches in flight finish
      for (uint64_t t : srv->pending) fail_request(srv, t, BO_E_STATE);
      srv->pending.clear();
      srv->cv_done.notify_all();
      bool any = false;
      for (auto& L : srv->launches) any |= L->busy;
      if (!any) break;
    }
    dispatch(srv);
    bool inflight = false;
    for (auto& L : srv->launches) inflight |= L->busy;
    if (inflight) {
      // poll the launches' completion events between wake-ups
      srv->cv_work.wait_for(lk, std::chrono::microseconds(10));
    } else if (!srv->stop) {
      srv->cv_work.wait(lk);
    }
  }
}

}  // namespace

extern "C" {

bo_status bo_server_session_bytes(const bo_problem* prob, size_t* bytes) {
  if (!prob || !bytes) return set_error(BO_E_INVALID_ARG, "NULL argument");
  size_t ws = 0;
  const size_t b = session_bytes(*prob, &ws);
  if (!b) return set_error(BO_E_INVALID_ARG, "problem outside limits");
  *bytes = b;
  return BO_OK;
}

bo_status bo_server_create(bo_server** out, const bo_server_config* cfg) {
  if (!out || !cfg) return set_error(BO_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->max_batch > 4096) return set_error(BO_E_INVALID_ARG, "max_batch must be 1..4096");
  if (cfg->streams < 1 || cfg->streams > 8) return set_error(BO_E_INVALID_ARG, "streams must be 1..8");
  if (cfg->hbm_budget == 0) return set_error(BO_E_BUDGET, "memory budget is zero");
  const bo_batch_config& t = cfg->tiles;
  if ((t.post_order != 0 && t.post_order != 1) || t.acq_chunk < 2048 || t.acq_chunk % 2048 ||
      (t.fit_order != 0 && t.fit_order != 1))
    return set_error(BO_E_INVALID_ARG, "bad tile configuration");
  bo_server* srv = new (std::nothrow) bo_server();
  if (!srv) return set_error(BO_E_INVALID_ARG, "out of host memory");
  srv->cfg = *cfg;
  hipError_t e = hipGetDevice(&srv->device);
  const size_t per = a256(BatchCtx::bytes(cfg->max_batch));
  // streams that do not wait for the null stream (nor it for them), so that
  // session setup and teardown never hold up the launches
  if (e == hipSuccess) e = hipMalloc(&srv->ctx_mem, per * cfg->streams);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&srv->setup_stream, hipStreamNonBlocking);
  for (int i = 0; e == hipSuccess && i < cfg->streams; ++i) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) srv->launch_streams.push_back(st);
  }
  auto undo = [&]() {
    for (auto& M : srv->launches) M->ctx.destroy();
    for (hipStream_t st : srv->launch_streams) (void)hipStreamDestroy(st);
    if (srv->setup_stream) (void)hipStreamDestroy(srv->setup_stream);
    if (srv->ctx_mem) (void)hipFree(srv->ctx_mem);
    delete srv;
  };
  if (e != hipSuccess) {
    const char* msg = hipGetErrorString(e);
    undo();
    return set_error(BO_E_HIP, "server create: %s", msg);
  }
  for (int i = 0; i < cfg->streams; ++i) {
    std::unique_ptr<Launch> L(new Launch());
    bo_status rc = L->ctx.init(cfg->max_batch, (unsigned char*)srv->ctx_mem + per * i, per, srv->launch_streams[i]);
    if (rc == BO_OK) rc = L->ctx.set_timing(1);
    if (rc != BO_OK) {
      L->ctx.destroy();
      undo();
      return rc;
    }
    srv->launches.push_back(std::move(L));
  }
  srv->worker = std::thread(worker_main, srv);
  srv->setup_worker = std::thread(setup_main, srv);
  *out = srv;
  return BO_OK;
}

void bo_server_destroy(bo_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  srv->cv_setup.notify_all();
  srv->worker.join();
  srv->setup_worker.join();
  for (auto& x : srv->free_q) {
    if (x.s) bo_session_destroy(x.s);
    if (x.dev) (void)hipFree(x.dev);
  }
  for (auto& kv : srv->sessions) free_session_memory(srv, kv.second.get());
  for (auto& L : srv->launches) L->ctx.destroy();
  for (hipStream_t st : srv->launch_streams) (void)hipStreamDestroy(st);
  if (srv->staging) (void)hipFree(srv->staging);
  (void)hipFree(srv->ctx_mem);
  (void)hipStreamDestroy(srv->setup_stream);
  delete srv;
}

bo_status bo_server_open(bo_server* srv, const bo_problem* prob, const bo_gp_params* gp, const int32_t* levels,
                         const int64_t* cand, const uint8_t* invalid, const int64_t* obs_idx, const double* y,
                         int32_t n0, int32_t* id) {
  if (!srv || !prob || !levels || !obs_idx || !y || !id) return set_error(BO_E_INVALID_ARG, "NULL argument");
  if (prob->precision == BO_BF16X3) return set_error(BO_E_INVALID_ARG, "served sessions are FP64 or FP32");
  if (prob->n_max > kSmallFitMax) return set_error(BO_E_INVALID_ARG, "served sessions hold at most 256 observations");
  if (n0 < 1 || n0 > prob->n_max) return set_error(BO_E_INVALID_ARG, "initial observations must be 1..n_max");
  size_t ws = 0;
  const size_t bytes = session_bytes(*prob, &ws);
  if (!bytes) return set_error(BO_E_INVALID_ARG, "problem outside limits");
  std::unique_ptr<SrvSession> ss(new (std::nothrow) SrvSession());
  if (!ss) return set_error(BO_E_INVALID_ARG, "out of host memory");
  ss->prob = *prob;
  ss->gp = gp ? *gp : bo_gp_params{5, 7, 1.0, 1.0, 1e-6};
  ss->levels.assign(levels, levels + prob->d);
  if (cand) ss->cand.assign(cand, cand + prob->N);
  if (invalid) ss->invalid.assign(invalid, invalid + prob->N);
  ss->obs0.assign(obs_idx, obs_idx + n0);
  ss->y0.assign(y, y + n0);
  ss->bytes = bytes;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (bytes > srv->cfg.hbm_budget)
    return set_error(BO_E_BUDGET, "session needs %zu bytes, budget %zu", bytes, srv->cfg.hbm_budget);
  ss->id = srv->next_id++;
  *id = ss->id;
  srv->waiting.push_back(ss->id);
  srv->sessions[ss->id] = std::move(ss);
  admit(srv);
  srv->cv_work.notify_all();
  return BO_OK;
}

bo_status bo_server_close(bo_server* srv, int32_t id) {
  if (!srv) return set_error(BO_E_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->sessions.find(id);
  if (it == srv->sessions.end()) return set_error(BO_E_INVALID_ARG, "no session %d", id);
  SrvSession* ss = it->second.get();
  if (ss->state == 0) {
    srv->waiting.erase(std::remove(srv->waiting.begin(), srv->waiting.end(), id), srv->waiting.end());
    for (uint64_t t : srv->pending)
      if (srv->reqs[t].sid == id) fail_request(srv, t, BO_E_STATE);
    srv->pending.erase(std::remove_if(srv->pending.begin(), srv->pending.end(),
                                      [&](uint64_t t) { return srv->reqs[t].sid == id; }),
                       srv->pending.end());
    srv->sessions.erase(it);
    srv->cv_done.notify_all();
  } else if (ss->state == 4) {
    ss->close_requested = true;  // closed once its setup ends
  } else {
    ss->state = 2;  // its queued steps still run; memory is freed once idle
  }
  srv->cv_work.notify_all();
  return BO_OK;
}

bo_status bo_server_submit(bo_server* srv, int32_t id, int64_t idx, double y, int32_t valid,
                           const bo_acq_params* acq, uint64_t* ticket) {
  if (!srv || !acq || !ticket) return set_error(BO_E_INVALID_ARG, "NULL argument");
  AcqArgs a;
  bo_status rc = acq_params_check(acq, &a);
  if (rc != BO_OK) return rc;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->sessions.find(id);
  if (it == srv->sessions.end() || it->second->state == 2 || it->second->close_requested)
    return set_error(BO_E_INVALID_ARG, "no open session %d", id);
  if (idx < 0 || idx >= it->second->prob.N) return set_error(BO_E_INVALID_ARG, "index %lld out of range", (long long)idx);
  if (valid && !std::isfinite(y)) return set_error(BO_E_INVALID_ARG, "y is not finite");
  Request r;
  r.sid = id;
  r.idx = idx;
  r.y = y;
  r.valid = valid ? 1 : 0;
  r.acq = a;
  r.t_submit = Clock::now();
  const uint64_t t = srv->next_ticket++;
  srv->reqs[t] = r;
  srv->pending.push_back(t);
  *ticket = t;
  srv->cv_work.notify_all();
  return BO_OK;
}

bo_status bo_server_poll(bo_server* srv, uint64_t ticket, int32_t* done) {
  if (!srv || !done) return set_error(BO_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return set_error(BO_E_INVALID_ARG, "unknown ticket");
  *done = it->second.done ? 1 : 0;
  return BO_OK;
}

bo_status bo_server_wait(bo_server* srv, uint64_t ticket, bo_acq_result* out, double* latency_ms) {
  if (!srv || !out) return set_error(BO_E_INVALID_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return set_error(BO_E_INVALID_ARG, "unknown ticket");
  srv->cv_done.wait(lk, [&] { return it->second.done; });
  *out = it->second.res;
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(it->second.t_done - it->second.t_submit).count();
  srv->reqs.erase(it);
  return BO_OK;
}

bo_status bo_server_wait_any(bo_server* srv, int32_t max, int32_t timeout_us, uint64_t* tickets,
                             bo_acq_result* out, double* latency_ms, int32_t* count) {
  if (!srv || !tickets || !out || !count) return set_error(BO_E_INVALID_ARG, "NULL argument");
  if (max < 1) return set_error(BO_E_INVALID_ARG, "max must be >= 1");
  if (timeout_us < 0) return set_error(BO_E_INVALID_ARG, "timeout must be >= 0");
  *count = 0;
  std::unique_lock<std::mutex> lk(srv->mu);
  // tickets already taken by bo_server_wait are gone from the table
  auto drop_taken = [&] {
    while (!srv->completed.empty() && srv->reqs.find(srv->completed.front()) == srv->reqs.end())
      srv->completed.pop_front();
  };
  drop_taken();
  if (srv->completed.empty() && timeout_us > 0)
    srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] {
      drop_taken();
      return !srv->completed.empty();
    });
  int32_t k = 0;
  while (k < max && !srv->completed.empty()) {
    const uint64_t t = srv->completed.front();
    srv->completed.pop_front();
    auto it = srv->reqs.find(t);
    if (it == srv->reqs.end()) continue;
    tickets[k] = t;
    out[k] = it->second.res;
    if (latency_ms)
      latency_ms[k] = std::chrono::duration<double, std::milli>(it->second.t_done - it->second.t_submit).count();
    srv->reqs.erase(it);
    ++k;
  }
  *count = k;
  return BO_OK;
}

bo_status bo_server_stats(bo_server* srv, bo_server_info* out) {
  if (!srv || !out) return set_error(BO_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  bo_server_info s{};
  s.steps_done = srv->steps_done;
  s.launches = srv->n_launches;
  s.mean_batch = srv->n_launches ? (double)srv->items_launched / (double)srv->n_launches : 0.0;
  s.bytes_in_use = srv->used;
  for (auto& kv : srv->sessions) {
    if (kv.second->state == 1 || kv.second->state == 2 || kv.second->state == 4) ++s.sessions_resident;
    else if (kv.second->state == 0) ++s.sessions_waiting;
    if (kv.second->state == 4) ++s.sessions_setting_up;
  }
  s.mean_wait_us = srv->steps_done ? 1e6 * srv->wait_s / (double)srv->steps_done : 0.0;
  s.mean_launch_us = srv->n_launches ? 1e6 * srv->launch_s / (double)srv->n_launches : 0.0;
  s.mean_gpu_us = srv->gpu_timed ? 1e3 * srv->gpu_ms / (double)srv->gpu_timed : 0.0;
  s.pending = (int64_t)srv->pending.size();
  *out = s;
  return BO_OK;
}

}  // extern "C"
