// Batched BO steps: many independent sessions (uneven candidate counts,
// dimensions and observation counts) advance one step in one captured HIP
// graph, replayed every step:
//
//   plan copy -> fits -> posterior (d <= 8, d > 8) -> exploration factors ->
//   acquisition chunks -> selections -> result copy.
//
//  - fits: one workgroup per session (FP64, fit_small_run or append_run,
//    n <= 256), largest first when the plan asks for it;
//  - posterior: one launch per coordinate class (d <= 8, d > 8) over every
//    session's 64-candidate slots, FP64 and FP32 sessions alike, one slot per
//    workgroup, by default the sessions of the costliest slots first (longest
//    first keeps the tail short).  Each slot is the
//    single-session kernel's workgroup (four waves of 16 rows in the
//    register-resident posterior, their partials added in wave order), with
//    the session's shape chosen at run time from specialised, inlined bodies;
//  - exploration factor: one workgroup per session reduces its slots in the
//    single-session order (Section III-F);
//  - acquisition: (session, chunk of `acq_chunk` candidates) workgroups, then
//    one workgroup per session combines the chunks.
// So every result equals the single-session path's bit for bit.  Kernel
// boundaries order the phases, so no workgroup waits on another.  Everything
// that changes between steps (observation pointers and counts, masks,
// acquisition parameters, work lists) is in the plan, copied from pinned host
// memory by the graph's first node; the grid of each kernel node is set to
// the step's work before each replay, so the graph is captured once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "acq_common.h"
#include "batch_ctx.h"
#include "bo_device.h"
#include "bo_internal.h"
#include "fit_body.h"
#include "post_common.h"
#include "session_impl.h"

namespace bo {
namespace {

constexpr int kSlotRows = 64;      // candidates of a variance slot: one single-session posterior workgroup
constexpr int kSlotThreads = 256;  // threads of that workgroup, which fix the reduction orders

struct BatchSession {
  FitArgs fit;
  PostArgs post;
  AcqKArgs acq;
  int64_t new_idx;    // write_obs: observation written at position n - 1 first
  double new_y;
  uint8_t* mark;      // nullable: mark[new_idx] = 1 before the fit
  int32_t fit_kind;   // 0: full fit, 1: rank-1 append, 2: keep the current fit
  int32_t write_obs;
  int32_t f32;        // FP32 (1) or FP64 (0) posterior
  int32_t n_slots;    // 64-candidate variance slots, ceil(n_valid / 64), at least 1
  int32_t n_acq;      // acquisition chunks
  int32_t acq_chunk;  // candidates per acquisition chunk
};

struct PlanHdr {
  int32_t count;
  int32_t pad0;
  uint32_t wg_post[2];        // posterior workgroups (slots), d <= 8 and d > 8
  uint32_t wg_acq;            // acquisition workgroups
  uint32_t pad[3];
};

// Plan layout: PlanHdr | BatchSession[cap] | fit order[cap] |
// per class q (d <= 8, d > 8): session list[cap], workgroup offsets[cap + 1] |
// acquisition offsets[cap + 1]
struct PlanView {
  PlanHdr* hdr;
  BatchSession* ses;
  int32_t* order;
  int32_t* list[2];
  uint32_t* off[2];
  uint32_t* acq_off;
};

__host__ __device__ inline PlanView plan_view(unsigned char* base, int cap) {
  PlanView v;
  v.hdr = (PlanHdr*)base;
  v.ses = (BatchSession*)(base + sizeof(PlanHdr));
  v.order = (int32_t*)(v.ses + cap);
  unsigned char* q = (unsigned char*)(v.order + cap);
  for (int k = 0; k < 2; ++k) {
    v.list[k] = (int32_t*)q;
    v.off[k] = (uint32_t*)(v.list[k] + cap);
    q = (unsigned char*)(v.off[k] + cap + 1);
  }
  v.acq_off = (uint32_t*)q;
  return v;
}

inline size_t plan_bytes(int cap) {
  return sizeof(PlanHdr) + (sizeof(BatchSession) + 3 * sizeof(int32_t)) * cap + 3 * sizeof(uint32_t) * (cap + 1);
}

// Largest i with off[i] <= v, for off[0] = 0 <= v < off[count].
__device__ __forceinline__ int find_owner(const uint32_t* off, int count, uint32_t v) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= v) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Fits: one workgroup per session, in the plan's order.
__global__ __launch_bounds__(kSmallThreads) void k_bfit(unsigned char* plan, int cap) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  const PlanView v = plan_view(plan, cap);
  const int s = v.order[blockIdx.x];
  const BatchSession& S = v.ses[s];
  if (threadIdx.x == 0) {
    const int64_t i = S.new_idx;
    if (S.write_obs) {
      // the observation arrays belong to the caller that asked for this
      const_cast<int64_t*>(S.fit.obs_idx)[S.fit.n - 1] = i;
      const_cast<double*>(S.fit.y_in)[S.fit.n - 1] = S.new_y;
    }
    if (S.mark && i >= 0 && i < S.fit.N) S.mark[i] = 1;
  }
  __threadfence_block();
  __syncthreads();
  if (S.fit_kind == 0) fit_small_run(S.fit, s_raw);
  else if (S.fit_kind == 1) append_run(S.fit, s_raw);
}

// Posterior of the sessions of one class (DM = 8: d <= 8; DM = kMaxD: the
// others), both precisions: workgroup g takes one slot of one session,
// computed as the single-session kernel's workgroup does (k_post16r: same
// bodies, same order of the four waves' partials; the class only sets how
// many coordinates the distance loop runs over, and the zero coordinates
// past d add exact zeros), and publishes it in the session's slot array.  (A
// loop over several slots per workgroup, or both classes in one kernel, costs
// the shape bodies their spill-free register allocation.)
template <int DM>
__global__ __launch_bounds__(kSlotThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_bpost(
    unsigned char* plan, int cap) {
  __shared__ double s_xo[16 * kRegJB * kObsPitch];
  __shared__ double s_alpha[16 * kRegJB];
  __shared__ double s_wsum[4];
  __shared__ int64_t s_wcnt[4];
  const PlanView v = plan_view(plan, cap);
  constexpr int q = DM == 8 ? 0 : 1;
  if (blockIdx.x >= v.hdr->wg_post[q]) return;  // an empty list still launches one workgroup
  const int k = find_owner(v.off[q], v.hdr->count, blockIdx.x);
  const BatchSession& S = v.ses[v.list[q][k]];
  const PostArgs p = S.post;
  if (p.st->status != BO_OK) return;
  const int slot = (int)(blockIdx.x - v.off[q][k]);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int jb = reg_jb(p.n);
  stage_obs(p, 16 * jb, s_xo, s_alpha);
  {
    const int64_t row0 = ((int64_t)slot * 4 + w) * 16;
    double part;
    int64_t cnt;
    switch (jb) {
#define BO_REG_CASE(J) \
  case J: post16_wave_reg<J, DM>(p, row0, s_xo, s_alpha, &part, &cnt); break;
      BO_REG_CASE(1) BO_REG_CASE(2) BO_REG_CASE(3) BO_REG_CASE(4) BO_REG_CASE(5) BO_REG_CASE(6)
      BO_REG_CASE(7) BO_REG_CASE(8) BO_REG_CASE(9) BO_REG_CASE(10) BO_REG_CASE(11) BO_REG_CASE(12)
      BO_REG_CASE(13) BO_REG_CASE(14) BO_REG_CASE(15)
#undef BO_REG_CASE
      default: post16_wave_reg<16, DM>(p, row0, s_xo, s_alpha, &part, &cnt); break;
    }
    if (l == 0) {
      s_wsum[w] = part;
      s_wcnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0;
      int64_t c = 0;
      for (int i = 0; i < 4; ++i) {
        a += s_wsum[i];
        c += s_wcnt[i];
      }
      p.vslots[slot].sum = a;
      p.vslots[slot].count = c;
    }
  }
}

// Mean variance and exploration factor of each session from its slots.
__global__ __launch_bounds__(kSlotThreads) void k_blam(unsigned char* plan, int cap) {
  __shared__ double s_sum[kSlotThreads];
  __shared__ int64_t s_cnt[kSlotThreads];
  const PlanView v = plan_view(plan, cap);
  const BatchSession& S = v.ses[blockIdx.x];
  if (S.post.st->status != BO_OK) return;
  finish_lambda(S.post, S.n_slots, s_sum, s_cnt, kSlotThreads);
}

// Acquisitions of one chunk of one session.
__global__ __launch_bounds__(kAcqThreads) void k_bacq(unsigned char* plan, int cap) {
  __shared__ Best s_best[kAcqThreads / 64];
  __shared__ int s_nan[kAcqThreads / 64];
  const PlanView v = plan_view(plan, cap);
  const int s = find_owner(v.acq_off, v.hdr->count, blockIdx.x);
  const int j = (int)(blockIdx.x - v.acq_off[s]);
  const BatchSession& S = v.ses[s];
  const int64_t c0 = (int64_t)j * S.acq_chunk;
  const int64_t c1 = c0 + S.acq_chunk < S.acq.n_valid ? c0 + S.acq_chunk : S.acq.n_valid;
  if (S.f32) acq_range<true>(S.acq, c0, c1, &S.acq.slots[j], s_best, s_nan);
  else acq_range<false>(S.acq, c0, c1, &S.acq.slots[j], s_best, s_nan);
}

// Selection of each session from its chunks.
__global__ __launch_bounds__(kAcqThreads) void k_bsel(unsigned char* plan, int cap) {
  __shared__ Best s_best[kAcqThreads / 64];
  __shared__ int s_nan[kAcqThreads / 64];
  const PlanView v = plan_view(plan, cap);
  const BatchSession& S = v.ses[blockIdx.x];
  acq_finish(S.acq, S.n_acq, s_best, s_nan);
}

constexpr size_t kFitLds = kSmallLdsBytes;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

#define BHIP(expr)                                                                               \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return set_error(BO_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

}  // namespace


// ------------------------------------------------------------ BatchCtx --

size_t BatchCtx::bytes(int cap) { return align256(plan_bytes(cap)) + align256(sizeof(bo_acq_result) * cap); }

bo_status BatchCtx::init(int cap_, void* workspace, size_t nbytes, hipStream_t stream_) {
  if (cap_ < 1) return set_error(BO_E_INVALID_ARG, "batch capacity must be >= 1");
  if (!workspace || ((uintptr_t)workspace & 255u)) return set_error(BO_E_WORKSPACE, "workspace NULL or misaligned");
  if (nbytes < bytes(cap_)) return set_error(BO_E_WORKSPACE, "workspace %zu bytes < %zu needed", nbytes, bytes(cap_));
  BHIP(hipFuncSetAttribute((const void*)k_bfit, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFitLds));
  cap = cap_;
  stream = stream_;
  if (!stream) {
    // a graph cannot be captured on the null stream; a blocking stream keeps
    // the ordering with the caller's null-stream work
    BHIP(hipStreamCreate(&stream));
    own_stream = 1;
  }
  unsigned char* w = (unsigned char*)workspace;
  plan_sz = plan_bytes(cap);
  plan_dev = w;
  w += align256(plan_sz);
  res_dev = (bo_acq_result*)w;
  res_sz = sizeof(bo_acq_result) * cap;
  BHIP(hipHostMalloc((void**)&plan_host, plan_sz, hipHostMallocDefault));
  BHIP(hipHostMalloc((void**)&res_host, res_sz, hipHostMallocDefault));
  BHIP(hipEventCreateWithFlags(&done_ev, hipEventDisableTiming));
  return BO_OK;
}

void BatchCtx::destroy() {
  if (stream) (void)hipStreamSynchronize(stream);
  if (have_graph) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    have_graph = 0;
  }
  if (timing) {
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    timing = 0;
  }
  if (done_ev) (void)hipEventDestroy(done_ev);
  if (plan_host) (void)hipHostFree(plan_host);
  if (res_host) (void)hipHostFree(res_host);
  if (own_stream) (void)hipStreamDestroy(stream);
  done_ev = nullptr;
  plan_host = res_host = nullptr;
  stream = nullptr;
  own_stream = 0;
}

bo_status BatchCtx::set_timing(int enable) {
  if (enable && !timing) {
    BHIP(hipEventCreate(&ev[0]));
    BHIP(hipEventCreate(&ev[1]));
    timing = 1;
  } else if (!enable && timing) {
    BHIP(hipStreamSynchronize(stream));
    BHIP(hipEventDestroy(ev[0]));
    BHIP(hipEventDestroy(ev[1]));
    timing = 0;
  }
  return BO_OK;
}

bo_status BatchCtx::build_plan(const BatchItem* items, int count, const bo_batch_config& cfg) {
  if (count < 1 || count > cap) return set_error(BO_E_INVALID_ARG, "%d steps for a batch of capacity %d", count, cap);
  const PlanView v = plan_view(plan_host, cap);
  uint32_t ta = 0;
  for (int i = 0; i < count; ++i) {
    const BatchItem& it = items[i];
    bo_session* s = it.s;
    if (!s) return set_error(BO_E_INVALID_ARG, "step %d: session is NULL", i);
    if (s->lo.prec == BO_BF16X3) return set_error(BO_E_INVALID_ARG, "step %d: BF16X3 sessions are not batched", i);
    if (!s->have_cand) return set_error(BO_E_STATE, "step %d: no candidate set", i);
    if (it.n < 1) return set_error(BO_E_STATE, "step %d: a fit needs at least one observation", i);
    if (it.n > s->prob.n_max || it.n > kSmallFitMax)
      return set_error(BO_E_INVALID_ARG, "step %d: n = %d exceeds n_max = %d or %d", i, it.n, s->prob.n_max,
                       kSmallFitMax);
    if (!it.obs_idx || !it.y) return set_error(BO_E_INVALID_ARG, "step %d: obs_idx or y is NULL", i);
    BatchSession& B = v.ses[i];
    memset(&B, 0, sizeof B);
    B.fit = make_args(s->P, s->lo, s->gp, it.obs_idx, it.y, it.n);
    B.post = make_post_args(s->P, s->lo, s->gp, it.n, s->n_valid, it.visited, it.acq);
    B.acq = make_acq_args(s->P, s->n_valid, it.visited, it.acq, res_dev + i);
    B.new_idx = it.new_idx;
    B.new_y = it.new_y;
    B.mark = it.mark;
    B.fit_kind = it.fit_kind;
    B.write_obs = it.write_obs;
    B.f32 = s->lo.prec == BO_FP32 ? 1 : 0;
    const int64_t nv = s->n_valid;
    B.n_slots = (int32_t)std::max<int64_t>(1, (nv + kSlotRows - 1) / kSlotRows);
    // the session's chunk slots hold kAcqMaxBlocks results
    int64_t chunk = cfg.acq_chunk;
    const int64_t least = (nv + kAcqMaxBlocks - 1) / kAcqMaxBlocks;
    if (chunk < least) chunk = (least + 2047) / 2048 * 2048;
    B.acq_chunk = (int32_t)chunk;
    B.n_acq = (int32_t)std::max<int64_t>(1, (nv + chunk - 1) / chunk);
    v.acq_off[i] = ta;
    ta += (uint32_t)B.n_acq;
  }
  v.acq_off[count] = ta;
  order_scratch.resize(count);
  for (int i = 0; i < count; ++i) order_scratch[i] = i;
  if (cfg.fit_order == 1)
    std::stable_sort(order_scratch.begin(), order_scratch.end(),
                     [&](int a, int c) { return items[a].n > items[c].n; });
  for (int i = 0; i < count; ++i) v.order[i] = order_scratch[i];
  // posterior lists, by coordinate class (d <= 8, d > 8): the sessions of the
  // costliest slots (most column blocks) first, or in the fit order
  for (int q = 0; q < 2; ++q) {
    int k = 0;
    uint32_t wg = 0;
    for (int i = 0; i < count; ++i) {
      const BatchSession& B = v.ses[order_scratch[i]];
      if ((B.post.d > 8 ? 1 : 0) != q) continue;
      v.list[q][k] = order_scratch[i];
      ++k;
    }
    if (cfg.post_order == 0)
      std::stable_sort(v.list[q], v.list[q] + k,
                       [&](int a, int c) { return reg_jb(v.ses[a].post.n) > reg_jb(v.ses[c].post.n); });
    for (int j = 0; j < k; ++j) {
      v.off[q][j] = wg;
      wg += (uint32_t)v.ses[v.list[q][j]].n_slots;
    }
    // entries past the list repeat its end (the owner search spans `count`)
    for (int j = k; j <= count; ++j) v.off[q][j] = wg;
    v.hdr->wg_post[q] = wg;
  }
  v.hdr->count = count;
  v.hdr->pad0 = 0;
  v.hdr->wg_acq = ta;
  grids[0] = (unsigned)count;
  grids[1] = std::max(1u, v.hdr->wg_post[0]);
  grids[2] = std::max(1u, v.hdr->wg_post[1]);
  grids[3] = (unsigned)count;
  grids[4] = ta;
  grids[5] = (unsigned)count;
  return BO_OK;
}

// The kernels of the graph in launch order, with their block sizes and LDS.
struct BatchKernel {
  const void* fn;
  unsigned threads;
  unsigned lds;
};

static const BatchKernel* batch_kernels() {
  static const BatchKernel k[kBatchNodes] = {
      {(const void*)k_bfit, (unsigned)kSmallThreads, (unsigned)kFitLds},
      {(const void*)k_bpost<8>, (unsigned)kSlotThreads, 0u},
      {(const void*)k_bpost<kMaxD>, (unsigned)kSlotThreads, 0u},
      {(const void*)k_blam, (unsigned)kSlotThreads, 0u},
      {(const void*)k_bacq, (unsigned)kAcqThreads, 0u},
      {(const void*)k_bsel, (unsigned)kAcqThreads, 0u},
  };
  return k;
}

bo_status BatchCtx::capture() {
  const BatchKernel* K = batch_kernels();
  karg_plan = plan_dev;
  karg_cap = cap;
  BHIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  (void)hipMemcpyAsync(plan_dev, plan_host, plan_sz, hipMemcpyHostToDevice, stream);
  for (int i = 0; i < kBatchNodes; ++i) {
    void* args[2] = {&karg_plan, &karg_cap};
    (void)hipLaunchKernel(K[i].fn, dim3(grids[i]), dim3(K[i].threads), args, K[i].lds, stream);
  }
  (void)hipMemcpyAsync(res_host, res_dev, res_sz, hipMemcpyDeviceToHost, stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(stream, &g);
  if (e != hipSuccess) return set_error(BO_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  // the kernel nodes, whose grids each replay sets
  size_t nn = 0;
  e = hipGraphGetNodes(g, nullptr, &nn);
  std::vector<hipGraphNode_t> nodes(nn);
  if (e == hipSuccess) e = hipGraphGetNodes(g, nodes.data(), &nn);
  int found = 0;
  for (size_t i = 0; e == hipSuccess && i < nn; ++i) {
    hipGraphNodeType t;
    e = hipGraphNodeGetType(nodes[i], &t);
    if (e != hipSuccess || t != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams kp{};
    e = hipGraphKernelNodeGetParams(nodes[i], &kp);
    for (int k = 0; e == hipSuccess && k < kBatchNodes; ++k)
      if (kp.func == K[k].fn) {
        knode[k] = nodes[i];
        kgrid[k] = grids[k];
        ++found;
      }
  }
  if (e == hipSuccess && found != kBatchNodes) e = hipErrorInvalidValue;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return set_error(BO_E_HIP, "graph setup: %s", hipGetErrorString(e));
  }
  graph = g;
  have_graph = 1;
  return BO_OK;
}

bo_status BatchCtx::launch(const BatchItem* items, int count, const bo_batch_config& cfg) {
  // the previous replay must be done before its plan is overwritten
  BHIP(hipEventSynchronize(done_ev));
  bo_status rc = build_plan(items, count, cfg);
  if (rc != BO_OK) return rc;
  if (!have_graph) {
    rc = capture();
    if (rc != BO_OK) return rc;
  }
  const BatchKernel* K = batch_kernels();
  for (int i = 0; i < kBatchNodes; ++i) {
    if (grids[i] == kgrid[i]) continue;
    void* args[2] = {&karg_plan, &karg_cap};
    hipKernelNodeParams kp{};
    kp.func = (void*)K[i].fn;
    kp.gridDim = dim3(grids[i]);
    kp.blockDim = dim3(K[i].threads);
    kp.sharedMemBytes = K[i].lds;
    kp.kernelParams = args;
    kp.extra = nullptr;
    BHIP(hipGraphExecKernelNodeSetParams(exec, knode[i], &kp));
    kgrid[i] = grids[i];
  }
  n_last = count;
  if (timing) BHIP(hipEventRecord(ev[0], stream));
  BHIP(hipGraphLaunch(exec, stream));
  if (timing) BHIP(hipEventRecord(ev[1], stream));
  BHIP(hipEventRecord(done_ev, stream));
  return BO_OK;
}

bool BatchCtx::done() const { return hipEventQuery(done_ev) == hipSuccess; }

bo_status BatchCtx::finish(bo_acq_result* out, float* ms) {
  BHIP(hipEventSynchronize(done_ev));
  if (ms) {
    *ms = -1.f;
    if (timing) BHIP(hipEventElapsedTime(ms, ev[0], ev[1]));
  }
  memcpy(out, res_host, sizeof(bo_acq_result) * n_last);
  return BO_OK;
}

}  // namespace bo

using namespace bo;

struct bo_batch {
  BatchCtx ctx;
  std::vector<bo_session*> ses;
  std::vector<BatchItem> items;
  bo_batch_config cfg;
};

namespace {

bo_status check_config(const bo_batch_config* c) {
  if (c->post_order != 0 && c->post_order != 1) return set_error(BO_E_INVALID_ARG, "post_order must be 0 or 1");
  if (c->acq_chunk < 2048 || c->acq_chunk % 2048)
    return set_error(BO_E_INVALID_ARG, "acq_chunk must be a positive multiple of 2048");
  if (c->fit_order != 0 && c->fit_order != 1) return set_error(BO_E_INVALID_ARG, "fit_order must be 0 or 1");
  return BO_OK;
}

bo_status run_step(bo_batch* b, const bo_batch_config& cfg, const int64_t* const* obs_idx, const double* const* y,
                   const int32_t* n, const uint8_t* const* visited, const bo_acq_params* params,
                   bo_acq_result* out, float* ms) {
  if (!obs_idx || !y || !n || !params || !out) return set_error(BO_E_INVALID_ARG, "NULL argument");
  const int count = (int)b->ses.size();
  b->items.assign(count, BatchItem{});
  for (int i = 0; i < count; ++i) {
    BatchItem& it = b->items[i];
    it.s = b->ses[i];
    it.obs_idx = obs_idx[i];
    it.y = y[i];
    it.n = n[i];
    it.visited = (visited && visited[i]) ? visited[i] : it.s->P.vis;
    bo_status rc = acq_params_check(&params[i], &it.acq);
    if (rc != BO_OK) return rc;
    it.fit_kind = 0;
  }
  bo_status rc = b->ctx.launch(b->items.data(), count, cfg);
  if (rc != BO_OK) return rc;
  rc = b->ctx.finish(out, ms);
  if (rc != BO_OK) return rc;
  for (int i = 0; i < count; ++i) {
    bo_session* s = b->ses[i];
    s->n = n[i];
    s->large_fit = 0;
    s->have_fit = 1;
  }
  return BO_OK;
}

}  // namespace

extern "C" {

bo_status bo_batch_workspace_query(int32_t count, size_t* bytes) {
  if (!bytes) return set_error(BO_E_INVALID_ARG, "bytes is NULL");
  if (count < 1 || count > 65536) return set_error(BO_E_INVALID_ARG, "count must be 1..65536");
  *bytes = BatchCtx::bytes(count);
  return BO_OK;
}

bo_status bo_batch_create(bo_batch** out, bo_session* const* sessions, int32_t count, void* workspace,
                          size_t bytes, void* stream) {
  if (!out) return set_error(BO_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!sessions || count < 1 || count > 65536) return set_error(BO_E_INVALID_ARG, "sessions NULL or bad count");
  for (int i = 0; i < count; ++i) {
    if (!sessions[i]) return set_error(BO_E_INVALID_ARG, "session %d is NULL", i);
    if (sessions[i]->lo.prec == BO_BF16X3)
      return set_error(BO_E_INVALID_ARG, "session %d: the batched step runs FP64 and FP32 sessions only", i);
    for (int j = 0; j < i; ++j)
      if (sessions[j] == sessions[i]) return set_error(BO_E_INVALID_ARG, "session %d appears twice", i);
  }
  bo_batch* b = new (std::nothrow) bo_batch();
  if (!b) return set_error(BO_E_INVALID_ARG, "out of host memory");
  bo_status rc = b->ctx.init(count, workspace, bytes, (hipStream_t)stream);
  if (rc != BO_OK) {
    b->ctx.destroy();
    delete b;
    return rc;
  }
  b->ses.assign(sessions, sessions + count);
  b->cfg = bo_batch_config{0, 8192, 1, 0};
  *out = b;
  return BO_OK;
}

void bo_batch_destroy(bo_batch* b) {
  if (!b) return;
  b->ctx.destroy();
  delete b;
}

bo_status bo_batch_set_config(bo_batch* b, const bo_batch_config* cfg) {
  if (!b || !cfg) return set_error(BO_E_INVALID_ARG, "NULL argument");
  bo_status rc = check_config(cfg);
  if (rc != BO_OK) return rc;
  b->cfg = *cfg;
  return BO_OK;
}

bo_status bo_batch_get_config(bo_batch* b, bo_batch_config* cfg) {
  if (!b || !cfg) return set_error(BO_E_INVALID_ARG, "NULL argument");
  *cfg = b->cfg;
  return BO_OK;
}

bo_status bo_batch_set_timing(bo_batch* b, int32_t enable) {
  if (!b) return set_error(BO_E_INVALID_ARG, "batch is NULL");
  return b->ctx.set_timing(enable);
}

bo_status bo_batch_step(bo_batch* b, const int64_t* const* obs_idx, const double* const* y, const int32_t* n,
                        const uint8_t* const* visited, const bo_acq_params* params, bo_acq_result* out,
                        float* graph_ms) {
  if (!b) return set_error(BO_E_INVALID_ARG, "batch is NULL");
  return run_step(b, b->cfg, obs_idx, y, n, visited, params, out, graph_ms);
}

bo_status bo_batch_tune(bo_batch* b, const int64_t* const* obs_idx, const double* const* y, const int32_t* n,
                        const uint8_t* const* visited, const bo_acq_params* params, int32_t reps,
                        bo_batch_config* chosen, bo_acq_result* out) {
  if (!b) return set_error(BO_E_INVALID_ARG, "batch is NULL");
  if (reps < 1 || reps > 100) return set_error(BO_E_INVALID_ARG, "reps must be 1..100");
  const int had_timing = b->ctx.timing;
  bo_status rc = b->ctx.set_timing(1);
  if (rc != BO_OK) return rc;
  const int post_orders[2] = {0, 1};
  const int chunks[3] = {4096, 8192, 32768};
  const int orders[2] = {1, 0};
  bo_batch_config best{};
  float best_ms = INFINITY;
  for (int r : post_orders)
    for (int c : chunks)
      for (int o : orders) {
        const bo_batch_config cfg{r, c, o, 0};
        std::vector<float> t;
        for (int k = 0; k < reps + 1; ++k) {
          float ms = 0.f;
          rc = run_step(b, cfg, obs_idx, y, n, visited, params, out, &ms);
          if (rc != BO_OK) return rc;
          if (k > 0) t.push_back(ms);  // the first replay warms caches
        }
        std::sort(t.begin(), t.end());
        const float med = t[t.size() / 2];
        if (med < best_ms) {
          best_ms = med;
          best = cfg;
        }
      }
  b->cfg = best;
  if (!had_timing) (void)b->ctx.set_timing(0);
  if (chosen) *chosen = best;
  return BO_OK;
}

}  // extern "C"
