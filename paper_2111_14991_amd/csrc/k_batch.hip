// Batched BO steps: many independent sessions (uneven candidate counts,
// dimensions and observation counts) advance one step in a single persistent
// launch, captured once in a HIP graph and replayed every step.
//
// Work items, handed out in this order by one global counter:
//   1. one fit per session (FP64, fit_small_run: n <= 256), largest first
//      when the plan asks for it;
//   2. posterior tiles: (session, tile) with `rows` candidates per tile, each
//      wave running post16_wave on 16 * rb of them;
//   3. acquisition chunks: (session, chunk of `acq_chunk` candidates).
// A tile waits for its session's fit, a chunk for its session's exploration
// factor (computed by the session's last tile).  Every item waits only on
// items handed out before it, and those are held by running workgroups that
// never wait on later items, so each wait ends; a wait is still bounded by a
// spin limit that turns into an error flag.  The last workgroup to leave
// resets the counters and flags for the next replay.
//
// Everything that changes between steps (observation pointers and counts,
// masks, acquisition parameters, tile shapes) is in the plan, a device buffer
// copied from pinned host memory by the first node of the graph, so the graph
// never needs to be captured again.
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

constexpr int kBThreads = kSmallThreads;  // one fit needs the whole workgroup
constexpr int kBWaves = kBThreads / 64;
constexpr uint32_t kSpinLimit = 1u << 20;  // ~0.1 s of s_sleep 4; legitimate waits are ~1 ms

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
  int32_t rb;         // row blocks of 16 candidates per wave
  int32_t waves;      // waves working on a posterior tile (power of two)
  int32_t rows;       // candidates per posterior tile = 16 * rb * waves
  int32_t n_post;     // posterior tiles
  int32_t n_acq;      // acquisition chunks
  int32_t acq_chunk;  // candidates per acquisition chunk
  int32_t pad;
};

struct BatchSync {
  uint32_t fit_done, post_done, lam_ready, acq_done;
};

struct BatchCtl {
  uint32_t next;     // work counter
  uint32_t exited;   // workgroups that found no more work
  uint32_t timeout;  // a wait hit the spin limit
  uint32_t pad;
};

struct PlanHdr {
  int32_t count;
  uint32_t total_post, total_acq, pad;
};

// Plan layout: PlanHdr | BatchSession[cap] | post_off[cap + 1] | acq_off[cap + 1] | order[cap]
inline size_t plan_bytes(int cap) {
  return sizeof(PlanHdr) + sizeof(BatchSession) * cap + sizeof(uint32_t) * 2 * (cap + 1) + sizeof(int32_t) * cap;
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

// Thread 0 waits until *f >= want; every thread returns whether it did.
__device__ bool wait_flag(uint32_t* f, uint32_t want, BatchCtl* ctl, int* s_ok) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    int ok = 1;
    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
      __builtin_amdgcn_s_sleep(4);
      if (++spins > kSpinLimit) {
        ok = 0;
        atomicExch(&ctl->timeout, 1u);
        break;
      }
    }
    *s_ok = ok;
  }
  __syncthreads();
  __threadfence();
  return *s_ok != 0;
}

// Ticket on *t out of `total`: true in the workgroup that takes the last one.
__device__ bool last_of(uint32_t* t, uint32_t total, int* s_flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) *s_flag = (atomicAdd(t, 1u) == total - 1) ? 1 : 0;
  __syncthreads();
  const bool last = *s_flag != 0;
  if (last) __threadfence();
  return last;
}

// rb blocks of 16 rows from row0 with the register-resident FP64 posterior of
// n_pad = 16 JB, a function of its own per shape so that each gets its own
// register allocation
template <int JB>
__device__ __attribute__((noinline)) void reg_rows(const PostArgs& p, int64_t row0, int rb, const double* xs,
                                                   double* part, int64_t* cnt) {
  const double* as = xs + 16 * kRegJB * kObsPitch;
  const bool small_d = uni(p.d) <= 8;
  for (int b = 0; b < rb; ++b) {
    double pb;
    int64_t cb;
    if (small_d) post16_wave_reg<JB, 8>(p, row0 + 16 * b, xs, as, &pb, &cb);
    else post16_wave_reg<JB, kMaxD>(p, row0 + 16 * b, xs, as, &pb, &cb);
    *part += pb;
    *cnt += cb;
  }
}

// Same for the register-resident FP32 (compensated) posterior; rbuf: this
// wave's kReg32Rbuf floats of LDS.
template <int JB>
__device__ __attribute__((noinline)) void reg32_rows(const PostArgs& p, int64_t row0, int rb, const double* xs,
                                                     float* rbuf, double* part, int64_t* cnt) {
  const double* as = xs + 16 * kRegJB * kObsPitch;
  const bool small_d = uni(p.d) <= 8;
  for (int b = 0; b < rb; ++b) {
    double pb;
    int64_t cb;
    if (small_d) post16_wave_reg32<JB, 8>(p, row0 + 16 * b, xs, as, rbuf, &pb, &cb);
    else post16_wave_reg32<JB, kMaxD>(p, row0 + 16 * b, xs, as, rbuf, &pb, &cb);
    *part += pb;
    *cnt += cb;
  }
}

template <bool F32>
__device__ void post_tile(const BatchSession& S, int t, unsigned char* s_raw, double* s_wsum, int64_t* s_wcnt) {
  const PostArgs& p = S.post;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  double part = 0.0;
  int64_t cnt = 0;
  // the register-resident posterior (observations staged in LDS, then the
  // FP32 mode's kept residuals, kReg32Rbuf floats per wave)
  const bool reg = p.n_pad <= 16 * kRegJB;
  if (reg) {
    double* xs = (double*)s_raw;
    stage_obs(p, xs, xs + 16 * kRegJB * kObsPitch);
  }
  if (w < S.waves) {
    double* kt = (double*)s_raw + (size_t)w * S.rb * (p.n_pad >> 2) * 64;
    const int64_t row0 = (int64_t)t * S.rows + (int64_t)w * 16 * S.rb;
    if (reg) {
      // register-resident FP64 posterior, one block of 16 rows at a time,
      // observations staged in LDS above
      const double* xs = (const double*)s_raw;
      float* rbuf = (float*)(s_raw + kStageBytes) + (size_t)w * kReg32Rbuf;
      if (F32) {
        switch (p.n_pad >> 4) {  // a multiple of 4
          case 4: reg32_rows<4>(p, row0, S.rb, xs, rbuf, &part, &cnt); break;
          case 8: reg32_rows<8>(p, row0, S.rb, xs, rbuf, &part, &cnt); break;
          case 12: reg32_rows<12>(p, row0, S.rb, xs, rbuf, &part, &cnt); break;
          default: reg32_rows<16>(p, row0, S.rb, xs, rbuf, &part, &cnt); break;
        }
      } else {
        switch (p.n_pad >> 4) {
          case 4: reg_rows<4>(p, row0, S.rb, xs, &part, &cnt); break;
          case 8: reg_rows<8>(p, row0, S.rb, xs, &part, &cnt); break;
          case 12: reg_rows<12>(p, row0, S.rb, xs, &part, &cnt); break;
          default: reg_rows<16>(p, row0, S.rb, xs, &part, &cnt); break;
        }
      }
    } else if (S.rb == 2) {
      post16_wave<F32, 2>(p, row0, kt, &part, &cnt);
    } else {
      post16_wave<F32, 1>(p, row0, kt, &part, &cnt);
    }
  }
  if (l == 0) {
    s_wsum[w] = part;
    s_wcnt[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    int64_t c = 0;
    for (int i = 0; i < kBWaves; ++i) {
      s += s_wsum[i];
      c += s_wcnt[i];
    }
    p.vslots[t].sum = s;
    p.vslots[t].count = c;
  }
}

__global__ __launch_bounds__(kBThreads) void k_batch(const unsigned char* plan, BatchSync* sync, BatchCtl* ctl,
                                                     int cap) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  __shared__ uint32_t s_item;
  __shared__ int s_flag;
  __shared__ double s_wsum[kBWaves];
  __shared__ int64_t s_wcnt[kBWaves];
  __shared__ Best s_best[kBWaves];
  __shared__ int s_nan[kBWaves];

  const PlanHdr* hdr = (const PlanHdr*)plan;
  const BatchSession* ses = (const BatchSession*)(plan + sizeof(PlanHdr));
  const uint32_t* post_off = (const uint32_t*)(ses + cap);
  const uint32_t* acq_off = post_off + cap + 1;
  const int32_t* order = (const int32_t*)(acq_off + cap + 1);
  const uint32_t count = (uint32_t)hdr->count;
  const uint32_t end_fit = count, end_post = count + hdr->total_post, end_acq = end_post + hdr->total_acq;

  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(&ctl->next, 1u);
    __syncthreads();
    const uint32_t u = s_item;
    if (u >= end_acq) break;
    if (u < end_fit) {
      const int s = order[u];
      const BatchSession& S = ses[s];
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
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) atomicExch(&sync[s].fit_done, 1u);
    } else if (u < end_post) {
      const uint32_t v = u - end_fit;
      const int s = find_owner(post_off, (int)count, v);
      const int t = (int)(v - post_off[s]);
      const BatchSession& S = ses[s];
      const bool ok = wait_flag(&sync[s].fit_done, 1u, ctl, &s_flag);
      if (ok && S.post.st->status == BO_OK) {
        if (S.f32) post_tile<true>(S, t, s_raw, s_wsum, s_wcnt);
        else post_tile<false>(S, t, s_raw, s_wsum, s_wcnt);
      }
      if (last_of(&sync[s].post_done, (uint32_t)S.n_post, &s_flag)) {
        if (S.post.st->status == BO_OK)
          finish_lambda(S.post, S.n_post, (double*)s_raw, (int64_t*)(s_raw + kBThreads * sizeof(double)));
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) atomicExch(&sync[s].lam_ready, 1u);
      }
    } else {
      const uint32_t v = u - end_post;
      const int s = find_owner(acq_off, (int)count, v);
      const int j = (int)(v - acq_off[s]);
      const BatchSession& S = ses[s];
      (void)wait_flag(&sync[s].lam_ready, 1u, ctl, &s_flag);
      const int64_t c0 = (int64_t)j * S.acq_chunk;
      const int64_t c1 = c0 + S.acq_chunk < S.acq.n_valid ? c0 + S.acq_chunk : S.acq.n_valid;
      if (S.f32) acq_range<true>(S.acq, c0, c1, &S.acq.slots[j], s_best, s_nan);
      else acq_range<false>(S.acq, c0, c1, &S.acq.slots[j], s_best, s_nan);
      if (last_of(&sync[s].acq_done, (uint32_t)S.n_acq, &s_flag)) acq_finish(S.acq, S.n_acq, s_best, s_nan);
    }
  }
  // the last workgroup out re-arms the counters for the next replay
  __threadfence();
  if (threadIdx.x == 0) {
    if (atomicAdd(&ctl->exited, 1u) == gridDim.x - 1) {
      __threadfence();
      for (uint32_t s = 0; s < count; ++s) {
        atomicExch(&sync[s].fit_done, 0u);
        atomicExch(&sync[s].post_done, 0u);
        atomicExch(&sync[s].lam_ready, 0u);
        atomicExch(&sync[s].acq_done, 0u);
      }
      atomicExch(&ctl->next, 0u);
      atomicExch(&ctl->exited, 0u);
    }
  }
}

__global__ void k_batch_clear(BatchSync* sync, int cap, BatchCtl* ctl) {
  for (int i = threadIdx.x; i < cap; i += blockDim.x) sync[i] = BatchSync{0u, 0u, 0u, 0u};
  if (threadIdx.x == 0) *ctl = BatchCtl{0u, 0u, 0u, 0u};
}

constexpr size_t kBatchLds = kSmallLdsBytes;
static_assert(kBatchLds >= 2 * kBThreads * sizeof(double), "finish_lambda scratch");
static_assert(kBatchLds >= kStageBytes + kBWaves * kReg32Rbuf * sizeof(float), "staged observations and residuals");

// Posterior tile shape of one session: row blocks per wave and active waves,
// within the kernel's LDS (each wave parks rb * n_pad * 16 operand entries).
void tile_shape(int f32, int n_pad, int want_rb, int* rb, int* waves) {
  if (n_pad <= 16 * kRegJB) {
    // the register-resident posterior parks no operand in LDS
    *rb = want_rb == 2 ? 2 : 1;
    *waves = kBWaves;
    return;
  }
  const size_t esz = 8;  // both modes park FP64 operands
  *rb = 1;
  if (want_rb == 2 && (size_t)kBWaves * 2 * n_pad * 16 * esz <= kBatchLds) *rb = 2;
  int w = kBWaves;
  while (w > 1 && (size_t)w * (*rb) * n_pad * 16 * esz > kBatchLds) w >>= 1;
  *waves = w;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

#define BHIP(expr)                                                                               \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return set_error(BO_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

}  // namespace


// ------------------------------------------------------------ BatchCtx --

size_t BatchCtx::bytes(int cap) {
  return align256(plan_bytes(cap)) + align256(sizeof(BatchSync) * cap) +
         align256(sizeof(bo_acq_result) * cap + sizeof(BatchCtl));
}

bo_status BatchCtx::init(int cap_, void* workspace, size_t nbytes, hipStream_t stream_) {
  if (cap_ < 1) return set_error(BO_E_INVALID_ARG, "batch capacity must be >= 1");
  if (!workspace || ((uintptr_t)workspace & 255u)) return set_error(BO_E_WORKSPACE, "workspace NULL or misaligned");
  if (nbytes < bytes(cap_)) return set_error(BO_E_WORKSPACE, "workspace %zu bytes < %zu needed", nbytes, bytes(cap_));
  int dev = 0, cus = 0, per_cu = 0;
  BHIP(hipGetDevice(&dev));
  BHIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  BHIP(hipFuncSetAttribute((const void*)k_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchLds));
  BHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batch, kBThreads, kBatchLds));
  if (per_cu < 1) return set_error(BO_E_HIP, "batched kernel does not fit on a compute unit");
  cap = cap_;
  grid = cus * per_cu;
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
  sync = w;
  w += align256(sizeof(BatchSync) * cap);
  res_dev = (bo_acq_result*)w;
  ctl = w + sizeof(bo_acq_result) * cap;
  res_sz = sizeof(bo_acq_result) * cap + sizeof(BatchCtl);
  BHIP(hipHostMalloc((void**)&plan_host, plan_sz, hipHostMallocDefault));
  BHIP(hipHostMalloc((void**)&res_host, res_sz, hipHostMallocDefault));
  BHIP(hipEventCreateWithFlags(&done_ev, hipEventDisableTiming));
  hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(256), 0, stream, (BatchSync*)sync, cap, (BatchCtl*)ctl);
  BHIP(hipGetLastError());
  BHIP(hipStreamSynchronize(stream));
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
  unsigned char* base = plan_host;
  PlanHdr* hdr = (PlanHdr*)base;
  BatchSession* ses = (BatchSession*)(base + sizeof(PlanHdr));
  uint32_t* post_off = (uint32_t*)(ses + cap);
  uint32_t* acq_off = post_off + cap + 1;
  int32_t* order = (int32_t*)(acq_off + cap + 1);
  uint32_t tp = 0, ta = 0;
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
    BatchSession& B = ses[i];
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
    tile_shape(B.f32, n_pad_of(it.n), cfg.tile_rows / 16, &B.rb, &B.waves);
    B.rows = 16 * B.rb * B.waves;
    const int64_t nv = s->n_valid;
    B.n_post = (int32_t)std::max<int64_t>(1, (nv + B.rows - 1) / B.rows);
    B.acq_chunk = cfg.acq_chunk;
    B.n_acq = (int32_t)std::max<int64_t>(1, (nv + cfg.acq_chunk - 1) / cfg.acq_chunk);
    post_off[i] = tp;
    acq_off[i] = ta;
    tp += (uint32_t)B.n_post;
    ta += (uint32_t)B.n_acq;
  }
  post_off[count] = tp;
  acq_off[count] = ta;
  order_scratch.resize(count);
  for (int i = 0; i < count; ++i) order_scratch[i] = i;
  if (cfg.fit_order == 1)
    std::stable_sort(order_scratch.begin(), order_scratch.end(),
                     [&](int a, int c) { return items[a].n > items[c].n; });
  for (int i = 0; i < count; ++i) order[i] = order_scratch[i];
  hdr->count = count;
  hdr->total_post = tp;
  hdr->total_acq = ta;
  hdr->pad = 0;
  return BO_OK;
}

bo_status BatchCtx::capture() {
  BHIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  (void)hipMemcpyAsync(plan_dev, plan_host, plan_sz, hipMemcpyHostToDevice, stream);
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBThreads), kBatchLds, stream, plan_dev, (BatchSync*)sync,
                     (BatchCtl*)ctl, cap);
  (void)hipMemcpyAsync(res_host, res_dev, res_sz, hipMemcpyDeviceToHost, stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(stream, &g);
  if (e != hipSuccess) return set_error(BO_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return set_error(BO_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
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
  const BatchCtl* c = (const BatchCtl*)(res_host + sizeof(bo_acq_result) * cap);
  if (c->timeout) {
    hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(256), 0, stream, (BatchSync*)sync, cap, (BatchCtl*)ctl);
    (void)hipStreamSynchronize(stream);
    return set_error(BO_E_HIP, "batched step: a work-queue wait hit its spin limit");
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
  if (c->tile_rows != 16 && c->tile_rows != 32) return set_error(BO_E_INVALID_ARG, "tile_rows must be 16 or 32");
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
  b->cfg = bo_batch_config{16, 8192, 1, 0};
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
  const int rows[2] = {16, 32};
  const int chunks[3] = {4096, 8192, 32768};
  const int orders[2] = {1, 0};
  bo_batch_config best{};
  float best_ms = INFINITY;
  for (int r : rows)
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
