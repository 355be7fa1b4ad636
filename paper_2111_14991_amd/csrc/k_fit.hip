// Kernels and launch sequences of the FP64 surrogate fit; the device code of
// every step is in fit_body.h.
#include <algorithm>

#include "fit_body.h"

namespace bo {
namespace {

__global__ __launch_bounds__(kSmallThreads) void k_fit_small(FitArgs a) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  fit_small_run(a, s_raw);
}

__global__ __launch_bounds__(kSmallThreads) void k_append(FitArgs a) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  append_run(a, s_raw);
}

// ======================= large fit: one launch per phase ==================
// Workgroup 0: observations, their mean and incumbent, the index check and
// the fit state; workgroup b >= 1: the coordinates of observations
// 64 (b - 1) .. 64 b - 1, one per thread of its first wave (the augmented
// rows of the BF16X3 form are long enough to be worth spreading).
__global__ __launch_bounds__(1024) void k_fitL_gather(FitArgs a) {
  __shared__ double s_red[2 * 1024];
  __shared__ int s_pos[kMaxN];
  __shared__ int s_flag;
  if (blockIdx.x == 0) {
    fit_gather<false>(a, s_red, s_pos, &s_flag);
    return;
  }
  const int i = ((int)blockIdx.x - 1) * 64 + (int)threadIdx.x;
  if (threadIdx.x < 64 && i < a.n_pad) gather_coords_row(a, i);
}

constexpr int kAThreads = 2 * TT;
constexpr uint32_t kGridSpinLimit = 1u << 20;  // ~0.1 s of s_sleep 2; a legitimate wait is ~20 us

// Grid-wide barrier of the persistent fit: barrier b (counted in *count by
// every workgroup) completes when every workgroup has arrived (arrivals
// counted cumulatively in st->gs_arrive; the last one publishes b in
// st->gs_release).  Waits are bounded: a wait that reaches the spin limit
// raises st->gs_abort, which ends every other wait too, so that all
// workgroups leave.  Returns false after an abort, in every thread.
__device__ bool grid_sync(DevState* st, uint32_t* count, int* s_ok) {
  __syncthreads();
  *count += 1;
  if (threadIdx.x == 0) {
    int ok = 1;
    __threadfence();
    const uint32_t want = *count;
    const uint32_t prev = atomicAdd(&st->gs_arrive, 1u);
    if (prev + 1 == gridDim.x * want) {
      __hip_atomic_store(&st->gs_release, want, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      while (__hip_atomic_load(&st->gs_release, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < want) {
        if (__hip_atomic_load(&st->gs_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kGridSpinLimit) {
          atomicExch(&st->gs_abort, 1u);
          ok = 0;
          break;
        }
      }
    }
    if (__hip_atomic_load(&st->gs_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) ok = 0;
    __threadfence();
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// The persistent fit's tile operations as separate functions, so that each
// is register-allocated on its own (inlined into one kernel they would all
// compete for the same registers).  LDS pointers cross the calls in the LDS
// address space, so that the accesses inside stay LDS instructions.
#define LDS __attribute__((address_space(3)))
typedef LDS Tile* LTiles;
typedef LDS double (*LBuf)[64];

__device__ __noinline__ void build_op(const FitArgs& a, int t, double delta, LDS double* lxs, int tt) {
  int i, j;
  tri_decode(t, &i, &j);
  op_build(a, i, j, delta, (double*)lxs, tt);
}

// Whether a pivot failed in a phase up to `phase` of the current attempt.
// Workgroup 0 records the phase of a failure in st->fail_at (once per
// attempt); a workgroup that reads it late, after workgroup 0 has moved on,
// still sees only failures of the phases it has passed, so every workgroup
// takes the same decision after the same barrier.
__device__ __forceinline__ bool failed_by(DevState* st, uint32_t phase) {
  return __hip_atomic_load(&st->fail_at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= phase;
}

// Items of block step k for the workgroups after the first (team 0 of each):
//   panels L_bk, k + 2 <= b < NB (L_{k+1,k} is the look-ahead's);
//   block row k of the inverse, X_kb, b < k;
//   step k-1's trailing tiles (i, j), k < j <= i, except (k+1, k+1) (the
//     look-ahead's), and its inverse tiles R_ij below row k (i > k, j < k).
// Panels and inverse tiles first bring their own input up to date with step
// k-1's update of it, as the blocked factorization's launch per half-step
// would have; every tile receives its updates in step order, so the factor
// does not depend on the schedule.
__device__ __forceinline__ int step_items(int NB, int k) {
  const int m = NB - k;
  const int npanel = NB - k - 2 > 0 ? NB - k - 2 : 0;
  const int ntr = k > 0 ? (m - 1) * m / 2 - (m >= 2 ? 1 : 0) : 0;
  const int ninv = k > 0 ? (m - 1) * k : 0;
  return npanel + k + ntr + ninv;
}

__device__ __forceinline__ void step_item(const FitArgs& a, int k, int it, Tile* tiles, int tt, bool active) {
  const int NB = a.NB, m = NB - k;
  const int npanel = NB - k - 2 > 0 ? NB - k - 2 : 0;
  if (it < npanel + k) {
    // panel (b > k) or inverse (b < k) item of step k
    const int b = it < npanel ? k + 2 + it : it - npanel;
    if (k > 0) {
      const int t = b > k ? (b - k) * (b - k + 1) / 2 : m * (m + 1) / 2 + b;
      stepB_item(a, k - 1, t, tiles[1], tiles[2], tt, active);
      __syncthreads();
    }
    stepA_item(a, k, b, tiles[0], tiles[1], tiles[2], tt, active);
    return;
  }
  const int e = it - npanel - k;
  const int ntr = (m - 1) * m / 2 - (m >= 2 ? 1 : 0);
  int t;
  if (e < ntr) {
    // trailing tiles with k + 1 <= j <= i, after (k + 1, k + 1)
    int i, j;
    tri_decode(e + 1, &i, &j);
    i += k + 1;
    j += k + 1;
    t = (i - k) * (i - k + 1) / 2 + (j - k);
  } else {
    t = m * (m + 1) / 2 + k + (e - ntr);
  }
  stepB_item(a, k - 1, t, tiles[1], tiles[2], tt, active);
}

// The look-ahead of step k (workgroup 0, both teams, k + 1 < NB): step
// k-1's updates of tiles (k+1, k) (team 0) and (k+1, k+1) (team 1) -- items
// 1 and 2 of its trailing list --, the panel L_{k+1,k} with L_kk^-1, then
// tile k+1 factored and inverted with step k's update applied in LDS and
// stored (L, L^-1 and the diagonal inverse).  A pivot failure is recorded in
// st->fail_at as phase k + 1.
__device__ __forceinline__ void lookahead(const FitArgs& a, int k, double delta, Tile* tiles, double (*colbuf)[64],
                                          double (*xbuf)[64]) {
  const int tid = threadIdx.x, team = tid / TT, tt = tid % TT;
  if (k > 0) stepB_item(a, k - 1, 1 + team, tiles[2 * team], tiles[2 * team + 1], tt, true);
  __syncthreads();
  if (team == 0) load_dinv(tiles[0], a, k, tt);
  __syncthreads();
  stepA_item(a, k, k + 1, tiles[0], tiles[1], tiles[2], tt, team == 0);
  __syncthreads();
  double pmin = INFINITY;
  const bool f = op_diag<kAThreads>(a, k + 1, delta, tiles[0], tiles[1], colbuf, xbuf, &pmin, &tiles[2]);
  if (f) {
    if (tid == 0) atomicExch(&a.st->fail_at, (uint32_t)(k + 1));
  } else {
    if (tid == 0) a.st->min_piv = fmin(a.st->min_piv, pmin);
    stepA_item(a, k + 1, k + 1, tiles[0], tiles[1], tiles[2], tt, team == 0);
  }
}

// Tile 0 factored and inverted (workgroup 0); failure recorded as phase 0.
__device__ __forceinline__ void diag0(const FitArgs& a, double delta, Tile* tiles, double (*colbuf)[64],
                                      double (*xbuf)[64]) {
  const int tid = threadIdx.x, team = tid / TT, tt = tid % TT;
  double pmin = INFINITY;
  const bool fail = op_diag<kAThreads>(a, 0, delta, tiles[0], tiles[1], colbuf, xbuf, &pmin);
  if (fail) {
    if (tid == 0) atomicExch(&a.st->fail_at, 0u);
  } else {
    if (tid == 0) a.st->min_piv = pmin;
    stepA_item(a, 0, 0, tiles[0], tiles[1], tiles[2], tt, team == 0);
  }
}

// The same pieces as separate functions for the persistent kernel.
__device__ __noinline__ void step_item_op(const FitArgs& a, int k, int it, LTiles lt, int tt, bool active) {
  step_item(a, k, it, (Tile*)lt, tt, active);
}
__device__ __noinline__ void lookahead_op(const FitArgs& a, int k, double delta, LTiles lt, LBuf lcol, LBuf lx) {
  lookahead(a, k, delta, (Tile*)lt, (double(*)[64])lcol, (double(*)[64])lx);
}
__device__ __noinline__ void diag0_op(const FitArgs& a, double delta, LTiles lt, LBuf lcol, LBuf lx) {
  diag0(a, delta, (Tile*)lt, (double(*)[64])lcol, (double(*)[64])lx);
}

// z = L^-1 (y - m) (one row per wave) and the packed operand, over the grid.
__device__ __forceinline__ void z_and_pack(const FitArgs& a, int wave, int nwave, int lane, int64_t thread,
                                           int64_t nthreads) {
  const double mean_y = a.st->mean_y;
  for (int i = wave; i < a.n_pad; i += nwave) alpha_z_row(a, i, mean_y, lane);
  int64_t nfrag;
  const int64_t ne = pack_count(a, &nfrag);
  for (int64_t e = thread; e < ne; e += nthreads) {
    if (a.prec == BO_BF16X3) pack_elem32(a, e, nfrag);
    else pack_elem16(a, e);
  }
}

// ---- first attempt: one launch per phase and step ----
__device__ __forceinline__ bool fit_stopped(const FitArgs& a) {
  return a.st->status != BO_OK || a.st->fail_at != 0xffffffffu;
}

__global__ __launch_bounds__(TT) void k_fitL_build(FitArgs a) {
  if (fit_stopped(a)) return;
  __shared__ double xs[128 * (kMaxD + 1)];
  int i, j;
  tri_decode(blockIdx.x, &i, &j);
  op_build(a, i, j, jitter_of(a.noise, a.amp, 0), xs, threadIdx.x);
}

// Step k of the first attempt in one launch.  Workgroups b < NB each
// factor the diagonal tile k (step k-1's update of it applied in LDS), then
// bring their own input up to date -- the trailing tile (b, k) or the
// inverse tile (k, b) of step k-1 -- and compute item b of step k: the panel
// tile L_bk (b > k), the tiles L_kk, L_kk^-1 (b = k), or the inverse tile
// X_kb (b < k).  The workgroups after NB take step k-1's other trailing and
// inverse tiles, which nothing in this launch reads.  Step k-1's items keep
// their arithmetic and order, so the factor is the one a launch per
// half-step would give (and the one the retry kernel's schedule gives).
__global__ __launch_bounds__(kAThreads) void k_fitL_step(FitArgs a, int k) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  Tile* tiles = reinterpret_cast<Tile*>(s_raw);
  __shared__ __align__(16) double s_colbuf[2][64];
  __shared__ __align__(16) double s_xbuf[2][64];
  if (fit_stopped(a)) return;
  const int NB = a.NB, tt = threadIdx.x;
  const int m = NB - k;  // step k-1's trailing tiles span rows and columns k .. NB-1
  if ((int)blockIdx.x >= NB) {
    // step k-1's trailing tiles off column k, then its inverse tiles below row k
    const int v = (int)blockIdx.x - NB, ntr = (m - 1) * m / 2;
    int t;
    if (v < ntr) {
      int i, j;
      tri_decode(v, &i, &j);
      t = (i + 1) * (i + 2) / 2 + j + 1;
    } else {
      t = m * (m + 1) / 2 + k + (v - ntr);
    }
    stepB_item(a, k - 1, t, tiles[0], tiles[1], tt % TT, tt < TT);
    return;
  }
  const int b = blockIdx.x;
  double pmin = INFINITY;
  const bool fail = op_diag<kAThreads>(a, k, jitter_of(a.noise, a.amp, 0), tiles[0], tiles[1], s_colbuf, s_xbuf,
                                       &pmin, k > 0 ? &tiles[2] : nullptr);
  // launches run in order: block 0 folds this tile's pivots into the factor's minimum
  if (!fail && b == 0 && tt == 0) a.st->min_piv = fmin(k == 0 ? INFINITY : a.st->min_piv, pmin);
  if (fail) {
    if (b == 0 && tt == 0) atomicExch(&a.st->fail_at, (uint32_t)k);
    return;
  }
  if (k > 0 && b != k) {
    // step k-1's item for tile (b, k) (trailing) or (k, b) (inverse); tiles
    // 1 and 2 are free here, tile 0 holds L_kk^-1
    const int t = b > k ? (b - k) * (b - k + 1) / 2 : m * (m + 1) / 2 + b;
    stepB_item(a, k - 1, t, tiles[1], tiles[2], tt % TT, tt < TT);
    __syncthreads();
  }
  stepA_item(a, k, b, tiles[0], tiles[1], tiles[2], tt % TT, tt < TT);
}

__global__ __launch_bounds__(TT) void k_fitL_zpack(FitArgs a) {
  if (fit_stopped(a)) return;
  const int64_t thread = (int64_t)blockIdx.x * TT + threadIdx.x;
  z_and_pack(a, (int)(thread >> 6), (int)(gridDim.x * (TT / 64)), threadIdx.x & 63, thread,
             (int64_t)gridDim.x * TT);
}

// alpha = L^-T z: one wave per column; up to 256 observations one
// workgroup of 512 in the one-workgroup fit's order (lt_cols_pair), so that
// both fits give the same bits.
__global__ __launch_bounds__(kAThreads) void k_fitL_alpha(FitArgs a) {
  __shared__ double s_part[256];
  if (fit_stopped(a)) return;
  if (a.n_pad <= kSmallFitMax) {
    lt_cols_pair(
        a, a.n_pad, a.n, [&](int j) { return a.z[j]; }, [&](int i, double v) { a.alpha[i] = i < a.n ? v : 0.0; },
        s_part);
  } else {
    const int i = blockIdx.x * (kAThreads / 64) + (threadIdx.x >> 6);
    if (i < a.n_pad) alpha_a_row(a, i, threadIdx.x & 63);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.st->jitter = jitter_of(a.noise, a.amp, 0);
    a.st->attempt = 0;
    a.st->need_retry = 0;
  }
}

// Attempts 1 .. tries-1 of the jitter schedule after a failed first attempt,
// in one launch of co-resident workgroups of two teams with grid-wide
// barriers between the phases (no host round trip, so asynchronous and
// graph-captured steps escalate like synchronous ones):
//   K_nn + delta I (all tile-teams), tile 0 (workgroup 0), then block steps
//   k = 0 .. NB-1 (workgroup 0 the look-ahead, the others the step's items
//   with L_kk^-1 from memory), then z and the packed operand, then alpha.
// A pivot failure (phase recorded by workgroup 0, read by every workgroup
// after the next barrier) ends the attempt; after the last one the status is
// BO_E_NOT_PD.  When the first attempt succeeded every workgroup leaves at
// once.
__global__ __launch_bounds__(kAThreads) void k_fitL(FitArgs a) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  Tile* tiles = reinterpret_cast<Tile*>(s_raw);  // four tiles
  __shared__ __align__(16) double s_colbuf[2][64];
  __shared__ __align__(16) double s_xbuf[2][64];
  __shared__ int s_ok;
  DevState* st = a.st;
  if (st->status != BO_OK) return;            // the gather rejected the observations
  if (!failed_by(st, 0xfffffffeu)) return;    // the first attempt succeeded
  const int G = gridDim.x, bid = blockIdx.x, tid = threadIdx.x;
  const int team = tid / TT, tt = tid % TT;
  const int NB = a.NB;
  uint32_t bars = 0;
  bool failed = true;
  int attempt = 1;
  for (; attempt < a.tries; ++attempt) {
    // every workgroup has read the record before it is cleared, and sees it
    // cleared before the attempt starts
    if (!grid_sync(st, &bars, &s_ok)) return;
    if (bid == 0 && tid == 0) atomicExch(&st->fail_at, 0xffffffffu);
    if (!grid_sync(st, &bars, &s_ok)) return;
    const double delta = jitter_of(a.noise, a.amp, attempt);
    // K_nn + delta I, one tile per team
    const int nlow = NB * (NB + 1) / 2;
    for (int base = 0; base < nlow; base += 2 * G) {
      const int t = base + 2 * bid + team;
      if (t < nlow) {
        build_op(a, t, delta, (LDS double*)&tiles[team][0][0], tt);
      } else {
        __syncthreads();
        __syncthreads();
      }
    }
    if (!grid_sync(st, &bars, &s_ok)) return;
    if (bid == 0) diag0_op(a, delta, (LTiles)tiles, (LBuf)s_colbuf, (LBuf)s_xbuf);
    if (!grid_sync(st, &bars, &s_ok)) return;
    bool fail = failed_by(st, 0u);
    for (int k = 0; k < NB && !fail; ++k) {
      if (bid == 0) {
        if (k + 1 < NB) lookahead_op(a, k, delta, (LTiles)tiles, (LBuf)s_colbuf, (LBuf)s_xbuf);
      } else {
        const int nit = step_items(NB, k);
        if (nit > 0) {
          if (team == 0) load_dinv(tiles[0], a, k, tt);
          __syncthreads();
          for (int it = bid - 1; it < nit; it += G - 1) step_item_op(a, k, it, (LTiles)tiles, tt, team == 0);
        }
      }
      if (!grid_sync(st, &bars, &s_ok)) return;
      fail = failed_by(st, (uint32_t)(k + 1));
    }
    if (!fail) {
      failed = false;
      break;
    }
  }
  if (failed) {
    if (bid == 0 && tid == 0) {
      st->attempt = a.tries - 1;
      st->need_retry = 0;
      st->status = BO_E_NOT_PD;
    }
    return;
  }
  const int wave = (bid * kAThreads + tid) >> 6, nwave = G * (kAThreads / 64), lane = tid & 63;
  z_and_pack(a, wave, nwave, lane, (int64_t)bid * kAThreads + tid, (int64_t)G * kAThreads);
  if (!grid_sync(st, &bars, &s_ok)) return;
  if (a.n_pad <= kSmallFitMax) {
    double* s_part = reinterpret_cast<double*>(s_raw);  // the tiles are free by now
    if (bid == 0)
      lt_cols_pair(
          a, a.n_pad, a.n, [&](int j) { return a.z[j]; }, [&](int i, double v) { a.alpha[i] = i < a.n ? v : 0.0; },
          s_part);
  } else {
    for (int i = wave; i < a.n_pad; i += nwave) alpha_a_row(a, i, lane);
  }
  if (bid == 0 && tid == 0) {
    st->jitter = jitter_of(a.noise, a.amp, attempt);
    st->attempt = attempt;
    st->need_retry = 0;
  }
}

// Status after a persistent fit whose barriers were aborted (a wait hit its
// spin limit: the workgroups were not all resident).
__global__ void k_fitL_check(DevState* st) {
  if (threadIdx.x == 0 && st->gs_abort != 0u && st->status == BO_OK) st->status = BO_E_HIP;
}

hipError_t set_lds(const void* f, size_t bytes) {
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}


hipError_t prepare() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = set_lds((const void*)k_fit_small, kSmallLdsBytes);
  if (e == hipSuccess) e = set_lds((const void*)k_append, kSmallLdsBytes);
  if (e == hipSuccess) e = set_lds((const void*)k_fitL, 4 * sizeof(Tile));
  if (e == hipSuccess) e = set_lds((const void*)k_fitL_step, 3 * sizeof(Tile));
  if (e == hipSuccess) done = true;
  return e;
}

}  // namespace

hipError_t launch_fit_small(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                            const double* y_in, int n, hipStream_t st) {
  hipError_t e = prepare();
  if (e != hipSuccess) return e;
  FitArgs a = make_args(P, Lo, g, obs_idx, y_in, n);
  hipLaunchKernelGGL(k_fit_small, dim3(1), dim3(kSmallThreads), kSmallLdsBytes, st, a);
  return hipGetLastError();
}

// Rank-1 append of observation n - 1 (n <= 256) to the current fit, or a
// refit when that is not possible (append_run).
hipError_t launch_fit_append(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                             const double* y_in, int n, hipStream_t st) {
  hipError_t e = prepare();
  if (e != hipSuccess) return e;
  FitArgs a = make_args(P, Lo, g, obs_idx, y_in, n);
  hipLaunchKernelGGL(k_append, dim3(1), dim3(kSmallThreads), kSmallLdsBytes, st, a);
  return hipGetLastError();
}

// The gather (one workgroup); the first attempt of the jitter schedule as
// one launch per phase and block step; then, on the device, the other
// attempts when the first one failed (k_fitL, which leaves at once
// otherwise): no host round trip, so asynchronous and graph-captured steps
// escalate the jitter like synchronous ones.  first_attempt is accepted for
// the interface and must be 0.
hipError_t launch_fit_large(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                            const double* y_in, int n, int first_attempt, hipStream_t st) {
  (void)first_attempt;
  hipError_t e = prepare();
  if (e != hipSuccess) return e;
  static int resident = 0;  // workgroups of k_fitL that fit on the device at once
  if (resident == 0) {
    int dev = 0, cus = 0, per = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_fitL, kAThreads, 4 * sizeof(Tile));
    if (e != hipSuccess) return e;
    resident = cus * (per > 0 ? per : 1);
  }
  FitArgs a = make_args(P, Lo, g, obs_idx, y_in, n);
  const int NB = a.NB;
  const size_t lds = 4 * sizeof(Tile);
  int most = 0;
  hipLaunchKernelGGL(k_fitL_gather, dim3(1 + a.n_pad / 64), dim3(1024), 0, st, a);
  // first attempt
  hipLaunchKernelGGL(k_fitL_build, dim3(NB * (NB + 1) / 2), dim3(TT), 0, st, a);
  for (int k = 0; k < NB; ++k) {
    // NB workgroups for step k, plus step k-1's tiles that no item of step k reads
    const int m = NB - k;
    const int extra = k > 0 ? (m - 1) * m / 2 + k * (m - 1) : 0;
    hipLaunchKernelGGL(k_fitL_step, dim3(NB + extra), dim3(kAThreads), 3 * sizeof(Tile), st, a, k);
    // the retry kernel's busiest step: look-ahead + items
    const int npanel = NB - k - 2 > 0 ? NB - k - 2 : 0;
    const int ntr = k > 0 ? (m - 1) * m / 2 - (m >= 2 ? 1 : 0) : 0;
    most = std::max(most, npanel + k + ntr + (k > 0 ? (m - 1) * k : 0));
  }
  hipLaunchKernelGGL(k_fitL_zpack, dim3(256), dim3(TT), 0, st, a);
  hipLaunchKernelGGL(k_fitL_alpha, dim3(a.n_pad <= kSmallFitMax ? 1 : a.n_pad / (kAThreads / 64)), dim3(kAThreads), 0,
                     st, a);
  // the other attempts, on the device, when the first one failed
  if (resident < 2) return hipErrorInvalidConfiguration;
  const int G = std::max(2, std::min(most + 1, resident));
  hipLaunchKernelGGL(k_fitL, dim3(G), dim3(kAThreads), lds, st, a);
  hipLaunchKernelGGL(k_fitL_check, dim3(1), dim3(64), 0, st, P.st);
  return hipGetLastError();
}

}  // namespace bo
