// Kernels and launch sequences of the FP64 surrogate fit; the device code of
// every step is in fit_body.h.
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
__global__ __launch_bounds__(1024) void k_fitL_gather(FitArgs a) {
  __shared__ double s_red[2 * 1024];
  __shared__ int s_pos[kMaxN];
  __shared__ int s_flag;
  fit_gather(a, s_red, s_pos, &s_flag);
}

__global__ __launch_bounds__(TT) void k_fitL_build(FitArgs a, int attempt) {
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  __shared__ double xs[128 * (kMaxD + 1)];
  int i, j;
  tri_decode(blockIdx.x, &i, &j);
  op_build(a, i, j, jitter_of(a.noise, a.amp, attempt), xs, threadIdx.x);
}

constexpr int kAThreads = 2 * TT;

// Step k of the large fit in one launch.  Workgroups b < NB each factor the
// diagonal tile k (step k-1's update of it applied in LDS), then bring their
// own input up to date -- the trailing tile (b, k) or the inverse tile
// (k, b) of step k-1 -- and compute item b of step k: the panel tile L_bk
// (b > k), the tiles L_kk, L_kk^-1 (b = k), or the inverse tile X_kb (b < k).
// The workgroups after NB take step k-1's other trailing and inverse tiles,
// which nothing in this launch reads.  Step k-1's items keep their
// arithmetic and order, so the factor is the one a launch per half-step
// would give.
__global__ __launch_bounds__(kAThreads) void k_fitL_step(FitArgs a, int k, int attempt) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  Tile* tiles = reinterpret_cast<Tile*>(s_raw);
  __shared__ __align__(16) double s_colbuf[2][64];
  __shared__ __align__(16) double s_xbuf[2][64];
  if (a.st->status != BO_OK || a.st->fail_flag) return;
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
  const bool fail = op_diag<kAThreads>(a, k, jitter_of(a.noise, a.amp, attempt), tiles[0], tiles[1], s_colbuf,
                                       s_xbuf, &pmin, k > 0 ? &tiles[2] : nullptr);
  // launches run in order: block 0 folds this tile's pivots into the factor's minimum
  if (!fail && b == 0 && tt == 0) a.st->min_piv = fmin(k == 0 ? INFINITY : a.st->min_piv, pmin);
  if (fail) {
    if (b == 0 && tt == 0) {
      a.st->fail_flag = 1;
      a.st->attempt = attempt;
    }
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

__global__ __launch_bounds__(TT) void k_fitL_alpha_z(FitArgs a) {
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  const int i = blockIdx.x * (TT / 64) + (threadIdx.x >> 6);
  if (i < a.n_pad) alpha_z_row(a, i, a.st->mean_y, threadIdx.x & 63);
}

__global__ __launch_bounds__(TT) void k_fitL_alpha_a(FitArgs a) {
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  const int i = blockIdx.x * (TT / 64) + (threadIdx.x >> 6);
  if (i < a.n_pad) alpha_a_row(a, i, threadIdx.x & 63);
}

__global__ __launch_bounds__(TT) void k_fitL_pack(FitArgs a, int attempt) {
  DevState* st = a.st;
  if (st->status != BO_OK) return;
  if (st->fail_flag) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->need_retry = (attempt + 1 < a.tries) ? 1 : 0;
      st->status = BO_E_NOT_PD;
    }
    return;
  }
  int64_t nfrag;
  const int64_t ne = pack_count(a, &nfrag);
  for (int64_t e = (int64_t)blockIdx.x * TT + threadIdx.x; e < ne; e += (int64_t)gridDim.x * TT) {
    if (a.prec == BO_BF16X3) pack_elem32(a, e, nfrag);
    else pack_elem16(a, e);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->jitter = jitter_of(a.noise, a.amp, attempt);
    st->attempt = attempt;
    st->need_retry = 0;
  }
}

// Re-arms the large fit for the next jitter attempt after a pivot failure.
__global__ void k_fitL_rearm(DevState* st) {
  if (threadIdx.x == 0 && st->status == BO_E_NOT_PD && st->need_retry) {
    st->status = BO_OK;
    st->fail_flag = 0;
    st->need_retry = 0;
  }
}

hipError_t set_lds(const void* f, size_t bytes) {
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}


hipError_t prepare() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = set_lds((const void*)k_fit_small, kSmallLdsBytes);
  if (e == hipSuccess) e = set_lds((const void*)k_append, kSmallLdsBytes);
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

// One attempt of the jitter schedule.  The gather phase runs only on the
// first attempt.  On a pivot failure st->need_retry is set and st->status =
// BO_E_NOT_PD; the host retries with the next attempt.
hipError_t launch_fit_large(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                            const double* y_in, int n, int attempt, hipStream_t st) {
  hipError_t e = prepare();
  if (e != hipSuccess) return e;
  FitArgs a = make_args(P, Lo, g, obs_idx, y_in, n);
  const int NB = a.NB;
  if (attempt == 0) hipLaunchKernelGGL(k_fitL_gather, dim3(1), dim3(1024), 0, st, a);
  else hipLaunchKernelGGL(k_fitL_rearm, dim3(1), dim3(64), 0, st, P.st);
  hipLaunchKernelGGL(k_fitL_build, dim3(NB * (NB + 1) / 2), dim3(TT), 0, st, a, attempt);
  for (int k = 0; k < NB; ++k) {
    // NB workgroups for step k, plus step k-1's tiles that no item of step k reads
    const int m = NB - k;
    const int extra = k > 0 ? (m - 1) * m / 2 + k * (m - 1) : 0;
    hipLaunchKernelGGL(k_fitL_step, dim3(NB + extra), dim3(kAThreads), 3 * sizeof(Tile), st, a, k, attempt);
  }
  const int rows = a.n_pad / (TT / 64);
  hipLaunchKernelGGL(k_fitL_alpha_z, dim3(rows), dim3(TT), 0, st, a);
  hipLaunchKernelGGL(k_fitL_alpha_a, dim3(rows), dim3(TT), 0, st, a);
  hipLaunchKernelGGL(k_fitL_pack, dim3(512), dim3(TT), 0, st, a, attempt);
  return hipGetLastError();
}

}  // namespace bo
