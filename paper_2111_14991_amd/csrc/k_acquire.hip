// Acquisition and selection (Sections III-C, III-D.2): EI, PI and LCB in their
// minimization form with the step's exploration factor, over the compacted
// candidates that have not been evaluated, and the arg-optimum of each:
// argmax EI, argmax PI, argmin LCB, ties to the lowest index, NaN never
// selected.  Per-workgroup winners go to fixed slots; the last workgroup
// reduces them and writes the step result.
#include "bo_internal.h"
#include "bo_device.h"

namespace bo {
namespace {

struct AcqKArgs {
  int64_t n_valid;
  uint32_t bits;
  const int32_t* orig;
  const uint8_t* visited;
  const void* mu;
  const void* var;
  AcqSlot* slots;
  DevState* st;
  bo_acq_result* out;
};

struct Best {
  double s[3];
  int32_t i[3];
};

__device__ __forceinline__ void take(Best& b, int q, double s, int32_t i) {
  if (better(s, i, b.s[q], b.i[q], q == 2)) {
    b.s[q] = s;
    b.i[q] = i;
  }
}

template <bool F32>
__global__ __launch_bounds__(kAcqThreads) void k_acquire(AcqKArgs a) {
  __shared__ Best s_best[kAcqThreads / 64];
  __shared__ int s_nan[kAcqThreads / 64];
  __shared__ int s_last;
  const DevState* st = a.st;
  const bool ok = st->status == BO_OK && st->post_status == BO_OK;
  Best b;
  for (int q = 0; q < 3; ++q) {
    b.s[q] = 0.0;
    b.i[q] = -1;
  }
  int nan_seen = 0;
  if (ok) {
    const double fb = st->f_best, lam = st->lambda;
    const int64_t c0 = (int64_t)blockIdx.x * kAcqThreads * kAcqPerThread + threadIdx.x;
    for (int q = 0; q < kAcqPerThread; ++q) {
      const int64_t c = c0 + (int64_t)q * kAcqThreads;
      if (c >= a.n_valid) break;
      if (a.visited && a.visited[a.orig[c]]) continue;
      double mu, var;
      if constexpr (F32) {
        mu = ((const float*)a.mu)[c];
        var = ((const float*)a.var)[c];
      } else {
        mu = ((const double*)a.mu)[c];
        var = ((const double*)a.var)[c];
      }
      double v[3];
      acquisitions64(mu, var, fb, lam, &v[0], &v[1], &v[2]);
      for (int k = 0; k < 3; ++k) {
        if (!(a.bits & (1u << k))) continue;
        if (v[k] != v[k]) {
          nan_seen = 1;
          continue;
        }
        take(b, k, v[k], (int32_t)c);
      }
    }
  }
  // wave reduction
  for (int off = 32; off > 0; off >>= 1) {
    for (int k = 0; k < 3; ++k) {
      const double os = __shfl_xor(b.s[k], off, 64);
      const int32_t oi = __shfl_xor(b.i[k], off, 64);
      take(b, k, os, oi);
    }
    nan_seen |= __shfl_xor(nan_seen, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_best[w] = b;
    s_nan[w] = nan_seen;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kAcqThreads / 64; ++i) {
      for (int k = 0; k < 3; ++k) take(b, k, s_best[i].s[k], s_best[i].i[k]);
      nan_seen |= s_nan[i];
    }
    AcqSlot& sl = a.slots[blockIdx.x];
    for (int k = 0; k < 3; ++k) {
      sl.score[k] = b.s[k];
      sl.idx[k] = b.i[k];
    }
    sl.nan_seen = nan_seen;
  }
  if (!last_block(&a.st->ticket_acq, &s_last)) return;
  // last workgroup: combine the slots (the order does not matter: the
  // comparison is a total order on (score, index))
  Best r;
  for (int q = 0; q < 3; ++q) {
    r.s[q] = 0.0;
    r.i[q] = -1;
  }
  int nn = 0;
  for (int s = threadIdx.x; s < (int)gridDim.x; s += kAcqThreads) {
    const AcqSlot sl = a.slots[s];
    for (int k = 0; k < 3; ++k) take(r, k, sl.score[k], sl.idx[k]);
    nn |= sl.nan_seen;
  }
  for (int off = 32; off > 0; off >>= 1) {
    for (int k = 0; k < 3; ++k) {
      const double os = __shfl_xor(r.s[k], off, 64);
      const int32_t oi = __shfl_xor(r.i[k], off, 64);
      take(r, k, os, oi);
    }
    nn |= __shfl_xor(nn, off, 64);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    s_best[w] = r;
    s_nan[w] = nn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kAcqThreads / 64; ++i) {
      for (int k = 0; k < 3; ++k) take(r, k, s_best[i].s[k], s_best[i].i[k]);
      nn |= s_nan[i];
    }
    bo_acq_result res;
    const double qnan = __longlong_as_double(0x7ff8000000000000LL);
    int status = st->status != BO_OK ? st->status : st->post_status;
    for (int k = 0; k < 3; ++k) {
      const bool have = status == BO_OK && r.i[k] >= 0;
      res.idx[k] = have ? (int64_t)a.orig[r.i[k]] : -1;
      res.score[k] = have ? r.s[k] : qnan;
    }
    if (status == BO_OK && nn) status = BO_E_NUMERIC;
    res.lambda = st->lambda;
    res.var_mean = st->var_mean;
    res.jitter = st->jitter;
    res.f_best = st->f_best;
    res.mean_y = st->mean_y;
    res.n_unmasked = st->status == BO_OK ? st->n_unmasked : 0;
    res.status = status;
    res.n_obs = st->n;
    *a.out = res;
    a.st->ticket_acq = 0;
  }
}

// Posterior written back in the caller's enumeration (NaN where excluded).
template <bool F32>
__global__ void k_scatter_post(int64_t N, const int32_t* inv_map, const uint8_t* visited, const void* mu,
                               const void* var, double* mu_out, double* var_out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const double qnan = __longlong_as_double(0x7ff8000000000000LL);
  const int32_t pos = inv_map[c];
  double m = qnan, v = qnan;
  if (pos >= 0 && !(visited && visited[c])) {
    if constexpr (F32) {
      m = ((const float*)mu)[pos];
      v = ((const float*)var)[pos];
    } else {
      m = ((const double*)mu)[pos];
      v = ((const double*)var)[pos];
    }
  }
  if (mu_out) mu_out[c] = m;
  if (var_out) var_out[c] = v;
}

}  // namespace

int64_t acquire_blocks(int64_t n_valid) {
  const int64_t per = (int64_t)kAcqThreads * kAcqPerThread;
  const int64_t g = (n_valid + per - 1) / per;
  return g > 0 ? g : 1;
}

hipError_t launch_acquire(const DevPtrs& P, const Layout& Lo, int64_t n_valid, const uint8_t* visited,
                          const AcqArgs& acq, bo_acq_result* out_dev, hipStream_t st) {
  AcqKArgs a{};
  a.n_valid = n_valid;
  a.bits = acq.bits ? acq.bits : 7u;
  a.orig = P.orig;
  a.visited = visited;
  a.mu = P.mu;
  a.var = P.var;
  a.slots = P.aslots;
  a.st = P.st;
  a.out = out_dev;
  const int grid = (int)acquire_blocks(n_valid);
  if (Lo.prec == BO_FP64)
    hipLaunchKernelGGL(k_acquire<false>, dim3(grid), dim3(kAcqThreads), 0, st, a);
  else
    hipLaunchKernelGGL(k_acquire<true>, dim3(grid), dim3(kAcqThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_scatter_posterior(const DevPtrs& P, const Layout& Lo, int64_t n_valid,
                                    const uint8_t* visited, double* mu, double* var, hipStream_t st) {
  (void)n_valid;
  const int grid = (int)((Lo.N + 255) / 256);
  if (Lo.prec == BO_FP64)
    hipLaunchKernelGGL(k_scatter_post<false>, dim3(grid), dim3(256), 0, st, Lo.N, P.inv_map, visited, P.mu,
                       P.var, mu, var);
  else
    hipLaunchKernelGGL(k_scatter_post<true>, dim3(grid), dim3(256), 0, st, Lo.N, P.inv_map, visited, P.mu, P.var,
                       mu, var);
  return hipGetLastError();
}

}  // namespace bo
