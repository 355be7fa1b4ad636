// Acquisition and selection (Sections III-C, III-D.2): EI, PI and LCB in their
// minimization form with the step's exploration factor over the compacted
// candidates that have not been evaluated, and the arg-optimum of each
// (argmax EI, argmax PI, argmin LCB, ties to the lowest index, NaN never
// selected).  A workgroup reduces a range of candidates to one slot; the last
// workgroup combines the slots and writes the step result.  Shared by the
// single-session and the batched kernels.
#pragma once
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
  double* vals[3];  // optional per-candidate EI, PI, LCB in the caller's enumeration
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

__device__ __forceinline__ void best_init(Best& b) {
  for (int q = 0; q < 3; ++q) {
    b.s[q] = 0.0;
    b.i[q] = -1;
  }
}

// Reduces (b, nan) over the workgroup; the result is valid in thread 0.
// s_best / s_nan: one entry per wave.
__device__ __forceinline__ void acq_block_reduce(Best& b, int& nan_seen, Best* s_best, int* s_nan) {
  for (int off = 32; off > 0; off >>= 1) {
    for (int k = 0; k < 3; ++k) {
      const double os = __shfl_xor(b.s[k], off, 64);
      const int32_t oi = __shfl_xor(b.i[k], off, 64);
      take(b, k, os, oi);
    }
    nan_seen |= __shfl_xor(nan_seen, off, 64);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    s_best[w] = b;
    s_nan[w] = nan_seen;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      for (int k = 0; k < 3; ++k) take(b, k, s_best[i].s[k], s_best[i].i[k]);
      nan_seen |= s_nan[i];
    }
  }
}

// Acquisitions of compacted candidates [c_begin, c_end) by the workgroup
// (thread stride blockDim.x), reduced into *slot.
template <bool F32>
__device__ void acq_range(const AcqKArgs& a, int64_t c_begin, int64_t c_end, AcqSlot* slot, Best* s_best,
                          int* s_nan) {
  const DevState* st = a.st;
  const bool ok = st->status == BO_OK && st->post_status == BO_OK;
  Best b;
  best_init(b);
  int nan_seen = 0;
  if (ok) {
    const double fb = st->f_best, lam = st->lambda;
    for (int64_t c = c_begin + threadIdx.x; c < c_end; c += blockDim.x) {
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
      if (a.vals[0] || a.vals[1] || a.vals[2]) {
        const int32_t o = a.orig[c];
        for (int k = 0; k < 3; ++k)
          if (a.vals[k] && (a.bits & (1u << k))) a.vals[k][o] = v[k];
      }
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
  acq_block_reduce(b, nan_seen, s_best, s_nan);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      slot->score[k] = b.s[k];
      slot->idx[k] = b.i[k];
    }
    slot->nan_seen = nan_seen;
  }
}

// Combines nslots slots (any order: the comparison is a total order on
// (score, index)) and writes the step result to *a.out (thread 0).
__device__ void acq_finish(const AcqKArgs& a, int nslots, Best* s_best, int* s_nan) {
  const DevState* st = a.st;
  Best r;
  best_init(r);
  int nn = 0;
  for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
    const AcqSlot sl = a.slots[s];
    for (int k = 0; k < 3; ++k) take(r, k, sl.score[k], sl.idx[k]);
    nn |= sl.nan_seen;
  }
  acq_block_reduce(r, nn, s_best, s_nan);
  if (threadIdx.x == 0) {
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

inline AcqKArgs make_acq_args(const DevPtrs& P, int64_t n_valid, const uint8_t* visited, const AcqArgs& acq,
                              bo_acq_result* out_dev) {
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
  return a;
}

}  // namespace
}  // namespace bo
