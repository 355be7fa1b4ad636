// Shared by the posterior kernels: launch arguments and the last-workgroup
// reduction of the mean variance and the exploration factor.
#pragma once
#include "bo_internal.h"
#include "bo_device.h"

namespace bo {

struct PostArgs {
  int n, n_pad, d, nu2;
  double inv_l, amp;
  int64_t n_valid, N_pad;
  const double* X64;
  const float* X32;
  const int32_t* orig;
  const uint8_t* visited;
  const double* Xo64;
  const float* Xo32;
  const double* alpha;
  const void* Bpk;
  const double* K0;
  void* mu;
  void* var;
  VarSlot* vslots;
  DevState* st;
  AcqArgs acq;
};

// Last workgroup of a posterior launch: fixed-order reduction of the slots,
// mean variance and exploration factor (Section III-F).
__device__ inline void finish_lambda(const PostArgs& p, int nslots, double* s_sum, int64_t* s_cnt) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (nslots + nt - 1) / nt;
  double sum = 0.0;
  int64_t cnt = 0;
  for (int s = t * per; s < (t + 1) * per && s < nslots; ++s) {
    sum += p.vslots[s].sum;
    cnt += p.vslots[s].count;
  }
  s_sum[t] = sum;
  s_cnt[t] = cnt;
  __syncthreads();
  for (int off = nt / 2; off > 0; off >>= 1) {
    if (t < off) {
      s_sum[t] += s_sum[t + off];
      s_cnt[t] += s_cnt[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    DevState* st = p.st;
    const int64_t nu = s_cnt[0];
    st->n_unmasked = nu;
    st->post_status = BO_OK;
    if (nu == 0) {
      st->var_mean = __longlong_as_double(0x7ff8000000000000LL);
      st->lambda = st->var_mean;
      st->post_status = BO_E_NO_CANDIDATE;
    } else {
      const double vm = s_sum[0] / (double)nu;
      st->var_mean = vm;
      if (p.acq.mode == 0) {
        st->lambda = p.acq.lambda_const;
      } else {
        const double fb = st->f_best;
        if (!(fb > 0.0) || !(p.acq.mu_s > 0.0)) {
          st->post_status = BO_E_INVALID_ARG;
          st->lambda = __longlong_as_double(0x7ff8000000000000LL);
        } else {
          const double vs = p.acq.var_s_mean > 0.0 ? p.acq.var_s_mean : vm;
          st->lambda = (vm / (p.acq.mu_s / fb)) / vs;
        }
      }
    }
    st->ticket_post = 0;
  }
}

}  // namespace bo
