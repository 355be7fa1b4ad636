// Exhaustive posterior prediction (Section III-G) in the FP64 and FP32 modes,
// one session per launch: each wave computes 16 compacted candidates with
// register-resident FP64 accumulators (post16_wave_reg up to 256
// observations, post16_wave_big in column passes above); a workgroup of four
// waves publishes the sum and count of variances over its not-yet-evaluated
// candidates in its slot; a one-workgroup launch after it reduces the slots in
// order to the mean variance and the exploration factor of Section III-F.
#include "bo_internal.h"
#include "bo_device.h"
#include "post_common.h"

namespace bo {

// FP64 posterior with register-resident accumulators, JB = reg_jb(n) <= 16,
// d <= DM: four waves of 16 candidates per workgroup, no LDS operand (the
// FP64 mode, and the FP32 mode's FP32 mean and variance from the same FP64
// products).
template <int JB, int DM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_post16r(PostArgs p) {
  __shared__ double s_wsum[4];
  __shared__ int64_t s_wcnt[4];
  __shared__ double s_xo[16 * JB * kObsPitch];
  __shared__ double s_alpha[16 * JB];
  if (p.st->status != BO_OK) return;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + w) * 16;
  stage_obs(p, 16 * JB, s_xo, s_alpha);
  double part;
  int64_t cnt;
  post16_wave_reg<JB, DM>(p, row0, s_xo, s_alpha, &part, &cnt);
  if (l == 0) {
    s_wsum[w] = part;
    s_wcnt[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    int64_t c = 0;
    for (int i = 0; i < 4; ++i) {
      s += s_wsum[i];
      c += s_wcnt[i];
    }
    p.vslots[blockIdx.x].sum = s;
    p.vslots[blockIdx.x].count = c;
  }
}

// Mean variance and exploration factor from the slots (one workgroup, after
// the posterior launch: a last-workgroup ticket in the posterior would need a
// device-scope fence in every one of its workgroups).
__global__ __launch_bounds__(256) void k_post_lambda(PostArgs p, int nslots) {
  __shared__ double s_rsum[256];
  __shared__ int64_t s_rcnt[256];
  if (p.st->status != BO_OK) return;
  finish_lambda(p, nslots, s_rsum, s_rcnt, 256);
}

template <int JB>
static void launch_post16r(const PostArgs& a, int grid, hipStream_t st) {
  if (a.d <= 8)
    hipLaunchKernelGGL((k_post16r<JB, 8>), dim3(grid), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_post16r<JB, kMaxD>), dim3(grid), dim3(256), 0, st, a);
}

// Above kRegMax observations: post16_wave_big, eight waves of 16 candidates
// (two slots of 64) per workgroup, one workgroup per compute unit, with every
// observation staged in LDS (dynamic: 16 reg_jb(n) rows).
constexpr int kBigThreads = 512;

inline size_t big_lds_bytes(int n) { return (size_t)16 * reg_jb(n) * (kObsPitch + 1) * sizeof(double); }

template <int DM>
__global__ __launch_bounds__(kBigThreads) void k_post16big(PostArgs p) {
  extern __shared__ __align__(16) double s_obs[];
  __shared__ double s_wsum[8];
  __shared__ int64_t s_wcnt[8];
  if (p.st->status != BO_OK) return;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int rows = 16 * reg_jb(p.n);
  double* xs = s_obs;
  double* as = s_obs + (size_t)rows * kObsPitch;
  stage_obs(p, rows, xs, as);
  const int64_t row0 = ((int64_t)blockIdx.x * 8 + w) * 16;
  double part;
  int64_t cnt;
  post16_wave_big<DM>(p, row0, xs, as, &part, &cnt);
  if (l == 0) {
    s_wsum[w] = part;
    s_wcnt[w] = cnt;
  }
  __syncthreads();
  // slot 2b from waves 0-3, slot 2b + 1 from waves 4-7
  const int64_t nslots = (p.n_valid + 63) / 64;
  if (threadIdx.x < 2) {
    const int h = threadIdx.x;
    double s = 0.0;
    int64_t c = 0;
    for (int i = 0; i < 4; ++i) {
      s += s_wsum[4 * h + i];
      c += s_wcnt[4 * h + i];
    }
    const int64_t slot = 2 * (int64_t)blockIdx.x + h;
    if (slot < nslots) {
      p.vslots[slot].sum = s;
      p.vslots[slot].count = c;
    }
  }
}

hipError_t launch_post_bf16x3(const PostArgs& a, hipStream_t st);

hipError_t launch_posterior(const DevPtrs& P, const Layout& Lo, const GpConst& g, int n, int64_t n_valid,
                            const uint8_t* visited, const AcqArgs& acq, hipStream_t st) {
  const PostArgs a = make_post_args(P, Lo, g, n, n_valid, visited, acq);
  if (Lo.prec == BO_BF16X3) return launch_post_bf16x3(a, st);
  int grid = (int)((n_valid + 63) / 64);
  grid = grid > 0 ? grid : 1;
  if (a.n_pad > kRegMax) {
    static bool attr_set = false;
    const size_t max_lds = big_lds_bytes(kMaxN);
    if (!attr_set) {
      hipError_t e = hipFuncSetAttribute((const void*)k_post16big<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)max_lds);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_post16big<kMaxD>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)max_lds);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    const int gbig = (grid + 1) / 2;
    const size_t lds = big_lds_bytes(a.n);
    if (a.d <= 8)
      hipLaunchKernelGGL(k_post16big<8>, dim3(gbig), dim3(kBigThreads), lds, st, a);
    else
      hipLaunchKernelGGL(k_post16big<kMaxD>, dim3(gbig), dim3(kBigThreads), lds, st, a);
  } else {
    switch (reg_jb(a.n)) {
#define BO_REG_CASE(J) \
  case J: launch_post16r<J>(a, grid, st); break;
      BO_REG_CASE(1) BO_REG_CASE(2) BO_REG_CASE(3) BO_REG_CASE(4) BO_REG_CASE(5) BO_REG_CASE(6)
      BO_REG_CASE(7) BO_REG_CASE(8) BO_REG_CASE(9) BO_REG_CASE(10) BO_REG_CASE(11) BO_REG_CASE(12)
      BO_REG_CASE(13) BO_REG_CASE(14) BO_REG_CASE(15) BO_REG_CASE(16)
#undef BO_REG_CASE
      default: return hipErrorInvalidValue;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_post_lambda, dim3(1), dim3(256), 0, st, a, grid);
  return hipGetLastError();
}

}  // namespace bo
