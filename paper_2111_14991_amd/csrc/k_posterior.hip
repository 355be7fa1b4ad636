// Exhaustive posterior prediction (Section III-G) in the FP64 and FP32 modes,
// one session per launch: each wave runs post16_wave on 16 compacted
// candidates; a workgroup publishes the sum and count of variances over its
// not-yet-evaluated candidates; the last workgroup reduces them in slot order
// to the mean variance and the exploration factor of Section III-F.
#include "bo_internal.h"
#include "bo_device.h"
#include "post_common.h"

namespace bo {

template <bool F32>
__global__ __launch_bounds__(256) void k_post16(PostArgs p) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  __shared__ double s_wsum[4];
  __shared__ int64_t s_wcnt[4];
  __shared__ double s_rsum[256];
  __shared__ int64_t s_rcnt[256];
  __shared__ int s_last;
  if (p.st->status != BO_OK) return;
  const int W = blockDim.x >> 6;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  double* kt = (double*)s_dyn + (size_t)w * (p.n_pad >> 2) * 64;
  const int64_t row0 = ((int64_t)blockIdx.x * W + w) * 16;
  double part;
  int64_t cnt;
  post16_wave<F32, 1>(p, row0, kt, &part, &cnt);
  if (l == 0) {
    s_wsum[w] = part;
    s_wcnt[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    int64_t c = 0;
    for (int i = 0; i < W; ++i) {
      s += s_wsum[i];
      c += s_wcnt[i];
    }
    p.vslots[blockIdx.x].sum = s;
    p.vslots[blockIdx.x].count = c;
  }
  if (last_block(&p.st->ticket_post, &s_last)) finish_lambda(p, gridDim.x, s_rsum, s_rcnt, blockDim.x);
}

// FP64 posterior with register-resident accumulators, JB = reg_jb(n) <= 16,
// d <= DM: four waves of 16 candidates per workgroup, no LDS operand (the
// FP64 mode, and the FP32 mode's FP32 mean and variance from the same FP64
// products).
template <int JB, int DM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_post16r(PostArgs p) {
  __shared__ double s_wsum[4];
  __shared__ int64_t s_wcnt[4];
  __shared__ double s_rsum[256];
  __shared__ int64_t s_rcnt[256];
  __shared__ int s_last;
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
  if (last_block(&p.st->ticket_post, &s_last)) finish_lambda(p, gridDim.x, s_rsum, s_rcnt, blockDim.x);
}

template <int JB>
static void launch_post16r(const PostArgs& a, int grid, hipStream_t st) {
  if (a.d <= 8)
    hipLaunchKernelGGL((k_post16r<JB, 8>), dim3(grid), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_post16r<JB, kMaxD>), dim3(grid), dim3(256), 0, st, a);
}

int post16_rows_per_block(int prec, int n_pad) { return 16 * post16_waves(prec, n_pad); }

hipError_t launch_post_bf16x3(const PostArgs& a, hipStream_t st);

hipError_t launch_posterior(const DevPtrs& P, const Layout& Lo, const GpConst& g, int n, int64_t n_valid,
                            const uint8_t* visited, const AcqArgs& acq, hipStream_t st) {
  const PostArgs a = make_post_args(P, Lo, g, n, n_valid, visited, acq);
  if (Lo.prec == BO_BF16X3) return launch_post_bf16x3(a, st);
  if (a.n_pad <= 16 * kRegJB) {
    int grid = (int)((n_valid + 63) / 64);
    grid = grid > 0 ? grid : 1;
    switch (reg_jb(a.n)) {
#define BO_REG_CASE(J) \
  case J: launch_post16r<J>(a, grid, st); break;
      BO_REG_CASE(1) BO_REG_CASE(2) BO_REG_CASE(3) BO_REG_CASE(4) BO_REG_CASE(5) BO_REG_CASE(6)
      BO_REG_CASE(7) BO_REG_CASE(8) BO_REG_CASE(9) BO_REG_CASE(10) BO_REG_CASE(11) BO_REG_CASE(12)
      BO_REG_CASE(13) BO_REG_CASE(14) BO_REG_CASE(15) BO_REG_CASE(16)
#undef BO_REG_CASE
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const int W = post16_waves(Lo.prec, a.n_pad);
  const int64_t rows = 16 * W;
  const int grid = (int)((n_valid + rows - 1) / rows);
  const size_t lds = (size_t)W * a.n_pad * 16 * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_post16<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       128 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_post16<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (Lo.prec == BO_FP64)
    hipLaunchKernelGGL(k_post16<false>, dim3(grid), dim3(64 * W), lds, st, a);
  else
    hipLaunchKernelGGL(k_post16<true>, dim3(grid), dim3(64 * W), lds, st, a);
  return hipGetLastError();
}

}  // namespace bo
