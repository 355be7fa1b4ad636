// Exhaustive posterior prediction (Section III-G) in the FP64 and FP32 modes.
//
// Each wave owns 16 compacted candidates.  For them it generates the FP64
// cross-covariance k* = amp Matern(|x_c - x_i|) against every observation,
// accumulates the mean mu = m + k*^T alpha in FP64, and parks k* (FP64, or
// rounded to FP32) in LDS in the A-operand order of a 16x16x4 matrix-core
// product.  The variance contraction W = K* L^-T runs on the matrix cores
// against the packed lower-triangular L^-1, column block by column block,
// skipping the all-zero tiles above the diagonal; FP32 products are summed in
// chunks of 16 observations and the chunks are added in FP64.  Then
// var = amp - sum_j W_cj^2, clamped at zero.  A workgroup publishes the sum and
// count of variances over its not-yet-evaluated candidates; the last
// workgroup reduces them in slot order to the mean variance and the
// exploration factor of Section III-F.
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
  typedef typename std::conditional<F32, float, double>::type KT;

  if (p.st->status != BO_OK) return;
  const int W = blockDim.x >> 6;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nt4 = p.n_pad >> 2;
  KT* kt = (KT*)s_dyn + (size_t)w * nt4 * 64;
  const int64_t row0 = ((int64_t)blockIdx.x * W + w) * 16;
  const int64_t my_row = row0 + (l & 15);
  const int my_k = l >> 4;

  // cross-covariance and mean
  double xr[kMaxD];
#pragma unroll
  for (int j = 0; j < kMaxD; ++j) xr[j] = j < p.d ? p.X64[(int64_t)j * p.N_pad + my_row] : 0.0;
  double mu_part = 0.0;
  for (int t = 0; t < nt4; ++t) {
    const int i = 4 * t + my_k;
    double kv = 0.0;
    if (i < p.n) {
      const double* xo = p.Xo64 + (size_t)i * kMaxD;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < kMaxD; ++j) {
        if (j < p.d) {
          const double df = xr[j] - xo[j];
          s += df * df;
        }
      }
      kv = p.amp * matern64(p.nu2, sqrt(s), p.inv_l);
      mu_part += kv * p.alpha[i];
    }
    kt[t * 64 + l] = (KT)kv;
  }
  mu_part += shfl_xor_d(mu_part, 16);
  mu_part += shfl_xor_d(mu_part, 32);

  // variance contraction on the matrix cores
  double sq[4] = {0.0, 0.0, 0.0, 0.0};
  const int JB = p.n_pad >> 4;
  for (int J = 0; J < JB; ++J) {
    const int tmax = 4 * J + 3;
    const size_t base = (size_t)2 * J * (J + 1);
    if constexpr (F32) {
      const float* B = (const float*)p.Bpk + base * 64 + l;
      double a64[4] = {0.0, 0.0, 0.0, 0.0};
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int t = 0; t <= tmax; ++t) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(kt[t * 64 + l], B[(size_t)t * 64], acc, 0, 0, 0);
        if ((t & 3) == 3) {
#pragma unroll
          for (int i = 0; i < 4; ++i) a64[i] += (double)acc[i];
          acc = (f32x4){0.f, 0.f, 0.f, 0.f};
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) sq[i] += a64[i] * a64[i];
    } else {
      const double* B = (const double*)p.Bpk + base * 64 + l;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int t = 0; t <= tmax; ++t)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(kt[t * 64 + l], B[(size_t)t * 64], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) sq[i] += acc[i] * acc[i];
    }
  }
  // sum over the 16 columns held by the lanes of each quarter-wave
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double v = sq[i];
    v += shfl_xor_d(v, 1);
    v += shfl_xor_d(v, 2);
    v += shfl_xor_d(v, 4);
    v += shfl_xor_d(v, 8);
    sq[i] = v;
  }

  // write mu (lanes 0..15: their own row) and var (lane 16q).  Output
  // register i of lane l holds row 4(l/16) + i for the FP32 product and row
  // l/16 + 4i for the FP64 product (the two 16x16x4 shapes order rows
  // differently).
  double part = 0.0;
  int64_t cnt = 0;
  if (l < 16 && my_row < p.n_valid) {
    if constexpr (F32) ((float*)p.mu)[my_row] = (float)(p.st->mean_y + mu_part);
    else ((double*)p.mu)[my_row] = p.st->mean_y + mu_part;
  }
  if ((l & 15) == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = F32 ? row0 + 4 * my_k + i : row0 + my_k + 4 * i;
      if (r < p.n_valid) {
        double v = p.amp - sq[i];
        v = v > 0.0 ? v : 0.0;
        if constexpr (F32) {
          const float vf = (float)v;
          ((float*)p.var)[r] = vf;
          v = (double)vf;
        } else {
          ((double*)p.var)[r] = v;
        }
        const bool vis = p.visited && p.visited[p.orig[r]];
        if (!vis) {
          part += v;
          ++cnt;
        }
      }
    }
  }
  // the four quarter-wave leaders hold rows in increasing order
  part += __shfl_down(part, 16, 64);
  part += __shfl_down(part, 32, 64);
  cnt += __shfl_down(cnt, 16, 64);
  cnt += __shfl_down(cnt, 32, 64);
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
  if (last_block(&p.st->ticket_post, &s_last)) finish_lambda(p, gridDim.x, s_rsum, s_rcnt);
}

// Posterior rows per workgroup for the FP64 / FP32 kernels.
static int post16_waves(int prec, int n_pad) {
  const int esz = prec == BO_FP64 ? 8 : 4;
  for (int W = 4; W >= 1; W >>= 1)
    if ((size_t)W * n_pad * 16 * esz <= 128 * 1024) return W;
  return 1;
}

int post16_rows_per_block(int prec, int n_pad) { return 16 * post16_waves(prec, n_pad); }

hipError_t launch_post_bf16x3(const PostArgs& a, hipStream_t st);

hipError_t launch_posterior(const DevPtrs& P, const Layout& Lo, const GpConst& g, int n, int64_t n_valid,
                            const uint8_t* visited, const AcqArgs& acq, hipStream_t st) {
  PostArgs a{};
  a.n = n;
  a.n_pad = n_pad_of(n);
  a.d = Lo.d;
  a.nu2 = g.nu2;
  a.inv_l = 1.0 / g.l;
  a.amp = g.amp;
  a.n_valid = n_valid;
  a.N_pad = Lo.N_pad;
  a.X64 = P.X64;
  a.X32 = P.X32;
  a.orig = P.orig;
  a.visited = visited;
  a.Xo64 = P.Xo64;
  a.Xo32 = P.Xo32;
  a.alpha = P.alpha;
  a.Bpk = P.Bpk;
  a.mu = P.mu;
  a.var = P.var;
  a.vslots = P.vslots;
  a.st = P.st;
  a.acq = acq;
  if (Lo.prec == BO_BF16X3) return launch_post_bf16x3(a, st);
  const int W = post16_waves(Lo.prec, a.n_pad);
  const int64_t rows = 16 * W;
  const int grid = (int)((n_valid + rows - 1) / rows);
  const size_t lds = (size_t)W * a.n_pad * 16 * (Lo.prec == BO_FP64 ? 8 : 4);
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
