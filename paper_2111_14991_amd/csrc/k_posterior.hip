// Exhaustive posterior prediction (Section III-G) in the FP64 and FP32 modes.
//
// Each wave owns 16 compacted candidates.  For them it generates the FP64
// cross-covariance k* = amp Matern(|x_c - x_i|) against every observation,
// accumulates the mean mu = m + k*^T alpha in FP64, and parks the operand of
// the variance contraction in LDS in the A-operand order of a 16x16x4
// matrix-core product.  The contraction W = (operand) L^-T runs on the matrix
// cores against the packed lower-triangular L^-1, column block by column
// block, skipping the all-zero tiles above the diagonal.
//
// FP64 mode: the operand is k* and var = amp - |W|^2.
//
// FP32 mode (compensated): products are summed on FP32 matrix cores in chunks
// of 16 observations and the chunks are added in FP64.  Rounding k* and L^-1
// to FP32 would leave errors proportional to |k*| |L^-1|, which is large next
// to the variance near the data.  Instead the operand is the residual
// r = k* - K e_p against the nearest observation p (K = K_nn with the accepted
// jitter delta).  Because L^-1 K e_p = L^T e_p exactly,
//     k*^T K^-1 k* = K_pp + 2 r_p + |L^-1 r|^2,
// hence var = 2 (amp - k*_p) + delta - |L^-1 r|^2, whose first two terms are
// exact in FP64 and whose rounded part shrinks with the distance to the data
// (the identity holds for any p; the nearest one minimizes |r|).
//
// A workgroup publishes the sum and count of variances over its
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
  double base = 0.0;  // FP32 mode: 2 (amp - k*_p) + delta, on every lane of the row
  if constexpr (!F32) {
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
  } else {
    // nearest observation of the row: the four lanes of a row scan disjoint
    // observations, then compare (distance, index) pairs
    double best = __builtin_inf();
    int bi = 0;
    for (int t = 0; t < nt4; ++t) {
      const int i = 4 * t + my_k;
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
        if (s < best) {
          best = s;
          bi = i;
        }
      }
    }
#pragma unroll
    for (int m = 16; m <= 32; m <<= 1) {
      const double ob = shfl_xor_d(best, m);
      const int oi = __shfl_xor(bi, m, 64);
      if (ob < best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const double jit = p.st->jitter;
    const double* krow = p.K0 + (size_t)bi * p.n_pad;
    for (int t = 0; t < nt4; ++t) {
      const int i = 4 * t + my_k;
      double rv = 0.0;
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
        const double kv = p.amp * matern64(p.nu2, sqrt(s), p.inv_l);
        mu_part += kv * p.alpha[i];
        rv = kv - krow[i];
        if (i == bi) {
          rv -= jit;
          base = 2.0 * (p.amp - kv) + jit;
        }
      }
      kt[t * 64 + l] = (KT)rv;
    }
    base += shfl_xor_d(base, 16);
    base += shfl_xor_d(base, 32);
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
  // FP32 mode: the row constant of output row 4 (l/16) + i sits on lane 4 (l/16) + i
  double base_o[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) base_o[i] = F32 ? __shfl(base, 4 * my_k + i, 64) : 0.0;
  if ((l & 15) == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = F32 ? row0 + 4 * my_k + i : row0 + my_k + 4 * i;
      if (r < p.n_valid) {
        double v = (F32 ? base_o[i] : p.amp) - sq[i];
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
  a.K0 = P.K0;
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
