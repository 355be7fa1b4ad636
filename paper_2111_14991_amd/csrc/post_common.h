// Shared by the posterior kernels: launch arguments, the per-wave posterior of
// the FP64 / FP32 modes, and the last-workgroup reduction of the mean variance
// and the exploration factor.
#pragma once
#include "bo_internal.h"
#include "bo_device.h"

namespace bo {

struct PostArgs {
  int n, n_pad, d, nu2;
  int out32;  // mean and variance stored in FP32 (the FP32 mode)
  int ld;  // row stride of K0
  double inv_l, amp;
  int64_t n_valid, N_pad;
  const double* X64;
  const uint16_t* Xc16;  // augmented FP16 candidate coordinates, rows of 2 * w16 (BF16X3)
  const int32_t* orig;
  const uint8_t* visited;
  const double* Xo64;
  const uint16_t* Xo16;  // augmented FP16 observation coordinates, rows of 2 * w16 (BF16X3)
  int w16;
  const double* alpha;
  const void* Bpk;
  const double* K0;
  const double* Linv;  // row stride ld
  void* mu;
  void* var;
  VarSlot* vslots;
  DevState* st;
  AcqArgs acq;
};

// Last workgroup of a posterior launch: fixed-order reduction of the slots,
// mean variance and exploration factor (Section III-F).  Every thread of the
// workgroup calls it; the first nt (a power of two, at most blockDim.x) do
// the reduction, whose order depends on nt alone, so that a workgroup of any
// size reproduces another's sum bit for bit; s_sum / s_cnt hold nt entries.
__device__ inline void finish_lambda(const PostArgs& p, int nslots, double* s_sum, int64_t* s_cnt, int nt) {
  const int t = threadIdx.x;
  const int per = (nslots + nt - 1) / nt;
  if (t < nt) {
    double sum = 0.0;
    int64_t cnt = 0;
    for (int s = t * per; s < (t + 1) * per && s < nslots; ++s) {
      sum += p.vslots[s].sum;
      cnt += p.vslots[s].count;
    }
    s_sum[t] = sum;
    s_cnt[t] = cnt;
  }
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

// ---------------------------------------------------------------------------
// Posterior of RB blocks of 16 compacted candidates by one wave, FP64 or FP32
// mode (Section III-G).
//
// The wave generates the FP64 cross-covariance k* = amp Matern(|x_c - x_i|)
// against every observation, accumulates the mean mu = m + k*^T alpha in FP64
// and parks the FP64 operand of the variance contraction in LDS (kt: RB
// regions of n_pad * 16 doubles) in the A-operand order of a 16x16x4
// matrix-core product: entry (row r, observation i) of block b at
// kt[b][(i/4) * 64 + 16 (i%4) + r].  The contraction W = (operand) L^-T runs
// on the matrix cores against the packed lower-triangular L^-1, column block
// by column block, skipping the all-zero tiles above the diagonal; each B
// fragment is loaded once for the RB row blocks.
//
// FP64 mode: the operand is k* and var = amp - |W|^2.
//
// FP32 mode (compensated, with an FP64 fallback): rounding k* and L^-1 to
// FP32 leaves errors proportional to |k*| |L^-1|, large next to the variance
// near the data.  The operand is instead the residual of k* after projecting
// out the nearest observation p: with K = K_nn + delta I,
// c = k*_p / K_pp and r = k* - c K e_p (so r_p = 0), L^-1 K e_p = L^T e_p
// gives exactly
//     k*^T K^-1 k* = k*_p^2 / K_pp + |L^-1 r|^2,
//     var = amp - k*_p^2 / K_pp - |L^-1 r|^2,
// whose first part is exact in FP64; only |L^-1 r|^2 goes through FP32
// products (summed over 16 observations, chunks added in FP64), and |r|
// shrinks with the distance to the data.  Where var is still small next to
// |L^-1 r|^2 (more than a quarter of it: cancellation would amplify the FP32
// rounding past what the acquisitions tolerate), the wave recomputes
// |L^-1 r|^2 for that block of 16 rows with FP64 products against L^-1 itself.
//
// Writes mu and var (FP64 or FP32) of the rows below n_valid and returns, on
// lane 0, the sum and count of the variances of the rows not yet evaluated.
// Cross-covariance of the FP32-mode posterior (Section III-B), the same
// arithmetic in every kernel that computes it, so that the single-session,
// batched and served paths agree to the last bit: the squared distance as two
// interleaved partial sums over the coordinates (zero past the d-th, which
// adds nothing), then amp (1 + rho (1 + c2 rho)) exp(-rho), rho = c1 sqrt(s).
struct KStar {
  double amp, c1, c2;
  __device__ KStar(const PostArgs& p) {
    const bool nu5 = p.nu2 == 5;
    amp = p.amp;
    c1 = (nu5 ? 2.23606797749978969641 : 1.73205080756887729353) * p.inv_l;
    c2 = nu5 ? 1.0 / 3.0 : 0.0;
  }
  __device__ double operator()(double s) const {
    const double rho = c1 * sqrt(s);
    return amp * (fma(rho, fma(c2, rho, 1.0), 1.0) * exp(-rho));
  }
};
template <int DM>
__device__ __forceinline__ double dist2_pairs(const double* xr, const double* xo) {
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int j = 0; j < DM; j += 2) {
    const double e0 = xr[j] - xo[j];
    s0 = fma(e0, e0, s0);
    if (j + 1 < DM) {
      const double e1 = xr[j + 1] - xo[j + 1];
      s1 = fma(e1, e1, s1);
    }
  }
  return s0 + s1;
}

// Element (i, j) of L^-1 as a B operand, zero outside the lower triangle of
// the current fit.
__device__ __forceinline__ double linv_b(const PostArgs& p, int row, int col) {
  return (col <= row && row < p.n) ? p.Linv[(size_t)row * p.ld + col] : 0.0;
}

template <bool F32, int RB>
__device__ void post16_wave(const PostArgs& p, int64_t row0, double* kt, double* part_out, int64_t* cnt_out) {
  const int l = threadIdx.x & 63;
  const int nt4 = p.n_pad >> 2;
  const int my_k = l >> 4;
  double base[RB];  // FP32 mode: amp - k*_p^2 / K_pp of the lane's row
  double mu_part[RB];

#pragma unroll
  for (int b = 0; b < RB; ++b) {
    double* ktb = kt + (size_t)b * nt4 * 64;
    const int64_t my_row = row0 + 16 * b + (l & 15);
    double xr[kMaxD];
#pragma unroll
    for (int j = 0; j < kMaxD; ++j) xr[j] = j < p.d ? p.X64[(int64_t)j * p.N_pad + my_row] : 0.0;
    double mp = 0.0, bs = 0.0;
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
          mp += kv * p.alpha[i];
        }
        ktb[t * 64 + l] = kv;
      }
    } else {
      // nearest observation of the row: the four lanes of a row scan disjoint
      // observations, then compare (distance, index) pairs.  The coordinates
      // past the d-th are zero on both sides.
      const KStar kstar(p);
      double xo[kMaxD];
      double best = __builtin_inf();
      int bi = 0;
      for (int t = 0; t < nt4; ++t) {
        const int i = 4 * t + my_k;
        if (i < p.n) {
#pragma unroll
          for (int j = 0; j < kMaxD; ++j) xo[j] = j < p.d ? p.Xo64[(size_t)i * kMaxD + j] : 0.0;
          const double s = dist2_pairs<kMaxD>(xr, xo);
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
      // k*_p from the same distance the scan found, on every lane of the row
      const double kp = kstar(best);
      const double kpp = p.amp + p.st->jitter;
      const double c = kp / kpp;
      bs = p.amp - kp * c;
      const double* krow = p.K0 + (size_t)bi * p.ld;
      for (int t = 0; t < nt4; ++t) {
        const int i = 4 * t + my_k;
        double rv = 0.0;
        if (i < p.n) {
#pragma unroll
          for (int j = 0; j < kMaxD; ++j) xo[j] = j < p.d ? p.Xo64[(size_t)i * kMaxD + j] : 0.0;
          const double kv = kstar(dist2_pairs<kMaxD>(xr, xo));
          mp = fma(kv, p.alpha[i], mp);
          rv = i == bi ? 0.0 : kv - c * krow[i];
        }
        ktb[t * 64 + l] = rv;
      }
    }
    mp += shfl_xor_d(mp, 16);
    mp += shfl_xor_d(mp, 32);
    mu_part[b] = mp;
    base[b] = bs;
  }

  // variance contraction on the matrix cores
  double sq[RB][4];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int i = 0; i < 4; ++i) sq[b][i] = 0.0;
  const int JB = p.n_pad >> 4;
  for (int J = 0; J < JB; ++J) {
    const int tmax = 4 * J + 3;
    const size_t fbase = (size_t)2 * J * (J + 1);
    if constexpr (F32) {
      const float* B = (const float*)p.Bpk + fbase * 64 + l;
      double a64[RB][4];
      f32x4 acc[RB];
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        acc[b] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i) a64[b][i] = 0.0;
      }
      // groups of four k-steps (tmax + 1 is a multiple of 4), the B fragments
      // of the next group loaded while this one runs
      float bq[4], bn[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) bq[u] = B[(size_t)u * 64];
      for (int t0 = 0; t0 <= tmax; t0 += 4) {
        const bool more = t0 + 4 <= tmax;
#pragma unroll
        for (int u = 0; u < 4; ++u) bn[u] = B[(size_t)(more ? t0 + 4 + u : u) * 64];  // in bounds either way
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int b = 0; b < RB; ++b)
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)kt[((size_t)b * nt4 + t0 + u) * 64 + l], bq[u],
                                                          acc[b], 0, 0, 0);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
#pragma unroll
          for (int i = 0; i < 4; ++i) a64[b][i] += (double)acc[b][i];
          acc[b] = (f32x4){0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) bq[u] = bn[u];
      }
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) sq[b][i] += a64[b][i] * a64[b][i];
    } else {
      const double* B = (const double*)p.Bpk + fbase * 64 + l;
      f64x4 acc[RB];
#pragma unroll
      for (int b = 0; b < RB; ++b) acc[b] = (f64x4){0.0, 0.0, 0.0, 0.0};
      double bq[4], bn[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) bq[u] = B[(size_t)u * 64];
      for (int t0 = 0; t0 <= tmax; t0 += 4) {
        const bool more = t0 + 4 <= tmax;
#pragma unroll
        for (int u = 0; u < 4; ++u) bn[u] = B[(size_t)(more ? t0 + 4 + u : u) * 64];  // in bounds either way
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int b = 0; b < RB; ++b)
            acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kt[((size_t)b * nt4 + t0 + u) * 64 + l], bq[u], acc[b],
                                                          0, 0, 0);
#pragma unroll
        for (int u = 0; u < 4; ++u) bq[u] = bn[u];
      }
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) sq[b][i] += acc[b][i] * acc[b][i];
    }
  }

  double part = 0.0;
  int64_t cnt = 0;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int64_t brow0 = row0 + 16 * b;
    // sum over the 16 columns held by the lanes of each quarter-wave
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double v = sq[b][i];
      v += shfl_xor_d(v, 1);
      v += shfl_xor_d(v, 2);
      v += shfl_xor_d(v, 4);
      v += shfl_xor_d(v, 8);
      sq[b][i] = v;
    }
    // FP32 mode: the row constant of output row 4 (l/16) + i sits on lane 4 (l/16) + i
    double base_o[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) base_o[i] = F32 ? __shfl(base[b], 4 * my_k + i, 64) : 0.0;
    if constexpr (F32) {
      // rows whose variance is dominated by cancellation: FP64 products
      bool flag = false;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = brow0 + 4 * my_k + i;
        flag |= r < p.n_valid && sq[b][i] > 4.0 * (base_o[i] - sq[b][i]);
      }
      if (__any(flag)) {
        double* ktb = kt + (size_t)b * nt4 * 64;
        double s64[4] = {0.0, 0.0, 0.0, 0.0};
        for (int J = 0; J < JB; ++J) {
          f64x4 acc = {0.0, 0.0, 0.0, 0.0};
          for (int t = 0; t <= 4 * J + 3; ++t) {
            const double bv = linv_b(p, 16 * J + (l & 15), 4 * t + my_k);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ktb[t * 64 + l], bv, acc, 0, 0, 0);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) s64[i] += acc[i] * acc[i];
        }
        // the FP64 product orders rows as l/16 + 4i; move them to the FP32 order 4(l/16) + i
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          double v = s64[i];
          v += shfl_xor_d(v, 1);
          v += shfl_xor_d(v, 2);
          v += shfl_xor_d(v, 4);
          v += shfl_xor_d(v, 8);
          s64[i] = v;
        }
        // row q = 4a + i (FP32 order) is FP64 row a' + 4i' with a' = q % 4, i' = q / 4,
        // held in register i' by the lanes with l / 16 = a'
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int q = 4 * my_k + i;
          const int src = 16 * (q & 3);
          double v = 0.0;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const double t = __shfl(s64[k], src, 64);
            v = (q >> 2) == k ? t : v;
          }
          sq[b][i] = v;
        }
      }
    }
    const int64_t my_row = brow0 + (l & 15);
    if (l < 16 && my_row < p.n_valid) {
      if constexpr (F32) ((float*)p.mu)[my_row] = (float)(p.st->mean_y + mu_part[b]);
      else ((double*)p.mu)[my_row] = p.st->mean_y + mu_part[b];
    }
    // output register i of lane l holds row 4(l/16) + i for the FP32 product
    // and row l/16 + 4i for the FP64 product
    if ((l & 15) == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = F32 ? brow0 + 4 * my_k + i : brow0 + my_k + 4 * i;
        if (r < p.n_valid) {
          double v = (F32 ? base_o[i] : p.amp) - sq[b][i];
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
  }
  // the four quarter-wave leaders hold rows in increasing order
  part += __shfl_down(part, 16, 64);
  part += __shfl_down(part, 32, 64);
  cnt += __shfl_down(cnt, 16, 64);
  cnt += __shfl_down(cnt, 32, 64);
  *part_out = part;
  *cnt_out = cnt;
}

constexpr int kRegJB = kRegMax / 16;  // n_pad <= kRegMax takes the register-resident posterior
constexpr int kObsPitch = kMaxD + 1;  // LDS row pitch of the staged observations

// Observations of the register-resident posterior: n rounded up to 16
// (16 jb, jb = 1 .. kRegJB column blocks; the blocks and k-steps of the
// 64-padded layout beyond them hold zeros only and are skipped).
__host__ __device__ inline int reg_jb(int n) { return (n + 15) >> 4; }

// Stages the observation coordinates (`rows` = 16 jb rows, pitch kObsPitch,
// zero past the d-th) and alpha (zero past n) of a fit into LDS for
// post16_wave_reg; every thread of the workgroup calls it.  The odd pitch
// puts the four observations a wave reads at once in different banks.
__device__ inline void stage_obs(const PostArgs& p, int rows, double* xs, double* as) {
  for (int e = threadIdx.x; e < rows * kObsPitch; e += blockDim.x) {
    const int i = e / kObsPitch, j = e - i * kObsPitch;
    const double v = p.Xo64[i * kMaxD + (j < kMaxD ? j : kMaxD - 1)];
    xs[e] = j < p.d ? v : 0.0;
  }
  for (int i = threadIdx.x; i < rows; i += blockDim.x) {
    const double v = p.alpha[i];
    as[i] = i < p.n ? v : 0.0;
  }
  __syncthreads();
}

// FP64 posterior of 16 candidates by one wave for JB = reg_jb(n), with the
// contraction in k-outer order: lane l generates its A element
// k*(row l%16, observation 4t + l/16) once per k-step t and feeds it to every
// column block J >= t/4 (the others are zero above the diagonal), whose
// accumulators stay in registers.  The observations (xs, as) come from LDS
// as stage_obs leaves them; the candidate's first DM coordinates (DM >= d)
// from HBM.  The shape is a template parameter, so every step is
// straight-line code: the B loads of its live blocks, the kernel value, their
// MFMAs.  Same outputs and slot partial as post16_wave<false>.  The FP32
// mode (p.out32) stores the mean and variance in FP32; its products stay FP64:
// an FP32 contraction cannot hold the variance to 1e-6 of itself where it is
// small next to the prior, which is most of a well-sampled space.
template <int JB, int DM>
__device__ void post16_wave_reg(const PostArgs& p, int64_t row0, const double* xs, const double* as,
                                double* part_out, int64_t* cnt_out) {
  static_assert(JB >= 1 && JB <= kRegJB && DM <= kMaxD, "shape");
  const int l = threadIdx.x & 63;
  const int my_k = l >> 4;
  // every field below is the same across the wave; in the batched kernel the
  // session is chosen at run time, so say so to keep them in scalar registers
  row0 = uni(row0);
  const int n = uni(p.n), d = uni(p.d);
  const bool nu5 = uni(p.nu2) == 5;
  const double amp = uni(p.amp);
  // Matern (Section III-B) as (1 + rho (1 + c2 rho)) exp(-rho), rho = c1 r
  const double c1 = (nu5 ? 2.23606797749978969641 : 1.73205080756887729353) * uni(p.inv_l);
  const double c2 = nu5 ? 1.0 / 3.0 : 0.0;
  const int64_t n_valid = uni(p.n_valid), N_pad = uni(p.N_pad);
  const auto X64 = gptr(uni(p.X64));
  const auto orig = gptr(uni(p.orig));
  const auto visited = gptr(uni(p.visited));
  const bool out32 = uni(p.out32) != 0;
  double* const mu = (double*)uni(p.mu);
  double* const var = (double*)uni(p.var);
  const double mean_y = uni(p.st)->mean_y;
  const int64_t my_row = row0 + (l & 15);
  double xr[DM];
#pragma unroll
  for (int j = 0; j < DM; ++j) {
    const double v = X64[(int64_t)(j < d ? j : d - 1) * N_pad + my_row];
    xr[j] = j < d ? v : 0.0;
  }
  // packed B of 16 JB column blocks: 2 JB (JB + 1) tiles of 64 lanes
  const __amdgpu_buffer_rsrc_t rB = buffer_of(uni(p.Bpk), 2 * JB * (JB + 1) * 64 * (int)sizeof(double));
  f64x4 acc[JB];
#pragma unroll
  for (int J = 0; J < JB; ++J) acc[J] = (f64x4){0.0, 0.0, 0.0, 0.0};
  double mp = 0.0;
  // phase J0 covers k-steps 4 J0 .. 4 J0 + 3, whose B values are nonzero in
  // blocks J0 .. JB - 1 only; the phases are unrolled, so each one's loads
  // and MFMAs are a fixed sequence
#pragma unroll
  for (int J0 = 0; J0 < JB; ++J0) {
#pragma unroll 1
    for (int tt = 0; tt < 4; ++tt) {
      const int t = 4 * J0 + tt;
      double bq[JB];
#pragma unroll
      for (int J = J0; J < JB; ++J) bq[J] = buffer_load_f64(rB, l * 8, (2 * J * (J + 1) + t) * 64 * 8);
      const int i = 4 * t + my_k;
      const double* xo = xs + i * kObsPitch;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int j = 0; j < DM; j += 2) {
        const double e0 = xr[j] - xo[j];
        s0 = fma(e0, e0, s0);
        if (j + 1 < DM) {
          const double e1 = xr[j + 1] - xo[j + 1];
          s1 = fma(e1, e1, s1);
        }
      }
      const double rho = c1 * sqrt(s0 + s1);
      double kv = amp * (fma(rho, fma(c2, rho, 1.0), 1.0) * exp(-rho));
      kv = i < n ? kv : 0.0;
      mp = fma(kv, as[i], mp);
#pragma unroll
      for (int J = J0; J < JB; ++J) acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv, bq[J], acc[J], 0, 0, 0);
    }
  }
  mp += shfl_xor_d(mp, 16);
  mp += shfl_xor_d(mp, 32);
  // output register i of lane l: row l/16 + 4i, column l%16 of block J
  double sq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int J = 0; J < JB; ++J)
#pragma unroll
    for (int i = 0; i < 4; ++i) sq[i] += acc[J][i] * acc[J][i];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double v = sq[i];
    v += shfl_xor_d(v, 1);
    v += shfl_xor_d(v, 2);
    v += shfl_xor_d(v, 4);
    v += shfl_xor_d(v, 8);
    sq[i] = v;
  }
  double part = 0.0;
  int64_t cnt = 0;
  if (l < 16 && my_row < n_valid) {
    const double m = mean_y + mp;
    if (out32) ((float*)mu)[my_row] = (float)m;
    else mu[my_row] = m;
  }
  if ((l & 15) == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = row0 + my_k + 4 * i;
      if (r < n_valid) {
        double v = amp - sq[i];
        v = v > 0.0 ? v : 0.0;
        if (out32) ((float*)var)[r] = (float)v;
        else var[r] = v;
        if (!(visited && visited[orig[r]])) {
          part += v;
          ++cnt;
        }
      }
    }
  }
  part += __shfl_down(part, 16, 64);
  part += __shfl_down(part, 32, 64);
  cnt += __shfl_down(cnt, 16, 64);
  cnt += __shfl_down(cnt, 32, 64);
  *part_out = part;
  *cnt_out = cnt;
}

// Rows per workgroup and row blocks per wave of the single-session FP64 / FP32
// posterior: up to 4 waves of 16 rows within 128 KB of LDS.
inline int post16_waves(int prec, int n_pad) {
  (void)prec;  // both modes park FP64 operands
  for (int W = 4; W >= 1; W >>= 1)
    if ((size_t)W * n_pad * 16 * sizeof(double) <= 128 * 1024) return W;
  return 1;
}

// Launch arguments of a session's posterior.
inline PostArgs make_post_args(const DevPtrs& P, const Layout& Lo, const GpConst& g, int n, int64_t n_valid,
                               const uint8_t* visited, const AcqArgs& acq) {
  PostArgs a{};
  a.n = n;
  a.n_pad = n_pad_of(n);
  a.out32 = Lo.prec == BO_FP64 ? 0 : 1;
  a.ld = Lo.n_max_pad;
  a.d = Lo.d;
  a.nu2 = g.nu2;
  a.inv_l = 1.0 / g.l;
  a.amp = g.amp;
  a.n_valid = n_valid;
  a.N_pad = Lo.N_pad;
  a.X64 = P.X64;
  a.Xc16 = P.Xc16;
  a.orig = P.orig;
  a.visited = visited;
  a.Xo64 = P.Xo64;
  a.Xo16 = P.Xo16;
  a.w16 = Lo.w16;
  a.alpha = P.alpha;
  a.Bpk = P.Bpk;
  a.K0 = P.K0;
  a.Linv = P.Linv;
  a.mu = P.mu;
  a.var = P.var;
  a.vslots = P.vslots;
  a.st = P.st;
  a.acq = acq;
  return a;
}

}  // namespace bo
