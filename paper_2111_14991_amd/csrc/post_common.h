// Shared by the posterior kernels: launch arguments, the per-wave posterior of
// the FP64 / FP32 modes, and the reduction of the slots to the mean variance
// and the exploration factor.
#pragma once
#include "bo_internal.h"
#include "bo_device.h"

namespace bo {

struct PostArgs {
  int n, n_pad, d, nu2;
  int out32;  // mean and variance stored in FP32 (the FP32 mode)
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
// Register-resident posterior of the FP64 and FP32 modes (Section III-G).

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

// End of a wave's 16 rows in the register-resident posteriors: the mean
// partial mp (lane l: row l%16, over the observations 4t + l/16) and the
// squared norms sq (lane l, register i: row l/16 + 4i, over the columns
// l%16 of the blocks) are reduced over the lanes; the mean and the variance
// (clamped at zero) are stored, FP32 in the FP32 mode; lane 0 returns the
// sum and count of the variances of the rows not yet evaluated.
__device__ __forceinline__ void post16_store(const PostArgs& p, int64_t row0, double mp, double* sq,
                                             double* part_out, int64_t* cnt_out) {
  const int l = threadIdx.x & 63;
  const int my_k = l >> 4;
  row0 = uni(row0);
  const double amp = uni(p.amp);
  const int64_t n_valid = uni(p.n_valid);
  const auto orig = gptr(uni(p.orig));
  const auto visited = gptr(uni(p.visited));
  const bool out32 = uni(p.out32) != 0;
  double* const mu = (double*)uni(p.mu);
  double* const var = (double*)uni(p.var);
  const double mean_y = uni(p.st)->mean_y;
  const int64_t my_row = row0 + (l & 15);
  mp += shfl_xor_d(mp, 16);
  mp += shfl_xor_d(mp, 32);
#pragma unroll
  for (int i = 0; i < 4; ++i) sq[i] = row_sum16_d(sq[i]);
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
  const int64_t N_pad = uni(p.N_pad);
  const auto X64 = gptr(uni(p.X64));
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
  // output register i of lane l: row l/16 + 4i, column l%16 of block J
  double sq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int J = 0; J < JB; ++J)
#pragma unroll
    for (int i = 0; i < 4; ++i) sq[i] += acc[J][i] * acc[J][i];
  post16_store(p, row0, mp, sq, part_out, cnt_out);
}

// FP64 posterior of 16 candidates by one wave above kRegMax observations
// (JB = reg_jb(n) up to 64 column blocks), the register-resident scheme of
// post16_wave_reg with the column blocks in passes: the first pass takes the
// JB - PW (P - 1) lowest blocks, each later one the next PW, and a pass runs
// every k-step up to its last block's diagonal, so that the accumulators of
// at most PW blocks are live.  The cross-covariances are generated again in
// every pass (the observations and alpha staged in LDS by stage_obs); the
// mean is taken in the last pass, which runs every k-step.  Same outputs and
// slot partial as post16_wave_reg.
template <int DM>
struct BigWave {
  const double* xs;
  const double* as;
  __amdgpu_buffer_rsrc_t rB;
  int l, my_k, n;
  double amp, c1, c2;
  double xr[DM];
  double mp;
  double sq[4];

  __device__ __forceinline__ double kval(int t, bool mean) {
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
    if (mean) mp = fma(kv, as[i], mp);
    return kv;
  }

  __device__ __forceinline__ double bval(int J, int t) const {
    return buffer_load_f64(rB, l * 8, (2 * J * (J + 1) + t) * 64 * 8);
  }

  // blocks jbase .. jbase + NB - 1 over k-steps 0 .. 4 (jbase + NB) - 1
  template <int NB>
  __device__ void pass(int jbase, bool mean) {
    f64x4 acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = (f64x4){0.0, 0.0, 0.0, 0.0};
    // k-steps below the pass's first diagonal: every block of the pass is live
#pragma unroll 1
    for (int t = 0; t < 4 * jbase; ++t) {
      double bq[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) bq[q] = bval(jbase + q, t);
      const double kv = kval(t, mean);
#pragma unroll
      for (int q = 0; q < NB; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv, bq[q], acc[q], 0, 0, 0);
    }
    // the pass's own triangle: k-steps 4 (jbase + q0) .. + 3 feed blocks q >= q0
#pragma unroll
    for (int q0 = 0; q0 < NB; ++q0) {
#pragma unroll 1
      for (int tt = 0; tt < 4; ++tt) {
        const int t = 4 * (jbase + q0) + tt;
        double bq[NB];
#pragma unroll
        for (int q = q0; q < NB; ++q) bq[q] = bval(jbase + q, t);
        const double kv = kval(t, mean);
#pragma unroll
        for (int q = q0; q < NB; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv, bq[q], acc[q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) sq[i] += acc[q][i] * acc[q][i];
  }
};

// PW: blocks per full pass.  With 16, the accumulators and the coordinates
// leave a few registers to reload once per phase, which still beats 14-block
// passes (fewer regenerated k-steps).
template <int DM, int PW = 16>
__device__ void post16_wave_big(const PostArgs& p, int64_t row0, const double* xs, const double* as,
                                double* part_out, int64_t* cnt_out) {
  static_assert(DM <= kMaxD && PW >= 1 && PW <= 16, "shape");
  BigWave<DM> W;
  W.l = threadIdx.x & 63;
  W.my_k = W.l >> 4;
  row0 = uni(row0);
  W.n = uni(p.n);
  const int d = uni(p.d);
  const bool nu5 = uni(p.nu2) == 5;
  W.amp = uni(p.amp);
  W.c1 = (nu5 ? 2.23606797749978969641 : 1.73205080756887729353) * uni(p.inv_l);
  W.c2 = nu5 ? 1.0 / 3.0 : 0.0;
  W.xs = xs;
  W.as = as;
  const int64_t N_pad = uni(p.N_pad);
  const auto X64 = gptr(uni(p.X64));
  const int64_t my_row = row0 + (W.l & 15);
#pragma unroll
  for (int j = 0; j < DM; ++j) {
    const double v = X64[(int64_t)(j < d ? j : d - 1) * N_pad + my_row];
    W.xr[j] = j < d ? v : 0.0;
  }
  const int jb = reg_jb(W.n);
  const int jp = uni(p.n_pad) / 16;  // blocks of the packed layout
  W.rB = buffer_of(uni(p.Bpk), 2 * jp * (jp + 1) * 64 * (int)sizeof(double));
  W.mp = 0.0;
  for (int i = 0; i < 4; ++i) W.sq[i] = 0.0;
  const int passes = (jb + PW - 1) / PW;
  const int first = jb - PW * (passes - 1);
  switch (first) {
#define BO_BIG_CASE(NB) \
  case NB: if constexpr (NB <= PW) W.template pass<NB>(0, passes == 1); break;
    BO_BIG_CASE(1) BO_BIG_CASE(2) BO_BIG_CASE(3) BO_BIG_CASE(4) BO_BIG_CASE(5) BO_BIG_CASE(6)
    BO_BIG_CASE(7) BO_BIG_CASE(8) BO_BIG_CASE(9) BO_BIG_CASE(10) BO_BIG_CASE(11) BO_BIG_CASE(12)
    BO_BIG_CASE(13) BO_BIG_CASE(14) BO_BIG_CASE(15)
#undef BO_BIG_CASE
    default: W.template pass<PW>(0, passes == 1); break;
  }
  for (int k = 1; k < passes; ++k) W.template pass<PW>(first + PW * (k - 1), k == passes - 1);
  post16_store(p, row0, W.mp, W.sq, part_out, cnt_out);
}

// Launch arguments of a session's posterior.
inline PostArgs make_post_args(const DevPtrs& P, const Layout& Lo, const GpConst& g, int n, int64_t n_valid,
                               const uint8_t* visited, const AcqArgs& acq) {
  PostArgs a{};
  a.n = n;
  a.n_pad = n_pad_of(n);
  a.out32 = Lo.prec == BO_FP64 ? 0 : 1;
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
  a.mu = P.mu;
  a.var = P.var;
  a.vslots = P.vslots;
  a.st = P.st;
  a.acq = acq;
  return a;
}

}  // namespace bo
