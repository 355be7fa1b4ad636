// Surrogate fit in FP64 (Section III-B, fixed lengthscale): K_nn with the
// jitter schedule, blocked Cholesky L L^T = K_nn + delta I, explicit L^-1,
// alpha = L^-T L^-1 (y - m), and the packing of L^-1 into the operand layout
// of the posterior kernels.
//
// All dense work is done on 32 x 32 FP64 tiles by "quads" of 256 threads.
// n <= 256: one 1024-thread workgroup (4 quads) runs the whole fit, jitter
// retries included.  n > 256: one launch per phase, one quad per tile.
#include "bo_internal.h"
#include "bo_device.h"

namespace bo {
namespace {

constexpr int T = 32;
constexpr int LDP = 33;
constexpr int QT = 256;

struct FitArgs {
  int n, n_pad, NB, d, nu2, tries, prec;
  double inv_l, amp, noise;
  const int64_t* obs_idx;
  const double* y_in;
  int64_t N, N_pad;
  const int32_t* inv_map;
  const double* X64;
  double* Xo64;
  float* Xo32;
  double* y;
  double* A;
  double* L;
  double* Dinv;
  double* Linv;
  double* alpha;
  double* z;
  void* Bpk;
  DevState* st;
};

typedef double Tile[T][LDP];

__device__ __forceinline__ size_t tix(const FitArgs& a, int ti, int tj, int r, int c) {
  return (size_t)(ti * T + r) * a.n_pad + tj * T + c;
}

__device__ __forceinline__ void tri_decode(int t, int* i, int* j) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  *i = r;
  *j = t - r * (r + 1) / 2;
}

__device__ __forceinline__ void load_tile(Tile& s, const double* M, const FitArgs& a, int ti, int tj, int qt) {
  for (int e = qt; e < T * T; e += QT) {
    const int r = e >> 5, c = e & 31;
    s[r][c] = M[tix(a, ti, tj, r, c)];
  }
}

// ---- phase 0: gather observations, validate, prior mean and incumbent ----
// Runs in one workgroup of 1024 threads (n <= 1024).
__device__ void fit_gather(const FitArgs& a, double* s_red, int* s_bad) {
  const int t = threadIdx.x;
  if (t == 0) *s_bad = 0;
  __syncthreads();
  double yv = 0.0, ymin = INFINITY;
  for (int i = t; i < a.n_pad; i += blockDim.x) {
    if (i < a.n) {
      const int64_t idx = a.obs_idx[i];
      const double v = a.y_in[i];
      int pos = -1;
      if (idx >= 0 && idx < a.N) pos = a.inv_map[idx];
      if (pos < 0 || !isfinite(v)) {
        atomicExch(s_bad, 1);
        pos = 0;
      }
      for (int j = 0; j < kMaxD; ++j) {
        const double x = j < a.d ? a.X64[(int64_t)j * a.N_pad + pos] : 0.0;
        a.Xo64[i * kMaxD + j] = x;
        a.Xo32[i * kMaxD + j] = (float)x;
      }
      a.y[i] = v;
      yv += v;
      ymin = fmin(ymin, v);
    } else {
      for (int j = 0; j < kMaxD; ++j) {
        a.Xo64[i * kMaxD + j] = 0.0;
        a.Xo32[i * kMaxD + j] = 0.f;
      }
      a.y[i] = 0.0;
    }
  }
  // fixed-order tree reductions of the sum and the minimum
  s_red[t] = yv;
  s_red[blockDim.x + t] = ymin;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (t < off) {
      s_red[t] += s_red[t + off];
      s_red[blockDim.x + t] = fmin(s_red[blockDim.x + t], s_red[blockDim.x + t + off]);
    }
    __syncthreads();
  }
  if (t == 0) {
    DevState* st = a.st;
    st->n = a.n;
    st->mean_y = s_red[0] / (double)a.n;
    st->f_best = s_red[blockDim.x];
    st->status = *s_bad ? (int)BO_E_INVALID_ARG : (int)BO_OK;
    st->need_retry = 0;
    st->fail_flag = 0;
    st->attempt = 0;
  }
  __syncthreads();
}

// ---- tile operations (one quad of 256 threads per tile) ----
// Each op is split at one barrier: load inputs into LDS, then compute.

// K_nn tile: amp * Matern(|xo_i - xo_j|) + delta on the diagonal; padded rows
// and columns form an identity block so the padded factor stays regular.
__device__ void op_build(const FitArgs& a, int ti, int tj, double delta, int qt) {
  for (int e = qt; e < T * T; e += QT) {
    const int r = e >> 5, c = e & 31;
    const int gi = ti * T + r, gj = tj * T + c;
    double v;
    if (gi < a.n && gj < a.n) {
      double s = 0.0;
      for (int k = 0; k < a.d; ++k) {
        const double df = a.Xo64[gi * kMaxD + k] - a.Xo64[gj * kMaxD + k];
        s += df * df;
      }
      v = a.amp * matern64(a.nu2, sqrt(s), a.inv_l) + (gi == gj ? delta : 0.0);
    } else {
      v = gi == gj ? 1.0 : 0.0;
    }
    a.A[tix(a, ti, tj, r, c)] = v;
  }
}

// Diagonal block: in-LDS Cholesky with the pivot test, then its inverse.
// Right-looking, one barrier per column: every thread reads the unscaled
// pivot column, writes the scaled column into s1 and updates the trailing
// columns of s0.  The inverse of the factor (into s0) is a row sweep of
// forward substitution with 8 threads per column.  Executed by one quad of
// 256 threads; in the 1024-thread fit the other quads only join the barriers.
__device__ bool op_diag(const FitArgs& a, int k, double delta, Tile& s0, Tile& s1, int* s_fail, int qt,
                        bool active) {
  (void)s_fail;
  if (active) load_tile(s0, a.A, a, k, k, qt);
  __syncthreads();
  const double thr = (double)a.n * 2.220446049250313e-16 * (a.amp + delta);
  bool fail = false;
  for (int c = 0; c < T; ++c) {
    const double piv = s0[c][c];
    const double lim = (k * T + c) < a.n ? thr : 0.0;
    if (!isfinite(piv) || !(piv > lim)) {
      fail = true;  // every thread sees the same pivot
      break;
    }
    if (active) {
      const double inv_piv = 1.0 / piv;
      const double sq = sqrt(piv);
      for (int e = qt; e < T * T; e += QT) {
        const int r = e >> 5, q = e & 31;
        if (q == c) {
          if (r >= c) s1[r][c] = (r == c) ? sq : s0[r][c] / sq;
        } else if (q > c && r >= q) {
          s0[r][q] -= s0[r][c] * s0[q][c] * inv_piv;
        }
      }
    }
    __syncthreads();
  }
  if (fail) {
    __syncthreads();
    return true;
  }
  // inverse of the lower-triangular factor s1 into s0, row by row
  const int q = qt >> 3, part = qt & 7;
  for (int r = 0; r < T; ++r) {
    if (active && q <= r) {
      double v = 0.0;
      for (int m = q + part; m < r; m += 8) v += s1[r][m] * s0[m][q];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      if (part == 0) s0[r][q] = ((r == q ? 1.0 : 0.0) - v) / s1[r][r];
    }
    if (active && q > r && part == 0) s0[r][q] = 0.0;
    __syncthreads();
  }
  if (active) {
    for (int e = qt; e < T * T; e += QT) {
      const int r = e >> 5, c = e & 31;
      a.L[tix(a, k, k, r, c)] = c <= r ? s1[r][c] : 0.0;
      a.Dinv[(size_t)k * T * T + r * T + c] = s0[r][c];
    }
  }
  __syncthreads();
  return false;
}

// L_ik = A_ik Dinv_k^T
__device__ void op_panel_load(const FitArgs& a, int i, int k, Tile& s0, Tile& s1, int qt) {
  load_tile(s0, a.A, a, i, k, qt);
  for (int e = qt; e < T * T; e += QT) s1[e >> 5][e & 31] = a.Dinv[(size_t)k * T * T + e];
}
__device__ void op_panel_comp(const FitArgs& a, int i, int k, Tile& s0, Tile& s1, int qt) {
  for (int e = qt; e < T * T; e += QT) {
    const int r = e >> 5, c = e & 31;
    double v = 0.0;
    for (int s = 0; s <= c; ++s) v += s0[r][s] * s1[c][s];
    a.L[tix(a, i, k, r, c)] = v;
  }
}

// A_ij -= L_ik L_jk^T
__device__ void op_update_load(const FitArgs& a, int i, int j, int k, Tile& s0, Tile& s1, int qt) {
  load_tile(s0, a.L, a, i, k, qt);
  load_tile(s1, a.L, a, j, k, qt);
}
__device__ void op_update_comp(const FitArgs& a, int i, int j, Tile& s0, Tile& s1, int qt) {
  for (int e = qt; e < T * T; e += QT) {
    const int r = e >> 5, c = e & 31;
    double v = a.A[tix(a, i, j, r, c)];
    for (int s = 0; s < T; ++s) v -= s0[r][s] * s1[c][s];
    a.A[tix(a, i, j, r, c)] = v;
  }
}

// Inverse, block row p: X_pj = Dinv_p R_pj (j < p), X_pp = Dinv_p, with the
// running right-hand side R kept in A.
__device__ void op_invf_load(const FitArgs& a, int p, int j, Tile& s0, Tile& s1, int qt) {
  for (int e = qt; e < T * T; e += QT) s0[e >> 5][e & 31] = a.Dinv[(size_t)p * T * T + e];
  if (j < p) load_tile(s1, a.A, a, p, j, qt);
}
__device__ void op_invf_comp(const FitArgs& a, int p, int j, Tile& s0, Tile& s1, int qt) {
  for (int e = qt; e < T * T; e += QT) {
    const int r = e >> 5, c = e & 31;
    double v;
    if (j == p) {
      v = s0[r][c];
    } else {
      v = 0.0;
      for (int s = 0; s <= r; ++s) v += s0[r][s] * s1[s][c];
    }
    a.Linv[tix(a, p, j, r, c)] = v;
  }
}

// R_ij -= L_ip X_pj (i > p >= j)
__device__ void op_invu_load(const FitArgs& a, int i, int j, int p, Tile& s0, Tile& s1, int qt) {
  load_tile(s0, a.L, a, i, p, qt);
  load_tile(s1, a.Linv, a, p, j, qt);
}
__device__ void op_invu_comp(const FitArgs& a, int i, int j, int p, Tile& s0, Tile& s1, int qt) {
  for (int e = qt; e < T * T; e += QT) {
    const int r = e >> 5, c = e & 31;
    // column block j is first touched in phase p == j: R starts at zero there
    double v = (j == p) ? 0.0 : a.A[tix(a, i, j, r, c)];
    for (int s = 0; s < T; ++s) v -= s0[r][s] * s1[s][c];
    a.A[tix(a, i, j, r, c)] = v;
  }
}

// ---- alpha = L^-T (L^-1 (y - m)) : one wave per row ----
__device__ void alpha_z_row(const FitArgs& a, int i, double m, int lane) {
  double v = 0.0;
  for (int j = lane; j <= i; j += 64) {
    const double r = j < a.n ? a.y[j] - m : 0.0;
    v += a.Linv[(size_t)i * a.n_pad + j] * r;
  }
  for (int off = 32; off > 0; off >>= 1) v += shfl_xor_d(v, off);
  if (lane == 0) a.z[i] = v;
}
__device__ void alpha_a_row(const FitArgs& a, int i, int lane) {
  double v = 0.0;
  for (int j = i + lane; j < a.n_pad; j += 64) v += a.Linv[(size_t)j * a.n_pad + i] * a.z[j];
  for (int off = 32; off > 0; off >>= 1) v += shfl_xor_d(v, off);
  if (lane == 0) a.alpha[i] = i < a.n ? v : 0.0;
}

// ---- packing of L^-1 for the matrix-core posterior kernels ----
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ double linv_at(const FitArgs& a, int row, int col) {
  return (col <= row && row < a.n && col < a.n) ? a.Linv[(size_t)row * a.n_pad + col] : 0.0;
}

// FP64 / FP32, 16x16x4 operand: fragment (J, t) at 2J(J+1) + t, t <= 4J+3;
// lane l holds L^-1[16J + l%16][4t + l/16] (the transpose, as the B operand).
__device__ void pack_elem16(const FitArgs& a, int64_t e) {
  const int64_t f = e >> 6;
  const int l = (int)(e & 63);
  int J = (int)((sqrt(2.0 * (double)f + 1.0) - 1.0) * 0.5);
  while (2LL * (J + 1) * (J + 2) <= f) ++J;
  while (2LL * J * (J + 1) > f) --J;
  const int t = (int)(f - 2LL * J * (J + 1));
  const double v = linv_at(a, 16 * J + (l & 15), 4 * t + (l >> 4));
  if (a.prec == BO_FP64) ((double*)a.Bpk)[e] = v;
  else ((float*)a.Bpk)[e] = (float)v;
}

// BF16X3, 32x32x16 operand: fragment (J, t) at J(J+1) + t, t <= 2J+1; lane l
// holds 8 values L^-1[32J + l%32][16t + 8(l/32) + e]; high parts first, then
// the low parts (value - high) in a second array of the same shape.
__device__ void pack_elem32(const FitArgs& a, int64_t e, int64_t nfrag) {
  const int64_t f = e >> 6;
  const int l = (int)(e & 63);
  int J = (int)((sqrt(4.0 * (double)f + 1.0) - 1.0) * 0.5);
  while ((int64_t)(J + 1) * (J + 2) <= f) ++J;
  while ((int64_t)J * (J + 1) > f) --J;
  const int t = (int)(f - (int64_t)J * (J + 1));
  uint16_t hi[8], lo[8];
  for (int q = 0; q < 8; ++q) {
    const float v = (float)linv_at(a, 32 * J + (l & 31), 16 * t + 8 * (l >> 5) + q);
    hi[q] = bf16_rne(v);
    const float rem = v - __uint_as_float((uint32_t)hi[q] << 16);
    lo[q] = bf16_rne(rem);
  }
  uint4 h, w;
  h.x = hi[0] | ((uint32_t)hi[1] << 16);
  h.y = hi[2] | ((uint32_t)hi[3] << 16);
  h.z = hi[4] | ((uint32_t)hi[5] << 16);
  h.w = hi[6] | ((uint32_t)hi[7] << 16);
  w.x = lo[0] | ((uint32_t)lo[1] << 16);
  w.y = lo[2] | ((uint32_t)lo[3] << 16);
  w.z = lo[4] | ((uint32_t)lo[5] << 16);
  w.w = lo[6] | ((uint32_t)lo[7] << 16);
  ((uint4*)a.Bpk)[e] = h;
  ((uint4*)a.Bpk)[nfrag * 64 + e] = w;
}

__device__ __forceinline__ int64_t pack_count(const FitArgs& a, int64_t* nfrag) {
  if (a.prec == BO_BF16X3) {
    const int64_t JB = a.n_pad / 32;
    *nfrag = JB * (JB + 1);
  } else {
    const int64_t JB = a.n_pad / 16;
    *nfrag = 2 * JB * (JB + 1);
  }
  return *nfrag * 64;
}

// ======================= small fit: one workgroup =========================
constexpr int kSmallThreads = 1024;
constexpr int NQ = kSmallThreads / QT;

__global__ __launch_bounds__(kSmallThreads) void k_fit_small(FitArgs a) {
  __shared__ Tile s_t[NQ][2];
  __shared__ double s_red[2 * kSmallThreads];
  __shared__ int s_flag;
  const int quad = threadIdx.x / QT, qt = threadIdx.x % QT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = kSmallThreads / 64;

  fit_gather(a, s_red, &s_flag);
  if (a.st->status != BO_OK) return;

  bool fail = true;
  double delta = 0.0;
  int attempt = 0;
  for (attempt = 0; attempt < a.tries; ++attempt) {
    delta = jitter_of(a.noise, a.amp, attempt);
    const int nlow = a.NB * (a.NB + 1) / 2;
    for (int t = quad; t < nlow; t += NQ) {
      int i, j;
      tri_decode(t, &i, &j);
      op_build(a, i, j, delta, qt);
    }
    __syncthreads();
    fail = false;
    for (int k = 0; k < a.NB && !fail; ++k) {
      fail = op_diag(a, k, delta, s_t[0][0], s_t[0][1], &s_flag, qt, quad == 0);
      if (fail) break;
      const int np = a.NB - k - 1;
      for (int base = 0; base < np; base += NQ) {
        const int t = base + quad;
        if (t < np) op_panel_load(a, k + 1 + t, k, s_t[quad][0], s_t[quad][1], qt);
        __syncthreads();
        if (t < np) op_panel_comp(a, k + 1 + t, k, s_t[quad][0], s_t[quad][1], qt);
        __syncthreads();
      }
      const int nu = np * (np + 1) / 2;
      for (int base = 0; base < nu; base += NQ) {
        const int t = base + quad;
        int i = 0, j = 0;
        if (t < nu) {
          tri_decode(t, &i, &j);
          i += k + 1;
          j += k + 1;
          op_update_load(a, i, j, k, s_t[quad][0], s_t[quad][1], qt);
        }
        __syncthreads();
        if (t < nu) op_update_comp(a, i, j, s_t[quad][0], s_t[quad][1], qt);
        __syncthreads();
      }
    }
    if (!fail) break;
  }
  if (fail) {
    if (threadIdx.x == 0) {
      a.st->status = BO_E_NOT_PD;
      a.st->attempt = a.tries - 1;
    }
    return;
  }
  // explicit inverse, block row by block row
  for (int p = 0; p < a.NB; ++p) {
    for (int base = 0; base <= p; base += NQ) {
      const int j = base + quad;
      if (j <= p) op_invf_load(a, p, j, s_t[quad][0], s_t[quad][1], qt);
      __syncthreads();
      if (j <= p) op_invf_comp(a, p, j, s_t[quad][0], s_t[quad][1], qt);
      __syncthreads();
    }
    const int ni = a.NB - p - 1, nt = ni * (p + 1);
    for (int base = 0; base < nt; base += NQ) {
      const int t = base + quad;
      const int i = p + 1 + (t / (p + 1)), j = t % (p + 1);
      if (t < nt) op_invu_load(a, i, j, p, s_t[quad][0], s_t[quad][1], qt);
      __syncthreads();
      if (t < nt) op_invu_comp(a, i, j, p, s_t[quad][0], s_t[quad][1], qt);
      __syncthreads();
    }
  }
  const double m = a.st->mean_y;
  for (int i = wave; i < a.n_pad; i += nwave) alpha_z_row(a, i, m, lane);
  __syncthreads();
  for (int i = wave; i < a.n_pad; i += nwave) alpha_a_row(a, i, lane);
  int64_t nfrag;
  const int64_t ne = pack_count(a, &nfrag);
  for (int64_t e = threadIdx.x; e < ne; e += kSmallThreads) {
    if (a.prec == BO_BF16X3) pack_elem32(a, e, nfrag);
    else pack_elem16(a, e);
  }
  if (threadIdx.x == 0) {
    a.st->jitter = delta;
    a.st->attempt = attempt;
    a.st->status = BO_OK;
  }
}

// ======================= large fit: one launch per phase ==================
__global__ __launch_bounds__(1024) void k_fitL_gather(FitArgs a) {
  __shared__ double s_red[2 * 1024];
  __shared__ int s_flag;
  fit_gather(a, s_red, &s_flag);
}

__global__ __launch_bounds__(QT) void k_fitL_build(FitArgs a, int attempt) {
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  int i, j;
  tri_decode(blockIdx.x, &i, &j);
  op_build(a, i, j, jitter_of(a.noise, a.amp, attempt), threadIdx.x);
}

__global__ __launch_bounds__(QT) void k_fitL_diag(FitArgs a, int k, int attempt) {
  __shared__ Tile s0, s1;
  __shared__ int s_flag;
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  const bool fail = op_diag(a, k, jitter_of(a.noise, a.amp, attempt), s0, s1, &s_flag, threadIdx.x, true);
  if (fail && threadIdx.x == 0) {
    a.st->fail_flag = 1;
    a.st->attempt = attempt;
  }
}

__global__ __launch_bounds__(QT) void k_fitL_panel(FitArgs a, int k) {
  __shared__ Tile s0, s1;
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  const int i = k + 1 + blockIdx.x;
  op_panel_load(a, i, k, s0, s1, threadIdx.x);
  __syncthreads();
  op_panel_comp(a, i, k, s0, s1, threadIdx.x);
}

__global__ __launch_bounds__(QT) void k_fitL_update(FitArgs a, int k) {
  __shared__ Tile s0, s1;
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  int i, j;
  tri_decode(blockIdx.x, &i, &j);
  i += k + 1;
  j += k + 1;
  op_update_load(a, i, j, k, s0, s1, threadIdx.x);
  __syncthreads();
  op_update_comp(a, i, j, s0, s1, threadIdx.x);
}

__global__ __launch_bounds__(QT) void k_fitL_invf(FitArgs a, int p) {
  __shared__ Tile s0, s1;
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  op_invf_load(a, p, blockIdx.x, s0, s1, threadIdx.x);
  __syncthreads();
  op_invf_comp(a, p, blockIdx.x, s0, s1, threadIdx.x);
}

__global__ __launch_bounds__(QT) void k_fitL_invu(FitArgs a, int p) {
  __shared__ Tile s0, s1;
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  const int t = blockIdx.x;
  const int i = p + 1 + t / (p + 1), j = t % (p + 1);
  op_invu_load(a, i, j, p, s0, s1, threadIdx.x);
  __syncthreads();
  op_invu_comp(a, i, j, p, s0, s1, threadIdx.x);
}

__global__ __launch_bounds__(QT) void k_fitL_alpha_z(FitArgs a) {
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  const int i = blockIdx.x * (QT / 64) + (threadIdx.x >> 6);
  if (i < a.n_pad) alpha_z_row(a, i, a.st->mean_y, threadIdx.x & 63);
}

__global__ __launch_bounds__(QT) void k_fitL_alpha_a(FitArgs a) {
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  const int i = blockIdx.x * (QT / 64) + (threadIdx.x >> 6);
  if (i < a.n_pad) alpha_a_row(a, i, threadIdx.x & 63);
}

__global__ __launch_bounds__(QT) void k_fitL_pack(FitArgs a, int attempt) {
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
  for (int64_t e = (int64_t)blockIdx.x * QT + threadIdx.x; e < ne; e += (int64_t)gridDim.x * QT) {
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

FitArgs make_args(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                  const double* y_in, int n) {
  FitArgs a{};
  a.n = n;
  a.n_pad = n_pad_of(n);
  a.NB = a.n_pad / T;
  a.d = Lo.d;
  a.nu2 = g.nu2;
  a.tries = g.tries;
  a.prec = Lo.prec;
  a.inv_l = 1.0 / g.l;
  a.amp = g.amp;
  a.noise = g.noise;
  a.obs_idx = obs_idx;
  a.y_in = y_in;
  a.N = Lo.N;
  a.N_pad = Lo.N_pad;
  a.inv_map = P.inv_map;
  a.X64 = P.X64;
  a.Xo64 = P.Xo64;
  a.Xo32 = P.Xo32;
  a.y = P.y;
  a.A = P.A;
  a.L = P.L;
  a.Dinv = P.Dinv;
  a.Linv = P.Linv;
  a.alpha = P.alpha;
  a.z = P.z;
  a.Bpk = P.Bpk;
  a.st = P.st;
  return a;
}

}  // namespace

hipError_t launch_fit_small(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                            const double* y_in, int n, hipStream_t st) {
  FitArgs a = make_args(P, Lo, g, obs_idx, y_in, n);
  hipLaunchKernelGGL(k_fit_small, dim3(1), dim3(kSmallThreads), 0, st, a);
  return hipGetLastError();
}

// One attempt of the jitter schedule (attempt = first_attempt).  The gather
// phase runs only on the first attempt.  On a pivot failure st->need_retry is
// set and st->status = BO_E_NOT_PD; the host retries with the next attempt.
hipError_t launch_fit_large(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                            const double* y_in, int n, int attempt, hipStream_t st) {
  FitArgs a = make_args(P, Lo, g, obs_idx, y_in, n);
  const int NB = a.NB;
  if (attempt == 0) hipLaunchKernelGGL(k_fitL_gather, dim3(1), dim3(1024), 0, st, a);
  else hipLaunchKernelGGL(k_fitL_rearm, dim3(1), dim3(64), 0, st, P.st);
  hipLaunchKernelGGL(k_fitL_build, dim3(NB * (NB + 1) / 2), dim3(QT), 0, st, a, attempt);
  for (int k = 0; k < NB; ++k) {
    hipLaunchKernelGGL(k_fitL_diag, dim3(1), dim3(QT), 0, st, a, k, attempt);
    const int np = NB - k - 1;
    if (np > 0) {
      hipLaunchKernelGGL(k_fitL_panel, dim3(np), dim3(QT), 0, st, a, k);
      hipLaunchKernelGGL(k_fitL_update, dim3(np * (np + 1) / 2), dim3(QT), 0, st, a, k);
    }
  }
  for (int p = 0; p < NB; ++p) {
    hipLaunchKernelGGL(k_fitL_invf, dim3(p + 1), dim3(QT), 0, st, a, p);
    const int nt = (NB - p - 1) * (p + 1);
    if (nt > 0) hipLaunchKernelGGL(k_fitL_invu, dim3(nt), dim3(QT), 0, st, a, p);
  }
  const int rows = a.n_pad / (QT / 64);
  hipLaunchKernelGGL(k_fitL_alpha_z, dim3(rows), dim3(QT), 0, st, a);
  hipLaunchKernelGGL(k_fitL_alpha_a, dim3(rows), dim3(QT), 0, st, a);
  hipLaunchKernelGGL(k_fitL_pack, dim3(512), dim3(QT), 0, st, a, attempt);
  return hipGetLastError();
}

}  // namespace bo
