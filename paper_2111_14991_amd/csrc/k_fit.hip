// Surrogate fit in FP64 (Section III-B, fixed lengthscale): K_nn with the
// jitter schedule, blocked Cholesky L L^T = K_nn + delta I, explicit L^-1,
// alpha = L^-T L^-1 (y - m), and the packing of L^-1 into the operand layout
// of the posterior kernels.
//
// Dense work runs on 64 x 64 FP64 tiles, one "team" of 256 threads per tile
// (each thread owns a 4 x 4 block of the tile).  Block step k:
//   A_k: factor the diagonal tile A_kk (in LDS, one barrier per column; the
//        pivot test decides the jitter schedule), invert the factor, then
//        either write the panel tile L_ik = A_ik L_kk^-T (i > k) or finalize
//        block row k of the inverse, X_kj = L_kk^-1 R_kj (j < k), X_kk;
//   B_k: trailing update A_ij -= L_ik L_jk^T (k < j <= i) and the running
//        right-hand side of the inverse R_ij -= L_ik X_kj (i > k >= j).
// n <= 256: one workgroup (two teams) runs every step, jitter retries
// included.  n > 256: one launch per A_k / B_k with one team per tile; the
// host retries the jitter schedule after a pivot failure.
#include "bo_internal.h"
#include "bo_device.h"

namespace bo {
namespace {

constexpr int T = 64;     // tile edge
constexpr int LDP = 65;   // LDS row pitch (doubles)
constexpr int TT = 256;   // threads per team

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
  double* A;     // working matrix, later the running right-hand side R of the inverse
  double* L;
  double* Dinv;  // inverses of the diagonal tiles of L
  double* Linv;  // X = L^-1
  double* K0;    // symmetric copy of amp * Matern without jitter, or null
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

__device__ __forceinline__ void load_tile(Tile& s, const double* M, const FitArgs& a, int ti, int tj, int tt) {
  for (int e = tt; e < T * T; e += TT) {
    const int r = e >> 6, c = e & 63;
    s[r][c] = M[tix(a, ti, tj, r, c)];
  }
}

__device__ __forceinline__ void load_dinv(Tile& s, const FitArgs& a, int k, int tt) {
  const double* D = a.Dinv + (size_t)k * T * T;
  for (int e = tt; e < T * T; e += TT) s[e >> 6][e & 63] = D[e];
}

// ---- phase 0: gather observations, validate, prior mean and incumbent ----
// Runs in one workgroup (n <= 1024); s_red holds 2 * blockDim.x doubles and
// s_pos 1024 ints.
__device__ void fit_gather(const FitArgs& a, double* s_red, int* s_pos, int* s_bad) {
  const int t = threadIdx.x, nt = blockDim.x;
  if (t == 0) *s_bad = 0;
  __syncthreads();
  double yv = 0.0, ymin = INFINITY;
  for (int i = t; i < a.n_pad; i += nt) {
    int pos = 0;
    double v = 0.0;
    if (i < a.n) {
      const int64_t idx = a.obs_idx[i];
      v = a.y_in[i];
      pos = (idx >= 0 && idx < a.N) ? a.inv_map[idx] : -1;
      if (pos < 0 || !isfinite(v)) {
        atomicExch(s_bad, 1);
        pos = 0;
      }
      yv += v;
      ymin = fmin(ymin, v);
    }
    s_pos[i] = pos;
    a.y[i] = v;
  }
  __syncthreads();
  // coordinates: one (observation, dimension) pair per thread and round
  for (int e = t; e < a.n_pad * kMaxD; e += nt) {
    const int i = e / kMaxD, j = e % kMaxD;
    const double x = (i < a.n && j < a.d) ? a.X64[(int64_t)j * a.N_pad + s_pos[i]] : 0.0;
    a.Xo64[e] = x;
    a.Xo32[e] = (float)x;
  }
  // fixed-order tree reductions of the sum and the minimum
  s_red[t] = yv;
  s_red[nt + t] = ymin;
  __syncthreads();
  for (int off = nt / 2; off > 0; off >>= 1) {
    if (t < off) {
      s_red[t] += s_red[t + off];
      s_red[nt + t] = fmin(s_red[nt + t], s_red[nt + t + off]);
    }
    __syncthreads();
  }
  if (t == 0) {
    DevState* st = a.st;
    st->n = a.n;
    st->mean_y = s_red[0] / (double)a.n;
    st->f_best = s_red[nt];
    st->status = *s_bad ? (int)BO_E_INVALID_ARG : (int)BO_OK;
    st->need_retry = 0;
    st->fail_flag = 0;
    st->attempt = 0;
  }
  __syncthreads();
}

// ---- tile operations (one team; thread tt = 64 w + lane owns rows
// 16w .. 16w+15 of column `lane`, so the lanes of a wave touch consecutive
// LDS words and the row operand is a broadcast) ----

// K_nn tile: amp * Matern(|xo_i - xo_j|) + delta on the diagonal; padded rows
// and columns form an identity block so the padded factor stays regular.
// xs holds the coordinates of row block ti (rows 0..63) and column block tj
// (rows 64..127) as [128][kMaxD + 1] doubles.
__device__ void op_build(const FitArgs& a, int ti, int tj, double delta, double* xs, int tt) {
  for (int e = tt; e < 128 * kMaxD; e += TT) {
    const int r = e / kMaxD, j = e % kMaxD;
    const int g = (r < 64 ? ti * T + r : tj * T + r - 64);
    xs[r * (kMaxD + 1) + j] = a.Xo64[g * kMaxD + j];
  }
  __syncthreads();
  const int w = tt >> 6, c = tt & 63;
  const int gj = tj * T + c;
  const double* xc = xs + (64 + c) * (kMaxD + 1);
  for (int i = 0; i < 16; ++i) {
    const int r = 16 * w + i;
    const int gi = ti * T + r;
    const double* xr = xs + r * (kMaxD + 1);
    double v, v0 = 0.0;
    if (gi < a.n && gj < a.n) {
      double s2 = 0.0;
      for (int k = 0; k < a.d; ++k) {
        const double df = xr[k] - xc[k];
        s2 += df * df;
      }
      v0 = a.amp * matern64(a.nu2, sqrt(s2), a.inv_l);
      v = v0 + (gi == gj ? delta : 0.0);
    } else {
      v = gi == gj ? 1.0 : 0.0;
    }
    a.A[tix(a, ti, tj, r, c)] = v;
    if (a.K0) {
      a.K0[(size_t)gi * a.n_pad + gj] = v0;
      a.K0[(size_t)gj * a.n_pad + gi] = v0;
    }
  }
  __syncthreads();
}

// C (global tile) = init - sign * A B^T (NT) or A B (NN), A and B in LDS.
// init is the current C when `accumulate`, else zero.
template <bool NT>
__device__ void op_gemm(double* C, const FitArgs& a, int ti, int tj, const Tile& A, const Tile& B, bool accumulate,
                        double sign, int tt) {
  const int w = tt >> 6, c = tt & 63;
  double acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0;
  for (int k = 0; k < T; ++k) {
    const double bv = NT ? B[c][k] : B[k][c];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = fma(A[16 * w + i][k], bv, acc[i]);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const size_t ix = tix(a, ti, tj, 16 * w + i, c);
    const double base = accumulate ? C[ix] : 0.0;
    C[ix] = base - sign * acc[i];
  }
}

// Diagonal tile k: Cholesky with the pivot test, then the inverse of the
// factor, with the tile held in registers by all NT threads of the workgroup
// (thread 64 w + q owns rows S w .. S w + S - 1 of column q, S = 4096 / NT).
// One barrier per column: the owner of column c publishes it through LDS
// (double-buffered), every thread updates its rows; the inverse is a
// right-looking forward substitution on the identity.  The factor is left in
// s1 and its inverse in s0.  Returns true when a pivot fails (the same answer
// in every thread).
template <int NT>
__device__ bool op_diag(const FitArgs& a, int k, double delta, Tile& s0, Tile& s1, double (*colbuf)[64],
                        double (*xbuf)[64]) {
  constexpr int S = 4096 / NT;
  const int tt = threadIdx.x;
  const int w = tt >> 6, q = tt & 63, r0 = S * w;
  double av[S], lv[S], xv[S];
#pragma unroll
  for (int i = 0; i < S; ++i) av[i] = a.A[tix(a, k, k, r0 + i, q)];
  const double thr = (double)a.n * 2.220446049250313e-16 * (a.amp + delta);
  for (int c = 0; c < T; ++c) {
    double* col = colbuf[c & 1];
    if (q == c) {
#pragma unroll
      for (int i = 0; i < S; ++i) col[r0 + i] = av[i];
    }
    __syncthreads();
    const double piv = col[c];
    const double lim = (k * T + c) < a.n ? thr : 0.0;
    if (!(piv > lim) || !(piv < INFINITY)) return true;
    if (r0 + S - 1 > c && q > c) {
      const double cqs = col[q] / piv;
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (r0 + i >= q) av[i] -= col[r0 + i] * cqs;
    }
    if (q == c) {
      const double sq = sqrt(piv);
      const double inv_sq = 1.0 / sq;
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const int r = r0 + i;
        lv[i] = r > c ? av[i] * inv_sq : (r == c ? sq : 0.0);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < S; ++i) xv[i] = (r0 + i == q) ? 1.0 : 0.0;
  for (int r = 0; r < T; ++r) {
    double* col = colbuf[r & 1];
    double* xr = xbuf[r & 1];
    if (q == r) {
#pragma unroll
      for (int i = 0; i < S; ++i) col[r0 + i] = lv[i];
    }
    if (r0 <= r && r < r0 + S) {
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (r0 + i == r) xr[q] = xv[i];
    }
    __syncthreads();
    if (r0 + S - 1 >= r) {
      const double x = xr[q] / col[r];
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const int rr = r0 + i;
        if (rr == r) xv[i] = x;
        else if (rr > r) xv[i] -= col[rr] * x;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < S; ++i) {
    s1[r0 + i][q] = lv[i];
    s0[r0 + i][q] = xv[i];
  }
  __syncthreads();
  return false;
}

// ---- block step k (shared by both paths) ----
// A_k work item b: b < k: X_kb = Dinv_k R_kb;  b == k: L_kk, Dinv_k, X_kk;
// b > k: L_bk = A_bk Dinv_k^T.  s0 holds Dinv_k, s1 the factor, s2 scratch.
__device__ void stepA_item(const FitArgs& a, int k, int b, Tile& s0, Tile& s1, Tile& s2, int tt, bool active) {
  if (active) {
    if (b < k) load_tile(s2, a.A, a, k, b, tt);
    else if (b > k) load_tile(s2, a.A, a, b, k, tt);
  }
  __syncthreads();
  if (!active) return;
  if (b < k) {
    op_gemm<false>(a.Linv, a, k, b, s0, s2, false, -1.0, tt);
  } else if (b > k) {
    op_gemm<true>(a.L, a, b, k, s2, s0, false, -1.0, tt);
  } else {
    for (int e = tt; e < T * T; e += TT) {
      const int r = e >> 6, c = e & 63;
      a.L[tix(a, k, k, r, c)] = c <= r ? s1[r][c] : 0.0;
      a.Linv[tix(a, k, k, r, c)] = s0[r][c];
      a.Dinv[(size_t)k * T * T + e] = s0[r][c];
    }
  }
}

// B_k work item t: first the trailing tiles (i, j), k < j <= i, then the
// inverse tiles (i, j), i > k >= j.
__device__ __forceinline__ int stepB_count(int NB, int k) {
  const int m = NB - 1 - k;
  return m * (m + 1) / 2 + m * (k + 1);
}

__device__ void stepB_item(const FitArgs& a, int k, int t, Tile& s0, Tile& s1, int tt, bool active) {
  const int m = a.NB - 1 - k;
  const int ntr = m * (m + 1) / 2;
  int i = 0, j = 0;
  const bool trailing = t < ntr;
  if (trailing) {
    tri_decode(t, &i, &j);
    i += k + 1;
    j += k + 1;
  } else {
    const int u = t - ntr;
    i = k + 1 + u / (k + 1);
    j = u % (k + 1);
  }
  if (active) {
    load_tile(s0, a.L, a, i, k, tt);
    if (trailing) load_tile(s1, a.L, a, j, k, tt);
    else load_tile(s1, a.Linv, a, k, j, tt);
  }
  __syncthreads();
  if (!active) return;
  if (trailing) op_gemm<true>(a.A, a, i, j, s0, s1, true, 1.0, tt);
  else op_gemm<false>(a.A, a, i, j, s0, s1, j != k, 1.0, tt);
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
constexpr int kSmallThreads = 2 * TT;
constexpr int NTEAM = kSmallThreads / TT;

__global__ __launch_bounds__(kSmallThreads) void k_fit_small(FitArgs a) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  // tiles[0], tiles[1]: Dinv / factor of the diagonal tile in step A, team 0's
  // operands in step B; tiles[2], tiles[3]: team scratch (A) / team 1 (B)
  Tile* tiles = reinterpret_cast<Tile*>(s_raw);
  double* s_red = reinterpret_cast<double*>(tiles + 4);
  __shared__ int s_flag;
  __shared__ int s_pos[kMaxN];
  __shared__ __align__(16) double s_colbuf[2][64];
  __shared__ __align__(16) double s_xbuf[2][64];
  const int team = threadIdx.x / TT, tt = threadIdx.x % TT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = kSmallThreads / 64;

  fit_gather(a, s_red, s_pos, &s_flag);
  if (a.st->status != BO_OK) return;

  bool fail = true;
  double delta = 0.0;
  int attempt = 0;
  for (attempt = 0; attempt < a.tries; ++attempt) {
    delta = jitter_of(a.noise, a.amp, attempt);
    const int nlow = a.NB * (a.NB + 1) / 2;
    for (int base = 0; base < nlow; base += NTEAM) {
      const int t = base + team;
      int i = 0, j = 0;
      if (t < nlow) tri_decode(t, &i, &j);
      // team scratch: the coordinates of the two blocks
      double* xs = reinterpret_cast<double*>(&tiles[2 + team][0][0]);
      if (t < nlow) {
        op_build(a, i, j, delta, xs, tt);
      } else {
        __syncthreads();
        __syncthreads();
      }
    }
    __syncthreads();
    fail = false;
    for (int k = 0; k < a.NB; ++k) {
      fail = op_diag<kSmallThreads>(a, k, delta, tiles[0], tiles[1], s_colbuf, s_xbuf);
      if (fail) break;
      for (int base = 0; base < a.NB; base += NTEAM) {
        const int b = base + team;
        stepA_item(a, k, b, tiles[0], tiles[1], tiles[2 + team], tt, b < a.NB);
        __syncthreads();
      }
      if (k + 1 < a.NB) {
        const int nb = stepB_count(a.NB, k);
        for (int base = 0; base < nb; base += NTEAM) {
          const int t = base + team;
          stepB_item(a, k, t, tiles[2 * team], tiles[2 * team + 1], tt, t < nb);
          __syncthreads();
        }
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
  __shared__ int s_pos[kMaxN];
  __shared__ int s_flag;
  fit_gather(a, s_red, s_pos, &s_flag);
}

__global__ __launch_bounds__(TT) void k_fitL_build(FitArgs a, int attempt) {
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  __shared__ double xs[128 * (kMaxD + 1)];
  int i, j;
  tri_decode(blockIdx.x, &i, &j);
  op_build(a, i, j, jitter_of(a.noise, a.amp, attempt), xs, threadIdx.x);
}

constexpr int kAThreads = 2 * TT;

__global__ __launch_bounds__(kAThreads) void k_fitL_A(FitArgs a, int k, int attempt) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  Tile* tiles = reinterpret_cast<Tile*>(s_raw);
  __shared__ __align__(16) double s_colbuf[2][64];
  __shared__ __align__(16) double s_xbuf[2][64];
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  const bool fail = op_diag<kAThreads>(a, k, jitter_of(a.noise, a.amp, attempt), tiles[0], tiles[1], s_colbuf,
                                       s_xbuf);
  if (fail) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.st->fail_flag = 1;
      a.st->attempt = attempt;
    }
    return;
  }
  stepA_item(a, k, blockIdx.x, tiles[0], tiles[1], tiles[2], threadIdx.x % TT, threadIdx.x < TT);
}

__global__ __launch_bounds__(TT) void k_fitL_B(FitArgs a, int k) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  Tile* tiles = reinterpret_cast<Tile*>(s_raw);
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  stepB_item(a, k, blockIdx.x, tiles[0], tiles[1], threadIdx.x, true);
}

__global__ __launch_bounds__(TT) void k_fitL_alpha_z(FitArgs a) {
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  const int i = blockIdx.x * (TT / 64) + (threadIdx.x >> 6);
  if (i < a.n_pad) alpha_z_row(a, i, a.st->mean_y, threadIdx.x & 63);
}

__global__ __launch_bounds__(TT) void k_fitL_alpha_a(FitArgs a) {
  if (a.st->status != BO_OK || a.st->fail_flag) return;
  const int i = blockIdx.x * (TT / 64) + (threadIdx.x >> 6);
  if (i < a.n_pad) alpha_a_row(a, i, threadIdx.x & 63);
}

__global__ __launch_bounds__(TT) void k_fitL_pack(FitArgs a, int attempt) {
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
  for (int64_t e = (int64_t)blockIdx.x * TT + threadIdx.x; e < ne; e += (int64_t)gridDim.x * TT) {
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
  a.K0 = P.K0;
  a.alpha = P.alpha;
  a.z = P.z;
  a.Bpk = P.Bpk;
  a.st = P.st;
  return a;
}

hipError_t set_lds(const void* f, size_t bytes) {
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

constexpr size_t kSmallLdsBytes = 4 * sizeof(Tile) + 2 * kSmallThreads * sizeof(double);

hipError_t prepare() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = set_lds((const void*)k_fit_small, kSmallLdsBytes);
  if (e == hipSuccess) e = set_lds((const void*)k_fitL_A, 3 * sizeof(Tile));
  if (e == hipSuccess) e = set_lds((const void*)k_fitL_B, 2 * sizeof(Tile));
  if (e == hipSuccess) done = true;
  return e;
}

}  // namespace

hipError_t launch_fit_small(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                            const double* y_in, int n, hipStream_t st) {
  hipError_t e = prepare();
  if (e != hipSuccess) return e;
  FitArgs a = make_args(P, Lo, g, obs_idx, y_in, n);
  hipLaunchKernelGGL(k_fit_small, dim3(1), dim3(kSmallThreads), kSmallLdsBytes, st, a);
  return hipGetLastError();
}

// One attempt of the jitter schedule.  The gather phase runs only on the
// first attempt.  On a pivot failure st->need_retry is set and st->status =
// BO_E_NOT_PD; the host retries with the next attempt.
hipError_t launch_fit_large(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                            const double* y_in, int n, int attempt, hipStream_t st) {
  hipError_t e = prepare();
  if (e != hipSuccess) return e;
  FitArgs a = make_args(P, Lo, g, obs_idx, y_in, n);
  const int NB = a.NB;
  if (attempt == 0) hipLaunchKernelGGL(k_fitL_gather, dim3(1), dim3(1024), 0, st, a);
  else hipLaunchKernelGGL(k_fitL_rearm, dim3(1), dim3(64), 0, st, P.st);
  hipLaunchKernelGGL(k_fitL_build, dim3(NB * (NB + 1) / 2), dim3(TT), 0, st, a, attempt);
  for (int k = 0; k < NB; ++k) {
    hipLaunchKernelGGL(k_fitL_A, dim3(NB), dim3(kAThreads), 3 * sizeof(Tile), st, a, k, attempt);
    if (k + 1 < NB) {
      const int m = NB - 1 - k;
      const int nb = m * (m + 1) / 2 + m * (k + 1);
      hipLaunchKernelGGL(k_fitL_B, dim3(nb), dim3(TT), 2 * sizeof(Tile), st, a, k);
    }
  }
  const int rows = a.n_pad / (TT / 64);
  hipLaunchKernelGGL(k_fitL_alpha_z, dim3(rows), dim3(TT), 0, st, a);
  hipLaunchKernelGGL(k_fitL_alpha_a, dim3(rows), dim3(TT), 0, st, a);
  hipLaunchKernelGGL(k_fitL_pack, dim3(512), dim3(TT), 0, st, a, attempt);
  return hipGetLastError();
}

}  // namespace bo
