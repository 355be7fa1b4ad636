// Surrogate fit in FP64 (Section III-B, fixed lengthscale): K_nn with the
// jitter schedule, blocked Cholesky L L^T = K_nn + delta I, explicit L^-1,
// alpha = L^-T L^-1 (y - m), and the packing of L^-1 into the operand layout
// of the posterior kernels.
//
// Dense work runs on 64 x 64 FP64 tiles, one "team" of 256 threads per tile
// (thread 64w + c owns rows 16w..16w+15 of column c).  Block step k:
//   A_k: factor the diagonal tile A_kk and invert the factor, both with the
//        tile held in registers as per-thread strips of one column (one
//        barrier per column; the pivot test decides the jitter schedule), then
//        either write the panel tile L_ik = A_ik L_kk^-T (i > k) or finalize
//        block row k of the inverse, X_kj = L_kk^-1 R_kj (j < k), X_kk;
//   B_k: trailing update A_ij -= L_ik L_jk^T (k < j <= i) and the running
//        right-hand side of the inverse R_ij -= L_ik X_kj (i > k >= j).
// Small fits: one workgroup (two teams) runs every step, jitter retries
// included.  Large fits: one launch of co-resident workgroups with grid-wide
// barriers between the steps and a look-ahead of the next diagonal tile,
// jitter retries included (k_fit.hip).
#pragma once
#include <type_traits>
#include "bo_internal.h"
#include "bo_device.h"

namespace bo {
namespace {

constexpr int T = 64;     // tile edge
constexpr int LDP = 65;   // LDS row pitch (doubles)
constexpr int TT = 256;   // threads per team

struct FitArgs {
  int n, n_pad, NB, d, nu2, tries, prec;
  int ld;  // row stride of A, L and L^-1: n_pad of n_max, fixed for the session
  double inv_l, amp, noise;
  const int64_t* obs_idx;
  const double* y_in;
  int64_t N, N_pad;
  const int32_t* inv_map;
  const double* X64;
  double* Xo64;
  uint16_t* Xo16;  // augmented FP16 observation coordinates (BF16X3 only), rows of 2 * w16
  int w16;
  double* y;
  double* A;     // working matrix, later the running right-hand side R of the inverse
  double* L;
  double* Dinv;  // inverses of the diagonal tiles of L
  double* Linv;  // X = L^-1
  double* alpha;
  double* z;
  void* Bpk;
  int64_t* obs;  // the session's copy of the observations' candidate indices
  DevState* st;
};

typedef double Tile[T][LDP];

__device__ __forceinline__ size_t tix(const FitArgs& a, int ti, int tj, int r, int c) {
  return (size_t)(ti * T + r) * a.ld + tj * T + c;
}

__device__ __forceinline__ void tri_decode(int t, int* i, int* j) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  *i = r;
  *j = t - r * (r + 1) / 2;
}

// Tile loads into LDS by a team of TT threads (tt < TT): every load of the
// thread is issued before the first store, so their latencies overlap.
__device__ __forceinline__ void load_tile(Tile& s, const double* M, const FitArgs& a, int ti, int tj, int tt) {
  constexpr int NQ = T * T / TT;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tt + q * TT;
    v[q] = M[tix(a, ti, tj, e >> 6, e & 63)];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tt + q * TT;
    s[e >> 6][e & 63] = v[q];
  }
}

__device__ __forceinline__ void load_dinv(Tile& s, const FitArgs& a, int k, int tt) {
  const double* D = a.Dinv + (size_t)k * T * T;
  constexpr int NQ = T * T / TT;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = D[tt + q * TT];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tt + q * TT;
    s[e >> 6][e & 63] = v[q];
  }
}

// ---- phase 0: gather observations, validate, prior mean and incumbent ----
// Runs in one workgroup (n <= 1024); s_red holds 2 * blockDim.x doubles and
// s_pos 1024 ints.
template <bool COORDS = true>
__device__ void fit_gather(const FitArgs& a, double* s_red, int* s_pos, int* s_bad) {
  const int t = threadIdx.x, nt = blockDim.x;
  if (t == 0) *s_bad = 0;
  __syncthreads();
  double yv = 0.0, ymin = INFINITY;
  // observations in groups of U per thread, every load of a group issued
  // before the first store (the stores could alias later loads as far as
  // the compiler knows, which would serialize the round trips)
  constexpr int U = 4;
  for (int i0 = t; i0 < a.n_pad; i0 += U * nt) {
    int64_t idx[U];
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * nt;
      idx[u] = i < a.n ? a.obs_idx[i] : -1;
      v[u] = i < a.n ? a.y_in[i] : 0.0;
    }
    int pos[U];
#pragma unroll
    for (int u = 0; u < U; ++u) pos[u] = (idx[u] >= 0 && idx[u] < a.N) ? a.inv_map[idx[u]] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * nt;
      if (i >= a.n_pad) continue;
      if (i < a.n) {
        if (pos[u] < 0 || !isfinite(v[u])) {
          atomicExch(s_bad, 1);
          pos[u] = 0;
        }
        yv += v[u];
        ymin = fmin(ymin, v[u]);
      } else {
        pos[u] = 0;
      }
      s_pos[i] = pos[u];
      a.y[i] = v[u];
      if (i < a.n) a.obs[i] = idx[u];
    }
  }
  __syncthreads();
  // coordinates: one observation per thread, its kMaxD loads issued
  // together (one round for n_pad <= blockDim.x); with COORDS false other
  // workgroups take them (gather_coords_row)
  for (int i = t; COORDS && i < a.n_pad; i += nt) {
    const bool live = i < a.n;
    const int pos = live ? s_pos[i] : 0;
    double x[kMaxD];
#pragma unroll
    for (int j = 0; j < kMaxD; ++j) x[j] = (live && j < a.d) ? a.X64[(int64_t)j * a.N_pad + pos] : 0.0;
#pragma unroll
    for (int j = 0; j < kMaxD; ++j) a.Xo64[(size_t)i * kMaxD + j] = x[j];
    if (a.Xo16) aug16_row(x, a.d, true, a.Xo16 + (size_t)i * 2 * a.w16, a.w16);
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
    st->min_piv = INFINITY;
    st->gs_arrive = 0;
    st->gs_release = 0;
    st->gs_abort = 0;
    st->fail_at = 0xffffffffu;
  }
  __syncthreads();
}

// The coordinate part of fit_gather for observation i alone, with the same
// values: its row of X in Xo64 (zeros past d and past n) and its augmented
// FP16 row for the BF16X3 distance products; an index the gather refuses
// reads row 0, as there.
__device__ __forceinline__ void gather_coords_row(const FitArgs& a, int i) {
  const bool live = i < a.n;
  int pos = 0;
  if (live) {
    const int64_t idx = a.obs_idx[i];
    const int p = (idx >= 0 && idx < a.N) ? a.inv_map[idx] : -1;
    pos = (p < 0 || !isfinite(a.y_in[i])) ? 0 : p;
  }
  double x[kMaxD];
#pragma unroll
  for (int j = 0; j < kMaxD; ++j) x[j] = (live && j < a.d) ? a.X64[(int64_t)j * a.N_pad + pos] : 0.0;
#pragma unroll
  for (int j = 0; j < kMaxD; ++j) a.Xo64[(size_t)i * kMaxD + j] = x[j];
  if (a.Xo16) aug16_row(x, a.d, true, a.Xo16 + (size_t)i * 2 * a.w16, a.w16);
}

// ---- tile operations (one team; thread tt = 64 w + lane owns rows
// 16w .. 16w+15 of column `lane`, so the lanes of a wave touch consecutive
// LDS words and the row operand is a broadcast) ----

// K_nn tile: amp * Matern(|xo_i - xo_j|) + delta on the diagonal; padded rows
// and columns form an identity block so the padded factor stays regular.
// xs holds the coordinates of row block ti (rows 0..63) and column block tj
// (rows 64..127) as [128][kMaxD + 1] doubles.
__device__ void op_build(const FitArgs& a, int ti, int tj, double delta, double* xs, int tt) {
  {
    constexpr int NQ = 128 * kMaxD / TT;
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tt + q * TT;
      const int r = e / kMaxD, j = e % kMaxD;
      const int g = (r < 64 ? ti * T + r : tj * T + r - 64);
      v[q] = a.Xo64[g * kMaxD + j];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tt + q * TT;
      xs[(e / kMaxD) * (kMaxD + 1) + e % kMaxD] = v[q];
    }
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
  }
  __syncthreads();
}

// C (global tile) = init - sign * A B^T (NT) or A B (NN), A and B in LDS;
// init is the current C when `accumulate`, else zero.  FP64 16x16x4 matrix-
// core products: wave w (thread tt = 64 w + l) computes rows 16w..16w+15 as
// four 16x16 output tiles; the A fragment of k-step t is A[16w + l%16][4t +
// l/16], the B fragment of tile j is B^T or B at [4t + l/16][16j + l%16], and
// output register i of lane l is row l/16 + 4i, column l%16.
template <bool NT>
__device__ void op_gemm(double* C, const FitArgs& a, int ti, int tj, const Tile& A, const Tile& B, bool accumulate,
                        double sign, int tt) {
  const int w = tt >> 6, l = tt & 63;
  const int r = l & 15, kq = l >> 4;
  f64x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = (f64x4){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int t = 0; t < T / 4; ++t) {
    const int kk = 4 * t + kq;
    const double av = A[16 * w + r][kk];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double bv = NT ? B[16 * j + r][kk] : B[kk][16 * j + r];
      acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[j], 0, 0, 0);
    }
  }
  // all of C's current values are read before the first store (the stores
  // could alias a later load as far as the compiler knows)
  double base[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) base[j][i] = accumulate ? C[tix(a, ti, tj, 16 * w + kq + 4 * i, 16 * j + r)] : 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) C[tix(a, ti, tj, 16 * w + kq + 4 * i, 16 * j + r)] = base[j][i] - sign * acc[j][i];
}

// Lane N of each row of 16 lanes broadcast to the whole row (DPP
// row_newbcast, a VALU move; N is a compile-time constant).
template <int N>
__device__ __forceinline__ double row_bcast_d(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + N, 0xf, 0xf, true);
}

// Row Q of v (lanes 16Q .. 16Q+15) copied to all four rows: the lane swaps
// of gfx950 (upper half with lower half, then odd rows with even rows), VALU
// moves only.
template <int Q>
__device__ __forceinline__ double row_copy_d(double v) {
  const unsigned wd[2] = {(unsigned)__double2loint(v), (unsigned)__double2hiint(v)};
  unsigned r[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // {lower half twice, upper half twice}
    const auto a = __builtin_amdgcn_permlane32_swap(wd[h], wd[h], false, false);
    const unsigned half = Q < 2 ? a[0] : a[1];
    // {even row of each pair everywhere, odd row everywhere}
    const auto b = __builtin_amdgcn_permlane16_swap(half, half, false, false);
    r[h] = (Q & 1) ? b[1] : b[0];
  }
  return __hiloint2double((int)r[1], (int)r[0]);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// 16 x 16 x 16 FP64 products of LDS blocks on the matrix cores, one wave.
// Result layout (as the 16x16x4 product leaves it): register i of lane l is
// row l/16 + 4i, column l%16.
// acc + A[ra.., ca..] * B[rb.., cb..]^T
__device__ __forceinline__ f64x4 mm16_nt(const Tile& A, int ra, int ca, const Tile& B, int rb, int cb, f64x4 acc,
                                         int lane) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[ra + (lane & 15)][ca + 4 * s + (lane >> 4)],
                                               B[rb + (lane & 15)][cb + 4 * s + (lane >> 4)], acc, 0, 0, 0);
  return acc;
}
// acc + A[ra.., ca..] * B[rb.., cb..]
__device__ __forceinline__ f64x4 mm16_nn(const Tile& A, int ra, int ca, const Tile& B, int rb, int cb, f64x4 acc,
                                         int lane) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[ra + (lane & 15)][ca + 4 * s + (lane >> 4)],
                                               B[rb + 4 * s + (lane >> 4)][cb + (lane & 15)], acc, 0, 0, 0);
  return acc;
}
// acc + A[ra.., ca..] * M, M in registers in the result layout above (its
// register s is exactly the B operand of k-step s)
__device__ __forceinline__ f64x4 mm16_nr(const Tile& A, int ra, int ca, const f64x4& M, f64x4 acc, int lane) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[ra + (lane & 15)][ca + 4 * s + (lane >> 4)], M[s], acc, 0, 0, 0);
  return acc;
}

// Diagonal tile k: Cholesky with the pivot test, then the inverse of the
// factor.  The pivots form one sequential chain, so the tile is factored by a
// single wave, blocked in 16 x 16 sub-blocks (kb = 0..3):
//  - the diagonal sub-block is held in registers (lane l: column l%16, rows
//    l/16 + 4i) and reduced by elimination without square roots (column p
//    kept as L_rp sqrt(D_pp), the square roots taken per column afterwards),
//    the values each step needs passed between lanes (within a row of 16
//    lanes by DPP broadcasts, across rows through the LDS crossbar or the
//    lane swaps); its inverse follows through the unit factor
//    L diag(L)^-1, row by row;
//  - the panel L_ib = A_ib L_bb^-T and the trailing update
//    A_ij -= L_ib L_jb^T are 16x16x16 FP64 matrix-core products, one per
//    wave and phase;
//  - the off-diagonal inverse blocks X_ij = -X_ii sum_m L_im X_mj, i > j.
// With `pre` (k > 0) the tile's last trailing update of the blocked
// factorization, A_kk -= L_k,k-1 L_k,k-1^T, is applied in LDS first (pre
// stages L_k,k-1), in the order of the matrix-core steps of op_gemm, so the
// tile is the one a separate trailing-update launch would have left.
// The pivot test: a pivot of a row below n must exceed n eps (amp + delta)
// and be finite (padding rows: positive).  The factor (zeros above the
// diagonal) is left in s1 and its inverse in s0.  Returns true when a pivot
// fails, in every thread; *pmin takes the smallest pivot of the rows below n.
template <int NT>
__device__ bool op_diag(const FitArgs& a, int k, double delta, Tile& s0, Tile& s1, double (*colbuf)[64],
                        double (*xbuf)[64], double* pmin, Tile* pre = nullptr) {
  const int tt = threadIdx.x;
  {
    constexpr int NQ = T * T / NT;
    double v[NQ], lv[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tt + q * NT;
      v[q] = a.A[tix(a, k, k, e >> 6, e & 63)];
      if (pre) lv[q] = a.L[tix(a, k, k - 1, e >> 6, e & 63)];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tt + q * NT;
      s1[e >> 6][e & 63] = v[q];
      if (pre) (*pre)[e >> 6][e & 63] = lv[q];
    }
  }
  __syncthreads();
  static_assert(NT >= 6 * 64, "one wave per trailing product");
  const int wv = uni(tt >> 6), lane = tt & 63, g = lane >> 4, c = lane & 15;
  if (pre) {
    // the ten lower 16 x 16 blocks, spread over the waves
    for (int blk = wv; blk < 10; blk += NT / 64) {
      int ib, jb;
      tri_decode(blk, &ib, &jb);
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = mm16_nt(*pre, 16 * ib, 16 * kk, *pre, 16 * jb, 16 * kk, acc, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double& t = s1[16 * ib + g + 4 * i][16 * jb + c];
        t = t - acc[i];
      }
    }
    __syncthreads();
  }
  const double thr = (double)a.n * 2.220446049250313e-16 * (a.amp + delta);
  bool bad = false;  // wave 0
  double pm = INFINITY;
#pragma unroll 1
  for (int kb = 0; kb < 4; ++kb) {
    const int o = 16 * kb;
    if (wv == 0) {
      // the sub-block from its lower triangle (the upper one is stale)
      double d[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = g + 4 * i;
        d[i] = r >= c ? s1[o + r][o + c] : s1[o + c][o + r];
      }
      // Elimination without square roots: step p subtracts D_rp D_pc / D_pp
      // from every column c > p (rows at or above p become rounding noise
      // above the diagonal, cleared below) and keeps column p, so that
      // column p ends as L_rp sqrt(D_pp) with D_pp the p-th pivot.  D_rp
      // comes from lane p of the lane's row, D_pc from row p of the lane's
      // column; only a reciprocal lies on the chain from pivot to pivot.
      double pcol = 1.0;  // the pivot of the lane's column
      auto step = [&](auto pc) {
        constexpr int p = decltype(pc)::value;
        const double piv = readlane_d(d[p >> 2], 16 * (p & 3) + p);
        // D_pc: row p of the lane's column (an LDS-crossbar read whose
        // latency the reciprocal's refinement covers)
        const double dpc = __shfl(d[p >> 2], 16 * (p & 3) + c, 64);
        double rp = __builtin_amdgcn_rcp(piv);
        double e = fma(-piv, rp, 1.0);
        rp = fma(rp, e, rp);
        e = fma(-piv, rp, 1.0);
        rp = fma(rp, e, rp);
        const double nw = c > p ? -(dpc * rp) : 0.0;
        pcol = c == p ? piv : pcol;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * i + 3 >= p) d[i] = fma(row_bcast_d<p>(d[i]), nw, d[i]);
      };
      step(std::integral_constant<int, 0>());
      step(std::integral_constant<int, 1>());
      step(std::integral_constant<int, 2>());
      step(std::integral_constant<int, 3>());
      step(std::integral_constant<int, 4>());
      step(std::integral_constant<int, 5>());
      step(std::integral_constant<int, 6>());
      step(std::integral_constant<int, 7>());
      step(std::integral_constant<int, 8>());
      step(std::integral_constant<int, 9>());
      step(std::integral_constant<int, 10>());
      step(std::integral_constant<int, 11>());
      step(std::integral_constant<int, 12>());
      step(std::integral_constant<int, 13>());
      step(std::integral_constant<int, 14>());
      step(std::integral_constant<int, 15>());
      // pivot test of the lane's column (every lane of a column holds its
      // pivot), reduced over the wave: off the pivot-to-pivot chain
      {
        const int R = k * T + o + c;
        const bool fails = !(pcol > (R < a.n ? thr : 0.0)) || !(pcol < INFINITY);
        bad |= __ballot(fails) != 0;
        double mn = R < a.n ? pcol : INFINITY;
        for (int off = 1; off < 16; off <<= 1) mn = fmin(mn, __shfl_xor(mn, off, 64));
        pm = fmin(pm, mn);
      }
      // sqrt(pivot) and 1 / sqrt(pivot) of the lane's column: hardware
      // reciprocal square root, two Goldschmidt steps, a Newton correction
      // of each
      double h = 0.5 * __builtin_amdgcn_rsq(pcol), q = 2.0 * h * pcol;
      double e = fma(-h, q, 0.5);
      q = fma(q, e, q);
      h = fma(h, e, h);
      e = fma(-h, q, 0.5);
      q = fma(q, e, q);
      h = fma(h, e, h);
      const double sq = fma(fma(-q, q, pcol), h, q);
      double y = 2.0 * h;
      y = fma(y, fma(-sq, y, 1.0), y);
      // L_rc = D_rc / sqrt(D_cc) below the diagonal, sqrt(D_cc) on it; the
      // unit factor U = L diag(L)^-1 (diagonal left at zero: never used)
      double u[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = g + 4 * i;
        const double lv = d[i] * y;
        d[i] = r > c ? lv : (r == c ? sq : 0.0);
        u[i] = r > c ? lv * y : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) s1[o + g + 4 * i][o + c] = d[i];
      // Z = U^-1 by rows: once row r of Z is final, every row m takes away
      // U_mr Z_r (rows at or above r meet a zero of U); then
      // L^-1 = diag(1 / L_rr) Z.  Row r of Z comes from row r%4, register
      // r/4; U_mr from lane r of the lane's row.
      double z[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) z[i] = g + 4 * i == c ? 1.0 : 0.0;
      auto istep = [&](auto rc) {
        constexpr int r = decltype(rc)::value;
        const double zr = row_copy_d<r & 3>(z[r >> 2]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * i + 3 > r) z[i] = fma(-row_bcast_d<r>(u[i]), zr, z[i]);
      };
      istep(std::integral_constant<int, 0>());
      istep(std::integral_constant<int, 1>());
      istep(std::integral_constant<int, 2>());
      istep(std::integral_constant<int, 3>());
      istep(std::integral_constant<int, 4>());
      istep(std::integral_constant<int, 5>());
      istep(std::integral_constant<int, 6>());
      istep(std::integral_constant<int, 7>());
      istep(std::integral_constant<int, 8>());
      istep(std::integral_constant<int, 9>());
      istep(std::integral_constant<int, 10>());
      istep(std::integral_constant<int, 11>());
      istep(std::integral_constant<int, 12>());
      istep(std::integral_constant<int, 13>());
      istep(std::integral_constant<int, 14>());
#pragma unroll
      for (int i = 0; i < 4; ++i) s0[o + g + 4 * i][o + c] = z[i] * __shfl(y, g + 4 * i, 64);
    }
    __syncthreads();
    // panel: wave w forms L_ib,kb = A_ib,kb X_kb,kb^T for ib = kb + 1 + w
    {
      const int ib = kb + 1 + wv;
      if (ib < 4) {
        const f64x4 lb = mm16_nt(s1, 16 * ib, o, s0, o, o, (f64x4){0.0, 0.0, 0.0, 0.0}, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i) s1[16 * ib + g + 4 * i][o + c] = lb[i];
      }
    }
    __syncthreads();
    // trailing update: wave w takes the w-th block (ib, jb), kb < jb <= ib
    {
      const int m = 3 - kb;  // blocks after kb
      if (wv < m * (m + 1) / 2) {
        int jb = 0, ib = 0, u = wv;
        for (int q = 0; q < m; ++q) {
          if (u < m - q) {
            jb = kb + 1 + q;
            ib = jb + u;
            break;
          }
          u -= m - q;
        }
        const f64x4 upd = mm16_nt(s1, 16 * ib, o, s1, 16 * jb, o, (f64x4){0.0, 0.0, 0.0, 0.0}, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          double& t = s1[16 * ib + g + 4 * i][16 * jb + c];
          t -= upd[i];
        }
      }
    }
    __syncthreads();
  }
  // X_ij = -X_ii sum_{m=j}^{i-1} L_im X_mj, block row by block row; wave w
  // takes block column jb = w
  for (int ib = 1; ib < 4; ++ib) {
    const int jb = wv;
    if (jb < ib) {
      f64x4 t = {0.0, 0.0, 0.0, 0.0};
      for (int m = jb; m < ib; ++m) t = mm16_nn(s1, 16 * ib, 16 * m, s0, 16 * m, 16 * jb, t, lane);
      const f64x4 xi = mm16_nr(s0, 16 * ib, 16 * ib, t, (f64x4){0.0, 0.0, 0.0, 0.0}, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i) s0[16 * ib + g + 4 * i][16 * jb + c] = -xi[i];
    }
    __syncthreads();
  }
  // zeros above the diagonal blocks: wave w < 6 clears the w-th upper block
  if (wv < 6) {
    const int ib = wv < 3 ? 0 : (wv < 5 ? 1 : 2);
    const int jb = wv < 3 ? wv + 1 : (wv < 5 ? wv - 1 : 3);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s0[16 * ib + g + 4 * i][16 * jb + c] = 0.0;
      s1[16 * ib + g + 4 * i][16 * jb + c] = 0.0;
    }
  }
  if (tt == 0) {
    xbuf[0][0] = bad ? 1.0 : 0.0;
    xbuf[0][1] = pm;
  }
  __syncthreads();
  const bool fail = xbuf[0][0] != 0.0;
  const double pmv = xbuf[0][1];
  __syncthreads();
  if (fail) return true;
  *pmin = fmin(*pmin, pmv);
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
// z = L^-1 (y - m) and alpha = L^-T z, one row per wave; rows and columns at
// or beyond n are never read (they may hold another fit's values).
__device__ void alpha_z_row(const FitArgs& a, int i, double m, int lane) {
  double v = 0.0;
  if (i < a.n)
#pragma unroll 4
    for (int j = lane; j <= i; j += 64) v += a.Linv[(size_t)i * a.ld + j] * (a.y[j] - m);
  v = wave_sum_d(v);
  if (lane == 0) a.z[i] = v;
}
__device__ void alpha_a_row(const FitArgs& a, int i, int lane) {
  double v = 0.0;
#pragma unroll 4
  for (int j = i + lane; j < a.n; j += 64) v += a.Linv[(size_t)j * a.ld + i] * a.z[j];
  v = wave_sum_d(v);
  if (lane == 0) a.alpha[i] = i < a.n ? v : 0.0;
}

// z in one workgroup (n_pad <= 256): each wave takes four of its rows at a
// time and issues all their loads before the first reduction, so a wave
// waits once per four rows instead of once per row.  Every lane sums its
// terms in the order of alpha_z_row and the reduction is the same, so the
// results are the same bits.
// out(i, sum_{j <= i} Linv[i][j] src(j)) for the rows i < ni of the wave
// (zero for rows at or beyond nv), four at a time (z = L^-1 (y - m); also
// L^-1 k in an append)
template <typename Src, typename Out>
__device__ __forceinline__ void l_rows_block(const FitArgs& a, int ni, int nv, Src src, Out out, int wave, int NW, int lane) {
  constexpr int R = 4;  // rows of a wave in flight together
  for (int i0 = wave; i0 < ni; i0 += R * NW) {
    double v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = 0.0;
#pragma unroll
    for (int c = 0; c < kSmallFitMax / 64; ++c) {
      const int j = 64 * c + lane;
      if (64 * c < ni) {
        // the source at a clamped index (a load behind a branch is waited
        // for before the branch joins)
        const double xv = src(j < nv ? j : nv - 1);
        const double x = j < nv ? xv : 0.0;
        double l[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = i0 + r * NW;
          l[r] = (i < nv && j <= i) ? a.Linv[(size_t)i * a.ld + j] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = i0 + r * NW;
          if (i < nv && j <= i) v[r] += l[r] * x;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = wave_sum_d(v[r]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + r * NW;
      if (i < ni) out(i, v[r]);
    }
  }
}


// l_rows_block for two source vectors at once over the same rows (one pass
// over L^-1); each lane sums its products as l_rows_block does, and the lane
// partials are added by wave_sum_d.
template <typename Src1, typename Src2, typename Out>
__device__ __forceinline__ void l_rows_block2(const FitArgs& a, int ni, int nv, Src1 src1, Src2 src2, Out out,
                                              int wave, int NW, int lane) {
  constexpr int R = 4;
  for (int i0 = wave; i0 < ni; i0 += R * NW) {
    double v[R], u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = u[r] = 0.0;
#pragma unroll
    for (int c = 0; c < kSmallFitMax / 64; ++c) {
      const int j = 64 * c + lane;
      if (64 * c < ni) {
        // the sources at a clamped index, so that their loads sit behind no
        // branch (a load behind one is waited for before the branch joins)
        const int jc = j < nv ? j : nv - 1;
        const double xv = src1(jc), yv = src2(jc);
        const double x = j < nv ? xv : 0.0;
        const double y = j < nv ? yv : 0.0;
        double l[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = i0 + r * NW;
          l[r] = (i < nv && j <= i) ? a.Linv[(size_t)i * a.ld + j] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = i0 + r * NW;
          if (i < nv && j <= i) {
            v[r] += l[r] * x;
            u[r] += l[r] * y;
          }
        }
      }
    }
    // the eight wave sums first (independent chains), then the outputs
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = wave_sum_d(v[r]);
      u[r] = wave_sum_d(u[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + r * NW;
      if (i < ni) out(i, v[r], u[r]);
    }
  }
}

// out(i, sum_{i <= j < nj} Linv[j][i] src(j)) for the columns i < ni <= 256
// of L^-T src (alpha = L^-T z; also l^T L^-1 in an append), two threads per
// column (a workgroup of 512): thread (i, h) sums the rows j = i + h, i + h + 2,
// ... in ascending order, reading row j's entries of consecutive columns
// together (coalesced); the odd rows' sum is then added to the even rows'.
// s_part: 256 doubles of LDS.  The one-workgroup fit, the append and the
// multi-workgroup fit's alpha (n_pad <= 256) all take this order, so their
// alphas are the same bits.
template <typename Src, typename Out>
__device__ __forceinline__ void lt_cols_pair(const FitArgs& a, int ni, int nj, Src src, Out out, double* s_part) {
  const int t = threadIdx.x, i = t & 255, h = t >> 8;
  double v = 0.0;
  if (i < ni) {
#pragma unroll 8
    for (int j = i + h; j < nj; j += 2) v += a.Linv[(size_t)j * a.ld + i] * src(j);
  }
  if (h) s_part[i] = v;
  __syncthreads();
  if (!h && i < ni) out(i, v + s_part[i]);
  __syncthreads();
}

// ---- packing of L^-1 for the matrix-core posterior kernels ----
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ double linv_at(const FitArgs& a, int row, int col) {
  return (col <= row && row < a.n && col < a.n) ? a.Linv[(size_t)row * a.ld + col] : 0.0;
}

// FP64 / FP32, 16x16x4 operand: fragment (J, t) at 2J(J+1) + t, t <= 4J+3;
// lane l holds L^-1[16J + l%16][4t + l/16] (the transpose, as the B operand).
// FP64 values: the posterior of both modes takes FP64 products.
__device__ __forceinline__ bool pack_f64(const FitArgs& a) { return a.prec != BO_BF16X3; }

__device__ void pack_elem16(const FitArgs& a, int64_t e) {
  const int64_t f = e >> 6;
  const int l = (int)(e & 63);
  int J = (int)((sqrt(2.0 * (double)f + 1.0) - 1.0) * 0.5);
  while (2LL * (J + 1) * (J + 2) <= f) ++J;
  while (2LL * J * (J + 1) > f) --J;
  const int t = (int)(f - 2LL * J * (J + 1));
  const double v = linv_at(a, 16 * J + (l & 15), 4 * t + (l >> 4));
  if (pack_f64(a)) ((double*)a.Bpk)[e] = v;
  else ((float*)a.Bpk)[e] = (float)v;
}

// BF16X3, 32x32x16 operand.  Column block J (32 columns of L^-T) has nonzero
// k-steps t <= 2J+1 (16 observations each); it is stored with 4(J/2 + 1)
// fragments, a whole number of 64-observation chunks, the extra ones zero:
// block J starts at fragment 4m(m+1) (J = 2m) or 4(m+1)^2 (J = 2m+1).  Lane
// l of fragment (J, t) holds 8 values L^-1[32J + l%32][16t + 8(l/32) + e];
// high parts first, then the low parts (value - high) in a second array of
// the same shape.
__device__ __forceinline__ int64_t frag32_base(int J) {
  const int64_t m = J >> 1;
  return (J & 1) ? 4 * (m + 1) * (m + 1) : 4 * m * (m + 1);
}

__device__ void pack_elem32(const FitArgs& a, int64_t e, int64_t nfrag) {
  const int64_t f = e >> 6;
  const int l = (int)(e & 63);
  // block pair m covers fragments [4m(m+1), 4(m+1)(m+2))
  int64_t m = (int64_t)((sqrt((double)f + 1.0) - 1.0) * 0.5);
  while (4 * (m + 1) * (m + 2) <= f) ++m;
  while (4 * m * (m + 1) > f) --m;
  const int64_t u = f - 4 * m * (m + 1);
  const int J = (int)(2 * m + (u >= 4 * (m + 1) ? 1 : 0));
  const int t = (int)(f - frag32_base(J));
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
    const int64_t M = a.n_pad / 64;  // block pairs
    *nfrag = 4 * M * (M + 1);
  } else {
    const int64_t JB = a.n_pad / 16;
    *nfrag = 2 * JB * (JB + 1);
  }
  return *nfrag * 64;
}

// ======================= small fit: one workgroup =========================
constexpr int kSmallThreads = 2 * TT;
constexpr int NTEAM = kSmallThreads / TT;

// The whole fit of n <= 256 observations by one workgroup of kSmallThreads
// threads: gather, build, factor and invert with the jitter schedule, alpha
// and the packed operand.  s_raw: kSmallLdsBytes of LDS.
__device__ __forceinline__ void fit_small_run(const FitArgs& a, unsigned char* s_raw) {
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
  double pmin = INFINITY;
  for (attempt = 0; attempt < a.tries; ++attempt) {
    delta = jitter_of(a.noise, a.amp, attempt);
    pmin = INFINITY;
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
      fail = op_diag<kSmallThreads>(a, k, delta, tiles[0], tiles[1], s_colbuf, s_xbuf, &pmin);
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
  l_rows_block(
      a, a.n_pad, a.n, [&](int j) { return a.y[j] - m; },
      [&](int i, double v) {
        if (lane == 0) a.z[i] = v;
      },
      wave, nwave, lane);
  __syncthreads();
  lt_cols_pair(
      a, a.n_pad, a.n, [&](int j) { return a.z[j]; }, [&](int i, double v) { a.alpha[i] = i < a.n ? v : 0.0; },
      s_red);
  int64_t nfrag;
  const int64_t ne = pack_count(a, &nfrag);
  for (int64_t e = threadIdx.x; e < ne; e += kSmallThreads) {
    if (a.prec == BO_BF16X3) pack_elem32(a, e, nfrag);
    else pack_elem16(a, e);
  }
  if (threadIdx.x == 0) {
    a.st->jitter = delta;
    a.st->attempt = attempt;
    a.st->min_piv = pmin;
    a.st->status = BO_OK;
  }
}

// Bordered (rank-1) append of one observation, n0 -> n0 + 1 = a.n, to the
// session's current factor (Section III-B: the surrogate is refit after each
// new observation).  With k the covariances of the new point to the old ones,
// l = L^-1 k and d^2 = amp + delta - |l|^2:
//     L' = [L 0; l^T d],   L'^-1 = [L^-1 0; -(l^T L^-1) / d  1/d],
// so only a new row of L and of L^-1 is written, alpha is recomputed in
// O(n^2) and only the column blocks of the packed operand that hold row n0
// are rewritten.  The new observation must already be at position n0 of
// a.obs_idx / a.y_in.  When the current fit is not a valid fit of n0 points,
// or a pivot (the new one, or the smallest old one) fails the test of an
// (n0 + 1)-point factorization, the whole fit is redone by fit_small_run,
// jitter schedule included: the result is then the refit's by construction.
// One workgroup of kSmallThreads threads, n <= 256; s_raw: kSmallLdsBytes.
__device__ __forceinline__ void append_run(const FitArgs& a, unsigned char* s_raw) {
  __shared__ int s_mode;  // 0: append, 1: refit, 2: bad observation
  __shared__ int s_pos0;
  double* s_k = reinterpret_cast<double*>(s_raw);    // [256]
  double* s_l = s_k + kSmallFitMax;                  // [256]
  double* s_red = s_l + kSmallFitMax;                // [2 * kSmallThreads]
  const int t = threadIdx.x, nt = blockDim.x;
  const int lane = t & 63, wave = t >> 6, nwave = nt >> 6;
  const int n0 = a.n - 1;
  DevState* st = a.st;
  if (t == 0) {
    int mode = 0;
    const int64_t idx = a.obs_idx[n0];
    const double v = a.y_in[n0];
    const int pos = (idx >= 0 && idx < a.N) ? a.inv_map[idx] : -1;
    if (pos < 0 || !isfinite(v)) mode = 2;
    else if (n0 < 1 || st->status != BO_OK || st->n != n0 || a.prec == BO_BF16X3) mode = 1;
    s_mode = mode;
    s_pos0 = pos < 0 ? 0 : pos;
  }
  __syncthreads();
  if (s_mode == 1) {
    fit_small_run(a, s_raw);
    return;
  }
  if (s_mode == 2) {
    if (t == 0) {
      st->status = BO_E_INVALID_ARG;
      st->n = a.n;
    }
    return;
  }
  const double delta = st->jitter;
  if (t < kMaxD) {
    const double x = t < a.d ? a.X64[(int64_t)t * a.N_pad + s_pos0] : 0.0;
    a.Xo64[(size_t)n0 * kMaxD + t] = x;
  }
  if (a.Xo16 && t == 0) {
    double x[kMaxD];
    for (int j = 0; j < a.d; ++j) x[j] = a.X64[(int64_t)j * a.N_pad + s_pos0];
    aug16_row(x, a.d, true, a.Xo16 + (size_t)n0 * 2 * a.w16, a.w16);
  }
  if (t == 0) {
    a.y[n0] = a.y_in[n0];
    a.obs[n0] = a.obs_idx[n0];
  }
  __syncthreads();
  // covariances of the new point to the old ones
  for (int i = t; i < n0; i += nt) {
    double s2 = 0.0;
    for (int j = 0; j < a.d; ++j) {
      const double df = a.Xo64[(size_t)n0 * kMaxD + j] - a.Xo64[(size_t)i * kMaxD + j];
      s2 += df * df;
    }
    s_k[i] = a.amp * matern64(a.nu2, sqrt(s2), a.inv_l);
  }
  __syncthreads();
  // mean and incumbent over all observations, in the reduction order of fit_gather
  s_red[t] = t < a.n ? a.y[t] : 0.0;
  s_red[nt + t] = t < a.n ? a.y[t] : INFINITY;
  __syncthreads();
  for (int off = nt / 2; off > 0; off >>= 1) {
    if (t < off) {
      s_red[t] += s_red[t + off];
      s_red[nt + t] = fmin(s_red[nt + t], s_red[nt + t + off]);
    }
    __syncthreads();
  }
  const double m = s_red[0] / (double)a.n;
  const double fb = s_red[nt];
  __syncthreads();
  // one pass over the old rows of L^-1: l = L^-1 k and the old rows of
  // z = L^-1 (y - m) (rows < n0 keep their entries in the new factor)
  l_rows_block2(
      a, n0, n0, [&](int j) { return s_k[j]; }, [&](int j) { return a.y[j] - m; },
      [&](int i, double v, double u) {
        if (lane == 0) {
          s_l[i] = v;
          a.z[i] = u;
        }
      },
      wave, nwave, lane);
  __syncthreads();
  // new pivot d^2 = amp + delta - |l|^2 (fixed-order tree)
  s_red[t] = t < n0 ? s_l[t] * s_l[t] : 0.0;
  __syncthreads();
  for (int off = nt / 2; off > 0; off >>= 1) {
    if (t < off) s_red[t] += s_red[t + off];
    __syncthreads();
  }
  const double piv = (a.amp + delta) - s_red[0];
  const double thr = (double)a.n * 2.220446049250313e-16 * (a.amp + delta);
  const bool ok = piv > thr && piv < INFINITY && st->min_piv > thr;
  __syncthreads();
  if (!ok) {
    fit_small_run(a, s_raw);
    return;
  }
  const double dg = sqrt(piv);
  const double inv_dg = 1.0 / dg;
  // new rows: L[n0] = (l, d), L^-1[n0] = (-(l^T L^-1) / d, 1 / d)
  lt_cols_pair(
      a, n0 + 1, n0, [&](int j) { return s_l[j]; },
      [&](int i, double w) {
        a.L[(size_t)n0 * a.ld + i] = i < n0 ? s_l[i] : dg;
        a.Linv[(size_t)n0 * a.ld + i] = i < n0 ? -w * inv_dg : inv_dg;
      },
      s_red);
  if (t == 0) {
    st->n = a.n;
    st->mean_y = m;
    st->f_best = fb;
    st->min_piv = fmin(st->min_piv, piv);
  }
  __threadfence_block();
  __syncthreads();
  // z's new row, each lane's terms and the reduction in the order of
  // l_rows_block, and zeros past it
  if (wave == 0) {
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < kSmallFitMax / 64; ++c) {
      const int j = 64 * c + lane;
      if (j <= n0) v += a.Linv[(size_t)n0 * a.ld + j] * (a.y[j] - m);
    }
    v = wave_sum_d(v);
    if (lane == 0) a.z[n0] = v;
  }
  if (t > n0 && t < a.n_pad) a.z[t] = 0.0;
  __syncthreads();
  lt_cols_pair(
      a, a.n_pad, a.n, [&](int j) { return a.z[j]; }, [&](int i, double v) { a.alpha[i] = i < a.n ? v : 0.0; },
      s_red);
  // packed operand: the column blocks from the one holding row n0 on (the
  // fragment order does not depend on n for the 16x16x4 layout)
  const int J0 = n0 / 16, JB = a.n_pad / 16;
  const int64_t e0 = (int64_t)2 * J0 * (J0 + 1) * 64, e1 = (int64_t)2 * JB * (JB + 1) * 64;
  for (int64_t e = e0 + t; e < e1; e += nt) pack_elem16(a, e);
  __syncthreads();
}

constexpr size_t kSmallLdsBytes = 4 * sizeof(Tile) + 2 * kSmallThreads * sizeof(double);

inline FitArgs make_args(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                  const double* y_in, int n) {
  FitArgs a{};
  a.n = n;
  a.n_pad = n_pad_of(n);
  a.NB = a.n_pad / T;
  a.ld = Lo.n_max_pad;
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
  a.Xo16 = P.Xo16;
  a.w16 = Lo.w16;
  a.y = P.y;
  a.A = P.A;
  a.L = P.L;
  a.Dinv = P.Dinv;
  a.Linv = P.Linv;
  a.alpha = P.alpha;
  a.z = P.z;
  a.Bpk = P.Bpk;
  a.obs = P.obs;
  a.st = P.st;
  return a;
}

}  // namespace
}  // namespace bo
