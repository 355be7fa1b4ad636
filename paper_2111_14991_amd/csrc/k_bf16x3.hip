// Posterior of the BF16X3 precision mode (exhaustive prediction, Section
// III-G) on the bfloat16 matrix cores.
//
// Persistent kernel: each workgroup of 8 waves loops over tiles of 64
// compacted candidates, with the observation coordinates and alpha parked in
// LDS once.  For a tile the observations are streamed in chunks of 64: all
// 512 threads generate the FP32 cross-covariance k* = amp Matern(|x_c - x_i|)
// (one candidate and 8 consecutive observations per thread), add k* alpha to
// an FP64 running mean, split each value into a bfloat16 high part and a
// bfloat16 remainder, and park both in LDS in the A-operand order of the
// 32x32x16 product.  The buffers are double-buffered and the generation of
// the next chunk is interleaved with the products of the current one.  Each
// wave owns up to four 32-column blocks of W = K* L^-T (blocks w, w+8, w+16,
// w+24) for all 64 candidates and accumulates hi*hi + hi*lo + lo*hi in FP32,
// skipping the all-zero tiles above the diagonal; its L^-1 fragments are
// issued ahead of the generation work of the same k-step.  The squared column sums are combined across
// waves in a fixed order, var = amp - sum |W_c|^2 is clamped at zero, and the
// tile's mean-variance partial goes to the tile's slot.
#include "bo_internal.h"
#include "bo_device.h"
#include "post_common.h"

namespace bo {
namespace {

constexpr int kRows = 64;
constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kChunk = 64;  // observations per LDS chunk (4 k-steps of 16)
constexpr int kXoStride = kMaxD;  // floats per observation in LDS

__device__ __forceinline__ uint32_t bf16_bits_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) {
  union {
    uint4 u;
    bf16x8 b;
  } c;
  c.u = v;
  return c.b;
}

struct __align__(16) ChunkBuf {
  uint4 a[2][2][4][64];  // [hi/lo][row group][k-step][lane]
};

struct __align__(16) Smem {
  ChunkBuf buf[2];
  float xo[kMaxN * kXoStride];
  double alpha[kMaxN];
  float sq[kWaves][kRows];
  double mu[kRows];
  double rsum[kThreads];
  int64_t rcnt[kThreads];
  int last;
};

template <int D>
__global__ __launch_bounds__(kThreads) void k_post_bf16x3(PostArgs p, int ntiles) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  Smem& S = *reinterpret_cast<Smem*>(s_raw);

  if (p.st->status != BO_OK) return;
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int JB = p.n_pad >> 5;
  const int NC = p.n_pad / kChunk;
  const float inv_l = (float)p.inv_l, amp = (float)p.amp;
  const double mean_y = p.st->mean_y;

  // observations and alpha into LDS (padded observations: far away, alpha 0)
  for (int e = tid; e < p.n_pad * kXoStride; e += kThreads) {
    const int i = e / kXoStride, j = e % kXoStride;
    S.xo[e] = (i < p.n && j < D) ? p.Xo32[(size_t)i * kMaxD + j] : 0.f;
  }
  for (int i = tid; i < p.n_pad; i += kThreads) S.alpha[i] = i < p.n ? p.alpha[i] : 0.0;

  const int gr = tid >> 3, gg = tid & 7;
  const int g_rg = gr >> 5, g_s = gg >> 1, g_lane = (gr & 31) + 32 * (gg & 1);
  const uint4* Bhi = (const uint4*)p.Bpk;
  const int64_t nfrag = (int64_t)JB * (JB + 1);
  const uint4* Blo = Bhi + nfrag * 64;

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row_base = (int64_t)tile * kRows;
    const int64_t grow = row_base + gr;
    float xr[D];
#pragma unroll
    for (int j = 0; j < D; ++j) xr[j] = j < p.d ? p.X32[(int64_t)j * p.N_pad + grow] : 0.f;
    double mu_acc = 0.0;

    // generate elements e0, e0 + 1 of this thread's 8 for chunk c and store
    // their bfloat16 high and low parts into buffer b
    auto gen2 = [&](int c, int e0, ChunkBuf& b) {
      uint32_t h2 = 0, l2 = 0;
#pragma unroll
      for (int e = e0; e < e0 + 2; ++e) {
        const int i = c * kChunk + 8 * gg + e;
        const float* xo = S.xo + i * kXoStride;
        float r2 = 0.f;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const float df = xr[j] - xo[j];
          r2 = fmaf(df, df, r2);
        }
        const float kv = i < p.n ? amp * matern32_r2(p.nu2, r2, inv_l) : 0.f;
        mu_acc += (double)kv * S.alpha[i];
        const uint32_t hb = bf16_bits_rne(kv);
        const uint32_t lb = bf16_bits_rne(kv - __uint_as_float(hb << 16));
        h2 |= hb << (16 * (e - e0));
        l2 |= lb << (16 * (e - e0));
      }
      reinterpret_cast<uint32_t*>(&b.a[0][g_rg][g_s][g_lane])[e0 >> 1] = h2;
      reinterpret_cast<uint32_t*>(&b.a[1][g_rg][g_s][g_lane])[e0 >> 1] = l2;
    };

    f32x16 acc[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int rg = 0; rg < 2; ++rg)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[q][rg][i] = 0.f;

    __syncthreads();  // LDS tables ready; previous tile done with the buffers
    gen2(0, 0, S.buf[0]);
    gen2(0, 2, S.buf[0]);
    gen2(0, 4, S.buf[0]);
    gen2(0, 6, S.buf[0]);
    __syncthreads();

    for (int c = 0; c < NC; ++c) {
      const ChunkBuf& cur = S.buf[c & 1];
      ChunkBuf& nxt = S.buf[(c + 1) & 1];
      const bool more = c + 1 < NC;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int t = 4 * c + s;
        // L^-1 fragments of this k-step first (always in bounds: f < nfrag),
        // then the generation work, then the products
        uint4 bh[4], bl[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int J = w + kWaves * q;
          const int Jc = J < JB ? J : 0;
          const int64_t f = (int64_t)Jc * (Jc + 1) + t;
          bh[q] = Bhi[f * 64 + lane];
          bl[q] = Blo[f * 64 + lane];
        }
        if (more) gen2(c + 1, 2 * s, nxt);
        const bf16x8 ah0 = as_bf16x8(cur.a[0][0][s][lane]);
        const bf16x8 ah1 = as_bf16x8(cur.a[0][1][s][lane]);
        const bf16x8 al0 = as_bf16x8(cur.a[1][0][s][lane]);
        const bf16x8 al1 = as_bf16x8(cur.a[1][1][s][lane]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int J = w + kWaves * q;
          if (J < JB && t <= 2 * J + 1) {
            const bf16x8 h = as_bf16x8(bh[q]);
            const bf16x8 l = as_bf16x8(bl[q]);
            acc[q][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, h, acc[q][0], 0, 0, 0);
            acc[q][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, h, acc[q][1], 0, 0, 0);
            acc[q][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, l, acc[q][0], 0, 0, 0);
            acc[q][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, l, acc[q][1], 0, 0, 0);
            acc[q][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al0, h, acc[q][0], 0, 0, 0);
            acc[q][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al1, h, acc[q][1], 0, 0, 0);
          }
        }
      }
      __syncthreads();
    }

    // squared column sums; output register i of lane L holds row
    // 8(i/4) + 4(L/32) + i%4 of the row group, column L%32
#pragma unroll
    for (int rg = 0; rg < 2; ++rg) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        float v = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) v = fmaf(acc[q][rg][i], acc[q][rg][i], v);
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        v += __shfl_xor(v, 16, 64);
        if ((lane & 31) == 0) S.sq[w][32 * rg + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3)] = v;
      }
    }
    mu_acc += shfl_xor_d(mu_acc, 1);
    mu_acc += shfl_xor_d(mu_acc, 2);
    mu_acc += shfl_xor_d(mu_acc, 4);
    if (gg == 0) S.mu[gr] = mu_acc;
    __syncthreads();

    if (tid < 64) {
      const int64_t row = row_base + tid;
      double part = 0.0;
      int64_t cnt = 0;
      if (row < p.n_valid) {
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < kWaves; ++i) sum += (double)S.sq[i][tid];
        double v = p.amp - sum;
        v = v > 0.0 ? v : 0.0;
        const float vf = (float)v;
        ((float*)p.var)[row] = vf;
        ((float*)p.mu)[row] = (float)(mean_y + S.mu[tid]);
        if (!(p.visited && p.visited[p.orig[row]])) {
          part = (double)vf;
          cnt = 1;
        }
      }
      // fixed-order tile sum within the first wave
      for (int off = 32; off > 0; off >>= 1) {
        part += __shfl_down(part, off, 64);
        cnt += __shfl_down(cnt, off, 64);
      }
      if (tid == 0) {
        p.vslots[tile].sum = part;
        p.vslots[tile].count = cnt;
      }
    }
  }
  if (last_block(&p.st->ticket_post, &S.last)) finish_lambda(p, ntiles, S.rsum, S.rcnt);
}

template <int D>
hipError_t launch_d(const PostArgs& a, hipStream_t st) {
  static int grid = 0;
  const size_t lds = sizeof(Smem);
  if (grid == 0) {
    hipError_t e = hipFuncSetAttribute((const void*)k_post_bf16x3<D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_post_bf16x3<D>, kThreads, lds);
    if (e != hipSuccess) return e;
    grid = cus * (per > 0 ? per : 1);
  }
  const int ntiles = (int)((a.n_valid + kRows - 1) / kRows);
  const int g = ntiles < grid ? ntiles : grid;
  hipLaunchKernelGGL(k_post_bf16x3<D>, dim3(g), dim3(kThreads), lds, st, a, ntiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_post_bf16x3(const PostArgs& a, hipStream_t st) {
  switch (a.d) {
    case 1: case 2: case 3: case 4: return launch_d<4>(a, st);
    case 5: case 6: case 7: case 8: return launch_d<8>(a, st);
    case 9: case 10: return launch_d<10>(a, st);
    case 11: case 12: return launch_d<12>(a, st);
    default: return launch_d<16>(a, st);
  }
}

}  // namespace bo
