// Posterior of the BF16X3 precision mode (exhaustive prediction, Section
// III-G) on the matrix cores.
//
// Persistent kernel: each workgroup of 8 waves loops over tiles of 64
// compacted candidates; the observation coordinates, their squared norms and
// alpha are parked in LDS once.  For a tile the observations are streamed in
// chunks of 64:
//  - generation: the cross products x_c . x_i of a 16 x 16 (observation x
//    candidate) block come from FP32 16x16x4 matrix-core products;
//    r^2 = |x_c|^2 + |x_i|^2 - 2 x_c . x_i, k* = amp Matern(r) in FP32; k*
//    alpha is added to an FP64 running mean; k* is split into a bfloat16
//    high part and a bfloat16 remainder, written to LDS in the A-operand
//    order of the 32x32x16 bfloat16 product (double-buffered: the next chunk
//    is generated while the current one is consumed);
//  - contraction: each wave owns up to four 32-column blocks of W = K* L^-T
//    (blocks w, 15 - w, 16 + w and 31 - w, so every wave has the same number
//    of k-steps at n_pad = 1024) for all 64 candidates and accumulates
//    hi*hi + hi*lo + lo*hi in FP32.  The all-zero tiles above the diagonal
//    are skipped: each block's fragments cover whole chunks, so the blocks a
//    wave updates are decided once per chunk.  The L^-1 fragments of the next k-step are
//    requested (buffer loads at scalar offsets) as soon as the current ones
//    have been consumed.
// The squared column sums are combined across waves in a fixed order,
// var = amp - sum |W_c|^2 is clamped at zero, and the tile's mean-variance
// partial goes to the tile's slot.
#include "bo_internal.h"
#include "bo_device.h"
#include "post_common.h"

namespace bo {
namespace {

constexpr int kRows = 64;
constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kQ = 32 / kWaves;     // column blocks per wave (n <= 1024)
constexpr int kGen = 16 / kWaves;   // 16x16 generation blocks per wave and chunk
constexpr int kChunk = 64;  // observations per LDS chunk (4 k-steps of 16)
constexpr int kFragBytes = 64 * 16;  // one 32x32x16 operand fragment
// row pitch of the observation coordinates in LDS: 17 floats, so that the 16
// observations a quarter-wave reads in the distance products fall in
// distinct banks (a pitch of 16 puts them in two)
constexpr int kXoPitch = kMaxD + 1;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const f32x2 v = {a, b};
  const bf16x2 r = __builtin_convertvector(v, bf16x2);
  return *reinterpret_cast<const uint32_t*>(&r);
}

__device__ __forceinline__ uint4 load_frag(__amdgpu_buffer_rsrc_t r, int lane_off, int off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, lane_off, off, 0);
  return make_uint4(v[0], v[1], v[2], v[3]);
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
  float xo[kMaxN * kXoPitch];  // observation coordinates, zero-padded
  float xn[kMaxN];          // their squared norms
  double alpha[kMaxN];
  float sq[kWaves][kRows];
  double mu[kWaves / 4][kRows];
  double rsum[kThreads];
  int64_t rcnt[kThreads];
  int last;
};

template <int KS>
__global__ __launch_bounds__(kThreads) void k_post_bf16x3(PostArgs p, int ntiles) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  Smem& S = *reinterpret_cast<Smem*>(s_raw);

  if (p.st->status != BO_OK) return;
  const int tid = threadIdx.x;
  // the wave index is uniform per wave: keep it (and everything derived from
  // it: column blocks, fragment offsets, branch conditions) in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int JB = p.n_pad >> 5;
  const int NC = p.n_pad / kChunk;
  const float inv_l = (float)p.inv_l, amp = (float)p.amp;
  const double mean_y = p.st->mean_y;
  const float c_rho = (p.nu2 == 5 ? 2.2360679775f : 1.73205080757f) * inv_l;
  const float c_poly = p.nu2 == 5 ? 0.333333333333f : 0.f;

  for (int e = tid; e < p.n_pad * kMaxD; e += kThreads) {
    const int i = e / kMaxD, j = e % kMaxD;
    S.xo[i * kXoPitch + j] = (i < p.n && j < p.d) ? p.Xo32[(size_t)i * kMaxD + j] : 0.f;
  }
  for (int i = tid; i < p.n_pad; i += kThreads) S.alpha[i] = i < p.n ? p.alpha[i] : 0.0;
  __syncthreads();
  for (int i = tid; i < p.n_pad; i += kThreads) {
    float s = 0.f;
    for (int j = 0; j < kMaxD; ++j) s = fmaf(S.xo[i * kXoPitch + j], S.xo[i * kXoPitch + j], s);
    S.xn[i] = s;
  }

  // generation role: row block rb (16 candidates), observation blocks
  // ob0 + (kWaves / 4) j, j < kGen, of each chunk; lane l works on candidate
  // rb*16 + l%16 and the four observations 4(l/16) .. 4(l/16)+3 of a block
  const int rb = w & 3, ob0 = w >> 2;
  const int lrow = rb * 16 + (lane & 15);
  const int g_rg = lrow >> 5;
  const int g_lane = (lrow & 31) + 32 * (lane >> 5);
  const int g_word = 2 * ((lane >> 4) & 1);  // 4-element half of the 16-byte slot

  // this wave's 32-column blocks of W in ascending order, w and 31 - w with
  // 16 waves (w, 15 - w, 16 + w, 31 - w with 8): the same number of k-steps
  // for every wave at n_pad = 1024; the first nact exist.  Block J's fragments
  // start at frag32 base(J) and cover whole chunks (zero past k-step 2J+1),
  // so the set of blocks a chunk updates changes only between chunks.
  int Jq[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) Jq[q] = (q & 1) ? kWaves * (q + 1) - 1 - w : kWaves * q + w;
  int nact = 0;
#pragma unroll
  for (int q = 0; q < kQ; ++q) nact += Jq[q] < JB ? 1 : 0;
  const int M = p.n_pad / 64;
  const int nfrag = 4 * M * (M + 1);
  const __amdgpu_buffer_rsrc_t rB = buffer_of(p.Bpk, nfrag * 2 * kFragBytes);
  const int lo_off = nfrag * kFragBytes;
  int fb[kQ];  // byte offset of fragment 0 of each block (high parts)
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int m = Jq[q] >> 1;
    fb[q] = ((Jq[q] & 1) ? 4 * (m + 1) * (m + 1) : 4 * m * (m + 1)) * kFragBytes;
  }
  const int loff = lane * 16;

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row_base = (int64_t)tile * kRows;
    // this lane's candidate coordinates as the B operand of the distance
    // products: k-step s holds coordinate 4s + l/16
    float bx[KS];
    float rnorm = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int j = 4 * s + (lane >> 4);
      bx[s] = j < p.d ? p.X32[(int64_t)j * p.N_pad + row_base + lrow] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4 * KS; ++j) {
      const float x = j < p.d ? p.X32[(int64_t)j * p.N_pad + row_base + lrow] : 0.f;
      rnorm = fmaf(x, x, rnorm);
    }
    double mu_acc = 0.0;

    // distance products of observation block ob (within chunk c)
    auto dist = [&](int c, int ob) -> f32x4 {
      f32x4 d = {0.f, 0.f, 0.f, 0.f};
      const int obs = c * kChunk + ob * 16 + (lane & 15);
#pragma unroll
      for (int s = 0; s < KS; ++s)
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(S.xo[obs * kXoPitch + 4 * s + (lane >> 4)], bx[s], d, 0, 0, 0);
      return d;
    };
    // Matern, mean, split and store of the four values of block ob; output
    // register q of lane l is observation 4(l/16) + q, candidate l%16
    auto finish = [&](int c, int ob, f32x4 d, ChunkBuf& b) {
      float kv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = c * kChunk + ob * 16 + 4 * (lane >> 4) + q;
        float r2 = fmaf(-2.f, d[q], rnorm + S.xn[i]);
        r2 = r2 > 0.f ? r2 : 0.f;
        const float rho = c_rho * __builtin_amdgcn_sqrtf(r2);
        const float e = __builtin_amdgcn_exp2f(-1.44269504089f * rho);
        float k = amp * fmaf(rho, fmaf(rho, c_poly, 1.0f), 1.0f) * e;
        k = i < p.n ? k : 0.f;
        mu_acc += (double)k * S.alpha[i];
        kv[q] = k;
      }
      const uint32_t h01 = pack_bf16x2(kv[0], kv[1]);
      const uint32_t h23 = pack_bf16x2(kv[2], kv[3]);
      const uint32_t l01 =
          pack_bf16x2(kv[0] - __uint_as_float(h01 << 16), kv[1] - __uint_as_float(h01 & 0xffff0000u));
      const uint32_t l23 =
          pack_bf16x2(kv[2] - __uint_as_float(h23 << 16), kv[3] - __uint_as_float(h23 & 0xffff0000u));
      uint32_t* ph = reinterpret_cast<uint32_t*>(&b.a[0][g_rg][ob][g_lane]) + g_word;
      uint32_t* pl = reinterpret_cast<uint32_t*>(&b.a[1][g_rg][ob][g_lane]) + g_word;
      *reinterpret_cast<uint2*>(ph) = make_uint2(h01, h23);
      *reinterpret_cast<uint2*>(pl) = make_uint2(l01, l23);
    };

    f32x16 acc[kQ][2];
#pragma unroll
    for (int q = 0; q < kQ; ++q)
#pragma unroll
      for (int rg = 0; rg < 2; ++rg)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[q][rg][i] = 0.f;

    __syncthreads();  // LDS tables ready; previous tile done with the buffers
#pragma unroll
    for (int j = 0; j < kGen; ++j) finish(0, ob0 + (kWaves / 4) * j, dist(0, ob0 + (kWaves / 4) * j), S.buf[0]);
    // L^-1 fragments of k-step 0
    uint4 bh[kQ], bl[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      if (q < nact) {
        bh[q] = load_frag(rB, loff, fb[q]);
        bl[q] = load_frag(rB, loff, lo_off + fb[q]);
      }
    }
    __syncthreads();

    for (int c = 0; c < NC; ++c) {
      const ChunkBuf& cur = S.buf[c & 1];
      ChunkBuf& nxt = S.buf[(c + 1) & 1];
      const bool more = c + 1 < NC;
      // block q has nonzero k-steps in chunks 0 .. J/2; the blocks are in
      // ascending order, so the active ones are those from q0 to nact - 1
      bool act[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) act[q] = q < nact && c <= (Jq[q] >> 1);
      f32x4 dd = {0.f, 0.f, 0.f, 0.f};
      // the chunk's four k-steps unrolled: a step's A fragments can be read
      // while the previous step's products run, and the generation pieces
      // are placed at compile time
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int t = 4 * c + s;
        // a quarter (8 waves) or half (16 waves) of the next chunk's
        // generation per k-step
        if (more) {
          if (kGen == 2) {
            if (s == 0) dd = dist(c + 1, ob0);
            if (s == 1) finish(c + 1, ob0, dd, nxt);
            if (s == 2) dd = dist(c + 1, ob0 + 2);
            if (s == 3) finish(c + 1, ob0 + 2, dd, nxt);
          } else {
            if (s == 0) dd = dist(c + 1, ob0);
            if (s == 2) finish(c + 1, ob0, dd, nxt);
          }
        }
        const bf16x8 ah0 = as_bf16x8(cur.a[0][0][s][lane]);
        const bf16x8 ah1 = as_bf16x8(cur.a[0][1][s][lane]);
        const bf16x8 al0 = as_bf16x8(cur.a[1][0][s][lane]);
        const bf16x8 al1 = as_bf16x8(cur.a[1][1][s][lane]);
        // three passes over the active blocks (hi*hi, hi*lo, lo*hi) so that
        // consecutive products write different accumulators
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          if (act[q]) {
            const bf16x8 h = as_bf16x8(bh[q]);
            acc[q][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, h, acc[q][0], 0, 0, 0);
            acc[q][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, h, acc[q][1], 0, 0, 0);
          }
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          if (act[q]) {
            const bf16x8 l = as_bf16x8(bl[q]);
            acc[q][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, l, acc[q][0], 0, 0, 0);
            acc[q][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, l, acc[q][1], 0, 0, 0);
          }
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          if (act[q]) {
            const bf16x8 h = as_bf16x8(bh[q]);
            acc[q][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al0, h, acc[q][0], 0, 0, 0);
            acc[q][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al1, h, acc[q][1], 0, 0, 0);
          }
          // the next k-step's fragments (past a block's end: the next
          // block's, or zero past the buffer; never used)
          if (act[q]) {
            const int off = fb[q] + (t + 1) * kFragBytes;
            bh[q] = load_frag(rB, loff, off);
            bl[q] = load_frag(rB, loff, lo_off + off);
          }
        }
      }
      __syncthreads();
    }

    // squared row sums over the wave's columns; output register i of lane L
    // holds row 8(i/4) + 4(L/32) + i%4 of the row group, column L%32.  A
    // transposing butterfly over the 32 lanes of a half-wave: at each of the
    // lane distances 16, 8, 4, 2 a lane keeps half of its partial sums and
    // adds its partner's copies of them, so 16 + 8 + 4 + 2 + 1 values move
    // instead of 16 x 5; lane L ends with register i = (L % 32) / 2.
#pragma unroll
    for (int rg = 0; rg < 2; ++rg) {
      float v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < kQ; ++q) t = fmaf(acc[q][rg][i], acc[q][rg][i], t);
        v[i] = t;
      }
#pragma unroll
      for (int h = 8; h >= 1; h >>= 1) {
        const bool up = (lane & (2 * h)) != 0;  // keeps the upper half
#pragma unroll
        for (int j = 0; j < h; ++j) {
          const float send = up ? v[j] : v[h + j];
          const float keep = up ? v[h + j] : v[j];
          v[j] = keep + __shfl_xor(send, 2 * h, 64);
        }
      }
      v[0] += __shfl_xor(v[0], 1, 64);
      const int i = (lane & 31) >> 1;
      if ((lane & 1) == 0) S.sq[w][32 * rg + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3)] = v[0];
    }
    // mean: the four lanes l, l+16, l+32, l+48 share a candidate
    mu_acc += shfl_xor_d(mu_acc, 16);
    mu_acc += shfl_xor_d(mu_acc, 32);
    if (lane < 16) S.mu[ob0][lrow] = mu_acc;
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
        double m = 0.0;
#pragma unroll
        for (int i = 0; i < kWaves / 4; ++i) m += S.mu[i][tid];
        ((float*)p.mu)[row] = (float)(mean_y + m);
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

template <int KS>
hipError_t launch_ks(const PostArgs& a, hipStream_t st) {
  static int grid = 0;
  const size_t lds = sizeof(Smem);
  if (grid == 0) {
    hipError_t e = hipFuncSetAttribute((const void*)k_post_bf16x3<KS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_post_bf16x3<KS>, kThreads, lds);
    if (e != hipSuccess) return e;
    grid = cus * (per > 0 ? per : 1);
  }
  const int ntiles = (int)((a.n_valid + kRows - 1) / kRows);
  const int g = ntiles < grid ? ntiles : grid;
  hipLaunchKernelGGL(k_post_bf16x3<KS>, dim3(g), dim3(kThreads), lds, st, a, ntiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_post_bf16x3(const PostArgs& a, hipStream_t st) {
  if (a.d <= 4) return launch_ks<1>(a, st);
  if (a.d <= 8) return launch_ks<2>(a, st);
  if (a.d <= 12) return launch_ks<3>(a, st);
  return launch_ks<4>(a, st);
}

}  // namespace bo
