// Candidate-set construction (Section III-D): linear normalization of each
// parameter's ordered levels to [0, 1] (Section III-D.1) and one-off
// compaction of the valid candidates, keeping their original indices, so that
// restriction-pruned points are never predicted (Section III-D.2).
#include "bo_internal.h"
#include "bo_device.h"

namespace bo {
namespace {

constexpr int kSetupThreads = 1024;

struct GridArgs {
  int32_t d;
  int32_t from_coords;  // 0: decode grid index; 1: FP64 X; 2: FP32 X
  int64_t total;        // grid size
  int32_t levels[kMaxD];
};

__device__ __forceinline__ bool cand_ok(const GridArgs& ga, const int64_t* cand, int64_t c) {
  if (ga.from_coords) return true;
  const int64_t g = cand ? cand[c] : c;
  return g >= 0 && g < ga.total;
}

// Pass 1: per 1024-candidate block, count valid candidates; flag bad indices.
__global__ __launch_bounds__(kSetupThreads) void k_setup_count(int64_t N, GridArgs ga, const int64_t* cand,
                                                               const uint8_t* invalid, int32_t* blk,
                                                               DevState* st) {
  const int64_t c = (int64_t)blockIdx.x * kSetupThreads + threadIdx.x;
  int valid = 0;
  if (c < N) {
    if (!cand_ok(ga, cand, c)) atomicExch(&st->post_status, (int)BO_E_INVALID_ARG);
    valid = invalid ? (invalid[c] == 0) : 1;
  }
  const int cnt = __syncthreads_count(valid);
  if (threadIdx.x == 0) blk[blockIdx.x] = cnt;
}

// Pass 2: exclusive scan of the block counts (one workgroup), total -> n_unmasked.
__global__ __launch_bounds__(kSetupThreads) void k_setup_scan(int nblk, int32_t* blk, DevState* st) {
  __shared__ int32_t s_part[kSetupThreads];
  const int per = (nblk + kSetupThreads - 1) / kSetupThreads;
  const int b0 = threadIdx.x * per;
  int32_t sum = 0;
  for (int b = b0; b < b0 + per && b < nblk; ++b) sum += blk[b];
  s_part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < kSetupThreads; off <<= 1) {
    int32_t v = threadIdx.x >= off ? s_part[threadIdx.x - off] : 0;
    __syncthreads();
    s_part[threadIdx.x] += v;
    __syncthreads();
  }
  int32_t run = threadIdx.x > 0 ? s_part[threadIdx.x - 1] : 0;
  for (int b = b0; b < b0 + per && b < nblk; ++b) {
    const int32_t v = blk[b];
    blk[b] = run;
    run += v;
  }
  if (threadIdx.x == kSetupThreads - 1) st->n_unmasked = s_part[kSetupThreads - 1];
}

// Pass 3: scatter valid candidates to their compacted position with their
// normalized coordinates: level i of k -> i / (k - 1) (0 when k = 1).
__global__ __launch_bounds__(kSetupThreads) void k_setup_scatter(int64_t N, int64_t N_pad, GridArgs ga,
                                                                 const int64_t* cand, const void* Xin,
                                                                 const uint8_t* invalid, const int32_t* blk,
                                                                 const DevState* st, double* X64,
                                                                 int32_t* orig, int32_t* inv_map) {
  __shared__ int32_t s_wave[kSetupThreads / 64];
  const int64_t c = (int64_t)blockIdx.x * kSetupThreads + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int valid = 0;
  if (c < N) valid = (invalid ? (invalid[c] == 0) : 1) && cand_ok(ga, cand, c);
  const uint64_t bal = __ballot(valid);
  if (lane == 0) s_wave[wave] = __popcll(bal);
  __syncthreads();
  int32_t before = 0;
  for (int w = 0; w < wave; ++w) before += s_wave[w];
  const int32_t rank = before + __popcll(bal & ((1ull << lane) - 1ull));
  if (c < N) {
    if (valid) {
      const int64_t pos = (int64_t)blk[blockIdx.x] + rank;
      orig[pos] = (int32_t)c;
      inv_map[c] = (int32_t)pos;
      if (ga.from_coords == 0) {
        int64_t g = cand ? cand[c] : c;
        for (int j = ga.d - 1; j >= 0; --j) {
          const int64_t k = ga.levels[j];
          const int64_t i = g % k;
          g /= k;
          const double x = k > 1 ? (double)i / (double)(k - 1) : 0.0;
          X64[(int64_t)j * N_pad + pos] = x;
        }
      } else {
        for (int j = 0; j < ga.d; ++j) {
          const double x = ga.from_coords == 1 ? ((const double*)Xin)[c * ga.d + j]
                                               : (double)((const float*)Xin)[c * ga.d + j];
          X64[(int64_t)j * N_pad + pos] = x;
        }
      }
    } else {
      inv_map[c] = -1;
    }
  }
  // padding rows beyond the valid count
  const int64_t nv = st->n_unmasked;
  if (c >= nv && c < N_pad) {
    orig[c] = -1;
    for (int j = 0; j < ga.d; ++j) X64[(int64_t)j * N_pad + c] = 0.0;
  }
}

// Augmented FP16 coordinates of every compacted candidate (padding rows
// included) for the BF16X3 distance products.
__global__ __launch_bounds__(kSetupThreads) void k_setup_aug16(int64_t N_pad, int d, int w16, const double* X64,
                                                               uint16_t* Xc16) {
  const int64_t c = (int64_t)blockIdx.x * kSetupThreads + threadIdx.x;
  if (c >= N_pad) return;
  double x[kMaxD];
  for (int j = 0; j < d; ++j) x[j] = X64[(int64_t)j * N_pad + c];
  aug16_row(x, d, false, Xc16 + c * 2 * w16, w16);
}

}  // namespace

hipError_t launch_grid_setup(const DevPtrs& P, const Layout& Lo, const int32_t* levels, int d,
                             const int64_t* cand, const void* Xin, int x_is_f32,
                             const uint8_t* invalid, int64_t N, hipStream_t st) {
  GridArgs ga{};
  ga.d = d;
  ga.from_coords = Xin ? (x_is_f32 ? 2 : 1) : 0;
  ga.total = 1;
  if (!Xin) {
    for (int j = 0; j < d; ++j) {
      ga.levels[j] = levels[j];
      ga.total *= levels[j];
    }
  }
  const int64_t span = Lo.N_pad > N ? Lo.N_pad : N;
  const int nblk = (int)((N + kSetupThreads - 1) / kSetupThreads);
  const int nblk_pad = (int)((span + kSetupThreads - 1) / kSetupThreads);
  hipLaunchKernelGGL(k_setup_count, dim3(nblk), dim3(kSetupThreads), 0, st, N, ga, cand, invalid, P.blk, P.st);
  hipLaunchKernelGGL(k_setup_scan, dim3(1), dim3(kSetupThreads), 0, st, nblk, P.blk, P.st);
  hipLaunchKernelGGL(k_setup_scatter, dim3(nblk_pad), dim3(kSetupThreads), 0, st, N, Lo.N_pad, ga, cand, Xin,
                     invalid, P.blk, P.st, P.X64, P.orig, P.inv_map);
  if (P.Xc16)
    hipLaunchKernelGGL(k_setup_aug16, dim3((unsigned)((Lo.N_pad + kSetupThreads - 1) / kSetupThreads)),
                       dim3(kSetupThreads), 0, st, Lo.N_pad, d, Lo.w16, P.X64, P.Xc16);
  return hipGetLastError();
}

}  // namespace bo
