// Acquisition kernels of one session (the device code is in acq_common.h),
// and the scatter of the posterior back to the caller's enumeration.
#include "bo_internal.h"
#include "bo_device.h"
#include "acq_common.h"

namespace bo {
namespace {

template <bool F32>
__global__ __launch_bounds__(kAcqThreads) void k_acquire(AcqKArgs a) {
  __shared__ Best s_best[kAcqThreads / 64];
  __shared__ int s_nan[kAcqThreads / 64];
  const int64_t per = (a.n_valid + gridDim.x - 1) / gridDim.x;
  const int64_t c0 = (int64_t)blockIdx.x * per;
  const int64_t c1 = c0 + per < a.n_valid ? c0 + per : a.n_valid;
  acq_range<F32>(a, c0, c1, &a.slots[blockIdx.x], s_best, s_nan);
}

// The step result from the slots (one workgroup, after the acquisition
// launch: a last-workgroup ticket would need a device-scope fence in every
// workgroup of it).
__global__ __launch_bounds__(kAcqThreads) void k_acquire_finish(AcqKArgs a, int nslots) {
  __shared__ Best s_best[kAcqThreads / 64];
  __shared__ int s_nan[kAcqThreads / 64];
  acq_finish(a, nslots, s_best, s_nan);
}

// Posterior written back in the caller's enumeration (NaN where excluded).
template <bool F32>
__global__ void k_scatter_post(int64_t N, const int32_t* inv_map, const uint8_t* visited, const void* mu,
                               const void* var, double* mu_out, double* var_out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const double qnan = __longlong_as_double(0x7ff8000000000000LL);
  const int32_t pos = inv_map[c];
  double m = qnan, v = qnan;
  if (pos >= 0 && !(visited && visited[c])) {
    if constexpr (F32) {
      m = ((const float*)mu)[pos];
      v = ((const float*)var)[pos];
    } else {
      m = ((const double*)mu)[pos];
      v = ((const double*)var)[pos];
    }
  }
  if (mu_out) mu_out[c] = m;
  if (var_out) var_out[c] = v;
}

}  // namespace

// Workgroups of one acquisition launch: kAcqPerThread candidates per thread,
// at most kAcqMaxBlocks (the slots of the session's workspace).
int64_t acquire_blocks(int64_t n_valid) {
  const int64_t per = (int64_t)kAcqThreads * kAcqPerThread;
  const int64_t g = (n_valid + per - 1) / per;
  return g < 1 ? 1 : (g > kAcqMaxBlocks ? kAcqMaxBlocks : g);
}

hipError_t launch_acquire(const DevPtrs& P, const Layout& Lo, int64_t n_valid, const uint8_t* visited,
                          const AcqArgs& acq, bo_acq_result* out_dev, hipStream_t st, double* ei, double* pi,
                          double* lcb) {
  AcqKArgs a = make_acq_args(P, n_valid, visited, acq, out_dev);
  a.vals[0] = ei;
  a.vals[1] = pi;
  a.vals[2] = lcb;
  const int grid = (int)acquire_blocks(n_valid);
  if (Lo.prec == BO_FP64)
    hipLaunchKernelGGL(k_acquire<false>, dim3(grid), dim3(kAcqThreads), 0, st, a);
  else
    hipLaunchKernelGGL(k_acquire<true>, dim3(grid), dim3(kAcqThreads), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_acquire_finish, dim3(1), dim3(kAcqThreads), 0, st, a, grid);
  return hipGetLastError();
}

hipError_t launch_scatter_posterior(const DevPtrs& P, const Layout& Lo, int64_t n_valid,
                                    const uint8_t* visited, double* mu, double* var, hipStream_t st) {
  (void)n_valid;
  const int grid = (int)((Lo.N + 255) / 256);
  if (Lo.prec == BO_FP64)
    hipLaunchKernelGGL(k_scatter_post<false>, dim3(grid), dim3(256), 0, st, Lo.N, P.inv_map, visited, P.mu,
                       P.var, mu, var);
  else
    hipLaunchKernelGGL(k_scatter_post<true>, dim3(grid), dim3(256), 0, st, Lo.N, P.inv_map, visited, P.mu, P.var,
                       mu, var);
  return hipGetLastError();
}

}  // namespace bo
