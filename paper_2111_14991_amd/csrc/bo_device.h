// Device helpers of the gfx950 BO-step library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bo {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

// Matern correlation at half-integer order (Section III-B), unit amplitude,
// scaled distance rho = sqrt(2 nu) r / l.  FP64.
__device__ __forceinline__ double matern64(int nu2, double r, double inv_l) {
  if (nu2 == 5) {
    const double rho = 2.23606797749978969641 * r * inv_l;
    return (1.0 + rho + rho * rho * (1.0 / 3.0)) * exp(-rho);
  }
  const double rho = 1.73205080756887729353 * r * inv_l;
  return (1.0 + rho) * exp(-rho);
}

// Same in FP32 from a squared distance, on the hardware exp2/sqrt units.
__device__ __forceinline__ float matern32_r2(int nu2, float r2, float inv_l) {
  r2 = r2 > 0.f ? r2 : 0.f;
  const float r = __builtin_amdgcn_sqrtf(r2);
  if (nu2 == 5) {
    const float rho = 2.2360679775f * r * inv_l;
    const float e = __builtin_amdgcn_exp2f(-1.44269504089f * rho);
    return fmaf(rho, fmaf(rho, 0.333333333333f, 1.0f), 1.0f) * e;
  }
  const float rho = 1.73205080757f * r * inv_l;
  const float e = __builtin_amdgcn_exp2f(-1.44269504089f * rho);
  return (1.0f + rho) * e;
}

// Diagonal addition of jitter attempt t: the noise first, then tenfold steps
// from max(noise, 1e-10 amp).
__device__ __host__ __forceinline__ double jitter_of(double noise, double amp, int t) {
  if (t == 0) return noise;
  double base = noise > 1e-10 * amp ? noise : 1e-10 * amp;
  double p = 1.0;
  for (int i = 0; i < t; ++i) p *= 10.0;
  return base * p;
}

// Minimization-form acquisitions at one point (Section III-C) in FP64:
// tau = f_best - lambda, z = (tau - mu) / sigma,
// EI = (tau - mu) Phi(z) + sigma phi(z), PI = Phi(z) = erfc(-z/sqrt2)/2,
// LCB = mu - lambda sigma; sigma = 0 uses the sigma -> 0 limits.
__device__ __forceinline__ void acquisitions64(double mu, double var, double f_best, double lambda,
                                               double* ei, double* pi, double* lcb) {
  const double tau = f_best - lambda;
  const double sigma = sqrt(var);
  if (sigma > 0.0) {
    const double z = (tau - mu) / sigma;
    const double Phi = 0.5 * erfc(-z * 0.70710678118654752440);
    const double phi = exp(-0.5 * z * z) * 0.39894228040143267794;
    *pi = Phi;
    *ei = (tau - mu) * Phi + sigma * phi;
  } else {
    *ei = tau - mu > 0.0 ? tau - mu : 0.0;
    *pi = tau > mu ? 1.0 : (tau == mu ? 0.5 : 0.0);
  }
  *lcb = mu - lambda * sigma;
}

// "a is a better candidate than b": higher score (or lower, for minimize),
// ties to the lower index; idx < 0 means "no candidate".
__device__ __forceinline__ bool better(double sa, int ia, double sb, int ib, bool minimize) {
  if (ia < 0) return false;
  if (ib < 0) return true;
  if (sa != sb) return minimize ? (sa < sb) : (sa > sb);
  return ia < ib;
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  return __shfl_xor(v, m, 64);
}

// Last-block ticket: returns true in exactly one workgroup of the launch,
// after every workgroup has published its partial with a device-scope fence.
__device__ __forceinline__ bool last_block(uint32_t* ticket, int* s_flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = atomicAdd(ticket, 1u);
    *s_flag = (t == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = *s_flag != 0;
  if (last) __threadfence();
  return last;
}

}  // namespace bo
