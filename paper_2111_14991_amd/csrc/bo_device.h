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

// Augmented FP16 coordinates of the BF16X3 posterior's distance products.
// With c = candidate, o = observation, S = kAugScale, T = kAugPair, the rows
//   c: S c[0..d-1],   T,  S^2|c|^2/T, T,  (.)_3
//   o: -2S o[0..d-1], S^2|o|^2/T, T, (.)_3, T
// multiply to S^2 (|c|^2 + |o|^2 - 2 c.o) = S^2 r^2.  Each entry is held as an
// FP16 high part and an FP16 remainder; the squared norms take a third FP16
// part (subscript 3) in the extra slot, so that the three products
// high*high + high*low + low*high of the matrix cores reproduce each norm to
// about 2^-33 of its size.  The scale keeps the remainders of coordinates in
// [0, 1] in the normal FP16 range (a remainder that would be subnormal is
// below 2^-14 / S of the coordinate), so that no significant part is lost to
// a flush of subnormal inputs; S^2|c|^2/T stays below 2^12 for d <= 16.
// w16 (16 or 32) entries per part; the row is hi[w16], lo[w16].
constexpr double kAugScale = 1024.0;
constexpr double kAugPair = 4096.0;

__device__ __forceinline__ uint32_t f16_bits(double v, double* used) {
  // any high part does (the remainder takes the difference); through FP32,
  // which has a hardware conversion
  const _Float16 h = (_Float16)(float)v;
  *used = (double)h;
  return __builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ void aug16_row(const double* x, int d, bool obs, uint16_t* row, int w16) {
  double nrm = 0.0;
  for (int j = 0; j < d; ++j) nrm += x[j] * x[j];
  nrm *= kAugScale * kAugScale / kAugPair;
  uint4* out = reinterpret_cast<uint4*>(row);
  // entries in groups of eight (one 16-byte store per part and group)
  for (int g = 0; g < w16; g += 8) {
    uint32_t hw[4], lw[4];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = g + q;
      double hi = 0.0, lo = 0.0, hv, lv;
      if (j < d) {
        hi = (obs ? -2.0 : 1.0) * kAugScale * x[j];
        lo = 1.0;  // marks "remainder of hi"
      } else if (j == d) {
        if (obs) { hi = nrm; lo = 1.0; } else hi = kAugPair;
      } else if (j == d + 1) {
        if (obs) hi = kAugPair; else { hi = nrm; lo = 1.0; }
      } else if (j == d + 2) {
        hi = obs ? 2.0 : kAugPair;  // obs: third part of the norm, below
      } else if (j == d + 3) {
        hi = obs ? kAugPair : 2.0;  // cand: third part of the norm, below
      }
      uint32_t hb, lb = 0;
      if ((obs && j == d + 2) || (!obs && j == d + 3)) {
        double n1, n2, n3;
        (void)f16_bits(nrm, &n1);
        (void)f16_bits(nrm - n1, &n2);
        hb = f16_bits(nrm - n1 - n2, &n3);
      } else {
        hb = f16_bits(hi, &hv);
        if (lo != 0.0) lb = f16_bits(hi - hv, &lv);
      }
      if (q & 1) {
        hw[q >> 1] |= hb << 16;
        lw[q >> 1] |= lb << 16;
      } else {
        hw[q >> 1] = hb;
        lw[q >> 1] = lb;
      }
    }
    out[g / 8] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
    out[(w16 + g) / 8] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
  }
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

// Sum of v over each row of 16 lanes, in every lane of the row: DPP moves
// only (quad permutations for lane distances 1 and 2, row rotations by 4 and
// 8), where a butterfly of lane exchanges would wait on the LDS crossbar at
// every step.
__device__ __forceinline__ double row_sum16_d(double v) {
  v += __builtin_amdgcn_update_dpp(0.0, v, 0xB1, 0xf, 0xf, true);   // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(0.0, v, 0x4E, 0xf, 0xf, true);   // quad_perm [2,3,0,1]
  v += __builtin_amdgcn_update_dpp(0.0, v, 0x124, 0xf, 0xf, true);  // row_ror:4
  v += __builtin_amdgcn_update_dpp(0.0, v, 0x128, 0xf, 0xf, true);  // row_ror:8
  return v;
}

// Sum of v over the 64 lanes of the wave, in every lane: the row sums, then
// two lane exchanges across the rows.
__device__ __forceinline__ double wave_sum_d(double v) {
  v = row_sum16_d(v);
  v += shfl_xor_d(v, 16);
  v += shfl_xor_d(v, 32);
  return v;
}

// A wave-uniform value the compiler cannot prove uniform (read through a
// pointer chosen at run time, or passed to a called function) moved to
// scalar registers: each 32-bit word is taken from the first active lane.
template <typename T>
__device__ __forceinline__ T uni(T v) {
  static_assert(sizeof(T) % 4 == 0, "32-bit words");
  union {
    T v;
    int w[sizeof(T) / 4];
  } u;
  u.v = v;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) u.w[i] = __builtin_amdgcn_readfirstlane(u.w[i]);
  return u.v;
}

// A device pointer known to address global memory (HBM): loads through it
// are global loads (addressed by a scalar base and a per-lane offset, counted
// by the vector memory counter only) rather than flat ones.
template <typename T>
using gptr_t = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr_t<T> gptr(T* p) {
  return (gptr_t<T>)p;
}

// Raw buffer over `bytes` bytes of device memory (gfx9 descriptor: no
// swizzle, no format; reads past the end return zero).  Loads through it take
// a per-lane offset and a scalar offset, so a sequence of loads at uniform
// distances costs scalar adds only.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ double buffer_load_f64(__amdgpu_buffer_rsrc_t r, int lane_off, int uniform_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, uniform_off, 0));
}

// Last-block ticket: returns true in exactly one workgroup of the launch,
// after every workgroup has published its partial.  The partial must be
// written by thread 0, which alone orders it before its ticket with a
// device-scope fence (one fence per workgroup, not one per wave).
__device__ __forceinline__ bool last_block(uint32_t* ticket, int* s_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t t = atomicAdd(ticket, 1u);
    *s_flag = (t == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = *s_flag != 0;
  if (last) __threadfence();
  return last;
}

}  // namespace bo
