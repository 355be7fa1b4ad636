// Internal declarations of the gfx950 BO-step library: device state layout,
// workspace carving, kernel launch wrappers and small device helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/bo.h"

namespace bo {

constexpr int kMaxD = 16;
constexpr int kMaxN = 1024;
constexpr int kTile = 32;           // fit tile edge (FP64)
constexpr int kSmallFitMax = 256;   // most observations of the one-workgroup fit (batched, served, append)
constexpr int kPlainSmallMax = 128; // a single session's fit above this uses the multi-workgroup fit
constexpr int kRegMax = 256;        // n_pad of the register-resident posterior (FP64 products, FP64 and FP32)
constexpr int kAcqThreads = 256;
constexpr int kAcqPerThread = 2;
constexpr int kAcqMaxBlocks = 512;

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Device-resident scalars of one session.
struct DevState {
  int32_t status;       // fit status (BO_OK or an error code)
  int32_t attempt;      // accepted jitter attempt, or the failed one
  int32_t n;            // observations in the current fit
  int32_t need_retry;   // unused (kept 0)
  double mean_y, f_best, jitter;
  double lambda, var_mean;
  double min_piv;       // smallest accepted Cholesky pivot of the current factor
  int64_t n_unmasked;
  int32_t post_status;  // posterior / lambda status
  int32_t pad0;
  uint32_t ticket_post, ticket_acq, ticket_fit, pad1;
  int32_t fail_flag;    // unused (kept 0)
  int32_t pad2;
  // grid-wide barriers of the persistent large fit: cumulative arrivals, the
  // last barrier released, a flag that ends every wait (a spin limit hit),
  // and the phase of the current attempt in which a pivot failed (0: tile 0,
  // k + 1: the look-ahead of step k; 0xffffffff: none)
  uint32_t gs_arrive, gs_release, gs_abort, fail_at;
};

// Per-workgroup partial of the mean posterior variance.
struct VarSlot {
  double sum;
  int64_t count;
};

// Per-workgroup best candidate of each acquisition.
struct AcqSlot {
  double score[3];
  int32_t idx[3];   // compacted index, -1 = none
  int32_t nan_seen;
};

// Parameters passed by value to the kernels that compute lambda.
struct AcqArgs {
  int32_t mode;
  uint32_t bits;
  double lambda_const, mu_s, var_s_mean;
};

// Everything a kernel needs about a session's device memory.
struct DevPtrs {
  DevState* st;
  bo_acq_result* res;
  double* X64;        // [d][N_pad] normalized coordinates (SoA)
  uint16_t* Xc16;     // [N_pad][2][w16] augmented FP16 candidate coordinates (BF16X3 only)
  int32_t* orig;      // [N_pad] original index of compacted candidate, -1 pad
  int32_t* inv_map;   // [N] compacted position or -1 when invalid
  int32_t* blk;       // block counts / offsets for compaction
  void* mu;           // [N_pad] double (FP64) or float
  void* var;          // [N_pad]
  VarSlot* vslots;
  AcqSlot* aslots;
  double* Xo64;       // [n_max_pad][kMaxD]
  uint16_t* Xo16;     // [n_max_pad][2][w16] augmented FP16 observation coordinates (BF16X3 only)
  double* y;          // [n_max_pad]
  double* A;          // [n_max_pad^2] working matrix
  double* L;          // [n_max_pad^2]
  double* Dinv;       // [NB][32][32]
  double* Linv;       // [n_max_pad^2]
  double* alpha;      // [n_max_pad]
  double* z;          // [n_max_pad]
  void* Bpk;          // packed L^-1 operand for the matrix cores
  int64_t* obs;       // [n_max_pad] candidate indices of the current fit's observations
  uint8_t* vis;       // [N_pad] the session's own record of evaluated candidates
};

struct Layout {
  int64_t N, N_pad;
  int d, n_max, n_max_pad, prec, w16;
  size_t off_st, off_res, off_X64, off_Xc16, off_orig, off_inv, off_blk, off_mu, off_var,
      off_vslots, off_aslots, off_Xo64, off_Xo16, off_y, off_A, off_L, off_Dinv, off_Linv,
      off_alpha, off_z, off_Bpk, off_obs, off_vis, total;
  int64_t n_vslots, n_aslots;
};

// Entries per part of a row of augmented FP16 coordinates (BF16X3 distance
// products): d coordinates and four norm slots, in one or two 16-wide k-steps.
__host__ __device__ inline int aug16_width(int d) { return d + 4 <= 16 ? 16 : 32; }

// Pad of the observation dimension used by every kernel for a fit of n points.
inline int n_pad_of(int n) { return (int)round_up(n < 1 ? 1 : n, 64); }

size_t bpk_bytes(int prec, int n_pad);
bool make_layout(const bo_problem& p, Layout* L);
DevPtrs carve(const Layout& L, uint8_t* base);

struct GpConst {
  int32_t nu2, tries;
  double l, amp, noise;
};

// ---- launch wrappers (each returns hipSuccess or the launch error) ----
hipError_t launch_grid_setup(const DevPtrs& P, const Layout& Lo, const int32_t* levels, int d,
                             const int64_t* cand, const void* Xin, int x_is_f32,
                             const uint8_t* invalid, int64_t N, hipStream_t st);
hipError_t launch_fit_small(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                            const double* y_in, int n, hipStream_t st);
hipError_t launch_fit_append(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                             const double* y_in, int n, hipStream_t st);
hipError_t launch_fit_large(const DevPtrs& P, const Layout& Lo, const GpConst& g, const int64_t* obs_idx,
                            const double* y_in, int n, int first_attempt, hipStream_t st);
hipError_t launch_posterior(const DevPtrs& P, const Layout& Lo, const GpConst& g, int n, int64_t n_valid,
                            const uint8_t* visited, const AcqArgs& a, hipStream_t st);
hipError_t launch_acquire(const DevPtrs& P, const Layout& Lo, int64_t n_valid, const uint8_t* visited,
                          const AcqArgs& a, bo_acq_result* out_dev, hipStream_t st, double* ei = nullptr,
                          double* pi = nullptr, double* lcb = nullptr);
hipError_t launch_scatter_posterior(const DevPtrs& P, const Layout& Lo, int64_t n_valid,
                                    const uint8_t* visited, double* mu, double* var, hipStream_t st);

}  // namespace bo
