// C ABI of the BO-step library: argument validation, workspace carving,
// session lifecycle and the launch sequence of one step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "bo_internal.h"
#include "session_impl.h"

using namespace bo;

namespace bo {
int64_t acquire_blocks(int64_t n_valid);
}

// Device memory of bo_step_noalloc: one copy per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on the
// host it is only a stand-in for the symbol); it uses the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];


namespace {

bo_status fail(bo_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vset_error(fmt, ap);
  va_end(ap);
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(BO_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool problem_ok(const bo_problem* p) {
  return p && p->N >= 1 && p->N < (int64_t(1) << 31) && p->d >= 1 && p->d <= kMaxD && p->n_max >= 1 &&
         p->n_max <= kMaxN && p->precision >= BO_FP64 && p->precision <= BO_BF16X3;
}

__global__ void k_state_clear(DevState* st, int full) {
  if (threadIdx.x == 0) {
    if (full) {
      DevState z{};
      z.status = BO_E_STATE;
      *st = z;
    } else {
      st->post_status = BO_OK;
      st->n_unmasked = 0;
    }
  }
}

__global__ void k_fill_u8(uint8_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_fill_nan(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = __longlong_as_double(0x7ff8000000000000LL);
}

// One evaluation recorded in the session (Section III-D.2): the candidate is
// marked evaluated; a valid evaluation is placed after the current fit's
// observations, at position `at` of the session's observation list.
__global__ void k_observe(uint8_t* vis, int64_t* obs, double* y, int64_t idx, double yv, int valid, int at) {
  if (threadIdx.x == 0) {
    vis[idx] = 1;
    if (valid) {
      obs[at] = idx;
      y[at] = yv;
    }
  }
}

bo_status sync_state(bo_session* s) {
  HIP_TRY(hipMemcpyAsync(s->hstate, s->P.st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return BO_OK;
}

bo_status check_acq(const bo_acq_params* a, AcqArgs* out) { return acq_params_check(a, out); }

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices];

// Address of the current device's scratch array, looked up once per device.
bo_status scratch_of_current_device(uint8_t** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(BO_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kScratchDevices) return fail(BO_E_HIP, "device %d beyond the %d supported", dev, kScratchDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(BO_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = (uint8_t*)g_scratch_ptr[dev];
  return BO_OK;
}

// GP parameters (NULL: the defaults) checked into *g.
bo_status gp_check(const bo_gp_params* gp, bo_gp_params* g) {
  *g = bo_gp_params{5, 7, 1.0, 1.0, 1e-6};
  if (gp) *g = *gp;
  if (g->nu2 != 3 && g->nu2 != 5) return fail(BO_E_INVALID_ARG, "nu2 must be 3 or 5");
  if (!(g->lengthscale > 0.0) || !std::isfinite(g->lengthscale)) return fail(BO_E_INVALID_ARG, "lengthscale");
  if (!(g->amp > 0.0) || !std::isfinite(g->amp)) return fail(BO_E_INVALID_ARG, "amp");
  if (!(g->noise >= 0.0) || !std::isfinite(g->noise)) return fail(BO_E_INVALID_ARG, "noise");
  if (g->jitter_tries < 1 || g->jitter_tries > 20) return fail(BO_E_INVALID_ARG, "jitter_tries must be 1..20");
  return BO_OK;
}

bo_status step_ready(bo_session* s) {
  if (!s) return fail(BO_E_INVALID_ARG, "session is NULL");
  if (!s->have_cand) return fail(BO_E_STATE, "no candidate set");
  if (!s->have_fit) return fail(BO_E_STATE, "no fit");
  return BO_OK;
}

bo_status mark(bo_session* s, int which) {
  if (s->timing) {
    HIP_TRY(hipEventRecord(s->ev[which], s->stream));
    if (which & 1) s->ev_have[which >> 1] = 1;
  }
  return BO_OK;
}

#define MARK(s, w)                   \
  do {                               \
    bo_status m_ = mark((s), (w));   \
    if (m_ != BO_OK) return m_;      \
  } while (0)

bo_status enqueue_posterior(bo_session* s, const uint8_t* visited, const AcqArgs& a) {
  MARK(s, 2);
  HIP_TRY(launch_posterior(s->P, s->lo, s->gp, s->n, s->n_valid, visited, a, s->stream));
  MARK(s, 3);
  return BO_OK;
}

bo_status enqueue_step(bo_session* s, const uint8_t* visited, const AcqArgs& a, bo_acq_result* out_dev,
                       double* ei = nullptr, double* pi = nullptr, double* lcb = nullptr) {
  bo_status rc = enqueue_posterior(s, visited, a);
  if (rc != BO_OK) return rc;
  MARK(s, 4);
  HIP_TRY(launch_acquire(s->P, s->lo, s->n_valid, visited, a, out_dev, s->stream, ei, pi, lcb));
  MARK(s, 5);
  return BO_OK;
}

// Refit after one new observation at position n - 1 of (obs_idx, y): the
// bordered extension of the current factor when it holds n - 1 points and
// n <= kSmallFitMax, otherwise a whole fit.
bo_status append_fit(bo_session* s, const int64_t* obs_idx, const double* y, int n) {
  const bool bordered = s->have_fit && s->n == n - 1 && n <= kSmallFitMax;
  s->n = n;
  s->large_fit = !bordered && n > kPlainSmallMax;
  MARK(s, 0);
  if (bordered)
    HIP_TRY(launch_fit_append(s->P, s->lo, s->gp, obs_idx, y, n, s->stream));
  else if (!s->large_fit)
    HIP_TRY(launch_fit_small(s->P, s->lo, s->gp, obs_idx, y, n, s->stream));
  else
    HIP_TRY(launch_fit_large(s->P, s->lo, s->gp, obs_idx, y, n, 0, s->stream));
  MARK(s, 1);
  s->have_fit = 1;
  return BO_OK;
}

bo_status set_candidates(bo_session* s, const int32_t* levels, const int64_t* cand, const void* X, int x_is_f32,
                         const uint8_t* invalid, int64_t* n_valid) {
  if (!s) return fail(BO_E_INVALID_ARG, "session is NULL");
  const int d = s->prob.d;
  const int64_t N = s->prob.N;
  if (!X) {
    if (!levels) return fail(BO_E_INVALID_ARG, "levels is NULL");
    __int128 total = 1;
    for (int j = 0; j < d; ++j) {
      if (levels[j] < 1) return fail(BO_E_INVALID_ARG, "levels[%d] = %d < 1", j, levels[j]);
      total *= levels[j];
      if (total > (__int128(1) << 62)) return fail(BO_E_INVALID_ARG, "grid too large");
    }
    if (!cand && (int64_t)total != N)
      return fail(BO_E_INVALID_ARG, "grid size %lld != N %lld without a candidate list", (long long)total,
                  (long long)N);
  }
  hipLaunchKernelGGL(k_state_clear, dim3(1), dim3(64), 0, s->stream, s->P.st, 0);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_grid_setup(s->P, s->lo, levels, d, cand, X, x_is_f32, invalid, N, s->stream));
  hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)((s->lo.N_pad + 255) / 256)), dim3(256), 0, s->stream, s->P.vis,
                     s->lo.N_pad);
  HIP_TRY(hipGetLastError());
  bo_status rc = sync_state(s);
  if (rc != BO_OK) return rc;
  s->have_fit = 0;
  if (s->hstate->post_status != BO_OK) {
    s->have_cand = 0;
    return fail(BO_E_INVALID_ARG, "candidate grid index out of range");
  }
  s->n_valid = s->hstate->n_unmasked;
  s->have_cand = 1;
  if (n_valid) *n_valid = s->n_valid;
  return BO_OK;
}

bo_status acquire_sync(bo_session* s, const uint8_t* visited, const bo_acq_params* params, bo_acq_result* out,
                       double* ei, double* pi, double* lcb) {
  bo_status rc = step_ready(s);
  if (rc != BO_OK) return rc;
  if (!out) return fail(BO_E_INVALID_ARG, "out is NULL");
  if (!visited) visited = s->P.vis;
  AcqArgs a;
  rc = check_acq(params, &a);
  if (rc != BO_OK) return rc;
  if (s->n_valid == 0) {
    bo_acq_result r{};
    for (int k = 0; k < 3; ++k) {
      r.idx[k] = -1;
      r.score[k] = NAN;
    }
    r.status = BO_E_NO_CANDIDATE;
    *out = r;
    return fail(BO_E_NO_CANDIDATE, "every candidate is invalid");
  }
  for (double* v : {ei, pi, lcb})
    if (v) {
      hipLaunchKernelGGL(k_fill_nan, dim3((unsigned)((s->prob.N + 255) / 256)), dim3(256), 0, s->stream, v,
                         s->prob.N);
      HIP_TRY(hipGetLastError());
    }
  rc = enqueue_step(s, visited, a, s->P.res, ei, pi, lcb);
  if (rc != BO_OK) return rc;
  HIP_TRY(hipMemcpyAsync(s->hres, s->P.res, sizeof(bo_acq_result), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  *out = *s->hres;
  if (out->status != BO_OK) return fail((bo_status)out->status, "step finished with status %d", out->status);
  return BO_OK;
}

}  // namespace

// ---------------------------------------------------------------- layout --
namespace bo {

namespace {
thread_local std::string g_err;
}

void vset_error(const char* fmt, va_list ap) {
  char buf[512];
  vsnprintf(buf, sizeof buf, fmt, ap);
  g_err = buf;
}

bo_status set_error(bo_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vset_error(fmt, ap);
  va_end(ap);
  return s;
}

const char* last_error_text() { return g_err.c_str(); }

bo_status acq_params_check(const bo_acq_params* a, AcqArgs* out) {
  if (!a) return set_error(BO_E_INVALID_ARG, "acq params are NULL");
  if (a->mode != 0 && a->mode != 1) return set_error(BO_E_INVALID_ARG, "acq mode %d is not 0 or 1", a->mode);
  if (a->acq_bits & ~7u) return set_error(BO_E_INVALID_ARG, "unknown acquisition bits 0x%x", a->acq_bits);
  if (a->mode == 0 && !std::isfinite(a->lambda_const)) return set_error(BO_E_INVALID_ARG, "lambda_const is not finite");
  if (a->mode == 1 && !(a->mu_s > 0.0 && std::isfinite(a->mu_s)))
    return set_error(BO_E_INVALID_ARG, "contextual variance needs mu_s > 0");
  if (a->mode == 1 && !std::isfinite(a->var_s_mean)) return set_error(BO_E_INVALID_ARG, "var_s_mean is not finite");
  out->mode = a->mode;
  out->bits = a->acq_bits ? a->acq_bits : 7u;
  out->lambda_const = a->lambda_const;
  out->mu_s = a->mu_s;
  out->var_s_mean = a->var_s_mean;
  return BO_OK;
}


size_t bpk_bytes(int prec, int n_pad) {
  if (prec == BO_BF16X3) {
    const size_t M = n_pad / 64;  // pairs of 32-column blocks, 4(m+1) fragments per block
    return 4 * M * (M + 1) * 64 * 16 * 2;
  }
  const size_t JB = n_pad / 16;  // FP64 values in both modes
  return 2 * JB * (JB + 1) * 64 * 8;
}

bool make_layout(const bo_problem& p, Layout* L) {
  if (!problem_ok(&p)) return false;
  Layout o{};
  o.N = p.N;
  o.N_pad = round_up(p.N, 256);
  o.d = p.d;
  o.n_max = p.n_max;
  o.n_max_pad = n_pad_of(p.n_max);
  o.prec = p.precision;
  o.w16 = aug16_width(p.d);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (size_t)round_up((int64_t)(off + bytes), 256);
    return at;
  };
  const size_t Np = (size_t)o.N_pad, np = (size_t)o.n_max_pad;
  const size_t post_el = p.precision == BO_FP64 ? 8 : 4;
  o.n_vslots = (int64_t)(Np / 16);
  // one slot per acquisition workgroup of a plain step, or per chunk of the
  // batched and served steps (at least 2048 candidates each)
  o.n_aslots = std::max<int64_t>(acquire_blocks(o.N_pad), (o.N_pad + 2047) / 2048);
  o.off_st = take(sizeof(DevState));
  o.off_res = take(sizeof(bo_acq_result));
  o.off_X64 = take((size_t)o.d * Np * 8);
  o.off_Xc16 = take(p.precision == BO_BF16X3 ? Np * 2 * o.w16 * 2 : 0);
  o.off_orig = take(Np * 4);
  o.off_inv = take((size_t)o.N * 4);
  o.off_blk = take(((Np > (size_t)o.N ? Np : (size_t)o.N) / 1024 + 2) * 4);
  o.off_mu = take(Np * post_el);
  o.off_var = take(Np * post_el);
  o.off_vslots = take((size_t)o.n_vslots * sizeof(VarSlot));
  o.off_aslots = take((size_t)o.n_aslots * sizeof(AcqSlot));
  o.off_Xo64 = take(np * kMaxD * 8);
  o.off_Xo16 = take(p.precision == BO_BF16X3 ? np * 2 * o.w16 * 2 : 0);
  o.off_y = take(np * 8);
  o.off_A = take(np * np * 8);
  o.off_L = take(np * np * 8);
  o.off_Dinv = take((np / 64) * 64 * 64 * 8);
  o.off_Linv = take(np * np * 8);
  o.off_alpha = take(np * 8);
  o.off_z = take(np * 8);
  o.off_Bpk = take(bpk_bytes(p.precision, (int)np));
  o.off_obs = take(np * 8);
  o.off_vis = take(Np);
  o.total = off;
  *L = o;
  return true;
}

DevPtrs carve(const Layout& o, uint8_t* b) {
  DevPtrs P{};
  P.st = (DevState*)(b + o.off_st);
  P.res = (bo_acq_result*)(b + o.off_res);
  P.X64 = (double*)(b + o.off_X64);
  P.Xc16 = o.prec == BO_BF16X3 ? (uint16_t*)(b + o.off_Xc16) : nullptr;
  P.orig = (int32_t*)(b + o.off_orig);
  P.inv_map = (int32_t*)(b + o.off_inv);
  P.blk = (int32_t*)(b + o.off_blk);
  P.mu = b + o.off_mu;
  P.var = b + o.off_var;
  P.vslots = (VarSlot*)(b + o.off_vslots);
  P.aslots = (AcqSlot*)(b + o.off_aslots);
  P.Xo64 = (double*)(b + o.off_Xo64);
  P.Xo16 = o.prec == BO_BF16X3 ? (uint16_t*)(b + o.off_Xo16) : nullptr;
  P.y = (double*)(b + o.off_y);
  P.A = (double*)(b + o.off_A);
  P.L = (double*)(b + o.off_L);
  P.Dinv = (double*)(b + o.off_Dinv);
  P.Linv = (double*)(b + o.off_Linv);
  P.alpha = (double*)(b + o.off_alpha);
  P.z = (double*)(b + o.off_z);
  P.Bpk = b + o.off_Bpk;
  P.obs = (int64_t*)(b + o.off_obs);
  P.vis = b + o.off_vis;
  return P;
}

}  // namespace bo

// ------------------------------------------------------------------ C ABI --
extern "C" {

const char* bo_version(void) { return "bo-mi355x 0.1 (gfx950)"; }

const char* bo_last_error(void) { return last_error_text(); }

bo_status bo_workspace_query(const bo_problem* prob, size_t* bytes) {
  if (!bytes) return fail(BO_E_INVALID_ARG, "bytes is NULL");
  Layout L;
  if (!make_layout(*prob, &L))
    return fail(BO_E_INVALID_ARG, "problem outside limits (1 <= N < 2^31, 1 <= d <= 16, 1 <= n_max <= 1024)");
  *bytes = L.total;
  return BO_OK;
}

bo_status bo_session_create(bo_session** out, const bo_problem* prob, const bo_gp_params* gp, void* workspace,
                            size_t bytes, void* stream) {
  if (!out) return fail(BO_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!problem_ok(prob)) return fail(BO_E_INVALID_ARG, "problem outside limits");
  bo_gp_params g;
  bo_status grc = gp_check(gp, &g);
  if (grc != BO_OK) return grc;
  Layout L;
  make_layout(*prob, &L);
  if (!workspace || ((uintptr_t)workspace & 255u)) return fail(BO_E_WORKSPACE, "workspace NULL or not 256-aligned");
  if (bytes < L.total)
    return fail(BO_E_WORKSPACE, "workspace %zu bytes < %zu needed", bytes, L.total);
  bo_session* s = new (std::nothrow) bo_session();
  if (!s) return fail(BO_E_INVALID_ARG, "out of host memory");
  s->prob = *prob;
  s->gp = GpConst{g.nu2, g.jitter_tries, g.lengthscale, g.amp, g.noise};
  s->lo = L;
  s->ws = (uint8_t*)workspace;
  s->ws_bytes = bytes;
  s->P = carve(L, s->ws);
  s->stream = (hipStream_t)stream;
  hipError_t e = hipHostMalloc((void**)&s->hres, sizeof(bo_acq_result), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->hstate, sizeof(DevState), hipHostMallocDefault);
  if (e != hipSuccess) {
    if (s->hres) (void)hipHostFree(s->hres);
    delete s;
    return fail(BO_E_HIP, "hipHostMalloc: %s", hipGetErrorString(e));
  }
  hipLaunchKernelGGL(k_state_clear, dim3(1), dim3(64), 0, s->stream, s->P.st, 1);
  e = hipGetLastError();
  if (e != hipSuccess) {
    (void)hipHostFree(s->hres);
    (void)hipHostFree(s->hstate);
    delete s;
    return fail(BO_E_HIP, "launch: %s", hipGetErrorString(e));
  }
  *out = s;
  return BO_OK;
}

void bo_session_destroy(bo_session* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  if (s->timing)
    for (int i = 0; i < 6; ++i) (void)hipEventDestroy(s->ev[i]);
  (void)hipHostFree(s->hres);
  (void)hipHostFree(s->hstate);
  delete s;
}

bo_status bo_session_set_stream(bo_session* s, void* stream) {
  if (!s) return fail(BO_E_INVALID_ARG, "session is NULL");
  s->stream = (hipStream_t)stream;
  return BO_OK;
}

bo_status bo_set_grid(bo_session* s, const int32_t* levels, const int64_t* cand, const uint8_t* invalid,
                      int64_t* n_valid) {
  return set_candidates(s, levels, cand, nullptr, 0, invalid, n_valid);
}

bo_status bo_set_candidates(bo_session* s, const void* X, int32_t x_is_f32, const uint8_t* invalid,
                            int64_t* n_valid) {
  if (!X) return fail(BO_E_INVALID_ARG, "X is NULL");
  if (x_is_f32 != 0 && x_is_f32 != 1) return fail(BO_E_INVALID_ARG, "x_is_f32 must be 0 or 1");
  return set_candidates(s, nullptr, nullptr, X, x_is_f32, invalid, n_valid);
}

bo_status bo_gp_fit(bo_session* s, const int64_t* obs_idx, const double* y, int32_t n) {
  if (!s) return fail(BO_E_INVALID_ARG, "session is NULL");
  if (!s->have_cand) return fail(BO_E_STATE, "no candidate set");
  if (n < 1) return fail(BO_E_STATE, "a fit needs at least one observation (n = %d)", n);
  if (n > s->prob.n_max) return fail(BO_E_INVALID_ARG, "n = %d exceeds n_max = %d", n, s->prob.n_max);
  if (!obs_idx || !y) return fail(BO_E_INVALID_ARG, "obs_idx or y is NULL");
  s->n = n;
  // one session: the multi-workgroup fit is faster above kPlainSmallMax
  s->large_fit = n > kPlainSmallMax;
  MARK(s, 0);
  if (!s->large_fit)
    HIP_TRY(launch_fit_small(s->P, s->lo, s->gp, obs_idx, y, n, s->stream));
  else
    HIP_TRY(launch_fit_large(s->P, s->lo, s->gp, obs_idx, y, n, 0, s->stream));
  MARK(s, 1);
  s->have_fit = 1;
  return BO_OK;
}

bo_status bo_gp_append(bo_session* s, const int64_t* obs_idx, const double* y, int32_t n) {
  if (!s) return fail(BO_E_INVALID_ARG, "session is NULL");
  if (!s->have_cand) return fail(BO_E_STATE, "no candidate set");
  if (n < 1) return fail(BO_E_STATE, "a fit needs at least one observation (n = %d)", n);
  if (n > s->prob.n_max) return fail(BO_E_INVALID_ARG, "n = %d exceeds n_max = %d", n, s->prob.n_max);
  if (!obs_idx || !y) return fail(BO_E_INVALID_ARG, "obs_idx or y is NULL");
  return append_fit(s, obs_idx, y, n);
}

bo_status bo_observe(bo_session* s, int64_t idx, double y, int32_t valid) {
  if (!s) return fail(BO_E_INVALID_ARG, "session is NULL");
  if (!s->have_cand) return fail(BO_E_STATE, "no candidate set");
  if (idx < 0 || idx >= s->prob.N) return fail(BO_E_INVALID_ARG, "idx %lld outside [0, N)", (long long)idx);
  if (valid != 0 && valid != 1) return fail(BO_E_INVALID_ARG, "valid must be 0 or 1");
  const int n_new = (s->have_fit ? s->n : 0) + 1;
  if (valid) {
    if (!std::isfinite(y)) return fail(BO_E_INVALID_ARG, "y is not finite");
    if (n_new > s->prob.n_max) return fail(BO_E_INVALID_ARG, "n = %d exceeds n_max = %d", n_new, s->prob.n_max);
  }
  hipLaunchKernelGGL(k_observe, dim3(1), dim3(64), 0, s->stream, s->P.vis, s->P.obs, s->P.y, idx, y, valid,
                     n_new - 1);
  HIP_TRY(hipGetLastError());
  if (!valid) return BO_OK;
  return append_fit(s, s->P.obs, s->P.y, n_new);
}

bo_status bo_fit_read(bo_session* s, bo_fit_info* info, double* alpha, double* Linv) {
  if (!s) return fail(BO_E_INVALID_ARG, "session is NULL");
  if (!s->have_fit) return fail(BO_E_STATE, "no fit");
  bo_status rc = sync_state(s);
  if (rc != BO_OK) return rc;
  const DevState& h = *s->hstate;
  if (info) {
    info->status = h.status;
    info->n = h.n;
    info->attempt = h.attempt;
    info->reserved = 0;
    info->jitter = h.jitter;
    info->mean_y = h.mean_y;
    info->f_best = h.f_best;
  }
  const int n = s->n;
  if (alpha) HIP_TRY(hipMemcpy(alpha, s->P.alpha, sizeof(double) * n, hipMemcpyDeviceToHost));
  if (Linv) {
    HIP_TRY(hipMemcpy2D(Linv, sizeof(double) * n, s->P.Linv, sizeof(double) * s->lo.n_max_pad, sizeof(double) * n, n,
                        hipMemcpyDeviceToHost));
    // only the lower triangle of L^-1 is kept on the device
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) Linv[(size_t)i * n + j] = 0.0;
  }
  if (h.status != BO_OK) return fail((bo_status)h.status, "fit failed with status %d", h.status);
  return BO_OK;
}

bo_status bo_posterior(bo_session* s, const uint8_t* visited, double* mu, double* var, double* var_mean) {
  bo_status rc = step_ready(s);
  if (rc != BO_OK) return rc;
  if (!visited) visited = s->P.vis;
  if (s->n_valid == 0) return fail(BO_E_NO_CANDIDATE, "every candidate is invalid");
  AcqArgs a{0, 7u, 0.0, 0.0, 0.0};
  rc = enqueue_posterior(s, visited, a);
  if (rc != BO_OK) return rc;
  if (mu || var) HIP_TRY(launch_scatter_posterior(s->P, s->lo, s->n_valid, visited, mu, var, s->stream));
  if (!var_mean) return BO_OK;
  rc = sync_state(s);
  if (rc != BO_OK) return rc;
  const DevState& h = *s->hstate;
  if (h.status != BO_OK) return fail((bo_status)h.status, "fit failed with status %d", h.status);
  *var_mean = h.var_mean;
  if (h.post_status != BO_OK) return fail((bo_status)h.post_status, "posterior status %d", h.post_status);
  return BO_OK;
}

bo_status bo_acquire(bo_session* s, const uint8_t* visited, const bo_acq_params* params, bo_acq_result* out) {
  return acquire_sync(s, visited, params, out, nullptr, nullptr, nullptr);
}

bo_status bo_acquire_values(bo_session* s, const uint8_t* visited, const bo_acq_params* params, double* ei,
                            double* pi, double* lcb, bo_acq_result* out) {
  return acquire_sync(s, visited, params, out, ei, pi, lcb);
}

bo_status bo_acquire_async(bo_session* s, const uint8_t* visited, const bo_acq_params* params,
                           bo_acq_result* out_dev) {
  bo_status rc = step_ready(s);
  if (rc != BO_OK) return rc;
  if (!out_dev) return fail(BO_E_INVALID_ARG, "out_dev is NULL");
  AcqArgs a;
  rc = check_acq(params, &a);
  if (rc != BO_OK) return rc;
  if (s->n_valid == 0) return fail(BO_E_NO_CANDIDATE, "every candidate is invalid");
  if (!visited) visited = s->P.vis;
  return enqueue_step(s, visited, a, out_dev);
}

bo_status bo_set_timing(bo_session* s, int32_t enable) {
  if (!s) return fail(BO_E_INVALID_ARG, "session is NULL");
  if (enable && !s->timing) {
    for (int i = 0; i < 6; ++i) HIP_TRY(hipEventCreate(&s->ev[i]));
    s->ev_have[0] = s->ev_have[1] = s->ev_have[2] = 0;
    s->timing = 1;
  } else if (!enable && s->timing) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int i = 0; i < 6; ++i) HIP_TRY(hipEventDestroy(s->ev[i]));
    s->timing = 0;
  }
  return BO_OK;
}

bo_status bo_get_timing(bo_session* s, float* fit_ms, float* posterior_ms, float* acquire_ms) {
  if (!s) return fail(BO_E_INVALID_ARG, "session is NULL");
  if (!s->timing) return fail(BO_E_STATE, "timing is not enabled");
  HIP_TRY(hipStreamSynchronize(s->stream));
  float* outs[3] = {fit_ms, posterior_ms, acquire_ms};
  for (int k = 0; k < 3; ++k) {
    if (!outs[k]) continue;
    *outs[k] = -1.f;
    if (s->ev_have[k]) HIP_TRY(hipEventElapsedTime(outs[k], s->ev[2 * k], s->ev[2 * k + 1]));
  }
  return BO_OK;
}

bo_status bo_step_noalloc(const bo_problem* prob, const bo_gp_params* gp, const void* X, int32_t x_is_f32,
                          const uint8_t* invalid, const uint8_t* visited, const int64_t* obs_idx, const double* y,
                          int32_t n, const bo_acq_params* params, bo_acq_result* out, void* stream) {
  if (!out) return fail(BO_E_INVALID_ARG, "out is NULL");
  if (!problem_ok(prob)) return fail(BO_E_INVALID_ARG, "problem outside limits");
  if (!X) return fail(BO_E_INVALID_ARG, "X is NULL");
  if (x_is_f32 != 0 && x_is_f32 != 1) return fail(BO_E_INVALID_ARG, "x_is_f32 must be 0 or 1");
  if (n < 1) return fail(BO_E_STATE, "a fit needs at least one observation (n = %d)", n);
  if (n > prob->n_max) return fail(BO_E_INVALID_ARG, "n = %d exceeds n_max = %d", n, prob->n_max);
  if (!obs_idx || !y) return fail(BO_E_INVALID_ARG, "obs_idx or y is NULL");
  bo_gp_params g;
  bo_status rc = gp_check(gp, &g);
  if (rc != BO_OK) return rc;
  AcqArgs a;
  rc = check_acq(params, &a);
  if (rc != BO_OK) return rc;
  Layout L;
  make_layout(*prob, &L);
  if (L.total > kScratchBytes)
    return fail(BO_E_WORKSPACE, "problem needs %zu bytes of device memory; the static scratch holds %zu", L.total,
                kScratchBytes);
  uint8_t* ws = nullptr;
  rc = scratch_of_current_device(&ws);
  if (rc != BO_OK) return rc;
  // a session on the stack over the scratch array; its host-side copies of
  // the result and the state are stack variables (pageable memory)
  bo_acq_result hres{};
  DevState hstate{};
  bo_session s{};
  s.prob = *prob;
  s.gp = GpConst{g.nu2, g.jitter_tries, g.lengthscale, g.amp, g.noise};
  s.lo = L;
  s.ws = ws;
  s.ws_bytes = kScratchBytes;
  s.P = carve(L, ws);
  s.stream = (hipStream_t)stream;
  s.hres = &hres;
  s.hstate = &hstate;
  // the array keeps the previous call's contents: start from a cleared state
  hipLaunchKernelGGL(k_state_clear, dim3(1), dim3(64), 0, s.stream, s.P.st, 1);
  HIP_TRY(hipGetLastError());
  rc = set_candidates(&s, nullptr, nullptr, X, x_is_f32, invalid, nullptr);
  if (rc != BO_OK) return rc;
  rc = bo_gp_fit(&s, obs_idx, y, n);
  if (rc != BO_OK) return rc;
  return acquire_sync(&s, visited, params, out, nullptr, nullptr, nullptr);
}

}  // extern "C"
