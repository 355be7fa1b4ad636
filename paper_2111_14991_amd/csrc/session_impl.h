// Host-side state of a session, shared by the single-session, batched and
// serving entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>

#include "bo_internal.h"

struct bo_session {
  bo_problem prob;
  bo::GpConst gp;
  bo::Layout lo;
  bo::DevPtrs P;
  hipStream_t stream;
  uint8_t* ws;
  size_t ws_bytes;
  int64_t n_valid;
  int have_cand;
  int have_fit;
  int n;
  int large_fit;        // the current fit runs on the multi-workgroup path
  bo_acq_result* hres;  // pinned host copy of the device result
  bo::DevState* hstate;     // pinned host copy of the device state
  int timing;
  hipEvent_t ev[6];     // fit begin/end, posterior begin/end, acquire begin/end
  int ev_have[3];
};

namespace bo {
// Thread-local last-error text of the C ABI.
void vset_error(const char* fmt, va_list ap);
bo_status set_error(bo_status s, const char* fmt, ...);
const char* last_error_text();
// Validates acquisition parameters (bo_acq_params) into kernel arguments.
bo_status acq_params_check(const bo_acq_params* a, AcqArgs* out);
}  // namespace bo
