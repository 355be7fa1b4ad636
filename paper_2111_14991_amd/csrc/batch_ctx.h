// One launch context of the batched step (the graph of kernels in
// k_batch.hip): device plan and results in a caller-owned workspace, pinned
// host mirrors, a stream and the captured graph.  Used by
// the bo_batch entry points and by the server, which keeps one context per
// stream so that launches overlap.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "bo_internal.h"
#include "session_impl.h"

namespace bo {

// One session's step in a launch.
struct BatchItem {
  bo_session* s;
  const int64_t* obs_idx;  // device, n entries (position n - 1 written first when write_obs)
  const double* y;
  int32_t n;
  int32_t fit_kind;        // 0: full fit, 1: rank-1 append, 2: keep the current fit
  const uint8_t* visited;  // device uint8[N] or NULL
  AcqArgs acq;
  int32_t write_obs;
  int32_t pad;
  int64_t new_idx;
  double new_y;
  uint8_t* mark;           // device, nullable: mark[new_idx] = 1 before the fit
};

constexpr int kBatchNodes = 6;  // fits, posterior (two classes), exploration factors, chunks, selections

class BatchCtx {
 public:
  static size_t bytes(int cap);
  bo_status init(int cap, void* workspace, size_t nbytes, hipStream_t stream);
  void destroy();
  bo_status set_timing(int enable);
  // Writes the plan and replays the graph (captured on first use); returns
  // without waiting.  The previous launch of this context must be finished.
  bo_status launch(const BatchItem* items, int count, const bo_batch_config& cfg);
  bool done() const;
  // Waits for the launch and copies its `count` results.
  bo_status finish(bo_acq_result* out, float* ms);

  int cap = 0, grid = 0, timing = 0, own_stream = 0, have_graph = 0, n_last = 0;
  hipStream_t stream = nullptr;

 private:
  bo_status build_plan(const BatchItem* items, int count, const bo_batch_config& cfg);
  bo_status capture();
  unsigned char* plan_dev = nullptr;
  bo_acq_result* res_dev = nullptr;
  unsigned char* plan_host = nullptr;
  unsigned char* res_host = nullptr;
  size_t plan_sz = 0, res_sz = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t knode[kBatchNodes] = {};  // the kernel nodes, in launch order
  unsigned kgrid[kBatchNodes] = {};        // their grids in the instantiated graph
  unsigned grids[kBatchNodes] = {};        // the grids the current plan needs
  unsigned char* karg_plan = nullptr;      // kernel arguments (stable addresses)
  int karg_cap = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t done_ev = nullptr;
  std::vector<int> order_scratch;
};

}  // namespace bo
