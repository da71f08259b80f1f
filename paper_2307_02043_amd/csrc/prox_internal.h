// Internals shared by the two weighted-prox implementations (metric
// rank <= 1 in prox.hip, rank >= 2 in prox_rank.hip).
#pragma once
#include <algorithm>
#include <string>

#include <hip/hip_runtime.h>

#include "../../include/bq.h"
#include "bq_common.h"

namespace bq {
struct ProxState;
struct ProxRankState;
}  // namespace bq

struct bq_prox {
  int nz = 0, ny = 0, nx = 0, prec = 0;
  size_t V = 0;
  hipStream_t stream = nullptr;  // caller's stream
  hipStream_t own = nullptr;     // library stream (capturable), default priority
  hipEvent_t ev = nullptr;
  std::string err;
  void* a = nullptr;
  void* P = nullptr;
  void* R = nullptr;
  double* partial = nullptr;     // np x PX_PART doubles
  void* Pbak = nullptr;          // copy of a caller's starting dual point (3V), for a rerun
  void* R2 = nullptr;            // second momentum buffer (3V) of the metric-tau-I path, on first use
  bq::ProxState* st = nullptr;
  bq::ProxRankState* rst = nullptr;
  int np = 0;
  int max_passes = 8;       // evaluations of phi per dual iteration, rank <= 1 (1 fused + 7 passes)
  int ssn_slots = 2;        // root passes launched per dual iteration, rank <= 1 (up to max_passes - 1)
  int ssn_slots_rank = 2;   // the same for rank >= 2 (up to max_passes_rank - 1)
  int max_passes_rank = 12;  // the same for rank >= 2 (Newton steps and backtracking)
  // Launch every kernel directly on `own` instead of replaying a captured
  // graph (instantiating one may allocate): set for the workspace the
  // no-allocation entry point builds over its static scratch array, whose
  // `own` is the caller's stream and which has no event.
  bool direct = false;
};

namespace bq {
constexpr int PX_PART = 64;  // partial-sum slots per workgroup
constexpr int PX_MAX_RANK = 8;

// Most dual iterations find their root within one or two evaluations, so a
// call first launches slots_pref root passes per dual iteration.  once(slots,
// &overflow, &seen) runs the whole iteration; if some dual iteration needed
// more passes (overflow) the call is run again from the caller's starting
// dual point with all `full` passes, so the result is always that of the
// full budget.  The object then keeps the observed need plus one spare pass.
template <class Once>
bq_status run_with_pass_budget(bq_prox* p, void* P_io, size_t bytes3, bool root, int& slots_pref, int full,
                               Once once) {
  int slots = root ? std::max(1, std::min(slots_pref, full)) : 0;
  if (P_io && root && slots < full) {  // keep the starting dual point for a rerun
    if (!p->Pbak && hipMalloc(&p->Pbak, bytes3) != hipSuccess) {
      p->Pbak = nullptr;
      (void)hipGetLastError();
      slots = full;  // no room for the copy: launch every pass
    } else if (hipMemcpyAsync(p->Pbak, P_io, bytes3, hipMemcpyDeviceToDevice, p->own) != hipSuccess) {
      p->err = "copy of the starting dual point failed";
      return BQ_EDEVICE;
    }
  }
  int overflow = 0, seen = 0;
  bq_status st = once(slots, &overflow, &seen);
  if (st == BQ_OK && overflow) {
    if (P_io && hipMemcpyAsync(P_io, p->Pbak, bytes3, hipMemcpyDeviceToDevice, p->own) != hipSuccess) {
      p->err = "restore of the starting dual point failed";
      return BQ_EDEVICE;
    }
    st = once(full, &overflow, &seen);
  }
  if (st == BQ_OK && root) slots_pref = std::max(2, std::min(full, seen));
  return st;
}

// z chunk per thread of the column-walking dual kernels (workgroups of wg
// threads walking (y, x) columns through zc planes) and their grid: about
// 2^18 columns-times-chunks in flight (8 planes at 128^3, 32 at 256^3: the
// best of 2..32 measured), at least 2; the grid covers the (chunk, y) rows,
// a multiple of the XCD count.
struct ZWalk {
  int zc;
  dim3 grid;
};
inline ZWalk zwalk_shape(const bq_prox* p, int wg) {
  int zc = 2;
  while (zc < 32 && (size_t)zc * 2 * 262144 <= p->V) zc *= 2;
  const size_t rows = (size_t)((p->nz + zc - 1) / zc) * p->ny;
  const size_t rps = p->nx >= wg ? 1 : (size_t)(wg / p->nx);
  size_t g0 = std::min<size_t>((rows + rps - 1) / rps, 2048);
  if (g0 >= NUM_XCD) g0 = (g0 + NUM_XCD - 1) / NUM_XCD * NUM_XCD;
  return {zc, dim3((unsigned)g0)};
}

// Runs body(stream) `count` times on p->own: one capture replayed as a graph,
// or direct launches for a workspace that may not allocate.  False if the
// capture, the instantiation or a launch failed.
template <class Body>
bool replay_iterations(bq_prox* p, int count, Body body) {
  if (count <= 0) return true;
  const hipStream_t s = p->own;
  if (p->direct) {
    for (int k = 0; k < count; ++k) body(s);
    return hipGetLastError() == hipSuccess;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    body(s);
    ok = hipStreamEndCapture(s, &graph) == hipSuccess && graph != nullptr;
  }
  ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
  for (int k = 0; ok && k < count; ++k) ok = hipGraphLaunch(exec, s) == hipSuccess;
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (!ok) (void)hipGetLastError();
  return ok;
}

// Orders the library stream after the work pending on the caller's stream
// (nothing to do when they are the same stream).
inline bool order_after_caller(bq_prox* p) {
  if (p->own == p->stream || !p->ev) return true;
  return hipEventRecord(p->ev, p->stream) == hipSuccess && hipStreamWaitEvent(p->own, p->ev, 0) == hipSuccess;
}

template <typename T>
bq_status run_wprox_rank(bq_prox* p, const void* v, double tau, const void* U, int r, double lam, int tv,
                         int cset, int n_iter, void* x_out, void* P_io, bq_prox_stats* stats);
size_t prox_rank_state_bytes();
}  // namespace bq
