// Internals shared by the two weighted-prox implementations (metric
// rank <= 1 in prox.hip, rank >= 2 in prox_rank.hip).
#pragma once
#include <algorithm>
#include <string>

#include <hip/hip_runtime.h>

#include "../../include/bq.h"

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
  void* xbuf = nullptr;          // x(R) for metrics of rank >= 2
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

template <typename T>
bq_status run_wprox_rank(bq_prox* p, const void* v, double tau, const void* U, int r, double lam, int tv,
                         int cset, int n_iter, void* x_out, void* P_io, bq_prox_stats* stats);
size_t prox_rank_state_bytes();
}  // namespace bq
