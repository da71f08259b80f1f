// Internals shared by the two weighted-prox implementations (metric
// rank <= 1 in prox.hip, rank >= 2 in prox_rank.hip).
#pragma once
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
  bq::ProxState* st = nullptr;
  bq::ProxRankState* rst = nullptr;
  int np = 0;
  int max_passes = 8;       // evaluations of phi per dual iteration, rank <= 1 (1 fused + 7 passes)
  int max_passes_rank = 12;  // the same for rank >= 2 (Newton steps and backtracking)
};

namespace bq {
constexpr int PX_PART = 64;  // partial-sum slots per workgroup
constexpr int PX_MAX_RANK = 8;

template <typename T>
bq_status run_wprox_rank(bq_prox* p, const void* v, double tau, const void* U, int r, double lam, int tv,
                         int cset, int n_iter, void* x_out, void* P_io, bq_prox_stats* stats);
size_t prox_rank_state_bytes();
}  // namespace bq
