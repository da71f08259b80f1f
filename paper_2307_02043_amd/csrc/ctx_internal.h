// The Lippmann-Schwinger context (shared with the outer-iteration driver,
// which checks its geometry and precision).
#pragma once
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/bq.h"
#include "bq_kernels.h"

struct bq_ctx {
  bq_geom g{};
  int L = 0;
  std::vector<bq_illum> dirs;
  std::vector<bq::C<double>> inc_tab;  // plane-wave factors per illumination, L x 3 x N
  hipStream_t stream = nullptr;
  std::string err;
  double kb = 0.0;
  size_t V = 0;
  size_t csz = 0;  // bytes per complex element
  int np_mv = 0, np_vec = 0, np_det = 0;
  int Bcap = 0;
  // device memory
  void* ghat = nullptr;
  void* twN = nullptr;
  void* twH = nullptr;
  void* dettab = nullptr;  // detector transfer function / N^2 (N x N, [ky][kx]) when det_dist_um > 0
  // camera (cam_n > 0): ndet = cam_n pixels per side, else the N x N window
  int ndet = 0;
  void* camD = nullptr;    // M x N trigonometric interpolation matrix (camera)
  void* camwin = nullptr;  // B window images (N x N) between the field and the camera
  void* camtmp = nullptr;  // B intermediate products (N x M)
  void* f[8] = {};  // u w r rhat p v s t
  void* zh = nullptr;
  void* xh = nullptr;
  void* rdet = nullptr;
  bq::C<double>* inc = nullptr;
  bq::SysState* state = nullptr;
  double* part_mv = nullptr;
  double* part_vec = nullptr;
  double* part_det = nullptr;
  // pinned host staging (hipHostMalloc), sized with the batch capacity
  bq::SysState* hstate = nullptr;
  bq::C<double>* hinc = nullptr;
  double* hpart = nullptr;
  bq::PassTimer timer;
  // iterations the previous batched forward / adjoint solve took: the next
  // solve checks for convergence first after that many iterations, then
  // after every iteration (0: no history, check every 4)
  int hint[2] = {0, 0};
  // launch shapes of the FFT passes (0: default), set by bq_autotune or
  // bq_set_plan; they change no value any call computes
  int plan_xtile = 0, plan_zf = 0;
  // magnitude of rho, <rhat, v> or omega below which BiCGSTAB reports a
  // breakdown (bq_set_breakdown_floor)
  double brk = 1e-300;
  // systems per launch set (0: as many as the free device memory holds);
  // larger batches run as consecutive sub-batches
  int batch_limit = 0;
  // BQ_FLAG_GRAPH: one BiCGSTAB iteration of the batched path captured as a
  // HIP graph per (batch size, potential, solution, incident table, launch
  // shapes of the FFT passes) and replayed on a stream of the library's own
  // (a graph cannot be captured on the legacy null stream a caller may use),
  // ordered after the caller's stream by an event.  Dropped whenever the
  // batch buffers change and after bq_autotune.
  struct IterGraph {
    int B;
    const void* x;
    const void* e;
    const void* inc;
    int xtile, zf;  // plan_xtile / plan_zf the graph was captured under
    hipGraphExec_t exec;
  };
  std::vector<IterGraph> graphs;
  long long graph_captures = 0;  // iteration graphs captured since creation
  hipStream_t gstream = nullptr;
  hipEvent_t gev = nullptr;
};

