// Host-side declarations of the kernel launchers of the bq library.
#pragma once

#include <cmath>
#include <vector>

#include "bq_state.h"

namespace bq {

// exp(-2 pi i k / len) style twiddles are built on the host in long double
// and rounded once, so FP32 and FP64 tables are correctly rounded.
inline double cospi_host(double a) { return (double)cosl(3.14159265358979323846264338327950288L * (long double)a); }
inline double sinpi_host(double a) { return (double)sinl(3.14159265358979323846264338327950288L * (long double)a); }

// ---- device timing of passes (HIP events on the launch stream) -------------
enum PassId { P_ZF = 0, P_XF, P_YC, P_XI, P_ZI, P_XY, P_VEC, P_COUNT };

struct PassTimer {
  bool on = false;
  unsigned mask = 0;  // passes timed (bit p for pass p)
  std::vector<hipEvent_t> ev;
  std::vector<std::pair<int, size_t>> rec;  // (pass, index of the start event)
  size_t next = 0;
  double total_ms[P_COUNT] = {};
  long long count[P_COUNT] = {};
  int open_pass = -1;

  void start(int pass, hipStream_t s) {
    if (!on || !((mask >> pass) & 1u)) return;
    while (ev.size() < next + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
      ev.push_back(e);
    }
    (void)hipEventRecord(ev[next], s);
    rec.push_back({pass, next});
    open_pass = pass;
    next += 2;
  }
  void stop(hipStream_t s) {
    if (!on || open_pass < 0) return;
    (void)hipEventRecord(ev[rec.back().second + 1], s);
    open_pass = -1;
  }
  // call after the stream has been synchronised
  void collect() {
    for (auto& r : rec) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[r.second], ev[r.second + 1]) == hipSuccess) {
        total_ms[r.first] += ms;
        count[r.first] += 1;
      }
    }
    rec.clear();
    next = 0;
  }
  // at the host synchronisation points of a call: read the events back only
  // once many are pending, so that timing adds no per-call host work
  void maybe_collect() {
    if (rec.size() >= 4096) collect();
  }
  void reset() {
    for (int i = 0; i < P_COUNT; ++i) { total_ms[i] = 0.0; count[i] = 0; }
    rec.clear();
    next = 0;
  }
  ~PassTimer() { for (auto e : ev) (void)hipEventDestroy(e); }
};

// ---- Green's operator ----------------------------------------------------
template <typename T> int green_apply(const PassArgs<T>& a, hipStream_t st, PassTimer* tm = nullptr);
template <typename T> int green_num_partials(int N);
template <typename T> bool xy_fused_supported(int N);
template <typename T> bool reg_supported(int N);
template <typename T, int N> void launch_xf_stockham(const PassArgs<T>& a, hipStream_t st);
template <typename T, int N> void launch_xi_stockham(const PassArgs<T>& a, hipStream_t st);
template <typename T> int reg_apply(const PassArgs<T>& a, hipStream_t st, PassTimer* tm);
// the padded register z and y passes of a grid whose x passes are the LDS
// Stockham ones (N = 96, complex64); false (nothing launched) otherwise;
// pad_num_partials: the z-inverse partials per system then, else -1
template <typename T> bool pad_zf_apply(const PassArgs<T>& a, hipStream_t st);
template <typename T> bool pad_y_apply(const PassArgs<T>& a, hipStream_t st);
template <typename T> bool pad_zi_apply(const PassArgs<T>& a, hipStream_t st);
template <typename T> int pad_num_partials(int N);
template <typename T>
int reg_num_partials(int N);
// launch shapes the autotuner may choose (valid for this size and precision)
template <typename T> bool xtile_valid(int N, int rows);
template <typename T> bool zf_threads_valid(int N, int threads);
template <typename T> int xy_fused_launch(const PassArgs<T>& a, hipStream_t st);
template <typename T> int ghat_precompute(int N, double h, double kb, C<T>* out, hipStream_t st);
template <typename T>
int plane_propagate(int B, int N, C<T>* planes, const C<T>* twN, const C<T>* tf, int adjoint, hipStream_t st);
// camera sampling D f D^T of B window images (N x N) into M x M, and its adjoint
template <typename T>
void camera_apply(int B, int N, int M, const C<T>* win, const C<T>* D, C<T>* tmp, C<T>* out, hipStream_t st);
template <typename T>
void camera_adjoint(int B, int N, int M, const C<T>* r, const C<T>* D, C<T>* tmp, C<T>* win, hipStream_t st);
int ghat_oversampling(int N);

// ---- BiCGSTAB and the data term -------------------------------------------
constexpr int VEC_WG = 256;  // threads per workgroup of the vector kernels
int vec_num_partials(size_t V);

template <typename T> struct VecArgs {
  int B;
  size_t V;
  int N;
  SysState* state;
  C<T>* e;       // iterate (u or w-bar)
  C<T>* r;
  C<T>* rhat;
  C<T>* p;
  C<T>* v;
  C<T>* s;
  C<T>* t;
  double* partial;  // B x NPV x 4
};

template <typename T> void vec_s(const VecArgs<T>& a, hipStream_t st);
template <typename T> void vec_xr(const VecArgs<T>& a, hipStream_t st);
template <typename T> void vec_norm(const VecArgs<T>& a, const C<T>* f, hipStream_t st);
template <typename T> void vec_fill_incident(int B, int N, const C<double>* inc, C<T>* out, hipStream_t st);
template <typename T> void vec_zero_if_b0(int B, size_t V, const SysState* st, C<T>* e, hipStream_t s);
template <typename T>
void det_residual(int B, int N, C<T>* rdet, const C<T>* ymeas, double* partial, int np, hipStream_t st);

void sc_init(int B, SysState* st, const double* part_r, int np_r, const double* part_b, int np_b,
             double bnorm2_fixed, double tol, int max_iter, double brk, hipStream_t s);
void sc_beta(int B, SysState* st, const double* part, int np, hipStream_t s);
void sc_alpha(int B, SysState* st, const double* part, int np, hipStream_t s);
void sc_s(int B, SysState* st, const double* part, int np, hipStream_t s);
void sc_omega(int B, SysState* st, const double* part, int np, hipStream_t s);

// Detector: H = S(field - u_in) (subtract_uin) or S(field); if ymeas is given
// writes r = H - y to out and FP64 partials of |r|^2 / 2, else writes H.
template <typename T>
void detector(int B, int N, const C<T>* field, int subtract_uin, const C<double>* inc,
              const C<T>* ymeas, C<T>* out, double* partial, int np, hipStream_t st);
int det_num_partials(int N);

// g (+)= scale * sum_b Re(u_b . wbar_b); u_b generated from inc if u == null.
template <typename T>
void gradient(int B, int N, const C<T>* u, const C<double>* inc, const C<T>* wbar, double scale,
              int accumulate, T* g, hipStream_t st);

}  // namespace bq
