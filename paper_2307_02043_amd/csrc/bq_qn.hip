// Outer iteration of the mini-batch quasi-Newton proximal method
// (Algorithm 4.1 with the choices of Section 4.3) on top of the library's
// mini-batch gradient (bq_grad) and weighted prox (bq_wprox).
//
// Per iteration k with chosen subset s':
//   g = grad F_{s'}(x_{k-1})                                  (bq_grad, scale S/L)
//   revisited subset: (tau_s', u_s') by Algorithm 4.2 from
//     s = x_{k-1} - xbar_s', m = g - gbar_s'  (FP64 inner products on the GPU,
//     the scalar branches of the listing on the host)
//   xbar_s' = x_{k-1}, gbar_s' = g
//   k <= S: x_k = WPM(x_{k-1} - (a / alpha) g; alpha I, a lambda)
//   k >  S: Btilde = tau* I + U U^T, tau* = sum_s tau_s, U = [u_1 .. u_S]
//           v = x_{k-1} - a S Btilde^-1 g (Woodbury, S x S solve on the host)
//           x_k = WPM(v; Btilde, a S lambda)
// State per subset: xbar_s, gbar_s, u_s (3S images) and tau_s; with warm
// starts also the forward and adjoint fields of the subset's illuminations,
// from which its next solves start (bq_grad_ws).  The first-order variant
// takes the k <= S step at every iteration.
#include <cmath>
#include <string>
#include <vector>

#include "../../include/bq.h"
#include "bq_common.h"
#include "ctx_internal.h"
#include "prox_internal.h"

namespace bq {

constexpr int QN_WG = 256;
constexpr int QN_RM = BQ_PROX_MAX_RANK;
constexpr int QN_NT = QN_RM * (QN_RM + 1) / 2;  // Gram upper triangle slots
constexpr int QN_K = QN_NT + QN_RM;             // + U^T g
constexpr double QN_DELTA1 = 1e-8, QN_DELTA2 = 1e-12;

__host__ __device__ constexpr int qn_tri(int i, int j) { return i * QN_RM - i * (i - 1) / 2 + (j - i); }

// mode 0: <m,m>, <s,m>, <s,s>;  mode 1: <r,s>, <r,r> with r = m - tau s;
// s = x - xb, m = g - gb formed in FP64
template <typename T>
__global__ void __launch_bounds__(QN_WG) k_qn_pair(const T* x, const T* xb, const T* g, const T* gb, size_t V,
                                                    double tau, int mode, double* part) {
  __shared__ double scratch[(QN_WG / 64) * 3];
  double acc[3] = {0.0, 0.0, 0.0};
  for (size_t i = blockIdx.x * (size_t)QN_WG + threadIdx.x; i < V; i += (size_t)gridDim.x * QN_WG) {
    const double s = (double)x[i] - (double)xb[i];
    const double m = (double)g[i] - (double)gb[i];
    if (mode == 0) {
      acc[0] += m * m;
      acc[1] += s * m;
      acc[2] += s * s;
    } else {
      const double r = m - tau * s;
      acc[0] += r * s;
      acc[1] += r * r;
    }
  }
  block_sum<QN_WG, 3>(acc, scratch);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) part[(size_t)blockIdx.x * QN_K + k] = acc[k];
}

// u = (m - tau s) * inv
template <typename T>
__global__ void __launch_bounds__(QN_WG) k_qn_ucol(const T* x, const T* xb, const T* g, const T* gb, size_t V,
                                                    double tau, double inv, T* u) {
  for (size_t i = blockIdx.x * (size_t)QN_WG + threadIdx.x; i < V; i += (size_t)gridDim.x * QN_WG) {
    const double s = (double)x[i] - (double)xb[i];
    const double m = (double)g[i] - (double)gb[i];
    u[i] = (T)((m - tau * s) * inv);
  }
}

template <typename T>
__global__ void k_qn_fill(T* d, size_t n, T val) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    d[i] = val;
}

// Gram matrix U^T U (upper triangle) and U^T g of the S columns
template <typename T>
__global__ void __launch_bounds__(QN_WG) k_qn_gram(const T* U, int S, const T* g, size_t V, double* part) {
  __shared__ double scratch[(QN_WG / 64) * QN_K];
  double acc[QN_K];
#pragma unroll
  for (int k = 0; k < QN_K; ++k) acc[k] = 0.0;
  for (size_t i = blockIdx.x * (size_t)QN_WG + threadIdx.x; i < V; i += (size_t)gridDim.x * QN_WG) {
    double u[QN_RM];
#pragma unroll
    for (int c = 0; c < QN_RM; ++c) u[c] = c < S ? (double)U[(size_t)c * V + i] : 0.0;
    const double gv = (double)g[i];
#pragma unroll
    for (int c = 0; c < QN_RM; ++c) {
#pragma unroll
      for (int e = c; e < QN_RM; ++e) acc[qn_tri(c, e)] += u[c] * u[e];
      acc[QN_NT + c] += u[c] * gv;
    }
  }
  block_sum<QN_WG, QN_K>(acc, scratch);
  if (threadIdx.x == 0)
    for (int k = 0; k < QN_K; ++k) part[(size_t)blockIdx.x * QN_K + k] = acc[k];
}

// out[k] = sum over the np workgroup rows (fixed order), k < K
__global__ void __launch_bounds__(256) k_qn_sum(const double* part, int np, int K, double* out) {
  __shared__ double scratch[4];
  for (int k = 0; k < K; ++k) {
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < np; i += 256) v[0] += part[(size_t)i * QN_K + k];
    block_sum<256, 1>(v, scratch);
    if (threadIdx.x == 0) out[k] = v[0];
  }
}

struct QnCoef {
  double w[QN_RM];
};

// v = x - c1 g + sum_c w_c U_c
template <typename T>
__global__ void __launch_bounds__(QN_WG) k_qn_v(const T* x, const T* g, const T* U, int S, double c1, QnCoef w, T* v,
                                                 size_t V) {
  for (size_t i = blockIdx.x * (size_t)QN_WG + threadIdx.x; i < V; i += (size_t)gridDim.x * QN_WG) {
    double acc = (double)x[i] - c1 * (double)g[i];
    for (int c = 0; c < S; ++c) acc += w.w[c] * (double)U[(size_t)c * V + i];
    v[i] = (T)acc;
  }
}

}  // namespace bq

using namespace bq;

struct bq_qn {
  bq_ctx* ls = nullptr;
  bq_prox* px = nullptr;
  bq_qn_params prm{};
  std::vector<int> idx, off, len;
  int N = 0, L = 0, prec = 0, S = 0, np = 0, k = 0, maxlen = 0;
  size_t V = 0, es = 0, csz = 0;
  hipStream_t stream = nullptr;
  void* xbar = nullptr;
  void* gbar = nullptr;
  void* U = nullptr;
  void* Uc = nullptr;  // the kept columns of U, packed (when only some are kept)
  void* g = nullptr;
  void* v = nullptr;
  void* ybuf = nullptr;
  void* ufields = nullptr;  // warm start: per subset, its illuminations' forward fields
  void* wfields = nullptr;  // and conjugated adjoint fields
  double* part = nullptr;
  double* res = nullptr;
  double* hres = nullptr;  // pinned
  std::vector<double> tau;
  std::vector<int> seen, kept;
  std::string err;
};

namespace {

thread_local std::string g_qn_create_error;

void free_qn(bq_qn* q) {
  if (!q) return;
  void* ptrs[] = {q->xbar, q->gbar, q->U, q->Uc, q->g, q->v, q->ybuf, q->ufields, q->wfields, q->part, q->res};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (q->hres) (void)hipHostFree(q->hres);
  delete q;
}

bq_status qn_fail(bq_qn* q, bq_status s, const std::string& m) {
  q->err = m;
  return s;
}

// reduce `K` slots of the partials and bring them to q->hres
bq_status qn_reduce(bq_qn* q, int K) {
  hipLaunchKernelGGL(k_qn_sum, dim3(1), dim3(256), 0, q->stream, (const double*)q->part, q->np, K, q->res);
  if (hipMemcpyAsync(q->hres, q->res, K * sizeof(double), hipMemcpyDeviceToHost, q->stream) != hipSuccess ||
      hipStreamSynchronize(q->stream) != hipSuccess)
    return qn_fail(q, BQ_EDEVICE, "device error in a reduction of the outer iteration");
  return BQ_OK;
}

template <typename T>
bq_status qn_pair(bq_qn* q, const T* x, const T* xb, const T* g, const T* gb, double tau, int mode) {
  hipLaunchKernelGGL((k_qn_pair<T>), dim3(q->np), dim3(QN_WG), 0, q->stream, x, xb, g, gb, q->V, tau, mode,
                     q->part);
  return qn_reduce(q, mode == 0 ? 3 : 2);
}

// SR1 metric tau I + u u^T of subset sp (Algorithm 4.2) from its pair
// s = x - xbar, m = g - gbar.  Along r(tau) = m - tau s the curvature
// <r, s> = <m, s> - tau <s, s> is linear in tau and <r, r> = <m, m> -
// 2 tau <m, s> + tau^2 <s, s>, so after the three inner products of the
// pair (and <r, s>, <r, r> at the first tau, reduced from the vectors) the
// halvings of tau that the curvature condition <r, s> > delta2 <s, s> asks
// for are found on the host from the closed form, with no further pass
// over the images.  The kept correction u = r / sqrt(<r, s>) is normalised
// by <r, s> reduced once more at the final tau; should that exact value
// still fail the condition (the closed form having cancelled), the halving
// goes on with reduced values.
template <typename T>
bq_status qn_sr1(bq_qn* q, int sp, const T* x, const T* g) {
  const size_t V = q->V;
  const T* xb = (const T*)q->xbar + (size_t)sp * V;
  const T* gb = (const T*)q->gbar + (size_t)sp * V;
  T* u = (T*)q->U + (size_t)sp * V;
  if (bq_status s = qn_pair<T>(q, x, xb, g, gb, 0.0, 0)) return s;
  const double mm = q->hres[0], sm = q->hres[1], ss = q->hres[2];
  if (!(ss > 0.0)) return BQ_OK;  // same iterate as the stored pair: keep the metric
  const double alpha = q->prm.alpha;
  double tau = std::fmin(mm / (q->prm.gamma * sm), q->prm.tau_max);
  bool keep = false;
  if (!(tau > 0.0)) {
    tau = alpha;
  } else {
    if (bq_status s = qn_pair<T>(q, x, xb, g, gb, tau, 1)) return s;
    const double rs0 = q->hres[0], rr0 = q->hres[1];
    // a correction whose curvature is negligible against |r| |s| is
    // dropped (tau kept); otherwise halve tau until <r, s> > delta2 <s, s>
    if (rs0 > QN_DELTA1 * std::sqrt(ss) * std::sqrt(rr0)) {
      keep = true;
      const double tau0 = tau;
      double rs = rs0;
      bool exact = true;  // rs reduced from the vectors at this tau
      for (;;) {
        if (rs > QN_DELTA2 * ss) {
          if (exact) break;
          if (bq_status s = qn_pair<T>(q, x, xb, g, gb, tau, 1)) return s;
          rs = q->hres[0];
          exact = true;
          continue;
        }
        if (tau < QN_DELTA2) {  // no usable curvature along r
          tau = alpha;
          keep = false;
          break;
        }
        tau *= 0.5;
        rs = rs0 + (tau0 - tau) * ss;  // <m - tau s, s> from its value at tau0
        exact = false;
      }
      if (keep)
        hipLaunchKernelGGL((k_qn_ucol<T>), dim3(q->np), dim3(QN_WG), 0, q->stream, x, xb, g, gb, V, tau,
                           1.0 / std::sqrt(rs), u);
    }
  }
  if (!keep) hipLaunchKernelGGL((k_qn_fill<T>), dim3(q->np), dim3(QN_WG), 0, q->stream, u, V, T(0));
  q->tau[sp] = tau;
  q->kept[sp] = keep ? 1 : 0;
  return BQ_OK;
}

// Cholesky solve of the SPD S x S system M c = b (host, FP64)
void qn_chol_solve(std::vector<double> M, int S, const double* b, double* c) {
  for (int j = 0; j < S; ++j) {
    double d = M[j * S + j];
    for (int k = 0; k < j; ++k) d -= M[j * S + k] * M[j * S + k];
    d = std::sqrt(d);
    M[j * S + j] = d;
    for (int i = j + 1; i < S; ++i) {
      double s = M[i * S + j];
      for (int k = 0; k < j; ++k) s -= M[i * S + k] * M[j * S + k];
      M[i * S + j] = s / d;
    }
  }
  std::vector<double> y(S);
  for (int i = 0; i < S; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= M[i * S + k] * y[k];
    y[i] = s / M[i * S + i];
  }
  for (int i = S - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < S; ++k) s -= M[k * S + i] * c[k];
    c[i] = s / M[i * S + i];
  }
}

template <typename T>
bq_status qn_step(bq_qn* q, void* xv, const void* y, int pick, bq_qn_info* info) {
  const int S = q->S;
  const size_t V = q->V;
  const bq_qn_params& p = q->prm;
  const int k = q->k + 1;
  int sp;
  if (k <= S) sp = k - 1;
  else if (pick < 0) sp = (k - 1) % S;
  else sp = pick;
  T* x = (T*)xv;
  T* g = (T*)q->g;
  T* v = (T*)q->v;
  // measurements of the subset, gathered in its index order
  const size_t row = (size_t)q->ls->ndet * q->ls->ndet * q->csz;
  for (int i = 0; i < q->len[sp]; ++i)
    if (hipMemcpyAsync((char*)q->ybuf + i * row, (const char*)y + (size_t)q->idx[q->off[sp] + i] * row, row,
                       hipMemcpyDeviceToDevice, q->stream) != hipSuccess)
      return qn_fail(q, BQ_EDEVICE, "gather of the subset measurements failed");
  if (hipStreamSynchronize(q->stream) != hipSuccess) return qn_fail(q, BQ_EDEVICE, "device error");
  double loss = 0.0;
  bq_status sg;
  if (p.warm_start) {
    const size_t fo = (size_t)q->off[sp] * V * q->csz;
    sg = bq_grad_ws(q->ls, x, q->ybuf, &q->idx[q->off[sp]], q->len[sp], (double)S / q->L, g, &loss, nullptr,
                    (char*)q->ufields + fo, (char*)q->wfields + fo, q->seen[sp]);
  } else {
    sg = bq_grad(q->ls, x, q->ybuf, &q->idx[q->off[sp]], q->len[sp], (double)S / q->L, g, &loss, nullptr);
  }
  if (sg < 0) return qn_fail(q, sg, std::string("gradient: ") + bq_last_error(q->ls));
  if (q->seen[sp] && !p.first_order)
    if (bq_status s = qn_sr1<T>(q, sp, x, g)) return s;
  if (hipMemcpyAsync((T*)q->xbar + (size_t)sp * V, x, V * sizeof(T), hipMemcpyDeviceToDevice, q->stream) !=
          hipSuccess ||
      hipMemcpyAsync((T*)q->gbar + (size_t)sp * V, g, V * sizeof(T), hipMemcpyDeviceToDevice, q->stream) !=
          hipSuccess)
    return qn_fail(q, BQ_EDEVICE, "copy of the subset pair failed");
  q->seen[sp] = 1;
  bq_prox_stats pst{};
  bq_status sx;
  double tau_sum;
  int rank;
  if (k <= S || p.first_order) {
    tau_sum = p.alpha;
    rank = 0;
    QnCoef w{};
    hipLaunchKernelGGL((k_qn_v<T>), dim3(q->np), dim3(QN_WG), 0, q->stream, x, g, (const T*)q->U, 0,
                       p.a / p.alpha, w, v, V);
    if (hipStreamSynchronize(q->stream) != hipSuccess) return qn_fail(q, BQ_EDEVICE, "device error");
    sx = bq_wprox(q->px, v, p.alpha, nullptr, 0, p.a * p.lambda, p.tv, p.cset, p.prox_iters, x, nullptr, &pst);
  } else {
    tau_sum = 0.0;
    for (int s = 0; s < S; ++s) tau_sum += q->tau[s];
    // Btilde = tau* I + U U^T: the columns of the subsets whose rank-one
    // correction was dropped are zero, so only the kept ones enter (packed
    // when some are missing); with none kept the metric is tau* I
    rank = 0;
    for (int s = 0; s < S; ++s) rank += q->kept[s] ? 1 : 0;
    const T* Uk = (const T*)q->U;
    if (rank > 0 && rank < S) {
      int c = 0;
      for (int s = 0; s < S; ++s)
        if (q->kept[s]) {
          if (hipMemcpyAsync((T*)q->Uc + (size_t)c * V, (const T*)q->U + (size_t)s * V, V * sizeof(T),
                             hipMemcpyDeviceToDevice, q->stream) != hipSuccess)
            return qn_fail(q, BQ_EDEVICE, "packing of the metric columns failed");
          ++c;
        }
      Uk = (const T*)q->Uc;
    }
    const double aS = p.a * S;
    QnCoef w{};
    if (rank > 0) {
      hipLaunchKernelGGL((k_qn_gram<T>), dim3(q->np), dim3(QN_WG), 0, q->stream, Uk, rank, g, V, q->part);
      if (bq_status s = qn_reduce(q, QN_K)) return s;
      std::vector<double> M((size_t)rank * rank);
      double ug[QN_RM], c[QN_RM];
      for (int i = 0; i < rank; ++i) {
        ug[i] = q->hres[QN_NT + i];
        for (int j = 0; j < rank; ++j)
          M[i * rank + j] = (i == j ? 1.0 : 0.0) + q->hres[i <= j ? qn_tri(i, j) : qn_tri(j, i)] / tau_sum;
      }
      qn_chol_solve(M, rank, ug, c);
      for (int i = 0; i < rank; ++i) w.w[i] = aS * c[i] / (tau_sum * tau_sum);
    }
    // v = x - a S (g / tau* - U c / tau*^2)
    hipLaunchKernelGGL((k_qn_v<T>), dim3(q->np), dim3(QN_WG), 0, q->stream, x, g, Uk, rank, aS / tau_sum, w, v, V);
    if (hipStreamSynchronize(q->stream) != hipSuccess) return qn_fail(q, BQ_EDEVICE, "device error");
    sx = bq_wprox(q->px, v, tau_sum, rank > 0 ? Uk : nullptr, rank, aS * p.lambda, p.tv, p.cset, p.prox_iters, x,
                  nullptr, &pst);
  }
  if (sx < 0) return qn_fail(q, sx, std::string("weighted prox: ") + bq_prox_last_error(q->px));
  q->k = k;
  if (info) {
    info->k = k;
    info->subset = sp;
    info->loss = loss;
    info->tau = q->tau[sp];
    info->u_kept = q->kept[sp];
    info->metric_rank = rank;
    info->tau_sum = tau_sum;
    info->prox_passes = pst.newton_total;
  }
  if (sg > 0) {
    q->err = std::string("gradient: ") + bq_last_error(q->ls);
    return sg;
  }
  if (sx > 0) {
    q->err = std::string("weighted prox: ") + bq_prox_last_error(q->px);
    return sx;
  }
  return BQ_OK;
}

}  // namespace

extern "C" {

bq_status bq_qn_create(bq_ctx* ls, bq_prox* px, const bq_qn_params* prm, const int* subset_idx,
                       const int* subset_len, bq_qn** out) {
  if (!out) { g_qn_create_error = "out is NULL"; return BQ_EINVAL; }
  *out = nullptr;
  if (!ls || !px || !prm || !subset_idx || !subset_len) {
    g_qn_create_error = "null argument";
    return BQ_EINVAL;
  }
  const bq_qn_params& p = *prm;
  if (p.S < 1 || p.S > BQ_PROX_MAX_RANK) { g_qn_create_error = "S must be in [1, BQ_PROX_MAX_RANK]"; return BQ_EINVAL; }
  if (!(p.a > 0) || !(p.lambda > 0) || !(p.alpha > 0) || !(p.gamma > 0) || !(p.gamma <= 1) || !(p.tau_max > 0) ||
      p.prox_iters < 0) {
    g_qn_create_error = "a, lambda, alpha, tau_max must be > 0, gamma in (0, 1], prox_iters >= 0";
    return BQ_EINVAL;
  }
  if ((p.tv != BQ_TV_ISO && p.tv != BQ_TV_ANISO) || (p.cset != BQ_SET_NONE && p.cset != BQ_SET_NONNEG)) {
    g_qn_create_error = "tv or cset";
    return BQ_EINVAL;
  }
  if (p.warm_start && ls->g.model != BQ_MODEL_LS) {
    g_qn_create_error = "warm starts need the LS model";
    return BQ_EUNSUPPORTED;
  }
  const int N = ls->g.N;
  if (px->prec != ls->g.precision || px->nz != N || px->ny != N || px->nx != N) {
    g_qn_create_error = "the prox workspace must have the context's precision and an N x N x N image";
    return BQ_EUNSUPPORTED;
  }
  bq_qn* q = new bq_qn();
  q->ls = ls;
  q->px = px;
  q->prm = p;
  q->S = p.S;
  q->N = N;
  q->L = ls->L;
  q->prec = ls->g.precision;
  q->V = (size_t)N * N * N;
  q->es = q->prec == BQ_F32 ? 4 : 8;
  q->csz = 2 * q->es;
  q->stream = ls->stream;
  int total = 0;
  for (int s = 0; s < p.S; ++s) {
    if (subset_len[s] < 1) { free_qn(q); g_qn_create_error = "empty subset"; return BQ_EINVAL; }
    q->off.push_back(total);
    q->len.push_back(subset_len[s]);
    total += subset_len[s];
    if (subset_len[s] > q->maxlen) q->maxlen = subset_len[s];
  }
  for (int i = 0; i < total; ++i) {
    if (subset_idx[i] < 0 || subset_idx[i] >= ls->L) {
      free_qn(q);
      g_qn_create_error = "illumination index out of range";
      return BQ_EINVAL;
    }
    q->idx.push_back(subset_idx[i]);
  }
  size_t g = (q->V + QN_WG * 4 - 1) / (QN_WG * 4);
  q->np = (int)(g > 1024 ? 1024 : g < 1 ? 1 : g);
  const size_t img = q->V * q->es;
  if (hipMalloc(&q->xbar, p.S * img) != hipSuccess || hipMalloc(&q->gbar, p.S * img) != hipSuccess ||
      hipMalloc(&q->U, p.S * img) != hipSuccess || hipMalloc(&q->Uc, p.S * img) != hipSuccess ||
      hipMalloc(&q->g, img) != hipSuccess ||
      hipMalloc(&q->v, img) != hipSuccess ||
      hipMalloc(&q->ybuf, (size_t)q->maxlen * ls->ndet * ls->ndet * q->csz) != hipSuccess ||
      hipMalloc((void**)&q->part, (size_t)q->np * QN_K * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&q->res, QN_K * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&q->hres, QN_K * sizeof(double)) != hipSuccess ||
      (p.warm_start && (hipMalloc(&q->ufields, (size_t)total * q->V * q->csz) != hipSuccess ||
                        hipMalloc(&q->wfields, (size_t)total * q->V * q->csz) != hipSuccess))) {
    free_qn(q);
    (void)hipGetLastError();  // not left for the next launch check to find
    g_qn_create_error = "out of memory";
    return BQ_ENOMEM;
  }
  if (q->prec == BQ_F32)
    hipLaunchKernelGGL((k_qn_fill<float>), dim3(1024), dim3(256), 0, q->stream, (float*)q->U, p.S * q->V, 0.0f);
  else
    hipLaunchKernelGGL((k_qn_fill<double>), dim3(1024), dim3(256), 0, q->stream, (double*)q->U, p.S * q->V, 0.0);
  if (hipStreamSynchronize(q->stream) != hipSuccess) {
    free_qn(q);
    g_qn_create_error = "device error";
    return BQ_EDEVICE;
  }
  q->tau.assign(p.S, p.alpha);
  q->seen.assign(p.S, 0);
  q->kept.assign(p.S, 0);
  *out = q;
  return BQ_OK;
}

bq_status bq_qn_destroy(bq_qn* q) {
  if (q) (void)hipStreamSynchronize(q->stream);
  free_qn(q);
  return BQ_OK;
}

const char* bq_qn_last_error(const bq_qn* q) { return q ? q->err.c_str() : g_qn_create_error.c_str(); }

bq_status bq_qn_step(bq_qn* q, void* x, const void* y, int pick, bq_qn_info* info) {
  if (!q) return BQ_EINVAL;
  if (!x || !y) return qn_fail(q, BQ_EINVAL, "null device pointer");
  if (q->k + 1 > q->S && (pick < -1 || pick >= q->S)) return qn_fail(q, BQ_EINVAL, "pick must be -1 or in [0, S)");
  return q->prec == BQ_F32 ? qn_step<float>(q, x, y, pick, info) : qn_step<double>(q, x, y, pick, info);
}

}  // extern "C"
