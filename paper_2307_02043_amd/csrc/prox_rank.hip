// Weighted proximal mapping of constrained TV for a metric tau I + U U^T
// whose factor U has r >= 2 columns (Section 4.3: the sum of the S rank-one
// corrected metrics of Algorithm 4.1 has this form with r = S).
//
// Same accelerated projected-gradient iteration on the dual as the
// rank-one path (Section 4.1, Lemma 4.1 step).  Per dual iteration:
//   d = sum_a (D^a)^T R_a,  a = v - (lambda / tau) d
//   c = U^T d,  kappa = lambda (I_r + G / tau)^-1 c / tau^2,  G = U^T U
//   w = v - lambda B^-1 d = a + U kappa                       (Woodbury)
//   x = max(w - U beta / tau, 0) = max(a - U theta, 0),  theta = beta / tau - kappa
// Theorem 3.1: beta* is the root of phi(beta) = U^T (w - max(w - U beta / tau, 0)) + beta,
// the gradient of the strongly convex Psi(beta) = |beta|^2 / 2 + beta^T U^T w
// + tau / 2 |max(w - U beta / tau, 0)|^2.  In theta, on the piece with active
// set A = {a - U theta > 0}:
//   psi(theta) = phi = U^T w + tau kappa - T_A + (S_A + tau I) theta
//   Psi        = tau^2 / 2 |theta + kappa|^2 + tau (theta + kappa)^T U^T w + tau / 2 Q_A
// with U^T w = U^T a + G kappa, S_A = U_A^T U_A, T_A = U_A^T a_A,
// Q_A = sum_A (a - U theta)^2.  The semi-smooth Newton step of Algorithm 4.3
// (generalised Jacobian S_A + tau I, up to the factor tau) is taken from the
// last accepted point; a trial point is accepted when Psi decreases
// (Armijo), otherwise the step is halved.  The iteration ends when the
// Newton step from an accepted point is below the image precision: the new
// point is the root of that point's piece.
//
// Kernels: k_div_r (a; FP64 partials of U^T d, U^T a and, at the warm-start
// theta, S_A, T_A, Q_A), k_ssn_r (S_A, T_A, Q_A at a trial theta), k_dual_r
// (x from a and U where the stencil needs it, P = Proj(R + sigma D x),
// momentum) and, for the output, k_xr (x).
// One-workgroup kernels reduce the partials in a fixed order and run the
// small dense algebra (Cholesky, r <= 8) on the device.
#include <cmath>
#include <string>

#include "../../include/bq.h"
#include "bq_common.h"
#include "prox_internal.h"

namespace bq {

constexpr int PR_WG = 256;
constexpr int RM = PX_MAX_RANK;

struct ProxRankState {
  double tau, lam, eps, t, mom;
  double G[RM * RM], Minv[RM * RM];
  double kappa[RM], uw[RM];     // kappa and U^T w = U^T a + G kappa
  double theta[RM];             // trial point read by the kernels
  double thk[RM], gk[RM], dir[RM];
  double psik, step, slope_k, phi_max, dmax_k;
  int r, nonneg, done, passes, total_passes, max_passes_seen, gaveup, have_k;
  int overflow;  // a dual iteration needed more root passes than were launched
};

template <int R>
struct RK {
  static constexpr int NS = R * (R + 1) / 2;  // upper triangle of S_A
  static constexpr int C = 0, UA = R, S = 2 * R, T = 2 * R + NS, Q = 3 * R + NS;
  static constexpr int K = 3 * R + NS + 1;
};
static_assert(RK<RM>::K <= PX_PART, "partial-sum slots");

template <int R>
__host__ __device__ constexpr int tri(int i, int j) {  // i <= j
  return i * R - i * (i - 1) / 2 + (j - i);
}

template <typename T>
struct PRArgs {
  int nz, ny, nx;
  size_t V;
  const T* v;
  const T* U;  // r x V
  T* a;
  T* P;
  T* R;
  double* partial;
  ProxRankState* st;
  double sigma;
  int iso;
};

// Cholesky factorisation of the SPD R x R matrix H (row-major, in place:
// lower triangle holds L) and solve H x = b.
template <int R>
__device__ inline void chol_factor(double* H) {
  for (int j = 0; j < R; ++j) {
    double d = H[j * R + j];
    for (int k = 0; k < j; ++k) d -= H[j * R + k] * H[j * R + k];
    d = sqrt(d);
    H[j * R + j] = d;
    for (int i = j + 1; i < R; ++i) {
      double s = H[i * R + j];
      for (int k = 0; k < j; ++k) s -= H[i * R + k] * H[j * R + k];
      H[i * R + j] = s / d;
    }
  }
}
template <int R>
__device__ inline void chol_solve(const double* L, const double* b, double* x) {
  double y[R];
  for (int i = 0; i < R; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i * R + k] * y[k];
    y[i] = s / L[i * R + i];
  }
  for (int i = R - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < R; ++k) s -= L[k * R + i] * x[k];
    x[i] = s / L[i * R + i];
  }
}

// Partials are stored value-major: value k of workgroup b at k np + b, so
// the reduction's loads are coalesced.  Sum values [K0, K0 + K) over the np
// workgroups (fixed order); result in thread 0.
template <int K0, int K>
__device__ inline void pr_sum(const double* part, int np, double* out, double* scratch) {
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] += part[(size_t)(K0 + k) * np + i];
  }
  block_sum<256, K>(out, scratch);
}

template <typename T, int R>
__global__ void __launch_bounds__(PR_WG) k_gram_r(PRArgs<T> p) {
  constexpr int NS = RK<R>::NS;
  __shared__ double scratch[(PR_WG / 64) * NS];
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  for (size_t i = blockIdx.x * (size_t)PR_WG + threadIdx.x; i < p.V; i += (size_t)gridDim.x * PR_WG) {
    double u[R];
#pragma unroll
    for (int c = 0; c < R; ++c) u[c] = (double)p.U[c * p.V + i];
#pragma unroll
    for (int c = 0; c < R; ++c)
#pragma unroll
      for (int e = c; e < R; ++e) acc[tri<R>(c, e)] += u[c] * u[e];
  }
  block_sum<PR_WG, NS>(acc, scratch);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) p.partial[(size_t)k * gridDim.x + blockIdx.x] = acc[k];
  }
}

// G = U^T U, Minv = (I + G / tau)^-1
template <int R>
__global__ void __launch_bounds__(256) k_pr_gram(ProxRankState* st, const double* part, int np) {
  constexpr int NS = RK<R>::NS;
  __shared__ double scratch[4 * NS];
  double g[NS];
  pr_sum<0, NS>(part, np, g, scratch);
  if (threadIdx.x != 0) return;
  ProxRankState& s = *st;
  double M[R * R];
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) {
      const double gij = g[i <= j ? tri<R>(i, j) : tri<R>(j, i)];
      s.G[i * RM + j] = gij;
      M[i * R + j] = (i == j ? 1.0 : 0.0) + gij / s.tau;
    }
  chol_factor<R>(M);
  for (int j = 0; j < R; ++j) {
    double e[R], col[R];
    for (int i = 0; i < R; ++i) e[i] = i == j ? 1.0 : 0.0;
    chol_solve<R>(M, e, col);
    for (int i = 0; i < R; ++i) s.Minv[i * RM + j] = col[i];
  }
}

// a = v - (lambda / tau) d(R); partials U^T d, U^T a, and S_A, T_A, Q_A at the warm-start theta
template <typename T, int R>
__global__ void __launch_bounds__(PR_WG) k_div_r(PRArgs<T> p) {
  using K_ = RK<R>;
  __shared__ double scratch[(PR_WG / 64) * K_::K];
  const ProxRankState* s = p.st;
  const double lt = s->lam / s->tau;
  T th[R];
#pragma unroll
  for (int c = 0; c < R; ++c) th[c] = (T)s->theta[c];
  const size_t V = p.V, sz = (size_t)p.ny * p.nx, sy = (size_t)p.nx;
  double acc[K_::K];
#pragma unroll
  for (int k = 0; k < K_::K; ++k) acc[k] = 0.0;
  const T* Rz = p.R;
  const T* Ry = p.R + V;
  const T* Rx = p.R + 2 * V;
  const unsigned nrows = (unsigned)p.nz * (unsigned)p.ny;
  for_rows<PR_WG>(p.nx, nrows, [&](unsigned row, int x) {
    const int z = (int)(row / (unsigned)p.ny), y = (int)(row - (unsigned)z * (unsigned)p.ny);
    const size_t base = (size_t)row * p.nx;
    const size_t i = base + x;
    // all loads issued (at the low faces the backward neighbour is replaced
    // by the forward one, every dimension being >= 2), boundaries as selects
    const T zm = Rz[z > 0 ? i - sz : i + sz], zc = Rz[i];
    const T ym = Ry[y > 0 ? i - sy : i + sy], yc = Ry[i];
    const T xm = Rx[x > 0 ? i - 1 : i + 1], xc = Rx[i];
    T d = 0;
    d += z > 0 ? zm : T(0);
    d -= z < p.nz - 1 ? zc : T(0);
    d += y > 0 ? ym : T(0);
    d -= y < p.ny - 1 ? yc : T(0);
    d += x > 0 ? xm : T(0);
    d -= x < p.nx - 1 ? xc : T(0);
    const T av = nt_ld(&p.v[i]) - (T)lt * d;
    p.a[i] = av;
    T u[R];
#pragma unroll
    for (int c = 0; c < R; ++c) u[c] = p.U[c * V + i];
    T zr = av;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      acc[K_::C + c] += (double)u[c] * d;
      acc[K_::UA + c] += (double)u[c] * av;
      zr -= u[c] * th[c];
    }
    if (zr > T(0)) {
#pragma unroll
      for (int c = 0; c < R; ++c) {
#pragma unroll
        for (int e = c; e < R; ++e) acc[K_::S + tri<R>(c, e)] += (double)u[c] * u[e];
        acc[K_::T + c] += (double)u[c] * av;
      }
      acc[K_::Q] += (double)zr * zr;
    }
  });
  block_sum<PR_WG, K_::K>(acc, scratch);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K_::K; ++k) p.partial[(size_t)k * gridDim.x + blockIdx.x] = acc[k];
  }
}

// S_A, T_A, Q_A at the trial theta
template <typename T, int R>
__global__ void __launch_bounds__(PR_WG) k_ssn_r(PRArgs<T> p) {
  using K_ = RK<R>;
  constexpr int KS = K_::K - K_::S;
  __shared__ double scratch[(PR_WG / 64) * KS];
  if (p.st->done) return;
  T th[R];
#pragma unroll
  for (int c = 0; c < R; ++c) th[c] = (T)p.st->theta[c];
  double acc[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) acc[k] = 0.0;
  for (size_t i = blockIdx.x * (size_t)PR_WG + threadIdx.x; i < p.V; i += (size_t)gridDim.x * PR_WG) {
    const T av = p.a[i];
    T u[R];
    T zr = av;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      u[c] = p.U[c * p.V + i];
      zr -= u[c] * th[c];
    }
    if (zr > T(0)) {
#pragma unroll
      for (int c = 0; c < R; ++c) {
#pragma unroll
        for (int e = c; e < R; ++e) acc[tri<R>(c, e)] += (double)u[c] * u[e];
        acc[K_::NS + c] += (double)u[c] * av;
      }
      acc[K_::NS + R] += (double)zr * zr;
    }
  }
  block_sum<PR_WG, KS>(acc, scratch);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < KS; ++k) p.partial[(size_t)(K_::S + k) * gridDim.x + blockIdx.x] = acc[k];
  }
}

// One evaluation at s.theta with the piece sums S (upper triangle), Tv, Q:
// accept or backtrack, then the next trial point or termination.
template <int R>
__device__ inline void pr_eval(ProxRankState& s, const double* S, const double* Tv, double Q, int max_passes) {
  const double tau = s.tau;
  double psi[R], scale = 0.0, pmax = 0.0;
  double Psi = 0.0, Qt = 0.0;
  for (int i = 0; i < R; ++i) {
    double v = s.uw[i] + tau * s.kappa[i] - Tv[i] + tau * s.theta[i];
    double sc = fabs(s.uw[i]) + tau * fabs(s.kappa[i]) + fabs(Tv[i]) + tau * fabs(s.theta[i]);
    for (int j = 0; j < R; ++j) {
      const double sij = S[i <= j ? tri<R>(i, j) : tri<R>(j, i)];
      v += sij * s.theta[j];
      sc += fabs(sij * s.theta[j]);
    }
    psi[i] = v;
    scale = fmax(scale, sc);
    pmax = fmax(pmax, fabs(v));
    const double tk = s.theta[i] + s.kappa[i];
    Psi += 0.5 * tau * tau * tk * tk + tau * tk * s.uw[i];
    Qt += fabs(0.5 * tau * tau * tk * tk) + fabs(tau * tk * s.uw[i]);
  }
  Psi += 0.5 * tau * Q;
  Qt += 0.5 * tau * Q;
  s.phi_max = pmax;
  s.passes += 1;
  s.total_passes += 1;
  if (s.passes > s.max_passes_seen) s.max_passes_seen = s.passes;
  const double e64 = 2.220446049250313e-16;
  // Armijo test; the slack covers the rounding of Psi in the image precision
  // (Q_A is a sum of squares of image-precision values)
  const bool accept =
      !s.have_k || Psi <= s.psik + 1e-4 * s.step * s.slope_k + 16.0 * s.eps * (Qt + fabs(s.psik));
  if (accept) {
    for (int i = 0; i < R; ++i) { s.thk[i] = s.theta[i]; s.gk[i] = psi[i]; }
    s.psik = Psi;
    s.have_k = 1;
    double H[R * R];
    for (int i = 0; i < R; ++i)
      for (int j = 0; j < R; ++j) H[i * R + j] = S[i <= j ? tri<R>(i, j) : tri<R>(j, i)] + (i == j ? tau : 0.0);
    chol_factor<R>(H);
    double stepv[R];
    chol_solve<R>(H, psi, stepv);
    double dmax = 0.0, tmax = 0.0, sl = 0.0;
    for (int i = 0; i < R; ++i) {
      s.dir[i] = -stepv[i];
      dmax = fmax(dmax, fabs(stepv[i]));
      tmax = fmax(tmax, fabs(s.theta[i]));
      sl += psi[i] * s.dir[i];
    }
    s.slope_k = tau * sl;
    s.dmax_k = dmax;
    if (pmax == 0.0 || dmax <= 4.0 * s.eps * fmax(1.0, tmax) || pmax <= 16.0 * e64 * scale) {
      // on the root's piece the Newton point is the exact root
      for (int i = 0; i < R; ++i) s.theta[i] = s.thk[i] + s.dir[i];
      s.done = 1;
      return;
    }
    s.step = 1.0;
    for (int i = 0; i < R; ++i) s.theta[i] = s.thk[i] + s.dir[i];
  } else {
    s.step *= 0.5;
    double tmax = 0.0;
    for (int i = 0; i < R; ++i) tmax = fmax(tmax, fabs(s.thk[i]));
    if (s.step * s.dmax_k <= 4.0 * s.eps * fmax(1.0, tmax)) {
      // no representable progress left: the accepted point is the root to
      // the image precision
      for (int i = 0; i < R; ++i) s.theta[i] = s.thk[i];
      s.done = 1;
      return;
    }
    for (int i = 0; i < R; ++i) s.theta[i] = s.thk[i] + s.step * s.dir[i];
  }
  if (s.passes >= max_passes) {  // give up: best accepted point
    for (int i = 0; i < R; ++i) s.theta[i] = s.thk[i];
    s.done = 1;
    s.gaveup += 1;
  }
}

template <int R>
__global__ void __launch_bounds__(256) k_pr_after_div(ProxRankState* st, const double* part, int np,
                                                      int max_passes) {
  using K_ = RK<R>;
  __shared__ double scratch[4 * K_::K];
  double v[K_::K];
  pr_sum<0, K_::K>(part, np, v, scratch);
  if (threadIdx.x != 0) return;
  ProxRankState& s = *st;
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * s.t * s.t));
  s.mom = (s.t - 1.0) / tn;
  s.t = tn;
  const double f = s.lam / (s.tau * s.tau);
  for (int i = 0; i < R; ++i) {
    double k = 0.0;
    for (int j = 0; j < R; ++j) k += s.Minv[i * RM + j] * v[K_::C + j];
    s.kappa[i] = f * k;
  }
  for (int i = 0; i < R; ++i) {
    double g = v[K_::UA + i];
    for (int j = 0; j < R; ++j) g += s.G[i * RM + j] * s.kappa[j];
    s.uw[i] = g;
  }
  s.have_k = 0;
  s.passes = 0;
  s.done = 0;
  s.step = 1.0;
  s.slope_k = 0.0;
  if (!s.nonneg) {  // x = w = a + U kappa
    for (int i = 0; i < R; ++i) s.theta[i] = -s.kappa[i];
    s.done = 1;
    return;
  }
  pr_eval<R>(s, &v[K_::S], &v[K_::T], v[K_::Q], max_passes);
}

// last_slot: no further pass follows in this dual iteration; a root still
// open there is flagged (the host then reruns with every pass launched)
template <int R>
__global__ void __launch_bounds__(256) k_pr_after_ssn(ProxRankState* st, const double* part, int np,
                                                      int max_passes, int last_slot) {
  using K_ = RK<R>;
  constexpr int KS = K_::K - K_::S;
  __shared__ double scratch[4 * KS];
  if (st->done) return;
  double v[KS];
  pr_sum<K_::S, KS>(part, np, v, scratch);
  if (threadIdx.x != 0) return;
  pr_eval<R>(*st, &v[0], &v[K_::NS], v[K_::NS + R], max_passes);
  if (last_slot && !st->done) {
    st->overflow = 1;
    st->done = 1;
  }
}

// x = max(a - U theta, 0) (or a - U theta without the constraint) at voxel i
template <typename T, int R>
__device__ inline T xr_at(const PRArgs<T>& p, size_t i, const T* th, bool nonneg) {
  T z = p.a[i];
#pragma unroll
  for (int c = 0; c < R; ++c) z -= p.U[c * p.V + i] * th[c];
  return nonneg ? (z > T(0) ? z : T(0)) : z;
}

// x into out (the output of a call)
template <typename T, int R>
__global__ void __launch_bounds__(PR_WG) k_xr(PRArgs<T> p, T* out) {
  T th[R];
#pragma unroll
  for (int c = 0; c < R; ++c) th[c] = (T)p.st->theta[c];
  const bool nonneg = p.st->nonneg;
  for (size_t i = blockIdx.x * (size_t)PR_WG + threadIdx.x; i < p.V; i += (size_t)gridDim.x * PR_WG)
    out[i] = xr_at<T, R>(p, i, th, nonneg);
}

// P_k = Proj(R_k + sigma D x_k); R_{k+1} = P_k + mom (P_k - P_{k-1}), with x
// formed from a and U where the stencil needs it (as k_xr forms it, so the
// iterates do not depend on which thread forms it).  Each thread walks one
// (y, x) column through a chunk of zc planes: x at plane z + 1 is the next
// step's centre and x at x + 1 the next lane's (a cross-lane shift; the last
// lane of a wave forms it itself).  On a high face the voxel itself stands
// in for the forward neighbour, whose difference is discarded.  R and P are
// streamed (non-temporal).
template <typename T, int R>
__global__ void __launch_bounds__(PR_WG) k_dual_r(PRArgs<T> p, int zc) {
  T th[R];
#pragma unroll
  for (int c = 0; c < R; ++c) th[c] = (T)p.st->theta[c];
  const bool nonneg = p.st->nonneg;
  const T sig = (T)p.sigma, mom = (T)p.st->mom;
  const size_t V = p.V, sz = (size_t)p.ny * p.nx, sy = (size_t)p.nx;
  const unsigned nchunk = (unsigned)((p.nz + zc - 1) / zc);
  const bool last_lane = (threadIdx.x & 63) == 63;
  for_rows<PR_WG>(p.nx, nchunk * (unsigned)p.ny, [&](unsigned row, int x) {
    const int ch = (int)(row / (unsigned)p.ny), y = (int)(row - (unsigned)ch * (unsigned)p.ny);
    const int z0 = ch * zc, z1 = min(z0 + zc, p.nz);
    const bool hy = y < p.ny - 1, hx = x < p.nx - 1;
    const size_t dy = hy ? sy : 0;  // offset of (z, y + 1) from the voxel
    size_t i = ((size_t)z0 * p.ny + y) * p.nx + x;
    T xc = xr_at<T, R>(p, i, th, nonneg);
    for (int z = z0; z < z1; ++z) {
      const bool hz = z < p.nz - 1;
      const T xz = xr_at<T, R>(p, hz ? i + sz : i, th, nonneg);
      const T xy = xr_at<T, R>(p, i + dy, th, nonneg);
      T xx = __shfl_down(xc, 1, 64);
      if (last_lane && hx) xx = xr_at<T, R>(p, i + 1, th, nonneg);
      const T gz = hz ? xz - xc : T(0);
      const T gy = hy ? xy - xc : T(0);
      const T gx = hx ? xx - xc : T(0);
      T qz = nt_ld(&p.R[i]) + sig * gz;
      T qy = nt_ld(&p.R[V + i]) + sig * gy;
      T qx = nt_ld(&p.R[2 * V + i]) + sig * gx;
      if (p.iso) {
        const T n = sqrt(qz * qz + qy * qy + qx * qx);
        if (n > T(1)) {
          const T inv = T(1) / n;
          qz *= inv; qy *= inv; qx *= inv;
        }
      } else {
        qz = fmin(fmax(qz, T(-1)), T(1));
        qy = fmin(fmax(qy, T(-1)), T(1));
        qx = fmin(fmax(qx, T(-1)), T(1));
      }
      const T oz = nt_ld(&p.P[i]), oy = nt_ld(&p.P[V + i]), ox = nt_ld(&p.P[2 * V + i]);
      nt_st(&p.P[i], qz); nt_st(&p.P[V + i], qy); nt_st(&p.P[2 * V + i], qx);
      nt_st(&p.R[i], qz + mom * (qz - oz));
      nt_st(&p.R[V + i], qy + mom * (qy - oy));
      nt_st(&p.R[2 * V + i], qx + mom * (qx - ox));
      xc = xz;
      i += sz;
    }
  });
}

template <typename T>
__global__ void k_fill_r(T* d, size_t n, T val) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    d[i] = val;
}

__global__ void k_pr_init(ProxRankState* st, double tau, double lam, int r, int nonneg, double eps) {
  if (threadIdx.x != 0) return;
  ProxRankState s{};
  s.tau = tau;
  s.lam = lam;
  s.eps = eps;
  s.t = 1.0;
  s.r = r;
  s.nonneg = nonneg;
  s.done = 1;
  s.step = 1.0;
  *st = s;
}

size_t prox_rank_state_bytes() { return sizeof(ProxRankState); }

static int pr_grid(size_t V) {
  size_t g = (V + PR_WG * 4 - 1) / (PR_WG * 4);
  if (g > 2048) g = 2048;
  if (g >= NUM_XCD) g = (g + NUM_XCD - 1) / NUM_XCD * NUM_XCD;  // one row slab per XCD
  if (g < 1) g = 1;
  return (int)g;
}

// One run of the iteration with `slots` root passes launched per dual
// iteration; the final device state goes to *hs_out.
template <typename T, int R>
static bq_status run_rank_once(bq_prox* p, const void* v, double tau, const void* U, double lam, int tv,
                               int cset, int n_iter, void* x_out, void* P_io, int slots, ProxRankState* hs_out) {
  const size_t V = p->V;
  const hipStream_t s = p->own;
  const int np = pr_grid(V);
  if (np > p->np) {
    p->err = "partial-sum buffer too small";
    return BQ_EDEVICE;
  }
  const dim3 g(np), b(PR_WG);
  PRArgs<T> a{};
  a.nz = p->nz; a.ny = p->ny; a.nx = p->nx; a.V = V;
  a.v = (const T*)v;
  a.U = (const T*)U;
  a.a = (T*)p->a;
  a.P = P_io ? (T*)P_io : (T*)p->P;
  a.R = (T*)p->R;
  a.partial = p->partial;
  a.st = p->rst;
  a.iso = (tv == BQ_TV_ISO);
  a.sigma = tau / (4.0 * 3.0 * lam);  // 1 / Lipschitz (Lemma 4.1, omega_min = tau, D = 3), x 2 lambda
  const int nonneg = (cset == BQ_SET_NONNEG);
  const double eps = sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
  hipLaunchKernelGGL(k_pr_init, dim3(1), dim3(64), 0, s, p->rst, tau, lam, R, nonneg, eps);
  hipLaunchKernelGGL((k_gram_r<T, R>), g, b, 0, s, a);
  hipLaunchKernelGGL((k_pr_gram<R>), dim3(1), dim3(256), 0, s, p->rst, (const double*)p->partial, np);
  if (!P_io) hipLaunchKernelGGL((k_fill_r<T>), dim3(1024), dim3(256), 0, s, a.P, 3 * V, T(0));
  if (hipMemcpyAsync(a.R, a.P, 3 * V * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess) {
    p->err = "copy of the starting dual point failed";
    return BQ_EDEVICE;
  }
  const int mp = p->max_passes_rank;
  const int n_ssn = nonneg ? slots : 0;
  // divergence and root finding for the current momentum R
  auto primal = [&]() {
    hipLaunchKernelGGL((k_div_r<T, R>), g, b, 0, s, a);
    hipLaunchKernelGGL((k_pr_after_div<R>), dim3(1), dim3(256), 0, s, p->rst, (const double*)p->partial, np, mp);
    for (int j = 0; j < n_ssn; ++j) {
      hipLaunchKernelGGL((k_ssn_r<T, R>), g, b, 0, s, a);
      hipLaunchKernelGGL((k_pr_after_ssn<R>), dim3(1), dim3(256), 0, s, p->rst, (const double*)p->partial, np,
                         mp, j == n_ssn - 1 ? 1 : 0);
    }
  };
  const ZWalk zw = zwalk_shape(p, PR_WG);
  if (!replay_iterations(p, n_iter, [&](hipStream_t) {
        primal();
        hipLaunchKernelGGL((k_dual_r<T, R>), zw.grid, b, 0, s, a, zw.zc);
      })) {
    p->err = "graph capture or launch of the dual iteration failed";
    return BQ_EDEVICE;
  }
  if (hipMemcpyAsync(a.R, a.P, 3 * V * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess) {
    p->err = "copy failed";
    return BQ_EDEVICE;
  }
  primal();
  hipLaunchKernelGGL((k_xr<T, R>), g, b, 0, s, a, (T*)x_out);
  if (hipGetLastError() != hipSuccess) {
    p->err = "kernel launch failed";
    return BQ_EDEVICE;
  }
  if (hipMemcpyAsync(hs_out, p->rst, sizeof(ProxRankState), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    p->err = "device error in the proximal mapping";
    return BQ_EDEVICE;
  }
  return BQ_OK;
}

template <typename T, int R>
static bq_status run_rank(bq_prox* p, const void* v, double tau, const void* U, double lam, int tv, int cset,
                          int n_iter, void* x_out, void* P_io, bq_prox_stats* stats) {
  if (!order_after_caller(p)) {
    p->err = "stream synchronisation failed";
    return BQ_EDEVICE;
  }
  ProxRankState hs{};
  const bq_status st = run_with_pass_budget(
      p, P_io, 3 * p->V * sizeof(T), cset == BQ_SET_NONNEG, p->ssn_slots_rank, p->max_passes_rank - 1,
      [&](int slots, int* overflow, int* seen) {
        const bq_status r = run_rank_once<T, R>(p, v, tau, U, lam, tv, cset, n_iter, x_out, P_io, slots, &hs);
        *overflow = hs.overflow;
        *seen = hs.max_passes_seen;
        return r;
      });
  if (st != BQ_OK) return st;
  if (stats) {
    stats->newton_total = hs.total_passes;
    stats->newton_max = hs.max_passes_seen;
    stats->beta_last = hs.tau * (hs.theta[0] + hs.kappa[0]);
    stats->phi_last = hs.phi_max;
  }
  if (hs.gaveup > 0) {
    p->err = "semi-smooth Newton hit its pass limit in " + std::to_string(hs.gaveup) + " dual iterations";
    return BQ_NOTCONV;
  }
  return BQ_OK;
}

template <typename T>
bq_status run_wprox_rank(bq_prox* p, const void* v, double tau, const void* U, int r, double lam, int tv,
                         int cset, int n_iter, void* x_out, void* P_io, bq_prox_stats* stats) {
  switch (r) {
    case 2: return run_rank<T, 2>(p, v, tau, U, lam, tv, cset, n_iter, x_out, P_io, stats);
    case 3: return run_rank<T, 3>(p, v, tau, U, lam, tv, cset, n_iter, x_out, P_io, stats);
    case 4: return run_rank<T, 4>(p, v, tau, U, lam, tv, cset, n_iter, x_out, P_io, stats);
    case 5: return run_rank<T, 5>(p, v, tau, U, lam, tv, cset, n_iter, x_out, P_io, stats);
    case 6: return run_rank<T, 6>(p, v, tau, U, lam, tv, cset, n_iter, x_out, P_io, stats);
    case 7: return run_rank<T, 7>(p, v, tau, U, lam, tv, cset, n_iter, x_out, P_io, stats);
    case 8: return run_rank<T, 8>(p, v, tau, U, lam, tv, cset, n_iter, x_out, P_io, stats);
    default:
      p->err = "metric rank out of range";
      return BQ_EINVAL;
  }
}

template bq_status run_wprox_rank<float>(bq_prox*, const void*, double, const void*, int, double, int, int, int,
                                         void*, void*, bq_prox_stats*);
template bq_status run_wprox_rank<double>(bq_prox*, const void*, double, const void*, int, double, int, int, int,
                                          void*, void*, bq_prox_stats*);

}  // namespace bq
