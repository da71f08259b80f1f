// Weighted proximal mapping of constrained TV on gfx950:
//   x = argmin_{x in C} 1/2 ||x - v||^2_B + lambda TV(x),  B = tau I + u u^T
// by the accelerated projected gradient iteration on the dual (Section 4.1,
// Lemma 4.1 step tau / (4 D lambda)), the Woodbury inverse of B (Section
// 4.3) and the projection onto the nonnegative orthant of Theorem 3.1,
// whose scalar root is found by a safeguarded semi-smooth Newton iteration
// (Algorithm 4.3) that stops exactly once the active set repeats.
//
// Variables per dual iteration (V = voxels):
//   d  = sum_a (D^a)^T R_a                       (divergence of the momentum)
//   a  = v - (lambda / tau) d                    (stored, the only V temp)
//   w  = v - lambda B^-1 d = a + kappa u,  kappa = lambda (u.d) / (tau^2 M),
//        M = 1 + u.u / tau
//   x  = max(w - u beta / tau, 0) = max(a - u theta, 0),  theta = beta/tau - kappa
//   psi(theta) = phi(beta) = u.a + kappa u.u - sum_{A} u_n (a_n - u_n theta)
//                + tau (theta + kappa),  A = {a_n - u_n theta > 0}
// so on the active set A, psi is linear: psi = K0 + theta (S_A + tau) with
// K0 = u.a + kappa u.u - T_A + tau kappa, S_A = sum_A u^2, T_A = sum_A u a.
//
// Kernels: k_div (a, and FP64 partials of u.d, u.a, S_A, T_A at the warm
// start theta), k_ssn (partials S_A, T_A at the current theta), k_dual
// (x at the voxel and its three forward neighbours, P = Proj(R + sigma D x),
// momentum), k_out.  One-workgroup scalar kernels reduce the partials in a
// fixed order and run the Newton / bisection logic on the device.  Without
// u (metric tau I) x is pointwise in d and there is no root: one kernel,
// k_dual0, carries the whole dual iteration, and k_out0 the output.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bq.h"
#include "bq_common.h"
#include "prox_internal.h"

namespace bq {

constexpr int PX_WG = 256;


struct ProxState {
  double tau, lam;
  double unorm2, M;
  double kappa;
  double ua;          // u . a
  double theta;       // current / final theta
  double lo, hi;      // bracket of the root in theta
  double K0, slope;   // line of the last evaluated piece
  double psi, psi_scale;
  int done;           // root found for this dual iteration
  int passes;         // evaluations in this dual iteration
  int total_passes;
  int max_passes_seen;
  int has_u, nonneg;
  int gaveup;         // dual iterations whose root was not pinned down
  int overflow;       // a dual iteration needed more root passes than were launched
  double eps;         // unit roundoff of the image precision
  double t, mom;      // FISTA sequence t_k and the momentum (t_k - 1) / t_{k+1}
  double tt[2];       // t_k of the metric-tau-I path, alternating between two slots
};

template <typename T>
struct ProxArgs {
  int nz, ny, nx;
  size_t V;
  const T* v;
  const T* u;       // may be null
  T* a;             // V
  T* P;             // 3V (P_{k-1} in, P_k out)
  T* R;             // 3V (R_k in, R_{k+1} out)
  T* x_out;
  double* partial;  // NP x 4
  ProxState* st;
  double sigma;     // dual step
  int iso;
};

// x = max(a - u theta, 0) (or a - u theta without the constraint, a when
// there is no u); the two cases are compile-time, so that no load sits
// behind a branch and the caller's loads stay in flight together.
template <typename T, bool HAS_U, bool NONNEG>
__device__ inline T xval(const ProxArgs<T>& a, size_t i, T theta) {
  T w = a.a[i];
  if constexpr (HAS_U) w = w - a.u[i] * theta;
  if constexpr (NONNEG) w = w > T(0) ? w : T(0);
  return w;
}

// a = v - (lambda / tau) d(R); partials: u.d, u.a, S_A(theta0), T_A(theta0).
// Rows (z, y) over workgroups, x over threads; two rows per step with all
// their loads issued before any arithmetic, to keep enough bytes in flight.
template <typename T>
__global__ void __launch_bounds__(PX_WG) k_div(ProxArgs<T> p) {
  __shared__ double scratch[(PX_WG / 64) * 4];
  const ProxState s = *p.st;
  const double lt = s.lam / s.tau;
  const T theta0 = (T)s.theta;
  const size_t V = p.V, sz = (size_t)p.ny * p.nx, sy = (size_t)p.nx;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const T* Rz = p.R;
  const T* Ry = p.R + V;
  const T* Rx = p.R + 2 * V;
  const unsigned nrows = (unsigned)p.nz * (unsigned)p.ny;
  // (D^a)^T q at i: q[i - e_a] (if i_a > 0) - q[i] (if i_a < n_a - 1)
  // every load is issued (at the low faces the backward neighbour is
  // replaced by the forward one, every dimension being >= 2) and the
  // boundary cases are selects, so that the loads of a row are in flight
  // together instead of behind one branch-and-wait each
  auto divergence = [&](unsigned row, int x) {
    const int z = (int)(row / (unsigned)p.ny), y = (int)(row - (unsigned)z * (unsigned)p.ny);
    const size_t i = (size_t)row * p.nx + x;
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
    return d;
  };
  auto finish = [&](size_t i, T d, T vv, T uv) {
    const T av = vv - (T)lt * d;
    p.a[i] = av;
    if (s.has_u) {
      acc[0] += (double)uv * d;
      acc[1] += (double)uv * av;
      if (av - uv * theta0 > T(0)) {
        acc[2] += (double)uv * uv;
        acc[3] += (double)uv * av;
      }
    }
  };
  for_row_pairs<PX_WG>(p.nx, nrows, [&](unsigned row0, unsigned row1, bool two, int x) {
    const size_t i0 = (size_t)row0 * p.nx + x, i1 = (size_t)row1 * p.nx + x;
    const T d0 = divergence(row0, x);
    const T v0 = nt_ld(&p.v[i0]), u0 = s.has_u ? p.u[i0] : T(0);
    T d1 = 0, v1 = 0, u1 = 0;
    if (two) {
      d1 = divergence(row1, x);
      v1 = nt_ld(&p.v[i1]);
      u1 = s.has_u ? p.u[i1] : T(0);
    }
    finish(i0, d0, v0, u0);
    if (two) finish(i1, d1, v1, u1);
  });
  if (!s.has_u) return;
  block_sum<PX_WG, 4>(acc, scratch);
  if (threadIdx.x == 0) {
    double* q = p.partial + (size_t)blockIdx.x * 4;
    q[0] = acc[0]; q[1] = acc[1]; q[2] = acc[2]; q[3] = acc[3];
  }
}

// partials S_A, T_A at the current theta
template <typename T>
__global__ void __launch_bounds__(PX_WG) k_ssn(ProxArgs<T> p) {
  __shared__ double scratch[(PX_WG / 64) * 2];
  if (p.st->done) return;
  const T theta = (T)p.st->theta;
  double acc[2] = {0.0, 0.0};
  for (size_t i = blockIdx.x * (size_t)PX_WG + threadIdx.x; i < p.V; i += (size_t)gridDim.x * PX_WG) {
    const T av = p.a[i], uv = p.u[i];
    if (av - uv * theta > T(0)) {
      acc[0] += (double)uv * uv;
      acc[1] += (double)uv * av;
    }
  }
  block_sum<PX_WG, 2>(acc, scratch);
  if (threadIdx.x == 0) {
    double* q = p.partial + (size_t)blockIdx.x * 4;
    q[2] = acc[0];
    q[3] = acc[1];
  }
}

template <int K0_, int K1_>
__device__ inline void px_sum(const double* part, int np, double* out, double* scratch) {
  constexpr int K = K1_ - K0_;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += part[(size_t)i * 4 + K0_ + k];
  }
  block_sum<256, K>(v, scratch);
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = v[k];
}

// Evaluate psi on the piece just measured, update the bracket, decide.
__device__ inline void px_step(ProxState& s, double SA, double TA, int max_passes) {
  const double th = s.theta;
  s.K0 = s.ua + s.kappa * s.unorm2 - TA + s.tau * s.kappa;
  s.slope = SA + s.tau;
  s.psi = s.K0 + th * s.slope;
  s.psi_scale = fabs(s.ua) + fabs(s.kappa) * s.unorm2 + fabs(TA) + fabs(th) * s.slope + s.tau * fabs(s.kappa);
  s.passes += 1;
  s.total_passes += 1;
  if (s.passes > s.max_passes_seen) s.max_passes_seen = s.passes;
  if (s.psi <= 0.0 && th > s.lo) s.lo = th;
  if (s.psi >= 0.0 && th < s.hi) s.hi = th;
  const double newton = -s.K0 / s.slope;  // root of this piece's line
  const double tol_t = 4.0 * s.eps * fmax(1.0, fabs(th));
  if (s.psi == 0.0 || fabs(newton - th) <= tol_t || s.hi - s.lo <= tol_t ||
      fabs(s.psi) <= 16.0 * 2.220446049250313e-16 * s.psi_scale) {
    // on the root's piece the Newton point is the exact root
    if (newton >= s.lo && newton <= s.hi) s.theta = newton;
    s.done = 1;
    return;
  }
  if (s.passes >= max_passes) {  // give up: best bracket point
    s.theta = (s.lo > -INFINITY && s.hi < INFINITY) ? 0.5 * (s.lo + s.hi) : th;
    s.done = 1;
    s.gaveup += 1;
    return;
  }
  double next = newton;
  if (!(next > s.lo && next < s.hi)) {
    if (s.lo > -INFINITY && s.hi < INFINITY) next = 0.5 * (s.lo + s.hi);
    else if (s.lo > -INFINITY) next = s.lo + 2.0 * fabs(s.psi) / s.tau;  // slope >= tau
    else next = s.hi - 2.0 * fabs(s.psi) / s.tau;
  }
  s.theta = next;
}

__global__ void __launch_bounds__(256) k_px_after_div(ProxState* st, const double* part, int np, int max_passes) {
  __shared__ double scratch[4 * 4];
  double v[4];
  px_sum<0, 4>(part, np, v, scratch);
  if (threadIdx.x != 0) return;
  ProxState s = *st;
  // momentum of the dual update that follows this divergence
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * s.t * s.t));
  s.mom = (s.t - 1.0) / tn;
  s.t = tn;
  s.kappa = s.lam * v[0] / (s.tau * s.tau * s.M);
  s.ua = v[1];
  s.lo = -INFINITY;
  s.hi = INFINITY;
  s.passes = 0;
  s.done = 0;
  if (!s.nonneg) {  // no constraint: x = w = a + kappa u, i.e. theta = -kappa
    s.theta = -s.kappa;
    s.done = 1;
  } else {
    px_step(s, v[2], v[3], max_passes);
  }
  *st = s;
}

// last_slot: no further pass follows in this dual iteration; a root still
// open there is flagged (the host then reruns with every pass launched)
__global__ void __launch_bounds__(256) k_px_after_ssn(ProxState* st, const double* part, int np, int max_passes,
                                                      int last_slot) {
  __shared__ double scratch[4 * 2];
  if (st->done) return;
  double v[2];
  px_sum<2, 4>(part, np, v, scratch);
  if (threadIdx.x != 0) return;
  ProxState s = *st;
  px_step(s, v[0], v[1], max_passes);
  if (last_slot && !s.done) {
    s.overflow = 1;
    s.done = 1;
  }
  *st = s;
}

__global__ void __launch_bounds__(256) k_px_unorm(ProxState* st, const double* part, int np) {
  __shared__ double scratch[4];
  double v[1];
  px_sum<0, 1>(part, np, v, scratch);
  if (threadIdx.x != 0) return;
  st->unorm2 = v[0];
  st->M = 1.0 + v[0] / st->tau;
}

template <typename T>
__global__ void __launch_bounds__(PX_WG) k_unorm(ProxArgs<T> p) {
  __shared__ double scratch[(PX_WG / 64)];
  double acc[1] = {0.0};
  for (size_t i = blockIdx.x * (size_t)PX_WG + threadIdx.x; i < p.V; i += (size_t)gridDim.x * PX_WG)
    acc[0] += (double)p.u[i] * p.u[i];
  block_sum<PX_WG, 1>(acc, scratch);
  if (threadIdx.x == 0) p.partial[(size_t)blockIdx.x * 4] = acc[0];
}

// P_k = Proj(R_k + sigma D x_k); R_{k+1} = P_k + mom (P_k - P_{k-1}).
// R and P are read and written once per voxel (non-temporal); a and u are
// re-read as stencil neighbours and keep the default cache policy.
// Each thread walks one (y, x) column through a chunk of zc planes: x at
// plane z + 1, formed for the z difference, is the next step's centre, and
// x at x + 1 is the next lane's centre (a cross-lane shift; the last lane
// of a wave forms it itself).  On a high face the voxel itself stands in
// for the forward neighbour, whose difference is discarded (in-bounds
// loads, no branch).  Traversal rows are (chunk, y) pairs.
template <typename T, bool HAS_U, bool NONNEG>
__global__ void __launch_bounds__(PX_WG) k_dual(ProxArgs<T> p, int zc) {
  const ProxState* stp = p.st;
  const T theta = (T)stp->theta;
  const T sig = (T)p.sigma, mom = (T)stp->mom;
  const size_t V = p.V, sz = (size_t)p.ny * p.nx, sy = (size_t)p.nx;
  const unsigned nchunk = (unsigned)((p.nz + zc - 1) / zc);
  const bool last_lane = (threadIdx.x & 63) == 63;
  for_rows<PX_WG>(p.nx, nchunk * (unsigned)p.ny, [&](unsigned row, int x) {
    const int ch = (int)(row / (unsigned)p.ny), y = (int)(row - (unsigned)ch * (unsigned)p.ny);
    const int z0 = ch * zc, z1 = min(z0 + zc, p.nz);
    const bool hy = y < p.ny - 1, hx = x < p.nx - 1;
    const size_t dy = hy ? sy : 0;  // offset of (z, y + 1) from the voxel
    size_t i = ((size_t)z0 * p.ny + y) * p.nx + x;
    T xc = xval<T, HAS_U, NONNEG>(p, i, theta);
    for (int z = z0; z < z1; ++z) {
      const bool hz = z < p.nz - 1;
      const T xz = xval<T, HAS_U, NONNEG>(p, hz ? i + sz : i, theta);
      const T xy = xval<T, HAS_U, NONNEG>(p, i + dy, theta);
      T xx = __shfl_down(xc, 1, 64);
      if (last_lane && hx) xx = xval<T, HAS_U, NONNEG>(p, i + 1, theta);
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

template <typename T, bool HAS_U, bool NONNEG>
__global__ void __launch_bounds__(PX_WG) k_out(ProxArgs<T> p) {
  const T theta = (T)p.st->theta;
  for (size_t i = blockIdx.x * (size_t)PX_WG + threadIdx.x; i < p.V; i += (size_t)gridDim.x * PX_WG)
    p.x_out[i] = xval<T, HAS_U, NONNEG>(p, i, theta);
}

// launch k_dual / k_out of the rank-one path, specialised on the constraint
// (without u the metric-tau-I path below runs instead)
template <typename T>
void launch_dual(bool nonneg, dim3 g, dim3 b, hipStream_t s, const ProxArgs<T>& a, int zc) {
  if (nonneg) hipLaunchKernelGGL((k_dual<T, true, true>), g, b, 0, s, a, zc);
  else hipLaunchKernelGGL((k_dual<T, true, false>), g, b, 0, s, a, zc);
}
template <typename T>
void launch_out(bool nonneg, dim3 g, dim3 b, hipStream_t s, const ProxArgs<T>& a) {
  if (nonneg) hipLaunchKernelGGL((k_out<T, true, true>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_out<T, true, false>), g, b, 0, s, a);
}

// Metric tau I (no u): x = Proj_C(v - (lambda / tau) d(R)) is pointwise in
// d, so one kernel carries a whole dual iteration: x from R_k at the voxel
// and at its three forward neighbours (a divergence each), P_k = Proj(R_k +
// sigma D x), R_{k+1} = P_k + mom (P_k - P_{k-1}).  R_{k+1} goes to a second
// buffer, since neighbouring threads still read R_k; P is read and written
// only at the voxel and is updated in place.  The arithmetic of x, of the
// projection and of the momentum is that of k_div / k_px_after_div /
// k_dual, operation for operation, so x does not depend on which thread
// forms it.
//
// x at (z, y, x) from the six R values of its divergence (the backward
// neighbour m and the voxel c of each component; a backward neighbour off
// the low face is not used) and v there.
template <typename T, bool NONNEG>
__device__ inline T x_of(const ProxArgs<T>& p, T lt, int z, int y, int x, T zm, T zc, T ym, T yc, T xm, T xc,
                         T vv) {
  T d = 0;
  d += z > 0 ? zm : T(0);
  d -= z < p.nz - 1 ? zc : T(0);
  d += y > 0 ? ym : T(0);
  d -= y < p.ny - 1 ? yc : T(0);
  d += x > 0 ? xm : T(0);
  d -= x < p.nx - 1 ? xc : T(0);
  T w = vv - lt * d;
  if constexpr (NONNEG) w = w > T(0) ? w : T(0);
  return w;
}

// x at (z, y, x), voxel j, with its loads; the three components of R at
// that voxel are returned in c[] (the caller reuses them for the dual step).
template <typename T, bool NONNEG>
__device__ inline T x_tau(const ProxArgs<T>& p, const T* __restrict__ R, T lt, int z, int y, int x, size_t j,
                          T* c) {
  const size_t V = p.V, sz = (size_t)p.ny * p.nx, sy = (size_t)p.nx;
  const T* Rz = R;
  const T* Ry = R + V;
  const T* Rx = R + 2 * V;
  const T zm = Rz[z > 0 ? j - sz : j + sz], zc = Rz[j];
  const T ym = Ry[y > 0 ? j - sy : j + sy], yc = Ry[j];
  const T xm = Rx[x > 0 ? j - 1 : j + 1], xc = Rx[j];
  c[0] = zc; c[1] = yc; c[2] = xc;
  return x_of<T, NONNEG>(p, lt, z, y, x, zm, zc, ym, yc, xm, xc, p.v[j]);
}

// Each thread walks one (y, x) column through a chunk of zc planes, so x and
// R at plane z + 1, formed for the z difference, are the next step's centre;
// x at x + 1 is the next lane's centre (a cross-lane shift; the last lane of
// a wave forms it itself).  Of the divergences of x at (z + 1, y) and at
// (z, y + 1), three R values are already held: R_z and R_y at the voxel and
// R_z at (z - 1, y + 1), loaded by the previous step.  On a high face the
// forward neighbour's x is not used, and the voxel itself stands in for it
// (in-bounds loads, no branch).  Traversal "rows" are (chunk, y) pairs, so
// rows y and y + 1 of one chunk are neighbours in the XCD row slabs.
//
// par: slot of t_k in the state (t_{k+1} is written to the other slot by
// one thread; no other thread reads that slot in this launch)
template <typename T, bool NONNEG>
__global__ void __launch_bounds__(PX_WG) k_dual0(ProxArgs<T> p, const T* __restrict__ Rin, T* __restrict__ Rout,
                                                 int par, int zc) {
  const double t = p.st->tt[par];
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
  const T mom = (T)((t - 1.0) / tn);
  if (blockIdx.x == 0 && threadIdx.x == 0) p.st->tt[par ^ 1] = tn;
  const T lt = (T)(p.st->lam / p.st->tau);
  const T sig = (T)p.sigma;
  const size_t V = p.V, sz = (size_t)p.ny * p.nx, sy = (size_t)p.nx;
  const unsigned nchunk = (unsigned)((p.nz + zc - 1) / zc);
  const bool last_lane = (threadIdx.x & 63) == 63;
  const T* Rz = Rin;
  const T* Ry = Rin + V;
  const T* Rx = Rin + 2 * V;
  for_rows<PX_WG>(p.nx, nchunk * (unsigned)p.ny, [&](unsigned row, int x) {
    const int ch = (int)(row / (unsigned)p.ny), y = (int)(row - (unsigned)ch * (unsigned)p.ny);
    const int z0 = ch * zc, z1 = min(z0 + zc, p.nz);
    const bool hy = y < p.ny - 1, hx = x < p.nx - 1;
    const size_t dy = hy ? sy : 0;  // offset of (z, y + 1) from the voxel
    size_t i = ((size_t)z0 * p.ny + y) * p.nx + x;
    T rc[3];
    T xc = x_tau<T, NONNEG>(p, Rin, lt, z0, y, x, i, rc);
    // R_z at (z - 1, y + 1) and, for the last lane, at (z - 1, y, x + 1);
    // not used at z = 0
    T rzy = Rz[(z0 > 0 && hy) ? i + sy - sz : i];
    T rzx = T(0);
    if (last_lane && hx) rzx = Rz[z0 > 0 ? i + 1 - sz : i + 1];
    for (int z = z0; z < z1; ++z) {
      const bool hz = z < p.nz - 1;
      const size_t j1 = hz ? i + sz : i;  // (z + 1, y)
      const size_t j2 = i + dy;           // (z, y + 1)
      const T z1c = Rz[j1], y1m = Ry[y > 0 ? j1 - sy : j1 + sy], y1c = Ry[j1];
      const T x1m = Rx[x > 0 ? j1 - 1 : j1 + 1], x1c = Rx[j1], v1 = p.v[j1];
      const T z2c = Rz[j2], y2c = Ry[j2], x2m = Rx[x > 0 ? j2 - 1 : j2 + 1], x2c = Rx[j2], v2 = p.v[j2];
      const T xz = x_of<T, NONNEG>(p, lt, hz ? z + 1 : z, y, x, rc[0], z1c, y1m, y1c, x1m, x1c, v1);
      const T xy = x_of<T, NONNEG>(p, lt, z, hy ? y + 1 : y, x, rzy, z2c, rc[1], y2c, x2m, x2c, v2);
      T xx = __shfl_down(xc, 1, 64);
      if (last_lane && hx) {  // x at (z, y, x + 1): R_x at the voxel is its backward neighbour
        const size_t j3 = i + 1;
        const T z3c = Rz[j3], y3m = Ry[y > 0 ? j3 - sy : j3 + sy], y3c = Ry[j3], x3c = Rx[j3], v3 = p.v[j3];
        xx = x_of<T, NONNEG>(p, lt, z, y, x + 1, rzx, z3c, y3m, y3c, rc[2], x3c, v3);
        rzx = z3c;
      }
      const T gz = hz ? xz - xc : T(0);
      const T gy = hy ? xy - xc : T(0);
      const T gx = hx ? xx - xc : T(0);
      T qz = rc[0] + sig * gz;
      T qy = rc[1] + sig * gy;
      T qx = rc[2] + sig * gx;
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
      nt_st(&Rout[i], qz + mom * (qz - oz));
      nt_st(&Rout[V + i], qy + mom * (qy - oy));
      nt_st(&Rout[2 * V + i], qx + mom * (qx - ox));
      xc = xz;
      rc[0] = z1c; rc[1] = y1c; rc[2] = x1c;
      rzy = z2c;
      i += sz;
    }
  });
}

// x(Q) = Proj_C(v - (lambda / tau) d(Q)) for the metric tau I
template <typename T, bool NONNEG>
__global__ void __launch_bounds__(PX_WG) k_out0(ProxArgs<T> p, const T* __restrict__ Q) {
  const T lt = (T)(p.st->lam / p.st->tau);
  const unsigned nrows = (unsigned)p.nz * (unsigned)p.ny;
  for_rows<PX_WG>(p.nx, nrows, [&](unsigned row, int x) {
    const int z = (int)(row / (unsigned)p.ny), y = (int)(row - (unsigned)z * (unsigned)p.ny);
    const size_t i = (size_t)row * p.nx + x;
    T c[3];
    p.x_out[i] = x_tau<T, NONNEG>(p, Q, lt, z, y, x, i, c);
  });
}

template <typename T>
__global__ void k_fill(T* d, size_t n, T val) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    d[i] = val;
}

__global__ void k_px_init(ProxState* st, double tau, double lam, int has_u, int nonneg, double eps) {
  if (threadIdx.x != 0) return;
  ProxState s{};
  s.eps = eps;
  s.tau = tau;
  s.lam = lam;
  s.M = 1.0;
  s.has_u = has_u;
  s.nonneg = nonneg;
  s.theta = 0.0;
  s.done = 1;
  s.t = 1.0;
  s.tt[0] = s.tt[1] = 1.0;
  *st = s;
}

}  // namespace bq

using namespace bq;

namespace {

thread_local std::string g_prox_create_error;

int px_grid(size_t V) {
  size_t g = (V + PX_WG * 4 - 1) / (PX_WG * 4);
  if (g > 2048) g = 2048;
  if (g >= NUM_XCD) g = (g + NUM_XCD - 1) / NUM_XCD * NUM_XCD;  // one row slab per XCD
  if (g < 1) g = 1;
  return (int)g;
}

// One run of the rank-one iteration (u not null) with `slots` root passes
// launched per dual iteration; the final device state goes to *hs.
template <typename T>
bq_status run_wprox_once(bq_prox* p, const void* v, double tau, const void* u, double lam, int tv, int cset,
                         int n_iter, void* x_out, void* P_io, int slots, ProxState* hs_out) {
  const size_t V = p->V;
  const hipStream_t s = p->own;
  const dim3 g(p->np), b(PX_WG);
  ProxArgs<T> a{};
  a.nz = p->nz; a.ny = p->ny; a.nx = p->nx; a.V = V;
  a.v = (const T*)v;
  a.u = (const T*)u;
  a.a = (T*)p->a;
  a.P = P_io ? (T*)P_io : (T*)p->P;
  a.R = (T*)p->R;
  a.x_out = (T*)x_out;
  a.partial = p->partial;
  a.st = p->st;
  a.iso = (tv == BQ_TV_ISO);
  a.sigma = tau / (4.0 * 3.0 * lam);  // 1 / Lipschitz (Lemma 4.1, omega_min = tau, D = 3), x 2 lambda
  const int has_u = u != nullptr, nonneg = (cset == BQ_SET_NONNEG);
  const double eps = sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
  hipLaunchKernelGGL(k_px_init, dim3(1), dim3(64), 0, s, p->st, tau, lam, has_u, nonneg, eps);
  if (has_u) {
    hipLaunchKernelGGL((k_unorm<T>), g, b, 0, s, a);
    hipLaunchKernelGGL(k_px_unorm, dim3(1), dim3(256), 0, s, p->st, (const double*)p->partial, p->np);
  }
  // P_0 (given or zero); R_1 = P_0
  if (!P_io) hipLaunchKernelGGL((k_fill<T>), dim3(1024), dim3(256), 0, s, a.P, 3 * V, T(0));  // P_0 = 0
  if (hipMemcpyAsync(a.R, a.P, 3 * V * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess) {
    p->err = "copy of the starting dual point failed";
    return BQ_EDEVICE;
  }
  const int max_launch = (has_u && nonneg) ? slots : 0;  // SSN passes per dual iteration
  // divergence + root finding for the current momentum R (all arguments are
  // iteration invariant: the momentum coefficient lives on the device)
  auto primal = [&]() {
    hipLaunchKernelGGL((k_div<T>), g, b, 0, s, a);
    hipLaunchKernelGGL(k_px_after_div, dim3(1), dim3(256), 0, s, p->st, (const double*)p->partial, p->np,
                       p->max_passes);
    for (int j = 0; j < max_launch; ++j) {
      hipLaunchKernelGGL((k_ssn<T>), g, b, 0, s, a);
      hipLaunchKernelGGL(k_px_after_ssn, dim3(1), dim3(256), 0, s, p->st, (const double*)p->partial, p->np,
                         p->max_passes, j == max_launch - 1 ? 1 : 0);
    }
  };
  // one dual iteration captured as a graph and replayed n_iter times
  const ZWalk zw = zwalk_shape(p, PX_WG);
  if (!replay_iterations(p, n_iter, [&](hipStream_t) {
        primal();
        launch_dual<T>(nonneg, zw.grid, b, s, a, zw.zc);
      })) {
    p->err = "graph capture or launch of the dual iteration failed";
    return BQ_EDEVICE;
  }
  // x(P_K): divergence of P_K itself, then the projection
  if (hipMemcpyAsync(a.R, a.P, 3 * V * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess) {
    p->err = "copy failed";
    return BQ_EDEVICE;
  }
  primal();
  launch_out<T>(nonneg, g, b, s, a);
  if (hipGetLastError() != hipSuccess) {
    p->err = "kernel launch failed";
    return BQ_EDEVICE;
  }
  if (hipMemcpyAsync(hs_out, p->st, sizeof(ProxState), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    p->err = "device error in the proximal mapping";
    return BQ_EDEVICE;
  }
  return BQ_OK;
}

// Metric tau I: one fused kernel per dual iteration (k_dual0), R_k and
// R_{k+1} alternating between p->R and p->R2.  Two dual iterations are
// captured as one graph (even: R -> R2, t in slot 0; odd: R2 -> R, slot 1)
// and replayed; an odd count ends with one even iteration launched alone.
template <typename T>
bq_status run_wprox_tau(bq_prox* p, const void* v, double tau, double lam, int tv, int cset, int n_iter,
                        void* x_out, void* P_io, bq_prox_stats* stats) {
  const size_t V = p->V;
  const hipStream_t s = p->own;
  const dim3 g(p->np), b(PX_WG);
  if (!p->R2 && hipMalloc(&p->R2, 3 * V * sizeof(T)) != hipSuccess) {
    p->R2 = nullptr;
    (void)hipGetLastError();
    p->err = "out of device memory";
    return BQ_ENOMEM;
  }
  ProxArgs<T> a{};
  a.nz = p->nz; a.ny = p->ny; a.nx = p->nx; a.V = V;
  a.v = (const T*)v;
  a.P = P_io ? (T*)P_io : (T*)p->P;
  a.x_out = (T*)x_out;
  a.st = p->st;
  a.iso = (tv == BQ_TV_ISO);
  a.sigma = tau / (4.0 * 3.0 * lam);  // as in the rank-one path
  const bool nonneg = (cset == BQ_SET_NONNEG);
  T* R0 = (T*)p->R;
  T* R1 = (T*)p->R2;
  const double eps = sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
  hipLaunchKernelGGL(k_px_init, dim3(1), dim3(64), 0, s, p->st, tau, lam, 0, nonneg ? 1 : 0, eps);
  if (!P_io) hipLaunchKernelGGL((k_fill<T>), dim3(1024), dim3(256), 0, s, a.P, 3 * V, T(0));  // P_0 = 0
  if (hipMemcpyAsync(R0, a.P, 3 * V * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess) {  // R_1 = P_0
    p->err = "copy of the starting dual point failed";
    return BQ_EDEVICE;
  }
  const ZWalk zw = zwalk_shape(p, PX_WG);
  const dim3 gd = zw.grid;
  const int zc = zw.zc;
  auto dual = [&](const T* rin, T* rout, int par) {
    if (nonneg) hipLaunchKernelGGL((k_dual0<T, true>), gd, b, 0, s, a, rin, rout, par, zc);
    else hipLaunchKernelGGL((k_dual0<T, false>), gd, b, 0, s, a, rin, rout, par, zc);
  };
  if (!replay_iterations(p, n_iter / 2, [&](hipStream_t) {
        dual(R0, R1, 0);
        dual(R1, R0, 1);
      })) {
    p->err = "graph capture or launch of the dual iteration failed";
    return BQ_EDEVICE;
  }
  if (n_iter % 2) dual(R0, R1, 0);
  // x(P_K)
  if (nonneg) hipLaunchKernelGGL((k_out0<T, true>), g, b, 0, s, a, (const T*)a.P);
  else hipLaunchKernelGGL((k_out0<T, false>), g, b, 0, s, a, (const T*)a.P);
  if (hipGetLastError() != hipSuccess) {
    p->err = "kernel launch failed";
    return BQ_EDEVICE;
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    p->err = "device error in the proximal mapping";
    return BQ_EDEVICE;
  }
  if (stats) {  // no root to find
    stats->newton_total = 0;
    stats->newton_max = 0;
    stats->beta_last = 0.0;
    stats->phi_last = 0.0;
  }
  return BQ_OK;
}

template <typename T>
bq_status run_wprox(bq_prox* p, const void* v, double tau, const void* u, double lam, int tv, int cset,
                    int n_iter, void* x_out, void* P_io, bq_prox_stats* stats) {
  // order after the caller's pending work, then run on the library stream
  if (!order_after_caller(p)) {
    p->err = "stream synchronisation failed";
    return BQ_EDEVICE;
  }
  if (!u) return run_wprox_tau<T>(p, v, tau, lam, tv, cset, n_iter, x_out, P_io, stats);
  ProxState hs{};
  const bq_status st = run_with_pass_budget(
      p, P_io, 3 * p->V * sizeof(T), u != nullptr && cset == BQ_SET_NONNEG, p->ssn_slots, p->max_passes - 1,
      [&](int slots, int* overflow, int* seen) {
        const bq_status r = run_wprox_once<T>(p, v, tau, u, lam, tv, cset, n_iter, x_out, P_io, slots, &hs);
        *overflow = hs.overflow;
        *seen = hs.max_passes_seen;
        return r;
      });
  if (st != BQ_OK) return st;
  if (stats) {
    stats->newton_total = hs.total_passes;
    stats->newton_max = hs.max_passes_seen;
    stats->beta_last = hs.tau * (hs.theta + hs.kappa);
    stats->phi_last = fabs(hs.psi);
  }
  if (hs.gaveup > 0) {
    p->err = "semi-smooth Newton hit its pass limit in " + std::to_string(hs.gaveup) + " dual iterations";
    return BQ_NOTCONV;
  }
  return BQ_OK;
}

void free_prox(bq_prox* p) {
  if (!p) return;
  void* ptrs[] = {p->a, p->P, p->R, p->R2, p->partial, p->st, p->rst, p->Pbak};
  for (void* q : ptrs) if (q) (void)hipFree(q);
  if (p->ev) (void)hipEventDestroy(p->ev);
  if (p->own) (void)hipStreamDestroy(p->own);
  delete p;
}

// Scratch memory of bq_wprox_noalloc: one array per device, allocated with
// the code object when the library is loaded on that device and kept until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// the device array: kernels get the device address that
// hipGetSymbolAddress returns for the current device (scratch_address).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(96) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per
// device (on its first call).  Null on failure, with the reason in *why.
void* scratch_address(const char** why) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    (void)hipGetLastError();
    *why = "no current HIP device (or device index above 63)";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      *why = "hipGetSymbolAddress of the scratch array failed";
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

extern "C" {

bq_status bq_prox_create(int nz, int ny, int nx, int precision, void* stream, bq_prox** out) {
  if (!out) { g_prox_create_error = "out is NULL"; return BQ_EINVAL; }
  *out = nullptr;
  if (nz < 2 || ny < 2 || nx < 2) { g_prox_create_error = "each image dimension must be >= 2"; return BQ_EINVAL; }
  if (precision != BQ_F32 && precision != BQ_F64) { g_prox_create_error = "precision"; return BQ_EINVAL; }
  bq_prox* p = new bq_prox();
  p->nz = nz; p->ny = ny; p->nx = nx; p->prec = precision;
  p->V = (size_t)nz * ny * nx;
  p->stream = (hipStream_t)stream;
  p->np = px_grid(p->V);
  const size_t es = precision == BQ_F32 ? 4 : 8;
  if (hipMalloc(&p->a, p->V * es) != hipSuccess || hipMalloc(&p->P, 3 * p->V * es) != hipSuccess ||
      hipMalloc(&p->R, 3 * p->V * es) != hipSuccess ||
      hipMalloc((void**)&p->partial, (size_t)p->np * PX_PART * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&p->st, sizeof(ProxState)) != hipSuccess ||
      hipMalloc((void**)&p->rst, prox_rank_state_bytes()) != hipSuccess) {
    free_prox(p);
    (void)hipGetLastError();  // not left for the next launch check to find
    g_prox_create_error = "out of device memory";
    return BQ_ENOMEM;
  }
  if (hipStreamCreateWithFlags(&p->own, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev, hipEventDisableTiming) != hipSuccess) {
    free_prox(p);
    g_prox_create_error = "could not create the library stream";
    return BQ_EDEVICE;
  }
  *out = p;
  return BQ_OK;
}

bq_status bq_prox_destroy(bq_prox* p) {
  if (p) (void)hipStreamSynchronize(p->own);
  free_prox(p);
  return BQ_OK;
}

const char* bq_prox_last_error(const bq_prox* p) { return p ? p->err.c_str() : g_prox_create_error.c_str(); }

bq_status bq_wprox(bq_prox* p, const void* v, double tau, const void* U, int r, double lambda, int tv,
                   int cset, int n_iter, void* x_out, void* P_io, bq_prox_stats* st) {
  if (!p) return BQ_EINVAL;
  if (!v || !x_out) { p->err = "null device pointer"; return BQ_EINVAL; }
  if (!(tau > 0) || !(lambda > 0) || n_iter < 0) { p->err = "tau, lambda must be > 0 and n_iter >= 0"; return BQ_EINVAL; }
  if (tv != BQ_TV_ISO && tv != BQ_TV_ANISO) { p->err = "tv"; return BQ_EINVAL; }
  if (cset != BQ_SET_NONE && cset != BQ_SET_NONNEG) { p->err = "cset"; return BQ_EINVAL; }
  if (r < 0 || r > BQ_PROX_MAX_RANK) { p->err = "metric rank r must be in [0, BQ_PROX_MAX_RANK]"; return BQ_EINVAL; }
  if (r > 0 && !U) { p->err = "U is NULL with r > 0"; return BQ_EINVAL; }
  if (r >= 2)
    return p->prec == BQ_F32 ? run_wprox_rank<float>(p, v, tau, U, r, lambda, tv, cset, n_iter, x_out, P_io, st)
                             : run_wprox_rank<double>(p, v, tau, U, r, lambda, tv, cset, n_iter, x_out, P_io, st);
  const void* u = r == 1 ? U : nullptr;
  return p->prec == BQ_F32 ? run_wprox<float>(p, v, tau, u, lambda, tv, cset, n_iter, x_out, P_io, st)
                           : run_wprox<double>(p, v, tau, u, lambda, tv, cset, n_iter, x_out, P_io, st);
}

bq_status bq_wprox_noalloc(int nz, int ny, int nx, int precision, const void* v, double tau, const void* U,
                           int r, double lambda, int tv, int cset, int n_iter, void* x_out, void* P_io,
                           bq_prox_stats* st, void* stream) {
  auto fail = [](bq_status s, const char* msg) {
    g_prox_create_error = msg;
    return s;
  };
  if (nz < 2 || ny < 2 || nx < 2) return fail(BQ_EINVAL, "each image dimension must be >= 2");
  if (precision != BQ_F32 && precision != BQ_F64) return fail(BQ_EINVAL, "precision");
  if (!v || !x_out) return fail(BQ_EINVAL, "null device pointer");
  if (!(tau > 0) || !(lambda > 0) || n_iter < 0) return fail(BQ_EINVAL, "tau, lambda must be > 0 and n_iter >= 0");
  if (tv != BQ_TV_ISO && tv != BQ_TV_ANISO) return fail(BQ_EINVAL, "tv");
  if (cset != BQ_SET_NONE && cset != BQ_SET_NONNEG) return fail(BQ_EINVAL, "cset");
  if (r < 0 || r > BQ_PROX_MAX_RANK) return fail(BQ_EINVAL, "metric rank r must be in [0, BQ_PROX_MAX_RANK]");
  if (r > 0 && !U) return fail(BQ_EINVAL, "U is NULL with r > 0");
  // the workspace of a bq_prox object, laid out in the scratch array: the
  // image a, the dual point P (unless the caller's), the momentum R, the
  // second momentum buffer of the metric tau I, the partial sums and the
  // two device states
  const size_t V = (size_t)nz * ny * nx;
  const size_t es = precision == BQ_F32 ? 4 : 8;
  const int np = px_grid(V);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
  const size_t o_a = take(V * es);
  const size_t o_P = P_io ? 0 : take(3 * V * es);
  const size_t o_R = take(3 * V * es);
  const size_t o_R2 = r == 0 ? take(3 * V * es) : 0;
  const size_t o_part = take((size_t)np * PX_PART * sizeof(double));
  const size_t o_st = take(sizeof(ProxState));
  const size_t o_rst = take(prox_rank_state_bytes());
  if (off > NOALLOC_SCRATCH_BYTES) {
    g_prox_create_error = "image too large for bq_wprox_noalloc: it needs " + std::to_string(off) +
                          " bytes of scratch, the maximum is " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                          " (use bq_prox_create and bq_wprox)";
    return BQ_EINVAL;
  }
  const char* why = nullptr;
  unsigned char* base = (unsigned char*)scratch_address(&why);
  if (!base) return fail(BQ_EDEVICE, why);
  bq_prox p;
  p.nz = nz; p.ny = ny; p.nx = nx; p.prec = precision;
  p.V = V;
  p.stream = p.own = (hipStream_t)stream;
  p.direct = true;
  p.np = np;
  p.a = base + o_a;
  p.P = P_io ? nullptr : base + o_P;
  p.R = base + o_R;
  p.R2 = r == 0 ? base + o_R2 : nullptr;
  p.partial = (double*)(base + o_part);
  p.st = (ProxState*)(base + o_st);
  p.rst = (ProxRankState*)(base + o_rst);
  // every root pass launched: no rerun, so no copy of the starting point
  p.ssn_slots = p.max_passes - 1;
  p.ssn_slots_rank = p.max_passes_rank - 1;
  bq_status res;
  if (r >= 2)
    res = precision == BQ_F32 ? run_wprox_rank<float>(&p, v, tau, U, r, lambda, tv, cset, n_iter, x_out, P_io, st)
                              : run_wprox_rank<double>(&p, v, tau, U, r, lambda, tv, cset, n_iter, x_out, P_io, st);
  else
    res = precision == BQ_F32
              ? run_wprox<float>(&p, v, tau, r == 1 ? U : nullptr, lambda, tv, cset, n_iter, x_out, P_io, st)
              : run_wprox<double>(&p, v, tau, r == 1 ? U : nullptr, lambda, tv, cset, n_iter, x_out, P_io, st);
  if (res != BQ_OK) g_prox_create_error = p.err;
  return res;
}

}  // extern "C"
