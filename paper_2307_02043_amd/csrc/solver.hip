// BiCGSTAB vector updates, per-system scalar updates, detector and gradient
// reduction of the Lippmann-Schwinger data term (gfx950).
//
// Every kernel covers all systems of a mini-batch (blockIdx.z / blockIdx.x =
// system) and skips the systems whose solve has ended, so converged
// illuminations retire individually while the others keep iterating.  Inner
// products and norms are accumulated in FP64 whatever the field precision;
// per-workgroup partial sums are reduced by the scalar kernels in a fixed
// order, so results are bitwise reproducible.
#include "bq_kernels.h"

namespace bq {

int vec_num_partials(size_t V) {
  size_t wg = (V + VEC_WG * 8 - 1) / (VEC_WG * 8);
  if (wg > 512) wg = 512;
  if (wg < 1) wg = 1;
  return (int)wg;
}

template <typename T>
__device__ inline C<double> c2d(C<T> a) { return C<double>{(double)a.x, (double)a.y}; }

// s = r - alpha v ; partial ||s||^2
template <typename T>
__global__ void __launch_bounds__(VEC_WG) k_vec_s(VecArgs<T> a) {
  __shared__ double scratch[(VEC_WG / 64) * 1];
  const int b = blockIdx.z;
  const SysState& s = a.state[b];
  if (s.status != SYS_RUNNING) return;
  const C<T> alpha{(T)s.alpha_x, (T)s.alpha_y};
  const size_t off = (size_t)b * a.V;
  double acc[1] = {0.0};
  for (size_t i = blockIdx.x * (size_t)VEC_WG + threadIdx.x; i < a.V; i += (size_t)gridDim.x * VEC_WG) {
    const C<T> sv = sld(&a.r[off + i]) - cmul(alpha, sld(&a.v[off + i]));
    sst(&a.s[off + i], sv);
    acc[0] += (double)sv.x * sv.x + (double)sv.y * sv.y;
  }
  block_sum<VEC_WG, 1>(acc, scratch);
  if (threadIdx.x == 0) {
    double* p = a.partial + ((size_t)b * gridDim.x + blockIdx.x) * 4;
    p[0] = acc[0];
  }
}

// e += alpha p (+ omega s) ; r = s - omega t ; partials ||r||^2, <rhat, r>
template <typename T>
__global__ void __launch_bounds__(VEC_WG) k_vec_xr(VecArgs<T> a) {
  __shared__ double scratch[(VEC_WG / 64) * 3];
  const int b = blockIdx.z;
  const SysState& s = a.state[b];
  if (s.status != SYS_RUNNING) return;
  const bool half = s.sflag;
  const C<T> alpha{(T)s.alpha_x, (T)s.alpha_y}, omega{(T)s.omega_x, (T)s.omega_y};
  const size_t off = (size_t)b * a.V;
  double acc[3] = {0.0, 0.0, 0.0};
  for (size_t i = blockIdx.x * (size_t)VEC_WG + threadIdx.x; i < a.V; i += (size_t)gridDim.x * VEC_WG) {
    const size_t k = off + i;
    if (half) {
      sst(&a.e[k], sld(&a.e[k]) + cmul(alpha, sld(&a.p[k])));
    } else {
      const C<T> sv = sld(&a.s[k]);
      sst(&a.e[k], sld(&a.e[k]) + cmul(alpha, sld(&a.p[k])) + cmul(omega, sv));
      const C<T> r = sv - cmul(omega, sld(&a.t[k]));
      sst(&a.r[k], r);
      const C<T> rh = sld(&a.rhat[k]);
      acc[0] += (double)r.x * r.x + (double)r.y * r.y;
      acc[1] += (double)rh.x * r.x + (double)rh.y * r.y;
      acc[2] += (double)rh.x * r.y - (double)rh.y * r.x;
    }
  }
  block_sum<VEC_WG, 3>(acc, scratch);
  if (threadIdx.x == 0) {
    double* p = a.partial + ((size_t)b * gridDim.x + blockIdx.x) * 4;
    p[0] = acc[0];
    p[1] = acc[1];
    p[2] = acc[2];
  }
}

template <typename T>
__global__ void __launch_bounds__(VEC_WG) k_vec_norm(VecArgs<T> a, const C<T>* f) {
  __shared__ double scratch[(VEC_WG / 64) * 1];
  const int b = blockIdx.z;
  const size_t off = (size_t)b * a.V;
  double acc[1] = {0.0};
  for (size_t i = blockIdx.x * (size_t)VEC_WG + threadIdx.x; i < a.V; i += (size_t)gridDim.x * VEC_WG) {
    const C<T> v = f[off + i];
    acc[0] += (double)v.x * v.x + (double)v.y * v.y;
  }
  block_sum<VEC_WG, 1>(acc, scratch);
  if (threadIdx.x == 0) a.partial[((size_t)b * gridDim.x + blockIdx.x) * 4] = acc[0];
}

template <typename T>
__global__ void __launch_bounds__(VEC_WG) k_fill_incident(int N, const C<double>* inc, C<T>* out) {
  const int b = blockIdx.z;
  const size_t V = (size_t)N * N * N;
  const C<double>* t = inc + (size_t)b * 3 * N;
  for (size_t i = blockIdx.x * (size_t)VEC_WG + threadIdx.x; i < V; i += (size_t)gridDim.x * VEC_WG) {
    const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / ((size_t)N * N));
    const C<double> u = cmul(cmul(t[x], t[N + y]), t[2 * N + z]);
    out[(size_t)b * V + i] = C<T>{(T)u.x, (T)u.y};
  }
}

// e_b = 0 for the systems whose right-hand side is zero (their solution),
// after a solve started from a given point
template <typename T>
__global__ void __launch_bounds__(VEC_WG) k_zero_if_b0(const SysState* st, C<T>* e, size_t V) {
  const int b = blockIdx.z;
  if (st[b].bnorm2 != 0.0) return;
  for (size_t i = blockIdx.x * (size_t)VEC_WG + threadIdx.x; i < V; i += (size_t)gridDim.x * VEC_WG)
    e[(size_t)b * V + i] = C<T>{0, 0};
}

template <typename T>
void vec_zero_if_b0(int B, size_t V, const SysState* st, C<T>* e, hipStream_t s) {
  hipLaunchKernelGGL((k_zero_if_b0<T>), dim3(vec_num_partials(V), 1, B), dim3(VEC_WG), 0, s, st, e, V);
}

template <typename T>
void vec_s(const VecArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_vec_s<T>), dim3(vec_num_partials(a.V), 1, a.B), dim3(VEC_WG), 0, st, a);
}
template <typename T>
void vec_xr(const VecArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_vec_xr<T>), dim3(vec_num_partials(a.V), 1, a.B), dim3(VEC_WG), 0, st, a);
}
template <typename T>
void vec_norm(const VecArgs<T>& a, const C<T>* f, hipStream_t st) {
  hipLaunchKernelGGL((k_vec_norm<T>), dim3(vec_num_partials(a.V), 1, a.B), dim3(VEC_WG), 0, st, a, f);
}
template <typename T>
void vec_fill_incident(int B, int N, const C<double>* inc, C<T>* out, hipStream_t st) {
  const size_t V = (size_t)N * N * N;
  hipLaunchKernelGGL((k_fill_incident<T>), dim3(vec_num_partials(V), 1, B), dim3(VEC_WG), 0, st, N, inc, out);
}

// ---------------------------------------------------------------------------
// Scalar updates: one workgroup per system sums the partials in a fixed order.
// ---------------------------------------------------------------------------
template <int K>
__device__ inline void sum_partials(const double* part, int np, int b, double* out, double* scratch) {
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) {
    const double* p = part + ((size_t)b * np + i) * 4;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += p[k];
  }
  block_sum<256, K>(v, scratch);
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = v[k];
}

__device__ inline bool finite3(double a, double b, double c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

__global__ void __launch_bounds__(256) k_sc_init(SysState* st, const double* part_r, int np_r,
                                                 const double* part_b, int np_b, double bfix,
                                                 double tol, int max_iter, double brk) {
  __shared__ double scratch[4 * 3];
  const int b = blockIdx.x;
  double rv[3], bv[1] = {bfix};
  sum_partials<3>(part_r, np_r, b, rv, scratch);
  if (part_b) sum_partials<1>(part_b, np_b, b, bv, scratch);
  if (threadIdx.x != 0) return;
  SysState s{};
  s.tol = tol;
  s.max_iter = max_iter;
  s.brk = brk;
  s.bnorm2 = bv[0];
  const double rn2 = rv[2];
  s.rho_x = rn2;  // rhat = r0, so <rhat, r0> = ||r0||^2
  s.rho_y = 0.0;
  s.alpha_x = 1.0;
  s.omega_x = 1.0;
  s.first = 1;
  s.iters = 0;
  if (!(isfinite(rn2) && isfinite(s.bnorm2))) {
    s.status = SYS_NONFINITE;
    s.res = NAN;
  } else if (s.bnorm2 == 0.0) {
    s.status = SYS_CONVERGED;
    s.res = 0.0;
  } else {
    s.res = sqrt(rn2 / s.bnorm2);
    s.status = (s.res <= tol) ? SYS_CONVERGED : SYS_RUNNING;
  }
  st[b] = s;
}

__global__ void __launch_bounds__(256) k_sc_beta(SysState* st, const double* part, int np) {
  __shared__ double scratch[4 * 3];
  const int b = blockIdx.x;
  if (st[b].status != SYS_RUNNING) return;
  double v[3];
  const bool first = st[b].first;
  if (!first) sum_partials<3>(part, np, b, v, scratch);
  if (threadIdx.x != 0) return;
  SysState s = st[b];
  double rnx, rny;
  if (!first) {
    if (s.sflag) {
      s.status = SYS_CONVERGED;
      st[b] = s;
      return;
    }
    if (!finite3(v[0], v[1], v[2])) {
      s.status = SYS_NONFINITE;
      st[b] = s;
      return;
    }
    s.res = sqrt(v[0] / s.bnorm2);
    if (s.res <= s.tol) {
      s.status = SYS_CONVERGED;
      st[b] = s;
      return;
    }
    if (hypot(s.omega_x, s.omega_y) < s.brk) {
      s.status = SYS_BREAKDOWN;
      st[b] = s;
      return;
    }
    rnx = v[1];
    rny = v[2];
  } else {
    rnx = s.rho_x;
    rny = s.rho_y;
  }
  if (s.iters >= s.max_iter) {
    s.status = SYS_NOTCONV;
    st[b] = s;
    return;
  }
  if (hypot(rnx, rny) < s.brk) {
    s.status = SYS_BREAKDOWN;
    st[b] = s;
    return;
  }
  // beta = (rho_new / rho) (alpha / omega)
  const C<double> rn{rnx, rny}, rho{s.rho_x, s.rho_y}, al{s.alpha_x, s.alpha_y}, om{s.omega_x, s.omega_y};
  const double d1 = rho.x * rho.x + rho.y * rho.y, d2 = om.x * om.x + om.y * om.y;
  const C<double> q1 = cmulc(rn, rho) * (1.0 / d1);
  const C<double> q2 = cmulc(al, om) * (1.0 / d2);
  const C<double> beta = cmul(q1, q2);
  s.beta_x = beta.x;
  s.beta_y = beta.y;
  s.rhon_x = rnx;
  s.rhon_y = rny;
  s.iters += 1;
  st[b] = s;
}

__global__ void __launch_bounds__(256) k_sc_alpha(SysState* st, const double* part, int np) {
  __shared__ double scratch[4 * 2];
  const int b = blockIdx.x;
  if (st[b].status != SYS_RUNNING) return;
  double v[2];
  sum_partials<2>(part, np, b, v, scratch);
  if (threadIdx.x != 0) return;
  SysState s = st[b];
  s.first = 0;
  s.mvs += 1;  // the matvec A p of this iteration ran for this system
  const double d = v[0] * v[0] + v[1] * v[1];
  if (!(isfinite(v[0]) && isfinite(v[1]))) {
    s.status = SYS_NONFINITE;
  } else if (d == 0.0 || hypot(v[0], v[1]) < s.brk) {
    s.status = SYS_BREAKDOWN;
  } else {
    const C<double> a = cmulc(C<double>{s.rhon_x, s.rhon_y}, C<double>{v[0], v[1]}) * (1.0 / d);
    s.alpha_x = a.x;
    s.alpha_y = a.y;
  }
  st[b] = s;
}

__global__ void __launch_bounds__(256) k_sc_s(SysState* st, const double* part, int np) {
  __shared__ double scratch[4];
  const int b = blockIdx.x;
  if (st[b].status != SYS_RUNNING) return;
  double v[1];
  sum_partials<1>(part, np, b, v, scratch);
  if (threadIdx.x != 0) return;
  SysState s = st[b];
  if (!isfinite(v[0])) {
    s.status = SYS_NONFINITE;
  } else {
    const double rs = sqrt(v[0] / s.bnorm2);
    if (rs <= s.tol) {
      s.sflag = 1;
      s.res = rs;
    }
  }
  st[b] = s;
}

__global__ void __launch_bounds__(256) k_sc_omega(SysState* st, const double* part, int np) {
  __shared__ double scratch[4 * 3];
  const int b = blockIdx.x;
  if (st[b].status != SYS_RUNNING || st[b].sflag) return;
  double v[3];
  sum_partials<3>(part, np, b, v, scratch);
  if (threadIdx.x != 0) return;
  SysState s = st[b];
  s.mvs += 1;  // the matvec A s of this iteration ran for this system
  if (!finite3(v[0], v[1], v[2])) {
    s.status = SYS_NONFINITE;
  } else {
    const double tt = v[2];
    s.omega_x = tt > 0.0 ? v[0] / tt : 0.0;
    s.omega_y = tt > 0.0 ? v[1] / tt : 0.0;
    s.rho_x = s.rhon_x;
    s.rho_y = s.rhon_y;
  }
  st[b] = s;
}

void sc_init(int B, SysState* st, const double* part_r, int np_r, const double* part_b, int np_b,
             double bfix, double tol, int max_iter, double brk, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_init, dim3(B), dim3(256), 0, s, st, part_r, np_r, part_b, np_b, bfix, tol, max_iter,
                     brk);
}
void sc_beta(int B, SysState* st, const double* part, int np, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_beta, dim3(B), dim3(256), 0, s, st, part, np);
}
void sc_alpha(int B, SysState* st, const double* part, int np, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_alpha, dim3(B), dim3(256), 0, s, st, part, np);
}
void sc_s(int B, SysState* st, const double* part, int np, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_s, dim3(B), dim3(256), 0, s, st, part, np);
}
void sc_omega(int B, SysState* st, const double* part, int np, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_omega, dim3(B), dim3(256), 0, s, st, part, np);
}

// ---------------------------------------------------------------------------
// Detector and gradient
// ---------------------------------------------------------------------------
int det_num_partials(int N) {
  int wg = (N * N + 255) / 256;
  return wg > 64 ? 64 : wg;
}

template <typename T>
__global__ void __launch_bounds__(256) k_detector(int N, const C<T>* field, int sub, const C<double>* inc,
                                                  const C<T>* ymeas, C<T>* out, double* partial) {
  __shared__ double scratch[4];
  const int b = blockIdx.z;
  const size_t N2 = (size_t)N * N, V = N2 * N;
  const C<double>* t = inc + (size_t)b * 3 * N;
  double acc[1] = {0.0};
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < N2; i += (size_t)gridDim.x * 256) {
    const int x = (int)(i % N), y = (int)(i / N);
    C<T> H = field[(size_t)b * V + (size_t)(N - 1) * N2 + i];
    if (sub) {
      const C<double> u = cmul(cmul(t[x], t[N + y]), t[2 * N + (N - 1)]);
      H = H - C<T>{(T)u.x, (T)u.y};
    }
    if (ymeas) {
      const C<T> r = H - ymeas[(size_t)b * N2 + i];
      out[(size_t)b * N2 + i] = r;
      acc[0] += 0.5 * ((double)r.x * r.x + (double)r.y * r.y);
    } else {
      out[(size_t)b * N2 + i] = H;
    }
  }
  if (partial) {
    block_sum<256, 1>(acc, scratch);
    if (threadIdx.x == 0) partial[(size_t)b * gridDim.x + blockIdx.x] = acc[0];
  }
}

template <typename T>
void detector(int B, int N, const C<T>* field, int sub, const C<double>* inc, const C<T>* ymeas,
              C<T>* out, double* partial, int np, hipStream_t st) {
  hipLaunchKernelGGL((k_detector<T>), dim3(np, 1, B), dim3(256), 0, st, N, field, sub, inc, ymeas, out, partial);
}

// r = H - y in place on the (propagated) detector images; partial 1/2 |r|^2
template <typename T>
__global__ void __launch_bounds__(256) k_det_residual(int N, C<T>* rdet, const C<T>* ymeas, double* partial) {
  __shared__ double scratch[4];
  const int b = blockIdx.z;
  const size_t N2 = (size_t)N * N;
  double acc[1] = {0.0};
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < N2; i += (size_t)gridDim.x * 256) {
    const C<T> r = rdet[(size_t)b * N2 + i] - ymeas[(size_t)b * N2 + i];
    rdet[(size_t)b * N2 + i] = r;
    acc[0] += 0.5 * ((double)r.x * r.x + (double)r.y * r.y);
  }
  block_sum<256, 1>(acc, scratch);
  if (threadIdx.x == 0) partial[(size_t)b * gridDim.x + blockIdx.x] = acc[0];
}

template <typename T>
void det_residual(int B, int N, C<T>* rdet, const C<T>* ymeas, double* partial, int np, hipStream_t st) {
  hipLaunchKernelGGL((k_det_residual<T>), dim3(np, 1, B), dim3(256), 0, st, N, rdet, ymeas, partial);
}

template <typename T>
__global__ void __launch_bounds__(256) k_gradient(int B, int N, const C<T>* u, const C<double>* inc,
                                                  const C<T>* wbar, double scale, int accumulate, T* g) {
  const size_t V = (size_t)N * N * N;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < V; i += (size_t)gridDim.x * 256) {
    double acc = 0.0;
    const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / ((size_t)N * N));
    for (int b = 0; b < B; ++b) {
      C<double> ub;
      if (u) {
        ub = c2d(u[(size_t)b * V + i]);
      } else {
        const C<double>* t = inc + (size_t)b * 3 * N;
        ub = cmul(cmul(t[x], t[N + y]), t[2 * N + z]);
        if (sizeof(T) == 4) ub = C<double>{(double)(float)ub.x, (double)(float)ub.y};
      }
      const C<double> w = c2d(wbar[(size_t)b * V + i]);
      acc += ub.x * w.x - ub.y * w.y;  // Re(u wbar) = Re(conj(u) w)
    }
    acc *= scale;
    g[i] = accumulate ? (T)((double)g[i] + acc) : (T)acc;
  }
}

template <typename T>
void gradient(int B, int N, const C<T>* u, const C<double>* inc, const C<T>* wbar, double scale,
              int accumulate, T* g, hipStream_t st) {
  const size_t V = (size_t)N * N * N;
  size_t wg = (V + 255) / 256;
  if (wg > 8192) wg = 8192;
  hipLaunchKernelGGL((k_gradient<T>), dim3((unsigned)wg), dim3(256), 0, st, B, N, u, inc, wbar, scale, accumulate, g);
}

#define BQ_INST(T)                                                                                   \
  template void vec_s<T>(const VecArgs<T>&, hipStream_t);                                           \
  template void vec_xr<T>(const VecArgs<T>&, hipStream_t);                                          \
  template void vec_norm<T>(const VecArgs<T>&, const C<T>*, hipStream_t);                           \
  template void vec_fill_incident<T>(int, int, const C<double>*, C<T>*, hipStream_t);               \
  template void vec_zero_if_b0<T>(int, size_t, const SysState*, C<T>*, hipStream_t);                 \
  template void det_residual<T>(int, int, C<T>*, const C<T>*, double*, int, hipStream_t);             \
  template void detector<T>(int, int, const C<T>*, int, const C<double>*, const C<T>*, C<T>*,        \
                            double*, int, hipStream_t);                                             \
  template void gradient<T>(int, int, const C<T>*, const C<double>*, const C<T>*, double, int, T*,   \
                            hipStream_t);
BQ_INST(float)
BQ_INST(double)
#undef BQ_INST

}  // namespace bq
