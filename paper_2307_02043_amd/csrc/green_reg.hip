// Green's operator passes with register-resident line FFTs (power-of-two N).
//
// Same passes and data layout as the LDS-Stockham passes of green.hip, but
// for the strided lines (z forward with prologue, y transfer-function
// convolution, z inverse with epilogue) every N-point line transform is held
// in registers by R2 threads (R1 points each) with a single exchange through
// LDS, which cuts LDS traffic about fourfold.  The x passes keep the
// Stockham kernels (whole contiguous rows per access measured faster).
//
// Lane mapping: consecutive lanes take consecutive lines, so global
// accesses are coalesced along x and the LDS exchange (line stride N + 1) is
// conflict free.
#include "bq_kernels.h"

namespace bq {

template <int N> struct RegCfg { static constexpr bool ok = false; static constexpr int R1 = 1, R2 = 1; };
#define BQ_RC(NN, A, B_) \
  template <> struct RegCfg<NN> { static constexpr bool ok = true; static constexpr int R1 = A, R2 = B_; };
BQ_RC(16, 4, 4)
BQ_RC(32, 8, 4)
BQ_RC(64, 8, 8)
BQ_RC(128, 16, 8)
BQ_RC(256, 16, 16)
#undef BQ_RC

constexpr int RT = 256;  // threads per workgroup

template <typename T>
__device__ inline C<T> cvt_r(C<double> a) { return C<T>{(T)a.x, (T)a.y}; }

// z lines.  Line L = y N + x of the N^2 lines; element z at z N^2 + L.
// grid (N^2 / LPW, 1, B)
template <typename T, int N>
__global__ void __launch_bounds__(RT) k_zf_r(PassArgs<T> a) {
  constexpr int R1 = RegCfg<N>::R1, R2 = RegCfg<N>::R2, LPW = RT / R2, LS = N + 1, NI = R1 / R2;
  __shared__ C<T> lds[LPW * LS];
  __shared__ C<T> tw[N];
  __shared__ C<T> th[N];
  const int b = blockIdx.z, tid = threadIdx.x, line = tid % LPW, j = tid / LPW;
  if (sys_skip(a.state, a.mask, b)) return;
  for (int i = tid; i < N; i += RT) { tw[i] = a.twN[i]; th[i] = a.twH[i]; }
  const size_t N2 = (size_t)N * N, V = N2 * N;
  const int L = blockIdx.x * LPW + line;
  const int y = L / N, x = L - y * N;
  C<T> orig[R1], d[R1];
#pragma unroll
  for (int m = 0; m < R1; ++m) {
    const int z = j + R2 * m;
    const size_t n = (size_t)z * N2 + L;
    C<T> val;
    switch (a.zf_mode) {
      case ZF_XV: val = a.vin[b * V + n] * a.xpot[n]; break;
      case ZF_XUIN: {
        const C<double>* t = a.inc + (size_t)b * 3 * N;
        val = cvt_r<T>(cmul(cmul(t[x], t[N + y]), t[2 * N + z])) * a.xpot[n];
      } break;
      case ZF_DETCONJ:
        val = (z == N - 1) ? conj(a.rdet[(size_t)b * N2 + L]) : C<T>{0, 0};
        break;
      case ZF_V: val = a.vin[b * V + n]; break;
      default: val = conj(a.vin[b * V + n]); break;
    }
    orig[m] = val;
  }
  __syncthreads();  // tables
  for (int pz = 0; pz < 2; ++pz) {
#pragma unroll
    for (int m = 0; m < R1; ++m) d[m] = pz ? cmul(orig[m], th[j + R2 * m]) : orig[m];
    line_fft<T, N, R1, R2, false>(d, &lds[line * LS], 1, j, tw);
    C<T>* dst = a.zh + (size_t)(b * 2 + pz) * V + L;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int kz = (j + R2 * i) + R1 * k2;
        dst[(size_t)kz * N2] = d[i * R2 + k2];
      }
  }
}

// y columns of class (pz, px): line L = kz N + kx; element y at
// (kz N + y) N + kx.  grid (N^2 / LPW, 1, 4 B)
template <typename T, int N>
__device__ __forceinline__ void yc_body(const PassArgs<T>& a) {
  constexpr int R1 = RegCfg<N>::R1, R2 = RegCfg<N>::R2, LPW = RT / R2, LS = N + 1, NI = R1 / R2;
  __shared__ C<T> lds[LPW * LS];
  __shared__ C<T> tw[N];
  __shared__ C<T> th[N];
  const int b = blockIdx.z >> 2, cls = blockIdx.z & 3, pz = cls >> 1, px = cls & 1;
  const int tid = threadIdx.x, line = tid % LPW, j = tid / LPW;
  if (sys_skip(a.state, a.mask, b)) return;
  for (int i = tid; i < N; i += RT) { tw[i] = a.twN[i]; th[i] = a.twH[i]; }
  const size_t N2 = (size_t)N * N, V = N2 * N;
  const int L = blockIdx.x * LPW + line;
  const int kz = L / N, kx = L - kz * N;
  C<T>* col = a.xh + ((size_t)b * 4 + cls) * V + (size_t)kz * N2 + kx;
  C<T> orig[R1], acc[R1], d[R1];
#pragma unroll
  for (int m = 0; m < R1; ++m) {
    orig[m] = col[(size_t)(j + R2 * m) * N];
    acc[m] = C<T>{0, 0};
  }
  __syncthreads();
  for (int py = 0; py < 2; ++py) {
#pragma unroll
    for (int m = 0; m < R1; ++m) d[m] = py ? cmul(orig[m], th[j + R2 * m]) : orig[m];
    line_fft<T, N, R1, R2, false>(d, &lds[line * LS], 1, j, tw);
    const C<T>* g = a.ghat + (size_t)((pz * 2 + py) * 2 + px) * V + (size_t)kz * N2 + kx;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int ky = (j + R2 * i) + R1 * k2;
        d[i * R2 + k2] = cmul(d[i * R2 + k2], g[(size_t)ky * N]);
      }
    line_ifft<T, N, R1, R2>(d, &lds[line * LS], 1, j, tw);
#pragma unroll
    for (int m = 0; m < R1; ++m) acc[m] = acc[m] + (py ? cmulc(d[m], th[j + R2 * m]) : d[m]);
  }
#pragma unroll
  for (int m = 0; m < R1; ++m) col[(size_t)(j + R2 * m) * N] = acc[m];
}

// z lines, inverse, both z parities summed, epilogue and FP64 partials.
// grid (N^2 / LPW, 1, B); partials[(b * NP + blockIdx.x) * 4 + k]
template <typename T, int N>
__device__ __forceinline__ void zi_body(const PassArgs<T>& a) {
  constexpr int R1 = RegCfg<N>::R1, R2 = RegCfg<N>::R2, LPW = RT / R2, LS = N + 1, NI = R1 / R2;
  __shared__ C<T> lds[LPW * LS];
  __shared__ C<T> tw[N];
  __shared__ C<T> th[N];
  __shared__ double red_scratch[(RT / 64) * 3];
  const int b = blockIdx.z, tid = threadIdx.x, line = tid % LPW, j = tid / LPW;
  if (sys_skip(a.state, a.mask, b)) return;
  for (int i = tid; i < N; i += RT) { tw[i] = a.twN[i]; th[i] = a.twH[i]; }
  const size_t N2 = (size_t)N * N, V = N2 * N;
  const int L = blockIdx.x * LPW + line;
  C<T> acc[R1], d[R1];
#pragma unroll
  for (int m = 0; m < R1; ++m) acc[m] = C<T>{0, 0};
  __syncthreads();
  for (int pz = 0; pz < 2; ++pz) {
    const C<T>* src = a.zh + (size_t)(b * 2 + pz) * V + L;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) d[i * R2 + k2] = src[(size_t)((j + R2 * i) + R1 * k2) * N2];
    line_ifft<T, N, R1, R2>(d, &lds[line * LS], 1, j, tw);
#pragma unroll
    for (int m = 0; m < R1; ++m) acc[m] = acc[m] + (pz ? cmulc(d[m], th[j + R2 * m]) : d[m]);
  }
  double red[3] = {0.0, 0.0, 0.0};
  const int mode = a.zi_mode;
#pragma unroll
  for (int m = 0; m < R1; ++m) {
    const size_t n = (size_t)b * V + (size_t)(j + R2 * m) * N2 + L;
    const C<T> gw = acc[m];
    if (mode == ZI_G) {
      a.out[n] = gw;
    } else if (mode == ZI_GCONJ) {
      a.out[n] = conj(gw);
    } else if (mode == ZI_AV_RHAT) {
      const C<T> o = a.vz[n] - gw;
      a.out[n] = o;
      const C<T> rh = a.rhat[n];
      red[0] += (double)rh.x * o.x + (double)rh.y * o.y;
      red[1] += (double)rh.x * o.y - (double)rh.y * o.x;
    } else if (mode == ZI_AS_TS) {
      const C<T> sv = a.vz[n];
      const C<T> o = sv - gw;
      a.out[n] = o;
      red[0] += (double)o.x * sv.x + (double)o.y * sv.y;
      red[1] += (double)o.x * sv.y - (double)o.y * sv.x;
      red[2] += (double)o.x * o.x + (double)o.y * o.y;
    } else {  // ZI_G_NORM
      a.out[n] = gw;
      if (a.out2) a.out2[n] = gw;
      red[2] += (double)gw.x * gw.x + (double)gw.y * gw.y;
    }
  }
  if (mode >= ZI_AV_RHAT) {
    block_sum<RT, 3>(red, red_scratch);
    if (tid == 0) {
      double* p = a.partial + ((size_t)b * gridDim.x + blockIdx.x) * 4;
      p[0] = red[0];
      p[1] = red[1];
      p[2] = red[2];
      p[3] = 0.0;
    }
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(RT) k_yc_r(PassArgs<T> a) { yc_body<T, N>(a); }
template <typename T, int N>
__global__ void __launch_bounds__(RT) k_zi_r(PassArgs<T> a) { zi_body<T, N>(a); }

template <typename T>
bool reg_supported(int N) {
  switch (N) {
    case 16: case 32: case 64: case 128: case 256: return true;
    default: return false;
  }
}

int reg_num_partials(int N) {
  switch (N) {
    case 16: return N * N / (RT / RegCfg<16>::R2);
    case 32: return N * N / (RT / RegCfg<32>::R2);
    case 64: return N * N / (RT / RegCfg<64>::R2);
    case 128: return N * N / (RT / RegCfg<128>::R2);
    case 256: return N * N / (RT / RegCfg<256>::R2);
    default: return -1;
  }
}

template <typename T, int N>
static void launch_reg_N(const PassArgs<T>& a, hipStream_t st, PassTimer* tm, bool fused_xy) {
  constexpr int LPW = RT / RegCfg<N>::R2;
  const dim3 blk(RT);
  if (tm) tm->start(P_ZF, st);
  hipLaunchKernelGGL((k_zf_r<T, N>), dim3(N * N / LPW, 1, a.B), blk, 0, st, a);
  if (fused_xy) {
    if (tm) { tm->stop(st); tm->start(P_XY, st); }
    xy_fused_launch<T>(a, st);
  } else {
    // x passes: the LDS-Stockham kernels read and write whole contiguous rows,
    // which measured faster than the register kernels' 64-byte row segments
    if (tm) { tm->stop(st); tm->start(P_XF, st); }
    launch_xf_stockham<T, N>(a, st);
    if (tm) { tm->stop(st); tm->start(P_YC, st); }
    hipLaunchKernelGGL((k_yc_r<T, N>), dim3(N * N / LPW, 1, 4 * a.B), blk, 0, st, a);
    if (tm) { tm->stop(st); tm->start(P_XI, st); }
    launch_xi_stockham<T, N>(a, st);
  }
  if (tm) { tm->stop(st); tm->start(P_ZI, st); }
  hipLaunchKernelGGL((k_zi_r<T, N>), dim3(N * N / LPW, 1, a.B), blk, 0, st, a);
  if (tm) tm->stop(st);
}

template <typename T>
int reg_apply(const PassArgs<T>& a, hipStream_t st, PassTimer* tm) {
  const bool fused = a.xy_fused && xy_fused_supported<T>(a.N);
  switch (a.N) {
    case 16: launch_reg_N<T, 16>(a, st, tm, fused); break;
    case 32: launch_reg_N<T, 32>(a, st, tm, fused); break;
    case 64: launch_reg_N<T, 64>(a, st, tm, fused); break;
    case 128: launch_reg_N<T, 128>(a, st, tm, fused); break;
    case 256: launch_reg_N<T, 256>(a, st, tm, fused); break;
    default: return -1;
  }
  return 0;
}

template bool reg_supported<float>(int);
template bool reg_supported<double>(int);
template int reg_apply<float>(const PassArgs<float>&, hipStream_t, PassTimer*);
template int reg_apply<double>(const PassArgs<double>&, hipStream_t, PassTimer*);

}  // namespace bq
