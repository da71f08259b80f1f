// Fused x/y pass of the Green's operator: one workgroup per (system, pz, kz)
// plane, the whole N x N plane resident in LDS (128^2 complex64 = 136 KB
// with padding on gfx950's 160 KB LDS).
//
// For each x parity px:
//   rows    : twiddle exp(-i pi px x / N), N-point FFT
//   columns : for py in {0,1}: twiddle, FFT, multiply by the transfer-function
//             class (pz, py, px), inverse FFT, conjugate twiddle, summed
//   rows    : inverse FFT, conjugate twiddle, accumulated over px in registers
// Reads the plane (twice, the second time from cache), writes it once.
// Only the column pass reads the transfer function.
//
// Line FFTs are register resident: a line of N = R1 R2 points is held by R2
// threads with R1 points each (thread j holds x[j + R2 m]); a radix-R1 DFT in
// registers, twiddles W_N^{j k1}, one exchange through LDS, and radix-R2 DFTs
// give X[k1 + R1 k2] (k1 = j + R2 i).  The inverse runs the mirror sequence.
// The LDS row stride is padded so that consecutive rows start 64 bytes apart
// modulo 256 bytes, spreading row and column accesses over the banks.
//
// Workgroups are mapped XCD-aware: hardware workgroup h runs on XCD h mod 8;
// all B systems of one plane are given consecutive slots of the same XCD so
// that the four transfer-function planes they read are shared in its L2.
#include "bq_kernels.h"

namespace bq {

template <typename T, int N> struct XYCfg { static constexpr bool ok = false; };
#define BQ_XY(TT, NN, A, B_, NTH)                 \
  template <> struct XYCfg<TT, NN> {              \
    static constexpr bool ok = true;              \
    static constexpr int R1 = A, R2 = B_, NTHR = NTH; \
  };
BQ_XY(float, 16, 4, 4, 64)
BQ_XY(float, 32, 8, 4, 128)
BQ_XY(float, 64, 8, 8, 512)
BQ_XY(float, 128, 16, 8, 512)
BQ_XY(double, 16, 4, 4, 64)
BQ_XY(double, 32, 8, 4, 128)
BQ_XY(double, 64, 8, 8, 512)
#undef BQ_XY

// Smallest row stride >= N + 1 (complex elements) with stride * size = 64 mod 256 bytes.
template <typename T>
constexpr int xy_stride(int N) {
  int ls = N + 1;
  while ((ls * (int)sizeof(C<T>)) % 256 != 64) ++ls;
  return ls;
}

template <typename T, int N>
__global__ void __launch_bounds__((XYCfg<T, N>::NTHR)) k_xy(PassArgs<T> a) {
  constexpr int R1 = XYCfg<T, N>::R1, R2 = XYCfg<T, N>::R2, NTHR = XYCfg<T, N>::NTHR;
  constexpr int LS = xy_stride<T>(N), RPR = NTHR / R2, NR = N / RPR, NI = R1 / R2;
  // With two row rounds per thread the px accumulator would not fit in
  // registers: the px = 0 result then goes to a scratch plane (cache
  // resident) and is added back during px = 1.
  constexpr bool SCRATCH = NR > 1;
  __shared__ C<T> buf[N * LS];
  __shared__ C<T> tw[N];
  __shared__ C<T> th[N];
  const int B = a.B;
  const int h = blockIdx.x;
  const int jq = h >> 3;
  const int b = jq % B;
  const int q = (jq / B) * 8 + (h & 7);
  const int pz = q / N, kz = q - pz * N;
  if (sys_skip(a.state, a.mask, b)) return;
  const int tid = threadIdx.x, j = tid % R2, l = tid / R2;
  // Column phase: within a wavefront the R2 threads of a column are 64 / R2
  // lanes apart and consecutive lanes take consecutive columns, so that a
  // column access touches 64/R2 columns x R2 rows spread over all banks.
  constexpr int CPW = (64 / R2) < RPR ? (64 / R2) : RPR;  // columns per wave
  const int lane = tid & 63, wv = tid >> 6;
  const int jc = (RPR >= 64 / R2) ? lane / CPW : j;
  const int lc = (RPR >= 64 / R2) ? wv * CPW + lane % CPW : l;
  for (int i = tid; i < N; i += NTHR) { tw[i] = a.twN[i]; th[i] = a.twH[i]; }
  const size_t N2 = (size_t)N * N, V = N2 * N;
  C<T>* plane = a.zh + ((size_t)b * 2 + pz) * V + (size_t)kz * N2;
  C<T>* scratch = a.xh + ((size_t)b * 2 + pz) * V + (size_t)kz * N2;
  constexpr int NRA = SCRATCH ? 1 : NR;
  C<T> acc[NRA][R1];
#pragma unroll
  for (int r = 0; r < NRA; ++r)
#pragma unroll
    for (int m = 0; m < R1; ++m) acc[r][m] = C<T>{0, 0};
  C<T> d[R1], c[R1], accc[R1];
  __syncthreads();
  for (int px = 0; px < 2; ++px) {
    // ---- rows: forward FFT of the px class --------------------------------
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int y = r * RPR + l;
#pragma unroll
      for (int m = 0; m < R1; ++m) {
        const int xi = j + R2 * m;
        const C<T> v = plane[(size_t)y * N + xi];
        d[m] = px ? cmul(v, th[xi]) : v;
      }
      line_fft<T, N, R1, R2, false>(d, &buf[y * LS], 1, j, tw);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) buf[y * LS + (j + R2 * i) + R1 * k2] = d[i * R2 + k2];
    }
    __syncthreads();
    // ---- columns: both y parities, transfer function ----------------------
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int kx = r * RPR + lc;
#pragma unroll
      for (int m = 0; m < R1; ++m) {
        c[m] = buf[(jc + R2 * m) * LS + kx];
        accc[m] = C<T>{0, 0};
      }
      __syncthreads();
      for (int py = 0; py < 2; ++py) {
#pragma unroll
        for (int m = 0; m < R1; ++m) d[m] = py ? cmul(c[m], th[jc + R2 * m]) : c[m];
        line_fft<T, N, R1, R2, false>(d, &buf[kx], LS, jc, tw);
        const C<T>* g = a.ghat + (size_t)((pz * 2 + py) * 2 + px) * V + (size_t)kz * N2 + kx;
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int k2 = 0; k2 < R2; ++k2) {
            const int ky = (jc + R2 * i) + R1 * k2;
            d[i * R2 + k2] = cmul(d[i * R2 + k2], g[(size_t)ky * N]);
          }
        line_ifft<T, N, R1, R2>(d, &buf[kx], LS, jc, tw);
#pragma unroll
        for (int m = 0; m < R1; ++m) accc[m] = accc[m] + (py ? cmulc(d[m], th[jc + R2 * m]) : d[m]);
      }
#pragma unroll
      for (int m = 0; m < R1; ++m) buf[(jc + R2 * m) * LS + kx] = accc[m];
    }
    __syncthreads();
    // ---- rows: inverse FFT, accumulate the px classes -----------------------
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int y = r * RPR + l;
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) d[i * R2 + k2] = buf[y * LS + (j + R2 * i) + R1 * k2];
      __syncthreads();
      line_ifft<T, N, R1, R2>(d, &buf[y * LS], 1, j, tw);
      if constexpr (SCRATCH) {
#pragma unroll
        for (int m = 0; m < R1; ++m) {
          const size_t o = (size_t)y * N + j + R2 * m;
          if (px == 0) scratch[o] = d[m];
          else plane[o] = scratch[o] + cmulc(d[m], th[j + R2 * m]);
        }
      } else {
#pragma unroll
        for (int m = 0; m < R1; ++m) acc[r][m] = acc[r][m] + (px ? cmulc(d[m], th[j + R2 * m]) : d[m]);
      }
    }
    __syncthreads();
  }
  if constexpr (!SCRATCH) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int y = r * RPR + l;
#pragma unroll
      for (int m = 0; m < R1; ++m) plane[(size_t)y * N + j + R2 * m] = acc[r][m];
    }
  }
}

template <typename T>
bool xy_fused_supported(int N) {
  switch (N) {
    case 16: return XYCfg<T, 16>::ok;
    case 32: return XYCfg<T, 32>::ok;
    case 64: return XYCfg<T, 64>::ok;
    case 128: return XYCfg<T, 128>::ok;
    default: return false;
  }
}

template <typename T, int N>
static void launch_xy_N(const PassArgs<T>& a, hipStream_t st) {
  if constexpr (XYCfg<T, N>::ok)
    hipLaunchKernelGGL((k_xy<T, N>), dim3(2 * N * a.B), dim3(XYCfg<T, N>::NTHR), 0, st, a);
}

template <typename T>
int xy_fused_launch(const PassArgs<T>& a, hipStream_t st) {
  switch (a.N) {
    case 16: launch_xy_N<T, 16>(a, st); break;
    case 32: launch_xy_N<T, 32>(a, st); break;
    case 64: launch_xy_N<T, 64>(a, st); break;
    case 128: launch_xy_N<T, 128>(a, st); break;
    default: return -1;
  }
  return 0;
}

template bool xy_fused_supported<float>(int);
template bool xy_fused_supported<double>(int);
template int xy_fused_launch<float>(const PassArgs<float>&, hipStream_t);
template int xy_fused_launch<double>(const PassArgs<double>&, hipStream_t);

}  // namespace bq
