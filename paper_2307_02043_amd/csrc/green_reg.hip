// Green's operator passes with register-resident line FFTs (power-of-two N).
//
// Same passes and data layout as the LDS-Stockham passes of green.hip, but
// for the strided lines (z forward with prologue, y transfer-function
// convolution, z inverse with epilogue) every line transform is held in
// registers by R2 threads (R1 points each) with a single exchange through
// LDS, which cuts LDS traffic about fourfold.  The x passes keep the
// Stockham kernels (whole contiguous rows per access measured faster).
//
// Lane mapping: consecutive lanes take consecutive lines, so global
// accesses are coalesced along x; the exchange layout and the per-thread
// twiddle rows of line_fft_t make every LDS access a base address plus a
// constant offset (no bank conflicts measured).  The strided sweeps of the y
// pass and of the transform sides of the z passes are raw buffer accesses
// with the stride in the scalar offset, which keeps address arithmetic off
// the vector ALU -- the y pass is bound by vector-ALU issue.
#include <cstdio>
#include <string>
#include <vector>

#include "bq_kernels.h"
#include "raw_offsets.h"

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

// Prologue of the z-forward passes: the H values z = j + R2 m (m < H) of
// line L = y N + x of system b.  Each mode has a loop of its own so that all
// loads of a thread are in flight before the first use.
template <typename T, int N, int R2, int H>
__device__ __forceinline__ void zf_prologue(const PassArgs<T>& a, int b, int j, int L, C<T>* d) {
  const size_t N2 = (size_t)N * N, V = N2 * N;
  switch (a.zf_mode) {
    case ZF_XV: {
      const C<T>* v = a.vin + (size_t)b * V + L;
      const T* xp = a.xpot + L;
      T xr[H];
#pragma unroll
      for (int m = 0; m < H; ++m) {
        d[m] = sld(&v[(size_t)(j + R2 * m) * N2]);
        xr[m] = xp[(size_t)(j + R2 * m) * N2];
      }
#pragma unroll
      for (int m = 0; m < H; ++m) d[m] = d[m] * xr[m];
    } break;
    case ZF_XUIN: {
      const int y = L / N, x = L - y * N;
      const C<double>* t = a.inc + (size_t)b * 3 * N;
      const C<double> txy = cmul(t[x], t[N + y]);
      const T* xp = a.xpot + L;
      T xr[H];
#pragma unroll
      for (int m = 0; m < H; ++m) xr[m] = xp[(size_t)(j + R2 * m) * N2];
#pragma unroll
      for (int m = 0; m < H; ++m) d[m] = cvt_r<T>(cmul(txy, t[2 * N + j + R2 * m])) * xr[m];
    } break;
    case ZF_DETCONJ: {
      const C<T> r = conj(a.rdet[(size_t)b * N2 + L]);
#pragma unroll
      for (int m = 0; m < H; ++m) d[m] = (j + R2 * m == N - 1) ? r : C<T>{0, 0};
    } break;
    case ZF_V: {
      const C<T>* v = a.vin + (size_t)b * V + L;
#pragma unroll
      for (int m = 0; m < H; ++m) d[m] = sld(&v[(size_t)(j + R2 * m) * N2]);
    } break;
    case ZF_XP_UPD: {
      const SysState& st = a.state[b];
      const bool first = st.first;
      const C<T> beta{(T)st.beta_x, (T)st.beta_y}, omega{(T)st.omega_x, (T)st.omega_y};
      C<T>* pp = a.pio + (size_t)b * V + L;
      const C<T>* rr = a.rvec + (size_t)b * V + L;
      const C<T>* vv = a.vvec + (size_t)b * V + L;
      const T* xp = a.xpot + L;
      C<T> r[H], po[H], vo[H];
      T xr[H];
#pragma unroll
      for (int m = 0; m < H; ++m) {
        const size_t o = (size_t)(j + R2 * m) * N2;
        r[m] = sld(&rr[o]);
        xr[m] = xp[o];
        if (!first) {
          po[m] = sld(&pp[o]);
          vo[m] = sld(&vv[o]);
        }
      }
#pragma unroll
      for (int m = 0; m < H; ++m) {
        const C<T> pn = first ? r[m] : r[m] + cmul(beta, po[m] - cmul(omega, vo[m]));
        sst(&pp[(size_t)(j + R2 * m) * N2], pn);
        d[m] = pn * xr[m];
      }
    } break;
    default: {
      const C<T>* v = a.vin + (size_t)b * V + L;
#pragma unroll
      for (int m = 0; m < H; ++m) d[m] = conj(sld(&v[(size_t)(j + R2 * m) * N2]));
    } break;
  }
}

// Epilogue of the z-inverse passes: G w at z = j + R2 m (m < H) of line L of
// system b, combined and stored by mode, with the FP64 products of the mode
// accumulated into red (in ascending m).  Operand loads of a mode are all
// issued before the first use.
template <typename T, int N, int R2, int H>
__device__ __forceinline__ void zi_epilogue(const PassArgs<T>& a, int b, int j, int L, const C<T>* gw,
                                            double* red) {
  const size_t N2 = (size_t)N * N, V = N2 * N;
  C<T>* out = a.out + (size_t)b * V + L;
  switch (a.zi_mode) {
    case ZI_G:
#pragma unroll
      for (int m = 0; m < H; ++m) sst(&out[(size_t)(j + R2 * m) * N2], gw[m]);
      break;
    case ZI_GCONJ:
#pragma unroll
      for (int m = 0; m < H; ++m) sst(&out[(size_t)(j + R2 * m) * N2], conj(gw[m]));
      break;
    case ZI_AV_RHAT: {
      const C<T>* vz = a.vz + (size_t)b * V + L;
      const C<T>* rhat = a.rhat + (size_t)b * V + L;
      C<T> o[H], rh[H];
#pragma unroll
      for (int m = 0; m < H; ++m) {
        o[m] = sld(&vz[(size_t)(j + R2 * m) * N2]);
        rh[m] = sld(&rhat[(size_t)(j + R2 * m) * N2]);
      }
#pragma unroll
      for (int m = 0; m < H; ++m) {
        o[m] = o[m] - gw[m];
        sst(&out[(size_t)(j + R2 * m) * N2], o[m]);
        red[0] += (double)rh[m].x * o[m].x + (double)rh[m].y * o[m].y;
        red[1] += (double)rh[m].x * o[m].y - (double)rh[m].y * o[m].x;
      }
    } break;
    case ZI_AS_TS: {
      const C<T>* vz = a.vz + (size_t)b * V + L;
      C<T> sv[H];
#pragma unroll
      for (int m = 0; m < H; ++m) sv[m] = sld(&vz[(size_t)(j + R2 * m) * N2]);
#pragma unroll
      for (int m = 0; m < H; ++m) {
        const C<T> o = sv[m] - gw[m];
        sst(&out[(size_t)(j + R2 * m) * N2], o);
        red[0] += (double)o.x * sv[m].x + (double)o.y * sv[m].y;
        red[1] += (double)o.x * sv[m].y - (double)o.y * sv[m].x;
        red[2] += (double)o.x * o.x + (double)o.y * o.y;
      }
    } break;
    case ZI_RES_NORM: {  // r0 = b - e0 + G w for a solve started from e0
      const C<T>* e0 = a.vz + (size_t)b * V + L;
      C<T> o[H];
      if (a.bsrc) {
        const C<T>* bs = a.bsrc + (size_t)b * V + L;
#pragma unroll
        for (int m = 0; m < H; ++m) o[m] = sld(&bs[(size_t)(j + R2 * m) * N2]) - sld(&e0[(size_t)(j + R2 * m) * N2]);
      } else {
        const int y = L / N, x = L - y * N;
        const C<double>* t = a.inc + (size_t)b * 3 * N;
        const C<double> txy = cmul(t[x], t[N + y]);
#pragma unroll
        for (int m = 0; m < H; ++m)
          o[m] = cvt_r<T>(cmul(txy, t[2 * N + j + R2 * m])) - sld(&e0[(size_t)(j + R2 * m) * N2]);
      }
      C<T>* out2 = a.out2 + (size_t)b * V + L;
#pragma unroll
      for (int m = 0; m < H; ++m) {
        o[m] = o[m] + gw[m];
        sst(&out[(size_t)(j + R2 * m) * N2], o[m]);
        sst(&out2[(size_t)(j + R2 * m) * N2], o[m]);
        red[2] += (double)o[m].x * o[m].x + (double)o[m].y * o[m].y;
      }
    } break;
    default: {  // ZI_G_NORM
      C<T>* out2 = a.out2 ? a.out2 + (size_t)b * V + L : nullptr;
#pragma unroll
      for (int m = 0; m < H; ++m) {
        sst(&out[(size_t)(j + R2 * m) * N2], gw[m]);
        if (out2) sst(&out2[(size_t)(j + R2 * m) * N2], gw[m]);
        red[2] += (double)gw[m].x * gw[m].x + (double)gw[m].y * gw[m].y;
      }
    } break;
  }
}

// Twiddle tables of line_fft_t / line_ifft_t for N-point lines: W_N^n from
// the table exp(-2 pi i n / N), n < N.
template <typename T, int R1, int R2>
__device__ inline void load_twtab_n(C<T>* t, const C<T>* twN, int tid) {
  for (int e = tid; e < R1 * R2; e += RT) {
    const int a = e / R1, b = e - a * R1;
    const C<T> v = twN[a * b];
    t[e] = v;
    if constexpr (R1 != R2) t[R1 * R2 + b * R2 + a] = v;
  }
}

// z lines.  Line L = y N + x of the N^2 lines; element z at z N^2 + L.
// grid (N^2 / LPW, 1, B)
template <typename T, int N>
__global__ void __launch_bounds__(RT) k_zf_r(PassArgs<T> a) {
  constexpr int R1 = RegCfg<N>::R1, R2 = RegCfg<N>::R2, LPW = RT / R2, LS = LineX<R1, R2>::LS, NI = R1 / R2;
  __shared__ C<T> lds[LPW * LS];
  __shared__ C<T> twt[LineX<R1, R2>::TW];
  __shared__ C<T> th[N];
  const int b = blockIdx.z, tid = threadIdx.x, line = tid % LPW, j = tid / LPW;
  if (sys_skip(a.state, a.mask, b)) return;
  load_twtab_n<T, R1, R2>(twt, a.twN, tid);
  for (int i = tid; i < N; i += RT) th[i] = a.twH[i];
  const size_t N2 = (size_t)N * N, V = N2 * N;
  const int L = blockIdx.x * LPW + line;
  C<T> orig[R1], d[R1];
  zf_prologue<T, N, R2, R1>(a, b, j, L, orig);
  __syncthreads();  // tables
  for (int pz = 0; pz < 2; ++pz) {
#pragma unroll
    for (int m = 0; m < R1; ++m) d[m] = pz ? cmul(orig[m], th[j + R2 * m]) : orig[m];
    line_fft_t<T, R1, R2, false>(d, &lds[line * LS], j, twt, pz == 0);
    C<T>* dst = a.zh + (size_t)(b * 2 + pz) * V + L;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int kz = (j + R2 * i) + R1 * k2;
        sst(&dst[(size_t)kz * N2], d[i * R2 + k2]);
      }
  }
}

// y columns of class (pz, px): line L = kz N + kx; element y at
// (kz N + y) N + kx.  grid (N^2 / LPW, 1, 4 B)
template <typename T, int N>
__device__ __forceinline__ void yc_body(const PassArgs<T>& a) {
  constexpr int R1 = RegCfg<N>::R1, R2 = RegCfg<N>::R2, LPW = RT / R2, LS = LineX<R1, R2>::LS, NI = R1 / R2;
  __shared__ C<T> lds[LPW * LS];
  __shared__ C<T> twt[LineX<R1, R2>::TW];
  __shared__ C<T> th[N];
  const int b = blockIdx.z >> 2, cls = blockIdx.z & 3, pz = cls >> 1, px = cls & 1;
  const int tid = threadIdx.x, line = tid % LPW, j = tid / LPW;
  if (sys_skip(a.state, a.mask, b)) return;
  load_twtab_n<T, R1, R2>(twt, a.twN, tid);
  for (int i = tid; i < N; i += RT) th[i] = a.twH[i];
  const size_t N2 = (size_t)N * N, V = N2 * N;
  const int L = blockIdx.x * LPW + line;
  const int kz = L / N, kx = L - kz * N;
  C<T>* col = a.xh + ((size_t)b * 4 + cls) * V + (size_t)kz * N2 + kx;
  C<T> orig[R1], acc[R1], d[R1];
#pragma unroll
  for (int m = 0; m < R1; ++m) {
    orig[m] = sld(&col[(size_t)(j + R2 * m) * N]);
    acc[m] = C<T>{0, 0};
  }
  __syncthreads();
  for (int py = 0; py < 2; ++py) {
#pragma unroll
    for (int m = 0; m < R1; ++m) d[m] = py ? cmul(orig[m], th[j + R2 * m]) : orig[m];
    line_fft_t<T, R1, R2, false>(d, &lds[line * LS], j, twt);
    const C<T>* g = a.ghat + (size_t)((pz * 2 + py) * 2 + px) * V + (size_t)kz * N2 + kx;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int ky = (j + R2 * i) + R1 * k2;
        d[i * R2 + k2] = cmul(d[i * R2 + k2], g[(size_t)ky * N]);
      }
    line_ifft_t<T, R1, R2>(d, &lds[line * LS], j, R1 == R2 ? twt : twt + R1 * R2, py == 0);
#pragma unroll
    for (int m = 0; m < R1; ++m) acc[m] = acc[m] + (py ? cmulc(d[m], th[j + R2 * m]) : d[m]);
  }
#pragma unroll
  for (int m = 0; m < R1; ++m) sst(&col[(size_t)(j + R2 * m) * N], acc[m]);
}

// z lines, inverse, both z parities summed, epilogue and FP64 partials.
// NTH threads, LPW = NTH / R2 lines per workgroup; grid (N^2 / LPW, 1, B);
// partials[(b * NP + blockIdx.x) * 4 + k]
template <typename T, int N, int NTH = RT>
__device__ __forceinline__ void zi_body(const PassArgs<T>& a) {
  constexpr int R1 = RegCfg<N>::R1, R2 = RegCfg<N>::R2, LPW = NTH / R2, LS = LineX<R1, R2>::LS, NI = R1 / R2;
  __shared__ C<T> lds[LPW * LS];
  __shared__ C<T> twt[LineX<R1, R2>::TW];
  __shared__ C<T> th[N];
  __shared__ double red_scratch[(NTH / 64) * 3];
  const int b = blockIdx.z, tid = threadIdx.x, line = tid % LPW, j = tid / LPW;
  if (sys_skip(a.state, a.mask, b)) return;
  for (int e = tid; e < R1 * R2; e += NTH) {  // twiddle table of the N-point lines
    const int ta = e / R1, tb = e - ta * R1;
    twt[e] = a.twN[ta * tb];
    if constexpr (R1 != R2) twt[R1 * R2 + tb * R2 + ta] = a.twN[ta * tb];
  }
  for (int i = tid; i < N; i += NTH) th[i] = a.twH[i];
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
      for (int k2 = 0; k2 < R2; ++k2) d[i * R2 + k2] = sld(&src[(size_t)((j + R2 * i) + R1 * k2) * N2]);
    line_ifft_t<T, R1, R2>(d, &lds[line * LS], j, R1 == R2 ? twt : twt + R1 * R2, pz == 0);
#pragma unroll
    for (int m = 0; m < R1; ++m) acc[m] = acc[m] + (pz ? cmulc(d[m], th[j + R2 * m]) : d[m]);
  }
  double red[3] = {0.0, 0.0, 0.0};
  const int mode = a.zi_mode;
  zi_epilogue<T, N, R2, R1>(a, b, j, L, acc, red);
  if (mode >= ZI_AV_RHAT) {
    block_sum<NTH, 3>(red, red_scratch);
    if (tid == 0) {
      double* p = a.partial + ((size_t)b * gridDim.x + blockIdx.x) * 4;
      p[0] = red[0];
      p[1] = red[1];
      p[2] = red[2];
      p[3] = 0.0;
    }
  }
}

// Threads per workgroup of the parity-split z-inverse pass: 32 lines of
// complex64 at N = 256 (72 KB of LDS, two workgroups per CU), so that one
// wave instruction covers two 256-byte runs of a z plane instead of four
// 128-byte pieces (90.5 -> 86.0 ms of z-inverse per 256^3 step; 1024
// threads spill); 16 lines otherwise.
template <typename T, int N>
constexpr int rtz_r() { return (N == 256 && sizeof(T) == 4) ? 512 : RT; }

template <typename T, int N>
__global__ void __launch_bounds__(RT) k_yc_r(PassArgs<T> a) { yc_body<T, N>(a); }
template <typename T, int N>
__global__ void __launch_bounds__((rtz_r<T, N>())) k_zi_r(PassArgs<T> a) { zi_body<T, N, rtz_r<T, N>()>(a); }


// ===========================================================================
// Padded-line variants (N = 16..128): a strided line of N points is
// transformed as one 2N-point line with zero upper half instead of two
// pre-twiddled N-point lines.  Padded frequency k' = 2k + p lands in parity
// class p at index k, and the sum over both classes of the conjugate-
// twiddled N-point inverses equals the first N outputs of the 2N-point
// inverse, so no input copy, accumulator or parity twiddle is needed.  The
// zero half of the input and the unused half of the inverse's outputs are
// removed by the compiler.
// ===========================================================================
template <int N> struct PadCfg { static constexpr bool ok = false; static constexpr int R1 = 1, R2 = 1; };
#define BQ_PC(NN, A, B_) \
  template <> struct PadCfg<NN> { static constexpr bool ok = true; static constexpr int R1 = A, R2 = B_; };
BQ_PC(16, 8, 4)
BQ_PC(32, 8, 8)
BQ_PC(64, 16, 8)
BQ_PC(96, 24, 8)
BQ_PC(128, 16, 16)
BQ_PC(256, 32, 16)
#undef BQ_PC
constexpr bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
// The padded form is used up to N = 128, and for the y pass at N = 256 in
// complex64 (a 512-point line takes 70 KB of LDS per 16 lines; complex128
// would need 139 KB, so it keeps the parity-split form).  At N = 96 (192-
// point lines of 24 x 8) only the y pass is padded, in complex64: the other
// passes of that grid are the LDS Stockham ones, which share its layouts,
// and complex128 keeps the LDS y pass (24 values per thread in FP64 would
// cost half the waves).
template <typename T, int N>
struct PadSel {
  static constexpr bool ok = PadCfg<N>::ok && (pow2(N) ? (N <= 128 || sizeof(T) == 4) : sizeof(T) == 4);
};


// Twiddle tables of line_fft_t / line_ifft_t for the padded 2N-point lines:
// W_{2N}^n = exp(-i pi n / N) from the half-angle table (n < 2N).
// INV_ROWS: also the inverse table (rows of k1) after the forward one; the
// split-exchange transforms read both directions from the forward table.
template <typename T, int N, int R1, int R2, int NTH = RT, bool INV_ROWS = true>
__device__ inline void load_twtab_pad(C<T>* t, const C<T>* twH, int tid) {
  for (int e = tid; e < R1 * R2; e += NTH) {
    const int a = e / R1, b = e - a * R1, n = a * b;
    const C<T> w = twH[n < N ? n : n - N];
    const C<T> v = n < N ? w : C<T>{-w.x, -w.y};
    t[e] = v;
    if constexpr (R1 != R2 && INV_ROWS) t[R1 * R2 + b * R2 + a] = v;
  }
}

// Threads per workgroup of the padded z passes: 64 lines of complex64 at
// N = 128, so that one wave instruction covers 512 contiguous bytes of a
// z plane instead of four 128-byte pieces (16 lines elsewhere; complex128
// would not fit in LDS).  The y pass keeps 16 lines: its 16-wave barrier
// would stall a pass bound by vector issue.
template <typename T, int N>
constexpr int rtz() { return (N == 128 && sizeof(T) == 4) ? 1024 : RT; }

// The z-forward pass writes no partial sums, so the autotuner may also run
// it 1024 threads wide at other sizes (complex64, where the lines fit in LDS).
template <typename T, int N>
constexpr bool zf_wide_ok() { return sizeof(T) == 4 && N <= 128 && pow2(N) && PadCfg<N>::ok; }

// Padded z lines of three or more exchange rounds (R1 = 3 R2 at N = 96) go
// through an LDS line of R2 rows per round (18 KB per workgroup instead of
// 55 KB for the whole 24-row line).
template <int N>
constexpr bool zsplit() { return PadCfg<N>::R1 / PadCfg<N>::R2 > 2; }

template <typename T, int N, int NTH = rtz<T, N>()>
__global__ void __launch_bounds__(NTH) k_zf_p(PassArgs<T> a) {
  constexpr int R1 = PadCfg<N>::R1, R2 = PadCfg<N>::R2, LPW = NTH / R2, NI = R1 / R2;
  constexpr bool SPLIT = zsplit<N>();
  constexpr int LS = SPLIT ? LineXS<R1, R2>::LS : LineX<R1, R2>::LS, H = R1 / 2;  // H: nonzero inputs per thread
  constexpr int TW = SPLIT ? LineXS<R1, R2>::TW : LineX<R1, R2>::TW;
  constexpr uint32_t SZ = sizeof(C<T>);
  __shared__ C<T> lds[LPW * LS];
  __shared__ C<T> twt[TW];
  const int b = blockIdx.z, tid = threadIdx.x, line = tid % LPW, j = tid / LPW;
  if (sys_skip(a.state, a.mask, b)) return;
  load_twtab_pad<T, N, R1, R2, NTH, !SPLIT>(twt, a.twH, tid);
  const size_t N2 = (size_t)N * N, V = N2 * N;
  const int L = blockIdx.x * LPW + line;
  C<T> d[R1];
  zf_prologue<T, N, R2, H>(a, b, j, L, d);
#pragma unroll
  for (int m = H; m < R1; ++m) d[m] = C<T>{0, 0};
  __syncthreads();  // twiddle table
  if constexpr (SPLIT)
    line_fft_ts<T, R1, R2, false>(d, &lds[line * LS], j, twt, false);
  else
    line_fft_t<T, R1, R2, false>(d, &lds[line * LS], j, twt, false);
  // padded frequency kp = k1 + R1 k2 (k1 = j + R2 i): class kp & 1 = j & 1,
  // plane kp >> 1; the two classes of system b are consecutive volumes
  using O = PadRaw<N, R1, R2, SZ>;
  const brsrc rz = make_rsrc(a.zh + (size_t)b * 2 * V, O::z_bytes);
  const uint32_t vo = O::z_v(j, L);
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2)
      bstore<T, true>(d[i * R2 + k2], rz, vo, O::z_s(i, k2));
}

// y columns of class (pz, px), line L = kz N + kx
template <typename T, int N>
__global__ void __launch_bounds__(RT) k_yc_p(PassArgs<T> a) {
  constexpr int R1 = PadCfg<N>::R1, R2 = PadCfg<N>::R2, LPW = RT / R2, NI = R1 / R2;
  // R1 > R2 (the 512-point lines at N = 256): the exchange runs in NI rounds
  // through an LDS line of R2 rows, so that 4 workgroups fit a CU (2 with
  // the whole line: 76 KB each)
  constexpr bool SPLIT = R1 != R2;
  constexpr int LS = SPLIT ? LineXS<R1, R2>::LS : LineX<R1, R2>::LS, H = R1 / 2;
  constexpr int TW = SPLIT ? LineXS<R1, R2>::TW : LineX<R1, R2>::TW;
  constexpr uint32_t SZ = sizeof(C<T>);
  __shared__ C<T> lds[LPW * LS];
  __shared__ C<T> twt[TW];
  // XCD-aware order: workgroup h runs on XCD h mod 8; the B systems of one
  // (class, line block) take consecutive slots of the same XCD, so the
  // transfer-function slab they share is fetched into that XCD's L2 once.
  constexpr int NLB = N * N / LPW;
  const YcSlot slot = yc_slot(blockIdx.x, a.B, NLB);
  const int b = slot.b, cls = slot.cls, lb = slot.lb, pz = cls >> 1, px = cls & 1;
  const int tid = threadIdx.x, line = tid % LPW, j = tid / LPW;
  if (sys_skip(a.state, a.mask, b)) return;
  load_twtab_pad<T, N, R1, R2, RT, !SPLIT>(twt, a.twH, tid);
  const size_t N2 = (size_t)N * N, V = N2 * N;
  const int L = lb * LPW + line;
  const int kz = L / N, kx = L - kz * N;
  // column: one resource per (system, class) slice, element y at (kz N + y) N + kx
  using O = PadRaw<N, R1, R2, SZ>;
  const brsrc rc = make_rsrc(a.xh + ((size_t)b * 4 + cls) * V, O::y_bytes);
  const uint32_t vo = O::y_v(kz, kx, j);
  C<T> d[R1];
#pragma unroll
  for (int m = 0; m < R1; ++m) d[m] = (m < H) ? bload<T, true>(rc, vo, O::y_s(m)) : C<T>{0, 0};
  // padded frequency kp = k1 + R1 k2 (k1 = j + R2 i) is py class kp & 1 = j & 1
  // at index kp >> 1; classes (pz, 0, px) and (pz, 1, px) are 2V apart
  const brsrc rg = make_rsrc(a.ghat + (size_t)(pz * 4 + px) * V, O::g_bytes);
  const uint32_t vg = O::g_v(j, kz, kx);
  // the transfer function is loaded before the forward transform (its
  // latency then overlaps the transform instead of stalling the product);
  // at R1 = 32 the 32 extra values would cost a wave per SIMD
  C<T> g[R1];
  if constexpr (!SPLIT) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) g[i * R2 + k2] = bload<T>(rg, vg, O::g_s(i, k2));
  }
  __syncthreads();
  if constexpr (SPLIT)
    line_fft_ts<T, R1, R2, false>(d, &lds[line * LS], j, twt);
  else
    line_fft_t<T, R1, R2, false>(d, &lds[line * LS], j, twt);
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2)
      d[i * R2 + k2] = cmul(d[i * R2 + k2], SPLIT ? bload<T>(rg, vg, O::g_s(i, k2)) : g[i * R2 + k2]);
  if constexpr (SPLIT)
    line_ifft_ts<T, R1, R2>(d, &lds[line * LS], j, twt, false);
  else
    line_ifft_t<T, R1, R2>(d, &lds[line * LS], j, twt, false);
#pragma unroll
  for (int m = 0; m < H; ++m) bstore<T, true>(d[m], rc, vo, O::y_s(m));
}

// z lines, inverse (first N outputs of the padded inverse), epilogue
template <typename T, int N>
__global__ void __launch_bounds__((rtz<T, N>())) k_zi_p(PassArgs<T> a) {
  constexpr int NTH = rtz<T, N>();
  constexpr int R1 = PadCfg<N>::R1, R2 = PadCfg<N>::R2, LPW = NTH / R2, NI = R1 / R2;
  constexpr bool SPLIT = zsplit<N>();
  constexpr int LS = SPLIT ? LineXS<R1, R2>::LS : LineX<R1, R2>::LS, H = R1 / 2;
  constexpr int TW = SPLIT ? LineXS<R1, R2>::TW : LineX<R1, R2>::TW;
  constexpr uint32_t SZ = sizeof(C<T>);
  __shared__ C<T> lds[LPW * LS];
  __shared__ C<T> twt[TW];
  __shared__ double red_scratch[(NTH / 64) * 3];
  const int b = blockIdx.z, tid = threadIdx.x, line = tid % LPW, j = tid / LPW;
  if (sys_skip(a.state, a.mask, b)) return;
  load_twtab_pad<T, N, R1, R2, NTH, !SPLIT>(twt, a.twH, tid);
  const int L = blockIdx.x * LPW + line;
  using O = PadRaw<N, R1, R2, SZ>;
  const brsrc rz = make_rsrc(a.zh + (size_t)b * 2 * N * N * N, O::z_bytes);
  const uint32_t vo = O::z_v(j, L);
  C<T> d[R1];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2)
      d[i * R2 + k2] = bload<T, true>(rz, vo, O::z_s(i, k2));
  __syncthreads();
  if constexpr (SPLIT)
    line_ifft_ts<T, R1, R2>(d, &lds[line * LS], j, twt, false);
  else
    line_ifft_t<T, R1, R2>(d, &lds[line * LS], j, R1 == R2 ? twt : twt + R1 * R2, false);
  double red[3] = {0.0, 0.0, 0.0};
  const int mode = a.zi_mode;
  zi_epilogue<T, N, R2, H>(a, b, j, L, d, red);
  if (mode >= ZI_AV_RHAT) {
    block_sum<NTH, 3>(red, red_scratch);
    if (tid == 0) {
      double* p = a.partial + ((size_t)b * gridDim.x + blockIdx.x) * 4;
      p[0] = red[0];
      p[1] = red[1];
      p[2] = red[2];
      p[3] = 0.0;
    }
  }
}

template <typename T>
bool reg_supported(int N) {
  switch (N) {
    case 16: case 32: case 64: case 128: case 256: return true;
    default: return false;
  }
}

template <typename T>
int reg_num_partials(int N) {
  switch (N) {  // grid of the z-inverse kernel (padded variant up to 128)
    case 16: return N * N / (rtz<T, 16>() / PadCfg<16>::R2);
    case 32: return N * N / (rtz<T, 32>() / PadCfg<32>::R2);
    case 64: return N * N / (rtz<T, 64>() / PadCfg<64>::R2);
    case 128: return N * N / (rtz<T, 128>() / PadCfg<128>::R2);
    case 256: return N * N / (rtz_r<T, 256>() / RegCfg<256>::R2);
    default: return -1;
  }
}

template <typename T, int N>
static void launch_reg_N(const PassArgs<T>& a, hipStream_t st, PassTimer* tm, bool fused_xy) {
  // The y pass and the z passes choose their line form separately (same
  // layouts): at N = 256 the padded 512-point y lines cut the y pass's
  // vector work by ~30 %, while the z passes, bound by memory, keep the
  // parity-split form at twice the occupancy (padded z passes measured slower).
  constexpr bool PADY = PadSel<T, N>::ok;
  constexpr bool PADZ = PadSel<T, N>::ok && N <= 128;
  constexpr int NTZ = PADZ ? rtz<T, N>() : RT;  // threads of the z kernels
  constexpr int LPWZ = NTZ / (PADZ ? PadCfg<N>::R2 : RegCfg<N>::R2);
  constexpr int LPWY = RT / (PADY ? PadCfg<N>::R2 : RegCfg<N>::R2);
  const dim3 blk(RT);
  if (tm) tm->start(P_ZF, st);
  if constexpr (PADZ) {
    if constexpr (zf_wide_ok<T, N>()) {
      if (a.zf_threads == 1024 || a.zf_threads == RT) {  // tuned width
        if (a.zf_threads == 1024)
          hipLaunchKernelGGL((k_zf_p<T, N, 1024>), dim3(N * N / (1024 / PadCfg<N>::R2), 1, a.B), dim3(1024), 0,
                             st, a);
        else
          hipLaunchKernelGGL((k_zf_p<T, N, RT>), dim3(N * N / (RT / PadCfg<N>::R2), 1, a.B), dim3(RT), 0, st, a);
      } else {
        hipLaunchKernelGGL((k_zf_p<T, N>), dim3(N * N / LPWZ, 1, a.B), dim3(NTZ), 0, st, a);
      }
    } else {
      hipLaunchKernelGGL((k_zf_p<T, N>), dim3(N * N / LPWZ, 1, a.B), dim3(NTZ), 0, st, a);
    }
  } else
    hipLaunchKernelGGL((k_zf_r<T, N>), dim3(N * N / LPWZ, 1, a.B), blk, 0, st, a);
  if (fused_xy) {
    if (tm) { tm->stop(st); tm->start(P_XY, st); }
    xy_fused_launch<T>(a, st);
  } else {
    // x passes: the LDS-Stockham kernels read and write whole contiguous rows,
    // which measured faster than the register kernels' 64-byte row segments
    if (tm) { tm->stop(st); tm->start(P_XF, st); }
    launch_xf_stockham<T, N>(a, st);
    if (tm) { tm->stop(st); tm->start(P_YC, st); }
    if constexpr (PADY)  // 4 N^2 / LPW is a multiple of 8 for every padded size
      hipLaunchKernelGGL((k_yc_p<T, N>), dim3(4 * (N * N / LPWY) * a.B), blk, 0, st, a);
    else
      hipLaunchKernelGGL((k_yc_r<T, N>), dim3(N * N / LPWY, 1, 4 * a.B), blk, 0, st, a);
    if (tm) { tm->stop(st); tm->start(P_XI, st); }
    launch_xi_stockham<T, N>(a, st);
  }
  if (tm) { tm->stop(st); tm->start(P_ZI, st); }
  if constexpr (PADZ) {
    hipLaunchKernelGGL((k_zi_p<T, N>), dim3(N * N / LPWZ, 1, a.B), dim3(NTZ), 0, st, a);
  } else {
    constexpr int NTI = rtz_r<T, N>(), LPWI = NTI / RegCfg<N>::R2;
    hipLaunchKernelGGL((k_zi_r<T, N>), dim3(N * N / LPWI, 1, a.B), dim3(NTI), 0, st, a);
  }
  if (tm) tm->stop(st);
}

// The padded register z and y passes of a grid whose x passes are the LDS
// Stockham ones (N = 96 in complex64); false (nothing launched) if the grid
// has none.  The z-inverse pass then writes N^2 / LPW partials per system.
template <typename T>
bool pad_zf_apply(const PassArgs<T>& a, hipStream_t st) {
  if constexpr (PadSel<T, 96>::ok) {
    if (a.N == 96) {
      constexpr int LPW = rtz<T, 96>() / PadCfg<96>::R2;
      hipLaunchKernelGGL((k_zf_p<T, 96>), dim3(96 * 96 / LPW, 1, a.B), dim3(rtz<T, 96>()), 0, st, a);
      return true;
    }
  }
  return false;
}
template <typename T>
bool pad_y_apply(const PassArgs<T>& a, hipStream_t st) {
  if constexpr (PadSel<T, 96>::ok) {
    if (a.N == 96) {
      constexpr int LPWY = RT / PadCfg<96>::R2;
      hipLaunchKernelGGL((k_yc_p<T, 96>), dim3(4 * (96 * 96 / LPWY) * a.B), dim3(RT), 0, st, a);
      return true;
    }
  }
  return false;
}
template <typename T>
bool pad_zi_apply(const PassArgs<T>& a, hipStream_t st) {
  if constexpr (PadSel<T, 96>::ok) {
    if (a.N == 96) {
      constexpr int LPW = rtz<T, 96>() / PadCfg<96>::R2;
      hipLaunchKernelGGL((k_zi_p<T, 96>), dim3(96 * 96 / LPW, 1, a.B), dim3(rtz<T, 96>()), 0, st, a);
      return true;
    }
  }
  return false;
}
template <typename T>
int pad_num_partials(int N) {
  if constexpr (PadSel<T, 96>::ok)
    if (N == 96) return 96 * 96 / (rtz<T, 96>() / PadCfg<96>::R2);
  return -1;
}
template bool pad_zf_apply<float>(const PassArgs<float>&, hipStream_t);
template bool pad_zf_apply<double>(const PassArgs<double>&, hipStream_t);
template bool pad_y_apply<float>(const PassArgs<float>&, hipStream_t);
template bool pad_y_apply<double>(const PassArgs<double>&, hipStream_t);
template bool pad_zi_apply<float>(const PassArgs<float>&, hipStream_t);
template bool pad_zi_apply<double>(const PassArgs<double>&, hipStream_t);
template int pad_num_partials<float>(int);
template int pad_num_partials<double>(int);

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
template int reg_num_partials<float>(int);
template int reg_num_partials<double>(int);

template <typename T>
bool zf_threads_valid(int N, int nth) {
  if (nth != RT && nth != 1024) return false;
  switch (N) {
    case 16: return nth == RT || zf_wide_ok<T, 16>();
    case 32: return nth == RT || zf_wide_ok<T, 32>();
    case 64: return nth == RT || zf_wide_ok<T, 64>();
    case 128: return nth == RT || zf_wide_ok<T, 128>();
    default: return false;  // N = 256: parity-split z passes, one shape
  }
}
template bool zf_threads_valid<float>(int, int);
template bool zf_threads_valid<double>(int, int);
template int reg_apply<float>(const PassArgs<float>&, hipStream_t, PassTimer*);
template int reg_apply<double>(const PassArgs<double>&, hipStream_t, PassTimer*);

// ---------------------------------------------------------------------------
// Host-side audit of the raw buffer accesses (bq_audit_raw_ranges): every
// offset the padded kernels can form, over their launch grids, against the
// size of the resource it goes through.
// ---------------------------------------------------------------------------
namespace {

struct Audit {
  long long accesses = 0;
  int bad = 0;
  std::string msg;
  void fail(const std::string& m) {
    if (bad++ < 8) msg += m + "\n";
  }
  // one access: a 32-bit per-thread part and a 32-bit compile-time part
  // (computed exactly in 64 bits), an element of esz bytes, a resource of
  // `bytes`
  void check(const char* what, int N, int esz, uint64_t v, uint64_t s, size_t bytes) {
    ++accesses;
    if (v >= (1ull << 32) || s >= (1ull << 32) || v + s >= (1ull << 32) || v + s + esz > bytes)
      fail(std::string(what) + " N=" + std::to_string(N) + " esz=" + std::to_string(esz) + ": offset " +
           std::to_string(v + s) + " outside " + std::to_string(bytes) + " bytes");
  }
  void check_resource(const char* what, int N, size_t bytes, size_t base_elems, size_t alloc_elems, int esz) {
    if (bytes >= (1ull << 31)) fail(std::string(what) + " N=" + std::to_string(N) + ": resource over 2^31 bytes");
    if (base_elems * esz + bytes > alloc_elems * esz)
      fail(std::string(what) + " N=" + std::to_string(N) + ": resource passes the end of its allocation");
  }
};

// z passes of NTH threads: lines L = block * LPW + tid % LPW, j = tid / LPW
template <typename T, int N, int NTH>
void audit_z(Audit& A, const char* what) {
  constexpr int R1 = PadCfg<N>::R1, R2 = PadCfg<N>::R2, LPW = NTH / R2, NI = R1 / R2;
  constexpr uint32_t SZ = sizeof(C<T>);
  using O = PadRaw<N, R1, R2, SZ>;
  const size_t V = O::V;
  if ((N * N) % LPW != 0) A.fail(std::string(what) + ": N^2 lines not a whole number of workgroups");
  // system b's two classes from zh + 2 V b, inside a workspace of 2 V B (B = 1 is the tightest)
  A.check_resource(what, N, O::z_bytes, 0, 2 * V, SZ);
  for (int blk = 0; blk < N * N / LPW; ++blk)
    for (int tid = 0; tid < NTH; ++tid) {
      const int L = blk * LPW + tid % LPW, j = tid / LPW;
      if (L < 0 || L >= N * N) A.fail(std::string(what) + ": line out of range");
      for (int i = 0; i < NI; ++i)
        for (int k2 = 0; k2 < R2; ++k2) A.check(what, N, SZ, O::z_v64(j, L), O::z_s64(i, k2), O::z_bytes);
    }
}

template <typename T, int N>
void audit_y(Audit& A) {
  constexpr int R1 = PadCfg<N>::R1, R2 = PadCfg<N>::R2, LPW = RT / R2, NI = R1 / R2, H = R1 / 2;
  constexpr int NLB = N * N / LPW;
  constexpr uint32_t SZ = sizeof(C<T>);
  using O = PadRaw<N, R1, R2, SZ>;
  const size_t V = O::V;
  A.check_resource("y column", N, O::y_bytes, 0, V, SZ);
  // class (pz, px) base (pz * 4 + px) V of the 8 V transfer function, the
  // largest base being class (1, 0, 1)
  A.check_resource("transfer function", N, O::g_bytes, 5 * V, 8 * V, SZ);
  // workgroup -> (system, class, line block) is a bijection for every batch
  // size up to 40 (4 NLB is a multiple of 8)
  if ((4 * NLB) % 8 != 0) A.fail("y pass: 4 N^2 / LPW not a multiple of 8");
  for (int B = 1; B <= 40; ++B) {
    std::vector<unsigned char> seen((size_t)4 * NLB * B, 0);
    for (int h = 0; h < 4 * NLB * B; ++h) {
      const YcSlot t = yc_slot(h, B, NLB);
      if (t.b < 0 || t.b >= B || t.cls < 0 || t.cls >= 4 || t.lb < 0 || t.lb >= NLB) {
        A.fail("y pass N=" + std::to_string(N) + " B=" + std::to_string(B) + ": workgroup outside the grid");
        break;
      }
      unsigned char& c = seen[((size_t)t.b * 4 + t.cls) * NLB + t.lb];
      if (c++) A.fail("y pass N=" + std::to_string(N) + " B=" + std::to_string(B) + ": slot taken twice");
    }
  }
  for (int lb = 0; lb < NLB; ++lb)
    for (int tid = 0; tid < RT; ++tid) {
      const int L = lb * LPW + tid % LPW, j = tid / LPW;
      const int kz = L / N, kx = L - kz * N;
      for (int m = 0; m < H; ++m) A.check("y column", N, SZ, O::y_v64(kz, kx, j), O::y_s64(m), O::y_bytes);
      for (int i = 0; i < NI; ++i)
        for (int k2 = 0; k2 < R2; ++k2)
          A.check("transfer function", N, SZ, O::g_v64(j, kz, kx), O::g_s64(i, k2), O::g_bytes);
    }
}

template <typename T, int N>
void audit_N(Audit& A) {
  if constexpr (PadSel<T, N>::ok && N <= 128) {
    audit_z<T, N, rtz<T, N>()>(A, "z lines");
    if constexpr (zf_wide_ok<T, N>()) {
      audit_z<T, N, 1024>(A, "z lines (1024-wide forward)");
      audit_z<T, N, RT>(A, "z lines (256-wide forward)");
    }
  }
  if constexpr (PadSel<T, N>::ok) audit_y<T, N>(A);
}

template <typename T>
void audit_T(Audit& A) {
  audit_N<T, 16>(A);
  audit_N<T, 32>(A);
  audit_N<T, 64>(A);
  audit_N<T, 96>(A);
  audit_N<T, 128>(A);
  audit_N<T, 256>(A);
}

}  // namespace

}  // namespace bq

extern "C" int bq_audit_raw_ranges(char* report, int report_len, long long* accesses) {
  bq::Audit A;
  bq::audit_T<float>(A);
  bq::audit_T<double>(A);
  if (accesses) *accesses = A.accesses;
  if (report && report_len > 0) {
    const std::string m = A.bad ? A.msg : std::string("all raw buffer accesses in range");
    std::snprintf(report, (size_t)report_len, "%s", m.c_str());
  }
  return A.bad;
}
