// Green's operator of the discretised Lippmann-Schwinger equation on gfx950.
//
// G v = crop(IFFT_2N(ghat_P . FFT_2N(pad v))) is evaluated without ever
// materialising the (2N)^3 padded grid.  Splitting every padded frequency
// k' = 2k + p by parity p in {0,1}^3 turns the padded convolution into eight
// N^3 circular convolutions of the pre-twiddled field v . exp(-i pi p.n / N)
// with the parity classes of ghat_P; the twiddles are scalars per line and
// are applied inside the passes, so only N-point FFTs are ever run.
//
// Power-of-two grids run the register-resident line passes of green_reg.hip;
// at N = 96 in complex64 the z and y passes are register passes as well
// (padded 24 x 8 lines) between the LDS x passes here.
//
// Passes (one system per blockIdx.z, all systems of a batch in one launch):
//   Zf  : z lines, prologue (x . v, x . u_in, S^T conj r, ...), both z parities
//   Xf  : x rows, both x parities              (split path)
//   Yc  : y columns, FFT -> . ghat -> IFFT, both y parities summed
//   Xi  : x rows, IFFT, x parities summed
//   Zi  : z lines, IFFT, z parities summed, epilogue + FP64 partial sums
//
// ghat_P itself is precomputed here too (truncated Helmholtz kernel,
// oversampled by Q per axis, cropped to the lags -N..N-1, transformed on the
// 2N grid), in FP64 with the same FFT machinery.
#include <type_traits>

#include "bq_kernels.h"

namespace bq {

constexpr int NT = 256;  // threads per workgroup for all line passes

// Largest divisor of N that keeps one tile of lines within ~32 KB of LDS
// and at most 16 lines wide (16 complex64 = 128 contiguous bytes per row).
template <typename T>
constexpr int tile_w(int N) {
  int lim = 32768 / (N * (int)sizeof(C<T>));
  if (lim > 16) lim = 16;
  if (lim < 1) lim = 1;
  for (int t = lim; t >= 1; --t)
    if (N % t == 0) return t;
  return 1;
}

template <typename T>
__device__ inline C<T> cvt(C<double> a) { return C<T>{(T)a.x, (T)a.y}; }

// ---------------------------------------------------------------------------
// Zf: z-direction forward FFTs of both z parities, with the prologue.
// grid (N/TX, N, B)
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(NT) k_zf(PassArgs<T> a) {
  constexpr int TX = tile_w<T>(N), LS = N + 1, TOT = TX * N, EPT = (TOT + NT - 1) / NT;
  __shared__ C<T> lds[TX * LS];
  __shared__ C<T> tw[N];
  __shared__ C<T> th[N];
  const int b = blockIdx.z, y = blockIdx.y, x0 = blockIdx.x * TX, tid = threadIdx.x;
  if (sys_skip(a.state, a.mask, b)) return;
  for (int i = tid; i < N; i += NT) { tw[i] = a.twN[i]; th[i] = a.twH[i]; }
  const size_t V = (size_t)N * N * N;
  // Prologue: one loop per mode, so that all loads are in flight before use.
  C<T> orig[EPT];
  auto valid = [&](int s) { return (TOT % NT) == 0 || tid + s * NT < TOT; };
  auto zof = [&](int s) { return (tid + s * NT) / TX; };
  auto xof = [&](int s) { return x0 + (tid + s * NT) - zof(s) * TX; };
  auto nof = [&](int s) { return ((size_t)zof(s) * N + y) * N + xof(s); };
  switch (a.zf_mode) {
    case ZF_XV: {
      T xr[EPT];
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) { orig[s] = a.vin[b * V + nof(s)]; xr[s] = a.xpot[nof(s)]; }
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) orig[s] = orig[s] * xr[s];
    } break;
    case ZF_XUIN: {
      const C<double>* t = a.inc + (size_t)b * 3 * N;
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) {
          const C<double> u = cmul(cmul(t[xof(s)], t[N + y]), t[2 * N + zof(s)]);
          orig[s] = cvt<T>(u) * a.xpot[nof(s)];
        }
    } break;
    case ZF_DETCONJ:
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s))
          orig[s] = (zof(s) == N - 1) ? conj(a.rdet[(size_t)b * N * N + (size_t)y * N + xof(s)]) : C<T>{0, 0};
      break;
    case ZF_V:
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) orig[s] = a.vin[b * V + nof(s)];
      break;
    case ZF_XP_UPD: {
      const SysState& st = a.state[b];
      const bool first = st.first;
      const C<T> beta{(T)st.beta_x, (T)st.beta_y}, omega{(T)st.omega_x, (T)st.omega_y};
      C<T> po[EPT], vo[EPT];
      T xr[EPT];
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) {
          orig[s] = a.rvec[b * V + nof(s)];
          xr[s] = a.xpot[nof(s)];
          if (!first) {
            po[s] = a.pio[b * V + nof(s)];
            vo[s] = a.vvec[b * V + nof(s)];
          }
        }
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) {
          const C<T> pn = first ? orig[s] : orig[s] + cmul(beta, po[s] - cmul(omega, vo[s]));
          a.pio[b * V + nof(s)] = pn;
          orig[s] = pn * xr[s];
        }
    } break;
    default:
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) orig[s] = conj(a.vin[b * V + nof(s)]);
      break;
  }
  for (int pz = 0; pz < 2; ++pz) {
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int z = e / TX, xo = e - z * TX;
        lds[xo * LS + z] = pz ? cmul(orig[s], th[z]) : orig[s];
      }
    }
    __syncthreads();
    lds_fft<T, N, TX, NT, false>(lds, LS, 1, tw);
    C<T>* dst = a.zh + (size_t)(b * 2 + pz) * V + (size_t)y * N + x0;
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int kz = e / TX, xo = e - kz * TX;
        dst[(size_t)kz * N * N + xo] = lds[xo * LS + kz];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Xf: x-direction forward FFTs of rows (pz, kz, y), both x parities.
// grid (2 N^2 / TL, 1, B); writes xh[b][pz][px][kz][y][kx]
// ---------------------------------------------------------------------------
template <typename T, int N, int TL = tile_w<T>(N)>
__global__ void __launch_bounds__(NT) k_xf(PassArgs<T> a) {
  constexpr int LS = N + 1, TOT = TL * N, EPT = (TOT + NT - 1) / NT;
  __shared__ C<T> lds[TL * LS];
  __shared__ C<T> tw[N];
  __shared__ C<T> th[N];
  const int b = blockIdx.z, row0 = blockIdx.x * TL, tid = threadIdx.x;
  if (sys_skip(a.state, a.mask, b)) return;
  for (int i = tid; i < N; i += NT) { tw[i] = a.twN[i]; th[i] = a.twH[i]; }
  const size_t N2 = (size_t)N * N, V = N2 * N;
  const C<T>* src = a.zh + (size_t)b * 2 * V + (size_t)row0 * N;
  C<T> orig[EPT];
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) orig[s] = sld(&src[e]);
  }
  const int pz = row0 / (int)N2;  // TL divides N, so a tile never straddles pz
  const size_t rest0 = (size_t)row0 - (size_t)pz * N2;
  for (int px = 0; px < 2; ++px) {
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int rl = e / N, x = e - rl * N;
        lds[rl * LS + x] = px ? cmul(orig[s], th[x]) : orig[s];
      }
    }
    __syncthreads();
    lds_fft<T, N, TL, NT, false>(lds, LS, 1, tw);
    C<T>* dst = a.xh + ((size_t)b * 4 + pz * 2 + px) * V + rest0 * N;
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int rl = e / N, x = e - rl * N;
        sst(&dst[e], lds[rl * LS + x]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Yc: y columns of class (pz, px): for py in {0,1}: twiddle, FFT, . ghat,
// IFFT, conj twiddle, sum.  In place on xh.  grid (N/TX, N (kz), 4 B)
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(NT) k_yc(PassArgs<T> a) {
  constexpr int TX = tile_w<T>(N), LS = N + 1, TOT = TX * N, EPT = (TOT + NT - 1) / NT;
  __shared__ C<T> lds[TX * LS];
  __shared__ C<T> tw[N];
  __shared__ C<T> th[N];
  const int b = blockIdx.z >> 2, cls = blockIdx.z & 3, pz = cls >> 1, px = cls & 1;
  const int kz = blockIdx.y, x0 = blockIdx.x * TX, tid = threadIdx.x;
  if (sys_skip(a.state, a.mask, b)) return;
  for (int i = tid; i < N; i += NT) { tw[i] = a.twN[i]; th[i] = a.twH[i]; }
  const size_t N2 = (size_t)N * N, V = N2 * N;
  C<T>* plane = a.xh + ((size_t)b * 4 + cls) * V + (size_t)kz * N2 + x0;
  C<T> orig[EPT], acc[EPT];
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) {
      const int y = e / TX, xo = e - y * TX;
      orig[s] = plane[(size_t)y * N + xo];
      acc[s] = C<T>{0, 0};
    }
  }
  for (int py = 0; py < 2; ++py) {
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int y = e / TX, xo = e - y * TX;
        lds[xo * LS + y] = py ? cmul(orig[s], th[y]) : orig[s];
      }
    }
    __syncthreads();
    lds_fft<T, N, TX, NT, false>(lds, LS, 1, tw);
    const C<T>* g = a.ghat + (size_t)((pz * 2 + py) * 2 + px) * V + (size_t)kz * N2 + x0;
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int ky = e / TX, xo = e - ky * TX;
        lds[xo * LS + ky] = cmul(lds[xo * LS + ky], g[(size_t)ky * N + xo]);
      }
    }
    __syncthreads();
    lds_fft<T, N, TX, NT, true>(lds, LS, 1, tw);
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int y = e / TX, xo = e - y * TX;
        C<T> v = lds[xo * LS + y];
        acc[s] = acc[s] + (py ? cmulc(v, th[y]) : v);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) {
      const int y = e / TX, xo = e - y * TX;
      plane[(size_t)y * N + xo] = acc[s];
    }
  }
}

// ---------------------------------------------------------------------------
// Xi: x-direction inverse FFTs, x parities summed; writes back into zh.
// grid (2 N^2 / TL, 1, B)
// ---------------------------------------------------------------------------
template <typename T, int N, int TL = tile_w<T>(N)>
__global__ void __launch_bounds__(NT) k_xi(PassArgs<T> a) {
  constexpr int LS = N + 1, TOT = TL * N, EPT = (TOT + NT - 1) / NT;
  __shared__ C<T> lds[TL * LS];
  __shared__ C<T> tw[N];
  __shared__ C<T> th[N];
  const int b = blockIdx.z, row0 = blockIdx.x * TL, tid = threadIdx.x;
  if (sys_skip(a.state, a.mask, b)) return;
  for (int i = tid; i < N; i += NT) { tw[i] = a.twN[i]; th[i] = a.twH[i]; }
  const size_t N2 = (size_t)N * N, V = N2 * N;
  const int pz = row0 / (int)N2;
  const size_t rest0 = (size_t)row0 - (size_t)pz * N2;
  C<T> acc[EPT];
#pragma unroll
  for (int s = 0; s < EPT; ++s) acc[s] = C<T>{0, 0};
  for (int px = 0; px < 2; ++px) {
    const C<T>* src = a.xh + ((size_t)b * 4 + pz * 2 + px) * V + rest0 * N;
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int rl = e / N, x = e - rl * N;
        lds[rl * LS + x] = sld(&src[e]);
      }
    }
    __syncthreads();
    lds_fft<T, N, TL, NT, true>(lds, LS, 1, tw);
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int rl = e / N, x = e - rl * N;
        C<T> v = lds[rl * LS + x];
        acc[s] = acc[s] + (px ? cmulc(v, th[x]) : v);
      }
    }
    __syncthreads();
  }
  C<T>* dst = a.zh + (size_t)b * 2 * V + (size_t)row0 * N;
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) sst(&dst[e], acc[s]);
  }
}

// ---------------------------------------------------------------------------
// Zi: z-direction inverse FFTs, z parities summed, epilogue.
// grid (N/TX, N, B); partials[(b * NP + wg) * 4 + k]
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(NT) k_zi(PassArgs<T> a) {
  constexpr int TX = tile_w<T>(N), LS = N + 1, TOT = TX * N, EPT = (TOT + NT - 1) / NT;
  __shared__ C<T> lds[TX * LS];
  __shared__ C<T> tw[N];
  __shared__ C<T> th[N];
  __shared__ double red_scratch[(NT / 64) * 3];
  const int b = blockIdx.z, y = blockIdx.y, x0 = blockIdx.x * TX, tid = threadIdx.x;
  if (sys_skip(a.state, a.mask, b)) return;
  for (int i = tid; i < N; i += NT) { tw[i] = a.twN[i]; th[i] = a.twH[i]; }
  const size_t N2 = (size_t)N * N, V = N2 * N;
  C<T> acc[EPT];
#pragma unroll
  for (int s = 0; s < EPT; ++s) acc[s] = C<T>{0, 0};
  for (int pz = 0; pz < 2; ++pz) {
    const C<T>* src = a.zh + (size_t)(b * 2 + pz) * V + (size_t)y * N + x0;
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int kz = e / TX, xo = e - kz * TX;
        lds[xo * LS + kz] = src[(size_t)kz * N2 + xo];
      }
    }
    __syncthreads();
    lds_fft<T, N, TX, NT, true>(lds, LS, 1, tw);
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = tid + s * NT;
      if ((TOT % NT) == 0 || e < TOT) {
        const int z = e / TX, xo = e - z * TX;
        C<T> v = lds[xo * LS + z];
        acc[s] = acc[s] + (pz ? cmulc(v, th[z]) : v);
      }
    }
    __syncthreads();
  }
  // Epilogue: one loop per mode (operand loads first), FP64 products in
  // ascending s.
  double red[3] = {0.0, 0.0, 0.0};
  const int mode = a.zi_mode;
  auto valid = [&](int s) { return (TOT % NT) == 0 || tid + s * NT < TOT; };
  auto nof = [&](int s) {
    const int e = tid + s * NT, z = e / TX, xo = e - z * TX;
    return (size_t)b * V + ((size_t)z * N + y) * N + x0 + xo;
  };
  switch (mode) {
    case ZI_G:
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) a.out[nof(s)] = acc[s];
      break;
    case ZI_GCONJ:
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) a.out[nof(s)] = conj(acc[s]);
      break;
    case ZI_AV_RHAT: {
      C<T> o[EPT], rh[EPT];
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) { o[s] = a.vz[nof(s)]; rh[s] = a.rhat[nof(s)]; }
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) {
          o[s] = o[s] - acc[s];
          a.out[nof(s)] = o[s];
          red[0] += (double)rh[s].x * o[s].x + (double)rh[s].y * o[s].y;
          red[1] += (double)rh[s].x * o[s].y - (double)rh[s].y * o[s].x;
        }
    } break;
    case ZI_AS_TS: {
      C<T> sv[EPT];
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) sv[s] = a.vz[nof(s)];
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) {
          const C<T> o = sv[s] - acc[s];
          a.out[nof(s)] = o;
          red[0] += (double)o.x * sv[s].x + (double)o.y * sv[s].y;
          red[1] += (double)o.x * sv[s].y - (double)o.y * sv[s].x;
          red[2] += (double)o.x * o.x + (double)o.y * o.y;
        }
    } break;
    case ZI_RES_NORM: {  // r0 = b - e0 + G w for a solve started from e0
      C<T> o[EPT];
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) {
          const size_t n = nof(s);
          C<T> bv;
          if (a.bsrc) {
            bv = a.bsrc[n];
          } else {
            const int e = tid + s * NT, z = e / TX, x = x0 + (e - z * TX);
            const C<double>* t = a.inc + (size_t)b * 3 * N;
            bv = cvt<T>(cmul(cmul(t[x], t[N + y]), t[2 * N + z]));
          }
          o[s] = bv - a.vz[n];
        }
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) {
          o[s] = o[s] + acc[s];
          a.out[nof(s)] = o[s];
          a.out2[nof(s)] = o[s];
          red[2] += (double)o[s].x * o[s].x + (double)o[s].y * o[s].y;
        }
    } break;
    default:  // ZI_G_NORM
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) {
          a.out[nof(s)] = acc[s];
          if (a.out2) a.out2[nof(s)] = acc[s];
          red[2] += (double)acc[s].x * acc[s].x + (double)acc[s].y * acc[s].y;
        }
      break;
  }
  if (mode >= ZI_AV_RHAT) {
    block_sum<NT, 3>(red, red_scratch);
    if (tid == 0) {
      const int NP = gridDim.x * gridDim.y;
      const int wg = blockIdx.y * gridDim.x + blockIdx.x;
      double* p = a.partial + ((size_t)b * NP + wg) * 4;
      p[0] = red[0];
      p[1] = red[1];
      p[2] = red[2];
      p[3] = 0.0;
    }
  }
}

template <typename T, int N>
static void launch_split_N(const PassArgs<T>& a, hipStream_t st, PassTimer* tm) {
  constexpr int TX = tile_w<T>(N);
  const dim3 blk(NT);
  if (tm) tm->start(P_ZF, st);
  if (!pad_zf_apply<T>(a, st)) hipLaunchKernelGGL((k_zf<T, N>), dim3(N / TX, N, a.B), blk, 0, st, a);
  if (tm) { tm->stop(st); tm->start(P_XF, st); }
  hipLaunchKernelGGL((k_xf<T, N>), dim3(2 * N * N / TX, 1, a.B), blk, 0, st, a);
  if (tm) { tm->stop(st); tm->start(P_YC, st); }
  if (!pad_y_apply<T>(a, st)) hipLaunchKernelGGL((k_yc<T, N>), dim3(N / TX, N, 4 * a.B), blk, 0, st, a);
  if (tm) { tm->stop(st); tm->start(P_XI, st); }
  hipLaunchKernelGGL((k_xi<T, N>), dim3(2 * N * N / TX, 1, a.B), blk, 0, st, a);
  if (tm) { tm->stop(st); tm->start(P_ZI, st); }
  if (!pad_zi_apply<T>(a, st)) hipLaunchKernelGGL((k_zi<T, N>), dim3(N / TX, N, a.B), blk, 0, st, a);
  if (tm) tm->stop(st);
}

template <typename T>
int green_num_partials(int N) {
  if (reg_supported<T>(N)) return reg_num_partials<T>(N);
  if (pad_num_partials<T>(N) > 0) return pad_num_partials<T>(N);
  switch (N) {
#define BQ_NP(n) case n: return (n / tile_w<T>(n)) * n;
    BQ_NP(8) BQ_NP(12) BQ_NP(16) BQ_NP(24) BQ_NP(32) BQ_NP(48) BQ_NP(64) BQ_NP(96) BQ_NP(128) BQ_NP(256)
#undef BQ_NP
    default: return -1;
  }
}

// Power-of-two grids use the register-resident passes (green_reg.hip); the
// other supported sizes (factors of 3) use the LDS Stockham passes here.
template <typename T>
int green_apply(const PassArgs<T>& a, hipStream_t st, PassTimer* tm) {
  if (reg_supported<T>(a.N)) {
    if (reg_apply<T>(a, st, tm)) return -1;
    return hipGetLastError() == hipSuccess ? 0 : -2;
  }
  switch (a.N) {
#define BQ_CASE(n) case n: launch_split_N<T, n>(a, st, tm); break;
    BQ_CASE(8) BQ_CASE(12) BQ_CASE(16) BQ_CASE(24) BQ_CASE(32) BQ_CASE(48) BQ_CASE(64) BQ_CASE(96)
    BQ_CASE(128) BQ_CASE(256)
#undef BQ_CASE
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Rows per workgroup of the x passes: the default tile, or one the
// autotuner chose among 8, 16 and 32 (a divisor of N within 64 KB of LDS).
// Every tile computes the same values; only the launch shape changes.
template <typename T, int N, int TL>
constexpr bool xtile_ok() { return N % TL == 0 && TL * (N + 1) * (int)sizeof(C<T>) <= 65536; }

template <typename T, int N, bool INV>
static void launch_x_stockham(const PassArgs<T>& a, hipStream_t st) {
  auto go = [&](auto tl) {
    constexpr int TL = decltype(tl)::value;
    if constexpr (INV)
      hipLaunchKernelGGL((k_xi<T, N, TL>), dim3(2 * N * N / TL, 1, a.B), dim3(NT), 0, st, a);
    else
      hipLaunchKernelGGL((k_xf<T, N, TL>), dim3(2 * N * N / TL, 1, a.B), dim3(NT), 0, st, a);
  };
  switch (a.xtile) {
    case 8: if constexpr (xtile_ok<T, N, 8>()) { go(std::integral_constant<int, 8>{}); return; } break;
    case 16: if constexpr (xtile_ok<T, N, 16>()) { go(std::integral_constant<int, 16>{}); return; } break;
    case 32: if constexpr (xtile_ok<T, N, 32>()) { go(std::integral_constant<int, 32>{}); return; } break;
    default: break;
  }
  go(std::integral_constant<int, tile_w<T>(N)>{});
}
template <typename T, int N>
void launch_xf_stockham(const PassArgs<T>& a, hipStream_t st) { launch_x_stockham<T, N, false>(a, st); }
template <typename T, int N>
void launch_xi_stockham(const PassArgs<T>& a, hipStream_t st) { launch_x_stockham<T, N, true>(a, st); }

template <typename T>
bool xtile_valid(int N, int tl) {
  auto ok = [&](auto n) {
    constexpr int NN = decltype(n)::value;
    return (tl == 8 && xtile_ok<T, NN, 8>()) || (tl == 16 && xtile_ok<T, NN, 16>()) ||
           (tl == 32 && xtile_ok<T, NN, 32>());
  };
  switch (N) {
    case 16: return ok(std::integral_constant<int, 16>{});
    case 32: return ok(std::integral_constant<int, 32>{});
    case 64: return ok(std::integral_constant<int, 64>{});
    case 128: return ok(std::integral_constant<int, 128>{});
    case 256: return ok(std::integral_constant<int, 256>{});
    default: return false;
  }
}
template bool xtile_valid<float>(int, int);
template bool xtile_valid<double>(int, int);
#define BQ_XI(T, n) \
  template void launch_xf_stockham<T, n>(const PassArgs<T>&, hipStream_t); \
  template void launch_xi_stockham<T, n>(const PassArgs<T>&, hipStream_t);
BQ_XI(float, 16) BQ_XI(float, 32) BQ_XI(float, 64) BQ_XI(float, 128) BQ_XI(float, 256)
BQ_XI(double, 16) BQ_XI(double, 32) BQ_XI(double, 64) BQ_XI(double, 128) BQ_XI(double, 256)
#undef BQ_XI

// ===========================================================================
// Propagation of B detector planes (N x N, [y][x]) by a transfer function on
// the lateral frequency grid: out = F^-1 diag(t) F in, t in FFT order
// [ky][kx] with the 1/N^2 of the inverse folded in (conj(t) for the
// adjoint).  Rows forward, columns forward-multiply-inverse, rows inverse,
// in place.
// ===========================================================================
template <typename T, int N, bool INV>
__global__ void __launch_bounds__(NT) k_plane_rows(C<T>* planes, const C<T>* twN) {
  constexpr int TL = tile_w<T>(N), LS = N + 1, TOT = TL * N, EPT = (TOT + NT - 1) / NT;
  __shared__ C<T> lds[TL * LS];
  __shared__ C<T> tw[N];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) tw[i] = twN[i];
  C<T>* rows = planes + (size_t)blockIdx.z * N * N + (size_t)blockIdx.x * TL * N;
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) {
      const int rl = e / N, x = e - rl * N;
      lds[rl * LS + x] = rows[e];
    }
  }
  __syncthreads();
  lds_fft<T, N, TL, NT, INV>(lds, LS, 1, tw);
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) {
      const int rl = e / N, x = e - rl * N;
      rows[e] = lds[rl * LS + x];
    }
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(NT) k_plane_cols(C<T>* planes, const C<T>* twN, const C<T>* tf, int conj_tf) {
  constexpr int TX = tile_w<T>(N), LS = N + 1, TOT = TX * N, EPT = (TOT + NT - 1) / NT;
  __shared__ C<T> lds[TX * LS];
  __shared__ C<T> tw[N];
  const int tid = threadIdx.x, x0 = blockIdx.x * TX;
  for (int i = tid; i < N; i += NT) tw[i] = twN[i];
  C<T>* pl = planes + (size_t)blockIdx.z * N * N;
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) {
      const int y = e / TX, xo = e - y * TX;
      lds[xo * LS + y] = pl[(size_t)y * N + x0 + xo];
    }
  }
  __syncthreads();
  lds_fft<T, N, TX, NT, false>(lds, LS, 1, tw);
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) {
      const int ky = e / TX, xo = e - ky * TX;
      const C<T> t = tf[(size_t)ky * N + x0 + xo];
      lds[xo * LS + ky] = conj_tf ? cmulc(lds[xo * LS + ky], t) : cmul(lds[xo * LS + ky], t);
    }
  }
  __syncthreads();
  lds_fft<T, N, TX, NT, true>(lds, LS, 1, tw);
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) {
      const int y = e / TX, xo = e - y * TX;
      pl[(size_t)y * N + x0 + xo] = lds[xo * LS + y];
    }
  }
}

template <typename T, int N>
static void plane_propagate_N(int B, C<T>* planes, const C<T>* twN, const C<T>* tf, int adjoint, hipStream_t st) {
  constexpr int TL = tile_w<T>(N);
  hipLaunchKernelGGL((k_plane_rows<T, N, false>), dim3(N / TL, 1, B), dim3(NT), 0, st, planes, twN);
  hipLaunchKernelGGL((k_plane_cols<T, N>), dim3(N / TL, 1, B), dim3(NT), 0, st, planes, twN, tf, adjoint);
  hipLaunchKernelGGL((k_plane_rows<T, N, true>), dim3(N / TL, 1, B), dim3(NT), 0, st, planes, twN);
}

template <typename T>
int plane_propagate(int B, int N, C<T>* planes, const C<T>* twN, const C<T>* tf, int adjoint, hipStream_t st) {
  switch (N) {
#define BQ_CASE(n) case n: plane_propagate_N<T, n>(B, planes, twN, tf, adjoint, st); break;
    BQ_CASE(8) BQ_CASE(12) BQ_CASE(16) BQ_CASE(24) BQ_CASE(32) BQ_CASE(48) BQ_CASE(64) BQ_CASE(96)
    BQ_CASE(128) BQ_CASE(256)
#undef BQ_CASE
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
template int plane_propagate<float>(int, int, C<float>*, const C<float>*, const C<float>*, int, hipStream_t);
template int plane_propagate<double>(int, int, C<double>*, const C<double>*, const C<double>*, int, hipStream_t);

template int green_apply<float>(const PassArgs<float>&, hipStream_t, PassTimer*);
template int green_apply<double>(const PassArgs<double>&, hipStream_t, PassTimer*);
template int green_num_partials<float>(int);
template int green_num_partials<double>(int);

// ===========================================================================
// Precomputation of the parity classes of ghat_P (FP64).
// ===========================================================================

// Integral of exp(i a t) over [0, R] (FP64).  A power series for |a R| < 0.5
// avoids the cancellation of (e^{i a R} - 1) / (i a).
__device__ inline C<double> e_int(double a, double R) {
  const double z = a * R;
  if (fabs(z) >= 0.5) {
    double sn, cs;
    sincos(z, &sn, &cs);
    // (cs - 1 + i sn) / (i a) = (sn - i (cs - 1)) / a
    return C<double>{sn / a, (1.0 - cs) / a};
  }
  // R * sum_{n>=0} (i z)^n / (n+1)!
  C<double> acc{0.0, 0.0}, term{1.0, 0.0};
  double fact = 1.0;
  for (int n = 0; n < 22; ++n) {
    fact *= (double)(n + 1);
    acc.x += term.x / fact;
    acc.y += term.y / fact;
    term = C<double>{-term.y * z, term.x * z};
  }
  return C<double>{acc.x * R, acc.y * R};
}

// Fourier transform of exp(i kb r) / (4 pi r) truncated at r = R, at |xi| = s:
// (1/s) int_0^R exp(i kb t) sin(s t) dt.
__device__ inline C<double> ghat_trunc(double s, double kb, double R) {
  if (s < 0.5 * kb) {
    double sk, ck, ss, cs;
    sincos(kb * R, &sk, &ck);
    sincos(s * R, &ss, &cs);
    const double sinc = (s > 0.0) ? ss / s : R;
    // 1 + e^{i kb R} (i kb sinc - cos(sR))
    const C<double> m{-cs, kb * sinc};
    const C<double> num = C<double>{1.0, 0.0} + cmul(C<double>{ck, sk}, m);
    const double den = s * s - kb * kb;
    return C<double>{num.x / den, num.y / den};
  }
  const C<double> d = e_int(kb + s, R) - e_int(kb - s, R);
  // d / (2 i s) = (d.y - i d.x) / (2 s)
  return C<double>{d.y / (2.0 * s), -d.x / (2.0 * s)};
}

__global__ void k_ghat_sample(C<double>* out, int Q, double h, double kb, double R) {
  const size_t Q3 = (size_t)Q * Q * Q;
  const double dk = 2.0 * M_PI / ((double)Q * h);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < Q3;
       i += (size_t)gridDim.x * blockDim.x) {
    const int ix = (int)(i % Q), iy = (int)((i / Q) % Q), iz = (int)(i / ((size_t)Q * Q));
    const double fx = (ix < Q / 2 ? ix : ix - Q) * dk;
    const double fy = (iy < Q / 2 ? iy : iy - Q) * dk;
    const double fz = (iz < Q / 2 ? iz : iz - Q) * dk;
    out[i] = ghat_trunc(sqrt(fz * fz + fy * fy + fx * fx), kb, R);
  }
}

// FFT of lines along one axis of a contiguous 3D array (n x n x n), in place.
// Lines of axis 2 are contiguous rows; for axes 0/1 a tile of TX lines that
// are adjacent along axis 2 is processed together for coalescing.
template <int LEN, bool INV>
__global__ void __launch_bounds__(NT) k_fft_axis(C<double>* data, int axis, const C<double>* twg) {
  constexpr int TX = tile_w<double>(LEN), LS = LEN + 1, TOT = TX * LEN, EPT = (TOT + NT - 1) / NT;
  __shared__ C<double> lds[TX * LS];
  __shared__ C<double> tw[LEN];
  const int tid = threadIdx.x;
  for (int i = tid; i < LEN; i += NT) tw[i] = twg[i];
  const size_t n = LEN, n2 = n * n;
  size_t base, lstep, estep;
  if (axis == 2) {  // rows: blockIdx.x enumerates tiles of TX rows
    base = (size_t)blockIdx.x * TX * n;
    lstep = n;
    estep = 1;
  } else {
    const size_t outer = blockIdx.y;  // the remaining axis
    const size_t x0 = (size_t)blockIdx.x * TX;
    base = (axis == 1 ? outer * n2 : outer * n) + x0;
    lstep = 1;
    estep = (axis == 1 ? n : n2);
  }
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) {
      int l, k;
      if (axis == 2) { l = e / LEN; k = e - l * LEN; } else { k = e / TX; l = e - k * TX; }
      lds[l * LS + k] = data[base + l * lstep + k * estep];
    }
  }
  __syncthreads();
  lds_fft<double, LEN, TX, NT, INV>(lds, LS, 1, tw);
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = tid + s * NT;
    if ((TOT % NT) == 0 || e < TOT) {
      int l, k;
      if (axis == 2) { l = e / LEN; k = e - l * LEN; } else { k = e / TX; l = e - k * TX; }
      data[base + l * lstep + k * estep] = lds[l * LS + k];
    }
  }
}

template <int LEN, bool INV>
static void fft3d_axis_all(C<double>* d, const C<double>* tw, hipStream_t st) {
  constexpr int TX = tile_w<double>(LEN);
  hipLaunchKernelGGL((k_fft_axis<LEN, INV>), dim3((LEN * LEN) / TX), dim3(NT), 0, st, d, 2, tw);
  hipLaunchKernelGGL((k_fft_axis<LEN, INV>), dim3(LEN / TX, LEN), dim3(NT), 0, st, d, 1, tw);
  hipLaunchKernelGGL((k_fft_axis<LEN, INV>), dim3(LEN / TX, LEN), dim3(NT), 0, st, d, 0, tw);
}

static int fft3d(int len, bool inv, C<double>* d, const C<double>* tw, hipStream_t st) {
  switch (len) {
#define BQ_F(L) case L: if (inv) fft3d_axis_all<L, true>(d, tw, st); else fft3d_axis_all<L, false>(d, tw, st); break;
    BQ_F(8) BQ_F(12) BQ_F(16) BQ_F(24) BQ_F(32) BQ_F(48) BQ_F(64) BQ_F(96) BQ_F(128) BQ_F(192)
    BQ_F(256) BQ_F(384) BQ_F(512) BQ_F(768)
#undef BQ_F
    default: return -1;
  }
  return 0;
}

// Lag-cropped kernel folded into the 8 parity classes (with the 1/Q^3 of the
// inverse DFT):  cls[p][m] = exp(-i pi p.m / N) sum_{w in {0,1}^3}
// (-1)^{p.w} K_P[m + N w],  K_P[j] = Kq[lag(j) mod Q] / Q^3 with lag(j) = j
// for j < N and j - 2N otherwise.
__global__ void k_ghat_fold(const C<double>* Kq, C<double>* cls, int N, int Q) {
  const size_t N3 = (size_t)N * N * N;
  const double invQ3 = 1.0 / ((double)Q * Q * Q);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < 8 * N3;
       i += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(i / N3);
    const size_t m = i - (size_t)p * N3;
    const int mx = (int)(m % N), my = (int)((m / N) % N), mz = (int)(m / ((size_t)N * N));
    const int pz = (p >> 2) & 1, py = (p >> 1) & 1, px = p & 1;
    C<double> acc{0.0, 0.0};
    for (int w = 0; w < 8; ++w) {
      const int wz = (w >> 2) & 1, wy = (w >> 1) & 1, wx = w & 1;
      const int jz = mz + N * wz, jy = my + N * wy, jx = mx + N * wx;
      const int qz = (jz < N ? jz : jz - 2 * N + Q);
      const int qy = (jy < N ? jy : jy - 2 * N + Q);
      const int qx = (jx < N ? jx : jx - 2 * N + Q);
      C<double> k = Kq[((size_t)qz * Q + qy) * Q + qx];
      const int sgn = (pz & wz) ^ (py & wy) ^ (px & wx);
      acc = sgn ? acc - k : acc + k;
    }
    double sn, cs;
    sincospi(-(double)(pz * mz + py * my + px * mx) / (double)N, &sn, &cs);
    cls[i] = cmul(acc, C<double>{cs, sn}) * invQ3;
  }
}

template <typename T>
__global__ void k_ghat_final(const C<double>* cls, C<T>* out, size_t n, double scale) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = C<T>{(T)(cls[i].x * scale), (T)(cls[i].y * scale)};
}

static void twiddles(int len, std::vector<C<double>>& w) {
  w.resize(len);
  for (int k = 0; k < len; ++k) {
    // exp(-2 pi i k / len) with the angle reduced exactly via sincospi
    const double a = -2.0 * (double)k / (double)len;
    w[k] = C<double>{cospi_host(a), sinpi_host(a)};
  }
}

int ghat_oversampling(int N) { return N <= 128 ? 4 * N : 3 * N; }

template <typename T>
int ghat_precompute(int N, double h, double kb, C<T>* out, hipStream_t st) {
  const int Q = ghat_oversampling(N);
  const size_t Q3 = (size_t)Q * Q * Q, N3 = (size_t)N * N * N;
  C<double>* dq = nullptr;
  C<double>* dcls = nullptr;
  C<double>* twq = nullptr;
  C<double>* twn = nullptr;
  std::vector<C<double>> hq, hn;
  twiddles(Q, hq);
  twiddles(N, hn);
  int rc = 0;
  if (hipMalloc(&dq, Q3 * sizeof(C<double>)) != hipSuccess) return -3;
  if (hipMalloc(&dcls, 8 * N3 * sizeof(C<double>)) != hipSuccess) { (void)hipFree(dq); return -3; }
  if (hipMalloc(&twq, Q * sizeof(C<double>)) != hipSuccess ||
      hipMalloc(&twn, N * sizeof(C<double>)) != hipSuccess) { rc = -3; goto done; }
  if (hipMemcpyAsync(twq, hq.data(), Q * sizeof(C<double>), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(twn, hn.data(), N * sizeof(C<double>), hipMemcpyHostToDevice, st) != hipSuccess) {
    rc = -2; goto done;
  }
  {
    const double R = sqrt(3.0) * N * h;
    hipLaunchKernelGGL(k_ghat_sample, dim3(4096), dim3(256), 0, st, dq, Q, h, kb, R);
    if (fft3d(Q, true, dq, twq, st)) { rc = -1; goto done; }
    hipLaunchKernelGGL(k_ghat_fold, dim3(4096), dim3(256), 0, st, dq, dcls, N, Q);
    for (int p = 0; p < 8; ++p)
      if (fft3d(N, false, dcls + p * N3, twn, st)) { rc = -1; goto done; }
    // 1/(2N)^3 of the padded inverse transform is folded into the table
    const double scale = 1.0 / (8.0 * (double)N * N * N);
    hipLaunchKernelGGL((k_ghat_final<T>), dim3(4096), dim3(256), 0, st, dcls, out, 8 * N3, scale);
    if (hipGetLastError() != hipSuccess) rc = -2;
    if (hipStreamSynchronize(st) != hipSuccess) rc = -2;
  }
done:
  (void)hipStreamSynchronize(st);
  if (twq) (void)hipFree(twq);
  if (twn) (void)hipFree(twn);
  (void)hipFree(dcls);
  (void)hipFree(dq);
  return rc;
}

template int ghat_precompute<float>(int, double, double, C<float>*, hipStream_t);
template int ghat_precompute<double>(int, double, double, C<double>*, hipStream_t);

}  // namespace bq
