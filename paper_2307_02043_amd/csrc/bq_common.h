// Shared device-side building blocks of the bq library (gfx950 / CDNA4).
//
// * complex arithmetic on interleaved (re, im) pairs in float or double;
// * radix-2/3/4/8 DFT butterflies;
// * an LDS-resident Stockham (self-sorting) mixed-radix FFT over a set of
//   lines held by one workgroup, used by every FFT pass of the Green's
//   operator and of the kernel precomputation;
// * wavefront / workgroup FP64 reductions (DPP shuffles + LDS), with a fixed
//   order so that results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bq {

template <typename T>
struct C {
  T x, y;
};

template <typename T>
__host__ __device__ inline C<T> mk(T a, T b) { return C<T>{a, b}; }
template <typename T>
__host__ __device__ inline C<T> operator+(C<T> a, C<T> b) { return C<T>{a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ inline C<T> operator-(C<T> a, C<T> b) { return C<T>{a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ inline C<T> operator*(C<T> a, T s) { return C<T>{a.x * s, a.y * s}; }
template <typename T>
__host__ __device__ inline C<T> cmul(C<T> a, C<T> b) {
  return C<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__host__ __device__ inline C<T> cmulc(C<T> a, C<T> b) {
  return C<T>{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__host__ __device__ inline C<T> conj(C<T> a) { return C<T>{a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__host__ __device__ inline C<T> rot90(C<T> a) {
  return INV ? C<T>{-a.y, a.x} : C<T>{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Small DFTs, forward: X[k] = sum_n x[n] exp(-2 pi i n k / R); INV flips the
// sign of the exponent (no scaling).
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__device__ inline void dft2(C<T>* v) {
  C<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T, bool INV>
__device__ inline void dft3(C<T>* v) {
  const T h = T(0.86602540378443864676372317075294);  // sin(2 pi / 3)
  C<T> t1 = v[1] + v[2];
  C<T> t2 = v[1] - v[2];
  C<T> m = v[0] - t1 * T(0.5);
  C<T> r = rot90<T, INV>(t2) * h;  // -i h t2 (forward)
  v[0] = v[0] + t1;
  v[1] = m + r;
  v[2] = m - r;
}

template <typename T, bool INV>
__device__ inline void dft4(C<T>* v) {
  C<T> a0 = v[0] + v[2], a1 = v[0] - v[2];
  C<T> a2 = v[1] + v[3], a3 = rot90<T, INV>(v[1] - v[3]);
  v[0] = a0 + a2;
  v[2] = a0 - a2;
  v[1] = a1 + a3;
  v[3] = a1 - a3;
}

template <typename T, bool INV>
__device__ inline void dft8(C<T>* v) {
  const T r = T(0.70710678118654752440084436210485);
  C<T> a[4], b[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    a[n] = v[n] + v[n + 4];
    b[n] = v[n] - v[n + 4];
  }
  // b[n] *= W8^n (forward) or its conjugate (inverse)
  b[1] = C<T>{(b[1].x + (INV ? -b[1].y : b[1].y)) * r, (b[1].y + (INV ? b[1].x : -b[1].x)) * r};
  b[2] = rot90<T, INV>(b[2]);
  b[3] = C<T>{(-b[3].x + (INV ? -b[3].y : b[3].y)) * r, (-b[3].y + (INV ? b[3].x : -b[3].x)) * r};
  dft4<T, INV>(a);
  dft4<T, INV>(b);
  v[0] = a[0]; v[2] = a[1]; v[4] = a[2]; v[6] = a[3];
  v[1] = b[0]; v[3] = b[1]; v[5] = b[2]; v[7] = b[3];
}

template <typename T, bool INV, int R>
__device__ inline void dftR(C<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// Radix plans: product of radices == LEN.
// ---------------------------------------------------------------------------
template <int LEN> struct Plan;
#define BQ_PLAN(L, NS, A, B, C_, D) \
  template <> struct Plan<L> { static constexpr int n = NS; static constexpr int r[4] = {A, B, C_, D}; };
BQ_PLAN(8, 1, 8, 1, 1, 1)
BQ_PLAN(12, 2, 4, 3, 1, 1)
BQ_PLAN(16, 2, 4, 4, 1, 1)
BQ_PLAN(24, 2, 8, 3, 1, 1)
BQ_PLAN(32, 2, 8, 4, 1, 1)
BQ_PLAN(48, 3, 4, 4, 3, 1)
BQ_PLAN(64, 2, 8, 8, 1, 1)
BQ_PLAN(96, 3, 8, 4, 3, 1)
BQ_PLAN(128, 3, 8, 4, 4, 1)
BQ_PLAN(192, 3, 8, 8, 3, 1)
BQ_PLAN(256, 3, 8, 8, 4, 1)
BQ_PLAN(384, 4, 8, 4, 4, 3)
BQ_PLAN(512, 3, 8, 8, 8, 1)
BQ_PLAN(768, 4, 8, 8, 4, 3)
BQ_PLAN(1024, 4, 8, 8, 4, 4)
#undef BQ_PLAN

// One Stockham stage over NL lines of length LEN stored in LDS at
// buf[line * ls + elem * es].  Butterfly j of a line reads elements
// j + r LEN/R, applies twiddles W_{NS R}^{(j mod NS) r}, runs the radix-R DFT
// and writes to (j / NS) NS R + (j mod NS) + r NS.  tw holds W_LEN^k.
template <typename T, int LEN, int NL, int NTHR, bool INV, int R, int NS>
__device__ inline void stockham_stage(C<T>* buf, int ls, int es, const C<T>* tw) {
  constexpr int M = LEN / R;
  constexpr int NB = NL * M;
  constexpr int BPT = (NB + NTHR - 1) / NTHR;
  constexpr int STEP = LEN / (NS * R);
  C<T> v[BPT][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < BPT; ++s) {
    const int j = tid + s * NTHR;
    if ((NB % NTHR) == 0 || j < NB) {
      const int line = j / M, jj = j - line * M;
      const C<T>* base = buf + line * ls;
      const int k = jj % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C<T> a = base[(jj + r * M) * es];
        if (NS > 1 && r > 0) {
          C<T> w = tw[k * r * STEP];
          a = INV ? cmulc(a, w) : cmul(a, w);
        }
        v[s][r] = a;
      }
      dftR<T, INV, R>(v[s]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < BPT; ++s) {
    const int j = tid + s * NTHR;
    if ((NB % NTHR) == 0 || j < NB) {
      const int line = j / M, jj = j - line * M;
      C<T>* base = buf + line * ls;
      const int k = jj % NS;
      const int d = (jj / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) base[(d + r * NS) * es] = v[s][r];
    }
  }
  __syncthreads();
}

template <typename T, int LEN, int NL, int NTHR, bool INV, int S, int NS>
struct StockhamRun {
  static __device__ inline void run(C<T>* buf, int ls, int es, const C<T>* tw) {
    if constexpr (S < Plan<LEN>::n) {
      constexpr int R = Plan<LEN>::r[S];
      stockham_stage<T, LEN, NL, NTHR, INV, R, NS>(buf, ls, es, tw);
      StockhamRun<T, LEN, NL, NTHR, INV, S + 1, NS * R>::run(buf, ls, es, tw);
    }
  }
};

// In-place unnormalised FFT of NL lines held in LDS.  Caller must
// __syncthreads() before (data written) -- the routine ends synchronised.
template <typename T, int LEN, int NL, int NTHR, bool INV>
__device__ inline void lds_fft(C<T>* buf, int ls, int es, const C<T>* tw) {
  StockhamRun<T, LEN, NL, NTHR, INV, 0, 1>::run(buf, ls, es, tw);
}

// ---------------------------------------------------------------------------
// Reductions (FP64, deterministic order).
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum K values over the workgroup; result valid in thread 0.  scratch must
// hold (NTHR / 64) * K doubles.
template <int NTHR, int K>
__device__ inline void block_sum(double* vals, double* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) vals[k] = wave_sum(vals[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) scratch[wave * K + k] = vals[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < NTHR / 64; ++w) s += scratch[w * K + k];
      vals[k] = s;
    }
  }
  __syncthreads();
}

}  // namespace bq
