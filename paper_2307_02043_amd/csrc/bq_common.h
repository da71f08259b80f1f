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

// cos(m pi / 8), m mod 16 (exact decimal expansions of the four distinct values)
__host__ __device__ constexpr double cos16(int m) {
  constexpr double c[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                            0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                            -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                            0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
  return c[m & 15];
}
__host__ __device__ constexpr double sin16(int m) { return cos16(m + 12); }  // sin x = cos(x - pi/2)
constexpr double cabs_(double x) { return x < 0 ? -x : x; }

// Twiddled radix-2 butterfly (a, b) -> (a + W b, a - W b), W = W16^M (its
// conjugate for the inverse), with W written as cos(1 + i tan) or, when
// |tan| > 1, as sin(cot + i): 6 FMA-able operations instead of a complex
// product and two complex sums (8); multiples of a quarter turn are adds.
template <typename T, bool INV, int M>
__device__ inline void tbfly(C<T>& a, C<T>& b) {
  constexpr int m = M & 15;
  constexpr double wr = cos16(m), wi = INV ? sin16(m) : -sin16(m);
  C<T> wb;
  if constexpr (m == 0) {
    wb = b;
  } else if constexpr (m == 8) {
    wb = C<T>{-b.x, -b.y};
  } else if constexpr (m == 4 || m == 12) {  // W = i wi
    wb = wi > 0 ? C<T>{-b.y, b.x} : C<T>{b.y, -b.x};
  } else if constexpr (cabs_(wr) >= cabs_(wi)) {
    constexpr T t = T(wi / wr), c = T(wr);
    const C<T> mm{b.x - t * b.y, b.y + t * b.x};
    const C<T> y0{a.x + c * mm.x, a.y + c * mm.y}, y1{a.x - c * mm.x, a.y - c * mm.y};
    a = y0;
    b = y1;
    return;
  } else {
    constexpr T t = T(wr / wi), c = T(wi);
    const C<T> mm{t * b.x - b.y, t * b.y + b.x};
    const C<T> y0{a.x + c * mm.x, a.y + c * mm.y}, y1{a.x - c * mm.x, a.y - c * mm.y};
    a = y0;
    b = y1;
    return;
  }
  const C<T> y0 = a + wb, y1 = a - wb;
  a = y0;
  b = y1;
}

// 16-point DFT as 4 x 4: n = n1 + 4 n2, k = k2 + 4 k1; inner DFT-4 over n2,
// then for each k2 the DFT-4 over n1 of a[n1][k2] W16^{n1 k2}, taken as two
// radix-2 layers of twiddled butterflies:
//   e+- = a0 +- W^{2k2} a2,  f+- = a1 +- W^{2k2} a3,
//   X[k2] , X[k2+8]  = e+ +- W^{k2} f+,  X[k2+4], X[k2+12] = e- +- W^{k2+4} f-
// (W^{k2+4} = -i W^{k2}); natural-order output.
template <typename T, bool INV, int K2>
__device__ inline void dft16_col(C<T> (&a)[4][4], C<T>* v) {
  C<T> e0 = a[0][K2], e1 = a[2][K2], f0 = a[1][K2], f1 = a[3][K2];
  tbfly<T, INV, 2 * K2>(e0, e1);
  tbfly<T, INV, 2 * K2>(f0, f1);
  tbfly<T, INV, K2>(e0, f0);
  tbfly<T, INV, K2 + 4>(e1, f1);
  v[K2] = e0;
  v[K2 + 8] = f0;
  v[K2 + 4] = e1;
  v[K2 + 12] = f1;
}

template <typename T, bool INV>
__device__ inline void dft16(C<T>* v) {
  C<T> a[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) a[n1][n2] = v[n1 + 4 * n2];
    dft4<T, INV>(a[n1]);  // a[n1][k2]
  }
  dft16_col<T, INV, 0>(a, v);
  dft16_col<T, INV, 1>(a, v);
  dft16_col<T, INV, 2>(a, v);
  dft16_col<T, INV, 3>(a, v);
}

// cos(m pi / 16), m mod 32
__host__ __device__ constexpr double cos32(int m) {
  constexpr double c[9] = {1.0,
                           0.98078528040323044913,
                           0.92387953251128675613,
                           0.83146961230254523708,
                           0.70710678118654752440,
                           0.55557023301960222474,
                           0.38268343236508977173,
                           0.19509032201612826785,
                           0.0};
  const int r = m & 31;                     // angle r pi / 16 in [0, 2 pi)
  const int q = r <= 16 ? r : 32 - r;       // cos is even about pi
  return q <= 8 ? c[q] : -c[16 - q];        // cos(pi - t) = -cos t
}
__host__ __device__ constexpr double sin32(int m) { return cos32(m + 24); }  // sin x = cos(x - pi/2)

// (a, b) -> (a + W b, a - W b), W = W32^M (conjugate for the inverse); same
// tangent / cotangent forms as tbfly.
template <typename T, bool INV, int M>
__device__ inline void tbfly32(C<T>& a, C<T>& b) {
  constexpr int m = M & 31;
  if constexpr ((m & 1) == 0) {
    tbfly<T, INV, m / 2>(a, b);  // W32^{2k} = W16^k
  } else {
    constexpr double wr = cos32(m), wi = INV ? sin32(m) : -sin32(m);
    C<T> mm;
    T c;
    if constexpr (cabs_(wr) >= cabs_(wi)) {
      constexpr T t = T(wi / wr);
      c = T(wr);
      mm = C<T>{b.x - t * b.y, b.y + t * b.x};
    } else {
      constexpr T t = T(wr / wi);
      c = T(wi);
      mm = C<T>{t * b.x - b.y, t * b.y + b.x};
    }
    const C<T> y0{a.x + c * mm.x, a.y + c * mm.y}, y1{a.x - c * mm.x, a.y - c * mm.y};
    a = y0;
    b = y1;
  }
}

template <typename T, bool INV, int K>
__device__ inline void dft32_join(C<T>* e, C<T>* o, C<T>* v) {
  if constexpr (K < 16) {
    C<T> x0 = e[K], x1 = o[K];
    tbfly32<T, INV, K>(x0, x1);
    v[K] = x0;
    v[K + 16] = x1;
    dft32_join<T, INV, K + 1>(e, o, v);
  }
}

// 32-point DFT: radix-2 split into the even and odd samples (two DFT-16s),
// joined by the twiddled butterflies X[k], X[k+16] = E[k] +- W32^k O[k].
template <typename T, bool INV>
__device__ inline void dft32(C<T>* v) {
  C<T> e[16], o[16];
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    e[n] = v[2 * n];
    o[n] = v[2 * n + 1];
  }
  dft16<T, INV>(e);
  dft16<T, INV>(o);
  dft32_join<T, INV, 0>(e, o, v);
}

// cos(m pi / 12), m mod 24 (exact decimal expansions: cos 15 = (sqrt 6 +
// sqrt 2) / 4, cos 75 = (sqrt 6 - sqrt 2) / 4)
__host__ __device__ constexpr double cos24(int m) {
  constexpr double c[7] = {1.0,
                           0.96592582628906828674974319972890,
                           0.86602540378443864676372317075294,
                           0.70710678118654752440084436210485,
                           0.5,
                           0.25881904510252076234889883762405,
                           0.0};
  const int r = ((m % 24) + 24) % 24;  // angle r pi / 12 in [0, 2 pi)
  const int q = r <= 12 ? r : 24 - r;  // cos is even about pi
  return q <= 6 ? c[q] : -c[12 - q];   // cos(pi - t) = -cos t
}
__host__ __device__ constexpr double sin24(int m) { return cos24(m + 18); }  // sin x = cos(x - pi/2)

// a W24^M (its conjugate for the inverse); quarter turns are swaps
template <typename T, bool INV, int M>
__device__ inline C<T> tw24(C<T> a) {
  constexpr int m = M % 24;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 12) {
    return C<T>{-a.x, -a.y};
  } else if constexpr (m == 6) {
    return rot90<T, INV>(a);  // W24^6 = -i
  } else if constexpr (m == 18) {
    return rot90<T, !INV>(a);
  } else {
    constexpr T wr = T(cos24(m)), wi = T(INV ? sin24(m) : -sin24(m));
    return C<T>{a.x * wr - a.y * wi, a.x * wi + a.y * wr};
  }
}

// 24-point DFT as 3 x 8: n = 8 n1 + n2, k = k1 + 3 k2.  DFT-3 over n1 for
// each n2, twiddles W24^{n2 k1}, DFT-8 over n2 for each k1.
template <typename T, bool INV, int N2>
__device__ inline void dft24_col(const C<T>* v, C<T> (&a)[3][8]) {
  if constexpr (N2 < 8) {
    C<T> t[3] = {v[N2], v[8 + N2], v[16 + N2]};
    dft3<T, INV>(t);
    a[0][N2] = t[0];
    a[1][N2] = tw24<T, INV, N2>(t[1]);
    a[2][N2] = tw24<T, INV, 2 * N2>(t[2]);
    dft24_col<T, INV, N2 + 1>(v, a);
  }
}

template <typename T, bool INV>
__device__ inline void dft24(C<T>* v) {
  C<T> a[3][8];
  dft24_col<T, INV, 0>(v, a);
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    dft8<T, INV>(a[k1]);
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) v[k1 + 3 * k2] = a[k1][k2];
  }
}

template <typename T, bool INV, int R>
__device__ inline void dftR(C<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else if constexpr (R == 16) dft16<T, INV>(v);
  else if constexpr (R == 24) dft24<T, INV>(v);
  else if constexpr (R == 32) dft32<T, INV>(v);
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
      // lines vary fastest across lanes: lane-adjacent accesses are a line
      // stride apart, which the padded stride spreads over the LDS banks
      const int line = j % NL, jj = j / NL;
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
      const int line = j % NL, jj = j / NL;
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
// Register-resident line FFT: a line of N = R1 R2 points is held by R2
// threads with R1 points each (thread j holds x[j + R2 m]).  A radix-R1 DFT
// in registers, twiddles W_N^{j k1}, one exchange through LDS and radix-R2
// DFTs give X[k1 + R1 k2] with k1 = j + R2 i held by thread j at
// d[i R2 + k2].  One LDS write and one read per transform (against two per
// radix stage for the LDS Stockham routine).  All threads of the workgroup
// must call it together (it synchronises the workgroup).
// ---------------------------------------------------------------------------
// Exchange slot of value (k1, jj): the jj index is XOR-swizzled by k1 so that
// the R2 lanes of a line never hit the same LDS bank group.
template <int R2>
__device__ inline int xslot(int k1, int jj) { return k1 * R2 + (jj ^ (k1 & (R2 - 1))); }

// Forward (or inverse-signed) FFT of one line distributed over R2 threads.
// In: d[m] = x[j + R2 m].  Out: d[i R2 + k2] = X[k1 + R1 k2], k1 = j + R2 i.
template <typename T, int N, int R1, int R2, bool INV>
__device__ inline void line_fft(C<T>* d, C<T>* line, int es, int j, const C<T>* tw) {
  constexpr int NI = R1 / R2;
  dftR<T, INV, R1>(d);
#pragma unroll
  for (int k1 = 1; k1 < R1; ++k1) {
    const C<T> w = tw[j * k1];
    d[k1] = INV ? cmulc(d[k1], w) : cmul(d[k1], w);
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) line[xslot<R2>(k1, j) * es] = d[k1];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int k1 = j + R2 * i;
#pragma unroll
    for (int jj = 0; jj < R2; ++jj) d[i * R2 + jj] = line[xslot<R2>(k1, jj) * es];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NI; ++i) dftR<T, INV, R2>(&d[i * R2]);
}

// Inverse of line_fft (unnormalised): from the distributed spectrum back to
// d[m] = N x[j + R2 m].
template <typename T, int N, int R1, int R2>
__device__ inline void line_ifft(C<T>* d, C<T>* line, int es, int j, const C<T>* tw) {
  constexpr int NI = R1 / R2;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int k1 = j + R2 * i;
    dftR<T, true, R2>(&d[i * R2]);
#pragma unroll
    for (int jj = 0; jj < R2; ++jj) {
      C<T> v = d[i * R2 + jj];
      if (jj * k1) v = cmulc(v, tw[jj * k1]);
      line[xslot<R2>(k1, jj) * es] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) d[k1] = line[xslot<R2>(k1, j) * es];
  __syncthreads();
  dftR<T, true, R1>(d);
}

// ---------------------------------------------------------------------------
// Table-driven variant of the register line FFT for the strided-line passes.
// The exchange slot of value (k1, jj) is k1 P + jj with P = R2 + 1: each
// thread's writes and reads through LDS are then one base address plus
// compile-time offsets (no per-element address arithmetic), and the odd line
// stride LS spreads lanes of neighbouring lines over the banks.  Twiddles
// come from per-thread rows of a table:
//   tf[a R1 + b] = W^{a b} (a < R2, b < R1)   (forward, row of thread j)
//   ti[b R2 + a] = W^{a b}                    (inverse, row of k1 = b)
// which are the same table when R1 == R2.
// ---------------------------------------------------------------------------
template <int R1, int R2>
struct LineX {
  static constexpr int P = R2 + 1;
  static constexpr int SPAN = (R1 - 1) * P + R2;
  static constexpr int LS = SPAN | 1;
  static constexpr int TW = R1 == R2 ? R1 * R2 : 2 * R1 * R2;  // table entries
};

// In: d[m] = x[j + R2 m].  Out: d[i R2 + k2] = X[k1 + R1 k2], k1 = j + R2 i.
// tail = false drops the barrier after the exchange's reads, for a caller
// that touches this LDS line no more (the kernel's last exchange); it must
// be uniform over the workgroup.
template <typename T, int R1, int R2, bool INV>
__device__ inline void line_fft_t(C<T>* d, C<T>* line, int j, const C<T>* tf, bool tail = true) {
  constexpr int NI = R1 / R2, P = LineX<R1, R2>::P;
  dftR<T, INV, R1>(d);
  const C<T>* w = tf + j * R1;
#pragma unroll
  for (int k1 = 1; k1 < R1; ++k1) d[k1] = INV ? cmulc(d[k1], w[k1]) : cmul(d[k1], w[k1]);
  C<T>* wp = line + j;
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) wp[k1 * P] = d[k1];
  __syncthreads();
  const C<T>* rp = line + j * P;
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int jj = 0; jj < R2; ++jj) d[i * R2 + jj] = rp[i * R2 * P + jj];
  if (tail) __syncthreads();
#pragma unroll
  for (int i = 0; i < NI; ++i) dftR<T, INV, R2>(&d[i * R2]);
}

// Inverse of line_fft_t (unnormalised): back to d[m] = len x[j + R2 m].
template <typename T, int R1, int R2>
__device__ inline void line_ifft_t(C<T>* d, C<T>* line, int j, const C<T>* ti, bool tail = true) {
  constexpr int NI = R1 / R2, P = LineX<R1, R2>::P;
  C<T>* wp = line + j * P;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    dftR<T, true, R2>(&d[i * R2]);
    const C<T>* w = ti + (j + R2 * i) * R2;
#pragma unroll
    for (int jj = 0; jj < R2; ++jj) {
      C<T> v = d[i * R2 + jj];
      if (jj) v = cmulc(v, w[jj]);
      wp[i * R2 * P + jj] = v;
    }
  }
  __syncthreads();
  const C<T>* rp = line + j;
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) d[k1] = rp[k1 * P];
  if (tail) __syncthreads();
  dftR<T, true, R1>(d);
}

// Variants of line_fft_t / line_ifft_t for R1 = NI R2 > R2 whose exchange
// passes through LDS in NI rounds, one per group i of NI: the line then
// needs R2 rows of P slots instead of R1 (LineXS::LS), at one more barrier
// pair per round.  Both directions read their twiddles from the forward
// table alone (W^{(j + R2 i) jj} = tf[jj R1 + j + R2 i]), TW = R1 R2.
// The line stride is the odd one of the full exchange (the R1 = R2 layout
// of 16 x 16 lines at N = 128, whose exchanges the counters show free of
// bank conflicts); a stride of an odd multiple of 8 banks measured 13 times
// the conflict cycles and a slower pass.
template <int R1, int R2>
struct LineXS {
  static constexpr int P = R2 + 1;
  static constexpr int LS = ((R2 - 1) * P + R2) | 1;
  static constexpr int TW = R1 * R2;
};

template <typename T, int R1, int R2, bool INV>
__device__ inline void line_fft_ts(C<T>* d, C<T>* line, int j, const C<T>* tf, bool tail = true) {
  constexpr int NI = R1 / R2, P = LineXS<R1, R2>::P;
  dftR<T, INV, R1>(d);
  const C<T>* w = tf + j * R1;
#pragma unroll
  for (int k1 = 1; k1 < R1; ++k1) d[k1] = INV ? cmulc(d[k1], w[k1]) : cmul(d[k1], w[k1]);
  C<T>* wp = line + j;
  const C<T>* rp = line + j * P;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    // values k1 = R2 i + kk of every thread to slot (kk, thread); thread j
    // then reads its column k1 = j + R2 i over all threads into the same
    // registers (their values are in LDS by then)
#pragma unroll
    for (int kk = 0; kk < R2; ++kk) wp[kk * P] = d[i * R2 + kk];
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < R2; ++jj) d[i * R2 + jj] = rp[jj];
    if (tail || i + 1 < NI) __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NI; ++i) dftR<T, INV, R2>(&d[i * R2]);
}

template <typename T, int R1, int R2>
__device__ inline void line_ifft_ts(C<T>* d, C<T>* line, int j, const C<T>* tf, bool tail = true) {
  constexpr int NI = R1 / R2, P = LineXS<R1, R2>::P;
  C<T>* wp = line + j * P;
  const C<T>* rp = line + j;
  const C<T>* w = tf + j;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    dftR<T, true, R2>(&d[i * R2]);
#pragma unroll
    for (int jj = 0; jj < R2; ++jj) {
      C<T> v = d[i * R2 + jj];
      if (jj) v = cmulc(v, w[jj * R1 + R2 * i]);
      wp[jj] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < R2; ++kk) d[i * R2 + kk] = rp[kk * P];
    if (tail || i + 1 < NI) __syncthreads();
  }
  dftR<T, true, R1>(d);
}

// ---------------------------------------------------------------------------
// Row-wise traversal of an image with nrows rows (z, y) of nx points: rows
// over workgroups, x over threads.  When a row is shorter than the
// workgroup, one step covers rps = WG / nx rows (thread t takes row t / nx of
// the step at x = t mod nx; threads beyond rps rows idle).  Long rows keep
// the row index workgroup-uniform (scalar index arithmetic and branches).
// f(row0, row1, two, x) gets a pair of rows, row1 = row0 + the stride of
// the traversal, two = row1 exists; for_rows hands single rows to f(row, x).
//
// Workgroup h runs on XCD h mod 8, and each XCD has its own L2.  With a grid
// that is a multiple of 8, XCD j takes the contiguous rows [j nrows / 8,
// (j + 1) nrows / 8) and its G / 8 workgroups stride through them, so the
// neighbouring rows a stencil reads (y +- 1 in the same step, z +- 1 a step
// or two later) are fetched into the same L2 rather than from HBM again by
// another XCD.  Other grids take every row in one range.
// ---------------------------------------------------------------------------
constexpr unsigned NUM_XCD = 8;

struct RowSlab {
  unsigned r0, r1;  // rows of this workgroup's XCD
  unsigned k, per;  // rank of the workgroup among them, their number
};

__device__ inline RowSlab row_slab(unsigned nrows) {
  const unsigned G = gridDim.x;
  if (G >= NUM_XCD && G % NUM_XCD == 0) {
    const unsigned j = blockIdx.x % NUM_XCD;
    return {(unsigned)((unsigned long long)nrows * j / NUM_XCD),
            (unsigned)((unsigned long long)nrows * (j + 1) / NUM_XCD), blockIdx.x / NUM_XCD, G / NUM_XCD};
  }
  return {0u, nrows, blockIdx.x, G};
}

template <int WG, class F>
__device__ inline void for_row_pairs(int nx, unsigned nrows, F&& f) {
  const RowSlab sl = row_slab(nrows);
  if (nx >= WG) {
    for (unsigned row0 = sl.r0 + sl.k; row0 < sl.r1; row0 += 2 * sl.per) {
      const unsigned row1 = row0 + sl.per;
      for (int x = threadIdx.x; x < nx; x += WG) f(row0, row1, row1 < sl.r1, x);
    }
  } else {
    const unsigned rps = (unsigned)(WG / nx), rl = threadIdx.x / (unsigned)nx;
    const int x = (int)(threadIdx.x - rl * (unsigned)nx);
    const unsigned stride = sl.per * rps;
    if (rl < rps)
      for (unsigned rb = sl.r0 + sl.k * rps; rb < sl.r1; rb += 2 * stride) {
        const unsigned row0 = rb + rl, row1 = row0 + stride;
        if (row0 < sl.r1) f(row0, row1, row1 < sl.r1, x);
      }
  }
}

template <int WG, class F>
__device__ inline void for_rows(int nx, unsigned nrows, F&& f) {
  const RowSlab sl = row_slab(nrows);
  if (nx >= WG) {
    for (unsigned row = sl.r0 + sl.k; row < sl.r1; row += sl.per)
      for (int x = threadIdx.x; x < nx; x += WG) f(row, x);
  } else {
    const unsigned rps = (unsigned)(WG / nx), rl = threadIdx.x / (unsigned)nx;
    const int x = (int)(threadIdx.x - rl * (unsigned)nx);
    if (rl < rps)
      for (unsigned rb = sl.r0 + sl.k * rps; rb < sl.r1; rb += sl.per * rps) {
        const unsigned row = rb + rl;
        if (row < sl.r1) f(row, x);
      }
  }
}

// ---------------------------------------------------------------------------
// Streaming element access (non-temporal hint), for values that are read or
// written once per kernel and not reused from the caches.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T nt_ld(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ inline void nt_st(T* p, T v) { __builtin_nontemporal_store(v, p); }
template <typename T>
__device__ inline C<T> sld(const C<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return C<T>{v.x, v.y};
}
template <typename T>
__device__ inline void sst(C<T>* p, C<T> c) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = c.x;
  v.y = c.y;
  __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
}

// ---------------------------------------------------------------------------
// Raw buffer access: a resource per workgroup-uniform slice, a per-thread
// byte offset and a compile-time (scalar) byte offset per access, so that a
// strided sweep costs no vector address arithmetic.  Word 3 of the resource
// is the gfx9-family raw (untyped, 32-bit) format; accesses past `bytes`
// read zero and drop writes.
// ---------------------------------------------------------------------------
using brsrc = __amdgpu_buffer_rsrc_t;
__device__ inline brsrc make_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)(uint32_t)bytes, 0x00020000);
}
// STREAM: non-temporal hint (cache-policy bit nt) for single-use data
template <typename T, bool STREAM = false>
__device__ inline C<T> bload(brsrc r, uint32_t voff, uint32_t soff) {
  constexpr int aux = STREAM ? 2 : 0;
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(C<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, aux));
  } else {
    return __builtin_bit_cast(C<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, aux));
  }
}
template <typename T, bool STREAM = false>
__device__ inline void bstore(C<T> v, brsrc r, uint32_t voff, uint32_t soff) {
  constexpr int aux = STREAM ? 2 : 0;
  if constexpr (sizeof(T) == 4) {
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, soff, aux);
  } else {
    using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, v), r, voff, soff, aux);
  }
}

// ---------------------------------------------------------------------------
// Reductions (FP64, deterministic order).
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int clog2(int k) { return k <= 1 ? 0 : 1 + clog2((k + 1) / 2); }

// Sum K <= 64 values over the workgroup; result valid in thread 0.  scratch
// must hold (NTHR / 64) * K doubles.  Within a wave the sums form a
// reduce-scatter: each halving step keeps half of the values a lane still
// holds and exchanges the other half with the partner lane, so a wave pays
// about K shuffles instead of K log2(64).  Afterwards the lanes l with
// l mod 2^(6-M) == 0 hold the wave total of value l >> (6 - M), M =
// ceil(log2 K).  The order of every sum depends on lane and wave indices
// only, so results are reproducible.
template <int NTHR, int K>
__device__ inline void block_sum(double* vals, double* scratch) {
  static_assert(K >= 1 && K <= 64, "block_sum: 1..64 values");
  constexpr int M = clog2(K), KP = 1 << M, SH = 6 - M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) v[k] = k < K ? vals[k] : 0.0;
#pragma unroll
  for (int s = 0; s < M; ++s) {
    const int o = 32 >> s, h = KP >> (s + 1);
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int k = 0; k < h; ++k) {
      const double keep = up ? v[h + k] : v[k];
      const double send = up ? v[k] : v[h + k];
      v[k] = keep + __shfl_xor(send, o, 64);
    }
  }
  double t = v[0];
#pragma unroll
  for (int o = 32 >> M; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  if ((lane & ((1 << SH) - 1)) == 0 && (lane >> SH) < K) scratch[wave * K + (lane >> SH)] = t;
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
