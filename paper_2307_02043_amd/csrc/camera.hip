// Camera sampling of the detector-plane field: the M x M camera image of an
// N x N window field f is D f D^T, with D (M x N) the trigonometric
// interpolation of the window's samples at the camera's pixel centres
// (reading of the camera geometry; the paper's cameras have pixel counts of
// their own, Section 6).  The adjoint takes an M x M image r to D^H r conj(D).
// Both are two batched complex matrix products, run on the matrix cores.
#include "bq_kernels.h"

namespace bq {

// C_b(i, j) = sum_k opA(A_b(i, k)) opB(B_b(k, j)) for b < grid z, with
// element (i, k) of A_b at A + b sAb + i sAi + k sAk (sAb = 0: one matrix
// for all b), opA = conj when conjA; the same for B and C.
//
// Matrix cores: each wave owns a 16 x 16 output tile and steps through K
// four at a time with the 16 x 16 x 4 MFMA of the element type (FP32 or
// FP64 products, accumulation in the element type); a complex product is
// four real ones, Re += Ar Br - Ai Bi and Im += Ar Bi + Ai Br.  Lane l
// supplies A(i0 + l mod 16, k0 + l / 16) and B(k0 + l / 16, j0 + l mod 16);
// output r of lane l is C(i0 + 4 (l / 16) + r, j0 + l mod 16) for FP32 and
// C(i0 + l / 16 + 4 r, j0 + l mod 16) for FP64.  Operands past the matrix
// edges are zeros, so every lane of a wave issues every MFMA.  Four waves
// per workgroup take a 32 x 32 block of C.
struct GemmDesc {
  int I, J, K;
  long long sAb, sAi, sAk, sBb, sBk, sBj, sCb, sCi, sCj;
  int conjA, conjB;
};

typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using V = mfma_f4;
  static __device__ inline V mac(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
  using V = mfma_d4;
  static __device__ inline V mac(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <typename T>
__global__ void __launch_bounds__(256) k_cgemm(const C<T>* A, const C<T>* Bm, C<T>* Cm, GemmDesc d) {
  using M = Mfma<T>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = (blockIdx.y * 2 + (wave >> 1)) * 16, j0 = (blockIdx.x * 2 + (wave & 1)) * 16;
  const long long b = blockIdx.z;
  const C<T>* Ab = A + b * d.sAb;
  const C<T>* Bb = Bm + b * d.sBb;
  const int ia = i0 + (lane & 15), jb = j0 + (lane & 15), kl = lane >> 4;
  typename M::V re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
#pragma unroll 4
  for (int k0 = 0; k0 < d.K; k0 += 4) {
    const int k = k0 + kl;
    C<T> a{0, 0}, w{0, 0};
    if (ia < d.I && k < d.K) a = Ab[ia * d.sAi + k * d.sAk];
    if (k < d.K && jb < d.J) w = Bb[k * d.sBk + jb * d.sBj];
    if (d.conjA) a.y = -a.y;
    if (d.conjB) w.y = -w.y;
    re = M::mac(a.x, w.x, re);
    re = M::mac(-a.y, w.y, re);
    im = M::mac(a.x, w.y, im);
    im = M::mac(a.y, w.x, im);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + M::row(lane, r), j = jb;
    if (i < d.I && j < d.J) Cm[b * d.sCb + i * d.sCi + j * d.sCj] = C<T>{re[r], im[r]};
  }
}

template <typename T>
static void cgemm(int B, const C<T>* A, const C<T>* Bm, C<T>* Cm, const GemmDesc& d, hipStream_t st) {
  const dim3 grid((d.J + 31) / 32, (d.I + 31) / 32, B);
  hipLaunchKernelGGL((k_cgemm<T>), grid, dim3(256), 0, st, A, Bm, Cm, d);
}

// out_b (M x M) = D win_b D^T through tmp_b (N x M) = win_b D^T
template <typename T>
void camera_apply(int B, int N, int M, const C<T>* win, const C<T>* D, C<T>* tmp, C<T>* out, hipStream_t st) {
  const long long n = N, m = M;
  // tmp(y, a) = sum_x win(y, x) D(a, x)
  cgemm<T>(B, win, D, tmp, GemmDesc{N, M, N, n * n, n, 1, 0, 1, n, n * m, m, 1, 0, 0}, st);
  // out(a', a) = sum_y D(a', y) tmp(y, a)
  cgemm<T>(B, D, tmp, out, GemmDesc{M, M, N, 0, n, 1, n * m, m, 1, m * m, m, 1, 0, 0}, st);
}

// win_b (N x N) = D^H r_b conj(D) through tmp_b (M x N) = r_b conj(D)
template <typename T>
void camera_adjoint(int B, int N, int M, const C<T>* r, const C<T>* D, C<T>* tmp, C<T>* win, hipStream_t st) {
  const long long n = N, m = M;
  // tmp(a', x) = sum_a r(a', a) conj(D(a, x))
  cgemm<T>(B, r, D, tmp, GemmDesc{M, N, M, m * m, m, 1, 0, n, 1, m * n, n, 1, 0, 1}, st);
  // win(y, x) = sum_a' conj(D(a', y)) tmp(a', x)
  cgemm<T>(B, D, tmp, win, GemmDesc{N, N, M, 0, 1, n, m * n, n, 1, n * n, n, 1, 1, 0}, st);
}

template void camera_apply<float>(int, int, int, const C<float>*, const C<float>*, C<float>*, C<float>*,
                                  hipStream_t);
template void camera_apply<double>(int, int, int, const C<double>*, const C<double>*, C<double>*, C<double>*,
                                   hipStream_t);
template void camera_adjoint<float>(int, int, int, const C<float>*, const C<float>*, C<float>*, C<float>*,
                                    hipStream_t);
template void camera_adjoint<double>(int, int, int, const C<double>*, const C<double>*, C<double>*,
                                     C<double>*, hipStream_t);

}  // namespace bq
