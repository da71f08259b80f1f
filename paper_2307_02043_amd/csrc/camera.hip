// Camera sampling of the detector-plane field: the M x M camera image of an
// N x N window field f is D f D^T, with D (M x N) the trigonometric
// interpolation of the window's samples at the camera's pixel centres
// (reading of the camera geometry; the paper's cameras have pixel counts of
// their own, Section 6).  The adjoint takes an M x M image r to D^H r conj(D).
// Both are two batched complex matrix products, run by one tiled kernel.
#include "bq_kernels.h"

namespace bq {

// C_b(i, j) = sum_k opA(A_b(i, k)) opB(B_b(k, j)) for b < grid z, with
// element (i, k) of A_b at A + b sAb + i sAi + k sAk (sAb = 0: one matrix
// for all b), opA = conj when conjA; the same for B and C.  16 x 16 output
// tiles per 256-thread workgroup, K in chunks of 16 through LDS; the
// accumulation runs in the element type.
struct GemmDesc {
  int I, J, K;
  long long sAb, sAi, sAk, sBb, sBk, sBj, sCb, sCi, sCj;
  int conjA, conjB;
};

template <typename T>
__global__ void __launch_bounds__(256) k_cgemm(const C<T>* A, const C<T>* Bm, C<T>* Cm, GemmDesc d) {
  __shared__ C<T> As[16][17];
  __shared__ C<T> Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  const long long b = blockIdx.z;
  const C<T>* Ab = A + b * d.sAb;
  const C<T>* Bb = Bm + b * d.sBb;
  C<T> acc{0, 0};
  for (int k0 = 0; k0 < d.K; k0 += 16) {
    // A tile rows i0..i0+15, columns k0..k0+15; B tile rows k0.., columns j0..
    {
      const int ai = blockIdx.y * 16 + ty, ak = k0 + tx;
      C<T> v{0, 0};
      if (ai < d.I && ak < d.K) {
        v = Ab[ai * d.sAi + ak * d.sAk];
        if (d.conjA) v.y = -v.y;
      }
      As[ty][tx] = v;
      const int bk = k0 + ty, bj = blockIdx.x * 16 + tx;
      C<T> w{0, 0};
      if (bk < d.K && bj < d.J) {
        w = Bb[bk * d.sBk + bj * d.sBj];
        if (d.conjB) w.y = -w.y;
      }
      Bs[ty][tx] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const C<T> a = As[ty][kk], bb = Bs[kk][tx];
      acc.x = fma(a.x, bb.x, acc.x);
      acc.x = fma(-a.y, bb.y, acc.x);
      acc.y = fma(a.x, bb.y, acc.y);
      acc.y = fma(a.y, bb.x, acc.y);
    }
    __syncthreads();
  }
  if (i < d.I && j < d.J) Cm[b * d.sCb + i * d.sCi + j * d.sCj] = acc;
}

template <typename T>
static void cgemm(int B, const C<T>* A, const C<T>* Bm, C<T>* Cm, const GemmDesc& d, hipStream_t st) {
  const dim3 grid((d.J + 15) / 16, (d.I + 15) / 16, B);
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
