// Byte offsets of the raw buffer accesses of the padded-line passes of G
// (green_reg.hip), shared by the kernels and by the host-side range audit
// (bq_audit_raw_ranges), so that the audit checks the arithmetic the
// kernels run.  A raw buffer access reads zero or drops the write when its
// offset passes the resource's size, so an indexing error there would not
// fault: the audit proves, for every instantiated grid and precision, that
// each resource is under 2^31 bytes and that every offset a launch can form
// (its per-thread part plus its compile-time part, plus the element) lies
// inside it without wrapping 32 bits.
#pragma once
#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace bq {

// R1 points per thread, R2 threads per padded 2N-point line, SZ bytes per
// complex element.
template <int N, int R1, int R2, uint32_t SZ>
struct PadRaw {
  static constexpr size_t V = (size_t)N * N * N;
  // z-line spectrum of one system: the two z parity classes, N^3 each.
  // Value (i, k2) of thread j of line L = y N + x is padded frequency
  // kp = j + R2 i + R1 k2 (R1, R2 even): class kp & 1 = j & 1, plane
  // kp >> 1 = (j >> 1) + (R2 i + R1 k2) / 2.
  static constexpr size_t z_bytes = 2 * V * SZ;
  __host__ __device__ static constexpr uint64_t z_v64(int j, int L) {
    return ((uint64_t)(j & 1) * N * N * N + (uint64_t)(j >> 1) * N * N + (uint64_t)L) * SZ;
  }
  __host__ __device__ static constexpr uint64_t z_s64(int i, int k2) {
    return (uint64_t)((R2 * i + R1 * k2) >> 1) * N * N * SZ;
  }
  // y column (kz, kx) of one (system, (pz, px) class) slice of N^3: element
  // y at (kz N + y) N + kx; thread j holds y = j + R2 m, m < R1 / 2.
  static constexpr size_t y_bytes = V * SZ;
  __host__ __device__ static constexpr uint64_t y_v64(int kz, int kx, int j) {
    return ((uint64_t)kz * N * N + (uint64_t)kx + (uint64_t)j * N) * SZ;
  }
  __host__ __device__ static constexpr uint64_t y_s64(int m) { return (uint64_t)m * R2 * N * SZ; }
  // transfer function from class (pz, 0, px): classes (pz, py, px) are
  // 2 N^3 apart in py, each [kz][ky][kx]; value (i, k2) of thread j is
  // padded y frequency kp = j + R2 i + R1 k2, in class j & 1 at ky = kp >> 1.
  static constexpr size_t g_bytes = 3 * V * SZ;
  __host__ __device__ static constexpr uint64_t g_v64(int j, int kz, int kx) {
    return ((uint64_t)(j & 1) * 2 * N * N * N + (uint64_t)kz * N * N + (uint64_t)kx + (uint64_t)(j >> 1) * N) * SZ;
  }
  __host__ __device__ static constexpr uint64_t g_s64(int i, int k2) {
    return (uint64_t)((R2 * i + R1 * k2) >> 1) * N * SZ;
  }
  // the 32-bit offsets the kernels pass to the buffer instructions
  __host__ __device__ static constexpr uint32_t z_v(int j, int L) { return (uint32_t)z_v64(j, L); }
  __host__ __device__ static constexpr uint32_t z_s(int i, int k2) { return (uint32_t)z_s64(i, k2); }
  __host__ __device__ static constexpr uint32_t y_v(int kz, int kx, int j) { return (uint32_t)y_v64(kz, kx, j); }
  __host__ __device__ static constexpr uint32_t y_s(int m) { return (uint32_t)y_s64(m); }
  __host__ __device__ static constexpr uint32_t g_v(int j, int kz, int kx) { return (uint32_t)g_v64(j, kz, kx); }
  __host__ __device__ static constexpr uint32_t g_s(int i, int k2) { return (uint32_t)g_s64(i, k2); }
};

// Workgroup h of the y pass over B systems: system b, class cls = pz * 2 +
// px and line block lb.  Workgroup h runs on XCD h mod 8; the B systems of
// one (class, line block) take consecutive slots on one XCD, so the
// transfer-function slab they share is fetched into that XCD's L2 once.
// nlb = N^2 / lines per workgroup; the grid has 4 nlb B workgroups.
struct YcSlot {
  int b, cls, lb;
};
__host__ __device__ inline YcSlot yc_slot(int h, int B, int nlb) {
  const int sl = h >> 3;
  const int b = sl % B;
  const int q = (sl / B) * 8 + (h & 7);
  const int cls = q / nlb;
  return YcSlot{b, cls, q - cls * nlb};
}

}  // namespace bq
