// Gaussian random matrix R of the adaptive sampling (Alg. 3: the new
// columns drawn in every round), generated on the device from a counter-based
// generator so that entry R(i, j) depends only on (seed, i, j):
//   * Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011) with counter
//     (i >> 2, j, 0, 0) and key (seed, 0) gives four 64-bit words for the
//     rows 4q .. 4q+3 of column j;
//   * each word becomes a double in (0, 1] as ((w >> 11) + 1) 2^-53;
//   * Box and Muller (1958) in FP64 on the pairs (u0, u1), (u2, u3):
//     sqrt(-2 log u_a) times cos and sin of (2 pi) u_b.
// Columns appended in a later round never change the earlier ones, and a
// sample of any size is reproducible entry by entry.
#include "hss_internal.h"

namespace hss {

namespace {

constexpr uint64_t kPhM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhW1 = 0xBB67AE8584CAA73Bull;
constexpr double kTwoPi = 6.283185307179586;   // the double nearest to 2 pi

struct Words4 {
  uint64_t w[4];
};

__device__ __forceinline__ Words4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                                uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhW0;
      k1 += kPhW1;
    }
    const uint64_t hi0 = __umul64hi(kPhM0, c0), lo0 = kPhM0 * c0;
    const uint64_t hi1 = __umul64hi(kPhM1, c2), lo1 = kPhM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return Words4{{c0, c1, c2, c3}};
}

__device__ __forceinline__ double unit53(uint64_t w) { return ((double)(w >> 11) + 1.0) * 0x1.0p-53; }

// Thread (q, t) writes rows 4q .. 4q+3 of output column t (key column c0 + t).
template <bool WORDS>
__global__ __launch_bounds__(256) void k_randn(double* __restrict__ R, int64_t ldr, uint64_t* __restrict__ W,
                                               int64_t ldw, int64_t n, int32_t c0, uint64_t seed) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t t = blockIdx.y;
  const int64_t i0 = 4 * q;
  if (i0 >= n) return;
  const Words4 o = philox4x64_10((uint64_t)q, (uint64_t)(c0 + t), 0ull, 0ull, seed, 0ull);
  if (WORDS) {
    uint64_t* dst = W + (int64_t)t * ldw + i0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u < n) dst[u] = o.w[u];
    return;
  }
  double z[4];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double rho = sqrt(-2.0 * log(unit53(o.w[2 * p])));
    double s, c;
    sincos(kTwoPi * unit53(o.w[2 * p + 1]), &s, &c);
    z[2 * p] = rho * c;
    z[2 * p + 1] = rho * s;
  }
  double* dst = R + (int64_t)t * ldr + i0;
  if (i0 + 4 <= n && (((uintptr_t)dst) & 31) == 0) {
    reinterpret_cast<double4*>(dst)[0] = make_double4(z[0], z[1], z[2], z[3]);
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u < n) dst[u] = z[u];
  }
}

}  // namespace

void launch_randn(double* R, int64_t ldr, int64_t n, int32_t c0, int32_t ncols, uint64_t seed, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  const int64_t nq = (n + 3) / 4;
  for (int32_t t0 = 0; t0 < ncols; t0 += 65535) {   // grid.y limit
    const int32_t nc = std::min(65535, ncols - t0);
    const dim3 grid((unsigned)((nq + 255) / 256), (unsigned)nc);
    hipLaunchKernelGGL(k_randn<false>, grid, dim3(256), 0, s, R + (int64_t)t0 * ldr, ldr, (uint64_t*)nullptr,
                       (int64_t)0, n, c0 + t0, seed);
  }
}

void launch_rand_words(uint64_t* W, int64_t ldw, int64_t n, int32_t c0, int32_t ncols, uint64_t seed,
                       hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  const int64_t nq = (n + 3) / 4;
  for (int32_t t0 = 0; t0 < ncols; t0 += 65535) {
    const int32_t nc = std::min(65535, ncols - t0);
    const dim3 grid((unsigned)((nq + 255) / 256), (unsigned)nc);
    hipLaunchKernelGGL(k_randn<true>, grid, dim3(256), 0, s, (double*)nullptr, (int64_t)0, W + (int64_t)t0 * ldw,
                       ldw, n, c0 + t0, seed);
  }
}

}  // namespace hss
