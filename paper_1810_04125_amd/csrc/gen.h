// Entry generators of the permuted operator A_hat(i,j) = a(perm[i], perm[j]).
// The compression is partially matrix-free (Sec. 4): the library never
// stores A; the kernels evaluate entries where they need them.
#pragma once

#include "hss_internal.h"

namespace hss {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInv4Pi = 0.07957747154594767;  // 1/(4 pi)

__device__ __forceinline__ double toeplitz_entry(const GenDev& g, int64_t i, int64_t j) {
  int64_t k = g.perm[i] - g.perm[j];
  k = k < 0 ? -k : k;
  return g.tcol[k];
}

__device__ __forceinline__ double dist2(const double* __restrict__ pts, int64_t i, int64_t j) {
  const double dx = pts[3 * i] - pts[3 * j];
  const double dy = pts[3 * i + 1] - pts[3 * j + 1];
  const double dz = pts[3 * i + 2] - pts[3 * j + 2];
  return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ double laplace_entry(const GenDev& g, int64_t i, int64_t j) {
  if (i == j) return g.diag;
  return kInv4Pi / sqrt(dist2(g.pts, i, j));
}

__device__ __forceinline__ double gauss_entry(const GenDev& g, int64_t i, int64_t j) {
  double v = exp(-dist2(g.pts, i, j) * g.inv2s2);
  return i == j ? v + g.diag : v;
}

__device__ __forceinline__ double dense_entry(const GenDev& g, int64_t i, int64_t j) {
  return g.dense[g.perm[j] * g.ld + g.perm[i]];
}

__device__ __forceinline__ double gen_entry(const GenDev& g, int64_t i, int64_t j) {
  switch (g.family) {
    case HSS_FAM_TOEPLITZ: return toeplitz_entry(g, i, j);
    case HSS_FAM_LAPLACE: return laplace_entry(g, i, j);
    case HSS_FAM_GAUSS: return gauss_entry(g, i, j);
    default: return dense_entry(g, i, j);
  }
}

}  // namespace hss
