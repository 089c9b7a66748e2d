// Reduced-precision sampling S = A_hat R for the adaptive HSS compression
// (the sampling product of Sec. 2.2, eq. sample_off_diag, in FP32 or in
// split BF16): the stopping tests, the IDs and every other step stay FP64.
//
//   FP32    entries generated in FP32 (distances in FP64, then FP32
//           rsqrt / exp), R rounded to FP32, v_mfma_f32_16x16x4f32.
//   BF16x3  a = a_hi + a_lo and r = r_hi + r_lo with bf16 parts; three
//           v_mfma_f32_16x16x32_bf16 products a_hi r_hi + a_hi r_lo + a_lo r_hi.
//
// Both accumulate in FP32 over K chunks of 64 and add the chunk sums into
// FP64 accumulators; split-K partials are reduced in FP64 in fixed order.
// The FP32 sum is the largest error term of the FP32 path (about 1.4e-7
// relative on the n = 65536 Gaussian-kernel rows at 64, 3.9e-7 at 512;
// generation and operand rounding add 2e-8 to 5e-8 each); the BF16 split
// (16 bits per operand) sets the BF16x3 path's level, about 4e-6.  Scaling
// rows or columns by powers of two would not change these: the formats
// carry an exponent per value, and the generated families stay far inside
// their range.
// With `offdiag` set, entries inside a leaf's diagonal block are skipped,
// so the product is (A_hat - blockdiag(D_leaf)) R and the leaf local
// samples need no D R subtraction (no cancellation against the near field).
#include "gen.h"

namespace hss {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int LP_ROWS = 128;
constexpr int LP_COLS = 64;
constexpr int LP_BK = 32;
constexpr int LP_CHUNK = 64;    // FP32 accumulation length before the FP64 sum

template <int FAM>
__device__ __forceinline__ float entry32(const GenDev& g, int64_t i, int64_t j) {
  if constexpr (FAM == HSS_FAM_TOEPLITZ) {
    return (float)toeplitz_entry(g, i, j);
  } else if constexpr (FAM == HSS_FAM_LAPLACE) {
    if (i == j) return (float)g.diag;
    const float r2 = (float)dist2(g.pts, i, j);
    return (float)kInv4Pi * rsqrtf(r2);
  } else {
    const float v = expf(-(float)(dist2(g.pts, i, j) * g.inv2s2));
    return i == j ? v + (float)g.diag : v;
  }
}

template <int FAM, int TRANS>
__device__ __forceinline__ float lp_entry(const GenDev& g, int64_t row, int64_t col, int64_t llo, int64_t lhi,
                                          bool offdiag) {
  if (offdiag && col >= llo && col < lhi) return 0.0f;
  return TRANS ? entry32<FAM>(g, col, row) : entry32<FAM>(g, row, col);
}

// Kernel-family entry from the row point (px, py, pz) and a column point
// staged in LDS: distance in FP64, then FP32 rsqrt / exp.  Symmetric, so
// the transposed product uses the same value.
template <int FAM>
__device__ __forceinline__ float pts_entry32(double px, double py, double pz, const double* pj, bool diag_hit,
                                             float diag, double inv2s2) {
  const double dx = px - pj[0], dy = py - pj[1], dz = pz - pj[2];
  const double r2 = dx * dx + dy * dy + dz * dz;
  if constexpr (FAM == HSS_FAM_LAPLACE) {
    const float v = (float)kInv4Pi * rsqrtf((float)r2);
    return diag_hit ? diag : v;
  } else {
    const float v = expf(-(float)(r2 * inv2s2));
    return diag_hit ? v + diag : v;
  }
}

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

template <int FAM, int TRANS, int BF>
__global__ __launch_bounds__(512) void k_sample_lp(GenDev g, const double* __restrict__ R, int64_t ldr,
                                                   double* __restrict__ out, int64_t lds, int32_t ncols,
                                                   int64_t kchunk, int32_t nsplit, const int32_t* __restrict__ leaf_lo,
                                                   const int32_t* __restrict__ leaf_hi, int32_t offdiag) {
  constexpr bool PTS = FAM == HSS_FAM_LAPLACE || FAM == HSS_FAM_GAUSS;
  __shared__ float Rf[LP_BK][LP_COLS + 1];
  __shared__ __bf16 Rhi[LP_COLS][LP_BK + 8];
  __shared__ __bf16 Rlo[LP_COLS][LP_BK + 8];
  __shared__ double Ps[PTS ? LP_BK : 1][3];
  const int64_t n = g.n;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * LP_ROWS + wave * 16;
  const int col0 = blockIdx.y * LP_COLS;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = min(n, kb + kchunk);
  const int64_t my_row = row0 + (lane & 15);
  const bool row_ok = my_row < n;
  const int kq = lane >> 4;
  int64_t llo = -1, lhi = -1;
  if (offdiag && row_ok) {
    llo = leaf_lo[my_row];
    lhi = leaf_hi[my_row];
  }
  double px = 0.0, py = 0.0, pz = 0.0;
  if constexpr (PTS) {
    if (row_ok) {
      px = g.pts[3 * my_row];
      py = g.pts[3 * my_row + 1];
      pz = g.pts[3 * my_row + 2];
    }
  }
  const float fdiag = (float)g.diag;
  dbl4 acc64[4];
  flt4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    acc64[c] = dbl4{0.0, 0.0, 0.0, 0.0};
    acc[c] = flt4{0.f, 0.f, 0.f, 0.f};
  }
  int since = 0;
  for (int64_t kt = kb; kt < ke; kt += LP_BK) {
    for (int idx = threadIdx.x; idx < LP_BK * LP_COLS; idx += 512) {
      const int r = idx % LP_BK, c = idx / LP_BK;
      const int64_t gk = kt + r;
      const int gc = col0 + c;
      const float x = (gk < ke && gc < ncols) ? (float)R[(int64_t)gc * ldr + gk] : 0.0f;
      if (BF) {
        __bf16 hi, lo;
        split_bf16(x, hi, lo);
        Rhi[c][r] = hi;
        Rlo[c][r] = lo;
      } else {
        Rf[r][c] = x;
      }
    }
    if constexpr (PTS) {
      for (int idx = threadIdx.x; idx < LP_BK * 3; idx += 512) {
        const int64_t gk = kt + idx / 3;
        Ps[idx / 3][idx % 3] = gk < ke ? g.pts[3 * kt + idx] : 0.0;
      }
    }
    __syncthreads();
    if (BF) {
      const int64_t j0 = kt + 8 * kq;
      bf8 ahi, alo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t j = j0 + e;
        float a;
        if constexpr (PTS) {
          const float v = pts_entry32<FAM>(px, py, pz, Ps[8 * kq + e], my_row == j, fdiag, g.inv2s2);
          a = (row_ok && j < ke && !(offdiag && j >= llo && j < lhi)) ? v : 0.0f;
        } else {
          a = (row_ok && j < ke) ? lp_entry<FAM, TRANS>(g, my_row, j, llo, lhi, offdiag) : 0.0f;
        }
        __bf16 hi, lo;
        split_bf16(a, hi, lo);
        ahi[e] = hi;
        alo[e] = lo;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bf8 bhi = *reinterpret_cast<const bf8*>(&Rhi[c * 16 + (lane & 15)][8 * kq]);
        const bf8 blo = *reinterpret_cast<const bf8*>(&Rlo[c * 16 + (lane & 15)][8 * kq]);
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[c], 0, 0, 0);
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[c], 0, 0, 0);
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[c], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < LP_BK; kk += 4) {
        const int64_t j = kt + kk + kq;
        float a;
        if constexpr (PTS) {
          const float v = pts_entry32<FAM>(px, py, pz, Ps[kk + kq], my_row == j, fdiag, g.inv2s2);
          a = (row_ok && j < ke && !(offdiag && j >= llo && j < lhi)) ? v : 0.0f;
        } else {
          a = (row_ok && j < ke) ? lp_entry<FAM, TRANS>(g, my_row, j, llo, lhi, offdiag) : 0.0f;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float b = Rf[kk + kq][c * 16 + (lane & 15)];
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    since += LP_BK;
    if (since >= LP_CHUNK) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc64[c][v] += (double)acc[c][v];
        acc[c] = flt4{0.f, 0.f, 0.f, 0.f};
      }
      since = 0;
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc64[c][v] += (double)acc[c][v];
  // FP32-family result layout: D[i][j] with i = 4*(lane/16) + v, j = lane % 16
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int gc = col0 + c * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gr = row0 + 4 * kq + v;
      if (gr >= n || gc >= ncols) continue;
      if (nsplit == 1) {
        out[(int64_t)gc * lds + gr] = acc64[c][v];
      } else {
        const int64_t ncp = (int64_t)gridDim.y * LP_COLS;
        out[((int64_t)blockIdx.z * ncp + gc) * n + gr] = acc64[c][v];
      }
    }
  }
}

template <int FAM, int BF>
static void launch_lp_fam(const GenDev& g, int transpose, const double* R, int64_t ldr, double* out, int64_t lds,
                          int32_t ncols, int64_t kchunk, int nsplit, dim3 grid, const int32_t* llo,
                          const int32_t* lhi, int offdiag, hipStream_t s) {
  if (transpose)
    hipLaunchKernelGGL((k_sample_lp<FAM, 1, BF>), grid, dim3(512), 0, s, g, R, ldr, out, lds, ncols, kchunk,
                       nsplit, llo, lhi, offdiag);
  else
    hipLaunchKernelGGL((k_sample_lp<FAM, 0, BF>), grid, dim3(512), 0, s, g, R, ldr, out, lds, ncols, kchunk,
                       nsplit, llo, lhi, offdiag);
}

template <int BF>
static void launch_lp(const GenDev& g, int transpose, const double* R, int64_t ldr, double* out, int64_t lds,
                      int32_t ncols, int64_t kchunk, int nsplit, dim3 grid, const int32_t* llo, const int32_t* lhi,
                      int offdiag, hipStream_t s) {
  switch (g.family) {
    case HSS_FAM_TOEPLITZ:
      launch_lp_fam<HSS_FAM_TOEPLITZ, BF>(g, transpose, R, ldr, out, lds, ncols, kchunk, nsplit, grid, llo, lhi,
                                          offdiag, s);
      break;
    case HSS_FAM_LAPLACE:
      launch_lp_fam<HSS_FAM_LAPLACE, BF>(g, transpose, R, ldr, out, lds, ncols, kchunk, nsplit, grid, llo, lhi,
                                         offdiag, s);
      break;
    default:
      launch_lp_fam<HSS_FAM_GAUSS, BF>(g, transpose, R, ldr, out, lds, ncols, kchunk, nsplit, grid, llo, lhi,
                                       offdiag, s);
      break;
  }
}

void launch_sample_lp(const GenDev& g, int32_t transpose, int32_t bf16x3, const double* R, int64_t ldr,
                      double* out, int64_t lds, int32_t ncols, int64_t kchunk, int32_t nz, dim3 grid,
                      const int32_t* leaf_lo, const int32_t* leaf_hi, int32_t offdiag, hipStream_t s) {
  if (g.family == HSS_FAM_DENSE) throw Error(HSS_ERR_INVALID_ARG, "reduced-precision sampling needs a generated family");
  if (bf16x3)
    launch_lp<1>(g, transpose, R, ldr, out, lds, ncols, kchunk, nz, grid, leaf_lo, leaf_hi, offdiag, s);
  else
    launch_lp<0>(g, transpose, R, ldr, out, lds, ncols, kchunk, nz, grid, leaf_lo, leaf_hi, offdiag, s);
}

}  // namespace hss
