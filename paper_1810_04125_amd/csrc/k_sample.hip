// Matrix-free random sampling S = A_hat R (and S^c = A_hat^T R) for the
// adaptive HSS compression (Sec. 2.2, eq. sample_off_diag: the samples of
// every Hankel block derive from S^r = A R and S^c = A^* R).
//
// A is never stored: each lane generates the entries it feeds to the
// matrix core.  One workgroup = 4 waves computes a 128 x 64 tile of S
// (each wave 32 rows x 64 columns = eight 16x16 FP64 MFMA blocks), so every
// generated entry is reused for 64 columns of R and every value of R read
// from LDS for two row blocks.  With 128 or more columns the Toeplitz and
// Gaussian kernels take wider tiles that reuse each entry for 128 columns
// (see sample_tile).  R tiles are staged in LDS and shared by the 4 waves.
// The K dimension (n) is split over blockIdx.z when the tile grid alone
// would not fill the 256 CUs; split partial sums are reduced in fixed
// order, so results are deterministic.

#include <algorithm>

#include "gen.h"

namespace hss {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int SM_ROWS = 128;   // rows of S per workgroup (narrow tile)
constexpr int SM_T = 256;      // threads per workgroup: 4 waves of 32 rows
constexpr int SM_COLS = 64;    // columns of S per workgroup (narrow tile)
constexpr int SM_COLS_W = 128; // wide tile
constexpr int SM_BK = 32;      // K rows of R staged per LDS tile

__global__ void k_toeplitz_table(double* __restrict__ t, int64_t n, double h) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (k == 0) {
    t[0] = kPi * kPi / (6.0 * h * h);
  } else {
    const double kk = (double)k;
    const double sign = (k & 1) ? -1.0 : 1.0;
    t[k] = sign / (kk * kk * h * h);
  }
}

void launch_toeplitz_table(double* t, int64_t n, double h, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_toeplitz_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, n, h);
}

__global__ void k_permute_points(const double* __restrict__ pts, const int64_t* __restrict__ perm,
                                 int64_t n, double* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = perm[i];
  out[3 * i] = pts[3 * p];
  out[3 * i + 1] = pts[3 * p + 1];
  out[3 * i + 2] = pts[3 * p + 2];
}

void launch_permute_points(const double* pts, const int64_t* perm, int64_t n, double* out,
                           hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_permute_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts,
                     perm, n, out);
}

// 1/sqrt(x) from the hardware estimate y (about 2^-25 relative) refined by
// one third-order step of the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ...
// with e = 1 - x y^2 taken by an FMA: y <- y + y e (1/2 + 3e/8).  The
// truncation is about (5/16) e^3, far below FP64 rounding; five operations
// instead of the eight of two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-(x * y), y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

// Kernel variant of HSS_FAM_TOEPLITZ for the identity permutation (index
// bisection): entries from an LDS window of t(|i - j|) per tile pair.
constexpr int kFamToeplitzWindow = 16;

template <int FAM>
__device__ __forceinline__ double entry_t(const GenDev& g, int64_t i, int64_t j) {
  if constexpr (FAM == HSS_FAM_TOEPLITZ) return toeplitz_entry(g, i, j);
  else if constexpr (FAM == HSS_FAM_LAPLACE) return laplace_entry(g, i, j);
  else if constexpr (FAM == HSS_FAM_GAUSS) return gauss_entry(g, i, j);
  else return dense_entry(g, i, j);
}

// out(row, col) for rows [0,n), cols [0, ncols): either S directly
// (nsplit == 1, column-major with lds) or the split-K partial buffer
// P[z][col][row]: split z's partial sums column-major, ncp = gridDim.y * COLS
// columns of n rows each (the reduce then reads and writes along rows).
// Each wave computes NH x NCB blocks of 16 x 16: the workgroup's tile is
// ROWS = 64 NH rows by COLS = 16 NCB columns, and each generated entry
// feeds NCB MFMAs.
template <int FAM, int TRANS, int NH, int NCB>
__global__ __launch_bounds__(SM_T, 2) void k_sample_f64(GenDev g, const double* __restrict__ R,
                                                     int64_t ldr, double* __restrict__ out,
                                                     int64_t lds, int32_t ncols, int64_t kchunk,
                                                     int32_t nsplit) {
  constexpr bool PTS = FAM == HSS_FAM_LAPLACE || FAM == HSS_FAM_GAUSS;
  constexpr bool TOEP = FAM == kFamToeplitzWindow;
  constexpr int COLS = 16 * NCB;
  constexpr int ROWS = 64 * NH;
  constexpr int TW = ROWS + SM_BK - 1;   // Toeplitz window: t(|i - j|) over one tile pair
  __shared__ double Rs[SM_BK][COLS + 2];
  __shared__ double Ps[PTS ? SM_BK : 1][3];   // points of the K rows of the tile
  __shared__ double Tw[TOEP ? TW : 1];
  const int64_t n = g.n;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * ROWS + wave * 16 * NH;   // NH 16-row blocks per wave
  const int col0 = blockIdx.y * COLS;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = min(n, kb + kchunk);
  int64_t my_row[NH];
  bool row_ok[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    my_row[h] = row0 + 16 * h + (lane & 15);
    row_ok[h] = my_row[h] < n;
  }
  const int kq = lane >> 4;
  double px[NH], py[NH], pz[NH];   // this lane's row points
#pragma unroll
  for (int h = 0; h < NH; ++h) px[h] = py[h] = pz[h] = 0.0;
  if constexpr (PTS) {
#pragma unroll
    for (int h = 0; h < NH; ++h)
      if (row_ok[h]) {
        px[h] = g.pts[3 * my_row[h]];
        py[h] = g.pts[3 * my_row[h] + 1];
        pz[h] = g.pts[3 * my_row[h] + 2];
      }
  }

  dbl4 acc[NH][NCB];
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[h][c] = dbl4{0.0, 0.0, 0.0, 0.0};

  // R(kt:kt+BK, col0:col0+COLS) and the tile's points are loaded into
  // registers one tile ahead, then stored to LDS (Rs[k][c], Ps[k][xyz]).
  // With the identity permutation a Toeplitz entry t(|i - j|) of the tile
  // pair (rows rb0.., K rows kt..) is Tw[i - j - (rb0 - kt - BK + 1)]: the
  // window of its ROWS + BK - 1 distinct values is staged the same way.
  constexpr int RPT = SM_BK * COLS / SM_T;
  static_assert(TW <= SM_T, "one window value per thread");
  const int64_t rb0 = (int64_t)blockIdx.x * ROWS, rb1 = rb0 + ROWS;   // rows of the workgroup
  double rr[RPT];
  double pp = 0.0, tw = 0.0;
  auto load_tile = [&](int64_t kt) {
#pragma unroll
    for (int e = 0; e < RPT; ++e) {
      const int idx = threadIdx.x + SM_T * e;
      const int r = idx % SM_BK, c = idx / SM_BK;
      const int64_t gk = kt + r;
      const int gc = col0 + c;
      rr[e] = (gk < ke && gc < ncols) ? R[(int64_t)gc * ldr + gk] : 0.0;
    }
    if constexpr (PTS) {
      if (threadIdx.x < SM_BK * 3) {
        const int64_t gk = kt + threadIdx.x / 3;
        pp = gk < ke ? g.pts[3 * kt + threadIdx.x] : 0.0;
      }
    }
    if constexpr (TOEP) {
      if (threadIdx.x < TW) {
        int64_t o = rb0 - kt - (SM_BK - 1) + threadIdx.x;
        o = o < 0 ? -o : o;
        tw = o < n ? g.tcol[o] : 0.0;   // beyond n only for rows or K rows outside the matrix
      }
    }
  };
  if (kb < ke) load_tile(kb);
  for (int64_t kt = kb; kt < ke; kt += SM_BK) {
#pragma unroll
    for (int e = 0; e < RPT; ++e) {
      const int idx = threadIdx.x + SM_T * e;
      Rs[idx % SM_BK][idx / SM_BK] = rr[e];
    }
    if constexpr (PTS) {
      if (threadIdx.x < SM_BK * 3) Ps[threadIdx.x / 3][threadIdx.x % 3] = pp;
    }
    if constexpr (TOEP) {
      if (threadIdx.x < TW) Tw[threadIdx.x] = tw;
    }
    __syncthreads();
    if (kt + SM_BK < ke) load_tile(kt + SM_BK);
    // A tile inside the matrix and off its diagonal needs neither the
    // bounds nor the diagonal selects: the kernel families take a short
    // path there (all but the few tiles that meet the diagonal or an edge).
    if constexpr (TOEP) {
      // entries from the LDS window (the diagonal's t(0) included); rows
      // and K rows outside the matrix are masked on the edge tiles only
      const bool inner = rb1 <= n && kt + SM_BK <= ke;
      const int wb = wave * 16 * NH + (lane & 15) - kq + SM_BK - 1;
#pragma unroll 2
      for (int kk = 0; kk < SM_BK; kk += 4) {
        const bool k_ok = kt + kk + kq < ke;
        double a[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          a[h] = Tw[wb + 16 * h - kk];
          if (!inner) a[h] = (row_ok[h] && k_ok) ? a[h] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
          const double b = Rs[kk + kq][c * 16 + (lane & 15)];
#pragma unroll
          for (int h = 0; h < NH; ++h)
            acc[h][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h], b, acc[h][c], 0, 0, 0);
        }
      }
      __syncthreads();
      continue;
    }
    bool fast = false;
    if constexpr (PTS) fast = rb1 <= n && kt + SM_BK <= ke && (kt + SM_BK <= rb0 || kt >= rb1);
    if (fast) {
#pragma unroll
      for (int kk = 0; kk < SM_BK; kk += 4) {
        const double qx = Ps[kk + kq][0], qy = Ps[kk + kq][1], qz = Ps[kk + kq][2];
        double a[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const double dx = px[h] - qx, dy = py[h] - qy, dz = pz[h] - qz;
          const double r2 = dx * dx + dy * dy + dz * dz;
          if constexpr (FAM == HSS_FAM_LAPLACE) a[h] = kInv4Pi * rsqrt_nr(r2);
          else a[h] = exp(-r2 * g.inv2s2);
        }
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
          const double b = Rs[kk + kq][c * 16 + (lane & 15)];
#pragma unroll
          for (int h = 0; h < NH; ++h)
            acc[h][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h], b, acc[h][c], 0, 0, 0);
        }
      }
      __syncthreads();
      continue;
    }
#pragma unroll 2
    for (int kk = 0; kk < SM_BK; kk += 4) {
      const int64_t j = kt + kk + kq;
      double a[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const bool ok = row_ok[h] && j < ke;
        if constexpr (PTS) {
          // symmetric kernels: the transposed product reads the same entries;
          // computed unconditionally and selected, so the loop has no branches
          const double dx = px[h] - Ps[kk + kq][0];
          const double dy = py[h] - Ps[kk + kq][1];
          const double dz = pz[h] - Ps[kk + kq][2];
          const double r2 = dx * dx + dy * dy + dz * dz;
          double v;
          if constexpr (FAM == HSS_FAM_LAPLACE) {
            v = kInv4Pi * rsqrt_nr(r2);
            v = my_row[h] == j ? g.diag : v;
          } else {
            v = exp(-r2 * g.inv2s2);
            v = my_row[h] == j ? v + g.diag : v;
          }
          a[h] = ok ? v : 0.0;
        } else {
          a[h] = 0.0;
          if (ok) a[h] = TRANS ? entry_t<FAM>(g, j, my_row[h]) : entry_t<FAM>(g, my_row[h], j);
        }
      }
#pragma unroll
      for (int c = 0; c < NCB; ++c) {
        const double b = Rs[kk + kq][c * 16 + (lane & 15)];
#pragma unroll
        for (int h = 0; h < NH; ++h)
          acc[h][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h], b, acc[h][c], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // FP64 16x16x4 result layout: D[i][j] with i = 4*v + lane/16, j = lane % 16
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      const int gc = col0 + c * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gr = row0 + 16 * h + 4 * v + kq;
        if (gr >= n || gc >= ncols) continue;
        if (nsplit == 1) {
          out[(int64_t)gc * lds + gr] = acc[h][c][v];
        } else {
          const int64_t ncp = (int64_t)gridDim.y * COLS;
          out[((int64_t)blockIdx.z * ncp + gc) * n + gr] = acc[h][c][v];
        }
      }
    }
}

__global__ void k_splitk_reduce(const double* __restrict__ P, int64_t n, int32_t ncols, int64_t ncp,
                                int32_t nsplit, double* __restrict__ S, int64_t lds) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * ncols) return;
  const int64_t row = idx % n;
  const int64_t col = idx / n;
  double s = 0.0;   // added in split order; the loads of 8 splits in flight together
#pragma unroll 8
  for (int z = 0; z < nsplit; ++z) s += P[((int64_t)z * ncp + col) * n + row];
  S[col * lds + row] = s;
}

// Workgroup tile of the FP64 kernels: 128 x 64 (two row blocks and four
// column blocks per wave), or for large problems where the column count
// allows, 64 x 128 for the Gaussian kernel
// (one row block and eight column blocks per wave: half the entries per
// MFMA in the same registers; its exponential is the costliest entry) and
// 128 x 128 for Toeplitz (its table gathers leave registers for two row
// blocks).  The Laplace kernel keeps the narrow tile: its entries are
// cheap enough that the wide tile's doubled LDS reads per MFMA cancel the
// saving.
struct SampleTile {
  int32_t rows, cols;
};
constexpr SampleTile kTileNarrow{SM_ROWS, SM_COLS}, kTileWideGauss{SM_ROWS / 2, SM_COLS_W},
    kTileWideToep{SM_ROWS, SM_COLS_W};

static int sample_splits(int64_t n, int32_t ncols, SampleTile t) {
  const int64_t gx = (n + t.rows - 1) / t.rows;
  const int64_t gy = (ncols + t.cols - 1) / t.cols;
  const int64_t tiles = gx * gy;
  const int64_t target = tune().sample_wg;   // 2048 by default
  int64_t z = (target + tiles - 1) / tiles;
  const int64_t zmax = (n + 255) / 256;   // at least 256 K rows per split
  if (z > zmax) z = zmax;
  if (z < 1) z = 1;
  return (int)z;
}

static SampleTile sample_tile(int32_t precision, int32_t family, int64_t n, int32_t ncols) {
  // the wide tiles where they leave at most half a narrow tile's columns
  // idle (192 columns: three narrow tiles beat two wide ones)
  if (precision != HSS_SAMPLE_FP64 || ncols < SM_COLS_W) return kTileNarrow;
  const int32_t r = ncols % SM_COLS_W;
  if (r != 0 && r <= SM_COLS) return kTileNarrow;
  SampleTile t = kTileNarrow;
  if (family == HSS_FAM_TOEPLITZ) t = kTileWideToep;
  else if (family == HSS_FAM_GAUSS) t = kTileWideGauss;
  else return kTileNarrow;
  // only where the wide grid fills the device with at most four K splits:
  // with fewer tiles, the split count that restores the workgroup count
  // multiplies the split-K partial sums written and read (at n = 16384 the
  // wide Toeplitz tile ran slower than the narrow one)
  const int64_t tiles = ((n + t.rows - 1) / t.rows) * ((ncols + t.cols - 1) / t.cols);
  return 4 * tiles >= tune().sample_wg ? t : kTileNarrow;
}

// Partial-sum capacity covering every column count up to ncols_max in
// every tile shape (the split count is not monotone in the column count,
// so take the maximum).
size_t sample_partial_elems(int64_t n, int32_t ncols_max) {
  size_t best = 0;
  for (const SampleTile t : {kTileNarrow, kTileWideGauss, kTileWideToep}) {
    const int64_t gymax = (ncols_max + t.cols - 1) / t.cols;
    for (int64_t gy = 1; gy <= gymax; ++gy) {
      const int z = sample_splits(n, (int32_t)(gy * t.cols), t);
      if (z == 1) continue;
      best = std::max(best, (size_t)z * (size_t)n * (size_t)(gy * t.cols));
    }
  }
  return best;
}

template <int FAM, int NH, int NCB>
static void launch_fam(const GenDev& g, int transpose, const double* R, int64_t ldr, double* out,
                       int64_t lds, int32_t ncols, int64_t kchunk, int nsplit, dim3 grid,
                       hipStream_t s) {
  if (transpose)
    hipLaunchKernelGGL((k_sample_f64<FAM, 1, NH, NCB>), grid, dim3(SM_T), 0, s, g, R, ldr, out, lds,
                       ncols, kchunk, nsplit);
  else
    hipLaunchKernelGGL((k_sample_f64<FAM, 0, NH, NCB>), grid, dim3(SM_T), 0, s, g, R, ldr, out, lds,
                       ncols, kchunk, nsplit);
}

template <int FAM>
static void launch_fam(const GenDev& g, int transpose, const double* R, int64_t ldr, double* out,
                       int64_t lds, int32_t ncols, int64_t kchunk, int nsplit, dim3 grid,
                       SampleTile t, hipStream_t s) {
  if constexpr (FAM == HSS_FAM_TOEPLITZ) {
    // the entries are symmetric: the transposed product is the same one
    if (g.perm_id) {
      if (t.cols == SM_COLS_W)
        launch_fam<kFamToeplitzWindow, 2, 8>(g, 0, R, ldr, out, lds, ncols, kchunk, nsplit, grid, s);
      else
        launch_fam<kFamToeplitzWindow, 2, 4>(g, 0, R, ldr, out, lds, ncols, kchunk, nsplit, grid, s);
      return;
    }
    if (t.cols == SM_COLS_W) {
      launch_fam<FAM, 2, 8>(g, transpose, R, ldr, out, lds, ncols, kchunk, nsplit, grid, s);
      return;
    }
  }
  if constexpr (FAM == HSS_FAM_GAUSS) {
    if (t.cols == SM_COLS_W) {
      launch_fam<FAM, 1, 8>(g, transpose, R, ldr, out, lds, ncols, kchunk, nsplit, grid, s);
      return;
    }
  }
  launch_fam<FAM, 2, 4>(g, transpose, R, ldr, out, lds, ncols, kchunk, nsplit, grid, s);
}

void launch_sample_lp(const GenDev& g, int32_t transpose, int32_t bf16x3, const double* R, int64_t ldr,
                      double* out, int64_t lds, int32_t ncols, int64_t kchunk, int32_t nz, dim3 grid,
                      const int32_t* leaf_lo, const int32_t* leaf_hi, int32_t offdiag, hipStream_t s);

// Dense matrices in HBM: A_hat R = P A P^T R is a plain GEMM between two
// row permutations, X = P^T R (X(perm(i), :) = R(i, :)), Y = op(A) X on
// the FP64 matrix cores, S(i, :) = Y(perm(i), :).  The entry-generating kernel would
// load every entry of A through the permutation inside its MFMA loop.
__global__ void k_perm_rows(const double* __restrict__ src, int64_t lds_, double* __restrict__ dst, int64_t ldd,
                            const int64_t* __restrict__ perm, int64_t n, int32_t ncols, int32_t scatter) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * ncols) return;
  const int64_t i = idx % n, c = idx / n;
  const int64_t p = perm[i];
  if (scatter) dst[c * ldd + p] = src[c * lds_ + i];
  else dst[c * ldd + i] = src[c * lds_ + p];
}

// Returns false when the workspace cannot hold one 64-column chunk of X and Y.
// The product Y = op(A) X is one task of the library's FP64 MFMA GEMM
// (k_gemm.hip): 64 x 64 output tiles, so with 64 columns every tile row
// streams its 64 rows of A from HBM once.
static bool sample_dense_gemm(const GenDev& g, int32_t transpose, const double* R, int64_t ldr, double* S,
                              int64_t lds, int32_t ncols, double* partial, hipStream_t s,
                              unsigned long long* kcnt) {
  const int64_t n = g.n;
  const int64_t cap = (int64_t)sample_partial_elems(n, ncols);   // at most what the caller allocated
  constexpr int64_t kTaskElems = 32;                              // room for the GEMM task at the end
  const int64_t chunk = partial ? std::min<int64_t>(ncols, (cap - kTaskElems) / (2 * n) / 64 * 64) : 0;
  if (chunk < std::min<int64_t>(ncols, 64)) return false;
  double* X = partial;
  double* Y = partial + n * chunk;
  GemmTask* task = reinterpret_cast<GemmTask*>(partial + 2 * n * chunk);
  static_assert(sizeof(GemmTask) <= kTaskElems * sizeof(double), "GEMM task does not fit its slot");
  for (int64_t c0 = 0; c0 < ncols; c0 += chunk) {
    const int32_t c = (int32_t)std::min<int64_t>(chunk, ncols - c0);
    const unsigned blocks = (unsigned)((n * c + 255) / 256);
    hipLaunchKernelGGL(k_perm_rows, dim3(blocks), dim3(256), 0, s, R + c0 * ldr, ldr, X, n, g.perm, n, c, 1);
    GemmTask t;
    t.A = g.dense;
    t.a_rs = transpose ? g.ld : 1;
    t.a_cs = transpose ? 1 : g.ld;
    t.B = X; t.b_rs = 1; t.b_cs = n;
    t.C = Y; t.c_rs = 1; t.c_cs = n;
    t.M = (int32_t)n; t.N = c; t.K = (int32_t)n; t.pad = 0;
    t.alpha = 1.0; t.beta = 0.0;
    HSS_HIP_CHECK(hipMemcpyAsync(task, &t, sizeof(t), hipMemcpyHostToDevice, s));
    HSS_HIP_CHECK(hipStreamSynchronize(s));   // the host struct is gone after this scope
    launch_gemm(task, 1, (int32_t)n, c, s, nullptr, 0, nullptr, 0, HSS_K_SAMPLE);
    hipLaunchKernelGGL(k_perm_rows, dim3(blocks), dim3(256), 0, s, Y, n, S + c0 * lds, lds, g.perm, n, c, 0);
  }
  return true;
}

void launch_sample(const GenDev& g, int32_t transpose, int32_t precision, const double* R,
                   int64_t ldr, double* S, int64_t lds, int32_t ncols, double* partial,
                   hipStream_t s, unsigned long long* kcnt) {
  if (ncols <= 0 || g.n <= 0) return;
  if (precision == HSS_SAMPLE_FP64 && g.family == HSS_FAM_DENSE &&
      sample_dense_gemm(g, transpose, R, ldr, S, lds, ncols, partial, s, kcnt))
    return;
  const int64_t n = g.n;
  const SampleTile tile = sample_tile(precision, g.family, n, ncols);
  const int nsplit = sample_splits(n, ncols, tile);
  int64_t kchunk = (n + nsplit - 1) / nsplit;
  kchunk = (kchunk + SM_BK - 1) / SM_BK * SM_BK;
  const int nz = (int)((n + kchunk - 1) / kchunk);
  dim3 grid((unsigned)((n + tile.rows - 1) / tile.rows), (unsigned)((ncols + tile.cols - 1) / tile.cols),
            (unsigned)nz);
  double* out = nz == 1 ? S : partial;
  prof_begin(s);
  if (precision != HSS_SAMPLE_FP64)
    launch_sample_lp(g, transpose, precision == HSS_SAMPLE_BF16X3, R, ldr, out, lds, ncols, kchunk, nz, grid,
                     g.leaf_lo, g.leaf_hi, g.offdiag, s);
  else switch (g.family) {
    case HSS_FAM_TOEPLITZ: launch_fam<HSS_FAM_TOEPLITZ>(g, transpose, R, ldr, out, lds, ncols, kchunk, nz, grid, tile, s); break;
    case HSS_FAM_LAPLACE: launch_fam<HSS_FAM_LAPLACE>(g, transpose, R, ldr, out, lds, ncols, kchunk, nz, grid, tile, s); break;
    case HSS_FAM_GAUSS: launch_fam<HSS_FAM_GAUSS>(g, transpose, R, ldr, out, lds, ncols, kchunk, nz, grid, tile, s); break;
    default: launch_fam<HSS_FAM_DENSE>(g, transpose, R, ldr, out, lds, ncols, kchunk, nz, grid, tile, s); break;
  }
  prof_end(HSS_K_SAMPLE, s);
  if (nz > 1) {
    const int64_t ncp = (int64_t)grid.y * tile.cols;
    const int64_t tot = n * ncols;
    prof_begin(s);
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       partial, n, ncols, ncp, nz, S, lds);
    prof_end(HSS_K_SAMPLE_REDUCE, s);
  }
}

}  // namespace hss
