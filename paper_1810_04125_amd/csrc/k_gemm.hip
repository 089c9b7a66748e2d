// Grouped FP64 GEMM on the matrix cores for the per-level dense
// contractions of the compression: local samples (D R, B R; Alg. 2), the
// block Gram-Schmidt projections of the stopping test ((I - Q Q^T)^2 S;
// Alg. 5) and the reduced random matrices (x(J) + E x(rest); Alg. 2).
//
// Every task has its own pointers, strides and sizes (sizes are written
// by device kernels, since ranks live on the GPU).  blockIdx.z selects
// the task and the K slice, blockIdx.y/x the 64 x 64 output tile; tiles
// outside a task's actual size exit at once.  4 waves per workgroup, each
// a 32 x 32 block of 2 x 2 MFMA 16x16x4 FP64 tiles; A and B tiles of 32
// k-columns are staged in LDS, the next ones loaded into registers while
// the current ones are multiplied.
//
// Split K: products with few output tiles and a long K (the Gram-Schmidt
// projections against a large basis at the top of the tree) cut K into
// `ksplit` slices; each slice writes its 64 x 64 partial tile to a
// workspace and a second kernel adds the slices in slice order, so the
// result does not depend on scheduling.
#include "hss_internal.h"

namespace hss {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;   // output tile (square shape)
constexpr int GK = 32;   // K tile (square shape)
constexpr int GTILE = GT * GT;   // output elements of a tile, either shape

// Tile shapes: 64 x 64 with K tiles of 32 (the 4 waves 2 x 2), or, for
// products of at most 32 rows (the block ID's V^T A with one row per
// pivot), 32 x 128 with K tiles of 16 (the 4 waves side by side), so no
// matrix-core work goes to rows that do not exist.  Both keep 8 elements
// of each operand tile per thread.
template <int TM>
struct GemmShape {
  static constexpr int TN = GTILE / TM;
  static constexpr int KT = TM == 64 ? 32 : 16;
  static constexpr int APT = KT * TM / 256;   // A-tile elements per thread
  static constexpr int BPT = KT * TN / 256;   // B-tile elements per thread
  static constexpr int WPR = TN / 32;         // waves along a tile row
};

template <int TM>
__device__ __forceinline__ void gemm_coords(const GemmTask& t, int idx, bool a_side, int& k, int& x) {
  using S = GemmShape<TM>;
  // make the faster index follow the smaller stride
  if (a_side) {
    if (t.a_rs <= t.a_cs) { x = idx % TM; k = idx / TM; } else { k = idx % S::KT; x = idx / S::KT; }
  } else {
    if (t.b_cs <= t.b_rs) { x = idx % S::TN; k = idx / S::TN; } else { k = idx % S::KT; x = idx / S::KT; }
  }
}

template <int TM>
__global__ __launch_bounds__(256, 3) void k_gemm_grouped(const GemmTask* __restrict__ tasks, int ntasks, int ksplit,
                                                     double* __restrict__ part,
                                                     unsigned long long* __restrict__ kcnt) {
  using S = GemmShape<TM>;
  constexpr int TN = S::TN, KT = S::KT, APT = S::APT, BPT = S::BPT;
  static_assert(APT <= 16 && BPT <= 16, "valid-bit mask");
  const int task = blockIdx.z % ntasks, ks = blockIdx.z / ntasks;
  const GemmTask t = tasks[task];
  const int tm = blockIdx.y, tn = blockIdx.x;
  if (t.M <= 0 || t.N <= 0) return;
  if (ks == 0 && tm == 0 && tn == 0 && threadIdx.x == 0) {
    const double M = t.M, N = t.N, K = t.K;
    kcount(kcnt, HSS_K_GEMM, 8.0 * (M * K + K * N + M * N * (t.beta == 0.0 ? 1.0 : 2.0)), 2.0 * M * N * K);
  }
  if (tm * TM >= t.M || tn * TN >= t.N) return;
  __shared__ double As[KT][TM + 2];
  __shared__ double Bs[KT][TN + 2];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = (wave / S::WPR) * 32, wc = (wave % S::WPR) * 32;
  const int64_t i0 = (int64_t)tm * TM, j0 = (int64_t)tn * TN;
  // K slice of this workgroup
  int kb = 0, ke = t.K;
  if (ksplit > 1) {
    const int kchunk = ((t.K + ksplit - 1) / ksplit + KT - 1) / KT * KT;
    kb = min(t.K, ks * kchunk);
    ke = min(t.K, kb + kchunk);
  }
  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

  // Operand elements of a K tile, loaded without branches from clamped
  // indices: the column indices of a gathered A as one batch of loads, then
  // all values as another; the elements outside the operands are recorded
  // in a bit mask and written to LDS as 0.
  const HSS_GLOBAL double* gA = gview(t.A);
  const HSS_GLOBAL double* gB = gview(t.B);
  const HSS_GLOBAL int32_t* gcols = t.a_cols ? gview(t.a_cols) : nullptr;
  const HSS_GLOBAL int32_t* gbcols = t.b_cols ? gview(t.b_cols) : nullptr;
  // physical columns of B of this thread's elements (fixed over K)
  int64_t bcol[BPT];
#pragma unroll
  for (int e = 0; e < BPT; ++e) {
    int kk, j;
    gemm_coords<TM>(t, threadIdx.x + 256 * e, false, kk, j);
    const int64_t gj = min(j0 + j, (int64_t)t.N - 1);
    bcol[e] = gbcols ? (int64_t)gbcols[gj] : gj;
  }
  double ra[APT], rb[BPT];
  uint32_t valid = 0;
  auto load = [&](int k0) {
    int64_t col[APT];
#pragma unroll
    for (int e = 0; e < APT; ++e) {
      int k, i;
      gemm_coords<TM>(t, threadIdx.x + 256 * e, true, k, i);
      const int gk = min(k0 + k, ke - 1);
      col[e] = gcols ? (int64_t)gcols[gk] : (int64_t)gk;
    }
    valid = 0;
#pragma unroll
    for (int e = 0; e < APT; ++e) {
      int k, i;
      gemm_coords<TM>(t, threadIdx.x + 256 * e, true, k, i);
      const int64_t gi = i0 + i, gk = k0 + k;
      ra[e] = gA[min(gi, (int64_t)t.M - 1) * t.a_rs + col[e] * t.a_cs];
      valid |= (uint32_t)(gi < t.M && gk < ke) << e;
    }
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
      int kk, j;
      gemm_coords<TM>(t, threadIdx.x + 256 * e, false, kk, j);
      const int64_t gj = j0 + j, gkb = k0 + kk;
      rb[e] = gB[min(gkb, (int64_t)ke - 1) * t.b_rs + bcol[e] * t.b_cs];
      valid |= (uint32_t)(gj < t.N && gkb < ke) << (APT + e);
    }
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += KT) {
#pragma unroll
    for (int e = 0; e < APT; ++e) {
      int k, x;
      gemm_coords<TM>(t, threadIdx.x + 256 * e, true, k, x);
      As[k][x] = (valid >> e) & 1u ? ra[e] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
      int k, x;
      gemm_coords<TM>(t, threadIdx.x + 256 * e, false, k, x);
      Bs[k][x] = (valid >> (APT + e)) & 1u ? rb[e] : 0.0;
    }
    __syncthreads();
    if (k0 + KT < ke) load(k0 + KT);
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const int kq = kk + (lane >> 4);
      const double a0 = As[kq][wr + (lane & 15)];
      const double a1 = As[kq][wr + 16 + (lane & 15)];
      const double b0 = Bs[kq][wc + (lane & 15)];
      const double b1 = Bs[kq][wc + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  if (ksplit > 1) {
    // raw partial tile, row-major TM x TN, slot (ks, task, tm, tn)
    double* P = part + ((((int64_t)ks * ntasks + task) * gridDim.y + tm) * gridDim.x + tn) * GTILE;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          P[(wr + a * 16 + 4 * v + (lane >> 4)) * TN + wc + b * 16 + (lane & 15)] = acc[a][b][v];
    return;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // FP64 16x16x4 result layout: row 4*v + lane/16, column lane % 16
        const int64_t gi = i0 + wr + a * 16 + 4 * v + (lane >> 4);
        const int64_t gj = j0 + wc + b * 16 + (lane & 15);
        if (gi >= t.M || gj >= t.N) continue;
        const int64_t cj = t.c_cols ? (int64_t)t.c_cols[gj] : gj;
        HSS_GLOBAL double* c = gview_w(t.C + gi * t.c_rs + cj * t.c_cs);
        const double val = t.alpha * acc[a][b][v];
        *c = (t.beta == 0.0) ? val : val + t.beta * (*c);
      }
}

// C = alpha * (sum of the K-slice partials, in slice order) + beta * C.
// blockIdx.z = task * SUM_SPLIT + part: each workgroup adds one 256-element
// part of a tile, a thread one element, loading SUM_U slices at once.
constexpr int SUM_SPLIT = GTILE / 256;
constexpr int SUM_U = 8;
template <int TM>
__global__ __launch_bounds__(256) void k_gemm_splitk_sum(const GemmTask* __restrict__ tasks, int ntasks, int ksplit,
                                                        const double* __restrict__ part) {
  constexpr int TN = GemmShape<TM>::TN;
  const int task = blockIdx.z / SUM_SPLIT, piece = blockIdx.z % SUM_SPLIT;
  const GemmTask t = tasks[task];
  const int tm = blockIdx.y, tn = blockIdx.x;
  if (t.M <= 0 || t.N <= 0 || tm * TM >= t.M || tn * TN >= t.N) return;
  const int e = piece * 256 + threadIdx.x;
  const int r = e / TN, c = e % TN;
  const int64_t gi = (int64_t)tm * TM + r, gj = (int64_t)tn * TN + c;
  if (gi >= t.M || gj >= t.N) return;
  const int64_t tile = (((int64_t)task * gridDim.y + tm) * gridDim.x + tn) * GTILE;
  const int64_t stride = (int64_t)ntasks * gridDim.y * gridDim.x * GTILE;
  double sum = 0.0;
  for (int k0 = 0; k0 < ksplit; k0 += SUM_U) {
    double v[SUM_U];
#pragma unroll
    for (int u = 0; u < SUM_U; ++u) v[u] = part[min(k0 + u, ksplit - 1) * stride + tile + e];
#pragma unroll
    for (int u = 0; u < SUM_U; ++u)
      if (k0 + u < ksplit) sum += v[u];
  }
  const int64_t cj = t.c_cols ? (int64_t)t.c_cols[gj] : gj;
  HSS_GLOBAL double* cp = gview_w(t.C + gi * t.c_rs + cj * t.c_cs);
  const double val = t.alpha * sum;
  *cp = (t.beta == 0.0) ? val : val + t.beta * (*cp);
}

template <int TM>
static void launch_gemm_shape(const GemmTask* tasks, int32_t ntasks, int32_t mcap, int32_t ncap, hipStream_t s,
                              unsigned long long* kcnt, int32_t kcap, double* ws, int64_t ws_elems) {
  constexpr int TN = GemmShape<TM>::TN;
  const unsigned gx = (unsigned)((ncap + TN - 1) / TN), gy = (unsigned)((mcap + TM - 1) / TM);
  const int64_t tiles = (int64_t)gx * gy * ntasks;
  // split K until about tune().gemm_wg (2048) workgroups are busy, K slices
  // of at least 128 rows, at most tune().gemm_max_split, within the workspace
  const int64_t target = tune().gemm_wg, maxsplit = tune().gemm_max_split;
  int ksplit = 1;
  if (ws && kcap >= 8 * GK && tiles < target) {
    ksplit = (int)std::min<int64_t>(std::min<int64_t>(maxsplit, kcap / (4 * GK)), std::max<int64_t>(1, target / tiles));
    while (ksplit > 1 && (int64_t)ksplit * tiles * GTILE > ws_elems) --ksplit;
  }
  if (ksplit == 1) {
    // grid z is at most 65535: very large batches go in several launches
    constexpr int kMaxZ = 65535;
    for (int t0 = 0; t0 < ntasks; t0 += kMaxZ) {
      const int nt = std::min(kMaxZ, ntasks - t0);
      hipLaunchKernelGGL(k_gemm_grouped<TM>, dim3(gx, gy, (unsigned)nt), dim3(256), 0, s, tasks + t0, nt, 1, ws,
                         kcnt);
    }
  } else {
    hipLaunchKernelGGL(k_gemm_grouped<TM>, dim3(gx, gy, (unsigned)(ntasks * ksplit)), dim3(256), 0, s, tasks, ntasks,
                       ksplit, ws, kcnt);
    hipLaunchKernelGGL(k_gemm_splitk_sum<TM>, dim3(gx, gy, (unsigned)(ntasks * SUM_SPLIT)), dim3(256), 0, s, tasks,
                       ntasks, ksplit, ws);
  }
}

void launch_gemm(const GemmTask* tasks, int32_t ntasks, int32_t mcap, int32_t ncap, hipStream_t s,
                 unsigned long long* kcnt, int32_t kcap, double* ws, int64_t ws_elems, int cls) {
  if (ntasks <= 0 || mcap <= 0 || ncap <= 0) return;
  prof_begin(s);
  if (mcap <= 32) launch_gemm_shape<32>(tasks, ntasks, mcap, ncap, s, kcnt, kcap, ws, ws_elems);
  else launch_gemm_shape<64>(tasks, ntasks, mcap, ncap, s, kcnt, kcap, ws, ws_elems);
  prof_end(cls, s);
}

}  // namespace hss
