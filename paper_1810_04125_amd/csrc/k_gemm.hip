// Grouped FP64 GEMM on the matrix cores for the per-level dense
// contractions of the compression: local samples (D R, B R; Alg. 2), the
// block Gram-Schmidt projections of the stopping test ((I - Q Q^T)^2 S;
// Alg. 5) and the reduced random matrices (x(J) + E x(rest); Alg. 2).
//
// Every task has its own pointers, strides and sizes (sizes are written
// by device kernels, since ranks live on the GPU).  blockIdx.z selects
// the task, blockIdx.y/x the 64 x 64 output tile; tiles outside a task's
// actual size exit at once.  4 waves per workgroup, each a 32 x 32 block
// of 2 x 2 MFMA 16x16x4 FP64 tiles; A and B tiles are staged in LDS.
#include "hss_internal.h"

namespace hss {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;   // output tile
constexpr int GK = 16;   // K tile
constexpr int GLD = GT + 2;

__global__ __launch_bounds__(256) void k_gemm_grouped(const GemmTask* __restrict__ tasks,
                                                     unsigned long long* __restrict__ kcnt) {
  const GemmTask t = tasks[blockIdx.z];
  const int tm = blockIdx.y, tn = blockIdx.x;
  if (t.M <= 0 || t.N <= 0) return;
  if (tm == 0 && tn == 0 && threadIdx.x == 0) {
    const double M = t.M, N = t.N, K = t.K;
    kcount(kcnt, HSS_K_GEMM, 8.0 * (M * K + K * N + M * N * (t.beta == 0.0 ? 1.0 : 2.0)), 2.0 * M * N * K);
  }
  if (tm * GT >= t.M || tn * GT >= t.N) return;
  __shared__ double As[GK][GLD];
  __shared__ double Bs[GK][GLD];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int64_t i0 = (int64_t)tm * GT, j0 = (int64_t)tn * GT;
  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < t.K; k0 += GK) {
    for (int idx = threadIdx.x; idx < GK * GT; idx += 256) {
      // A tile: As[k][i]; make the faster index follow the smaller stride
      int k, i;
      if (t.a_rs <= t.a_cs) { i = idx % GT; k = idx / GT; } else { k = idx % GK; i = idx / GK; }
      const int64_t gi = i0 + i, gk = k0 + k;
      double av = 0.0;
      if (gi < t.M && gk < t.K) {
        const int64_t col = t.a_cols ? (int64_t)t.a_cols[gk] : gk;
        av = t.A[gi * t.a_rs + col * t.a_cs];
      }
      As[k][i] = av;
      int kb, j;
      if (t.b_cs <= t.b_rs) { j = idx % GT; kb = idx / GT; } else { kb = idx % GK; j = idx / GK; }
      const int64_t gj = j0 + j, gkb = k0 + kb;
      Bs[kb][j] = (gj < t.N && gkb < t.K) ? t.B[gkb * t.b_rs + gj * t.b_cs] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
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
        double* c = t.C + gi * t.c_rs + gj * t.c_cs;
        const double val = t.alpha * acc[a][b][v];
        *c = (t.beta == 0.0) ? val : val + t.beta * (*c);
      }
}

void launch_gemm(const GemmTask* tasks, int32_t ntasks, int32_t mcap, int32_t ncap, hipStream_t s,
                 unsigned long long* kcnt) {
  if (ntasks <= 0 || mcap <= 0 || ncap <= 0) return;
  dim3 grid((unsigned)((ncap + GT - 1) / GT), (unsigned)((mcap + GT - 1) / GT), (unsigned)ntasks);
  prof_begin(s);
  hipLaunchKernelGGL(k_gemm_grouped, grid, dim3(256), 0, s, tasks, kcnt);
  prof_end(HSS_K_GEMM, s);
}

}  // namespace hss
