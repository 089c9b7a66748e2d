// Explicit Q_k of the stopping test (Alg. 5: the basis grows by the
// orthonormal factor of the projected block's QR).  The Householder QR
// leaves the reflectors H_k = I - tau_k v_k v_k^T in the panel (column k:
// v_k(k) = W(k,k) - rdiag[k], v_k(i) = W(i,k) below, tau_k = 2 / v_k^T v_k).
//
// Compact WY ("UT") form: H_0 ... H_{b-1} = I - V S^{-1} V^T with S the
// upper triangle of V^T V whose diagonal is halved (S_kk = 1 / tau_k), so
//     Q_k = [I; 0] - V (S^{-1} V_1^T),   V_1 = the top b x b block of V:
// one GEMM for V^T V, a b x b triangular solve, one GEMM for the update.
// Blocks too wide for the node's workspace fall back to forming each
// column j = H_0 ... H_j e_j on its own.
#include "hss_internal.h"

namespace hss {

namespace {
constexpr int QFB = 256;
constexpr int QFW = QFB / 64;

__device__ __forceinline__ double qf_wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
}  // namespace

// Column-by-column formation for the tasks without a workspace.
__global__ __launch_bounds__(QFB) void k_qform(const QformTask* __restrict__ tasks, const int2* __restrict__ wg,
                                               int cpw, unsigned long long* __restrict__ kcnt) {
  const int2 w = wg[blockIdx.x];
  const QformTask& t = tasks[w.x];
  if (!t.active || t.wk) return;
  const int m = t.m;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jend = min(t.nc, w.y + cpw);
  if (w.y == 0 && threadIdx.x == 0) {
    const double mm = m, b = t.nc;
    kcount(kcnt, HSS_K_QFORM, 8.0 * mm * b * 2.0, 2.0 * mm * b * b);
  }
  for (int j = w.y + wv; j < jend; j += QFW) {
    double* y = t.Q + (int64_t)j * t.ldq;
    for (int i = lane; i < m; i += 64) y[i] = (i == j) ? 1.0 : 0.0;
    for (int k = j; k >= 0; --k) {
      const double alpha = t.rdiag[k];
      const double nu = fabs(alpha);
      if (nu == 0.0) continue;
      const double* x = t.W + (int64_t)k * t.ldw;
      const double x0 = x[k];
      const double tk = 1.0 / (nu * (nu + fabs(x0)));
      double dot = 0.0;
      for (int i = k + lane; i < m; i += 64) dot += (i == k ? x0 - alpha : x[i]) * y[i];
      dot = qf_wsum(dot) * tk;
      for (int i = k + lane; i < m; i += 64) y[i] -= dot * (i == k ? x0 - alpha : x[i]);
    }
  }
}

// V over W (zeros above the diagonal, v_k(k) = W(k,k) - rdiag[k]),
// Q_k = [I; 0], and the GEMM task G = V^T V (b x b, in wk).
__global__ __launch_bounds__(QFB) void k_qf_prep(const QformTask* __restrict__ tasks, GemmTask* __restrict__ gt,
                                                 unsigned long long* __restrict__ kcnt) {
  const QformTask& t = tasks[blockIdx.x];
  GemmTask* g = gt + blockIdx.x;
  const bool on = t.active && t.wk;
  if (blockIdx.y == 0 && threadIdx.x == 0) {
    g->M = 0;
    if (on) {
      GemmTask q;
      q.A = t.W; q.a_rs = t.ldw; q.a_cs = 1;   // V^T
      q.B = t.W; q.b_rs = 1; q.b_cs = t.ldw;   // V
      q.C = t.wk; q.c_rs = 1; q.c_cs = t.nc;
      q.M = t.nc; q.N = t.nc; q.K = t.m; q.pad = 0;
      q.alpha = 1.0; q.beta = 0.0;
      *g = q;
      const double mm = t.m, b = t.nc;
      kcount(kcnt, HSS_K_QFORM, 8.0 * mm * b * 3.0, 0.0);
    }
  }
  if (!on) return;
  const int m = t.m;
  const int64_t tot = (int64_t)m * t.nc;
  for (int64_t idx = threadIdx.x + (int64_t)blockIdx.y * QFB; idx < tot; idx += (int64_t)QFB * gridDim.y) {
    const int i = (int)(idx % m), k = (int)(idx / m);
    double* w = t.W + (int64_t)k * t.ldw + i;
    const double x = *w;
    *w = i < k ? 0.0 : (i == k ? x - t.rdiag[k] : x);
    t.Q[(int64_t)k * t.ldq + i] = (i == k) ? 1.0 : 0.0;
  }
}

// M = S^{-1} V_1^T (b x b) by right-looking back substitution over the
// whole workgroup (rows of M become final from the bottom up), held in LDS
// with G for b <= QF_LDS_B and in the workspace otherwise; then the GEMM
// task Q_k -= V M.  Thread (row group pg, column j) updates column j of the
// rows pg, pg + QFS/64, ... of each step.
constexpr int QFS = 1024;
constexpr int QF_LDS_B = 64;
constexpr int QF_RG = QFS / 64;   // row groups

__global__ __launch_bounds__(QFS) void k_qf_solve(const QformTask* __restrict__ tasks, GemmTask* __restrict__ gt,
                                                  unsigned long long* __restrict__ kcnt) {
  __shared__ double Rl[QF_LDS_B * QF_LDS_B];
  __shared__ double Gl[QF_LDS_B * QF_LDS_B];
  const QformTask& t = tasks[blockIdx.x];
  GemmTask* g = gt + blockIdx.x;
  if (threadIdx.x == 0) g->M = 0;
  if (!t.active || !t.wk) return;
  const int b = t.nc;
  const bool in_lds = b <= QF_LDS_B;
  double* Mg = t.wk + (int64_t)b * b;          // M, b x b column-major
  // working copies: R row-major b x b, G column-major b x b
  double* R = in_lds ? Rl : Mg;
  const double* G = in_lds ? Gl : t.wk;
  {
    const HSS_GLOBAL double* gW = gview(t.W);
    const HSS_GLOBAL double* gG = gview(t.wk);
    constexpr int LU = 4;
    const int tot = b * b;
    for (int base = threadIdx.x; base < tot; base += QFS * LU) {
      double rv[LU], gv[LU];
#pragma unroll
      for (int u = 0; u < LU; ++u) {
        const int idx = min(base + u * QFS, tot - 1);
        const int l = idx / b, j = idx - l * b;
        rv[u] = gW[(int64_t)l * t.ldw + j];   // R(l, j) = V(j, l), zero for j < l
        gv[u] = gG[idx];
      }
#pragma unroll
      for (int u = 0; u < LU; ++u) {
        const int idx = base + u * QFS;
        if (idx < tot) {
          const int l = idx / b, j = idx - l * b;
          R[idx] = j >= l ? rv[u] : 0.0;
          if (in_lds) Gl[idx] = gv[u];
        }
      }
    }
  }
  __syncthreads();
  const int jl = threadIdx.x & 63, pg = threadIdx.x >> 6;
  for (int l = b - 1; l >= 0; --l) {
    // row l is final: divide by S_ll = G_ll / 2
    const double inv = 2.0 / G[(int64_t)l * b + l];
    for (int j = threadIdx.x; j < b; j += QFS) R[l * b + j] *= inv;
    __syncthreads();
    // rows p < l: R(p, :) -= S(p, l) R(l, :), S(p, l) = G(p, l); in LDS the
    // rows of a thread are unrolled so that their reads are in flight together
    if (in_lds) {
      if (jl < b) {
        const double rl = Rl[l * b + jl];
#pragma unroll
        for (int u = 0; u < QF_LDS_B / QF_RG; ++u) {
          const int p = pg + QF_RG * u;
          const int pc = min(p, QF_LDS_B - 1);
          const double v = Rl[pc * b + jl] - Gl[l * b + pc] * rl;
          if (p < l) Rl[pc * b + jl] = v;
        }
      }
    } else {
      for (int j = jl; j < b; j += 64)
        for (int p = pg; p < l; p += QF_RG) R[p * b + j] -= G[(int64_t)l * b + p] * R[l * b + j];
    }
    __syncthreads();
  }
  // M column-major for the GEMM
  if (in_lds) {
    HSS_GLOBAL double* gM = gview_w(Mg);
    for (int idx = threadIdx.x; idx < b * b; idx += QFS) {
      const int l = idx / b, j = idx - l * b;
      gM[(int64_t)j * b + l] = Rl[idx];
    }
  }
  if (threadIdx.x == 0) {
    GemmTask q;
    q.A = t.W; q.a_rs = 1; q.a_cs = t.ldw;   // V
    q.B = Mg;
    if (in_lds) { q.b_rs = 1; q.b_cs = b; } else { q.b_rs = b; q.b_cs = 1; }   // M(l, j)
    q.C = t.Q; q.c_rs = 1; q.c_cs = t.ldq;
    q.M = t.m; q.N = b; q.K = b; q.pad = 0;
    q.alpha = -1.0; q.beta = 1.0;
    *g = q;
    const double bb = b;
    kcount(kcnt, HSS_K_QFORM, 8.0 * 2.0 * bb * bb, bb * bb * bb);
  }
}

void run_qform(QformTask* tasks, int32_t count, const int2* wg, int32_t nwg, int32_t cpw, int32_t ncmax,
               int32_t mmax, GemmTask* gt, double* gws, hipStream_t s, unsigned long long* kcnt) {
  if (count <= 0 || ncmax <= 0) return;
  const int64_t cells = (int64_t)std::max(mmax, 1) * ncmax;
  const unsigned chunks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (cells + 4095) / 4096));
  prof_begin(s);
  hipLaunchKernelGGL(k_qf_prep, dim3((unsigned)count, chunks), dim3(QFB), 0, s, tasks, gt, kcnt);
  prof_end(HSS_K_QFORM, s);
  launch_gemm(gt, count, ncmax, ncmax, s, kcnt, mmax, gws, kGemmSplitElems);
  prof_begin(s);
  hipLaunchKernelGGL(k_qf_solve, dim3((unsigned)count), dim3(QFS), 0, s, tasks, gt, kcnt);
  prof_end(HSS_K_QFORM, s);
  launch_gemm(gt, count, mmax, ncmax, s, kcnt);
  if (nwg > 0) {
    prof_begin(s);
    hipLaunchKernelGGL(k_qform, dim3(nwg), dim3(QFB), 0, s, tasks, wg, cpw, kcnt);
    prof_end(HSS_K_QFORM, s);
  }
}

}  // namespace hss
