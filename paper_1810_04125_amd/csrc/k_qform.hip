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

// M = S^{-1} V_1^T (b x b; S and V_1^T are upper triangular, so is M).
// For b <= QF_LDS_B: right-looking back substitution over the whole
// workgroup, M and G in LDS, rows of M final from the bottom up; then the
// GEMM task Q_k -= V M.  Thread (row group pg, column j) updates column j
// of the rows pg, pg + QFS/64, ... of each step.  For wider blocks this
// kernel only lays out M = V_1^T (column-major) and the blocked solve below
// finishes it.
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
  const HSS_GLOBAL double* gW = gview(t.W);
  if (!in_lds) {
    // M(l, j) = V(j, l) for j >= l, else 0, column-major
    HSS_GLOBAL double* gM = gview_w(Mg);
    for (int j = threadIdx.x / 64; j < b; j += QFS / 64)
      for (int l = threadIdx.x & 63; l < b; l += 64) gM[(int64_t)j * b + l] = j >= l ? gW[(int64_t)l * t.ldw + j] : 0.0;
    return;
  }
  {
    // working copies: R row-major b x b, G column-major b x b
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
          Rl[idx] = j >= l ? rv[u] : 0.0;
          Gl[idx] = gv[u];
        }
      }
    }
  }
  __syncthreads();
  const int jl = threadIdx.x & 63, pg = threadIdx.x >> 6;
  for (int l = b - 1; l >= 0; --l) {
    // row l is final: divide by S_ll = G_ll / 2
    const double inv = 2.0 / Gl[l * b + l];
    for (int j = threadIdx.x; j < b; j += QFS) Rl[l * b + j] *= inv;
    __syncthreads();
    // rows p < l: R(p, :) -= S(p, l) R(l, :), S(p, l) = G(p, l); the rows of
    // a thread are unrolled so that their reads are in flight together
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
    __syncthreads();
  }
  // M column-major for the GEMM
  HSS_GLOBAL double* gM = gview_w(Mg);
  for (int idx = threadIdx.x; idx < b * b; idx += QFS) {
    const int l = idx / b, j = idx - l * b;
    gM[(int64_t)j * b + l] = Rl[idx];
  }
  if (threadIdx.x == 0) {
    GemmTask q;
    q.A = t.W; q.a_rs = 1; q.a_cs = t.ldw;   // V
    q.B = Mg; q.b_rs = 1; q.b_cs = b;        // M(l, j)
    q.C = t.Q; q.c_rs = 1; q.c_cs = t.ldq;
    q.M = t.m; q.N = b; q.K = b; q.pad = 0;
    q.alpha = -1.0; q.beta = 1.0;
    *g = q;
    const double bb = b;
    kcount(kcnt, HSS_K_QFORM, 8.0 * 2.0 * bb * bb, bb * bb * bb);
  }
}

// Blocked back substitution for the blocks wider than QF_LDS_B: diagonal
// block ib (rows i0 = 64 ib ... i1) of S M = V_1^T, every column of M on its
// own thread (the 64 x 64 block of S in LDS, the column's 64 entries in
// registers); the workgroup with blockIdx.y == 0 then writes the GEMM task
// of the update of the rows above, M(0:i0, i0:b) -= S(0:i0, i0:i1) M(i0:i1, i0:b)
// (into gu), and with ib == 0 the final task Q_k -= V M (into gf).
constexpr int QFD = 64;
__global__ __launch_bounds__(256) void k_qf_diag(const QformTask* __restrict__ tasks, int ib,
                                                 GemmTask* __restrict__ gu, GemmTask* __restrict__ gf,
                                                 unsigned long long* __restrict__ kcnt) {
  __shared__ double Sd[QFD][QFD + 1];
  const QformTask& t = tasks[blockIdx.x];
  const bool wide = t.active && t.wk && t.nc > QF_LDS_B;
  const int b = t.nc;
  const int i0 = ib * QFD;
  if (blockIdx.y == 0 && threadIdx.x == 0) gu[blockIdx.x].M = 0;
  if (!wide || i0 >= b) return;
  const int i1 = min(b, i0 + QFD), nb = i1 - i0;
  const double* G = t.wk;                        // b x b column-major
  double* M = t.wk + (int64_t)b * b;             // b x b column-major
  const HSS_GLOBAL double* gG = gview(G);
  for (int idx = threadIdx.x; idx < QFD * QFD; idx += 256) {
    const int r = idx % QFD, c = idx / QFD;
    double v = 0.0;
    if (r < nb && c < nb && r <= c) {
      v = gG[(int64_t)(i0 + c) * b + i0 + r];
      if (r == c) v *= 0.5;                      // S_ll = G_ll / 2
    }
    Sd[r][c] = v;
  }
  __syncthreads();
  const int j = i0 + blockIdx.y * 256 + threadIdx.x;   // columns j < i0 are zero in these rows
  if (j < b) {
    HSS_GLOBAL double* col = gview_w(M + (int64_t)j * b + i0);
    double x[QFD];
#pragma unroll
    for (int u = 0; u < QFD; ++u) x[u] = u < nb ? col[u] : 0.0;
#pragma unroll
    for (int l = QFD - 1; l >= 0; --l) {
      if (l < nb) {
        const double xl = x[l] / Sd[l][l];
        x[l] = xl;
#pragma unroll
        for (int p = 0; p < l; ++p) x[p] -= Sd[p][l] * xl;
      }
    }
#pragma unroll
    for (int u = 0; u < QFD; ++u)
      if (u < nb) col[u] = x[u];
  }
  if (blockIdx.y != 0 || threadIdx.x != 0) return;
  const double bb = b, nn = nb;
  kcount(kcnt, HSS_K_QFORM, 16.0 * nn * bb, nn * nn * bb);
  if (i0 > 0) {
    GemmTask q;
    q.A = G + (int64_t)i0 * b; q.a_rs = 1; q.a_cs = b;   // S(0:i0, i0:i1) = G(0:i0, i0:i1)
    q.B = M + (int64_t)i0 * b + i0; q.b_rs = 1; q.b_cs = b;   // M(i0:i1, i0:b); its columns < i0 are zero
    q.C = M + (int64_t)i0 * b; q.c_rs = 1; q.c_cs = b;        // M(0:i0, i0:b)
    q.M = i0; q.N = b - i0; q.K = nb; q.pad = 0;
    q.alpha = -1.0; q.beta = 1.0;
    gu[blockIdx.x] = q;
  } else {
    GemmTask q;
    q.A = t.W; q.a_rs = 1; q.a_cs = t.ldw;               // V
    q.B = M; q.b_rs = 1; q.b_cs = b;                     // M(l, j), column-major
    q.C = t.Q; q.c_rs = 1; q.c_cs = t.ldq;
    q.M = t.m; q.N = b; q.K = b; q.pad = 0;
    q.alpha = -1.0; q.beta = 1.0;
    gf[blockIdx.x] = q;
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
  if (ncmax > QF_LDS_B) {
    // blocks of 64 rows from the bottom; updates on the matrix cores (their
    // tasks in the second half of gt, the final tasks stay in the first)
    const unsigned gy = (unsigned)((ncmax + 255) / 256);
    for (int ib = (ncmax + QFD - 1) / QFD - 1; ib >= 0; --ib) {
      prof_begin(s);
      hipLaunchKernelGGL(k_qf_diag, dim3((unsigned)count, gy), dim3(256), 0, s, tasks, ib, gt + count, gt, kcnt);
      prof_end(HSS_K_QFORM, s);
      if (ib > 0) launch_gemm(gt + count, count, ib * QFD, ncmax, s, kcnt, QFD, gws, kGemmSplitElems);
    }
  }
  launch_gemm(gt, count, mmax, ncmax, s, kcnt);
  if (nwg > 0) {
    prof_begin(s);
    hipLaunchKernelGGL(k_qform, dim3(nwg), dim3(QFB), 0, s, tasks, wg, cpw, kcnt);
    prof_end(HSS_K_QFORM, s);
  }
}

}  // namespace hss
