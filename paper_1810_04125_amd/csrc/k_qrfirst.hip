// QR first for tall panels of the interpolative decomposition.
//
// The ID factors the panel W = S^T (d x m, d samples, m rows of the local
// sample) with column pivoting (eqs. ID, QRCPSr).  When d >= 2 m, W is first
// reduced to its m x m triangle R by a blocked Householder QR without
// pivoting (W = Q R); the pivoted factorization then runs on R.  Column
// norms, and so the pivots, the ranks and E = R11^{-1} R12, are unchanged
// by the orthogonal Q: the result is the ID of S up to rounding, but each
// pivot step touches an m x m panel instead of a d x m one.
//
// Blocks of NBQ columns: one workgroup factors the block's columns (their
// rows c..d-1) with Householder reflectors, kept as V (zero above the
// diagonal); the trailing columns are updated on the matrix cores in the
// compact WY form H_c ... H_{c+nb-1} = I - V S^{-1} V^T, S the upper
// triangle of V^T V with its diagonal halved:
//     A <- A - V (S^{-T} (V^T A)).
#include "hss_internal.h"

namespace hss {

namespace {
constexpr int NBQ = 32;
constexpr int QRF_T = 1024;

struct QrfPtrs {
  double *alpha, *tau, *G, *X, *W2, *W3, *V;
  int64_t ldv;
};

__device__ __forceinline__ int64_t qrf_need(const QrcpTask& t) {
  return 2 * (int64_t)t.mcap + 2 * NBQ * NBQ + 2 * (int64_t)NBQ * t.mcap + (int64_t)t.d * NBQ + 64;
}

__device__ __forceinline__ bool qrf_tall(const QrcpTask& t) {
  return t.active && t.hmt_mn == 0.0 && !t.nopivot && t.qrf && t.m >= 64 && t.d >= 2 * t.m &&
         t.qrf_elems >= qrf_need(t);
}

__device__ __forceinline__ QrfPtrs qrf_ptrs(const QrcpTask& t) {
  QrfPtrs p;
  p.alpha = t.qrf;
  p.tau = p.alpha + t.mcap;
  p.G = p.tau + t.mcap;
  p.X = p.G + NBQ * NBQ;
  p.W2 = p.X + NBQ * NBQ;
  p.W3 = p.W2 + (int64_t)NBQ * t.mcap;
  p.V = p.W3 + (int64_t)NBQ * t.mcap;
  p.ldv = t.d;
  return p;
}

__device__ __forceinline__ double qrf_wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
}  // namespace

// out[0]: the largest m among the tall panels; out[1]: the cells the
// reduction takes out of the first pivot step, (d - m) m summed over them;
// out[2]: the number of active panels.  One workgroup; writes its result
// directly (out may be mapped host memory).
constexpr int QRS = 1024;
__global__ __launch_bounds__(QRS) void k_qrf_scan(const QrcpTask* __restrict__ tasks, int ntasks,
                                                 int64_t* __restrict__ out) {
  __shared__ int64_t s0[QRS / 64], s1[QRS / 64], s2[QRS / 64];
  int64_t mt = 0, cells = 0, act = 0;
  for (int i = threadIdx.x; i < ntasks; i += QRS) {
    const QrcpTask& t = tasks[i];
    act += t.active ? 1 : 0;
    if (qrf_tall(t)) {
      mt = max(mt, (int64_t)t.m);
      cells += (int64_t)(t.d - t.m) * t.m;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mt = max(mt, (int64_t)__shfl_xor(mt, o, 64));
    cells += __shfl_xor(cells, o, 64);
    act += __shfl_xor(act, o, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { s0[wv] = mt; s1[wv] = cells; s2[wv] = act; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t a = 0, b = 0, c = 0;
    for (int w = 0; w < QRS / 64; ++w) { a = max(a, s0[w]); b += s1[w]; c += s2[w]; }
    out[0] = a;
    out[1] = b;
    out[2] = c;
  }
}

// Pinned, device-mapped host words for the scan's result.
static int64_t* scan_words(int64_t** dev) {
  thread_local int64_t* p = nullptr;
  thread_local int64_t* d = nullptr;
  if (!p) {
    HSS_HIP_CHECK(hipHostMalloc((void**)&p, 64, hipHostMallocMapped | hipHostMallocPortable));
    HSS_HIP_CHECK(hipHostGetDevicePointer((void**)&d, p, 0));
  }
  *dev = d;
  return p;
}

// Householder factorization of columns [c, c1) over rows c..d-1, one
// workgroup per tall panel; V, alpha (the diagonal of R) and tau kept; the
// GEMM task G = V^T V.
__global__ __launch_bounds__(QRF_T) void k_qrf_panel(const QrcpTask* __restrict__ tasks, int c,
                                                    GemmTask* __restrict__ gt,
                                                    unsigned long long* __restrict__ kcnt) {
  __shared__ double red[QRF_T / 64];
  __shared__ double part[QRF_T / 64][NBQ];
  __shared__ double dots[NBQ];
  const QrcpTask& t = tasks[blockIdx.x];
  GemmTask* g = gt + blockIdx.x;
  if (threadIdx.x == 0) g->M = 0;
  if (!qrf_tall(t) || c >= t.m) return;
  const int m = t.m, d = t.d, c1 = min(m, c + NBQ);
  const QrfPtrs P = qrf_ptrs(t);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int NW = QRF_T / 64;
  for (int k = c; k < c1; ++k) {
    const double* x = t.W + (int64_t)k * t.ldw;
    double sq = 0.0;
    for (int i = k + threadIdx.x; i < d; i += QRF_T) sq += x[i] * x[i];
    sq = qrf_wsum(sq);
    if (lane == 0) red[wv] = sq;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += red[w];
    const double nu = sqrt(tot);
    const double x0 = x[k];
    // a zero column gets the identity (v = 0, tau = 0)
    const double alpha = nu == 0.0 ? 0.0 : (x0 >= 0.0 ? -nu : nu);
    const double tk = nu == 0.0 ? 0.0 : 1.0 / (nu * (nu + fabs(x0)));
    double* vk = P.V + (int64_t)(k - c) * P.ldv - c;   // vk[i], i in [c, d)
    for (int i = c + threadIdx.x; i < d; i += QRF_T) vk[i] = (nu == 0.0 || i < k) ? 0.0 : (i == k ? x0 - alpha : x[i]);
    if (threadIdx.x == 0) {
      P.alpha[k] = alpha;
      P.tau[k] = tk;
    }
    __syncthreads();
    // every thread owns rows k + tid, k + tid + QRF_T, ...: partial dot
    // products with all the block's columns at once, one reduction, then
    // each thread updates its own rows
    double acc[NBQ];
#pragma unroll
    for (int jj = 0; jj < NBQ; ++jj) acc[jj] = 0.0;
    for (int i = k + threadIdx.x; i < d; i += QRF_T) {
      const double vi = vk[i];
      const double* wi = t.W + i;
#pragma unroll
      for (int jj = 0; jj < NBQ; ++jj)
        if (c + jj > k && c + jj < c1) acc[jj] += vi * wi[(int64_t)(c + jj) * t.ldw];
    }
#pragma unroll
    for (int jj = 0; jj < NBQ; ++jj) {
      const double v = qrf_wsum(acc[jj]);
      if (lane == 0) part[wv][jj] = v;
    }
    __syncthreads();
    if (threadIdx.x < NBQ) {
      double sdot = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) sdot += part[w][threadIdx.x];
      dots[threadIdx.x] = sdot * tk;
    }
    __syncthreads();
    for (int i = k + threadIdx.x; i < d; i += QRF_T) {
      const double vi = vk[i];
      double* wi = t.W + i;
#pragma unroll
      for (int jj = 0; jj < NBQ; ++jj)
        if (c + jj > k && c + jj < c1) wi[(int64_t)(c + jj) * t.ldw] -= dots[jj] * vi;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int nb = c1 - c;
    GemmTask q;
    q.pad = 0;
    q.A = P.V; q.a_rs = P.ldv; q.a_cs = 1;   // V^T
    q.B = P.V; q.b_rs = 1; q.b_cs = P.ldv;
    q.C = P.G; q.c_rs = 1; q.c_cs = NBQ;
    q.M = nb; q.N = nb; q.K = d - c; q.alpha = 1.0; q.beta = 0.0;
    *g = q;
    const double cells = (double)(d - c) * nb;
    kcount(kcnt, HSS_K_QRCP_OTHER, 8.0 * cells * (nb + 1), 4.0 * cells * nb);
  }
}

// X = S^{-1} (S = striu(V^T V) + diag(V^T V) / 2; 1 on the diagonal of an
// identity reflector) in LDS; GEMM tasks W2 = V^T A_trail and W3 = X^T W2.
__global__ __launch_bounds__(256) void k_qrf_tfac(const QrcpTask* __restrict__ tasks, int c, GemmTask* __restrict__ gt,
                                                 int ntasks) {
  __shared__ double A[NBQ][NBQ + 1];
  __shared__ double dS[NBQ], dX[NBQ];
  GemmTask* g0 = gt + blockIdx.x;
  GemmTask* g1 = gt + ntasks + blockIdx.x;
  if (threadIdx.x == 0) {
    g0->M = 0;
    g1->M = 0;
  }
  const QrcpTask& t = tasks[blockIdx.x];
  if (!qrf_tall(t) || c >= t.m) return;
  const int m = t.m, c1 = min(m, c + NBQ), nb = c1 - c;
  const QrfPtrs P = qrf_ptrs(t);
  const int j = threadIdx.x & 31, ib = threadIdx.x >> 5;   // 8 row groups x 32 columns
  if (j < nb) {
    for (int i = ib; i < nb; i += 8) A[i][j] = i < j ? P.G[(int64_t)j * NBQ + i] : 0.0;   // strictly upper
    if (ib == 0) {
      dS[j] = P.tau[c + j] == 0.0 ? 1.0 : 0.5 * P.G[(int64_t)j * NBQ + j];
      dX[j] = 1.0;
    }
  }
  __syncthreads();
  // right-looking back substitution of S X = I: X strictly upper kept
  // transposed in the lower triangle of A, its diagonal in dX
  for (int k = nb - 1; k >= 0; --k) {
    for (int q = k + 1 + threadIdx.x; q < nb; q += 256) A[q][k] /= dS[k];
    if (threadIdx.x == 0) dX[k] /= dS[k];
    __syncthreads();
    for (int idx = threadIdx.x; idx < k * (nb - k); idx += 256) {
      const int p = idx % k, q = k + idx / k;
      const double xkq = q == k ? dX[k] : A[q][k];
      A[q][p] -= A[p][k] * xkq;
    }
    __syncthreads();
  }
  if (j < nb)
    for (int i = ib; i < nb; i += 8) P.X[(int64_t)j * NBQ + i] = i < j ? A[j][i] : (i == j ? dX[i] : 0.0);
  const int n2 = m - c1;
  if (threadIdx.x == 0 && n2 > 0) {
    GemmTask q;
    q.pad = 0;
    q.A = P.V; q.a_rs = P.ldv; q.a_cs = 1;                          // V^T
    q.B = t.W + (int64_t)c1 * t.ldw + c; q.b_rs = 1; q.b_cs = t.ldw;  // A_trail
    q.C = P.W2; q.c_rs = 1; q.c_cs = NBQ;
    q.M = nb; q.N = n2; q.K = t.d - c; q.alpha = 1.0; q.beta = 0.0;
    *g0 = q;
    q.A = P.X; q.a_rs = NBQ; q.a_cs = 1;                            // X^T
    q.B = P.W2; q.b_rs = 1; q.b_cs = NBQ;
    q.C = P.W3; q.c_rs = 1; q.c_cs = NBQ;
    q.M = nb; q.N = n2; q.K = nb; q.alpha = 1.0; q.beta = 0.0;
    *g1 = q;
  }
}

// GEMM task A_trail -= V W3
__global__ void k_qrf_upd(const QrcpTask* __restrict__ tasks, int ntasks, int c, GemmTask* __restrict__ gt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntasks) return;
  GemmTask* g = gt + i;
  g->M = 0;
  const QrcpTask& t = tasks[i];
  if (!qrf_tall(t) || c >= t.m) return;
  const int c1 = min(t.m, c + NBQ), nb = c1 - c, n2 = t.m - c1;
  if (n2 <= 0) return;
  const QrfPtrs P = qrf_ptrs(t);
  GemmTask q;
  q.pad = 0;
  q.A = P.V; q.a_rs = 1; q.a_cs = P.ldv;
  q.B = P.W3; q.b_rs = 1; q.b_cs = NBQ;
  q.C = t.W + (int64_t)c1 * t.ldw + c; q.c_rs = 1; q.c_cs = t.ldw;
  q.M = t.d - c; q.N = n2; q.K = nb; q.alpha = -1.0; q.beta = 1.0;
  *g = q;
}

// The triangle R becomes the panel: R(k,k) = alpha_k, zeros below the
// diagonal of the first m rows, d := m, column norms for the pivoted steps.
__global__ __launch_bounds__(256) void k_qrf_finish(QrcpTask* __restrict__ tasks) {
  QrcpTask& t = tasks[blockIdx.x];
  if (!qrf_tall(t)) return;
  const int m = t.m;
  const QrfPtrs P = qrf_ptrs(t);
  for (int64_t idx = threadIdx.x; idx < (int64_t)m * m; idx += 256) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    if (i >= j) t.W[(int64_t)j * t.ldw + i] = i == j ? P.alpha[j] : 0.0;
  }
  __syncthreads();
  double* nrm = t.scr + 16;   // norm buffer of step 0
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = wv; j < m; j += 4) {
    const double* y = t.W + (int64_t)j * t.ldw;
    double sq = 0.0;
    for (int i = lane; i <= j && i < m; i += 64) sq += y[i] * y[i];
    sq = qrf_wsum(sq);
    if (lane == 0) nrm[j] = sqrt(sq);
  }
  __syncthreads();
  if (threadIdx.x == 0) t.d = m;
}

QrfScan qrf_scan(const QrcpTask* tasks, int32_t ntasks, hipStream_t s) {
  QrfScan r;
  if (ntasks <= 0) return r;
  int64_t* sw_dev = nullptr;
  int64_t* sw = scan_words(&sw_dev);
  hipLaunchKernelGGL(k_qrf_scan, dim3(1), dim3(QRS), 0, s, tasks, ntasks, sw_dev);
  HSS_HIP_CHECK(hipStreamSynchronize(s));
  r.mtall = (int32_t)sw[0];
  r.cells = sw[1];
  r.nact = (int32_t)sw[2];
  return r;
}

void run_qr_first(QrcpTask* tasks, int32_t ntasks, int32_t dmax, int32_t mcap_max, const QrfScan& sc,
                  GemmTask* gtasks, double* gws, hipStream_t s, unsigned long long* kcnt) {
  const int32_t mtall = sc.mtall;
  if (ntasks <= 0 || mtall <= 0 || sc.cells < kQrFirstMinCells) return;
  const int64_t split_ws = gws ? kGemmSplitElems : 0;
  for (int c = 0; c < mtall; c += NBQ) {
    prof_begin(s);
    hipLaunchKernelGGL(k_qrf_panel, dim3(ntasks), dim3(QRF_T), 0, s, tasks, c, gtasks, kcnt);
    prof_end(HSS_K_QRCP_OTHER, s);
    launch_gemm(gtasks, ntasks, NBQ, NBQ, s, kcnt, dmax, gws, split_ws);
    prof_begin(s);
    hipLaunchKernelGGL(k_qrf_tfac, dim3(ntasks), dim3(256), 0, s, tasks, c, gtasks, ntasks);
    prof_end(HSS_K_QRCP_OTHER, s);
    launch_gemm(gtasks, ntasks, NBQ, mcap_max, s, kcnt, dmax, gws, split_ws);
    launch_gemm(gtasks + ntasks, ntasks, NBQ, mcap_max, s, kcnt);
    prof_begin(s);
    hipLaunchKernelGGL(k_qrf_upd, dim3((ntasks + 127) / 128), dim3(128), 0, s, tasks, ntasks, c, gtasks);
    prof_end(HSS_K_QRCP_OTHER, s);
    launch_gemm(gtasks, ntasks, dmax, mcap_max, s, kcnt);
  }
  prof_begin(s);
  hipLaunchKernelGGL(k_qrf_finish, dim3(ntasks), dim3(256), 0, s, tasks);
  prof_end(HSS_K_QRCP_OTHER, s);
  HSS_HIP_CHECK(hipGetLastError());
}

}  // namespace hss
