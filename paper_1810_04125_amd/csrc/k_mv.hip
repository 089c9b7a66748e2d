// HSS matrix-vector product and reconstruction error (verification of the
// compressed generators).  The HSS format of Sec. 2.1: leaves hold D, the
// sibling block A(I_nu1, I_nu2) ~= U^big_nu1 B12 (V^big_nu2)^T, and the
// bases are nested (eq. nestedUV).  Upward pass: x_hat = V^T x(I) on the
// leaves and V^T [x_hat_nu1; x_hat_nu2] above.  Downward pass: the parent's
// y_hat expanded through U_tau plus the sibling couplings B12 x_hat_nu2 and
// B21 x_hat_nu1; leaves finish with U y_hat + D x.  All in permuted order.
#include "gen.h"

namespace hss {

constexpr int MB = 256;

#define MV_FOR(idx, total) \
  for (int64_t idx = threadIdx.x + (int64_t)blockIdx.y * MB; idx < (total); idx += (int64_t)MB * gridDim.y)

__device__ __forceinline__ double* xh_of(const MvArgs& a, int g) { return a.xh + a.xh_off[g] * a.nrhs; }
__device__ __forceinline__ double* yh_of(const MvArgs& a, int g) { return a.yh + a.xh_off[g] * a.nrhs; }
__device__ __forceinline__ double* ws_of(const MvArgs& a, int g) { return a.ws + a.ws_off[g] * a.nrhs; }

// Upward pass, one level: x_hat = V^T x_in = x_in(J) + E x_in(rest) (side-1
// basis); x_in = x(I_tau) on a leaf, [x_hat_nu1; x_hat_nu2] above.  Copies
// x_in(J) into x_hat and x_in(rest) into the node's workspace; the product
// E x_in(rest) is the GEMM task t.
__global__ __launch_bounds__(MB) void k_mvu_gather(MvArgs a, GemmTask* __restrict__ tasks) {
  const int t = blockIdx.x;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  if (threadIdx.x == 0 && blockIdx.y == 0) tasks[t].M = 0;
  if (nd.parent < 0) return;
  const NodeState& st = a.st[g];
  const int r = st.rank[1], m = st.m[1];
  const int32_t* J = a.ipool + nd.J[1];
  double* xh = xh_of(a, g);
  double* xr = ws_of(a, g);
  int rl = 0, ldl = 1, ldr = 1;
  const double *xl = nullptr, *xrr = nullptr;
  if (!nd.leaf) {
    rl = a.st[nd.left].rank[1];
    xl = xh_of(a, nd.left);
    xrr = xh_of(a, nd.right);
    ldl = a.desc[nd.left].rcap;
    ldr = a.desc[nd.right].rcap;
  }
  MV_FOR(idx, (int64_t)m * a.nrhs) {
    const int i = (int)(idx % m), c = (int)(idx / m);
    const int row = J[i];
    double v;
    if (nd.leaf) v = a.X[(int64_t)c * a.n + nd.lo + row];
    else v = row < rl ? xl[(int64_t)c * ldl + row] : xrr[(int64_t)c * ldr + (row - rl)];
    if (i < r) xh[(int64_t)c * nd.rcap + i] = v;
    else xr[(int64_t)c * nd.mcap + (i - r)] = v;
  }
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    GemmTask k;
    k.A = a.epool + nd.E[1]; k.a_rs = 1; k.a_cs = nd.eld[1];
    k.B = xr; k.b_rs = 1; k.b_cs = nd.mcap;
    k.C = xh; k.c_rs = 1; k.c_cs = nd.rcap;
    k.M = r; k.N = a.nrhs; k.K = m - r; k.pad = 0; k.alpha = 1.0; k.beta = 1.0;
    tasks[t] = k;
  }
}

// Downward pass, one level, GEMM tasks before the scatter: z_rest = E^T y_hat
// (side-0 basis U = Pi [I; E^T]) into the workspace, and Y(I) = D x(I) on leaves.
__global__ void k_mvd_pre(MvArgs a, GemmTask* __restrict__ tasks) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count) return;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  const NodeState& st = a.st[g];
  GemmTask k;
  k.pad = 0; k.alpha = 1.0; k.beta = 0.0; k.N = a.nrhs;
  k.M = 0;
  if (nd.parent >= 0) {
    const int r = st.rank[0], m = st.m[0];
    k.A = a.epool + nd.E[0]; k.a_rs = nd.eld[0]; k.a_cs = 1;
    k.B = yh_of(a, g); k.b_rs = 1; k.b_cs = nd.rcap;
    k.C = ws_of(a, g); k.c_rs = 1; k.c_cs = nd.mcap;
    k.M = m - r; k.K = r;
  }
  tasks[t] = k;
  k.M = 0;
  if (nd.leaf) {
    const int m = nd.hi - nd.lo;
    k.A = a.dpool + nd.D; k.a_rs = 1; k.a_cs = m;
    k.B = a.X + nd.lo; k.b_rs = 1; k.b_cs = a.n;
    k.C = a.Y + nd.lo; k.c_rs = 1; k.c_cs = a.n;
    k.M = m; k.K = m;
  }
  tasks[a.count + t] = k;
}

// Downward pass, one level, after k_mvd_pre's products: z = U y_hat placed
// into the children's y_hat (rows J of z are y_hat, the rest E^T y_hat), or
// added to the output rows on a leaf; the GEMM tasks add the sibling
// couplings y_hat_nu1 += B12 x_hat_nu2, y_hat_nu2 += B21 x_hat_nu1.
__global__ __launch_bounds__(MB) void k_mvd_scatter(MvArgs a, GemmTask* __restrict__ tasks) {
  const int t = blockIdx.x;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  const NodeState& st = a.st[g];
  const bool root = nd.parent < 0;
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    tasks[t].M = 0;
    tasks[a.count + t].M = 0;
  }
  const int r = root ? 0 : st.rank[0];
  const double* yh = yh_of(a, g);
  const double* zr = ws_of(a, g);
  const int32_t* J = a.ipool + nd.J[0];
  if (nd.leaf) {
    if (root) return;
    const int m = st.m[0];
    MV_FOR(idx, (int64_t)m * a.nrhs) {
      const int i = (int)(idx % m), c = (int)(idx / m);
      const double v = i < r ? yh[(int64_t)c * nd.rcap + i] : zr[(int64_t)c * nd.mcap + (i - r)];
      a.Y[(int64_t)c * a.n + nd.lo + J[i]] += v;
    }
    return;
  }
  const NodeDesc& L = a.desc[nd.left];
  const NodeDesc& R = a.desc[nd.right];
  const int rl0 = a.st[nd.left].rank[0], rr0 = a.st[nd.right].rank[0];
  const int rl1 = a.st[nd.left].rank[1], rr1 = a.st[nd.right].rank[1];
  double* yl = yh_of(a, nd.left);
  double* yr = yh_of(a, nd.right);
  const int mz = rl0 + rr0;
  MV_FOR(idx, (int64_t)mz * a.nrhs) {
    const int i = (int)(idx % mz), c = (int)(idx / mz);
    double v = 0.0;
    int row = i;
    if (!root) {
      v = i < r ? yh[(int64_t)c * nd.rcap + i] : zr[(int64_t)c * nd.mcap + (i - r)];
      row = J[i];
    }
    if (row < rl0) yl[(int64_t)c * L.rcap + row] = v;
    else yr[(int64_t)c * R.rcap + (row - rl0)] = v;
  }
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    GemmTask k;
    k.pad = 0; k.alpha = 1.0; k.beta = 1.0; k.N = a.nrhs;
    k.A = a.epool + nd.B12; k.a_rs = 1; k.a_cs = nd.b12ld;
    k.B = xh_of(a, nd.right); k.b_rs = 1; k.b_cs = R.rcap;
    k.C = yl; k.c_rs = 1; k.c_cs = L.rcap;
    k.M = rl0; k.K = rr1;
    tasks[t] = k;
    k.A = a.epool + nd.B21; k.a_rs = 1; k.a_cs = nd.b21ld;
    k.B = xh_of(a, nd.left); k.b_rs = 1; k.b_cs = L.rcap;
    k.C = yr; k.c_rs = 1; k.c_cs = R.rcap;
    k.M = rr0; k.K = rl1;
    tasks[a.count + t] = k;
  }
}

static dim3 mv_grid(int count) {
  int g = (512 + count - 1) / count;
  g = g < 1 ? 1 : (g > 32 ? 32 : g);
  return dim3(count, g);
}

void launch_mv_up(const MvArgs& a, GemmTask* tasks, int32_t mcap, hipStream_t s) {
  if (a.count <= 0) return;
  hipLaunchKernelGGL(k_mvu_gather, mv_grid(a.count), dim3(MB), 0, s, a, tasks);
  launch_gemm(tasks, a.count, mcap, a.nrhs, s);
}

void launch_mv_down(const MvArgs& a, GemmTask* tasks, int32_t mcap, hipStream_t s) {
  if (a.count <= 0) return;
  hipLaunchKernelGGL(k_mvd_pre, dim3((a.count + 127) / 128), dim3(128), 0, s, a, tasks);
  launch_gemm(tasks, 2 * a.count, mcap, a.nrhs, s);
  hipLaunchKernelGGL(k_mvd_scatter, mv_grid(a.count), dim3(MB), 0, s, a, tasks);
  launch_gemm(tasks, 2 * a.count, mcap, a.nrhs, s);
}

// out(i,c) = X(perm[i], c) (inverse = 0) or out(perm[i], c) = X(i, c) (inverse = 1)
__global__ void k_gather_rows(const double* __restrict__ X, int64_t ldx, const int64_t* __restrict__ perm,
                              int64_t n, int32_t nrhs, double* __restrict__ out, int64_t ldo, int32_t inverse) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * nrhs) return;
  const int64_t i = idx % n, c = idx / n;
  if (inverse) out[c * ldo + perm[i]] = X[c * ldx + i];
  else out[c * ldo + i] = X[c * ldx + perm[i]];
}

void launch_gather_rows(const double* X, int64_t ldx, const int64_t* perm, int64_t n, int32_t nrhs,
                        double* out, int64_t ldo, int32_t inverse, hipStream_t s) {
  const int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, ldx, perm,
                     n, nrhs, out, ldo, inverse);
}

// accum[2*blockIdx.x + {0,1}] = partial sums of (A - H)^2 and A^2 over a
// column block of H (n x nb, column-major, ld ldh) starting at column j0.
__global__ __launch_bounds__(256) void k_err_block(GenDev g, const double* __restrict__ Hc, int64_t ldh,
                                                   int64_t j0, int32_t nb, double* __restrict__ accum) {
  __shared__ double r1[4], r2[4];
  const int64_t n = g.n;
  const int64_t tot = n * nb;
  double e = 0.0, a2 = 0.0;
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx % n, c = idx / n;
    const double av = gen_entry(g, i, j0 + c);
    const double df = av - Hc[c * ldh + i];
    e += df * df;
    a2 += av * av;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    e += __shfl_xor(e, o, 64);
    a2 += __shfl_xor(a2, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) { r1[w] = e; r2[w] = a2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    accum[2 * blockIdx.x] += r1[0] + r1[1] + r1[2] + r1[3];
    accum[2 * blockIdx.x + 1] += r2[0] + r2[1] + r2[2] + r2[3];
  }
}

// Same sums with the column block of A given explicitly (n x nb, ld lda):
// the columns a caller's sample routine returned for A_hat [e_j0 ...].
__global__ __launch_bounds__(256) void k_err_cols(const double* __restrict__ Ac, int64_t lda,
                                                 const double* __restrict__ Hc, int64_t ldh, int64_t n,
                                                 int32_t nb, double* __restrict__ accum) {
  __shared__ double r1[4], r2[4];
  const int64_t tot = n * nb;
  double e = 0.0, a2 = 0.0;
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx % n, c = idx / n;
    const double av = Ac[c * lda + i];
    const double df = av - Hc[c * ldh + i];
    e += df * df;
    a2 += av * av;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    e += __shfl_xor(e, o, 64);
    a2 += __shfl_xor(a2, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) { r1[w] = e; r2[w] = a2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    accum[2 * blockIdx.x] += r1[0] + r1[1] + r1[2] + r1[3];
    accum[2 * blockIdx.x + 1] += r2[0] + r2[1] + r2[2] + r2[3];
  }
}

// flag |= 1 if any entry of the rows x cols block (ld ld) is not finite
__global__ __launch_bounds__(256) void k_check_finite(const double* __restrict__ p, int64_t rows, int32_t cols,
                                                     int64_t ld, int32_t* __restrict__ flag) {
  const int64_t tot = rows * cols;
  int bad = 0;
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx % rows, c = idx / rows;
    bad |= !isfinite(p[c * ld + i]);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

void launch_check_finite(const double* p, int64_t rows, int32_t cols, int64_t ld, int32_t* flag, hipStream_t s) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(1024, (tot + 255) / 256);
  hipLaunchKernelGGL(k_check_finite, dim3(g), dim3(256), 0, s, p, rows, cols, ld, flag);
}

void launch_err_cols(const double* Ac, int64_t lda, const double* Hc, int64_t ldh, int64_t n, int32_t nb,
                     double* accum, hipStream_t s) {
  hipLaunchKernelGGL(k_err_cols, dim3(1024), dim3(256), 0, s, Ac, lda, Hc, ldh, n, nb, accum);
}

__global__ void k_eye_block(double* __restrict__ X, int64_t n, int64_t j0, int32_t nb) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * nb) return;
  const int64_t i = idx % n, c = idx / n;
  X[idx] = (i == j0 + c) ? 1.0 : 0.0;
}

void launch_eye_block(double* X, int64_t n, int64_t j0, int32_t nb, hipStream_t s) {
  const int64_t tot = n * nb;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_eye_block, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, n, j0, nb);
}

// out(a, b) = A_hat(I[a], J[b]) (Sec. 4: D and B generators are sub-blocks of A)
__global__ void k_extract_list(GenDev g, int32_t nI, const int64_t* __restrict__ I, int32_t nJ,
                               const int64_t* __restrict__ J, double* __restrict__ out, int64_t ldo) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nI * nJ) return;
  const int64_t a = idx % nI, b = idx / nI;
  out[b * ldo + a] = gen_entry(g, I[a], J[b]);
}

void launch_extract(const GenDev& g, int32_t nI, const int64_t* I, int32_t nJ, const int64_t* J,
                    double* out, int64_t ldo, hipStream_t s) {
  const int64_t tot = (int64_t)nI * nJ;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_extract_list, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g, nI, I, nJ, J,
                     out, ldo);
}

// Block copies: blockIdx.x selects the block, the gridDim.y workgroups of
// a block share its elements, and every thread loads 8 elements before it
// stores them.
__global__ __launch_bounds__(256) void k_copy2d(const Copy2D* __restrict__ tasks) {
  constexpr int U = 8;
  const Copy2D t = tasks[blockIdx.x];
  const int tot = t.rows * t.cols;
  const int stride = 256 * gridDim.y;
  const HSS_GLOBAL double* src = gview(t.src);
  HSS_GLOBAL double* dst = gview_w(t.dst);
  for (int base = threadIdx.x + blockIdx.y * 256; base < tot; base += stride * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = min(base + u * stride, tot - 1);
      const int i = idx % t.rows, j = idx / t.rows;
      v[u] = src[(int64_t)j * t.lds + i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * stride;
      if (idx < tot) {
        const int i = idx % t.rows, j = idx / t.rows;
        dst[(int64_t)j * t.ldd + i] = v[u];
      }
    }
  }
}

void launch_copy2d(const Copy2D* tasks, int32_t count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_copy2d, dim3(count, 8), dim3(256), 0, s, tasks);
}

void launch_err_block(const GenDev& g, const double* Hc, int64_t ldh, int64_t j0, int32_t nb,
                      double* accum, hipStream_t s) {
  hipLaunchKernelGGL(k_err_block, dim3(1024), dim3(256), 0, s, g, Hc, ldh, j0, nb, accum);
}

}  // namespace hss
