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

// x_hat(k,c) = xin(J[k],c) + sum_l E(k,l) xin(J[r+l],c)  (V^T from side 1)
__global__ __launch_bounds__(MB) void k_mv_up(MvArgs a) {
  const int g = a.nodes[blockIdx.x];
  const NodeDesc& nd = a.desc[g];
  if (nd.parent < 0) return;
  const NodeState& st = a.st[g];
  const int r = st.rank[1], m = st.m[1];
  const int32_t* J = a.ipool + nd.J[1];
  const double* E = a.dpool + nd.E[1];
  double* xh = a.xh + a.xh_off[g] * a.nrhs;
  const int ldh = nd.rcap;
  int rl = 0, ldl = 1, ldr = 1;
  const double *xl = nullptr, *xr = nullptr;
  if (!nd.leaf) {
    rl = a.st[nd.left].rank[1];
    xl = a.xh + a.xh_off[nd.left] * a.nrhs;
    xr = a.xh + a.xh_off[nd.right] * a.nrhs;
    ldl = a.desc[nd.left].rcap;
    ldr = a.desc[nd.right].rcap;
  }
  auto xin = [&](int i, int c) -> double {
    if (nd.leaf) return a.X[(int64_t)c * a.n + nd.lo + i];
    return i < rl ? xl[(int64_t)c * ldl + i] : xr[(int64_t)c * ldr + (i - rl)];
  };
  for (int64_t idx = threadIdx.x; idx < (int64_t)r * a.nrhs; idx += MB) {
    const int k = (int)(idx % r), c = (int)(idx / r);
    double s = xin(J[k], c);
    for (int l = 0; l < m - r; ++l) s += E[(int64_t)l * nd.rcap + k] * xin(J[r + l], c);
    xh[(int64_t)c * ldh + k] = s;
  }
}

// Inner node: y_hat of the children; leaf: output rows.
__global__ __launch_bounds__(MB) void k_mv_down(MvArgs a) {
  const int g = a.nodes[blockIdx.x];
  const NodeDesc& nd = a.desc[g];
  const NodeState& st = a.st[g];
  const bool root = nd.parent < 0;
  const int r = root ? 0 : st.rank[0];
  const double* yh = a.yh + a.xh_off[g] * a.nrhs;
  const int ldy = nd.rcap;
  const int32_t* J = a.ipool + nd.J[0];
  const double* E = a.dpool + nd.E[0];
  const int m0 = root ? 0 : st.m[0];
  if (nd.leaf) {
    const int m = nd.hi - nd.lo;
    const double* D = a.dpool + nd.D;
    for (int64_t idx = threadIdx.x; idx < (int64_t)m * a.nrhs; idx += MB) {
      const int i = (int)(idx % m), c = (int)(idx / m);
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += D[(int64_t)j * m + i] * a.X[(int64_t)c * a.n + nd.lo + j];
      a.Y[(int64_t)c * a.n + nd.lo + i] = s;
    }
    __syncthreads();
    if (root) return;
    // U y_hat: row J[k] gets y_hat(k); row J[r+l] gets sum_k E(k,l) y_hat(k)
    for (int64_t idx = threadIdx.x; idx < (int64_t)m0 * a.nrhs; idx += MB) {
      const int i = (int)(idx % m0), c = (int)(idx / m0);
      double s;
      if (i < r) s = yh[(int64_t)c * ldy + i];
      else {
        s = 0.0;
        const int l = i - r;
        for (int k = 0; k < r; ++k) s += E[(int64_t)l * nd.rcap + k] * yh[(int64_t)c * ldy + k];
      }
      a.Y[(int64_t)c * a.n + nd.lo + J[i]] += s;
    }
    return;
  }
  const NodeDesc& L = a.desc[nd.left];
  const NodeDesc& R = a.desc[nd.right];
  const int rl0 = a.st[nd.left].rank[0], rr0 = a.st[nd.right].rank[0];
  const int rl1 = a.st[nd.left].rank[1], rr1 = a.st[nd.right].rank[1];
  double* yl = a.yh + a.xh_off[nd.left] * a.nrhs;
  double* yr = a.yh + a.xh_off[nd.right] * a.nrhs;
  const double* xl = a.xh + a.xh_off[nd.left] * a.nrhs;
  const double* xr = a.xh + a.xh_off[nd.right] * a.nrhs;
  const double* B12 = a.dpool + nd.B12;
  const double* B21 = a.dpool + nd.B21;
  // z = U_tau y_hat (zero at the root), split into the children's y_hat
  const int mz = rl0 + rr0;
  for (int64_t idx = threadIdx.x; idx < (int64_t)mz * a.nrhs; idx += MB) {
    const int i = (int)(idx % mz), c = (int)(idx / mz);
    double s = 0.0;
    if (!root) {
      (void)m0;
      if (i < r) s = yh[(int64_t)c * ldy + i];
      else {
        const int l = i - r;
        for (int k = 0; k < r; ++k) s += E[(int64_t)l * nd.rcap + k] * yh[(int64_t)c * ldy + k];
      }
    }
    const int row = root ? i : J[i];
    if (row < rl0) yl[(int64_t)c * L.rcap + row] = s;
    else yr[(int64_t)c * R.rcap + (row - rl0)] = s;
  }
  __syncthreads();
  for (int64_t idx = threadIdx.x; idx < (int64_t)(rl0 + rr0) * a.nrhs; idx += MB) {
    const int i = (int)(idx % (rl0 + rr0)), c = (int)(idx / (rl0 + rr0));
    if (i < rl0) {
      double s = 0.0;
      for (int k = 0; k < rr1; ++k) s += B12[(int64_t)k * L.rcap + i] * xr[(int64_t)c * R.rcap + k];
      yl[(int64_t)c * L.rcap + i] += s;
    } else {
      const int ii = i - rl0;
      double s = 0.0;
      for (int k = 0; k < rl1; ++k) s += B21[(int64_t)k * R.rcap + ii] * xl[(int64_t)c * L.rcap + k];
      yr[(int64_t)c * R.rcap + ii] += s;
    }
  }
}

void launch_mv_up(const MvArgs& a, hipStream_t s) {
  if (a.count <= 0) return;
  hipLaunchKernelGGL(k_mv_up, dim3(a.count), dim3(MB), 0, s, a);
}

void launch_mv_down(const MvArgs& a, hipStream_t s) {
  if (a.count <= 0) return;
  hipLaunchKernelGGL(k_mv_down, dim3(a.count), dim3(MB), 0, s, a);
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

void launch_err_block(const GenDev& g, const double* Hc, int64_t ldh, int64_t j0, int32_t nb,
                      double* accum, hipStream_t s) {
  hipLaunchKernelGGL(k_err_block, dim3(1024), dim3(256), 0, s, g, Hc, ldh, j0, nb, accum);
}

}  // namespace hss
