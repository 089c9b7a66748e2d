// Direct factorization and solve of a compressed HSS matrix, the downstream
// use the paper times beside the compression (ULV factorization and solve,
// table sixdrivers).  The paper gives no algorithm for it; this is the one
// the interpolative bases of Sec. 2.2 lead to.
//
// A non-root node tau has the row basis U = Pi_r [I; E_r^T] and the column
// basis V = Pi_c [I; E_c^T].  In the order [redundant R; skeleton S] of its
// local rows, T_r = [[I, -E_r^T], [0, I]] maps U to [0; I] (T_c maps V
// likewise), so after the two transforms tau's redundant unknowns couple
// only to tau's local block D' (the leaf's D, or the children's skeleton
// Schur complements joined by B12 and B21, eq. HSSexamplematrix):
//
//   Dhat = T_r D' T_c^T:  Dhat_RR = D'_RR - E_r^T D'_SR - D'_RS E_c + E_r^T D'_SS E_c,
//                         Dhat_RS = D'_RS - E_r^T D'_SS,  Dhat_SR = D'_SR - D'_SS E_c.
//
// F_tau (m x m, column-major) holds Dhat in those orders; an LU with
// partial pivoting of its first k = m - r columns, the pivots taken among
// the redundant rows only, leaves L and U of Dhat_RR, L_SR and U_RS, and in
// the trailing r x r block the Schur complement S_tau, which the parent
// gathers into its own local block.  The root's block is factored whole.
//
// The LU is blocked by 32 columns: a panel kernel (one workgroup per node,
// the panel in global memory) picks the pivots and forms the multipliers
// and the inverses of the panel's diagonal L and U blocks; the row swaps
// then go to the columns right of the panel (the columns left of it keep
// the rows as they stood at their own step, which the solve replays in the
// same order); U12 = L11^{-1} A12 and the trailing update A22 -= L21 U12
// run on the matrix cores as grouped GEMMs over all nodes of a level.
//
// The solve: bottom-up, each node's right-hand side in [R; S] order, the
// row transform (b_R -= E_r^T b_S) and the forward substitution with the
// node's pivots and L, whose skeleton rows then hold the reduced
// right-hand side its parent gathers; at the root the whole block is
// solved.  Top-down: the node's skeleton unknowns come from its parent,
// x_R = U_RR^{-1} (y_R - U_RS x_S), x_S -= E_c x_R (x = T_c^T xhat), and
// the result goes to the children's skeleton rows or to the output.
#include <cstring>

#include "driver.h"

namespace hss {

constexpr int UNB = 32;   // panel width: the GEMM's K tile
constexpr int UPT = 1024; // threads of the panel kernel

// Local index i of F's [R; S] order -> the node's local row (column): R =
// J[r..m), S = J[0..r); the root has no basis (identity).
__device__ __forceinline__ int rs_index(const int32_t* __restrict__ J, int i, int k, int r) {
  if (!J) return i;
  return i < k ? J[r + i] : J[i - k];
}

// ---------------------------------------------------------------- gather
// F = D'(order_r, order_c): the leaf's D, or [[S_l, B12], [B21, S_r]] from
// the children's factors (their trailing blocks).
__global__ __launch_bounds__(256) void k_ulv_build(const UlvBuild* __restrict__ tasks) {
  const UlvBuild& t = tasks[blockIdx.x];
  const int m = t.m;
  const int64_t tot = (int64_t)m * m;
  for (int64_t e = threadIdx.x + (int64_t)blockIdx.y * 256; e < tot; e += (int64_t)256 * gridDim.y) {
    const int i = (int)(e % m), j = (int)(e / m);
    const int a = rs_index(t.Jr, i, t.k, t.r), b = rs_index(t.Jc, j, t.k, t.r);
    double v;
    if (t.D) {
      v = t.D[a + (int64_t)b * m];
    } else if (a < t.rl) {
      v = b < t.rl ? t.Fl[(t.kl + a) + (int64_t)(t.kl + b) * t.ml] : t.B12[a + (int64_t)(b - t.rl) * t.ld12];
    } else {
      const int a2 = a - t.rl;
      v = b < t.rl ? t.B21[a2 + (int64_t)b * t.ld21] : t.Fr[(t.kr + a2) + (int64_t)(t.kr + b - t.rl) * t.mr];
    }
    t.F[e] = v;
  }
}

// ---------------------------------------------------------------- panel
// LU with partial pivoting of F(jb:m, jb:jb+nb), pivots among rows [jb, k);
// the panel's row swaps stay in its own columns.  The panel is factored in
// sub-panels of USB columns: column by column inside a sub-panel (pivot,
// swap across the whole panel, multipliers, update of the sub-panel's
// later columns), then one blocked update of the panel's columns right of
// it (U12 = L11^{-1} A12 on its rows, A22 -= L21 U12 below), so each entry
// is read and written about USB + nb / USB times instead of nb.  Then Linv
// and Uinv, the inverses of the panel's diagonal block's unit-lower and
// upper parts (UNB x UNB, column-major, zero outside nb x nb).
constexpr int USB = 8;
static_assert(UNB % USB == 0, "whole sub-panels");
__global__ __launch_bounds__(UPT) void k_ulv_panel(const UlvPanel* __restrict__ tasks, int32_t* __restrict__ flag) {
  const UlvPanel& t = tasks[blockIdx.x];
  const int nb = t.nb;
  if (nb <= 0) return;
  const int m = t.m, k = t.k, jb = t.jb, tid = threadIdx.x;
  HSS_GLOBAL double* F = gview_w(t.F);
  HSS_GLOBAL double* P = F + (int64_t)jb * m;   // P(i, c) = F(i, jb + c), i absolute
  __shared__ double prow[UNB];
  __shared__ double U12[USB][UNB];
  __shared__ double rv[2 * 16];
  __shared__ int ri[2 * 16];
  static_assert(UPT / 64 <= 16, "wave partials");
  for (int c0 = 0; c0 < nb; c0 += USB) {
    const int ce = min(c0 + USB, nb);
    for (int c = c0; c < ce; ++c) {
      const int j = jb + c;
      // the pivot: largest |P(i, c)| over i in [j, k), the lowest i on ties
      double bv = -1.0;
      int bi = 0x7fffffff;
#pragma unroll 4
      for (int i = j + tid; i < k; i += UPT) {
        const double v = fabs(P[i + (int64_t)c * m]);
        if (v > bv) { bv = v; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_down(bv, off);
        const int oi = __shfl_down(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if ((tid & 63) == 0) { rv[(c & 1) * 16 + (tid >> 6)] = bv; ri[(c & 1) * 16 + (tid >> 6)] = bi; }
      __syncthreads();
      // every thread combines the waves' candidates (double-buffered by
      // column parity, so the next column's partials cannot overwrite them)
      double pv = rv[(c & 1) * 16];
      int p = ri[(c & 1) * 16];
      for (int w = 1; w < UPT / 64; ++w) {
        const double ov = rv[(c & 1) * 16 + w];
        const int oi = ri[(c & 1) * 16 + w];
        if (ov > pv || (ov == pv && oi < p)) { pv = ov; p = oi; }
      }
      if (!(pv > 0.0)) p = j;   // a zero (or non-finite) column: the block is singular
      if (tid == 0) {
        if (!(pv > 0.0)) atomicOr(flag, 1);
        t.piv[j] = p;
      }
      if (tid < nb) {   // the swap across the whole panel; the pivot row's sub-panel part to LDS
        HSS_GLOBAL double* a = P + j + (int64_t)tid * m;
        HSS_GLOBAL double* b = P + p + (int64_t)tid * m;
        const double x = *a, y = *b;
        if (p != j) { *a = y; *b = x; }
        prow[tid] = p != j ? y : x;
      }
      __syncthreads();
      const double d = prow[c];
      const double rinv = d != 0.0 ? 1.0 / d : 0.0;
      for (int i = j + 1 + tid; i < m; i += UPT) {
        HSS_GLOBAL double* pi = P + i;
        double v[USB];
#pragma unroll
        for (int q = 0; q < USB; ++q) v[q] = c0 + q > c && c0 + q < ce ? pi[(int64_t)(c0 + q) * m] : 0.0;
        const double l = pi[(int64_t)c * m] * rinv;
        pi[(int64_t)c * m] = l;
#pragma unroll
        for (int q = 0; q < USB; ++q)
          if (c0 + q > c && c0 + q < ce) pi[(int64_t)(c0 + q) * m] = v[q] - l * prow[c0 + q];
      }
      __syncthreads();
    }
    if (ce >= nb) break;
    // U12 = L11^{-1} A12 on the sub-panel's rows (one thread per column right
    // of it, the unit-lower L11 from the sub-panel's rows), into LDS and F
    const int w = nb - ce;
    if (tid < w) {
      const int cc = ce + tid;
      double u[USB];
#pragma unroll
      for (int q = 0; q < USB; ++q) u[q] = c0 + q < ce ? P[(jb + c0 + q) + (int64_t)cc * m] : 0.0;
#pragma unroll
      for (int q = 1; q < USB; ++q) {
        if (c0 + q >= ce) break;
        double s = u[q];
#pragma unroll
        for (int q2 = 0; q2 < q; ++q2) s -= P[(jb + c0 + q) + (int64_t)(c0 + q2) * m] * u[q2];
        u[q] = s;
      }
#pragma unroll
      for (int q = 0; q < USB; ++q) {
        U12[q][tid] = u[q];
        if (c0 + q < ce) P[(jb + c0 + q) + (int64_t)cc * m] = u[q];
      }
    }
    __syncthreads();
    // A22 -= L21 U12 for the rows below the sub-panel
    for (int i = jb + ce + tid; i < m; i += UPT) {
      HSS_GLOBAL double* pi = P + i;
      double l[USB];
#pragma unroll
      for (int q = 0; q < USB; ++q) l[q] = c0 + q < ce ? pi[(int64_t)(c0 + q) * m] : 0.0;
      double a[UNB - USB];
#pragma unroll
      for (int x = 0; x < UNB - USB; ++x) a[x] = x < w ? pi[(int64_t)(ce + x) * m] : 0.0;
#pragma unroll
      for (int x = 0; x < UNB - USB; ++x) {
        if (x >= w) break;
        double s = a[x];
#pragma unroll
        for (int q = 0; q < USB; ++q) s -= l[q] * U12[q][x];
        pi[(int64_t)(ce + x) * m] = s;
      }
    }
    __syncthreads();
  }
  // inverses of the diagonal block's L (unit lower) and U, one column per thread
  if (tid < UNB) {
    const int c = tid;
    HSS_GLOBAL double* Li = gview_w(t.inv);
    HSS_GLOBAL double* Ui = gview_w(t.inv + UNB * UNB);
    const HSS_GLOBAL double* A = F + jb + (int64_t)jb * m;   // A(i, q) = F(jb + i, jb + q)
    for (int i = 0; i < UNB; ++i) {
      Li[i + c * UNB] = 0.0;
      Ui[i + c * UNB] = 0.0;
    }
    if (c < nb) {
      // L X = e_c: X(c) = 1, X(i) = -sum_{q in [c, i)} L(i, q) X(q)
      Li[c + c * UNB] = 1.0;
      for (int i = c + 1; i < nb; ++i) {
        double s = 0.0;
        for (int q = c; q < i; ++q) s += A[i + (int64_t)q * m] * Li[q + c * UNB];
        Li[i + c * UNB] = -s;
      }
      // U X = e_c: X(c) = 1 / U(c, c), X(i) = -sum_{q in (i, c]} U(i, q) X(q) / U(i, i)
      Ui[c + c * UNB] = 1.0 / A[c + (int64_t)c * m];
      for (int i = c - 1; i >= 0; --i) {
        double s = 0.0;
        for (int q = i + 1; q <= c; ++q) s += A[i + (int64_t)q * m] * Ui[q + c * UNB];
        Ui[i + c * UNB] = -s / A[i + (int64_t)i * m];
      }
    }
  }
}

// The panel's row swaps applied to columns [c0, c1) of a matrix with
// leading dimension ld (F right of the panel, or a right-hand side block):
// one thread per column, the swaps in order.
__global__ __launch_bounds__(256) void k_ulv_swap(const UlvSwap* __restrict__ tasks) {
  const UlvSwap& t = tasks[blockIdx.x];
  const int64_t col = t.c0 + (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (t.nb <= 0 || col >= t.c1) return;
  HSS_GLOBAL double* X = gview_w(t.X + col * t.ld);
  for (int c = 0; c < t.nb; ++c) {
    const int j = t.jb + c, p = t.piv[j];
    if (p != j) {
      const double a = X[j], b = X[p];
      X[j] = b;
      X[p] = a;
    }
  }
}

// ---------------------------------------------------------------- solve moves
// Y (m x nrhs, column-major, ld m) = the node's right-hand side in [R; S] row
// order: permuted B rows (leaf), or the children's reduced right-hand sides
// (the skeleton rows of their Y).
__global__ __launch_bounds__(256) void k_ulv_rhs_in(const UlvMove* __restrict__ tasks, int32_t nrhs) {
  const UlvMove& t = tasks[blockIdx.x];
  const int m = t.m;
  const int64_t tot = (int64_t)m * nrhs;
  for (int64_t e = threadIdx.x + (int64_t)blockIdx.y * 256; e < tot; e += (int64_t)256 * gridDim.y) {
    const int i = (int)(e % m), c = (int)(e / m);
    const int a = rs_index(t.J, i, t.k, t.r);
    double v;
    if (t.ext) v = t.ext[(t.lo + a) + (int64_t)c * t.ldext];
    else if (a < t.rl) v = t.Yl[(t.kl + a) + (int64_t)c * t.ml];
    else v = t.Yr[(t.kr + a - t.rl) + (int64_t)c * t.mr];
    t.Y[i + (int64_t)c * m] = v;
  }
}

// The node's solution (Y in [R; S] column order) to its local column order:
// into the output rows (leaf) or the children's skeleton rows.
__global__ __launch_bounds__(256) void k_ulv_x_out(const UlvMove* __restrict__ tasks, int32_t nrhs) {
  const UlvMove& t = tasks[blockIdx.x];
  const int m = t.m;
  const int64_t tot = (int64_t)m * nrhs;
  for (int64_t e = threadIdx.x + (int64_t)blockIdx.y * 256; e < tot; e += (int64_t)256 * gridDim.y) {
    const int i = (int)(e % m), c = (int)(e / m);
    const int a = rs_index(t.J, i, t.k, t.r);
    const double v = t.Y[i + (int64_t)c * m];
    if (t.ext) t.ext[(t.lo + a) + (int64_t)c * t.ldext] = v;
    else if (a < t.rl) t.Yl[(t.kl + a) + (int64_t)c * t.ml] = v;
    else t.Yr[(t.kr + a - t.rl) + (int64_t)c * t.mr] = v;
  }
}

// ---------------------------------------------------------------- fused solves
// For few right-hand sides the block steps of a level's substitutions are
// too small for one launch each: one workgroup per node runs them all.
// Forward (after the row transform): for each 32-row block of the first k
// rows, its row swaps, y_j = Linv y_j, and Y(rows below, :) -= L(rows
// below, block) y_j (the skeleton rows included).  Backward (after
// y_R -= U_RS x_S): from the last block up, x_j = Uinv y_j and
// Y(rows above, :) -= U(rows above, block) x_j.
constexpr int UST = 1024;  // threads of the fused substitutions
__global__ __launch_bounds__(UST) void k_ulv_subst(const UlvSubst* __restrict__ tasks, int32_t nrhs, int32_t backward) {
  const UlvSubst& t = tasks[blockIdx.x];
  const int m = t.m, k = t.k, tid = threadIdx.x;
  if (k <= 0) return;
  HSS_GLOBAL double* Y = gview_w(t.Y);
  const HSS_GLOBAL double* F = gview(t.F);
  __shared__ double yj[UNB * UST_MAXR];
  const int nblk = (k + UNB - 1) / UNB;
  for (int s0 = 0; s0 < nblk; ++s0) {
    const int st = backward ? nblk - 1 - s0 : s0;
    const int jb = st * UNB, nb = min(UNB, k - jb);
    const HSS_GLOBAL double* inv = gview(t.inv + (int64_t)st * 2 * UNB * UNB + (backward ? UNB * UNB : 0));
    if (!backward && tid < nrhs) {   // the block's row swaps, in order, one column per thread
      HSS_GLOBAL double* y = Y + (int64_t)tid * m;
      for (int q = 0; q < nb; ++q) {
        const int j = jb + q, p = t.piv[j];
        if (p != j) {
          const double a = y[j], b = y[p];
          y[j] = b;
          y[p] = a;
        }
      }
    }
    __syncthreads();
    // y_j = inv y_j (inv: lower for the forward pass, upper for the backward)
    for (int e = tid; e < nb * nrhs; e += UST) {
      const int r = e % nb, c = e / nb;
      double acc = 0.0;
#pragma unroll 8
      for (int q = 0; q < nb; ++q) acc += inv[r + q * UNB] * Y[(jb + q) + (int64_t)c * m];
      yj[r + UNB * c] = acc;
    }
    __syncthreads();
    for (int e = tid; e < nb * nrhs; e += UST) {
      const int r = e % nb, c = e / nb;
      Y[(jb + r) + (int64_t)c * m] = yj[r + UNB * c];
    }
    // the other rows: below the block (forward) or above it (backward)
    const int lo = backward ? 0 : jb + nb, hi = backward ? jb : m;
    for (int64_t e = tid; e < (int64_t)(hi - lo) * nrhs; e += UST) {
      const int i = lo + (int)(e % (hi - lo)), c = (int)(e / (hi - lo));
      double f[UNB];   // the row's block entries, loaded together
#pragma unroll
      for (int q = 0; q < UNB; ++q) f[q] = q < nb ? F[i + (int64_t)(jb + q) * m] : 0.0;
      double acc = Y[i + (int64_t)c * m];
#pragma unroll
      for (int q = 0; q < UNB; ++q) acc -= f[q] * yj[q + UNB * c];
      Y[i + (int64_t)c * m] = acc;
    }
    __syncthreads();
  }
}

void launch_ulv_subst(const UlvSubst* t, int32_t count, int32_t nrhs, int32_t backward, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_ulv_subst, dim3(count), dim3(UST), 0, s, t, nrhs, backward);
}

void launch_ulv_build(const UlvBuild* t, int32_t count, int64_t maxelems, hipStream_t s) {
  if (count <= 0) return;
  const unsigned gy = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (maxelems + 4095) / 4096));
  hipLaunchKernelGGL(k_ulv_build, dim3(count, gy), dim3(256), 0, s, t);
}
void launch_ulv_panel(const UlvPanel* t, int32_t count, int32_t* flag, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_ulv_panel, dim3(count), dim3(UPT), 0, s, t, flag);
}
void launch_ulv_swap(const UlvSwap* t, int32_t count, int64_t maxcols, hipStream_t s) {
  if (count <= 0 || maxcols <= 0) return;
  hipLaunchKernelGGL(k_ulv_swap, dim3(count, (unsigned)((maxcols + 255) / 256)), dim3(256), 0, s, t);
}
void launch_ulv_rhs_in(const UlvMove* t, int32_t count, int32_t nrhs, int64_t maxelems, hipStream_t s) {
  if (count <= 0) return;
  const unsigned gy = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (maxelems * nrhs + 4095) / 4096));
  hipLaunchKernelGGL(k_ulv_rhs_in, dim3(count, gy), dim3(256), 0, s, t, nrhs);
}
void launch_ulv_x_out(const UlvMove* t, int32_t count, int32_t nrhs, int64_t maxelems, hipStream_t s) {
  if (count <= 0) return;
  const unsigned gy = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (maxelems * nrhs + 4095) / 4096));
  hipLaunchKernelGGL(k_ulv_x_out, dim3(count, gy), dim3(256), 0, s, t, nrhs);
}

}  // namespace hss
