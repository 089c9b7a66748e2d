// Per-level kernels of the adaptive HSS compression.  Every launch covers
// all nodes of one tree level of every problem of the job; one workgroup
// (256 threads) or one thread owns a node.  Sizes that depend on ranks are
// read from NodeState, so a whole round runs without host involvement.
//
//   k_plan          Alg. 3: which nodes take part, their column range
//   k_extract_nodes Alg. 3: D = A(I,I) on leaves, B12/B21 from skeletons
//   k_ls_gather     Alg. 2 ComputeLocalSamples (copy part; products on MFMA)
//   k_fn_copy/qr    Alg. 5 / eq. stopping_criteria: CGS2 (on MFMA), norms,
//                   Householder QR of the projected block, the two tests
//   k_qrcp          eqs. ID, QRCPSr: QR with column pivoting of S^T with
//                   threshold stopping (plain, or HMT-scaled for Alg. 4),
//                   then E = R1^{-1} R2
//   k_red_gather    Alg. 2 ReduceLocalSamples (gather part; E x(rest) on MFMA)
//   k_finalize      node state transitions of Alg. 3
#include <math.h>

#include <algorithm>

#include "gen.h"

namespace hss {

constexpr int NB = 256;  // threads per node workgroup
constexpr int NW = NB / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup; every thread gets the result.  `red` holds NW doubles.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Same for a workgroup of NT threads; `red` holds NT / 64 doubles.
template <int NT>
__device__ double block_sum_n(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Element loops of the per-node copy kernels are spread over gridDim.y
// workgroups of the same node.
#define CHUNKED_FOR(idx, total) \
  for (int64_t idx = threadIdx.x + (int64_t)blockIdx.y * NB; idx < (total); idx += (int64_t)NB * gridDim.y)

// Copy loops of the per-node kernels: the node's elements [0, total) are
// spread over the gridDim.y workgroups of the node, and every thread loads
// CU elements (addresses from `at`, which maps an element index to its
// source and destination) before it stores any, so that the loads of a
// thread are in flight together.
struct CopyAt {
  const HSS_GLOBAL double* src;
  HSS_GLOBAL double* dst;
};
constexpr int CU = 8;

template <class At>
__device__ __forceinline__ void copy_elems(int total, At at) {
  const int stride = NB * gridDim.y;
  for (int base = threadIdx.x + blockIdx.y * NB; base < total; base += stride * CU) {
    double v[CU];
    HSS_GLOBAL double* dst[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      const CopyAt p = at(min(base + u * stride, total - 1));
      v[u] = *p.src;
      dst[u] = p.dst;
    }
#pragma unroll
    for (int u = 0; u < CU; ++u)
      if (base + u * stride < total) *dst[u] = v[u];
  }
}

// m x nc block copied between a column-major and a row-major layout
// through 32 x 32 LDS tiles, so that both the loads and the stores run
// along the contiguous dimension of their side.  SRC_RM: the source is
// row-major (row i at src + i * sld) and the destination column-major;
// otherwise the reverse.  The node's tiles are spread over its gridDim.y
// workgroups; every thread of the workgroup must call it.
template <bool SRC_RM>
__device__ void copy_transpose(const double* src, int64_t sld, double* dst, int64_t dld, int m, int nc) {
  __shared__ double tile[32][33];
  const HSS_GLOBAL double* gs = gview(src);
  HSS_GLOBAL double* gd = gview_w(dst);
  const int tr = (m + 31) / 32, tcn = (nc + 31) / 32;
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;   // NB = 256: 32 x 8
  for (int t = blockIdx.y; t < tr * tcn; t += gridDim.y) {
    const int r0 = (t % tr) * 32, k0 = (t / tr) * 32;
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = ly + 8 * u;
      const int i = SRC_RM ? r0 + b : r0 + lx, c = SRC_RM ? k0 + lx : k0 + b;
      v[u] = (i < m && c < nc) ? (SRC_RM ? gs[(int64_t)i * sld + c] : gs[(int64_t)c * sld + i]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = ly + 8 * u;
      if (SRC_RM) tile[b][lx] = v[u];
      else tile[lx][b] = v[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = ly + 8 * u;
      const int ti = SRC_RM ? lx : b, tc = SRC_RM ? b : lx;
      const int i = r0 + ti, c = k0 + tc;
      if (i < m && c < nc) {
        if (SRC_RM) gd[(int64_t)c * dld + i] = tile[ti][tc];
        else gd[(int64_t)i * dld + c] = tile[ti][tc];
      }
    }
    __syncthreads();
  }
}

static dim3 node_grid(int count) {
  int g = (1024 + count - 1) / count;
  g = g < 1 ? 1 : (g > 64 ? 64 : g);
  return dim3(count, g);
}

__device__ __forceinline__ const double* cdp(const LevelArgs& a, int64_t off) { return a.dpool + off; }
__device__ __forceinline__ double* dp(const LevelArgs& a, int64_t off) { return a.dpool + off; }
__device__ __forceinline__ const double* ctp(const LevelArgs& a, int64_t off) { return a.tpool + off; }
__device__ __forceinline__ double* tp(const LevelArgs& a, int64_t off) { return a.tpool + off; }

// ------------------------------------------------------------------ plan
__global__ void k_plan(LevelArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count) return;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  NodeState& st = a.st[g];
  const ProbDev& P = a.prob[nd.prob];
  st.active = 0;
  st.extract = 0;
  st.go = 0;
  st.test = 0;
  st.need[0] = st.need[1] = 0;
  st.nc = 0;
  st.reo = 0;
  if (P.done) return;
  if (st.state == COMPRESSED && nd.parent < 0) return;
  const bool kids = nd.leaf || (a.st[nd.left].state == COMPRESSED && a.st[nd.right].state == COMPRESSED);
  if (!kids) return;
  st.fresh = st.state == UNTOUCHED;
  st.extract = st.fresh;
  if (nd.parent < 0) {  // root: extraction, then COMPRESSED
    st.go = 1;
    return;
  }
  st.active = 1;
  st.c0 = st.fresh ? 0 : P.d - P.b;
  st.nc = P.d - st.c0;
  for (int s = 0; s < 2; ++s)
    st.m[s] = nd.leaf ? (nd.hi - nd.lo) : a.st[nd.left].rank[s] + a.st[nd.right].rank[s];
  if (P.symmetric) st.m[1] = st.m[0];
  // the level's largest column count and row count size its GEMM launches
  atomicMax(a.flags + 5, st.nc);
  atomicMax(a.flags + 6, max(st.m[0], st.m[1]));
  st.test = st.state != COMPRESSED;
  if (!st.test) return;
  if (st.fresh) {
    for (int s = 0; s < 2; ++s) {
      st.passed[s] = 0;
      st.q[s] = 0;
      st.rho[s] = -1.0;
      st.rank[s] = 0;
    }
  }
  // Alg. 5 runs over the sampling blocks not yet tested: all of them the
  // first time a node is tested, afterwards only the newest one.
  st.tb = st.fresh ? 0 : P.nsched - 1;
  st.nblk = (st.fresh ? P.nsched : 1);
  if (P.strategy != HSS_DBL_HMT && !P.force && st.nc > 0) {
    for (int s = 0; s < 2; ++s) st.need[s] = !st.passed[s];
    if (st.need[0] || st.need[1]) atomicMax(a.flags + 1, st.nblk);
  }
}

void launch_plan(const LevelArgs& a, hipStream_t s) {
  if (a.count <= 0) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_plan, dim3((a.count + 127) / 128), dim3(128), 0, s, a);
  prof_end(HSS_K_MISC, s);
}

// ------------------------------------------------------------------ extraction
__global__ __launch_bounds__(NB) void k_extract_nodes(LevelArgs a) {
  const int g = a.nodes[blockIdx.x];
  const NodeDesc& nd = a.desc[g];
  const NodeState& st = a.st[g];
  if (!st.extract) return;
  const ProbDev& P = a.prob[nd.prob];
  const GenDev& gen = P.gen;
  if (gen.family == HSS_FAM_CALLBACK) return;   // served by the caller's extraction routine
  int bad = 0;
  if (nd.leaf) {
    const int m = nd.hi - nd.lo;
    double* D = dp(a, nd.D);
    CHUNKED_FOR(idx, (int64_t)m * m) {
      const int i = (int)(idx % m), j = (int)(idx / m);
      const double v = gen_entry(gen, nd.lo + i, nd.lo + j);
      bad |= !isfinite(v);
      D[idx] = v;
    }
  } else {
    const NodeDesc& L = a.desc[nd.left];
    const NodeDesc& Rn = a.desc[nd.right];
    const NodeState& sl = a.st[nd.left];
    const NodeState& sr = a.st[nd.right];
    // B12 = A(left.I^r, right.I^c), B21 = A(right.I^r, left.I^c)
    const int r1 = sl.rank[0], c2 = sr.rank[1];
    const int64_t* I1r = a.lpool + L.I[0];
    const int64_t* I2c = a.lpool + Rn.I[1];
    double* B12 = tp(a, nd.B12);
    CHUNKED_FOR(idx, (int64_t)r1 * c2) {
      const int i = (int)(idx % r1), j = (int)(idx / r1);
      const double v = gen_entry(gen, I1r[i], I2c[j]);
      bad |= !isfinite(v);
      B12[(int64_t)j * nd.b12ld + i] = v;
    }
    const int r2 = sr.rank[0], c1 = sl.rank[1];
    const int64_t* I2r = a.lpool + Rn.I[0];
    const int64_t* I1c = a.lpool + L.I[1];
    double* B21 = tp(a, nd.B21);
    CHUNKED_FOR(idx, (int64_t)r2 * c1) {
      const int i = (int)(idx % r2), j = (int)(idx / r2);
      const double v = gen_entry(gen, I2r[i], I1c[j]);
      bad |= !isfinite(v);
      B21[(int64_t)j * nd.b21ld + i] = v;
    }
  }
  if (bad) atomicOr(a.flags, 1);
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    double ent;
    if (nd.leaf) ent = (double)(nd.hi - nd.lo) * (nd.hi - nd.lo);
    else ent = (double)a.st[nd.left].rank[0] * a.st[nd.right].rank[1] +
               (double)a.st[nd.right].rank[0] * a.st[nd.left].rank[1];
    kcount(a.kcnt, HSS_K_EXTRACT, 8.0 * ent, 0.0);
  }
}

void launch_extract_nodes(const LevelArgs& a, hipStream_t s) {
  if (a.count <= 0) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_extract_nodes, node_grid(a.count), dim3(NB), 0, s, a);
  prof_end(HSS_K_EXTRACT, s);
}

// ------------------------------------------------------------------ local samples
// Copies the first term of ComputeLocalSamples into tau.S(:, c0:c0+nc) and
// writes the GEMM tasks of the product terms (two per node).
__global__ __launch_bounds__(NB) void k_ls_gather(LevelArgs a, int side) {
  const int t = blockIdx.x;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  const NodeState& st = a.st[g];
  GemmTask* T0 = a.tasks + t;
  GemmTask* T1 = a.tasks + a.count + t;
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    T0->M = 0;
    T1->M = 0;
  }
  if (!st.active || st.nc <= 0) return;
  const ProbDev& P = a.prob[nd.prob];
  const int dcap = P.dcap;
  const int c0 = st.c0, nc = st.nc;
  const int m = st.m[side];
  double* S = tp(a, nd.S[side]);
  if (threadIdx.x == 0 && blockIdx.y == 0) kcount(a.kcnt, HSS_K_GATHER, 16.0 * m * nc, 0.0);
  if (nd.leaf) {
    // global samples (column-major) into the node's rows
    const double* Sg = ctp(a, P.sglob[side]);
    copy_transpose<false>(Sg + (int64_t)c0 * P.n + nd.lo, P.n, S + c0, dcap, m, nc);
    if (threadIdx.x == 0 && blockIdx.y == 0 && !P.gen.offdiag) {  // off-diagonal samples need no D R
      GemmTask k;
      k.A = cdp(a, nd.D);
      if (side == 0) { k.a_rs = 1; k.a_cs = m; } else { k.a_rs = m; k.a_cs = 1; }
      k.B = P.R + nd.lo + (int64_t)c0 * P.ldr;
      k.b_rs = 1;
      k.b_cs = P.ldr;
      k.C = S + c0;
      k.c_rs = dcap;
      k.c_cs = 1;
      k.M = m; k.N = nc; k.K = m; k.pad = 0;
      k.alpha = -1.0; k.beta = 1.0;
      *T0 = k;
    }
    return;
  }
  const NodeDesc& L = a.desc[nd.left];
  const NodeDesc& Rn = a.desc[nd.right];
  const NodeState& sl = a.st[nd.left];
  const NodeState& sr = a.st[nd.right];
  const int r1 = sl.rank[side];
  const int32_t* J1 = a.ipool + L.J[side];
  const int32_t* J2 = a.ipool + Rn.J[side];
  const double* S1 = ctp(a, L.S[side]);
  const double* S2 = ctp(a, Rn.S[side]);
  const HSS_GLOBAL int32_t* gJ1 = gview(J1);
  const HSS_GLOBAL int32_t* gJ2 = gview(J2);
  copy_elems(m * nc, [&](int idx) {
    const int c = idx % nc, i = idx / nc;
    const double* src = i < r1 ? S1 + (int64_t)gJ1[i] * dcap : S2 + (int64_t)gJ2[max(i - r1, 0)] * dcap;
    return CopyAt{gview(src + c0 + c), gview_w(S + (int64_t)i * dcap + c0 + c)};
  });
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    GemmTask k;
    k.b_rs = dcap; k.b_cs = 1; k.c_rs = dcap; k.c_cs = 1; k.N = nc; k.pad = 0;
    k.alpha = -1.0; k.beta = 1.0;
    if (side == 0) {
      // [left.S^r(J) - B12 right.R^r ; right.S^r(J) - B21 left.R^r], R^r = V^T R (side-1 basis)
      k.A = ctp(a, nd.B12); k.a_rs = 1; k.a_cs = nd.b12ld;
      k.B = ctp(a, Rn.RR[1]) + c0; k.C = S + c0;
      k.M = sl.rank[0]; k.K = sr.rank[1];
      *T0 = k;
      k.A = ctp(a, nd.B21); k.a_rs = 1; k.a_cs = nd.b21ld;
      k.B = ctp(a, L.RR[1]) + c0; k.C = S + (int64_t)sl.rank[0] * dcap + c0;
      k.M = sr.rank[0]; k.K = sl.rank[1];
      *T1 = k;
    } else {
      // [left.S^c(J) - B21^T right.R^c ; right.S^c(J) - B12^T left.R^c], R^c = U^T R
      k.A = ctp(a, nd.B21); k.a_rs = nd.b21ld; k.a_cs = 1;
      k.B = ctp(a, Rn.RR[0]) + c0; k.C = S + c0;
      k.M = sl.rank[1]; k.K = sr.rank[0];
      *T0 = k;
      k.A = ctp(a, nd.B12); k.a_rs = nd.b12ld; k.a_cs = 1;
      k.B = ctp(a, L.RR[0]) + c0; k.C = S + (int64_t)sl.rank[1] * dcap + c0;
      k.M = sr.rank[1]; k.K = sl.rank[0];
      *T1 = k;
    }
  }
}

void launch_local_samples(const LevelArgs& a, int side, int32_t mcap_max, int32_t rcap_max,
                          int32_t ncap, hipStream_t s) {
  if (a.count <= 0) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_ls_gather, node_grid(a.count), dim3(NB), 0, s, a, side);
  prof_end(HSS_K_GATHER, s);
  launch_gemm(a.tasks, 2 * a.count, mcap_max, ncap, s, a.kcnt, std::max(mcap_max, rcap_max), a.gws,
              kGemmSplitElems);
}

// ------------------------------------------------------------------ F-norm test
// Iteration `iter` of the test tests block tb + iter of the sampling
// schedule, columns [sched[b-1], sched[b]).  A side passes at once when the
// samples up to that block are at least as many as its rows (they span the
// whole local range).
__global__ __launch_bounds__(NB) void k_fn_copy(LevelArgs a, int side, int iter) {
  const int t = blockIdx.x;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  NodeState& st = a.st[g];
  GemmTask* TA = a.tasks + t;
  GemmTask* TB = a.tasks + a.count + t;
  // every workgroup of the node takes the same decision from the state at
  // launch; only the first one writes the state and the GEMM tasks
  const bool first = blockIdx.y == 0;
  int go = 0, c0 = 0, nc = 0;
  if (st.need[side] && !st.passed[side] && iter < st.nblk) {
    const ProbDev& P = a.prob[nd.prob];
    const int b = st.tb + iter;
    const int b0 = b > 0 ? P.sched[b - 1] : 0;
    const int b1 = P.sched[b];
    if (b1 < st.m[side] && b1 > b0) {
      go = 1;
      c0 = b0;
      nc = b1 - b0;
    }
  }
  __syncthreads();
  if (first && threadIdx.x == 0) {
    TA->M = 0;
    TB->M = 0;
    st.run[side] = go;
    if (go) {
      st.bc0 = c0;
      st.bnc = nc;
    } else if (st.need[side] && !st.passed[side] && iter < st.nblk) {
      const ProbDev& P = a.prob[nd.prob];
      if (P.sched[st.tb + iter] >= st.m[side]) st.passed[side] = 1;
    }
  }
  if (!go) return;
  const ProbDev& P = a.prob[nd.prob];
  const int dcap = P.dcap, m = st.m[side], q = st.q[side];
  if (first && threadIdx.x == 0) kcount(a.kcnt, HSS_K_GATHER, 16.0 * m * nc, 0.0);
  const double* S = ctp(a, nd.S[side]);
  double* Sh = a.wsA + nd.ws;
  copy_transpose<true>(S + c0, dcap, Sh, nd.mcap, m, nc);   // node rows into the column-major block
  if (first && threadIdx.x == 0) {
    const double* Q = ctp(a, nd.Q[side]);
    double* W = a.wsB + nd.wsq;
    GemmTask k;
    k.pad = 0;
    // W = Q^T Sh
    k.A = Q; k.a_rs = nd.mcap; k.a_cs = 1;
    k.B = Sh; k.b_rs = 1; k.b_cs = nd.mcap;
    k.C = W; k.c_rs = 1; k.c_cs = nd.qcap;
    k.M = q; k.N = nc; k.K = m; k.alpha = 1.0; k.beta = 0.0;
    *TA = k;
    // Sh -= Q W
    k.A = Q; k.a_rs = 1; k.a_cs = nd.mcap;
    k.B = W; k.b_rs = 1; k.b_cs = nd.qcap;
    k.C = Sh; k.c_rs = 1; k.c_cs = nd.mcap;
    k.M = m; k.N = nc; k.K = q; k.alpha = -1.0; k.beta = 1.0;
    *TB = k;
  }
}

// The F-norm tests of eq. stopping_criteria on the projected block Sh
// (m x nc, column-major, ld mcap): pass if ||Sh|| < eps_r ||S_new|| or
// ||Sh|| / sqrt(nc) < eps_a; otherwise queue the Householder QR of Sh.
constexpr int NBN = 1024;  // threads of the norm kernel (one workgroup per node)

// Sums of squares of the block under test S(:, c0:c0+nc) and of its
// projection S_hat over contiguous chunks of the elements, one chunk per
// workgroup of the node (the chunk count capped by the node's slot of
// workspace B, free between the projection GEMMs and the QR); k_fn_norms
// adds the chunks in order.
constexpr int NBP = 256;
__device__ __forceinline__ int fn_chunks(const NodeDesc& nd, const ProbDev& P, int grid) {
  return min(grid, 8 + nd.mcap + P.dcap);
}

__global__ __launch_bounds__(NBP) void k_fn_partial(LevelArgs a, int side) {
  __shared__ double red[NBP / 64];
  const int t = blockIdx.x;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  const NodeState& st = a.st[g];
  if (!st.run[side]) return;
  const ProbDev& P = a.prob[nd.prob];
  const int nch = fn_chunks(nd, P, gridDim.y);
  if ((int)blockIdx.y >= nch) return;
  const int dcap = P.dcap, m = st.m[side], nc = st.bnc, c0 = st.bc0, ld = nd.mcap;
  const int tot = m * nc;
  const int per = (tot + nch - 1) / nch;
  const int e0 = blockIdx.y * per, e1 = min(tot, e0 + per);
  const HSS_GLOBAL double* gS = gview(ctp(a, nd.S[side]));
  const HSS_GLOBAL double* gSh = gview(a.wsA + nd.ws);
  // S rows are contiguous over the columns, S_hat columns over the rows;
  // each thread loads NU entries before it adds them
  constexpr int NU = 8;
  double p1 = 0.0, p2 = 0.0;
  for (int base = e0 + threadIdx.x; base < e1; base += NBP * NU) {
    double x[NU], y[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int idx = min(base + u * NBP, e1 - 1);
      const int c = idx % nc, i = idx / nc;
      x[u] = gS[(int64_t)i * dcap + c0 + c];
      const int i2 = idx % m, c2 = idx / m;
      y[u] = gSh[(int64_t)c2 * ld + i2];
    }
#pragma unroll
    for (int u = 0; u < NU; ++u)
      if (base + u * NBP < e1) {
        p1 += x[u] * x[u];
        p2 += y[u] * y[u];
      }
  }
  p1 = block_sum_n<NBP>(p1, red);
  p2 = block_sum_n<NBP>(p2, red);
  if (threadIdx.x == 0) {
    HSS_GLOBAL double* part = gview_w(a.wsB + nd.wsq);
    part[2 * blockIdx.y] = p1;
    part[2 * blockIdx.y + 1] = p2;
  }
}

__global__ __launch_bounds__(NBN) void k_fn_norms(LevelArgs a, int side, QrcpTask* __restrict__ qt,
                                                 CholTask* __restrict__ ct, int chunk_grid) {
  __shared__ double red[NBN / 64];
  const int t = blockIdx.x;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  NodeState& st = a.st[g];
  if (threadIdx.x == 0) {
    qt[t].active = 0;
    ct[t].active = 0;
    a.tasks[t].M = 0;
  }
  if (!st.run[side]) return;
  const ProbDev& P = a.prob[nd.prob];
  const int dcap = P.dcap, m = st.m[side], nc = st.bnc, c0 = st.bc0, ld = nd.mcap;
  const double lev = (double)nd.level;
  const double er = fmax(P.eps_r / lev, P.eps_floor), ea = P.eps_a / lev;
  double* Sh = a.wsA + nd.ws;
  const HSS_GLOBAL double* gSh = gview(Sh);
  const bool hmt = P.strategy == HSS_INC_HMT;
  double cmax = 0.0;
  if (hmt) {
    // eq. HMT_IQQH: the largest column norm of S_hat, one wave per column
    // (sums in lane order), the maximum over the waves
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double wmax = 0.0;
    for (int c = wv; c < nc; c += NBN / 64) {
      double s2 = 0.0;
      for (int i = lane; i < m; i += 64) {
        const double v = gSh[(int64_t)c * ld + i];
        s2 += v * v;
      }
      wmax = fmax(wmax, sqrt(wave_sum(s2)));
    }
    if (lane == 0) red[wv] = wmax;
    __syncthreads();
    for (int w = 0; w < NBN / 64; ++w) cmax = fmax(cmax, red[w]);
  }
  if (threadIdx.x != 0) return;
  kcount(a.kcnt, HSS_K_TEST_NORMS, 16.0 * m * nc, 4.0 * m * nc);
  double p1 = 0.0, p2 = 0.0;   // the chunks of k_fn_partial, in order
  {
    const HSS_GLOBAL double* part = gview(a.wsB + nd.wsq);
    const int nch = fn_chunks(nd, P, chunk_grid);
    for (int y = 0; y < nch; ++y) {
      p1 += part[2 * y];
      p2 += part[2 * y + 1];
    }
  }
  const double nS = sqrt(p1), nSh = sqrt(p2);
  const bool pass = hmt ? (nS == 0.0 || P.hmt_alpha * sqrt(2.0 / kPi) * cmax <= ea)
                        : (nS == 0.0 || nSh < er * nS || nSh / sqrt((double)nc) < ea);
  if (pass) {
    st.passed[side] = 1;
    st.run[side] = 0;
    return;
  }
  QrcpTask q;
  q.S = Sh; q.lds = ld; q.W = Sh; q.ldw = ld;
  q.scr = a.wsB + nd.wsq;
  q.J = nullptr; q.E = nullptr; q.lde = 1;
  q.rank_out = &st.qrank;
  q.er = 0.0; q.ea = 0.0; q.hmt_mn = 0.0;
  q.m = nc; q.d = m; q.mcap = nc; q.active = 1;
  q.nopivot = 1;
  qt[t] = q;
  // Cholesky QR first when the block is narrow and the node's workspace
  // slot (mcap x dcap) holds S_hat, Q1, G, X and d1 side by side
  const int64_t blk = ((int64_t)ld * nc + 7) / 8 * 8;
  const int64_t sq = (int64_t)nc * nc;
  // (the HMT-lemma test appends every failing block: Householder path)
  if (!hmt && nc <= kCholMaxB && 2 * blk + 2 * sq + nc + 16 <= (int64_t)ld * dcap) {
    CholTask c;
    c.S = Sh; c.lds = ld;
    c.Q1 = Sh + blk;
    c.G = Sh + 2 * blk;
    c.X = c.G + sq;
    c.d1 = c.X + sq;
    c.m = m; c.nc = nc; c.active = 1; c.pad = 0;
    ct[t] = c;
    GemmTask k;   // G = S_hat^T S_hat
    k.A = Sh; k.a_rs = ld; k.a_cs = 1;
    k.B = Sh; k.b_rs = 1; k.b_cs = ld;
    k.C = c.G; k.c_rs = 1; k.c_cs = nc;
    k.M = nc; k.N = nc; k.K = m; k.pad = 0;
    k.alpha = 1.0; k.beta = 0.0;
    a.tasks[t] = k;
  }
}

// One Cholesky pass of the test's block: R^T R = G (upper R in LDS),
// X = R^{-1}.  Pass 1: keep diag(R1), queue Q1 = S_hat X and G2 = Q1^T Q1.
// Pass 2: Rbar = R2 R1 decides the R-diagonal tests of eq.
// stopping_criteria when the block clearly fails them (min |Rbar_ii| at
// least 10 times the threshold) and Q1 was nearly orthonormal (|R2_ii - 1|
// <= 0.1); then Q = Q1 X2 is appended to the basis and the Householder QR
// of the block is skipped.  Anything else is left to the Householder path.
//
// 16 waves per node: thread (row group ib, column j) updates the rows ib,
// ib + CRG, ... of column j, at most CRW of them per step, unrolled so that
// their LDS reads are in flight together.  NB is the widest block the
// instance takes (64, or 128 for the first blocks of a replay, d0 wide);
// the NB x NB factor lives in dynamic LDS (about 130 KB at 128).
constexpr int CHT = 1024;               // threads of the Cholesky kernel

template <int NB>
constexpr size_t cq_lds_bytes() { return sizeof(double) * (size_t)NB * (NB + 1); }

template <int PASS, int NB>
__global__ __launch_bounds__(CHT) void k_cq_chol(LevelArgs a, int side, CholTask* __restrict__ ct,
                                                 QrcpTask* __restrict__ qt) {
  constexpr int CRG = CHT / NB;   // row groups
  constexpr int CRW = NB / CRG;   // rows per thread and step
  extern __shared__ double cq_lds[];
  double (*A)[NB + 1] = reinterpret_cast<double (*)[NB + 1]>(cq_lds);
  const int t = blockIdx.x;
  GemmTask* T0 = a.tasks + t;
  GemmTask* T1 = a.tasks + a.count + t;
  if (threadIdx.x == 0) {
    T0->M = 0;
    T1->M = 0;
  }
  CholTask& c = ct[t];
  if (!c.active) return;
  const int nc = c.nc;
  if (nc > NB) return;   // cannot happen: the launch takes the widest block
  const int j = threadIdx.x % NB, ib = threadIdx.x / NB;
  {
    const HSS_GLOBAL double* G = gview(c.G);
    double gv[CRW];
#pragma unroll
    for (int u = 0; u < CRW; ++u) gv[u] = G[(int64_t)min(j, nc - 1) * nc + min(ib + CRG * u, nc - 1)];
#pragma unroll
    for (int u = 0; u < CRW; ++u)
      if (j < nc && ib + CRG * u < nc) A[ib + CRG * u][j] = gv[u];
  }
  __syncthreads();
  // outer-product Cholesky on the unscaled rows: after step k the trailing
  // block holds G - sum_{p<=k} r_p^T r_p with r_p = A(p, p:) / sqrt(A(p,p))
  bool bad = false;
  for (int k = 0; k < nc; ++k) {
    const double dk = A[k][k];
    if (!(dk > 0.0)) {
      bad = true;
      break;
    }
    if (j > k && j < nc) {
      const double akj = A[k][j] / dk;
#pragma unroll
      for (int u = 0; u < CRW; ++u) {
        const int i = k + 1 + ib + CRG * u;
        const int ic = min(i, NB - 1);
        const double v = A[ic][j] - A[k][ic] * akj;
        if (i <= j) A[ic][j] = v;
      }
    }
    __syncthreads();
  }
  if (bad) {
    if (threadIdx.x == 0) c.active = 0;
    return;
  }
  // R(i, j) = A(i, j) / sqrt(A(i, i)); diag(R) kept apart for the inversion
  __shared__ double dR[NB];
  for (int i = threadIdx.x; i < nc; i += CHT) dR[i] = sqrt(A[i][i]);
  __syncthreads();
  if (j < nc)
    for (int i = ib; i <= j && i < nc; i += CRG) A[i][j] /= dR[i];
  __syncthreads();
  // X = R^{-1} by right-looking back substitution of R X = I, bottom row
  // first: R stays in the upper triangle of A, the right-hand side B(p, q)
  // (p < q) is kept transposed in the lower triangle (A[q][p]).  At step k
  // row k of B is final: the threads of column q form X(k, q) =
  // B(k, q) / R(k, k) (B(k, k) = 1), write it out and update the rows
  // p < k of their column, so a step reads and writes disjoint entries and
  // needs one barrier.
  __shared__ double rinv[NB];
  for (int i = threadIdx.x; i < nc; i += CHT) rinv[i] = 1.0 / dR[i];
  if (j < nc)
    for (int i = ib; i < j; i += CRG) A[j][i] = 0.0;
  HSS_GLOBAL double* X = gview_w(c.X);
  if (j < nc)
    for (int i = j + 1 + ib; i < nc; i += CRG) X[(int64_t)j * nc + i] = 0.0;   // below the diagonal
  __syncthreads();
  for (int k = nc - 1; k >= 0; --k) {
    // B(p, q) -= R(p, k) X(k, q) for p < k, q >= k: thread (ib, j) takes
    // column q = j and the rows p = ib + 16u
    if (j >= k && j < nc) {
      const double xkq = j == k ? rinv[k] : A[j][k] * rinv[k];
      if (ib == 0) X[(int64_t)j * nc + k] = xkq;
#pragma unroll
      for (int u = 0; u < CRW; ++u) {
        const int p = ib + CRG * u;
        const double v = A[j][p] - A[p][k] * xkq;
        if (p < k) A[j][p] = v;
      }
    }
    __syncthreads();
  }
  if constexpr (PASS == 1) {
    for (int i = threadIdx.x; i < nc; i += CHT) gview_w(c.d1)[i] = dR[i];
    if (threadIdx.x == 0) {
      GemmTask k;
      k.pad = 0;
      k.A = c.S; k.a_rs = 1; k.a_cs = c.lds;     // Q1 = S_hat X
      k.B = c.X; k.b_rs = 1; k.b_cs = nc;
      k.C = c.Q1; k.c_rs = 1; k.c_cs = c.lds;
      k.M = c.m; k.N = nc; k.K = nc; k.alpha = 1.0; k.beta = 0.0;
      *T0 = k;
      k.A = c.Q1; k.a_rs = c.lds; k.a_cs = 1;    // G2 = Q1^T Q1
      k.B = c.Q1; k.b_rs = 1; k.b_cs = c.lds;
      k.C = c.G; k.c_rs = 1; k.c_cs = nc;
      k.M = nc; k.N = nc; k.K = c.m; k.alpha = 1.0; k.beta = 0.0;
      *T1 = k;
    }
  } else {
    // diag(R1) of the first pass, loaded by all threads at once
    __shared__ double d1[NB];
    for (int i = threadIdx.x; i < nc; i += CHT) d1[i] = gview(c.d1)[i];
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int g = a.nodes[t];
    const NodeDesc& nd = a.desc[g];
    NodeState& st = a.st[g];
    const ProbDev& P = a.prob[nd.prob];
    const double lev = (double)nd.level;
    const double er = fmax(P.eps_r / lev, P.eps_floor), ea = P.eps_a / lev;
    double mn = INFINITY, dev = 0.0;
    for (int i = 0; i < nc; ++i) {
      mn = fmin(mn, fabs(dR[i] * d1[i]));
      dev = fmax(dev, fabs(dR[i] - 1.0));
    }
    const double rho = st.rho[side] < 0.0 ? fabs(dR[0] * d1[0]) : st.rho[side];
    const double thr = fmax(ea, er * rho);
    c.active = 0;
    // decide only away from the threshold (rounding of either QR is ~1e-16
    // of the block's norm, the thresholds ~1e-9 of it or more)
    if (!(dev <= 0.1) || !(mn >= 1.5 * thr || mn < thr / 1.5)) return;   // Householder decides
    st.rho[side] = rho;
    st.run[side] = 0;
    qt[t].active = 0;
    if (mn < thr / 1.5) {   // an R-diagonal test passes: no basis growth
      st.passed[side] = 1;
      return;
    }
    double* Qd = tp(a, nd.Q[side]) + (int64_t)st.q[side] * nd.mcap;
    st.q[side] += nc;
    GemmTask k;   // Q(:, q:q+nc) = Q1 X2
    k.pad = 0;
    k.A = c.Q1; k.a_rs = 1; k.a_cs = c.lds;
    k.B = c.X; k.b_rs = 1; k.b_cs = nc;
    k.C = Qd; k.c_rs = 1; k.c_cs = nd.mcap;
    k.M = c.m; k.N = nc; k.K = nc; k.alpha = 1.0; k.beta = 0.0;
    *T0 = k;
    kcount(a.kcnt, HSS_K_TEST_NORMS, 8.0 * 4.0 * nc * nc, 2.0 * nc * nc * nc);
  }
}

// R-diagonal tests of eq. stopping_criteria after the QR of the projected
// block: pass if min |Rbar_ii| < eps_a or < eps_r rho (rho = |Rbar_11| of the
// first block QR'd on this side); otherwise queue Q_k for Q <- [Q Q_k].
__global__ void k_fn_rtest(LevelArgs a, int side, QformTask* __restrict__ qf) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count) return;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  NodeState& st = a.st[g];
  qf[t].active = 0;
  if (!st.run[side]) return;
  const ProbDev& P = a.prob[nd.prob];
  const int m = st.m[side], nc = st.bnc;
  const double lev = (double)nd.level;
  const double er = fmax(P.eps_r / lev, P.eps_floor), ea = P.eps_a / lev;
  const double* rdiag = a.wsB + nd.wsq + 16 + 2 * (int64_t)nc;
  const int r = st.qrank;
  double mn = r < nc ? 0.0 : INFINITY;
  for (int k = 0; k < r; ++k) mn = fmin(mn, fabs(rdiag[k]));
  if (st.rho[side] < 0.0) st.rho[side] = r > 0 ? fabs(rdiag[0]) : 0.0;
  st.run[side] = 0;
  const bool hmt = P.strategy == HSS_INC_HMT;   // no R-diagonal tests there
  if (r < nc || (!hmt && (mn < ea || mn < er * st.rho[side]))) {  // an exactly zero Rbar_ii also passes
    st.passed[side] = 1;
    return;
  }
  if (hmt) st.reo = side + 1;
  QformTask f;
  f.W = a.wsA + nd.ws; f.ldw = nd.mcap;
  f.rdiag = rdiag;
  f.Q = tp(a, nd.Q[side]) + (int64_t)st.q[side] * nd.mcap; f.ldq = nd.mcap;
  f.m = m; f.nc = nc; f.active = 1; f.pad = 0;
  // compact WY formation needs 2 nc^2 doubles: the node's workspace slot
  // (mcap x dcap) holds the block in its first nc columns
  const int64_t used = ((int64_t)nd.mcap * nc + 7) / 8 * 8;
  const int64_t room = (int64_t)nd.mcap * P.dcap - used;
  f.wk = (mn > 0.0 && room >= 2 * (int64_t)nc * nc + 8) ? a.wsA + nd.ws + used : nullptr;
  qf[t] = f;
  st.q[side] += nc;
}

// HMT-lemma test, after a failing block's Q_k was appended at columns
// q - nc .. q of Q: columns of S_hat at rounding level give directions of
// Q_k that are not orthogonal to the earlier basis once normalised.  Q_k
// is projected off the earlier basis twice more (GEMM tasks as in
// k_fn_copy) and factored again; the second Q replaces Q_k.
__global__ __launch_bounds__(NB) void k_hmt_reo_copy(LevelArgs a, int side) {
  const int t = blockIdx.x;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  const NodeState& st = a.st[g];
  GemmTask* TA = a.tasks + t;
  GemmTask* TB = a.tasks + a.count + t;
  const bool first = blockIdx.y == 0;
  if (first && threadIdx.x == 0) {
    TA->M = 0;
    TB->M = 0;
  }
  if (st.reo != side + 1) return;
  const int m = st.m[side], nc = st.bnc, q0 = st.q[side] - nc;
  const double* Q = ctp(a, nd.Q[side]);
  double* Sh = a.wsA + nd.ws;
  copy_elems(m * nc, [&](int idx) {
    const int i = idx % m, c = idx / m;
    return CopyAt{gview(Q + (int64_t)(q0 + c) * nd.mcap + i), gview_w(Sh + (int64_t)c * nd.mcap + i)};
  });
  if (first && threadIdx.x == 0) {
    double* W = a.wsB + nd.wsq;
    GemmTask k;
    k.pad = 0;
    k.A = Q; k.a_rs = nd.mcap; k.a_cs = 1;     // W = Q(:, 0:q0)^T Sh
    k.B = Sh; k.b_rs = 1; k.b_cs = nd.mcap;
    k.C = W; k.c_rs = 1; k.c_cs = nd.qcap;
    k.M = q0; k.N = nc; k.K = m; k.alpha = 1.0; k.beta = 0.0;
    *TA = k;
    k.A = Q; k.a_rs = 1; k.a_cs = nd.mcap;     // Sh -= Q(:, 0:q0) W
    k.B = W; k.b_rs = 1; k.b_cs = nd.qcap;
    k.C = Sh; k.c_rs = 1; k.c_cs = nd.mcap;
    k.M = m; k.N = nc; k.K = q0; k.alpha = -1.0; k.beta = 1.0;
    *TB = k;
    kcount(a.kcnt, HSS_K_GATHER, 16.0 * m * nc, 0.0);
  }
}

// Householder QR (no pivoting) of the re-projected block.
__global__ void k_hmt_reo_qr(LevelArgs a, int side, QrcpTask* __restrict__ qt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count) return;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  NodeState& st = a.st[g];
  qt[t].active = 0;
  if (st.reo != side + 1) return;
  double* Sh = a.wsA + nd.ws;
  const int ld = nd.mcap;
  QrcpTask q;
  q.S = Sh; q.lds = ld; q.W = Sh; q.ldw = ld;
  q.scr = a.wsB + nd.wsq;
  q.J = nullptr; q.E = nullptr; q.lde = 1;
  q.rank_out = &st.qrank;
  q.er = 0.0; q.ea = 0.0; q.hmt_mn = 0.0;
  q.m = st.bnc; q.d = st.m[side]; q.mcap = st.bnc; q.active = 1;
  q.nopivot = 1;
  qt[t] = q;
}

// Explicit Q of that QR over Q_k's columns; the re-orthogonalization ends.
__global__ void k_hmt_reo_form(LevelArgs a, int side, QformTask* __restrict__ qf) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count) return;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  NodeState& st = a.st[g];
  qf[t].active = 0;
  if (st.reo != side + 1) return;
  st.reo = 0;
  const ProbDev& P = a.prob[nd.prob];
  const int m = st.m[side], nc = st.bnc;
  if (st.qrank < nc) return;   // cannot happen for orthonormal input; Q_k is kept then
  QformTask f;
  f.W = a.wsA + nd.ws; f.ldw = nd.mcap;
  f.rdiag = a.wsB + nd.wsq + 16 + 2 * (int64_t)nc;
  f.Q = tp(a, nd.Q[side]) + (int64_t)(st.q[side] - nc) * nd.mcap; f.ldq = nd.mcap;
  f.m = m; f.nc = nc; f.active = 1; f.pad = 0;
  const int64_t used = ((int64_t)nd.mcap * nc + 7) / 8 * 8;
  const int64_t room = (int64_t)nd.mcap * P.dcap - used;
  f.wk = room >= 2 * (int64_t)nc * nc + 8 ? a.wsA + nd.ws + used : nullptr;
  qf[t] = f;
}

void launch_fnorm_test(const LevelArgs& a, int side, int32_t iter, int32_t mcap_max, int32_t qcap_max,
                       int32_t ncap, const TestScratch& ts, hipStream_t s, bool hmt) {
  if (a.count <= 0) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_fn_copy, node_grid(a.count), dim3(NB), 0, s, a, side, iter);
  prof_end(HSS_K_GATHER, s);
  for (int pass = 0; pass < 2; ++pass) {  // block Gram-Schmidt, twice
    launch_gemm(a.tasks, a.count, qcap_max, ncap, s, a.kcnt, mcap_max, a.gws, kGemmSplitElems);
    launch_gemm(a.tasks + a.count, a.count, mcap_max, ncap, s, a.kcnt, qcap_max, a.gws, kGemmSplitElems);
  }
  // chunks per node: about 2048 workgroups in all, at most 64 per node
  const int chunk_grid = std::max(1, std::min(64, 2048 / std::max(a.count, 1)));
  prof_begin(s);
  hipLaunchKernelGGL(k_fn_partial, dim3(a.count, chunk_grid), dim3(NBP), 0, s, a, side);
  hipLaunchKernelGGL(k_fn_norms, dim3(a.count), dim3(NBN), 0, s, a, side, ts.qt, ts.ct, chunk_grid);
  prof_end(HSS_K_TEST_NORMS, s);
  // Cholesky QR of the narrow blocks: decides the clearly failing tests
  const int32_t nb = std::min(ncap, kCholMaxB);
  static thread_local bool cq_attr = false;   // dynamic LDS above 64 KB
  if (!cq_attr) {
    HSS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cq_chol<1, 128>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)cq_lds_bytes<128>()));
    HSS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cq_chol<2, 128>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)cq_lds_bytes<128>()));
    cq_attr = true;
  }
  auto cq = [&](int pass) {
    if (nb <= 64) {
      if (pass == 1) hipLaunchKernelGGL((k_cq_chol<1, 64>), dim3(a.count), dim3(CHT), cq_lds_bytes<64>(), s, a, side, ts.ct, ts.qt);
      else hipLaunchKernelGGL((k_cq_chol<2, 64>), dim3(a.count), dim3(CHT), cq_lds_bytes<64>(), s, a, side, ts.ct, ts.qt);
    } else {
      if (pass == 1) hipLaunchKernelGGL((k_cq_chol<1, 128>), dim3(a.count), dim3(CHT), cq_lds_bytes<128>(), s, a, side, ts.ct, ts.qt);
      else hipLaunchKernelGGL((k_cq_chol<2, 128>), dim3(a.count), dim3(CHT), cq_lds_bytes<128>(), s, a, side, ts.ct, ts.qt);
    }
  };
  launch_gemm(a.tasks, a.count, nb, nb, s, a.kcnt, mcap_max, a.gws, kGemmSplitElems);
  prof_begin(s);
  cq(1);
  prof_end(HSS_K_TEST_NORMS, s);
  launch_gemm(a.tasks, a.count, mcap_max, nb, s, a.kcnt);
  launch_gemm(a.tasks + a.count, a.count, nb, nb, s, a.kcnt, mcap_max, a.gws, kGemmSplitElems);
  prof_begin(s);
  cq(2);
  prof_end(HSS_K_TEST_NORMS, s);
  launch_gemm(a.tasks, a.count, mcap_max, nb, s, a.kcnt);
  run_qrcp(ts.qt, a.count, ts.wk, nullptr, 0, ncap, mcap_max, ncap, ts.flag, ts.gt, mcap_max, s, a.kcnt, false);
  prof_begin(s);
  hipLaunchKernelGGL(k_fn_rtest, dim3((a.count + 127) / 128), dim3(128), 0, s, a, side, ts.qf);
  prof_end(HSS_K_TEST_NORMS, s);
  run_qform(ts.qf, a.count, ts.wg, ts.nwg, ts.cpw, ncap, mcap_max, ts.gt, a.gws, s, a.kcnt);
  if (!hmt) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_hmt_reo_copy, node_grid(a.count), dim3(NB), 0, s, a, side);
  prof_end(HSS_K_GATHER, s);
  for (int pass = 0; pass < 2; ++pass) {
    launch_gemm(a.tasks, a.count, qcap_max, ncap, s, a.kcnt, mcap_max, a.gws, kGemmSplitElems);
    launch_gemm(a.tasks + a.count, a.count, mcap_max, ncap, s, a.kcnt, qcap_max, a.gws, kGemmSplitElems);
  }
  prof_begin(s);
  hipLaunchKernelGGL(k_hmt_reo_qr, dim3((a.count + 127) / 128), dim3(128), 0, s, a, side, ts.qt);
  prof_end(HSS_K_TEST_NORMS, s);
  run_qrcp(ts.qt, a.count, ts.wk, nullptr, 0, ncap, mcap_max, ncap, ts.flag, ts.gt, mcap_max, s, a.kcnt, false);
  prof_begin(s);
  hipLaunchKernelGGL(k_hmt_reo_form, dim3((a.count + 127) / 128), dim3(128), 0, s, a, side, ts.qf);
  prof_end(HSS_K_TEST_NORMS, s);
  run_qform(ts.qf, a.count, ts.wg, ts.nwg, ts.cpw, ncap, mcap_max, ts.gt, a.gws, s, a.kcnt);
}

// `unexpected` (when not null): the host skips this level's ID because no
// node ran a test and none is forced, so none can pass; a node that does
// is reported there.
__global__ void k_decide_fnorm(LevelArgs a, int32_t* unexpected) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count) return;
  const int g = a.nodes[t];
  NodeState& st = a.st[g];
  if (!st.active || !st.test) return;
  const ProbDev& P = a.prob[a.desc[g].prob];
  const bool ok = st.passed[0] && (P.symmetric || st.passed[1]);
  st.go = (ok || P.force) ? 1 : 0;
  if (st.go && unexpected) atomicOr(unexpected, 1);
}

void launch_decide_fnorm(const LevelArgs& a, hipStream_t s, int32_t* unexpected) {
  if (a.count <= 0) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_decide_fnorm, dim3((a.count + 127) / 128), dim3(128), 0, s, a, unexpected);
  prof_end(HSS_K_MISC, s);
}

// ------------------------------------------------------------------ QRCP / ID
// One QrcpTask per node of the level: the node's side-`side` local sample
// (m x d), its workspace slots and thresholds eta*eps/level(tau).  Nodes
// that do not compress this round get active = 0.
__global__ void k_build_qrcp(LevelArgs a, int side, int hmt, QrcpTask* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count) return;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  NodeState& st = a.st[g];
  const ProbDev& P = a.prob[nd.prob];
  QrcpTask q;
  q.active = st.active && st.test && (hmt || st.go);
  q.S = a.tpool + nd.S[side];
  q.lds = P.dcap;
  q.W = a.wsA + nd.ws;
  q.ldw = P.dcap;
  q.scr = a.wsB + nd.wsq;
  q.J = a.ipool + nd.J[side];
  q.E = a.tpool + nd.E[side];
  q.lde = nd.rcap;
  q.rank_out = &st.rank[side];
  const double lev = (double)nd.level;
  q.er = fmax(P.eps_r / lev, P.eps_floor);
  q.ea = P.eps_a / lev;
  const int64_t size = nd.hi - nd.lo;
  q.hmt_mn = hmt ? (double)min(size, P.n - size) : 0.0;
  q.m = st.m[side];
  q.d = P.d;
  q.mcap = nd.mcap;
  q.nopivot = 0;
  out[t] = q;
}

void launch_build_qrcp(const LevelArgs& a, int side, int32_t hmt, QrcpTask* out, hipStream_t s) {
  if (a.count <= 0) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_build_qrcp, dim3((a.count + 127) / 128), dim3(128), 0, s, a, side, hmt, out);
  prof_end(HSS_K_MISC, s);
}

__global__ void k_decide_hmt(LevelArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count) return;
  const int g = a.nodes[t];
  NodeState& st = a.st[g];
  if (!st.active || !st.test) return;
  const ProbDev& P = a.prob[a.desc[g].prob];
  bool ok = true;
  for (int s = 0; s < (P.symmetric ? 1 : 2); ++s)
    ok = ok && (st.rank[s] < P.d - P.p || st.rank[s] == st.m[s]);
  st.go = (ok || P.force) ? 1 : 0;
}

void launch_decide_hmt(const LevelArgs& a, hipStream_t s) {
  if (a.count <= 0) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_decide_hmt, dim3((a.count + 127) / 128), dim3(128), 0, s, a);
  prof_end(HSS_K_MISC, s);
}

// ------------------------------------------------------------------ reduce
// RR[side](:, cols) = U_side^T X(:, cols) = X(J,:) + E X(rest,:), X = R(I_tau)
// on a leaf or the stacked children's RR[side]; skeleton indices on compression.
__global__ __launch_bounds__(NB) void k_red_gather(LevelArgs a, int side) {
  const int t = blockIdx.x;
  const int g = a.nodes[t];
  const NodeDesc& nd = a.desc[g];
  const NodeState& st = a.st[g];
  GemmTask* T0 = a.tasks + t;
  if (threadIdx.x == 0 && blockIdx.y == 0) T0->M = 0;
  if (!st.active) return;
  if (!(st.state == COMPRESSED || st.go)) return;
  const ProbDev& P = a.prob[nd.prob];
  const int dcap = P.dcap;
  const int c0 = st.go ? 0 : st.c0;
  const int nc = P.d - c0;
  const int m = st.m[side], r = st.rank[side];
  const int32_t* J = a.ipool + nd.J[side];
  double* RR = tp(a, nd.RR[side]);
  if (threadIdx.x == 0 && blockIdx.y == 0) kcount(a.kcnt, HSS_K_GATHER, 16.0 * m * nc, 0.0);
  double* Xr = a.wsA + nd.ws;  // (m - r) x nc, column-major, ld = mcap
  int r1 = 0;
  const double *X1 = nullptr, *X2 = nullptr;
  if (!nd.leaf) {
    r1 = a.st[nd.left].rank[side];
    X1 = ctp(a, a.desc[nd.left].RR[side]);
    X2 = ctp(a, a.desc[nd.right].RR[side]);
  }
  // Rows J of the random block, m x nc, through 32 x 32 LDS tiles: a
  // leaf's source is R (column-major: loaded along the rows), a parent's
  // its children's reduced blocks (row-major: loaded along the columns);
  // rows below r go to RR (row-major: stored along the columns), the rest
  // to Xr (column-major: stored along the rows).
  {
    __shared__ double tile[32][33];
    const HSS_GLOBAL int32_t* gJ = gview(J);
    const HSS_GLOBAL double* gR = gview(P.R);
    const HSS_GLOBAL double* gX1 = gview(X1);
    const HSS_GLOBAL double* gX2 = gview(X2);
    HSS_GLOBAL double* gRR = gview_w(RR);
    HSS_GLOBAL double* gXr = gview_w(Xr);
    const int tr = (m + 31) / 32, tcn = (nc + 31) / 32;
    const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;   // NB = 256: 32 x 8
    for (int tt = blockIdx.y; tt < tr * tcn; tt += gridDim.y) {
      const int r0 = (tt % tr) * 32, k0 = (tt / tr) * 32;
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = ly + 8 * u;
        const int ti = nd.leaf ? lx : b, tc = nd.leaf ? b : lx;
        const int i = r0 + ti, c = k0 + tc;
        const int row = gJ[min(i, m - 1)];
        const int64_t cc = c0 + min(c, nc - 1);
        double x;
        if (nd.leaf) x = gR[cc * P.ldr + nd.lo + row];
        else x = row < r1 ? gX1[(int64_t)row * dcap + cc] : gX2[(int64_t)(row - r1) * dcap + cc];
        v[u] = x;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = ly + 8 * u;
        if (nd.leaf) tile[lx][b] = v[u];
        else tile[b][lx] = v[u];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = ly + 8 * u;
        {   // rows of RR, along the columns
          const int i = r0 + b, c = k0 + lx;
          if (i < r && c < nc) gRR[(int64_t)i * dcap + c0 + c] = tile[b][lx];
        }
        {   // rows of Xr, along the rows
          const int i = r0 + lx, c = k0 + b;
          if (i >= r && i < m && c < nc) gXr[(int64_t)c * nd.mcap + (i - r)] = tile[lx][b];
        }
      }
      __syncthreads();
    }
  }
  if (st.go && blockIdx.y == 0) {
    int64_t* I = a.lpool + nd.I[side];
    const int64_t* I1 = nd.leaf ? nullptr : a.lpool + a.desc[nd.left].I[side];
    const int64_t* I2 = nd.leaf ? nullptr : a.lpool + a.desc[nd.right].I[side];
    for (int k = threadIdx.x; k < r; k += NB) {
      const int row = J[k];
      I[k] = nd.leaf ? (int64_t)nd.lo + row : (row < r1 ? I1[row] : I2[row - r1]);
    }
  }
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    GemmTask k;
    k.A = ctp(a, nd.E[side]); k.a_rs = 1; k.a_cs = nd.rcap;
    k.B = Xr; k.b_rs = 1; k.b_cs = nd.mcap;
    k.C = RR + c0; k.c_rs = dcap; k.c_cs = 1;
    k.M = r; k.N = nc; k.K = m - r; k.pad = 0;
    k.alpha = 1.0; k.beta = 1.0;
    *T0 = k;
  }
}

void launch_reduce(const LevelArgs& a, int side, int32_t mcap_max, int32_t rcap_max,
                   int32_t ncap, hipStream_t s) {
  if (a.count <= 0) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_red_gather, node_grid(a.count), dim3(NB), 0, s, a, side);
  prof_end(HSS_K_GATHER, s);
  launch_gemm(a.tasks, a.count, rcap_max, ncap, s, a.kcnt, mcap_max, a.gws, kGemmSplitElems);
}

// ------------------------------------------------------------------ finalize
__global__ void k_finalize(LevelArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {   // the next level's test block count and sizes start from zero
    a.flags[1] = 0;
    a.flags[5] = 0;
    a.flags[6] = 0;
  }
  if (t >= a.count) return;
  const int g = a.nodes[t];
  NodeState& st = a.st[g];
  const NodeDesc& nd = a.desc[g];
  const ProbDev& P = a.prob[nd.prob];
  if (nd.parent < 0) {
    if (st.go) st.state = COMPRESSED;
    return;
  }
  if (!st.active) return;
  if (st.go) st.state = COMPRESSED;
  else if (st.state != COMPRESSED) st.state = PARTIAL;
  if (P.symmetric) {
    st.rank[1] = st.rank[0];
    st.passed[1] = st.passed[0];
    st.q[1] = st.q[0];
    st.rho[1] = st.rho[0];
  }
}

void launch_finalize(const LevelArgs& a, hipStream_t s) {
  if (a.count <= 0) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_finalize, dim3((a.count + 127) / 128), dim3(128), 0, s, a);
  prof_end(HSS_K_MISC, s);
}

}  // namespace hss
