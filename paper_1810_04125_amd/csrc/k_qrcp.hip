// Interpolative decomposition by QR with column pivoting (Sec. 2.2,
// eqs. ID and QRCPSr): for a local sample S (m x d), factor S^T (d x m)
// with column pivoting, stop before the first pivot whose residual norm
// nu_k is <= max(eps_a, eps_r nu_1) (divided by the HMT factor of
// eq. RRQRHMTstop for the doubling strategy), and return the selected
// rows J (pivot order, then the other rows ascending) and
// E = R1^{-1} R2, so that S(rest,:) ~= E^T S(J,:).
//
// The factorization runs on many workgroups per matrix: column j of the
// panel W = S^T (the j-th row of S, contiguous) belongs to one workgroup,
// and every pivot step is one launch covering all matrices of a batch.
// Each workgroup finds the pivot itself (argmax over the residual norms
// of the previous step, ties to the lowest index), rebuilds the
// Householder vector from the pivot column in LDS, and updates its own
// columns, recomputing their residual norms exactly from the updated
// values.  Norms are double-buffered between steps and the pivot column is
// never written during a step, so workgroups of one launch never race.
// E is then obtained by a blocked back substitution: 64 x 64 diagonal
// blocks solved in LDS, the off-diagonal updates on the FP64 matrix cores.
#include <algorithm>

#include "hss_internal.h"

namespace hss {

constexpr int QB = 256;          // threads per workgroup
constexpr int QW = QB / 64;
constexpr int TRB = 64;          // diagonal block of the triangular solve
constexpr int QBW = 1024;        // threads of the one-workgroup factorization

struct QrcpCtl {
  int32_t done;
  int32_t rank;
  double nu1;
};

__device__ __forceinline__ QrcpCtl* ctl_of(const QrcpTask& t) { return reinterpret_cast<QrcpCtl*>(t.scr); }
__device__ __forceinline__ double* nrm_of(const QrcpTask& t, int k) { return t.scr + 16 + (int64_t)(k & 1) * t.mcap; }
__device__ __forceinline__ double* rdiag_of(const QrcpTask& t) { return t.scr + 16 + 2 * (int64_t)t.mcap; }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Work map of one factorization call, built on the device from the tasks
// that are active: every active matrix's m panel columns are cut into
// chunks of cpw columns, cpw = ceil(active columns / target), so the
// launches of the pivot steps have about `target` busy workgroups however
// few matrices factor; the target doubles when it would leave 16 or more
// columns to a workgroup.  meta = {number of chunks, cpw}; the chunk count
// is at most 2 target + ntasks.
__global__ __launch_bounds__(QB) void k_qrcp_plan(const QrcpTask* __restrict__ tasks, int ntasks, int target,
                                                  int2* __restrict__ chunks, int32_t* __restrict__ meta) {
  __shared__ long long part[QB];
  __shared__ int s_cpw;
  const int tid = threadIdx.x;
  const int per = (ntasks + QB - 1) / QB;
  const int t0 = min(ntasks, tid * per), t1 = min(ntasks, t0 + per);
  long long cols = 0;
  for (int t = t0; t < t1; ++t)
    if (tasks[t].active && tasks[t].m > 0) cols += tasks[t].m;
  part[tid] = cols;
  __syncthreads();
  if (tid == 0) {
    long long tot = 0;
    for (int i = 0; i < QB; ++i) tot += part[i];
    // steps with at least 16 columns per workgroup get twice the workgroups
    const long long tg = tot >= 16LL * target ? 2LL * target : (long long)target;
    s_cpw = (int)max(1LL, (tot + tg - 1) / tg);
  }
  __syncthreads();
  const int cpw = s_cpw;
  long long nch = 0;
  for (int t = t0; t < t1; ++t)
    if (tasks[t].active && tasks[t].m > 0) nch += (tasks[t].m + cpw - 1) / cpw;
  __syncthreads();
  part[tid] = nch;
  __syncthreads();
  if (tid == 0) {
    long long acc = 0;
    for (int i = 0; i < QB; ++i) {
      const long long v = part[i];
      part[i] = acc;
      acc += v;
    }
    meta[0] = (int32_t)acc;
    meta[1] = cpw;
  }
  __syncthreads();
  long long pos = part[tid];
  for (int t = t0; t < t1; ++t) {
    if (!tasks[t].active) continue;
    for (int c = 0; c < tasks[t].m; c += cpw) chunks[pos++] = make_int2(t, c);
  }
}

__global__ __launch_bounds__(QB) void k_qrcp_init(const QrcpTask* __restrict__ tasks, const int2* __restrict__ wg,
                                                  const int32_t* __restrict__ meta, int32_t* __restrict__ kbuf) {
  if (kbuf && blockIdx.x == 0 && threadIdx.x == 0) kbuf[0] = 0;   // step counter of the graph replays
  if ((int)blockIdx.x >= meta[0]) return;
  const int cpw = meta[1];
  const int2 w = wg[blockIdx.x];
  const QrcpTask& t = tasks[w.x];
  if (!t.active) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (w.y == 0 && threadIdx.x == 0) {
    QrcpCtl* c = ctl_of(t);
    c->done = 0;
    c->rank = 0;
    c->nu1 = 0.0;
  }
  double* nrm = nrm_of(t, 0);
  const int jend = min(t.m, w.y + cpw);
  for (int j = w.y + wv; j < jend; j += QW) {
    const double* src = t.S + (int64_t)j * t.lds;
    double* dst = t.W + (int64_t)j * t.ldw;
    double sq = 0.0;
    for (int i = lane; i < t.d; i += 64) {
      const double x = src[i];
      dst[i] = x;
      sq += x * x;
    }
    sq = wsum(sq);
    if (lane == 0) nrm[j] = sqrt(sq);
  }
}

// Pivot step k of one matrix over its panel columns [c0, cend), by a
// workgroup of NT threads.  Returns true when the matrix is finished (the
// pivot norm fell to the threshold, or k is past min(m, d)); the decision
// is the same for every thread of the workgroup.
template <int NT>
__device__ __forceinline__ bool qrcp_step_body(const QrcpTask& t, int k, int c0, int cend, bool lead,
                                               unsigned long long* __restrict__ kcnt, int kcls, double* vsh,
                                               double* rv, int* ri) {
  constexpr int NW = NT / 64;
  const int m = t.m, d = t.d;
  if (k >= min(m, d)) return true;
  QrcpCtl* c = ctl_of(t);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double* nold = nrm_of(t, k);
  double* nnew = nrm_of(t, k + 1);
  // the first norms are loaded before the finished flag is known, so the
  // two reads overlap (in bounds either way)
  double v4[4];
  if (!t.nopivot) {
#pragma unroll
    for (int u = 0; u < 4; ++u) v4[u] = threadIdx.x + u * NT < m ? nold[threadIdx.x + u * NT] : -1.0;
  }
  // The lead workgroup of a matrix may set `done` during this very launch
  // (the other workgroups then reach the same stopping decision from the
  // same norms): the flag is read once per workgroup, so all its waves
  // return together or carry on together.
  if (__syncthreads_or(c->done != 0)) return true;
  double nu;
  int p;
  if (t.nopivot) {
    p = k;
    nu = nold[k];
  } else {
    // pivot: largest residual norm among the remaining columns, ties -> lowest index
    double bv = -1.0;
    int bi = 0x7fffffff;
    // four loads in flight per thread, then compared in ascending j
    for (int j0 = threadIdx.x; j0 < m; j0 += 4 * NT) {
      if (j0 != (int)threadIdx.x) {
#pragma unroll
        for (int u = 0; u < 4; ++u) v4[u] = j0 + u * NT < m ? nold[j0 + u * NT] : -1.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + u * NT;
        const double v = v4[u];
        if (v < 0.0) continue;
        if (v > bv || (v == bv && j < bi)) { bv = v; bi = j; }
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { rv[wv] = bv; ri[wv] = bi; }
    __syncthreads();
    nu = rv[0];
    p = ri[0];
    for (int i = 1; i < NW; ++i)
      if (rv[i] > nu || (rv[i] == nu && ri[i] < p)) { nu = rv[i]; p = ri[i]; }
  }
  const double nu1 = (k == 0) ? nu : c->nu1;
  double thr = fmax(t.ea, t.er * nu1);
  if (t.hmt_mn > 0.0) {
    const double over = (double)(d - (k + 1) - 1);
    thr = over <= 0.0 ? 0.0 : thr / (1.0 + 4.0 * sqrt((double)d) / over * sqrt(t.hmt_mn));
  }
  if (nu <= thr) {
    if (lead) {
      c->rank = k;
      c->done = 1;
    }
    return true;
  }
  const double* x = t.W + (int64_t)p * t.ldw;
  const double x0 = x[k];
  const double alpha = x0 >= 0.0 ? -nu : nu;
  for (int i0 = k + threadIdx.x; i0 < d; i0 += 4 * NT) {
    double x4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x4[u] = i0 + u * NT < d ? x[i0 + u * NT] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * NT;
      if (i < d) vsh[i - k] = (i == k) ? x0 - alpha : x4[u];
    }
  }
  const double tk = 1.0 / (nu * (nu + fabs(x0)));  // 2 / v^T v
  if (lead) {
    if (k == 0) c->nu1 = nu;
    rdiag_of(t)[k] = alpha;
    if (t.J) t.J[k] = p;
    const double cells = (double)(d - k) * (double)(m - k - 1);
    kcount(kcnt, kcls, 16.0 * cells, 4.0 * cells);
  }
  __syncthreads();
  const int ncol = cend - c0;
  if (ncol > 0 && 2 * ncol <= NW) {
    // fewer columns than waves: wpc waves share a column, each a slice of
    // its rows; partial sums meet in LDS (rv, free again after the pivot
    // search) and are added in wave order
    const int wpc = NW / ncol;
    const int cj = wv / wpc, seg = wv - cj * wpc;
    const bool act = cj < ncol;
    const int j = c0 + cj;
    const bool live = act && !(j == p || nold[j] < 0.0);
    double* y = t.W + (int64_t)j * t.ldw;
    double dot = 0.0;
    if (live) {
#pragma unroll 4
      for (int i = k + seg * 64 + lane; i < d; i += 64 * wpc) dot += vsh[i - k] * y[i];
    }
    dot = wsum(dot);
    if (lane == 0) rv[wv] = dot;
    __syncthreads();
    double tot = 0.0;
    if (act)
      for (int q = 0; q < wpc; ++q) tot += rv[cj * wpc + q];
    tot *= tk;
    double sq = 0.0;
    if (live) {
#pragma unroll 4
      for (int i = k + seg * 64 + lane; i < d; i += 64 * wpc) {
        const double yi = y[i] - tot * vsh[i - k];
        y[i] = yi;
        if (i > k) sq += yi * yi;
      }
    }
    sq = wsum(sq);
    __syncthreads();
    if (lane == 0) rv[wv] = sq;
    __syncthreads();
    if (act && seg == 0 && lane == 0) {
      if (!live) {
        nnew[j] = -1.0;
      } else {
        double s2 = 0.0;
        for (int q = 0; q < wpc; ++q) s2 += rv[cj * wpc + q];
        nnew[j] = sqrt(s2);
      }
    }
    return false;
  }
  for (int j = c0 + wv; j < cend; j += NW) {
    if (j == p || nold[j] < 0.0) {
      if (lane == 0) nnew[j] = -1.0;
      continue;
    }
    double* y = t.W + (int64_t)j * t.ldw;
    double dot = 0.0;
#pragma unroll 4
    for (int i = k + lane; i < d; i += 64) dot += vsh[i - k] * y[i];
    dot = wsum(dot) * tk;
    double sq = 0.0;
#pragma unroll 4
    for (int i = k + lane; i < d; i += 64) {
      const double yi = y[i] - dot * vsh[i - k];
      y[i] = yi;
      if (i > k) sq += yi * yi;
    }
    sq = wsum(sq);
    if (lane == 0) nnew[j] = sqrt(sq);
  }
  return false;
}

__device__ __forceinline__ void qrcp_step_wg(const QrcpTask* __restrict__ tasks, const int2* __restrict__ wg,
                                             const int32_t* __restrict__ meta, int k,
                                             unsigned long long* __restrict__ kcnt, double* vsh, double* rv,
                                             int* ri) {
  const int2 w = wg[blockIdx.x];   // in bounds: the grid never exceeds the map's entries
  if ((int)blockIdx.x >= meta[0]) return;
  const int cpw = meta[1];
  const QrcpTask& t = tasks[w.x];
  if (!t.active) return;
  qrcp_step_body<QB>(t, k, w.y, min(t.m, w.y + cpw), w.y == 0 && threadIdx.x == 0, kcnt,
                     t.nopivot ? HSS_K_TEST_QR : HSS_K_QRCP_STEP, vsh, rv, ri);
}

__global__ __launch_bounds__(QB) void k_qrcp_step(const QrcpTask* __restrict__ tasks, const int2* __restrict__ wg,
                                                  const int32_t* __restrict__ meta, int k,
                                                  unsigned long long* __restrict__ kcnt) {
  extern __shared__ double vsh[];
  __shared__ double rv[QW];
  __shared__ int ri[QW];
  qrcp_step_wg(tasks, wg, meta, k, kcnt, vsh, rv, ri);
}

// The same step with k read from device memory, for replay in a graph of
// back-to-back steps: kin holds k, and workgroup 0 writes k + 1 to kout (the
// next step's kin; the two words alternate, so no step writes the word it
// reads).
__global__ __launch_bounds__(QB) void k_qrcp_step_g(const QrcpTask* __restrict__ tasks,
                                                    const int2* __restrict__ wg, const int32_t* __restrict__ meta,
                                                    const int32_t* __restrict__ kin, int32_t* __restrict__ kout,
                                                    unsigned long long* __restrict__ kcnt) {
  extern __shared__ double vsh[];
  __shared__ double rv[QW];
  __shared__ int ri[QW];
  const int k = *kin;
  if (blockIdx.x == 0 && threadIdx.x == 0) *kout = k + 1;
  qrcp_step_wg(tasks, wg, meta, k, kcnt, vsh, rv, ri);
}

// A graph of kSegSteps pivot steps (k_qrcp_step_g, k from kbuf[0] back to
// kbuf[0]) for one grid size and LDS size; instantiated once per job and
// shape, replayed for every full segment.
hipGraphExec_t QrcpGraphs::segment(const QrcpTask* tasks, const QrcpWork& wk, int nwg, size_t lds,
                                   unsigned long long* kcnt) {
  const auto key = std::make_pair(nwg, lds);
  auto it = execs.find(key);
  if (it != execs.end()) return it->second;
  hipGraph_t g = nullptr;
  HSS_HIP_CHECK(hipGraphCreate(&g, 0));
  hipGraphNode_t prev = nullptr;
  // kernel arguments of the two alternating node kinds
  struct Args {
    const QrcpTask* tasks;
    const int2* wg;
    const int32_t* meta;
    const int32_t* kin;
    int32_t* kout;
    unsigned long long* kcnt;
  } args[2] = {{tasks, wk.chunks, wk.meta, wk.kbuf, wk.kbuf + 1, kcnt},
               {tasks, wk.chunks, wk.meta, wk.kbuf + 1, wk.kbuf, kcnt}};
  void* params[2][6];
  for (int a = 0; a < 2; ++a) {
    params[a][0] = &args[a].tasks;
    params[a][1] = &args[a].wg;
    params[a][2] = &args[a].meta;
    params[a][3] = &args[a].kin;
    params[a][4] = &args[a].kout;
    params[a][5] = &args[a].kcnt;
  }
  for (int i = 0; i < kSegSteps; ++i) {
    hipKernelNodeParams p{};
    p.func = reinterpret_cast<void*>(k_qrcp_step_g);
    p.gridDim = dim3(nwg);
    p.blockDim = dim3(QB);
    p.sharedMemBytes = (unsigned)lds;
    p.kernelParams = params[i & 1];
    p.extra = nullptr;
    hipGraphNode_t node = nullptr;
    HSS_HIP_CHECK(hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p));
    prev = node;
  }
  hipGraphExec_t ex = nullptr;
  HSS_HIP_CHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
  HSS_HIP_CHECK(hipGraphDestroy(g));
  execs[key] = ex;
  return ex;
}

QrcpGraphs::~QrcpGraphs() {
  for (auto& kv : execs) hipGraphExecDestroy(kv.second);
}

// The whole factorization of one matrix by one workgroup, every pivot step
// in this launch: for small panels, where a launch per step costs more
// than the step's work.  Same arithmetic and outputs as k_qrcp_init
// followed by k_qrcp_step for k = 0, 1, ...
__global__ __launch_bounds__(QBW) void k_qrcp_wg(const QrcpTask* __restrict__ tasks,
                                                unsigned long long* __restrict__ kcnt) {
  extern __shared__ double vsh[];
  __shared__ double rv[QBW / 64];
  __shared__ int ri[QBW / 64];
  const QrcpTask& t = tasks[blockIdx.x];
  if (!t.active) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    QrcpCtl* c = ctl_of(t);
    c->done = 0;
    c->rank = 0;
    c->nu1 = 0.0;
  }
  double* nrm = nrm_of(t, 0);
  for (int j = wv; j < t.m; j += QBW / 64) {
    const double* src = t.S + (int64_t)j * t.lds;
    double* dst = t.W + (int64_t)j * t.ldw;
    double sq = 0.0;
    for (int i = lane; i < t.d; i += 64) {
      const double x = src[i];
      dst[i] = x;
      sq += x * x;
    }
    sq = wsum(sq);
    if (lane == 0) nrm[j] = sqrt(sq);
  }
  __syncthreads();
  const int kmax = min(t.m, t.d);
  for (int k = 0; k < kmax; ++k) {
    if (qrcp_step_body<QBW>(t, k, 0, t.m, threadIdx.x == 0, kcnt, HSS_K_QRCP_WG, vsh, rv, ri)) break;
    __syncthreads();
  }
}

// out[0]: matrices still factoring after step k-1 has run; out[1]: the
// largest rank of the batch so far (the final one once out[0] is 0), with
// the rank rule of k_qrcp_fin.  One workgroup; writes its result directly.
constexpr int QAL = 1024;
__global__ __launch_bounds__(QAL) void k_qrcp_alive(const QrcpTask* __restrict__ tasks, int ntasks, int k,
                                                   int32_t* __restrict__ out) {
  __shared__ int sa[QAL / 64], sr[QAL / 64];
  int alive = 0, rmax = 0;
  for (int i = threadIdx.x; i < ntasks; i += QAL) {
    const QrcpTask& t = tasks[i];
    if (!t.active) continue;
    const int kmax = min(t.m, t.d);
    const QrcpCtl* c = ctl_of(t);
    const bool done = c->done != 0;
    if (k < kmax && !done) ++alive;
    rmax = max(rmax, (kmax > 0 && done) ? c->rank : kmax);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    alive += __shfl_xor(alive, o, 64);
    rmax = max(rmax, __shfl_xor(rmax, o, 64));
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { sa[wv] = alive; sr[wv] = rmax; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, r = 0;
    for (int w = 0; w < QAL / 64; ++w) { a += sa[w]; r = max(r, sr[w]); }
    out[0] = a;
    out[1] = r;
  }
}

// Pinned, device-mapped host words for the values the host decides on:
// the liveness poll writes them directly (no copy), the host reads them
// after the stream has drained.  `dev` is the device-side address.
static int32_t* host_words(int32_t** dev) {
  thread_local int32_t* p = nullptr;
  thread_local int32_t* d = nullptr;
  if (!p) {
    HSS_HIP_CHECK(hipHostMalloc((void**)&p, 64, hipHostMallocMapped | hipHostMallocPortable));
    HSS_HIP_CHECK(hipHostGetDevicePointer((void**)&d, p, 0));
  }
  *dev = d;
  return p;
}

// Active panels of a factorization call, written to out[0] (mapped host
// memory).  One workgroup.
__global__ __launch_bounds__(QAL) void k_qrcp_count(const QrcpTask* __restrict__ tasks, int ntasks,
                                                   int32_t* __restrict__ out) {
  __shared__ int sa[QAL / 64];
  int act = 0;
  for (int i = threadIdx.x; i < ntasks; i += QAL) act += tasks[i].active ? 1 : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) act += __shfl_xor(act, o, 64);
  if ((threadIdx.x & 63) == 0) sa[threadIdx.x >> 6] = act;
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0;
    for (int w = 0; w < QAL / 64; ++w) a += sa[w];
    out[0] = a;
  }
}

int32_t count_active_panels(const QrcpTask* tasks, int32_t ntasks, hipStream_t s) {
  if (ntasks <= 0) return 0;
  int32_t* hw_dev = nullptr;
  int32_t* hw = host_words(&hw_dev);
  hipLaunchKernelGGL(k_qrcp_count, dim3(1), dim3(QAL), 0, s, tasks, ntasks, hw_dev + 2);
  HSS_HIP_CHECK(hipStreamSynchronize(s));
  return hw[2];
}

// rank, the ascending rest of J, max rank of the batch
__global__ __launch_bounds__(QB) void k_qrcp_fin(const QrcpTask* __restrict__ tasks, int32_t* maxrank,
                                                 unsigned long long* __restrict__ kcnt) {
  const QrcpTask& t = tasks[blockIdx.x];
  if (!t.active) return;
  __shared__ int cnt[QB];
  const int m = t.m, d = t.d;
  const int kmax = min(m, d);
  const QrcpCtl* c = ctl_of(t);
  const int r = (kmax > 0 && c->done) ? c->rank : kmax;
  if (t.J) {
    // the columns never pivoted, ascending, after the r pivots: each thread
    // counts its contiguous share, an exclusive scan gives its offset
    const double* nfin = nrm_of(t, r);
    const int per = (m + QB - 1) / QB;
    const int j0 = min(m, (int)threadIdx.x * per), j1 = min(m, j0 + per);
    int n = 0;
    for (int j = j0; j < j1; ++j) n += nfin[j] >= 0.0;
    cnt[threadIdx.x] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = 0;
      for (int i = 0; i < QB; ++i) {
        const int v = cnt[i];
        cnt[i] = acc;
        acc += v;
      }
    }
    __syncthreads();
    int pos = r + cnt[threadIdx.x];
    for (int j = j0; j < j1; ++j)
      if (nfin[j] >= 0.0) t.J[pos++] = j;
  }
  if (threadIdx.x == 0) {
    *t.rank_out = r;
    if (maxrank) atomicMax(maxrank, r);
    // the ID's algorithmic work: the d x m panel read once, E written, and
    // 4 d m r flops of a QR with column pivoting to rank r
    if (!t.nopivot) kcount(kcnt, HSS_K_ID, 8.0 * (double)d * m + 8.0 * (double)r * (m - r), 4.0 * (double)d * m * r);
  }
}

// Right-hand side of the back substitution: E(:, l) = R(0:r, J(r + l)),
// the first r entries of panel column J(r + l).  The columns l of a matrix
// are spread over the gridDim.y workgroups; a workgroup copies one column
// at a time, every thread loading its EU entries together.
constexpr int EU = 4;
__global__ __launch_bounds__(QB) void k_qrcp_egather(const QrcpTask* __restrict__ tasks) {
  const QrcpTask& t = tasks[blockIdx.x];
  if (!t.active || !t.E) return;
  const int r = *t.rank_out;
  const int nrest = t.m - r;
  const HSS_GLOBAL int32_t* J = gview(t.J);
  for (int l = blockIdx.y; l < nrest; l += gridDim.y) {
    const HSS_GLOBAL double* src = gview(t.W + (int64_t)J[r + l] * t.ldw);
    HSS_GLOBAL double* dst = gview_w(t.E + (int64_t)l * t.lde);
    for (int i0 = threadIdx.x; i0 < r; i0 += QB * EU) {
      double v[EU];
#pragma unroll
      for (int u = 0; u < EU; ++u) v[u] = src[min(i0 + u * QB, r - 1)];
#pragma unroll
      for (int u = 0; u < EU; ++u)
        if (i0 + u * QB < r) dst[i0 + u * QB] = v[u];
    }
  }
}

// Diagonal block [i0, i1) of the back substitution R1 E = R2 for the
// columns [c0, c0 + QB) of E; the workgroup with c0 == 0 also writes the
// GEMM task of the update E(0:i0, :) -= R1(0:i0, i0:i1) E(i0:i1, :).
__global__ __launch_bounds__(QB) void k_trsm_diag(const QrcpTask* __restrict__ tasks, const int2* __restrict__ wg,
                                                  int ib, GemmTask* __restrict__ gt,
                                                  unsigned long long* __restrict__ kcnt) {
  __shared__ double T[TRB][TRB + 1];
  const int2 w = wg[blockIdx.x];
  const QrcpTask& t = tasks[w.x];
  GemmTask* g = gt + w.x;
  if (w.y == 0 && threadIdx.x == 0) g->M = 0;
  if (!t.active) return;
  const int r = *t.rank_out;
  const int i0 = ib * TRB;
  if (i0 >= r) return;
  const int i1 = min(r, i0 + TRB);
  const int nb = i1 - i0;
  const int nrest = t.m - r;
  {
    // R1 block: column jj is panel column J(i0 + jj); every thread loads its
    // TPT entries (their column indices first) before writing any to LDS
    constexpr int TPT = TRB * TRB / QB;
    const HSS_GLOBAL double* rdiag = gview(rdiag_of(t));
    const HSS_GLOBAL int32_t* J = gview(t.J);
    const HSS_GLOBAL double* W = gview(t.W);
    int col[TPT];
#pragma unroll
    for (int u = 0; u < TPT; ++u) col[u] = J[i0 + min((int)(threadIdx.x + QB * u) / TRB, nb - 1)];
    double v[TPT];
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const int idx = threadIdx.x + QB * u;
      const int ii = idx % TRB, jj = idx / TRB;
      v[u] = ii == jj ? rdiag[i0 + min(jj, nb - 1)] : W[(int64_t)col[u] * t.ldw + i0 + min(ii, nb - 1)];
    }
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const int idx = threadIdx.x + QB * u;
      const int ii = idx % TRB, jj = idx / TRB;
      T[ii][jj] = (ii < nb && jj < nb && ii <= jj) ? v[u] : 0.0;
    }
  }
  __syncthreads();
  const int l = w.y + threadIdx.x;
  if (l < nrest) {
    HSS_GLOBAL double* e = gview_w(t.E + (int64_t)l * t.lde + i0);
    double x[TRB];
#pragma unroll
    for (int ii = 0; ii < TRB; ++ii) x[ii] = ii < nb ? e[ii] : 0.0;
#pragma unroll
    for (int jj = TRB - 1; jj >= 0; --jj) {
      if (jj < nb) {
        const double xj = x[jj] / T[jj][jj];
        x[jj] = xj;
#pragma unroll
        for (int ii = 0; ii < jj; ++ii) x[ii] -= T[ii][jj] * xj;
      }
    }
#pragma unroll
    for (int ii = 0; ii < TRB; ++ii)
      if (ii < nb) e[ii] = x[ii];
  }
  if (w.y == 0 && threadIdx.x == 0) kcount(kcnt, HSS_K_TRSM, 16.0 * nb * nrest, (double)nb * nb * nrest);
  if (w.y == 0 && threadIdx.x == 0 && i0 > 0 && nrest > 0) {
    GemmTask q;
    q.A = t.W; q.a_rs = 1; q.a_cs = t.ldw; q.a_cols = t.J + i0;
    q.B = t.E + i0; q.b_rs = 1; q.b_cs = t.lde;
    q.C = t.E; q.c_rs = 1; q.c_cs = t.lde;
    q.M = i0; q.N = nrest; q.K = nb; q.pad = 0;
    q.alpha = -1.0; q.beta = 1.0;
    *g = q;
  }
}

QrcpPlan make_qrcp_plan(const std::vector<int32_t>& mcaps, int cpw) {
  QrcpPlan p;
  for (size_t t = 0; t < mcaps.size(); ++t) {
    const int mc = std::max(mcaps[t], 1);
    for (int c = 0; c < mc; c += cpw) p.step.push_back(make_int2((int)t, c));
    for (int c = 0; c < mc; c += QB) p.trsm.push_back(make_int2((int)t, c));
  }
  return p;
}

void run_qrcp(QrcpTask* tasks, int32_t ntasks, const QrcpWork& wk, const int2* wg_trsm, int32_t ntrsm,
              int32_t kmax, int32_t dmax, int32_t ncols_max, int32_t* flag, GemmTask* gtasks, int32_t mcap_max,
              hipStream_t s, unsigned long long* kcnt, bool solve_e, double* gws, const IdBlockWork* bw) {
  if (ntasks <= 0) return;
  if (ntasks > wk.max_tasks) throw Error(HSS_ERR_INTERNAL, "QRCP work map too small for the batch");
  const int target = tune().qrcp_wg;   // kQrcpTarget by default
  const int nwg = 2 * target + ntasks;
  const size_t lds = (size_t)std::max(dmax, 1) * sizeof(double);
  // The ID first counts its active panels: with none it is done, and the
  // count picks the factorization kernel.
  int32_t nact = 0;
  if (solve_e) {
    nact = count_active_panels(tasks, ntasks, s);
    if (nact == 0) return;
  }
  const bool known_active = solve_e;   // some panel is known to be active
  const int64_t cells = (int64_t)std::max(dmax, 1) * std::max(ncols_max, 1);
  bool one_wg = cells <= kQrcpWgCells && lds <= 48 * 1024;
  if (one_wg && solve_e) {
    // Per pivot step, the one-workgroup kernel walks the columns 16 at a
    // time (about 5 + 2.2 us per 16 columns, measured); the many-workgroup
    // step costs about 7 us, or its traffic at about 3.4 TB/s when larger
    // (2.35 ps per cell of all active panels), and a pivot of the blocked
    // ID about 10 us on the sphere-Laplace levels (a block of 12 launches
    // per 19 pivots on average), so small panels stay on one workgroup.
    const double t_wg = 5.0 + 2.2 * std::ceil(ncols_max / 16.0);
    const double t_step = std::max(7.0, 2.35e-6 * (double)nact * (double)cells);
    one_wg = t_wg < t_step;
  }
  const bool blocks = !one_wg && solve_e && bw && bw->blk && ncols_max <= kIdbMaxM;
  if (one_wg) {
    prof_begin(s);
    hipLaunchKernelGGL(k_qrcp_wg, dim3(ntasks), dim3(QBW), lds, s, tasks, kcnt);
    prof_end(HSS_K_QRCP_WG, s);
  } else {
    prof_begin(s);
    hipLaunchKernelGGL(k_qrcp_plan, dim3(1), dim3(QB), 0, s, tasks, ntasks, target, wk.chunks, wk.meta);
    hipLaunchKernelGGL(k_qrcp_init, dim3(nwg), dim3(QB), 0, s, tasks, wk.chunks, wk.meta, wk.kbuf);
    prof_end(HSS_K_QRCP_OTHER, s);
  }
  // pivot steps: launched back to back in segments of 32 after liveness
  // polls (none before the first segment when a panel is known to be
  // active); profiling times each segment as a whole.  The poll that finds
  // no matrix alive also gives the largest rank.
  int32_t* hw_dev = nullptr;
  int32_t* hw = host_words(&hw_dev);
  bool rank_known = false;
  if (blocks) run_id_blocks(tasks, ntasks, *bw, dmax, ncols_max, hw_dev, hw, gws, s, kcnt);
  const int ksteps = (one_wg || blocks) ? 0 : kmax;
  for (int k0 = 0; k0 < ksteps; k0 += kSegSteps) {
    if (k0 > 0 || !known_active) {
      hipLaunchKernelGGL(k_qrcp_alive, dim3(1), dim3(QAL), 0, s, tasks, ntasks, k0, hw_dev);
      HSS_HIP_CHECK(hipStreamSynchronize(s));
      if (hw[0] == 0) {
        rank_known = true;
        break;
      }
    }
    const int k1 = std::min(ksteps, k0 + kSegSteps);
    prof_begin(s);
    if (wk.graphs && wk.kbuf && k1 - k0 == kSegSteps) {
      // a full segment: one replay of the step graph (kbuf[0] == k0 here)
      HSS_HIP_CHECK(hipGraphLaunch(wk.graphs->segment(tasks, wk, nwg, lds, kcnt), s));
    } else {
      for (int k = k0; k < k1; ++k)
        hipLaunchKernelGGL(k_qrcp_step, dim3(nwg), dim3(QB), lds, s, tasks, wk.chunks, wk.meta, k, kcnt);
    }
    prof_end(solve_e ? HSS_K_QRCP_STEP : HSS_K_TEST_QR, s, k1 - k0);
  }
  int32_t rmax = rank_known ? hw[1] : 0;
  if (!rank_known) HSS_HIP_CHECK(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
  prof_begin(s);
  hipLaunchKernelGGL(k_qrcp_fin, dim3(ntasks), dim3(QB), 0, s, tasks, rank_known ? nullptr : flag, kcnt);
  prof_end(HSS_K_QRCP_OTHER, s);
  if (solve_e) prof_count(HSS_K_ID, 1);
  if (!solve_e) return;
  prof_begin(s);
  hipLaunchKernelGGL(k_qrcp_egather, dim3(ntasks, (unsigned)std::max(1, std::min(256, 4096 / ntasks))), dim3(QB),
                     0, s, tasks);
  prof_end(HSS_K_QRCP_OTHER, s);
  if (!rank_known) {
    HSS_HIP_CHECK(hipMemcpyAsync(hw, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HSS_HIP_CHECK(hipStreamSynchronize(s));
    rmax = hw[0];
  }
  for (int ib = (rmax + TRB - 1) / TRB - 1; ib >= 0; --ib) {
    prof_begin(s);
    hipLaunchKernelGGL(k_trsm_diag, dim3(ntrsm), dim3(QB), 0, s, tasks, wg_trsm, ib, gtasks, kcnt);
    prof_end(HSS_K_TRSM, s);
    if (ib > 0) launch_gemm(gtasks, ntasks, ib * TRB, mcap_max, s, kcnt);
  }
  HSS_HIP_CHECK(hipGetLastError());
}

}  // namespace hss
