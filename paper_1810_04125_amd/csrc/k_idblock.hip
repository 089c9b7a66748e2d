// Interpolative decomposition by QR with column pivoting (Sec. 2.2, eqs. ID
// and QRCPSr), with the pivots chosen a block at a time.
//
// The ID selects, step by step, the panel column (a row of the local sample)
// with the largest residual norm and stops before the first one at or below
// the threshold.  A step needs the residual norms of all remaining columns,
// so a plain implementation reads the whole trailing panel once per pivot.
// Here the pivots are found in blocks, with the same choices:
//   1. candidates (k_idb_select, k_idb_gather): the c = 256 remaining
//      columns of largest residual norm (ties to the lower index); `bound` is the
//      largest norm among the others, and no residual norm ever grows, so
//      while the best candidate's residual is at least `bound`, it is the
//      column the one-step method would pick;
//   2. their Gram matrix G = C^T C (C = candidates' residual columns, FP64
//      matrix cores) and its pivoted Cholesky factorization (k_idb_chol), which yields the candidates' residual norms after each
//      pivot (the Schur complement's diagonal): pivots are taken while the
//      best one beats `bound`, until the threshold stops the factorization,
//      or until the residuals fall 1e5-fold within the block (their
//      Gram-derived values then lose accuracy); R1 of the pivot columns;
//   3. Cholesky QR, twice, of the pivot columns C_P (k_idb_rows1: Q1 =
//      C_P R1^{-1} and Q1^T Q1 by rows over many workgroups; k_idb_small:
//      R2, R = R2 R1) and the block's Householder reflectors rebuilt from Q
//      with their triangular factor T (k_idb_small, k_idb_rows2);
//   4. the remaining columns are updated as A <- A - (V T^T)(V^T A) by two
//      GEMMs on the matrix cores, and their residual norms are recomputed
//      exactly for the next block (k_idb_norms).
// R and the skeleton order are stored in the panel and the task as by the
// one-step kernels (k_qrcp.hip), whose back substitution then forms E.
//
// The factorizations of steps 2 and 3 are chains of dependent small steps,
// run by one workgroup per task: their code is kept compact (loops rather
// than fully unrolled straight-line code, which would be fetched into the
// instruction cache anew at every launch), and a step costs one barrier or
// none (the pivoted Cholesky runs on one wave).
#include <algorithm>

#include "hss_internal.h"

namespace hss {

namespace {

constexpr int SELT = 256;    // threads of the selection kernel
constexpr int PCT = 256;     // threads of the factorization kernel (one wave per SIMD: 512 VGPRs each)
constexpr int NRMW = 4;      // columns (one per wave) per workgroup of the norm kernel

struct QrcpCtlB {
  int32_t done;
  int32_t rank;
  double nu1;
};
__device__ __forceinline__ QrcpCtlB* ctlb(const QrcpTask& t) { return reinterpret_cast<QrcpCtlB*>(t.scr); }
__device__ __forceinline__ double* nrmb(const QrcpTask& t, int par) { return t.scr + 16 + (int64_t)par * t.mcap; }
__device__ __forceinline__ double* rdiagb(const QrcpTask& t) { return t.scr + 16 + 2 * (int64_t)t.mcap; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Orders the LDS accesses of one wave around this point (lanes exchange
// data through LDS without a workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1 / x and 1 / sqrt(x) for normal x > 0: the hardware estimates refined by
// two Newton steps (a few ulps; no special cases).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Largest 64-bit key over the wave; every lane gets it (DPP within rows of
// 16 lanes, readlane across the four rows).
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
  const auto take = [](uint64_t& v, int lo, int hi) {
    const uint64_t o = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    v = o > v ? o : v;
  };
  take(x, dpp_i<0xB1>((int)x), dpp_i<0xB1>((int)(x >> 32)));
  take(x, dpp_i<0x4E>((int)x), dpp_i<0x4E>((int)(x >> 32)));
  take(x, dpp_i<0x141>((int)x), dpp_i<0x141>((int)(x >> 32)));
  take(x, dpp_i<0x140>((int)x), dpp_i<0x140>((int)(x >> 32)));
  uint64_t v = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    take(v, __builtin_amdgcn_readlane((int)x, 16 * r), __builtin_amdgcn_readlane((int)(x >> 32), 16 * r));
  return v;
}

// C = A B for upper triangular A, B (L x L, LDS with row stride LP); C's
// entries outside the upper L x L triangle are set to zero.  Lane l: column
// l % 32, rows 16 (l / 32) .. + 15.  The operands' lower parts are not read.
template <int LP>
__device__ __forceinline__ void upper_product(const double (*A)[LP], const double (*Bm)[LP], double (*C)[LP], int L,
                                              int lane) {
  constexpr int N = LP - 1;
  static_assert(N == 32, "one column per half wave");
  const int b = lane & 31, a0 = (lane >> 5) * 16;
  double bc[N];
#pragma unroll
  for (int c = 0; c < N; ++c) bc[c] = (c <= b && b < L) ? Bm[c][b] : 0.0;
  double out[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int a = a0 + u;
    double sv = 0.0;
#pragma unroll
    for (int c = 0; c < N; ++c)
      if (c >= a) sv += A[a][c] * bc[c];
    out[u] = (a <= b && b < L) ? sv : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) C[a0 + u][b] = out[u];
}

__device__ __forceinline__ uint64_t key_of(double v) { return (uint64_t)__double_as_longlong(v); }

// Exclusive prefix sum of v over a workgroup of NT threads (NT / 64 waves);
// returns the thread's offset, *total the sum.  sh: NT / 64 + 1 ints of LDS.
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < NT / 64; ++w) { const int t = sh[w]; sh[w] = acc; acc += t; }
    sh[NT / 64] = acc;
  }
  __syncthreads();
  const int r = sh[wv] + x - v;
  *total = sh[NT / 64];
  __syncthreads();
  return r;
}

}  // namespace

// Per task: k = 0 and an empty block.
__global__ void k_idb_start(const QrcpTask* __restrict__ tasks, IdBlk* __restrict__ blks, int ntasks) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntasks) return;
  IdBlk& B = blks[t];
  B.k = 0;
  B.ncand = 0;
  B.nrest = 0;
  B.L = 0;
  B.lc = 0;
  B.stop = 0;
  B.kb = 0;
}

// Step 1: candidates and bound.  One workgroup per task; writes the Gram task.
// The norms are staged in LDS as keys: 0 for a pivoted column, else 1 + the
// bit pattern of the (non-negative) norm, which orders like the norm.
__global__ __launch_bounds__(SELT) void k_idb_select(const QrcpTask* __restrict__ tasks, IdBlk* __restrict__ blks,
                                                     GemmTask* __restrict__ gt, int ntasks) {
  extern __shared__ uint64_t keys[];   // m keys
  __shared__ uint32_t hist[256];
  __shared__ int sh_int[SELT];
  __shared__ uint64_t sh_prefix;
  __shared__ int sh_remain;
  __shared__ uint64_t sh_max[SELT / 64];
  const int ti = blockIdx.x;
  const QrcpTask& t = tasks[ti];
  IdBlk& B = blks[ti];
  GemmTask* g = gt + ti;
  const int tid = threadIdx.x;
  if (tid == 0) g->M = 0;
  if (!t.active) return;
  const int m = t.m, d = t.d, k = B.k;
  QrcpCtlB* c = ctlb(t);
  if (c->done || k >= min(m, d)) {
    if (tid == 0) { B.ncand = 0; B.L = 0; }
    return;
  }
  const HSS_GLOBAL double* nrm = gview(nrmb(t, 0));
  int na = 0;
  for (int j = tid; j < m; j += SELT) {
    const double v = nrm[j];
    const uint64_t key = v >= 0.0 ? key_of(v) + 1 : 0;
    keys[j] = key;
    na += key != 0;
  }
  int nact = 0;
  (void)block_excl_scan<SELT>(na, sh_int, &nact);
  const int cmax = B.cmax;
  const int nc = min(nact, cmax);
  // threshold key tau: #(key > tau) < nc <= #(key >= tau), by 8-bit radix passes from the top
  uint64_t tau = 1;
  int need_eq = 0;
  const bool all = nact <= cmax;
  if (!all) {
    if (tid == 0) { sh_prefix = 0; sh_remain = nc; }
    __syncthreads();
    for (int pos = 7; pos >= 0; --pos) {
      for (int b = tid; b < 256; b += SELT) hist[b] = 0;
      __syncthreads();
      const uint64_t prefix = sh_prefix;
      const int shift = 8 * pos;
      for (int j = tid; j < m; j += SELT) {
        const uint64_t key = keys[j];
        if (key == 0) continue;
        if (pos < 7 && (key >> (shift + 8)) != prefix) continue;
        atomicAdd(&hist[(key >> shift) & 255u], 1u);
      }
      __syncthreads();
      if (tid < 64) {
        // bins 255 .. 0 from the top: lane l holds bins 255 - 4l .. 252 - 4l;
        // the bin where the count from the top reaches `remain`
        const int remain = sh_remain;
        uint32_t h[4], own = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) { h[u] = hist[255 - 4 * tid - u]; own += h[u]; }
        uint32_t incl = own;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t y = __shfl_up(incl, o, 64);
          if (tid >= o) incl += y;
        }
        uint32_t before = incl - own;
        if ((int)before < remain && (int)incl >= remain) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if ((int)(before + h[u]) >= remain) {
              sh_remain = remain - (int)before;
              sh_prefix = (prefix << 8) | (uint64_t)(255 - 4 * tid - u);
              break;
            }
            before += h[u];
          }
        }
      }
      __syncthreads();
    }
    tau = sh_prefix;
    need_eq = sh_remain;   // candidates with key == tau, lowest indices first
  }
  // ordered compaction over contiguous column chunks (from LDS)
  const int per = (m + SELT - 1) / SELT;
  const int j0 = min(m, tid * per), j1 = min(m, j0 + per);
  int neq = 0;
  if (!all)
    for (int j = j0; j < j1; ++j) neq += keys[j] == tau;
  int dummy = 0;
  const int eq_before = block_excl_scan<SELT>(neq, sh_int, &dummy);
  int nsel = 0;
  uint64_t best_out = 0;
  {
    int eq = eq_before;
    for (int j = j0; j < j1; ++j) {
      const uint64_t key = keys[j];
      if (key == 0) continue;
      const bool sel = all || key > tau || (key == tau && eq++ < need_eq);
      if (sel) ++nsel;
      else best_out = max(best_out, key);
    }
  }
  const int sel_before = block_excl_scan<SELT>(nsel, sh_int, &dummy);
  {
    int pos = sel_before, eq = eq_before;
    for (int j = j0; j < j1; ++j) {
      const uint64_t key = keys[j];
      if (key == 0) continue;
      const bool sel = all || key > tau || (key == tau && eq++ < need_eq);
      if (sel) B.cand[pos++] = j;
    }
  }
  // bound: the largest norm among the non-candidates
  uint64_t bm = best_out;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t ob = (uint64_t)__shfl_xor((long long)bm, o, 64);
    bm = max(bm, ob);
  }
  if ((tid & 63) == 0) sh_max[tid >> 6] = bm;
  __syncthreads();
  if (tid == 0) {
    uint64_t b = 0;
    for (int w = 0; w < SELT / 64; ++w) b = max(b, sh_max[w]);
    B.bound = b == 0 ? -1.0 : __longlong_as_double((long long)(b - 1));
    B.ncand = nc;
    B.L = 0;
    // Gram of the gathered candidates: G = C^T C, C (d - k) x nc with leading dimension ldc
    GemmTask q;
    q.A = B.C; q.a_rs = B.ldc; q.a_cs = 1;
    q.B = B.C; q.b_rs = 1; q.b_cs = B.ldc;
    q.C = B.G; q.c_rs = 1; q.c_cs = B.cmax;
    q.M = nc; q.N = nc; q.K = d - k; q.pad = 0;
    q.alpha = 1.0; q.beta = 0.0;
    *g = q;
  }
}

// Step 1b: C(i, j) = W(k + i, cand[j]) for the rows k .. d of the candidates.
__global__ __launch_bounds__(256) void k_idb_gather(const QrcpTask* __restrict__ tasks, const IdBlk* __restrict__ blks) {
  const int ti = blockIdx.z;
  const QrcpTask& t = tasks[ti];
  if (!t.active) return;
  const IdBlk& B = blks[ti];
  const int j = blockIdx.y;
  if (j >= B.ncand) return;
  const int nr = t.d - B.k;
  const HSS_GLOBAL double* src = gview(t.W + (int64_t)B.cand[j] * t.ldw + B.k);
  HSS_GLOBAL double* dst = gview_w(B.C + (int64_t)j * B.ldc);
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nr; i += gridDim.x * 256) dst[i] = src[i];
}

// Step 2: pivoted Cholesky of the candidates' Gram matrix, left-looking:
// the block's pivots and the stopping decision, and R1 of the pivot
// columns (C_P = Q1 R1).  The first wave factors (lane l: candidates l,
// l + 64, ...), with no barriers; each step reads the pivot's row of the
// Gram matrix from global memory (it stays in the L2 of the compute unit's
// die after the first steps touch it) and the Cholesky entries from LDS.
__global__ __launch_bounds__(PCT) void k_idb_chol(const QrcpTask* __restrict__ tasks, IdBlk* __restrict__ blks) {
  constexpr int CPL = kIdbCmax / 64;   // candidates per lane
  static_assert(kIdbCmax % 64 == 0 && kIdbCmax <= 256, "whole lanes; an 8-bit index in the pivot key");
  extern __shared__ double Ls[];
  __shared__ int piv[kIdbLmax];
  __shared__ double spv[kIdbLmax];
  const int ti = blockIdx.x;
  const QrcpTask& t = tasks[ti];
  IdBlk& B = blks[ti];
  const int tid = threadIdx.x, lane = tid & 63;
  if (!t.active) return;
  const int nc = B.ncand;
  if (nc <= 0) return;
  const int m = t.m, d = t.d, k = B.k, cm = B.cmax;
  // per-candidate entries of rows q, q + 1 (q even) side by side: entry (q, a)
  // at (q / 2) PR + 2 a + q % 2, so that a lane's pair and the pivot's pair
  // are 16-byte loads without bank conflicts.  LDL^T form: Lu holds
  // u(q, a), the Schur complement entry of pivot q in column a; Lc holds
  // l(q, a) = u(q, a) / s_q with s_q the pivot's residual; the Cholesky
  // factor is l(q, a) sqrt(s_q).  Rows >= i are zero.
  constexpr int PR = 2 * kIdbCmax;
  double* Lc = Ls;
  double* Lu = Ls + (kIdbLmax / 2) * PR;
  for (int e = tid; e < kIdbLmax * PR; e += PCT) Ls[e] = 0.0;
  __syncthreads();
  const HSS_GLOBAL double* Gg = gview(B.G);
  if (tid >= 64) {
    // the other waves read the candidates' columns of G once (one load per
    // 128-byte line), so that the pivot rows the first wave reads later
    // come from this die's L2 rather than from another die's
    double acc = 0.0;
    const int64_t lines = ((int64_t)nc * cm + 15) / 16;
    for (int64_t e = tid - 64; e < lines; e += PCT - 64) acc += Gg[16 * e];
    asm volatile("" ::"v"(acc));
    return;
  }
  QrcpCtlB* ctl = ctlb(t);
  const double bound = B.bound;
  int au[CPL];
  bool cu[CPL];     // taken as a pivot, or past the candidates
  double sd[CPL];   // residual of each of this lane's candidates
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    au[u] = lane + 64 * u;
    cu[u] = au[u] >= nc;
    sd[u] = cu[u] ? 0.0 : Gg[au[u] + (int64_t)au[u] * cm];
  }
  double s0 = 0.0;
  double nu1 = ctl->nu1;
  const int kmax = min(m, d);
  const int lcap = min(min(kIdbLmax, nc), kmax - k);
  const double hmt_c = t.hmt_mn > 0.0 ? 4.0 * sqrt((double)d) * sqrt(t.hmt_mn) : 0.0;
  const double bound2 = bound >= 0.0 ? bound * bound : -1.0;
  double thr2_l = 0.0;   // lane i: the squared threshold of pivot k + i
  // the pivot: the largest residual, by a key that keeps the residual's top
  // 56 bits (a relative 2^-44) and prefers the lower index among equal keys;
  // its exact residual comes from the lane that holds it.  The next pivot
  // is found as soon as the residuals are updated, and its row of G is
  // loaded while the entries of its Cholesky column are read from LDS.
  int L = 0;
  bool stop = false;
#pragma unroll 1
  for (int i = 0; i < lcap; ++i) {
    // the pivot: the largest residual, by a key that keeps the residual's
    // top 56 bits (a relative 2^-44) and prefers the lower index among equal
    // keys; its exact residual comes from the lane that holds it
    uint64_t kl = 0;
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      if (cu[u]) continue;
      const uint64_t hb = ((uint64_t)__double_as_longlong(fmax(sd[u], 0.0)) >> 8) + 1;
      const uint64_t key = (hb << 8) | (uint64_t)(255 - au[u]);
      kl = key > kl ? key : kl;
    }
    const uint64_t kb = wave_max_u64(kl);
    const int p = 255 - (int)(kb & 255);
    double own = sd[0];
#pragma unroll
    for (int u = 1; u < CPL; ++u)
      if ((p >> 6) == u) own = sd[u];
    const double sp = readlane_d(own, p & 63);
    const double spp = fmax(sp, 0.0);
    if (i == 0) {
      s0 = sp;
      if (k == 0) nu1 = sqrt(spp);
      double thr = fmax(t.ea, t.er * nu1);
      if (hmt_c > 0.0) {
        const double over = (double)(d - (k + lane + 1) - 1);
        thr = over <= 0.0 ? 0.0 : thr / (1.0 + hmt_c / over);
      }
      thr2_l = thr * thr;
    }
    const double thr2 = readlane_d(thr2_l, i);
    if (i > 0 && spp < bound2) break;        // a non-candidate may be larger now
    if (spp <= thr2) { stop = true; break; } // every residual is at or below the threshold
    if (i > 0 && sp < 1e-10 * s0) break;     // Gram-derived residuals lose accuracy below this
    const double inv = sp >= 1e-290 ? rcp_nr(sp) : 1.0 / sp;
    // u_a = G(p, a) - sum_q u(q, a) l(q, p)
    // the row of G is added last, so that the LDS reads and products run
    // while its load is in flight
    double gp[CPL], g[CPL], h[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      gp[u] = cu[u] ? 0.0 : Gg[au[u] + (int64_t)p * cm];
      g[u] = 0.0;
      h[u] = 0.0;
    }
    for (int q0 = 0; q0 < i; q0 += 8) {   // rows >= i are zero: whole chunks of 8 rows
#pragma unroll
      for (int q = q0; q < q0 + 8; q += 2) {
        const int row = (q >> 1) * PR;
        const double2 w = *reinterpret_cast<const double2*>(Lc + row + 2 * p);
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
          const double2 x = *reinterpret_cast<const double2*>(Lu + row + 2 * au[u]);
          g[u] -= x.x * w.x;
          h[u] -= x.y * w.y;
        }
      }
    }
    wave_sync();   // every lane has read the pivot's entries
    const int wi = (i >> 1) * PR + (i & 1);
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const double ua = cu[u] ? 0.0 : gp[u] + (g[u] + h[u]);
      const double l = ua * inv;
      Lc[wi + 2 * au[u]] = l;
      Lu[wi + 2 * au[u]] = ua;
      if (!cu[u]) {
        if (au[u] == p) cu[u] = true;
        else sd[u] -= ua * l;
      }
    }
    if (lane == 0) { piv[i] = p; spv[i] = spp; }
    wave_sync();
    L = i + 1;
  }
  // R1 (row-major, L x L upper, zero elsewhere): R1(q, i') = l(q, p_i') sqrt(s_q)
  for (int e = lane; e < kIdbLmax * kIdbLmax; e += 64) {
    const int a = e / kIdbLmax, b = e % kIdbLmax;
    double v = 0.0;
    if (a < L && b < L && a <= b)
      v = a == b ? sqrt(spv[a]) : Lc[(a >> 1) * PR + 2 * piv[b] + (a & 1)] * sqrt(spv[a]);
    B.F[e] = v;
  }
  if (lane < L) B.piv[lane] = piv[lane];
  if (lane == 0) {
    if (k == 0) ctl->nu1 = nu1;
    B.lc = L;
    B.stop = stop;
  }
}

// Step 3a: Q1 = C_P R1^{-1}, one panel row per thread (forward substitution
// of x R1 = c), into V; each workgroup's share of Q1^T Q1 (upper 4 x 4
// blocks, 36 per group of rows, 7 row groups) into P.
constexpr int kNb4 = kIdbLmax / 4;
constexpr int kBlk4 = kNb4 * (kNb4 + 1) / 2;
constexpr int kGrp4 = kIdbRows / kBlk4;
static_assert(kBlk4 * 16 == kIdbPart, "partial layout");
__global__ __launch_bounds__(kIdbRows) void k_idb_rows1(const QrcpTask* __restrict__ tasks, IdBlk* __restrict__ blks) {
  extern __shared__ double Qc[];   // kIdbRows x kIdbLmax: R1 first, then the rows of Q1, then the group sums
  __shared__ int64_t colp[kIdbLmax];
  __shared__ double rinv[kIdbLmax];
  const int ti = blockIdx.y;
  const QrcpTask& t = tasks[ti];
  if (!t.active) return;
  const IdBlk& B = blks[ti];
  const int L = B.lc;
  if (B.ncand <= 0 || L <= 0) return;
  const int k = B.k, nr = t.d - k;
  const int r0 = blockIdx.x * kIdbRows;
  if (r0 >= nr) return;
  const int tid = threadIdx.x;
  constexpr int LP = kIdbLmax + 1;
  double* R1 = Qc;   // kIdbLmax x LP
#pragma unroll
  for (int e = tid; e < kIdbLmax * kIdbLmax; e += kIdbRows) R1[(e / kIdbLmax) * LP + e % kIdbLmax] = B.F[e];
  if (tid < L) colp[tid] = (int64_t)B.cand[B.piv[tid]] * t.ldw + k;
  __syncthreads();
  if (tid < L) rinv[tid] = 1.0 / R1[tid * LP + tid];
  __syncthreads();
  const int r = r0 + tid;
  double x[kIdbLmax];
#pragma unroll
  for (int j = 0; j < kIdbLmax; ++j) x[j] = 0.0;
  if (r < nr) {
    const HSS_GLOBAL double* W0 = gview(t.W);
#pragma unroll
    for (int j = 0; j < kIdbLmax; ++j)
      if (j < L) x[j] = W0[colp[j] + r];
#pragma unroll
    for (int j = 0; j < kIdbLmax; ++j) {
      if (j >= L) continue;
      double s = x[j];
#pragma unroll
      for (int i = 0; i < kIdbLmax; ++i)
        if (i < j) s -= x[i] * R1[i * LP + j];
      x[j] = s * rinv[j];
    }
#pragma unroll
    for (int j = 0; j < kIdbLmax; ++j)
      if (j < L) B.V[(int64_t)j * B.ldv + r] = x[j];
  }
  __syncthreads();   // R1 is overwritten by the rows
#pragma unroll
  for (int j = 0; j < kIdbLmax; j += 2)
    *reinterpret_cast<double2*>(&Qc[tid * kIdbLmax + j]) = make_double2(x[j], x[j + 1]);
  __syncthreads();
  // block (bi, bj), bi <= bj, of group grp: rows grp, grp + kGrp4, ...
  const int blk = tid % kBlk4, grp = tid / kBlk4;
  int bi = 0, rem = blk;
  while (rem >= kNb4 - bi) { rem -= kNb4 - bi; ++bi; }
  const int bj = bi + rem;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  const int rows = min(kIdbRows, nr - r0);
  if (grp < kGrp4) {
#pragma unroll 4
    for (int w = grp; w < rows; w += kGrp4) {
      const double2 a01 = *reinterpret_cast<const double2*>(&Qc[w * kIdbLmax + 4 * bi]);
      const double2 a23 = *reinterpret_cast<const double2*>(&Qc[w * kIdbLmax + 4 * bi + 2]);
      const double2 b01 = *reinterpret_cast<const double2*>(&Qc[w * kIdbLmax + 4 * bj]);
      const double2 b23 = *reinterpret_cast<const double2*>(&Qc[w * kIdbLmax + 4 * bj + 2]);
      const double a[4] = {a01.x, a01.y, a23.x, a23.y}, b[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u * 4 + v] += a[u] * b[v];
    }
  }
  __syncthreads();   // the rows are overwritten by the group sums
  if (grp < kGrp4) {
#pragma unroll
    for (int q = 0; q < 16; ++q) Qc[(grp * kBlk4 + blk) * 16 + q] = acc[q];
  }
  __syncthreads();
  double* P = B.P + (int64_t)blockIdx.x * kIdbPart;
  for (int e = tid; e < kIdbPart; e += kIdbRows) {
    double s = 0.0;
    for (int g = 0; g < kGrp4; ++g) s += Qc[g * kIdbPart + e];
    P[e] = s;
  }
}

// Step 3b: the block's small factors.  G2 = Q1^T Q1 (the row workgroups'
// sums, in order); Cholesky QR again: R2 = chol(G2), R = R2 R1, Q_1 = the
// top L rows of Q1 R2^{-1}; the reflectors rebuilt from Q (Ballard et al.,
// "Reconstructing Householder vectors from tall-skinny QR", 2015): with
// S = -sign(diag Q_1) and the LU factorization Q_1 - S = Y_1 Uf, the
// reflectors are Y = [Y_1; Q_2 (Uf R2)^{-1}] with T = -Uf S Y_1^{-T}, so that
// (I - Y T Y^T)^T C_P = [S R; 0].  Writes R of the pivots into the panel
// and the pivot order; M = Uf R2, T and Y_1 for the second row pass, which
// also lists the remaining columns and writes the GEMM tasks of the update.
// One workgroup of kIdbLmax^2 threads per task, thread (a, b) on entry
// (a, b); each elimination step is one barrier (the step's pivot row and
// column are read from the input, the step's results go to another array).
constexpr int SMT = kIdbLmax * kIdbLmax;
__global__ __launch_bounds__(SMT) void k_idb_small(const QrcpTask* __restrict__ tasks, IdBlk* __restrict__ blks,
                                                   GemmTask* __restrict__ gt, int ntasks,
                                                   unsigned long long* __restrict__ kcnt) {
  constexpr int LP = kIdbLmax + 1;
  __shared__ double R1[kIdbLmax][LP], Wk[kIdbLmax][LP], R2[kIdbLmax][LP], Q[kIdbLmax][LP], X[kIdbLmax][LP],
      Y1[kIdbLmax][LP];
  __shared__ double Sg[kIdbLmax], rdg[kIdbLmax];
  __shared__ int piv[kIdbLmax];
  const int ti = blockIdx.x;
  const QrcpTask& t = tasks[ti];
  IdBlk& B = blks[ti];
  const int tid = threadIdx.x;
  if (tid == 0) { gt[ntasks + ti].M = 0; gt[2 * ntasks + ti].M = 0; }
  if (!t.active) return;
  if (B.ncand <= 0) return;
  const int m = t.m, d = t.d, k = B.k;
  const int nr = d - k;
  const int Lchol = B.lc;
  const int a = tid / kIdbLmax, b = tid % kIdbLmax;
  {
    const int nrb = (nr + kIdbRows - 1) / kIdbRows;
    const HSS_GLOBAL double* P = gview(B.P);
    R1[a][b] = B.F[tid];
    // G2(a, b) from the upper 4 x 4 blocks of the row workgroups' partial sums
    double g = 0.0;
    if (a < Lchol && b < Lchol) {
      const int lo = min(a, b), hi = max(a, b);
      const int i4 = lo >> 2, j4 = hi >> 2;
      const int blk = i4 * kNb4 - i4 * (i4 - 1) / 2 + (j4 - i4);
      const int q = (lo == a) ? (a & 3) * 4 + (b & 3) : (b & 3) * 4 + (a & 3);
      const HSS_GLOBAL double* pp = P + blk * 16 + q;
      double g1 = 0.0;
      int pb = 0;
      for (; pb + 1 < nrb; pb += 2) { g += pp[(int64_t)pb * kIdbPart]; g1 += pp[(int64_t)(pb + 1) * kIdbPart]; }
      if (pb < nrb) g += pp[(int64_t)pb * kIdbPart];
      g += g1;
    }
    Wk[a][b] = g;
    R2[a][b] = 0.0;
    Q[a][b] = (a < Lchol && b < Lchol) ? B.V[(int64_t)b * B.ldv + a] : 0.0;
    if (tid < Lchol) piv[tid] = B.piv[tid];
  }
  __syncthreads();
  // R2 = chol(G2), right-looking on Wk (upper part); a pivot whose second
  // Cholesky step breaks down ends the block before it
  int L = Lchol;
  for (int j = 0; j < L; ++j) {
    const double dj = Wk[j][j];
    if (!(dj > 1e-290)) { L = j; break; }
    const double inv = rsq_nr(dj);
    if (a == j && b >= j && b < L) R2[j][b] = b == j ? dj * inv : Wk[j][b] * inv;
    if (tid == 0) rdg[j] = inv;
    if (a > j && a <= b && b < L) Wk[a][b] -= Wk[j][a] * Wk[j][b] * (inv * inv);
    __syncthreads();
  }
  // X = Q_1 = Q1_1 R2^{-1} by columns: column j final at step j; Q holds the
  // right-hand sides still to reduce
  for (int j = 0; j < L; ++j) {
    const double r = rdg[j];
    if (b == j && a < L) X[a][j] = Q[a][j] * r;
    if (b > j && b < L && a < L) Q[a][b] -= Q[a][j] * r * R2[j][b];
    __syncthreads();
  }
  // R = R2 R1 (upper) into Wk
  {
    double sv = 0.0;
    if (a <= b && b < L)
      for (int c = a; c <= b; ++c) sv += R2[a][c] * R1[c][b];
    Wk[a][b] = sv;
  }
  // S = -sign(diag Q_1); Q = Q_1 - S for the LU without pivoting
  if (tid < L) Sg[tid] = X[tid][tid] >= 0.0 ? -1.0 : 1.0;
  __syncthreads();
  Q[a][b] = (a < L && b < L) ? X[a][b] - (a == b ? Sg[a] : 0.0) : 0.0;
  Y1[a][b] = a == b ? 1.0 : 0.0;
  __syncthreads();
  // LU: the multipliers of step j go to Y1's column j; Q's upper part becomes Uf
  for (int j = 0; j < L; ++j) {
    const double r = rcp_nr(Q[j][j]);   // |Uf_jj| >= 1
    if (b == j && a > j && a < L) Y1[a][j] = Q[a][j] * r;
    if (a > j && b > j && a < L && b < L) Q[a][b] -= Q[a][j] * r * Q[j][b];
    __syncthreads();
  }
  // M = Uf R2 (upper) into R1 (R = R2 R1 is done); X = -Uf S, the right-hand
  // sides of T Y_1^T = -Uf S
  {
    double sv = 0.0;
    if (a <= b && b < L)
      for (int c = a; c <= b; ++c) sv += Q[a][c] * R2[c][b];
    R1[a][b] = sv;
    X[a][b] = (a <= b && b < L) ? -Q[a][b] * Sg[b] : 0.0;
  }
  __syncthreads();
  // T by columns (Y_1^T unit upper): column j final at step j, into R2
  for (int j = 0; j < L; ++j) {
    if (b == j) R2[a][j] = a <= j ? X[a][j] : 0.0;
    if (b > j && b < L) X[a][b] -= X[a][j] * Y1[b][j];
    __syncthreads();
  }
  // M, T, Y_1 for the second row pass
  {
    constexpr int LL = kIdbLmax * kIdbLmax;
    const bool in = a < L && b < L;
    B.F[LL + tid] = in ? R1[a][b] : 0.0;
    B.F[2 * LL + tid] = in && a <= b ? R2[a][b] : 0.0;
    B.F[3 * LL + tid] = in ? Y1[a][b] : (a == b ? 1.0 : 0.0);
  }
  // R of the pivots (S R) into the panel rows k .. k + L - 1, the diagonal,
  // the pivot order; pivots leave the norm buffers
  if (a < b && b < L) t.W[(int64_t)B.cand[piv[b]] * t.ldw + k + a] = Sg[a] * Wk[a][b];
  if (tid < L) {
    const int col = B.cand[piv[tid]];
    rdiagb(t)[k + tid] = Sg[tid] * Wk[tid][tid];
    if (t.J) t.J[k + tid] = col;
    nrmb(t, 0)[col] = -1.0;
    nrmb(t, 1)[col] = -1.0;
  }
  if (tid == 0) {
    const double cells = (double)nr * (double)(m - k);
    kcount(kcnt, HSS_K_QRCP_STEP, 8.0 * cells * 3.0, 4.0 * cells * L);
    B.L = L;
    B.kb = k;
    B.k = k + L;
    if (B.stop && L == Lchol) {
      QrcpCtlB* ctl = ctlb(t);
      ctl->rank = k + L;
      ctl->done = 1;
    }
  }
}

// Step 3c: the reflectors V (Y_1 on top, the rows of Q1 times M^{-1} below)
// and U_w = V T^T, one panel row per thread; the last workgroup of a task
// lists the columns left after the block (ascending) and writes the GEMM
// tasks of the update.
__global__ __launch_bounds__(kIdbRows) void k_idb_rows2(const QrcpTask* __restrict__ tasks, IdBlk* __restrict__ blks,
                                                        GemmTask* __restrict__ gt, int ntasks) {
  constexpr int LP = kIdbLmax + 1;
  __shared__ double Ms[kIdbLmax][LP], Ts[kIdbLmax][LP], Ys[kIdbLmax][LP];
  __shared__ double rinv[kIdbLmax];
  const int ti = blockIdx.y;
  const QrcpTask& t = tasks[ti];
  if (!t.active) return;
  IdBlk& B = blks[ti];
  const int L = B.L;
  if (L <= 0) return;
  const int nr = t.d - B.kb;
  const int tid = threadIdx.x;
  if (blockIdx.x == gridDim.x - 1) {
    __shared__ int sh_cnt[kIdbRows / 64 + 1];
    const int m = t.m, k = B.kb;
    const HSS_GLOBAL double* nrm = gview(nrmb(t, 0));
    const int per = (m + kIdbRows - 1) / kIdbRows;
    const int j0 = min(m, tid * per), j1 = min(m, j0 + per);
    int cnt = 0;
    for (int j = j0; j < j1; ++j) cnt += nrm[j] >= 0.0;
    int nrest = 0;
    int pos = block_excl_scan<kIdbRows>(cnt, sh_cnt, &nrest);
    for (int j = j0; j < j1; ++j)
      if (nrm[j] >= 0.0) B.rest[pos++] = j;
    if (tid == 0) {
      B.nrest = nrest;
      if (nrest > 0) {
        // Y = V^T W(k:d, rest)
        GemmTask q;
        q.A = B.V; q.a_rs = B.ldv; q.a_cs = 1;
        q.B = t.W + k; q.b_rs = 1; q.b_cs = t.ldw; q.b_cols = B.rest;
        q.C = B.Y; q.c_rs = 1; q.c_cs = kIdbLmax;
        q.M = L; q.N = nrest; q.K = nr; q.pad = 0;
        q.alpha = 1.0; q.beta = 0.0;
        gt[ntasks + ti] = q;
        // W(k:d, rest) -= U_w Y
        GemmTask u;
        u.A = B.U; u.a_rs = 1; u.a_cs = B.ldv;
        u.B = B.Y; u.b_rs = 1; u.b_cs = kIdbLmax;
        u.C = t.W + k; u.c_rs = 1; u.c_cs = t.ldw; u.c_cols = B.rest;
        u.M = nr; u.N = nrest; u.K = L; u.pad = 0;
        u.alpha = -1.0; u.beta = 1.0;
        gt[2 * ntasks + ti] = u;
      }
    }
    return;
  }
  const int r0 = blockIdx.x * kIdbRows;
  if (r0 >= nr) return;
  constexpr int LL = kIdbLmax * kIdbLmax;
#pragma unroll
  for (int e = tid; e < LL; e += kIdbRows) {
    const int a = e / kIdbLmax, b = e % kIdbLmax;
    Ms[a][b] = B.F[LL + e];
    Ts[a][b] = B.F[2 * LL + e];
    Ys[a][b] = B.F[3 * LL + e];
  }
  __syncthreads();
  if (tid < L) rinv[tid] = 1.0 / Ms[tid][tid];
  __syncthreads();
  const int r = r0 + tid;
  if (r >= nr) return;
  double v[kIdbLmax];
  if (r < L) {
#pragma unroll
    for (int j = 0; j < kIdbLmax; ++j) v[j] = j < r ? Ys[r][j] : (j == r ? 1.0 : 0.0);
  } else {
#pragma unroll
    for (int j = 0; j < kIdbLmax; ++j) v[j] = j < L ? B.V[(int64_t)j * B.ldv + r] : 0.0;
#pragma unroll
    for (int j = 0; j < kIdbLmax; ++j) {
      if (j >= L) continue;
      double sv = v[j];
#pragma unroll
      for (int i = 0; i < kIdbLmax; ++i)
        if (i < j) sv -= v[i] * Ms[i][j];
      v[j] = sv * rinv[j];
    }
  }
#pragma unroll
  for (int j = 0; j < kIdbLmax; ++j)
    if (j < L) B.V[(int64_t)j * B.ldv + r] = v[j];
#pragma unroll
  for (int j = 0; j < kIdbLmax; ++j) {
    if (j >= L) continue;
    double sv = 0.0;
#pragma unroll
    for (int i = 0; i < kIdbLmax; ++i)
      if (i >= j && i < L) sv += v[i] * Ts[j][i];
    B.U[(int64_t)j * B.ldv + r] = sv;
  }
}

// Step 4b: exact residual norms of the remaining columns (rows k .. d after
// the block's update), one wave per column, into both norm buffers.
__global__ __launch_bounds__(64 * NRMW) void k_idb_norms(const QrcpTask* __restrict__ tasks,
                                                         const IdBlk* __restrict__ blks) {
  const int ti = blockIdx.y;
  const QrcpTask& t = tasks[ti];
  if (!t.active) return;
  const IdBlk& B = blks[ti];
  if (B.L <= 0) return;
  const int pos = blockIdx.x * NRMW + (threadIdx.x >> 6);
  if (pos >= B.nrest) return;
  const int lane = threadIdx.x & 63;
  const int col = B.rest[pos];
  const HSS_GLOBAL double* y = gview(t.W + (int64_t)col * t.ldw);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int r = B.k + lane;
  for (; r + 192 < t.d; r += 256) {
    const double a = y[r], b = y[r + 64], c = y[r + 128], e = y[r + 192];
    s0 += a * a; s1 += b * b; s2 += c * c; s3 += e * e;
  }
  for (; r < t.d; r += 64) { const double a = y[r]; s0 += a * a; }
  const double s = wave_sum((s0 + s1) + (s2 + s3));
  if (lane == 0) {
    const double v = sqrt(s);
    nrmb(t, 0)[col] = v;
    nrmb(t, 1)[col] = v;
  }
}

// Tasks still factoring: not done and k below min(m, d).  One workgroup.
__global__ __launch_bounds__(1024) void k_idb_alive(const QrcpTask* __restrict__ tasks, const IdBlk* __restrict__ blks,
                                                    int ntasks, int32_t* __restrict__ out) {
  __shared__ int sa[16];
  int alive = 0;
  for (int i = threadIdx.x; i < ntasks; i += 1024) {
    const QrcpTask& t = tasks[i];
    if (!t.active) continue;
    alive += !ctlb(t)->done && blks[i].k < min(t.m, t.d);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) alive += __shfl_xor(alive, o, 64);
  if ((threadIdx.x & 63) == 0) sa[threadIdx.x >> 6] = alive;
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0;
    for (int w = 0; w < 16; ++w) a += sa[w];
    out[0] = a;
  }
}

void run_id_blocks(QrcpTask* tasks, int32_t ntasks, const IdBlockWork& bw, int32_t dmax, int32_t mmax,
                   int32_t* hw_dev, const int32_t* hw, double* gws, hipStream_t s, unsigned long long* kcnt) {
  if (ntasks > bw.max_tasks) throw Error(HSS_ERR_INTERNAL, "block ID workspace too small for the batch");
  hipLaunchKernelGGL(k_idb_start, dim3((ntasks + 127) / 128), dim3(128), 0, s, tasks, bw.blk, ntasks);
  const int cm = kIdbCmax;
  // dynamic LDS: Cholesky rows + packed Gram (k_idb_chol); Q1 rows (k_idb_rows1)
  constexpr size_t kLdsChol = sizeof(double) * 2 * (size_t)kIdbLmax * kIdbCmax;   // Lc and Lu
  constexpr size_t kLdsRows = sizeof(double) * (size_t)kIdbRows * kIdbLmax;
  static_assert(kLdsChol <= 160 * 1024 && kLdsRows <= 160 * 1024, "block ID LDS");
  static_assert(kLdsRows >= sizeof(double) * kGrp4 * kIdbPart, "group sums fit the rows' LDS");
  static thread_local bool attr_set = false;   // dynamic LDS above 64 KB
  if (!attr_set) {
    HSS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_idb_chol),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsChol));
    HSS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_idb_rows1),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsRows));
    HSS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_idb_select),
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)(sizeof(uint64_t) * kIdbMaxM)));
    attr_set = true;
  }
  const unsigned nrb = (unsigned)std::max(1, (dmax + kIdbRows - 1) / kIdbRows);
  const int kmax = std::max(1, std::min(dmax, mmax));
  constexpr int kPoll = 4;
  for (int b = 0; b < kmax; ++b) {
    if (b > 0 && b % kPoll == 0) {
      hipLaunchKernelGGL(k_idb_alive, dim3(1), dim3(1024), 0, s, tasks, bw.blk, ntasks, hw_dev);
      HSS_HIP_CHECK(hipStreamSynchronize(s));
      if (hw[0] == 0) break;
    }
    prof_begin(s);
    hipLaunchKernelGGL(k_idb_select, dim3(ntasks), dim3(SELT), sizeof(uint64_t) * (size_t)std::max(mmax, 1), s, tasks,
                       bw.blk, bw.gt, ntasks);
    const unsigned gx = (unsigned)std::max(1, std::min(16, (dmax + 255) / 256));
    hipLaunchKernelGGL(k_idb_gather, dim3(gx, cm, ntasks), dim3(256), 0, s, tasks, bw.blk);
    prof_end(HSS_K_QRCP_STEP, s, 2);
    launch_gemm(bw.gt, ntasks, cm, cm, s, nullptr, dmax, gws, kGemmSplitElems, HSS_K_QRCP_STEP);
    prof_begin(s);
    hipLaunchKernelGGL(k_idb_chol, dim3(ntasks), dim3(PCT), kLdsChol, s, tasks, bw.blk);
    hipLaunchKernelGGL(k_idb_rows1, dim3(nrb, ntasks), dim3(kIdbRows), kLdsRows, s, tasks, bw.blk);
    hipLaunchKernelGGL(k_idb_small, dim3(ntasks), dim3(SMT), 0, s, tasks, bw.blk, bw.gt, ntasks, kcnt);
    hipLaunchKernelGGL(k_idb_rows2, dim3(nrb + 1, ntasks), dim3(kIdbRows), 0, s, tasks, bw.blk, bw.gt, ntasks);
    prof_end(HSS_K_QRCP_STEP, s);
    launch_gemm(bw.gt + ntasks, ntasks, kIdbLmax, mmax, s, nullptr, dmax, gws, kGemmSplitElems, HSS_K_QRCP_STEP);
    launch_gemm(bw.gt + 2 * ntasks, ntasks, dmax, mmax, s, nullptr, 0, nullptr, 0, HSS_K_QRCP_STEP);
    prof_begin(s);
    hipLaunchKernelGGL(k_idb_norms, dim3((unsigned)((mmax + NRMW - 1) / NRMW), ntasks), dim3(64 * NRMW), 0, s, tasks,
                       bw.blk);
    prof_end(HSS_K_QRCP_STEP, s);
  }
  HSS_HIP_CHECK(hipGetLastError());
}

}  // namespace hss
