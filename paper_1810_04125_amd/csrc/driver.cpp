// Host driver of the adaptive HSS compression (Alg. 3, HSSCompressAdaptive).
//
// A job holds one or more independent problems.  All their nodes live in
// one node table; the per-level kernels cover one tree level of every
// problem per launch (Sec. 4: level-synchronised traversal), and the
// sampling step covers every problem still open.  Device memory is sized
// once from capacities (rank <= min(m, d_max)), so no allocation or
// host round trip happens inside a round; the host reads back only the
// root states at the end of each round to decide whether to sample more.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "driver.h"

namespace hss {

thread_local Prof* g_prof = nullptr;

void prof_begin(hipStream_t s) {
  if (g_prof && g_prof->on) hipEventRecord(g_prof->e0, s);
}

void prof_end(int cls, hipStream_t s, int nlaunch) {
  if (!g_prof) return;
  g_prof->launches[cls] += nlaunch;
  if (!g_prof->on) return;
  hipEventRecord(g_prof->e1, s);
  hipEventSynchronize(g_prof->e1);
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, g_prof->e0, g_prof->e1) == hipSuccess) g_prof->ms[cls] += ms;
}

void prof_count(int cls, int n) {
  if (g_prof) g_prof->launches[cls] += n;
}

// Makes the job's profiler current for the calling thread while alive.
struct ProfScope {
  Prof* saved;
  explicit ProfScope(Prof* p) : saved(g_prof) { g_prof = p; }
  ~ProfScope() { g_prof = saved; }
};

// Relative noise level of the reduced-precision samples below which the
// relative thresholds are not lowered: the measured sample accuracy (FP32
// 1.4e-7 overall, 5.4e-7 in the worst column; BF16x3 4.0e-6 and 1.7e-5, on
// the n = 65536 Gaussian-kernel workload), with margin.
constexpr double kFloorFp32 = 5e-7;
constexpr double kFloorBf16x3 = 1e-5;

int64_t align8(int64_t x) { return (x + 7) & ~int64_t(7); }

Job::~Job() {
  if (stream) hipStreamSynchronize(stream);
  arena_return();
  for (void* p : transients) dfree(p);
  for (void* p : allocs) dfree(p);
  hipStreamSynchronize(stream);
  if (ev0) hipEventDestroy(ev0);
  if (ev1) hipEventDestroy(ev1);
  if (ev_flag) hipEventDestroy(ev_flag);
  if (hflags) hipHostFree(hflags);
  if (sched_h) hipHostFree(sched_h);
  if (prof.e0) hipEventDestroy(prof.e0);
  if (prof.e1) hipEventDestroy(prof.e1);
}

// Device memory comes from the device's stream-ordered memory pool with
// the release threshold raised, so memory freed by one job is kept mapped
// and reused by the next one instead of being returned and re-mapped.
static void keep_pool_memory() {
  static bool done = false;
  if (done) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  hipGetLastError();
  done = true;
}

// After an out-of-memory failure: memory freed into the stream-ordered pool
// stays mapped (the release threshold above), and plain allocations cannot
// use it; give it back to the device before one retry.
static void trim_pool_memory() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  hipDeviceSynchronize();
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) hipMemPoolTrimTo(pool, 0);
  hipGetLastError();
}

// The transient buffers of a compression (local samples, bases, level
// workspaces: sized from d_max, often tens of GB) are carved from one
// block per device that outlives the job: freeing and re-mapping that much
// memory for every call costs seconds, reusing it costs nothing.  A job
// takes the block if it is idle and large enough, replaces it by a larger
// one if needed, and hands it back when the compression ends; a job that
// finds it busy (another thread) allocates its own.  hss_release_cache
// frees idle blocks.
namespace {
struct Arena {
  void* p = nullptr;
  size_t bytes = 0;
  bool busy = false;
};
std::mutex g_arena_mu;
std::map<int, Arena> g_arena;
}  // namespace

size_t arena_idle_bytes() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(g_arena_mu);
  auto it = g_arena.find(dev);
  return (it == g_arena.end() || it->second.busy) ? 0 : it->second.bytes;
}

void arena_release_idle() {
  int dev = 0;
  HSS_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_arena_mu);
  auto it = g_arena.find(dev);
  if (it == g_arena.end() || it->second.busy || !it->second.p) return;
  HSS_HIP_CHECK(hipDeviceSynchronize());
  HSS_HIP_CHECK(hipFree(it->second.p));
  g_arena.erase(it);
}

void* Job::arena_acquire(size_t bytes) {
  if (ualloc.alloc) return dalloc(bytes, true);   // the caller's allocator keeps its own cache
  keep_pool_memory();
  int dev = 0;
  HSS_HIP_CHECK(hipGetDevice(&dev));
  const auto t0 = std::chrono::steady_clock::now();
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_arena_mu);
    Arena& a = g_arena[dev];
    if (!a.busy) {
      if (a.bytes < bytes) {
        if (a.p) {
          HSS_HIP_CHECK(hipDeviceSynchronize());
          hipFree(a.p);
        }
        a.p = nullptr;
        a.bytes = 0;
        hipError_t e = hipMalloc(&a.p, bytes);
        if (e == hipErrorOutOfMemory) {
          hipGetLastError();
          trim_pool_memory();
          e = hipMalloc(&a.p, bytes);
        }
        if (e != hipSuccess) {
          hipGetLastError();
          a.p = nullptr;
          throw Error(e == hipErrorOutOfMemory ? HSS_ERR_OUT_OF_MEMORY : HSS_ERR_DEVICE,
                      "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
        }
        a.bytes = bytes;
      }
      a.busy = true;
      p = a.p;
      arena_dev = dev;
    }
  }
  if (!p) p = dalloc(bytes, true);   // block in use by another job
  alloc_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return p;
}

void Job::arena_return() {
  if (arena_dev < 0) return;
  std::lock_guard<std::mutex> lk(g_arena_mu);
  g_arena[arena_dev].busy = false;
  arena_dev = -1;
}

void* Job::dalloc(size_t bytes, bool transient) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  const auto t0 = std::chrono::steady_clock::now();
  if (ualloc.alloc) {
    p = ualloc.alloc(ualloc.ctx, bytes, stream);
    alloc_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (!p) throw Error(HSS_ERR_OUT_OF_MEMORY, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
    (transient ? transients : allocs).push_back(p);
    return p;
  }
  keep_pool_memory();
  hipError_t e = hipMallocAsync(&p, bytes, stream);
  if (e == hipErrorOutOfMemory) {
    hipGetLastError();
    trim_pool_memory();
    e = hipMallocAsync(&p, bytes, stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);   // usable from any stream from now on
  alloc_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (e != hipSuccess) {
    hipGetLastError();
    throw Error(e == hipErrorOutOfMemory ? HSS_ERR_OUT_OF_MEMORY : HSS_ERR_DEVICE,
                "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  (transient ? transients : allocs).push_back(p);
  return p;
}

void Job::dfree(void* p) {
  if (!p) return;
  if (ualloc.alloc) {
    if (ualloc.free) ualloc.free(ualloc.ctx, p, stream);
  } else {
    hipFreeAsync(p, stream);
  }
}

void Job::drop(void* p) {
  if (!p) return;
  for (std::vector<void*>* v : {&allocs, &transients}) {
    auto it = std::find(v->begin(), v->end(), p);
    if (it != v->end()) v->erase(it);
  }
  dfree(p);
}

// E of every node side and B12 / B21 of every non-leaf move from their
// capacity-sized slots in the transient pool to exactly sized blocks of the
// persistent E pool (E: rank x (m - rank); B: ranks of the children).
void Job::compact_e() {
  std::vector<Copy2D> cp;
  int64_t tot = 0;
  std::vector<int64_t> newoff(4 * desc.size(), 0);
  for (size_t g = 0; g < desc.size(); ++g) {
    const NodeDesc& d = desc[g];
    if (d.left >= 0) {   // B12: rank_r(left) x rank_c(right), B21: rank_r(right) x rank_c(left)
      const NodeState &sl = st_h[d.left], &sr = st_h[d.right];
      newoff[4 * g + 2] = tot;
      tot += align8((int64_t)std::max(sl.rank[0], 1) * std::max(sr.rank[1], 1));
      newoff[4 * g + 3] = tot;
      tot += align8((int64_t)std::max(sr.rank[0], 1) * std::max(sl.rank[1], 1));
    }
    if (d.parent < 0) continue;
    const int nsides = probs[d.prob].sym ? 1 : 2;
    for (int s = 0; s < nsides; ++s) {
      const int32_t r = st_h[g].rank[s], m = st_h[g].m[s];
      newoff[4 * g + s] = tot;
      tot += align8((int64_t)std::max(r, 1) * std::max(m - r, 1));
    }
  }
  epool = (double*)dalloc(sizeof(double) * std::max<int64_t>(tot, 1));
  for (size_t g = 0; g < desc.size(); ++g) {
    NodeDesc& d = desc[g];
    if (d.left >= 0) {
      const NodeState &sl = st_h[d.left], &sr = st_h[d.right];
      const int32_t r1 = sl.rank[0], c2 = sr.rank[1], r2 = sr.rank[0], c1 = sl.rank[1];
      if (r1 > 0 && c2 > 0) cp.push_back(Copy2D{tpool + d.B12, d.b12ld, epool + newoff[4 * g + 2], r1, r1, c2});
      if (r2 > 0 && c1 > 0) cp.push_back(Copy2D{tpool + d.B21, d.b21ld, epool + newoff[4 * g + 3], r2, r2, c1});
      d.B12 = newoff[4 * g + 2];
      d.b12ld = std::max(r1, 1);
      d.B21 = newoff[4 * g + 3];
      d.b21ld = std::max(r2, 1);
    }
    if (d.parent < 0) continue;
    const int nsides = probs[d.prob].sym ? 1 : 2;
    for (int s = 0; s < nsides; ++s) {
      const int32_t r = st_h[g].rank[s], m = st_h[g].m[s];
      if (r > 0 && m > r) cp.push_back(Copy2D{tpool + d.E[s], d.rcap, epool + newoff[4 * g + s], r, r, m - r});
      d.E[s] = newoff[4 * g + s];
      d.eld[s] = std::max(r, 1);
    }
    if (probs[d.prob].sym) {
      d.E[1] = d.E[0];
      d.eld[1] = d.eld[0];
    }
  }
  if (!cp.empty()) {
    Copy2D* cd = (Copy2D*)dalloc(sizeof(Copy2D) * cp.size(), true);
    HSS_HIP_CHECK(hipMemcpy(cd, cp.data(), sizeof(Copy2D) * cp.size(), hipMemcpyHostToDevice));
    launch_copy2d(cd, (int32_t)cp.size(), stream);
  }
  HSS_HIP_CHECK(hipMemcpyAsync(desc_d, desc.data(), sizeof(NodeDesc) * desc.size(), hipMemcpyHostToDevice, stream));
  HSS_HIP_CHECK(hipStreamSynchronize(stream));
}

// After compression only D, B, E, J, I, the node states and the tables the
// matvec needs stay on the device.
void Job::release_transients() {
  HSS_HIP_CHECK(hipStreamSynchronize(stream));
  arena_return();
  for (void* p : transients) dfree(p);
  HSS_HIP_CHECK(hipStreamSynchronize(stream));
  transients.clear();
  tpool = wsa = wsb = partial = gemm_ws = nullptr;
}

void Job::validate(const hss_generator& g, const hss_tree* t, const hss_options& o, int k) {
  const std::string who = "problem " + std::to_string(k) + ": ";
  if (!t || !t->perm || !t->lo || !t->hi || !t->left || !t->right || !t->parent || !t->level)
    throw Error(HSS_ERR_INVALID_ARG, who + "incomplete tree");
  if (g.n != t->n || g.n < 1) throw Error(HSS_ERR_INVALID_ARG, who + "generator n != tree n");
  if ((o.allocator.alloc == nullptr) != (o.allocator.free == nullptr))
    throw Error(HSS_ERR_INVALID_ARG, who + "allocator needs both alloc and free");
  if (g.family < 0 || g.family > HSS_FAM_CALLBACK) throw Error(HSS_ERR_INVALID_ARG, who + "unknown family");
  if (g.family == HSS_FAM_CALLBACK && (!g.sample || !g.extract))
    throw Error(HSS_ERR_INVALID_ARG, who + "callback family needs sample and extract routines");
  if ((g.family == HSS_FAM_LAPLACE || g.family == HSS_FAM_GAUSS) && !g.points)
    throw Error(HSS_ERR_INVALID_ARG, who + "kernel family needs points");
  if (g.family == HSS_FAM_DENSE && (!g.dense || g.ld < g.n))
    throw Error(HSS_ERR_INVALID_ARG, who + "dense family needs dense and ld >= n");
  if (g.family == HSS_FAM_TOEPLITZ && !(g.h > 0.0)) throw Error(HSS_ERR_INVALID_ARG, who + "toeplitz needs h > 0");
  if (g.family == HSS_FAM_GAUSS && !(g.sigma > 0.0)) throw Error(HSS_ERR_INVALID_ARG, who + "gauss needs sigma > 0");
  if (!(o.rtol >= 0.0) || !(o.atol >= 0.0) || !(o.eta > 0.0))
    throw Error(HSS_ERR_INVALID_ARG, who + "need rtol >= 0, atol >= 0, eta > 0");
  if (o.strategy < 0 || o.strategy > 3) throw Error(HSS_ERR_INVALID_ARG, who + "unknown strategy");
  if ((!o.predictor && o.d0 < 1) || o.d_max < 1) throw Error(HSS_ERR_INVALID_ARG, who + "need d0 >= 1 and d_max >= 1");
  if (o.predictor && (!gen_formula(g.family) || (o.strategy != HSS_INC_FNORM && o.strategy != HSS_INC_HMT)))
    throw Error(HSS_ERR_INVALID_ARG, who + "the predictor needs a generated family and an incrementing strategy");
  if (o.predictor && !(o.rtol > 0.0)) throw Error(HSS_ERR_INVALID_ARG, who + "the predictor needs rtol > 0");
  if ((o.strategy == HSS_INC_FNORM || o.strategy == HSS_INC_HMT) && o.delta_d < 1)
    throw Error(HSS_ERR_INVALID_ARG, who + "need delta_d >= 1");
  if (o.strategy == HSS_INC_HMT && !(o.hmt_alpha >= 0.0)) throw Error(HSS_ERR_INVALID_ARG, who + "need hmt_alpha >= 0");
  if (o.strategy == HSS_DBL_HMT && o.oversample_p < 0) throw Error(HSS_ERR_INVALID_ARG, who + "need p >= 0");
  if (std::min<int64_t>(o.d_max, g.n) > HSS_MAX_D)
    throw Error(HSS_ERR_INVALID_ARG, who + "d_max above HSS_MAX_D (" + std::to_string(HSS_MAX_D) +
                                         "): the ID's pivot step keeps one double per sample in LDS");
  if (o.R && (o.ldr < g.n || o.ncols_R < std::min<int64_t>(o.d_max, g.n)))
    throw Error(HSS_ERR_INVALID_ARG, who + "R must be n x ncols_R with ncols_R >= min(d_max, n)");
  if (o.sample_precision < 0 || o.sample_precision > 2) throw Error(HSS_ERR_INVALID_ARG, who + "bad precision");
  if (o.sample_precision != HSS_SAMPLE_FP64 && !gen_formula(g.family))
    throw Error(HSS_ERR_INVALID_ARG, who + "reduced-precision sampling needs a generated family");
  // tree structure
  const int32_t nn = t->num_nodes;
  if (nn < 1 || t->lo[0] != 0 || t->hi[0] != g.n || t->parent[0] != -1 || t->level[0] != 0)
    throw Error(HSS_ERR_INVALID_ARG, who + "root must own [0, n) at level 0");
  {
    // perm gathers points and indexes generated entries on the device: it
    // must hold every index of [0, n) exactly once
    std::vector<uint8_t> seen((size_t)g.n, 0);
    for (int64_t i = 0; i < g.n; ++i) {
      const int64_t v = t->perm[i];
      if (v < 0 || v >= g.n || seen[(size_t)v]) throw Error(HSS_ERR_INVALID_ARG, who + "perm is not a permutation of [0, n)");
      seen[(size_t)v] = 1;
    }
  }
  for (int32_t v = 0; v < nn; ++v) {
    if (t->hi[v] <= t->lo[v]) throw Error(HSS_ERR_INVALID_ARG, who + "empty tree node");
    const int32_t l = t->left[v], r = t->right[v];
    if ((l < 0) != (r < 0)) throw Error(HSS_ERR_INVALID_ARG, who + "nodes need zero or two children");
    if (l >= 0) {
      if (l <= v || r <= v || l >= nn || r >= nn || t->lo[l] != t->lo[v] || t->hi[l] != t->lo[r] ||
          t->hi[r] != t->hi[v] || t->parent[l] != v || t->parent[r] != v || t->level[l] != t->level[v] + 1 ||
          t->level[r] != t->level[v] + 1)
        throw Error(HSS_ERR_INVALID_ARG, who + "children must partition their parent (BFS numbering)");
    }
  }
}

// Device bytes one problem adds to a job (node pools, its share of the level
// workspaces, global samples, generator tables), from the same capacities
// setup() uses; the batched entry point groups problems by this estimate.
size_t Job::estimate_bytes(const hss_generator& g, const hss_tree* t, const hss_options& o, size_t* shared) {
  const int32_t nn = t->num_nodes;
  const int64_t dc = std::min<int64_t>(o.d_max, t->n);
  const bool sym = gen_symmetric(g);
  const int nsides = sym ? 1 : 2;
  std::vector<int64_t> mcap(nn), rcap(nn);
  int64_t dbl = 0, ints = 0;
  int32_t maxlev = 0;
  for (int32_t v = nn - 1; v >= 0; --v) {
    const int64_t size = t->hi[v] - t->lo[v];
    mcap[v] = t->left[v] < 0 ? size : std::min<int64_t>(size, rcap[t->left[v]] + rcap[t->right[v]]);
    rcap[v] = std::max<int64_t>(1, std::min<int64_t>(mcap[v], dc));
    maxlev = std::max(maxlev, t->level[v]);
  }
  std::vector<int64_t> wsa(maxlev + 1, 0), wsb(maxlev + 1, 0);
  for (int32_t v = 0; v < nn; ++v) {
    const int64_t qcap = o.strategy == HSS_DBL_HMT ? 0 : rcap[v];
    if (t->parent[v] >= 0)
      dbl += nsides * (align8(mcap[v] * dc) + align8(rcap[v] * dc) + align8(mcap[v] * qcap) + align8(rcap[v] * mcap[v]));
    ints += nsides * (align8(mcap[v]) + 2 * align8(rcap[v]));
    if (t->left[v] < 0) dbl += align8((t->hi[v] - t->lo[v]) * (t->hi[v] - t->lo[v]));
    else dbl += 2 * align8(rcap[t->left[v]] * rcap[t->right[v]]);
    wsa[t->level[v]] += align8(mcap[v] * dc);
    wsb[t->level[v]] += align8(std::max<int64_t>(qcap * dc, 16 + 2 * (mcap[v] + dc)));
    dbl += 2 * mcap[v] + 2 * rcap[v];   // matvec slots
  }
  dbl += nsides * align8(t->n * dc) + 8 * t->n;
  if (!o.R) dbl += align8(t->n * dc);   // R drawn by the library
  dbl += *std::max_element(wsa.begin(), wsa.end()) + *std::max_element(wsb.begin(), wsb.end());
  // one split-K partial buffer and one GEMM split workspace serve the whole
  // job (sized for its largest problem)
  *shared = 8 * (sample_partial_elems(t->n, (int32_t)dc) + (size_t)kGemmSplitElems);
  {
    // block-ID slots of the largest level
    std::vector<int64_t> ld(maxlev + 1, 0), li(maxlev + 1, 0);
    for (int32_t v = 0; v < nn; ++v) {
      ld[t->level[v]] += idblk_doubles(dc, mcap[v]);
      li[t->level[v]] += idblk_ints(mcap[v]);
    }
    dbl += *std::max_element(ld.begin(), ld.end()) + *std::max_element(li.begin(), li.end()) / 2 + 1;
  }
  return (size_t)(8 * dbl + 4 * ints + 64 * nn + (16 << 20));
}

void Job::setup(int32_t count, const hss_generator* gens, const hss_tree* const* trees,
                const hss_options* opts) {
  if (count < 1) throw Error(HSS_ERR_INVALID_ARG, "count must be >= 1");
  strategy = opts[0].strategy;
  stream = (hipStream_t)opts[0].stream;
  ualloc = opts[0].allocator;
  for (int k = 0; k < count; ++k) {
    validate(gens[k], trees[k], opts[k], k);
    if (opts[k].strategy != strategy || opts[k].stream != opts[0].stream)
      throw Error(HSS_ERR_INVALID_ARG, "batched problems must share strategy and stream");
  }
  HSS_HIP_CHECK(hipEventCreate(&ev0));
  HSS_HIP_CHECK(hipEventCreate(&ev1));
  HSS_HIP_CHECK(hipEventCreateWithFlags(&ev_flag, hipEventDisableTiming));
  HSS_HIP_CHECK(hipHostMalloc((void**)&hflags, 64, 0));
  HSS_HIP_CHECK(hipEventCreate(&prof.e0));
  HSS_HIP_CHECK(hipEventCreate(&prof.e1));
  prof.on = false;
  for (int k = 0; k < count; ++k) prof.on = prof.on || opts[k].profile != 0;
  probs.resize(count);
  int64_t dtot = 0, ttot = 0, itot = 0, ltot = 0;
  int32_t gnodes = 0;
  maxlevel = 0;
  for (int k = 0; k < count; ++k) {
    Problem& P = probs[k];
    const hss_tree* t = trees[k];
    P.gen = gens[k];
    P.opt = opts[k];
    P.n = t->n;
    P.nn = t->num_nodes;
    P.sym = gen_symmetric(gens[k]) ? 1 : 0;
    P.dcap = (int32_t)std::min<int64_t>(opts[k].d_max, t->n);
    P.node0 = gnodes;
    P.perm.assign(t->perm, t->perm + t->n);
    gnodes += P.nn;
    for (int32_t v = 0; v < P.nn; ++v) maxlevel = std::max(maxlevel, t->level[v]);
  }
  desc.resize(gnodes);
  // capacities bottom-up, then pool offsets
  for (int k = 0; k < count; ++k) {
    Problem& P = probs[k];
    const hss_tree* t = trees[k];
    const int64_t dc = P.dcap;
    for (int32_t v = P.nn - 1; v >= 0; --v) {
      NodeDesc& d = desc[P.node0 + v];
      std::memset(&d, 0, sizeof(d));
      d.prob = k;
      d.level = t->level[v];
      d.leaf = t->left[v] < 0;
      d.parent = t->parent[v] < 0 ? -1 : P.node0 + t->parent[v];
      d.left = t->left[v] < 0 ? -1 : P.node0 + t->left[v];
      d.right = t->right[v] < 0 ? -1 : P.node0 + t->right[v];
      d.lo = t->lo[v];
      d.hi = t->hi[v];
      const int32_t size = d.hi - d.lo;
      if (d.leaf) d.mcap = size;
      else d.mcap = std::min<int32_t>(size, desc[d.left].rcap + desc[d.right].rcap);
      d.rcap = (int32_t)std::min<int64_t>(d.mcap, dc);
      d.qcap = strategy == HSS_DBL_HMT ? 0 : d.rcap;
      d.rcap = std::max(d.rcap, 1);
    }
    for (int32_t v = 0; v < P.nn; ++v) {
      NodeDesc& d = desc[P.node0 + v];
      const bool root = d.parent < 0;
      const int nsides = P.sym ? 1 : 2;
      for (int s = 0; s < nsides; ++s) {
        if (!root) {
          d.S[s] = ttot; ttot += align8((int64_t)d.mcap * dc);
          d.RR[s] = ttot; ttot += align8((int64_t)d.rcap * dc);
          d.Q[s] = ttot; ttot += align8((int64_t)d.mcap * d.qcap);
          d.E[s] = ttot; ttot += align8((int64_t)d.rcap * d.mcap);
          d.eld[s] = d.rcap;
          d.J[s] = itot; itot += align8(d.mcap);
          d.I[s] = ltot; ltot += align8(d.rcap);
        }
      }
      if (P.sym) {
        d.S[1] = d.S[0]; d.RR[1] = d.RR[0]; d.Q[1] = d.Q[0]; d.E[1] = d.E[0]; d.eld[1] = d.eld[0];
        d.J[1] = d.J[0]; d.I[1] = d.I[0];
      }
      if (d.leaf) { d.D = dtot; dtot += align8((int64_t)(d.hi - d.lo) * (d.hi - d.lo)); }
      else {
        d.B12 = ttot; ttot += align8((int64_t)desc[d.left].rcap * desc[d.right].rcap);
        d.B21 = ttot; ttot += align8((int64_t)desc[d.right].rcap * desc[d.left].rcap);
        d.b12ld = desc[d.left].rcap;
        d.b21ld = desc[d.right].rcap;
      }
    }
    for (int s = 0; s < (P.sym ? 1 : 2); ++s) {
      P.sglob[s] = ttot;
      ttot += align8(P.n * dc);
    }
    if (P.sym) P.sglob[1] = P.sglob[0];
    if (!P.opt.R) {   // the library draws R: n x dcap, column-major
      P.rglob = ttot;
      ttot += align8(P.n * dc);
    }
  }
  // levels and workspaces
  levels.assign(maxlevel + 1, LevelInfo());
  for (int32_t g = 0; g < gnodes; ++g) levels[desc[g].level].nodes.push_back(g);
  int64_t wsA = 0, wsB = 0;
  int32_t maxcount = 0;
  for (auto& L : levels) {
    int64_t a = 0, b = 0;
    for (int32_t g : L.nodes) {
      NodeDesc& d = desc[g];
      const int64_t dc = probs[d.prob].dcap;
      d.ws = a;
      a += align8((int64_t)d.mcap * dc);
      d.wsq = b;
      b += align8(std::max<int64_t>((int64_t)d.qcap * dc, 16 + 2 * ((int64_t)d.mcap + dc)));
      L.mcap = std::max(L.mcap, d.mcap);
      L.rcap = std::max(L.rcap, d.rcap);
      L.qcap = std::max(L.qcap, d.qcap);
      L.dcap = std::max<int32_t>(L.dcap, probs[d.prob].dcap);
    }
    wsA = std::max(wsA, a);
    wsB = std::max(wsB, b);
    maxcount = std::max<int32_t>(maxcount, (int32_t)L.nodes.size());
  }
  size_t part = 0;
  for (auto& P : probs) part = std::max(part, sample_partial_elems(P.n, P.dcap));
  // block-pivoted ID workspace: one slot per node of a level, sized from its
  // capacities; the levels take turns, so the largest level's total is kept
  int64_t idb_d = 0, idb_i = 0;
  for (auto& L : levels) {
    int64_t dsum = 0, isum = 0;
    for (int32_t g : L.nodes) {
      dsum += idblk_doubles(probs[desc[g].prob].dcap, desc[g].mcap);
      isum += idblk_ints(desc[g].mcap);
    }
    idb_d = std::max(idb_d, dsum);
    idb_i = std::max(idb_i, isum);
  }
  dpool = (double*)dalloc(sizeof(double) * std::max<int64_t>(dtot, 1));
  ipool = (int32_t*)dalloc(sizeof(int32_t) * std::max<int64_t>(itot, 1));
  lpool = (int64_t*)dalloc(sizeof(int64_t) * std::max<int64_t>(ltot, 1));
  {
    // tpool | wsA | wsB | split-K partials, each 256-byte aligned
    auto a256 = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t bt = a256(sizeof(double) * std::max<int64_t>(ttot, 1));
    const size_t ba = a256(sizeof(double) * std::max<int64_t>(wsA, 1));
    const size_t bb = a256(sizeof(double) * std::max<int64_t>(wsB, 1));
    const size_t bp = a256(sizeof(double) * part);
    const size_t bg = a256(sizeof(double) * kGemmSplitElems);
    const size_t bd = a256(sizeof(double) * std::max<int64_t>(idb_d, 1));
    const size_t bi = a256(sizeof(int32_t) * std::max<int64_t>(idb_i, 1));
    char* base = (char*)arena_acquire(bt + ba + bb + bp + bg + bd + bi);
    tpool = (double*)base;
    wsa = (double*)(base + bt);
    wsb = (double*)(base + bt + ba);
    partial = part ? (double*)(base + bt + ba + bb) : nullptr;
    gemm_ws = (double*)(base + bt + ba + bb + bp);
    idb_dpool = (double*)(base + bt + ba + bb + bp + bg);
    idb_ipool = (int32_t*)(base + bt + ba + bb + bp + bg + bd);
  }
  desc_d = (NodeDesc*)dalloc(sizeof(NodeDesc) * gnodes);
  st_d = (NodeState*)dalloc(sizeof(NodeState) * gnodes);
  prob_d = (ProbDev*)dalloc(sizeof(ProbDev) * count);
  tasks_d = (GemmTask*)dalloc(sizeof(GemmTask) * 2 * std::max(maxcount, 1));
  qtasks_d = (QrcpTask*)dalloc(sizeof(QrcpTask) * std::max(maxcount, 1));
  qwork.max_tasks = std::max(maxcount, 1);
  qwork.chunks = (int2*)dalloc(sizeof(int2) * qrcp_work_entries(qwork.max_tasks));
  qwork.meta = (int32_t*)dalloc(sizeof(int32_t) * 2);
  qwork.kbuf = (int32_t*)dalloc(sizeof(int32_t) * 2);
  qwork.graphs = &qgraphs;
  qform_d = (QformTask*)dalloc(sizeof(QformTask) * std::max(maxcount, 1));
  chol_d = (CholTask*)dalloc(sizeof(CholTask) * std::max(maxcount, 1));
  mvtasks_d = (GemmTask*)dalloc(sizeof(GemmTask) * 2 * std::max(maxcount, 1));
  idb_gt = (GemmTask*)dalloc(sizeof(GemmTask) * 3 * std::max(maxcount, 1));
  for (auto& L : levels) {
    // block-ID slots of this level's nodes (task t of an ID call = node t)
    std::vector<IdBlk> hb(L.nodes.size());
    int64_t doff = 0, ioff = 0;
    for (size_t t = 0; t < L.nodes.size(); ++t) {
      const NodeDesc& d = desc[L.nodes[t]];
      const int64_t dc = probs[d.prob].dcap, mc = d.mcap;
      const auto a8 = [](int64_t x) { return (x + 7) & ~int64_t(7); };
      IdBlk& B = hb[t];
      std::memset(&B, 0, sizeof(B));
      double* dp = idb_dpool + doff;
      B.C = dp; dp += a8(dc * kIdbCmax);
      B.G = dp; dp += a8((int64_t)kIdbCmax * kIdbCmax);
      B.V = dp; dp += a8(dc * kIdbLmax);
      B.U = dp; dp += a8(dc * kIdbLmax);
      B.Y = dp; dp += a8(kIdbLmax * mc);
      B.F = dp; dp += a8(4 * (int64_t)kIdbLmax * kIdbLmax);
      B.P = dp;
      B.ldc = dc;
      B.ldv = dc;
      B.cmax = kIdbCmax;
      B.cand = idb_ipool + ioff;
      B.piv = B.cand + kIdbCmax;
      B.rest = B.piv + kIdbLmax;
      doff += idblk_doubles(dc, mc);
      ioff += idblk_ints(mc);
    }
    L.idb.blk = (IdBlk*)dalloc(sizeof(IdBlk) * std::max<size_t>(hb.size(), 1));
    HSS_HIP_CHECK(hipMemcpy(L.idb.blk, hb.data(), sizeof(IdBlk) * hb.size(), hipMemcpyHostToDevice));
    L.idb.gt = idb_gt;
    L.idb.max_tasks = (int32_t)L.nodes.size();
  }
  for (auto& L : levels) {
    std::vector<int32_t> mc;
    for (int32_t g : L.nodes) mc.push_back(desc[g].mcap);
    QrcpPlan qp = make_qrcp_plan(mc);
    L.ntrsm = (int32_t)qp.trsm.size();
    L.wg_trsm = (int2*)dalloc(sizeof(int2) * std::max<size_t>(qp.trsm.size(), 1));
    HSS_HIP_CHECK(hipMemcpy(L.wg_trsm, qp.trsm.data(), sizeof(int2) * qp.trsm.size(), hipMemcpyHostToDevice));
  }
  flags_d = (int32_t*)dalloc(sizeof(int32_t) * 8);
  kcnt_d = (unsigned long long*)dalloc(sizeof(unsigned long long) * 2 * HSS_K_COUNT);
  HSS_HIP_CHECK(hipMemset(kcnt_d, 0, sizeof(unsigned long long) * 2 * HSS_K_COUNT));
  nodes_d = (int32_t*)dalloc(sizeof(int32_t) * gnodes);
  {
    std::vector<int64_t> mo(gnodes);
    int64_t acc = 0;
    for (int32_t g = 0; g < gnodes; ++g) { mo[g] = acc; acc += desc[g].rcap; }
    mvtot = acc;
    mvoff_d = (int64_t*)dalloc(sizeof(int64_t) * gnodes);
    HSS_HIP_CHECK(hipMemcpy(mvoff_d, mo.data(), sizeof(int64_t) * gnodes, hipMemcpyHostToDevice));
    acc = 0;
    for (int32_t g = 0; g < gnodes; ++g) { mo[g] = acc; acc += desc[g].mcap; }
    mvwstot = acc;
    mvws_d = (int64_t*)dalloc(sizeof(int64_t) * gnodes);
    HSS_HIP_CHECK(hipMemcpy(mvws_d, mo.data(), sizeof(int64_t) * gnodes, hipMemcpyHostToDevice));
  }
  int32_t off = 0;
  std::vector<int32_t> all;
  for (auto& L : levels) {
    L.off = off;
    off += (int32_t)L.nodes.size();
    all.insert(all.end(), L.nodes.begin(), L.nodes.end());
  }
  HSS_HIP_CHECK(hipMemcpy(nodes_d, all.data(), sizeof(int32_t) * all.size(), hipMemcpyHostToDevice));
  HSS_HIP_CHECK(hipMemcpy(desc_d, desc.data(), sizeof(NodeDesc) * gnodes, hipMemcpyHostToDevice));
  HSS_HIP_CHECK(hipMemsetAsync(st_d, 0, sizeof(NodeState) * gnodes, stream));
  HSS_HIP_CHECK(hipMemsetAsync(flags_d, 0, sizeof(int32_t) * 8, stream));
  // per-problem generator data
  for (auto& P : probs) {
    GenDev& g = P.dev.gen;
    std::memset(&g, 0, sizeof(g));
    g.family = P.gen.family;
    g.symmetric = P.sym;
    g.n = P.n;
    g.diag = P.gen.diag;
    g.inv2s2 = P.gen.family == HSS_FAM_GAUSS ? 1.0 / (2.0 * P.gen.sigma * P.gen.sigma) : 0.0;
    int64_t* perm = (int64_t*)dalloc(sizeof(int64_t) * P.n);
    HSS_HIP_CHECK(hipMemcpy(perm, P.perm.data(), sizeof(int64_t) * P.n, hipMemcpyHostToDevice));
    g.perm = perm;
    if (P.gen.family == HSS_FAM_TOEPLITZ) {
      double* t = (double*)dalloc(sizeof(double) * P.n);
      launch_toeplitz_table(t, P.n, P.gen.h, stream);
      g.tcol = t;
      g.perm_id = 1;   // index bisection keeps the order: entries from the sampling window
      for (int64_t i = 0; i < P.n; ++i)
        if (P.perm[i] != i) {
          g.perm_id = 0;
          break;
        }
    }
    if (P.gen.family == HSS_FAM_LAPLACE || P.gen.family == HSS_FAM_GAUSS) {
      double* pts = (double*)dalloc(sizeof(double) * 3 * P.n);
      launch_permute_points(P.gen.points, perm, P.n, pts, stream);
      g.pts = pts;
    }
    if (P.gen.family == HSS_FAM_DENSE) {
      g.dense = P.gen.dense;
      g.ld = P.gen.ld;
    }
    if (P.gen.family == HSS_FAM_CALLBACK) {
      // permuted positions 0..n-1: the row and column lists of the leaves'
      // diagonal blocks handed to the extraction routine
      std::vector<int64_t> pos(P.n);
      for (int64_t i = 0; i < P.n; ++i) pos[i] = i;
      P.pos_d = (int64_t*)dalloc(sizeof(int64_t) * P.n);
      HSS_HIP_CHECK(hipMemcpy(P.pos_d, pos.data(), sizeof(int64_t) * P.n, hipMemcpyHostToDevice));
      has_callback = true;
    }
    if (P.opt.sample_precision != HSS_SAMPLE_FP64) {
      // reduced-precision sampling skips the leaf diagonal blocks
      std::vector<int32_t> llo(P.n), lhi(P.n);
      const hss_tree* t = trees[&P - probs.data()];
      for (int32_t v = 0; v < P.nn; ++v)
        if (t->left[v] < 0)
          for (int32_t i = t->lo[v]; i < t->hi[v]; ++i) { llo[i] = t->lo[v]; lhi[i] = t->hi[v]; }
      int32_t* dlo = (int32_t*)dalloc(sizeof(int32_t) * P.n);
      int32_t* dhi = (int32_t*)dalloc(sizeof(int32_t) * P.n);
      HSS_HIP_CHECK(hipMemcpy(dlo, llo.data(), sizeof(int32_t) * P.n, hipMemcpyHostToDevice));
      HSS_HIP_CHECK(hipMemcpy(dhi, lhi.data(), sizeof(int32_t) * P.n, hipMemcpyHostToDevice));
      g.leaf_lo = dlo;
      g.leaf_hi = dhi;
      g.offdiag = 1;
    }
    ProbDev& pd = P.dev;
    pd.dcap = P.dcap;
    pd.strategy = strategy;
    pd.p = P.opt.oversample_p;
    pd.symmetric = P.sym;
    pd.n = P.n;
    pd.eps_r = strategy == HSS_INC_HMT ? 0.0 : P.opt.eta * P.opt.rtol;   // HMT-lemma test: absolute only
    pd.eps_a = P.opt.eta * P.opt.atol;
    pd.hmt_alpha = P.opt.hmt_alpha > 0.0 ? P.opt.hmt_alpha : 10.0;
    // precision floor of the relative thresholds for reduced-precision samples
    pd.eps_floor = P.opt.sample_precision == HSS_SAMPLE_FP32 ? kFloorFp32
                 : P.opt.sample_precision == HSS_SAMPLE_BF16X3 ? kFloorBf16x3 : 0.0;
    {
      int32_t maxlev = 1;
      const hss_tree* t = trees[&P - probs.data()];
      for (int32_t v = 0; v < P.nn; ++v) maxlev = std::max(maxlev, t->level[v]);
      if (pd.eps_floor > 0.0 && pd.eps_r / maxlev < pd.eps_floor) P.status = HSS_TOL_BELOW_SAMPLING_PRECISION;
    }
    pd.sglob[0] = P.sglob[0];
    pd.sglob[1] = P.sglob[1];
    pd.R = P.rglob >= 0 ? tpool + P.rglob : P.opt.R;
    pd.ldr = P.rglob >= 0 ? P.n : P.opt.ldr;
  }
  // sampling schedules of all problems in one device array (one copy per
  // round from a pinned staging array)
  sched_stride = 2;
  for (const Problem& P : probs) sched_stride = std::max(sched_stride, (int64_t)P.dcap + 2);
  sched_all_d = (int32_t*)dalloc(sizeof(int32_t) * sched_stride * probs.size());
  HSS_HIP_CHECK(hipHostMalloc((void**)&sched_h, sizeof(int32_t) * sched_stride * probs.size(), 0));
  for (size_t k = 0; k < probs.size(); ++k) {
    probs[k].sched_d = sched_all_d + sched_stride * (int64_t)k;
    probs[k].dev.sched = probs[k].sched_d;
  }
  HSS_HIP_CHECK(hipGetLastError());
}

// Sampling step of a round: all problems' new columns, asynchronously; the
// HIP events bracket the whole step (one host wait per round).
void Job::sample_begin() { HSS_HIP_CHECK(hipEventRecord(ev0, stream)); }

void Job::sample_end() {
  HSS_HIP_CHECK(hipEventRecord(ev1, stream));
  HSS_HIP_CHECK(hipGetLastError());
  HSS_HIP_CHECK(hipEventSynchronize(ev1));
  float ms = 0.f;
  HSS_HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
  sample_ms += ms;
}

void Job::sample(Problem& P, int32_t c0, int32_t ncols) {
  if (ncols <= 0) return;
  double* Rc = const_cast<double*>(P.dev.R) + (int64_t)c0 * P.dev.ldr;   // the new columns of R
  if (P.rglob >= 0) {   // drawn here, only the new columns (Alg. 3)
    prof_begin(stream);
    launch_randn(Rc, P.dev.ldr, P.n, c0, ncols, P.opt.seed, stream);
    prof_end(HSS_K_RNG, stream);
    host_bytes[HSS_K_RNG] += 8.0 * (double)P.n * ncols;
  }
  if (P.gen.family == HSS_FAM_CALLBACK) {
    double* S0 = tpool + P.sglob[0] + (int64_t)c0 * P.n;
    double* S1 = P.sym ? nullptr : tpool + P.sglob[1] + (int64_t)c0 * P.n;
    const int32_t rc = P.gen.sample(P.gen.ctx, P.n, ncols, Rc, P.dev.ldr, S0, S1, P.n, stream);
    if (rc != 0) throw Error(HSS_ERR_CALLBACK, "sample routine returned " + std::to_string(rc));
    launch_check_finite(S0, P.n, ncols, P.n, flags_d, stream);
    if (S1) launch_check_finite(S1, P.n, ncols, P.n, flags_d, stream);
    require_finite("the sample routine");
    sample_flops += 2.0 * (double)P.n * (double)P.n * ncols * (P.sym ? 1 : 2);
    return;
  }
  const int prec = P.opt.sample_precision;
  for (int s = 0; s < (P.sym ? 1 : 2); ++s) {
    launch_sample(P.dev.gen, s, prec, Rc, P.dev.ldr,
                  tpool + P.sglob[s] + (int64_t)c0 * P.n, P.n, ncols, partial, stream, kcnt_d);
    host_flops[HSS_K_SAMPLE] += 2.0 * (double)P.n * (double)P.n * ncols;
    host_bytes[HSS_K_SAMPLE] += 16.0 * (double)P.n * ncols + 24.0 * (double)P.n;
  }
  sample_flops += 2.0 * (double)P.n * (double)P.n * ncols * (P.sym ? 1 : 2);
}

// The sub-blocks of A that the nodes of one level need this round (leaf
// diagonal blocks, couplings of nodes whose children just compressed), for
// the problems with caller routines: one extraction call per problem and
// level with all of its blocks.  Block sizes are ranks, decided on the
// device, so the node states come to the host first.
void Job::extract_callbacks(int lev) {
  const LevelInfo& L = levels[lev];
  st_h.resize(desc.size());
  HSS_HIP_CHECK(hipMemcpyAsync(st_h.data(), st_d, sizeof(NodeState) * desc.size(), hipMemcpyDeviceToHost, stream));
  HSS_HIP_CHECK(hipStreamSynchronize(stream));
  std::vector<std::vector<hss_block>> blocks(probs.size());
  for (int32_t g : L.nodes) {
    const NodeDesc& nd = desc[g];
    const Problem& P = probs[nd.prob];
    if (P.gen.family != HSS_FAM_CALLBACK || !st_h[g].extract) continue;
    std::vector<hss_block>& B = blocks[nd.prob];
    if (nd.leaf) {
      const int32_t m = nd.hi - nd.lo;
      B.push_back(hss_block{m, m, P.pos_d + nd.lo, P.pos_d + nd.lo, dpool + nd.D, m});
    } else {
      const NodeDesc& L1 = desc[nd.left];
      const NodeDesc& L2 = desc[nd.right];
      const NodeState& s1 = st_h[nd.left];
      const NodeState& s2 = st_h[nd.right];
      // B12 = A(left.I^r, right.I^c), B21 = A(right.I^r, left.I^c)
      if (s1.rank[0] > 0 && s2.rank[1] > 0)
        B.push_back(hss_block{s1.rank[0], s2.rank[1], lpool + L1.I[0], lpool + L2.I[1], tpool + nd.B12,
                              (int64_t)nd.b12ld});
      if (s2.rank[0] > 0 && s1.rank[1] > 0)
        B.push_back(hss_block{s2.rank[0], s1.rank[1], lpool + L2.I[0], lpool + L1.I[1], tpool + nd.B21,
                              (int64_t)nd.b21ld});
    }
  }
  for (size_t k = 0; k < probs.size(); ++k) {
    const std::vector<hss_block>& B = blocks[k];
    if (B.empty()) continue;
    const hss_generator& G = probs[k].gen;
    const int32_t rc = G.extract(G.ctx, (int32_t)B.size(), B.data(), stream);
    if (rc != 0) throw Error(HSS_ERR_CALLBACK, "extract routine returned " + std::to_string(rc));
    for (const hss_block& b : B) {
      launch_check_finite(b.out, b.nI, b.nJ, b.ldo, flags_d, stream);
      host_bytes[HSS_K_EXTRACT] += 8.0 * (double)b.nI * b.nJ;
    }
    require_finite("the extract routine");
  }
}

// Caller data is checked before any kernel uses it: a non-finite value
// ends the call here.
void Job::require_finite(const char* who) {
  int32_t bad = 0;
  HSS_HIP_CHECK(hipGetLastError());
  HSS_HIP_CHECK(hipMemcpyAsync(&bad, flags_d, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HSS_HIP_CHECK(hipStreamSynchronize(stream));
  if (bad) throw Error(HSS_ERR_NONFINITE, std::string("non-finite value from ") + who);
}

void Job::run_level(int lev, int32_t ncap) {
  LevelInfo& L = levels[lev];
  LevelArgs a;
  a.desc = desc_d;
  a.st = st_d;
  a.prob = prob_d;
  a.nodes = nodes_d + L.off;
  a.count = (int32_t)L.nodes.size();
  a.dpool = dpool;
  a.tpool = tpool;
  a.ipool = ipool;
  a.lpool = lpool;
  a.wsA = wsa;
  a.wsB = wsb;
  a.tasks = tasks_d;
  a.flags = flags_d;
  a.kcnt = kcnt_d;
  a.gws = gemm_ws;
  const int nsides = all_sym ? 1 : 2;
  const int32_t nc = std::min(ncap, L.dcap);
  launch_plan(a, stream);   // flags_d[1], [5], [6] are zero here: set up so, reset by each level's finalize
  int32_t max_b = 1;
  for (const Problem& P : probs)
    if (!P.done) max_b = std::max(max_b, P.b);
  // The level's test block count, largest column count and largest row
  // count are read back while the extraction runs.  The capacities alone
  // would size the GEMMs of the local samples for all d columns and
  // capacity rows, though most nodes take only the newest block; launched
  // that large, their K dimension is not split.  The local samples wait for
  // the counts only where d is well above the newest block (a host round
  // trip costs more than it saves on small levels); the later launches of
  // the level use them in any case.
  HSS_HIP_CHECK(hipMemcpyAsync(hflags, flags_d + 1, 6 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HSS_HIP_CHECK(hipEventRecord(ev_flag, stream));
  if (has_callback) extract_callbacks(lev);
  launch_extract_nodes(a, stream);
  const bool wait_counts = nc > 2 * max_b;
  if (wait_counts) HSS_HIP_CHECK(hipEventSynchronize(ev_flag));
  const int32_t ls_nc = wait_counts ? std::max(1, std::min(nc, hflags[4])) : nc;
  const int32_t ls_m = wait_counts ? std::max(1, std::min(L.mcap, hflags[5])) : L.mcap;
  // local samples: T0 has M = left rows (at most ls_m), K = right rank or the leaf size
  for (int s = 0; s < nsides; ++s) launch_local_samples(a, s, ls_m, std::min(L.rcap, ls_m), ls_nc, stream);
  if (!wait_counts) HSS_HIP_CHECK(hipEventSynchronize(ev_flag));
  const int32_t nblk = hflags[0];
  const int32_t lv_m = std::max(1, std::min(L.mcap, hflags[5]));
  int32_t red_nc = nc;
  auto id_phase = [&](int hmt) {
    for (int s = 0; s < nsides; ++s) {
      launch_build_qrcp(a, s, hmt, qtasks_d, stream);
      // panels of P.d <= ncap rows and st.m <= lv_m columns
      run_qrcp(qtasks_d, a.count, qwork, L.wg_trsm, L.ntrsm, std::min(lv_m, ncap), ncap, lv_m, flags_d + 4,
               tasks_d, lv_m, stream, kcnt_d, true, gemm_ws, kBlockId ? &L.idb : nullptr);
    }
  };
  if (strategy == HSS_DBL_HMT) {
    id_phase(1);
    launch_decide_hmt(a, stream);
  } else {
    if (nblk > 0) {
      // widest block of any schedule; with a single block to test, every
      // node tests its problem's newest block (a node tested before) or
      // its only one (the first round), at most max_b wide
      const int32_t nb_all = std::min(max_block, L.dcap);
      const int32_t nb = nblk == 1 ? std::min(nb_all, max_b) : nb_all;
      constexpr int kTestCpw = 4;
      if (L.test_ncap != nb_all) {   // workgroup map: kTestCpw block columns per workgroup
        std::vector<int32_t> caps(L.nodes.size(), nb_all);
        QrcpPlan qp = make_qrcp_plan(caps, kTestCpw);
        if (L.wg_test == nullptr || (int32_t)qp.step.size() > L.ntest)
          L.wg_test = (int2*)dalloc(sizeof(int2) * qp.step.size());
        HSS_HIP_CHECK(hipMemcpy(L.wg_test, qp.step.data(), sizeof(int2) * qp.step.size(), hipMemcpyHostToDevice));
        L.ntest = (int32_t)qp.step.size();
        L.test_ncap = nb_all;
      }
      TestScratch ts{qtasks_d, qform_d, chol_d, L.wg_test, L.ntest, kTestCpw, flags_d + 3, tasks_d, qwork};
      // A replay's first iteration may test a schedule's first block (d0
      // wide); the later ones test the blocks sampled after it, at most the
      // widest of those, so their launches are sized for that
      int32_t later = 0;
      for (const Problem& P : probs)
        if (!P.done)
          for (size_t i = 1; i < P.sched.size(); ++i) later = std::max(later, P.sched[i] - P.sched[i - 1]);
      for (int it = 0; it < nblk; ++it) {
        const int32_t nb_it = (it > 0 && later > 0) ? std::min(nb, later) : nb;
        // The basis a tested block is projected against holds at most the
        // columns sampled before the block: d - b for a node tested before
        // (its newest block, iteration 0), sched[it - 1] for one replaying
        // its blocks; the projections are sized for that, not for the
        // basis capacity.
        int32_t qb = 1;
        for (const Problem& P : probs) {
          if (P.done) continue;
          if (it == 0) qb = std::max(qb, P.d - P.b);
          else if ((size_t)it <= P.sched.size()) qb = std::max(qb, P.sched[it - 1]);
        }
        const int32_t q_it = std::max(1, std::min(std::min(L.qcap, lv_m), qb));
        for (int s = 0; s < nsides; ++s)
          launch_fnorm_test(a, s, it, lv_m, q_it, nb_it, ts, stream, strategy == HSS_INC_HMT);
      }
    }
    // A node passes only through a test of this round (a side that passed
    // earlier passed with the other, and the node compressed then) or when
    // its problem is forced: without either no node can go, and the ID of
    // the level, with its host round trips, is skipped.  The decision
    // kernel reports a node that goes anyway (checked after the round).
    bool any_force = false;
    for (const Problem& P : probs) any_force = any_force || (P.force && !P.done);
    const bool skip_id = nblk == 0 && !any_force;
    launch_decide_fnorm(a, stream, skip_id ? flags_d + 2 : nullptr);
    if (!skip_id) id_phase(0);
    red_nc = skip_id ? std::min(nc, max_b) : nc;
  }
  // reduce (M = rank, K = rows - rank): a node compressed earlier takes its
  // problem's newest block, one compressed now all d columns
  for (int s = 0; s < nsides; ++s) launch_reduce(a, s, lv_m, std::min(L.rcap, lv_m), red_nc, stream);
  launch_finalize(a, stream);
  HSS_HIP_CHECK(hipGetLastError());
}

void Job::compress() {
  ProfScope scope(&prof);
  auto t0 = std::chrono::steady_clock::now();
  all_sym = true;
  for (auto& P : probs) all_sym = all_sym && P.sym;
  sample_begin();
  for (auto& P : probs) {
    P.d = std::min(P.opt.d0, P.dcap);
    P.b = P.d;
    P.force = 0;
    P.done = 0;
    P.rounds = 0;
    P.sched.push_back(P.d);
    sample(P, 0, P.d);
  }
  sample_end();
  std::vector<NodeState> roots(probs.size());
  std::vector<ProbDev> pdev(probs.size());
  int32_t flags[4];
  for (int round = 0;; ++round) {
    int32_t ncap = 0;
    max_block = 0;
    for (size_t k = 0; k < probs.size(); ++k) {
      Problem& P = probs[k];
      P.dev.d = P.d;
      P.dev.b = P.b;
      P.dev.force = P.force;
      P.dev.done = P.done;
      P.dev.nsched = (int32_t)P.sched.size();
      std::memcpy(sched_h + sched_stride * (int64_t)k, P.sched.data(), sizeof(int32_t) * P.sched.size());
      for (size_t i = 0; i < P.sched.size(); ++i)
        max_block = std::max(max_block, P.sched[i] - (i ? P.sched[i - 1] : 0));
      pdev[k] = P.dev;
      if (!P.done) {
        ncap = std::max(ncap, P.d);
        P.rounds++;
      }
    }
    HSS_HIP_CHECK(hipMemcpyAsync(sched_all_d, sched_h, sizeof(int32_t) * sched_stride * probs.size(),
                                 hipMemcpyHostToDevice, stream));
    HSS_HIP_CHECK(hipMemcpyAsync(prob_d, pdev.data(), sizeof(ProbDev) * pdev.size(), hipMemcpyHostToDevice, stream));
    for (int lev = maxlevel; lev >= 0; --lev) run_level(lev, ncap);
    for (size_t k = 0; k < probs.size(); ++k)
      HSS_HIP_CHECK(hipMemcpyAsync(&roots[k], st_d + probs[k].node0, sizeof(NodeState), hipMemcpyDeviceToHost, stream));
    HSS_HIP_CHECK(hipMemcpyAsync(flags, flags_d, sizeof(flags), hipMemcpyDeviceToHost, stream));
    HSS_HIP_CHECK(hipStreamSynchronize(stream));
    if (flags[0]) throw Error(HSS_ERR_NONFINITE, "non-finite matrix entry generated");
    if (flags[2]) throw Error(HSS_ERR_INTERNAL, "a node passed in a level whose factorization was skipped");
    bool all_done = true;
    sample_begin();
    for (size_t k = 0; k < probs.size(); ++k) {
      Problem& P = probs[k];
      if (P.done) continue;
      if (roots[k].state == COMPRESSED) {
        P.done = 1;
        continue;
      }
      all_done = false;
      if (P.force) throw Error(HSS_ERR_INTERNAL, "forced round left the root open");
      if (P.d >= P.dcap) {
        P.force = 1;
        P.b = 0;
        if (P.status == HSS_OK) P.status = HSS_NOT_CONVERGED;
        continue;
      }
      int32_t b = (strategy == HSS_INC_FNORM || strategy == HSS_INC_HMT) ? P.opt.delta_d : P.d;
      b = std::min(b, P.dcap - P.d);
      sample(P, P.d, b);
      P.b = b;
      P.d += b;
      P.sched.push_back(P.d);
    }
    sample_end();
    if (all_done) break;
  }
  st_h.resize(desc.size());
  HSS_HIP_CHECK(hipMemcpyAsync(st_h.data(), st_d, sizeof(NodeState) * desc.size(), hipMemcpyDeviceToHost, stream));
  unsigned long long kc[2 * HSS_K_COUNT];
  HSS_HIP_CHECK(hipMemcpyAsync(kc, kcnt_d, sizeof(kc), hipMemcpyDeviceToHost, stream));
  HSS_HIP_CHECK(hipStreamSynchronize(stream));
  compact_e();
  release_transients();
  for (int c = 0; c < HSS_K_COUNT; ++c) {
    kstats[c].launches = prof.launches[c];
    kstats[c].ms = prof.ms[c];
    kstats[c].bytes = (double)kc[2 * c] + host_bytes[c];
    kstats[c].flops = (double)kc[2 * c + 1] + host_flops[c];
  }
  total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace hss
