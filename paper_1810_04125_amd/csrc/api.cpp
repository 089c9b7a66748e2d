// C ABI of libhss (declared in include/hss.h).  Every entry point catches
// all C++ exceptions, records a thread-local message and returns a status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "driver.h"

using namespace hss;

namespace {

thread_local std::string g_last_error;

hss_status fail(hss_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

template <class F>
hss_status guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(HSS_ERR_INTERNAL, e.what());
  } catch (...) {
    return fail(HSS_ERR_INTERNAL, "unknown error");
  }
}

// Device copies of the generator tables needed by the standalone kernels.
struct GenHolder {
  GenDev g;
  std::vector<void*> mem;
  ~GenHolder() {
    for (void* p : mem) hipFree(p);
  }
  void* alloc(size_t b) {
    void* p = nullptr;
    HSS_HIP_CHECK(hipMalloc(&p, std::max<size_t>(b, 8)));
    mem.push_back(p);
    return p;
  }
  GenHolder(const hss_generator& gen, const int64_t* perm, hipStream_t s) {
    if (!perm) throw Error(HSS_ERR_INVALID_ARG, "perm must be a device int64[n] array");
    if (gen.n < 1 || !(gen_formula(gen.family) || gen.family == HSS_FAM_DENSE))
      throw Error(HSS_ERR_INVALID_ARG, "bad generator");
    std::memset(&g, 0, sizeof(g));
    g.family = gen.family;
    g.n = gen.n;
    g.diag = gen.diag;
    g.perm = perm;
    g.symmetric = gen_symmetric(gen);
    if (gen.family == HSS_FAM_TOEPLITZ) {
      if (!(gen.h > 0.0)) throw Error(HSS_ERR_INVALID_ARG, "toeplitz needs h > 0");
      double* t = (double*)alloc(sizeof(double) * gen.n);
      launch_toeplitz_table(t, gen.n, gen.h, s);
      g.tcol = t;
      std::vector<int64_t> hp((size_t)gen.n);
      HSS_HIP_CHECK(hipMemcpyAsync(hp.data(), perm, sizeof(int64_t) * gen.n, hipMemcpyDeviceToHost, s));
      HSS_HIP_CHECK(hipStreamSynchronize(s));
      g.perm_id = 1;
      for (int64_t i = 0; i < gen.n; ++i)
        if (hp[i] != i) {
          g.perm_id = 0;
          break;
        }
    } else if (gen.family == HSS_FAM_DENSE) {
      if (!gen.dense || gen.ld < gen.n) throw Error(HSS_ERR_INVALID_ARG, "dense needs dense, ld >= n");
      g.dense = gen.dense;
      g.ld = gen.ld;
    } else {
      if (!gen.points) throw Error(HSS_ERR_INVALID_ARG, "kernel family needs points");
      if (gen.family == HSS_FAM_GAUSS) {
        if (!(gen.sigma > 0.0)) throw Error(HSS_ERR_INVALID_ARG, "gauss needs sigma > 0");
        g.inv2s2 = 1.0 / (2.0 * gen.sigma * gen.sigma);
      }
      double* pts = (double*)alloc(sizeof(double) * 3 * gen.n);
      launch_permute_points(gen.points, perm, gen.n, pts, s);
      g.pts = pts;
    }
  }
};

}  // namespace

hss_status hss::record_error(hss_status code, const std::string& msg) { return fail(code, msg); }

// Permuted-space matvec on the compressed job: Yp = H Xp, both n x nrhs (ld n).
void hss::matvec_permuted(const hss_matrix* h, int32_t nrhs, const double* Xp, double* Yp, double* xh,
                          double* yh, double* ws, hipStream_t s) {
  Job& J = *h->job;
  const Problem& P = J.probs[h->k];
  // The level lists mix problems; run per problem with its own sub-lists.
  for (int lev = J.maxlevel; lev >= 0; --lev) {
    MvArgs a;
    const LevelInfo& L = J.levels[lev];
    int32_t first = -1, cnt = 0;
    for (size_t i = 0; i < L.nodes.size(); ++i)
      if (J.desc[L.nodes[i]].prob == h->k) {
        if (first < 0) first = (int32_t)i;
        ++cnt;
      }
    if (cnt == 0) continue;
    a.desc = J.desc_d; a.st = J.st_d; a.nodes = J.nodes_d + L.off + first; a.count = cnt;
    a.dpool = J.dpool; a.epool = J.epool; a.ipool = J.ipool; a.xh = xh; a.yh = yh; a.xh_off = J.mvoff_d;
    a.X = Xp; a.Y = Yp; a.n = P.n; a.nrhs = nrhs; a.ws = ws; a.ws_off = J.mvws_d;
    launch_mv_up(a, J.mvtasks_d, J.levels[lev].mcap, s);
  }
  for (int lev = 0; lev <= J.maxlevel; ++lev) {
    MvArgs a;
    const LevelInfo& L = J.levels[lev];
    int32_t first = -1, cnt = 0;
    for (size_t i = 0; i < L.nodes.size(); ++i)
      if (J.desc[L.nodes[i]].prob == h->k) {
        if (first < 0) first = (int32_t)i;
        ++cnt;
      }
    if (cnt == 0) continue;
    a.desc = J.desc_d; a.st = J.st_d; a.nodes = J.nodes_d + L.off + first; a.count = cnt;
    a.dpool = J.dpool; a.epool = J.epool; a.ipool = J.ipool; a.xh = xh; a.yh = yh; a.xh_off = J.mvoff_d;
    a.X = Xp; a.Y = Yp; a.n = P.n; a.nrhs = nrhs; a.ws = ws; a.ws_off = J.mvws_d;
    launch_mv_down(a, J.mvtasks_d, J.levels[lev].mcap, s);
  }
  HSS_HIP_CHECK(hipGetLastError());
}

namespace {

struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t bytes) { HSS_HIP_CHECK(hipMalloc(&p, std::max<size_t>(bytes, 8))); }
  ~DevBuf() { if (p) hipFree(p); }
  template <class T> T* as() const { return (T*)p; }
};

// Stream-ordered scratch: allocated and freed in the order of `s`, so
// asynchronous calls may return while their kernels still use it; from the
// caller's allocator when one is given.
struct StreamBuf {
  void* p = nullptr;
  hipStream_t s;
  hss_allocator a{};
  StreamBuf(size_t bytes, hipStream_t st, const hss_allocator* ua = nullptr) : s(st) {
    if (ua && ua->alloc) {
      a = *ua;
      p = a.alloc(a.ctx, std::max<size_t>(bytes, 8), s);
      if (!p) throw Error(HSS_ERR_OUT_OF_MEMORY, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
      return;
    }
    hipError_t e = hipMallocAsync(&p, std::max<size_t>(bytes, 8), s);
    if (e != hipSuccess) {
      hipGetLastError();
      p = nullptr;
      throw Error(e == hipErrorOutOfMemory ? HSS_ERR_OUT_OF_MEMORY : HSS_ERR_DEVICE,
                  "hipMallocAsync of " + std::to_string(bytes) + " bytes failed");
    }
  }
  ~StreamBuf() {
    if (!p) return;
    if (a.alloc) {
      if (a.free) a.free(a.ctx, p, s);
    } else {
      hipFreeAsync(p, s);
    }
  }
  template <class T> T* as() const { return (T*)p; }
};

uint64_t splitmix64(uint64_t& x) {  // Steele, Lea and Flood (2014)
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// i -> (a i + c) mod n, a coprime to n: the sample order of one epoch
void epoch_order(uint64_t seed, int64_t epoch, int64_t n, int64_t& a, int64_t& c) {
  if (n <= 1) {
    a = 1;
    c = 0;
    return;
  }
  uint64_t x = seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(epoch + 1));
  a = 1 + (int64_t)(splitmix64(x) % (uint64_t)(n - 1));
  while (gcd64(a, n) != 1) a = a % (n - 1) + 1;
  c = (int64_t)(splitmix64(x) % (uint64_t)n);
}

MlpAdam adam_consts(float lr, float b1, float b2, float eps, int64_t step) {
  MlpAdam a;
  a.lr = lr;
  a.b1 = b1;
  a.b2 = b2;
  a.eps = eps;
  a.bc1 = (float)(1.0 - std::pow((double)b1, (double)step));
  a.bc2 = (float)(1.0 - std::pow((double)b2, (double)step));
  return a;
}

// The single-step entry points take device index arrays that select points
// and generated entries: they are copied back and checked on the host.
void check_device_perm(const int64_t* perm, int64_t n) {
  if (!perm) throw Error(HSS_ERR_INVALID_ARG, "perm must be a device int64[n] array");
  std::vector<int64_t> h((size_t)n);
  HSS_HIP_CHECK(hipMemcpy(h.data(), perm, sizeof(int64_t) * n, hipMemcpyDeviceToHost));
  std::vector<uint8_t> seen((size_t)n, 0);
  for (int64_t v : h) {
    if (v < 0 || v >= n || seen[(size_t)v]) throw Error(HSS_ERR_INVALID_ARG, "perm is not a permutation of [0, n)");
    seen[(size_t)v] = 1;
  }
}

void check_device_index(const int64_t* idx, int32_t cnt, int64_t n, const char* what) {
  if (cnt <= 0) return;
  std::vector<int64_t> h((size_t)cnt);
  HSS_HIP_CHECK(hipMemcpy(h.data(), idx, sizeof(int64_t) * cnt, hipMemcpyDeviceToHost));
  for (int64_t v : h)
    if (v < 0 || v >= n) throw Error(HSS_ERR_INVALID_ARG, std::string(what) + " holds an index outside [0, n)");
}

// Learned start (hss_predictor): the network's prediction of the final
// sample count from one feature row per tree level, turned into d0.
int32_t predict_d0(const hss_generator& g, const hss_tree* t, const hss_options& o, hipStream_t s,
                   double* dpred) {
  const hss_predictor& pr = *o.predictor;
  if (!pr.params) throw Error(HSS_ERR_INVALID_ARG, "predictor: params is NULL");
  const MlpShape S = mlp_shape(pr.net);
  if (pr.net.sizes[0] != 8 || pr.net.sizes[pr.net.n_layers] != 2)
    throw Error(HSS_ERR_INVALID_ARG, "predictor: the network must map 8 features to 2 outputs");
  int32_t L = 0;
  for (int32_t v = 0; v < t->num_nodes; ++v) L = std::max(L, t->level[v]);
  std::vector<double> sum(L + 1, 0.0), cnt(L + 1, 0.0);
  for (int32_t v = 0; v < t->num_nodes; ++v) {
    sum[t->level[v]] += (double)(t->hi[v] - t->lo[v]);
    cnt[t->level[v]] += 1.0;
  }
  const int fam = g.family == HSS_FAM_TOEPLITZ ? 0 : g.family == HSS_FAM_LAPLACE ? 1 : 2;
  const double param = g.family == HSS_FAM_TOEPLITZ ? g.h : g.family == HSS_FAM_GAUSS ? g.sigma : 0.0;
  std::vector<float> X((size_t)(L + 1) * 8, 0.0f), Y((size_t)(L + 1) * 2, 0.0f);
  for (int32_t l = 0; l <= L; ++l) {
    float* f = X.data() + 8 * l;
    f[fam] = 1.0f;
    f[3] = fam == 1 ? 0.0f : (float)(0.5 * std::log2(param));
    f[4] = (float)((std::log2((double)g.n) - 14.0) / 3.0);
    f[5] = (float)(l / 8.0);
    f[6] = (float)((std::log2(std::max(1.0, sum[l] / cnt[l])) - 10.0) / 4.0);
    f[7] = (float)((-std::log10(o.rtol) - 6.0) / 2.0);
  }
  DevBuf xd(sizeof(float) * X.size()), yd(sizeof(float) * Y.size());
  HSS_HIP_CHECK(hipMemcpyAsync(xd.p, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, s));
  launch_mlp_tile(S, pr.params, xd.as<float>(), nullptr, nullptr, 0, L + 1, 1, 0, L + 1, yd.as<float>(), nullptr,
                  nullptr, 0, s);
  HSS_HIP_CHECK(hipGetLastError());
  HSS_HIP_CHECK(hipMemcpyAsync(Y.data(), yd.p, sizeof(float) * Y.size(), hipMemcpyDeviceToHost, s));
  HSS_HIP_CHECK(hipStreamSynchronize(s));
  const double d = std::exp2((double)Y[1]);   // root row, output 1: log2 of the final sample count
  if (!std::isfinite(d)) throw Error(HSS_ERR_NONFINITE, "predictor output is not finite");
  *dpred = d;
  const int32_t dd = o.delta_d;
  const int64_t cap = std::min<int64_t>(o.d_max, g.n);
  const double q = std::floor(std::min(d, (double)cap) / dd + 0.5);   // the nearest multiple of delta_d
  int64_t d0 = std::max<int64_t>(dd, (int64_t)dd * (int64_t)q);
  return (int32_t)std::min<int64_t>(d0, cap);
}

void need(const void* p, const char* what) {
  if (!p) throw Error(HSS_ERR_INVALID_ARG, std::string(what) + " must not be NULL");
}

}  // namespace

extern "C" {

const char* hss_last_error(void) { return g_last_error.c_str(); }
const char* hss_version(void) { return "libhss 0.1 (gfx950)"; }

hss_status hss_tree_build(int64_t n, const double* points_host, int32_t leaf_size, int32_t method,
                          hss_tree** out) {
  return guarded([&]() -> hss_status {
    if (!out) throw Error(HSS_ERR_INVALID_ARG, "out is NULL");
    *out = tree_build(n, points_host, leaf_size, method);
    return HSS_OK;
  });
}

void hss_tree_free(hss_tree* tree) { tree_free(tree); }

hss_status hss_compress_batched(int32_t count, const hss_generator* gens, const hss_tree* const* trees,
                                const hss_options* opts, hss_matrix** out) {
  return guarded([&]() -> hss_status {
    if (count < 1 || !gens || !trees || !opts || !out) throw Error(HSS_ERR_INVALID_ARG, "NULL argument");
    for (int32_t k = 0; k < count; ++k) out[k] = nullptr;
    for (int32_t k = 0; k < count; ++k)
      if (!trees[k]) throw Error(HSS_ERR_INVALID_ARG, "NULL tree");
    // every argument is checked on the host before the first HIP call
    for (int32_t k = 0; k < count; ++k) Job::validate(gens[k], trees[k], opts[k], k);
    // learned starts: the predictor's d0 replaces options.d0, and its
    // predicted final count sizes the compression's sample capacity (the
    // transient buffers grow with d_max): twice the prediction, at least
    // four rounds past d0, at most the caller's d_max.  A run that reaches
    // that capacity before its root compresses is restarted from scratch
    // with the caller's d_max, starting from the capacity it reached.
    std::vector<hss_options> op(opts, opts + count);
    std::vector<double> dpred(count, 0.0);
    std::vector<int32_t> cap_dmax(count, 0);
    for (int32_t k = 0; k < count; ++k) {
      if (!op[k].predictor) continue;
      op[k].d0 = predict_d0(gens[k], trees[k], op[k], (hipStream_t)op[k].stream, &dpred[k]);
      const int64_t dd = op[k].delta_d;
      const int64_t want = std::max<int64_t>((int64_t)op[k].d0 + 4 * dd,
                                             dd * (int64_t)std::ceil(2.0 * dpred[k] / (double)dd));
      if (want < op[k].d_max) {
        cap_dmax[k] = op[k].d_max;   // the caller's, for a restart
        op[k].d_max = (int32_t)want;
      }
    }
    std::vector<std::unique_ptr<hss_matrix>> res(count);
    hss_status worst = HSS_OK;
    // Problems are taken in order into groups whose estimated device memory
    // fits the free HBM at the time the group starts (earlier groups keep only
    // their generators); every group is one level-batched job.
    auto run_groups = [&](const std::vector<int32_t>& idx) {
      std::vector<hss_generator> gv;
      std::vector<const hss_tree*> tv;
      std::vector<hss_options> ov;
      for (int32_t k : idx) {
        gv.push_back(gens[k]);
        tv.push_back(trees[k]);
        ov.push_back(op[k]);
      }
      const int32_t cnt = (int32_t)idx.size();
      int32_t g0 = 0;
      while (g0 < cnt) {
        size_t free_b = 0, total_b = 0;
        HSS_HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
        free_b += arena_idle_bytes();   // the cached transient block is reusable
        const size_t budget = std::min<size_t>((size_t)(0.6 * (double)free_b), (size_t)80 << 30);
        size_t acc = 0, shared = 0;
        int32_t g1 = g0;
        while (g1 < cnt) {
          size_t sh = 0;
          const size_t b = Job::estimate_bytes(gv[g1], tv[g1], ov[g1], &sh);
          if (g1 > g0 && acc + b + std::max(shared, sh) > budget) break;
          acc += b;
          shared = std::max(shared, sh);
          ++g1;
        }
        acc += shared;
        auto job = std::make_shared<Job>();
        // launch shapes from the tunables table (the group's first problem)
        const hss_tunables tu = tunables_for(gv[g0].family, ov[g0].sample_precision, gv[g0].n);
        TuneScope scope(tu);
        const auto t0 = std::chrono::steady_clock::now();
        job->setup(g1 - g0, gv.data() + g0, tv.data() + g0, ov.data() + g0);
        const auto t1 = std::chrono::steady_clock::now();
        job->compress();
        if (std::getenv("HSS_TRACE")) {
          const auto t2 = std::chrono::steady_clock::now();
          std::fprintf(stderr,
                       "[hss] group %d..%d: est %.1f GB (free %.1f GB), setup %.1f ms (alloc %.1f ms), compress "
                       "%.1f ms, sample %.1f ms\n",
                       g0, g1, acc / 1e9, free_b / 1e9, std::chrono::duration<double, std::milli>(t1 - t0).count(),
                       job->alloc_ms, std::chrono::duration<double, std::milli>(t2 - t1).count(), job->sample_ms);
        }
        for (int32_t q = g0; q < g1; ++q) {
          const int32_t k = idx[q];
          job->probs[q - g0].d_pred = dpred[k];
          res[k].reset(new hss_matrix);
          res[k]->job = job;
          res[k]->k = q - g0;
        }
        g0 = g1;
      }
    };
    std::vector<int32_t> all(count);
    for (int32_t k = 0; k < count; ++k) all[k] = k;
    run_groups(all);
    // hard restarts of the learned starts that outgrew their capacity
    std::vector<int32_t> again;
    for (int32_t k = 0; k < count; ++k) {
      // (force: d reached the capacity with the root open, whatever the status)
      if (!cap_dmax[k] || !res[k]->job->probs[res[k]->k].force) continue;
      op[k].d0 = op[k].d_max;
      op[k].d_max = cap_dmax[k];
      res[k].reset();
      again.push_back(k);
    }
    if (!again.empty()) run_groups(again);
    for (int32_t k = 0; k < count; ++k) {
      const hss_status st = res[k]->job->probs[res[k]->k].status;
      if (st > worst) worst = st;
    }
    for (int32_t k = 0; k < count; ++k) out[k] = res[k].release();
    if (worst == HSS_NOT_CONVERGED) g_last_error = "d reached d_max before the root compressed";
    return worst;
  });
}

hss_status hss_compress(const hss_generator* gen, const hss_tree* tree, const hss_options* opt,
                        hss_matrix** out) {
  if (!tree) return fail(HSS_ERR_INVALID_ARG, "tree is NULL");
  const hss_tree* trees[1] = {tree};
  return hss_compress_batched(1, gen, trees, opt, out);
}

void hss_destroy(hss_matrix* h) { delete h; }

hss_status hss_get_info(const hss_matrix* h, hss_info* out) {
  return guarded([&]() -> hss_status {
    if (!h || !out) throw Error(HSS_ERR_INVALID_ARG, "NULL argument");
    const Job& J = *h->job;
    const Problem& P = J.probs[h->k];
    std::memset(out, 0, sizeof(*out));
    out->n = P.n;
    out->num_nodes = P.nn;
    out->rounds = P.rounds;
    out->d_final = P.d;
    int32_t r = 0;
    for (int32_t v = 1; v < P.nn; ++v) {
      const NodeState& s = J.st_h[P.node0 + v];
      r = std::max(r, std::max(s.rank[0], s.rank[1]));
    }
    out->hss_rank = r;
    out->status = P.status;
    out->symmetric = P.sym;
    out->sample_ms = J.sample_ms;
    out->total_ms = J.total_ms;
    out->sample_flops = 2.0 * (double)P.n * (double)P.n * P.d * (P.sym ? 1 : 2);
    out->d0 = P.sched.empty() ? 0 : P.sched[0];
    out->d_predicted = P.d_pred;
    return HSS_OK;
  });
}

hss_status hss_get_kernel_stats(const hss_matrix* h, int32_t kclass, hss_kernel_stats* out) {
  return guarded([&]() -> hss_status {
    if (!h || !out) throw Error(HSS_ERR_INVALID_ARG, "NULL argument");
    if (kclass < 0 || kclass >= HSS_K_COUNT) throw Error(HSS_ERR_INVALID_ARG, "unknown kernel class");
    *out = h->job->kstats[kclass];
    return HSS_OK;
  });
}

hss_status hss_get_node_info(const hss_matrix* h, int32_t node, hss_node_info* out) {
  return guarded([&]() -> hss_status {
    if (!h || !out) throw Error(HSS_ERR_INVALID_ARG, "NULL argument");
    const Job& J = *h->job;
    const Problem& P = J.probs[h->k];
    if (node < 0 || node >= P.nn) throw Error(HSS_ERR_INVALID_ARG, "node out of range");
    const NodeDesc& d = J.desc[P.node0 + node];
    const NodeState& s = J.st_h[P.node0 + node];
    std::memset(out, 0, sizeof(*out));
    out->state = s.state;
    out->is_leaf = d.leaf;
    out->lo = d.lo;
    out->hi = d.hi;
    if (d.parent >= 0) {
      out->m_r = s.m[0];
      out->m_c = s.m[1];
      out->rank_r = s.rank[0];
      out->rank_c = s.rank[1];
    }
    if (!d.leaf) {
      out->b_rows = J.st_h[d.left].rank[0];
      out->b_cols = J.st_h[d.right].rank[1];
    }
    return HSS_OK;
  });
}

hss_status hss_copy_node(const hss_matrix* h, int32_t node, int32_t what, void* host_dst, size_t bytes) {
  return guarded([&]() -> hss_status {
    if (!h || !host_dst) throw Error(HSS_ERR_INVALID_ARG, "NULL argument");
    const Job& J = *h->job;
    const Problem& P = J.probs[h->k];
    if (node < 0 || node >= P.nn) throw Error(HSS_ERR_INVALID_ARG, "node out of range");
    const NodeDesc& d = J.desc[P.node0 + node];
    const NodeState& s = J.st_h[P.node0 + node];
    const bool root = d.parent < 0;
    auto need = [&](size_t b) {
      if (bytes < b) throw Error(HSS_ERR_INVALID_ARG, "destination too small");
    };
    // copy a (rows x cols) block with device leading dimension ld into a dense
    // column-major host array
    auto copy2d = [&](const double* src, int64_t ld, int32_t rows, int32_t cols) {
      need(sizeof(double) * (size_t)rows * cols);
      if (rows == 0 || cols == 0) return;
      HSS_HIP_CHECK(hipMemcpy2D(host_dst, sizeof(double) * rows, src, sizeof(double) * ld, sizeof(double) * rows,
                                cols, hipMemcpyDeviceToHost));
    };
    switch (what) {
      case HSS_NODE_D: {
        if (!d.leaf) throw Error(HSS_ERR_INVALID_ARG, "D exists on leaves only");
        const int32_t m = d.hi - d.lo;
        copy2d(J.dpool + d.D, m, m, m);
        break;
      }
      case HSS_NODE_B12:
      case HSS_NODE_B21: {
        if (d.leaf) throw Error(HSS_ERR_INVALID_ARG, "B exists on non-leaves only");
        const NodeDesc& L = J.desc[d.left];
        const NodeDesc& R = J.desc[d.right];
        const NodeState& sl = J.st_h[d.left];
        const NodeState& sr = J.st_h[d.right];
        if (what == HSS_NODE_B12) copy2d(J.epool + d.B12, d.b12ld, sl.rank[0], sr.rank[1]);
        else copy2d(J.epool + d.B21, d.b21ld, sr.rank[0], sl.rank[1]);
        break;
      }
      case HSS_NODE_JR:
      case HSS_NODE_JC: {
        if (root) throw Error(HSS_ERR_INVALID_ARG, "the root has no basis");
        const int side = what == HSS_NODE_JC;
        need(sizeof(int32_t) * s.m[side]);
        if (s.m[side])
          HSS_HIP_CHECK(hipMemcpy(host_dst, J.ipool + d.J[side], sizeof(int32_t) * s.m[side], hipMemcpyDeviceToHost));
        break;
      }
      case HSS_NODE_ER:
      case HSS_NODE_EC: {
        if (root) throw Error(HSS_ERR_INVALID_ARG, "the root has no basis");
        const int side = what == HSS_NODE_EC;
        copy2d(J.epool + d.E[side], d.eld[side], s.rank[side], s.m[side] - s.rank[side]);
        break;
      }
      case HSS_NODE_IR:
      case HSS_NODE_IC: {
        if (root) throw Error(HSS_ERR_INVALID_ARG, "the root has no basis");
        const int side = what == HSS_NODE_IC;
        need(sizeof(int64_t) * s.rank[side]);
        if (s.rank[side])
          HSS_HIP_CHECK(hipMemcpy(host_dst, J.lpool + d.I[side], sizeof(int64_t) * s.rank[side], hipMemcpyDeviceToHost));
        break;
      }
      default:
        throw Error(HSS_ERR_INVALID_ARG, "unknown node object");
    }
    return HSS_OK;
  });
}

hss_status hss_matvec(const hss_matrix* h, int32_t nrhs, const double* X, int64_t ldx, double* Y, int64_t ldy,
                      void* stream) {
  return guarded([&]() -> hss_status {
    if (!h || !X || !Y || nrhs < 1) throw Error(HSS_ERR_INVALID_ARG, "bad arguments");
    const Job& J = *h->job;
    const Problem& P = J.probs[h->k];
    if (ldx < P.n || ldy < P.n) throw Error(HSS_ERR_INVALID_ARG, "leading dimension < n");
    hipStream_t s = (hipStream_t)stream;
    // stream-ordered temporaries: freed behind the kernels on `s`, so the
    // call returns without waiting for them
    const hss_allocator* ua = &J.ualloc;
    StreamBuf xp(sizeof(double) * P.n * nrhs, s, ua), yp(sizeof(double) * P.n * nrhs, s, ua);
    StreamBuf xh(sizeof(double) * J.mvtot * nrhs, s, ua), yh(sizeof(double) * J.mvtot * nrhs, s, ua);
    StreamBuf ws(sizeof(double) * J.mvwstot * nrhs, s, ua);
    const int64_t* perm = P.dev.gen.perm;
    launch_gather_rows(X, ldx, perm, P.n, nrhs, xp.as<double>(), P.n, 0, s);
    matvec_permuted(h, nrhs, xp.as<double>(), yp.as<double>(), xh.as<double>(), yh.as<double>(), ws.as<double>(), s);
    launch_gather_rows(yp.as<double>(), P.n, perm, P.n, nrhs, Y, ldy, 1, s);
    HSS_HIP_CHECK(hipGetLastError());
    return HSS_OK;
  });
}

hss_status hss_factor(hss_matrix* h) {
  return guarded([&]() -> hss_status {
    if (!h) throw Error(HSS_ERR_INVALID_ARG, "NULL matrix");
    ulv_factor(h);
    return HSS_OK;
  });
}

hss_status hss_solve(const hss_matrix* h, int32_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
                     void* stream) {
  return guarded([&]() -> hss_status {
    if (!h || !B || !X || nrhs < 1) throw Error(HSS_ERR_INVALID_ARG, "bad arguments");
    const Job& J = *h->job;
    const Problem& P = J.probs[h->k];
    if (ldb < P.n || ldx < P.n) throw Error(HSS_ERR_INVALID_ARG, "leading dimension < n");
    hipStream_t s = (hipStream_t)stream;
    const hss_allocator* ua = &J.ualloc;
    StreamBuf bp(sizeof(double) * P.n * nrhs, s, ua), xp(sizeof(double) * P.n * nrhs, s, ua);
    const int64_t* perm = P.dev.gen.perm;
    launch_gather_rows(B, ldb, perm, P.n, nrhs, bp.as<double>(), P.n, 0, s);
    ulv_solve_permuted(h, nrhs, bp.as<double>(), xp.as<double>(), s);
    launch_gather_rows(xp.as<double>(), P.n, perm, P.n, nrhs, X, ldx, 1, s);
    HSS_HIP_CHECK(hipGetLastError());
    return HSS_OK;
  });
}

hss_status hss_rel_error(const hss_matrix* h, const hss_generator* gen, double* rel_err) {
  return guarded([&]() -> hss_status {
    if (!h || !rel_err) throw Error(HSS_ERR_INVALID_ARG, "NULL argument");
    const Job& J = *h->job;
    const Problem& P = J.probs[h->k];
    // the built-in families: the job keeps its own generator tables
    const bool cb = P.gen.family == HSS_FAM_CALLBACK;
    if (cb && (!gen || gen->family != HSS_FAM_CALLBACK || !gen->sample || gen->n != P.n))
      throw Error(HSS_ERR_INVALID_ARG, "a caller operator needs its generator (same n, sample routine)");
    hipStream_t s = J.stream;
    const int32_t nb = (int32_t)std::min<int64_t>(P.n, 256);
    DevBuf xp(sizeof(double) * P.n * nb), yp(sizeof(double) * P.n * nb);
    DevBuf ac(cb ? sizeof(double) * P.n * nb : 8);
    DevBuf xh(sizeof(double) * J.mvtot * nb), yh(sizeof(double) * J.mvtot * nb);
    DevBuf ws(sizeof(double) * J.mvwstot * nb);
    DevBuf acc(sizeof(double) * 2 * 1024);
    HSS_HIP_CHECK(hipMemsetAsync(acc.p, 0, sizeof(double) * 2 * 1024, s));
    for (int64_t j0 = 0; j0 < P.n; j0 += nb) {
      const int32_t w = (int32_t)std::min<int64_t>(nb, P.n - j0);
      launch_eye_block(xp.as<double>(), P.n, j0, w, s);
      matvec_permuted(h, w, xp.as<double>(), yp.as<double>(), xh.as<double>(), yh.as<double>(), ws.as<double>(), s);
      if (cb) {   // A_hat [e_j0 ... e_j0+w-1] from the caller's product
        const int32_t rc = gen->sample(gen->ctx, P.n, w, xp.as<double>(), P.n, ac.as<double>(), nullptr, P.n, s);
        if (rc != 0) throw Error(HSS_ERR_CALLBACK, "sample routine returned " + std::to_string(rc));
        launch_err_cols(ac.as<double>(), P.n, yp.as<double>(), P.n, P.n, w, acc.as<double>(), s);
      } else {
        launch_err_block(P.dev.gen, yp.as<double>(), P.n, j0, w, acc.as<double>(), s);
      }
    }
    std::vector<double> hacc(2 * 1024);
    HSS_HIP_CHECK(hipMemcpyAsync(hacc.data(), acc.p, sizeof(double) * 2 * 1024, hipMemcpyDeviceToHost, s));
    HSS_HIP_CHECK(hipStreamSynchronize(s));
    double e = 0.0, a = 0.0;
    for (int i = 0; i < 1024; ++i) {
      e += hacc[2 * i];
      a += hacc[2 * i + 1];
    }
    *rel_err = a > 0.0 ? std::sqrt(e / a) : std::sqrt(e);
    return HSS_OK;
  });
}

hss_status hss_sample(const hss_generator* gen, const int64_t* perm, int32_t ncols, const double* R, int64_t ldr,
                      double* S, int64_t lds, int32_t transpose, int32_t precision, void* stream) {
  return guarded([&]() -> hss_status {
    if (!gen || !R || !S || ncols < 0) throw Error(HSS_ERR_INVALID_ARG, "bad arguments");
    if (ldr < gen->n || lds < gen->n) throw Error(HSS_ERR_INVALID_ARG, "leading dimension < n");
    if (precision < 0 || precision > 2) throw Error(HSS_ERR_INVALID_ARG, "bad precision");
    if (precision != HSS_SAMPLE_FP64 && !gen_formula(gen->family))
      throw Error(HSS_ERR_INVALID_ARG, "reduced-precision sampling needs a generated family");
    hipStream_t s = (hipStream_t)stream;
    if (gen->family == HSS_FAM_CALLBACK) {
      if (!gen->sample) throw Error(HSS_ERR_INVALID_ARG, "callback family needs a sample routine");
      const int32_t rc = gen->sample(gen->ctx, gen->n, ncols, R, ldr, transpose ? nullptr : S,
                                     transpose ? S : nullptr, lds, s);
      if (rc != 0) throw Error(HSS_ERR_CALLBACK, "sample routine returned " + std::to_string(rc));
      HSS_HIP_CHECK(hipStreamSynchronize(s));
      return HSS_OK;
    }
    check_device_perm(perm, gen->n);
    GenHolder G(*gen, perm, s);
    const size_t pe = sample_partial_elems(gen->n, ncols);
    DevBuf part(sizeof(double) * std::max<size_t>(pe, 1));
    launch_sample(G.g, transpose ? 1 : 0, precision, R, ldr, S, lds, ncols, part.as<double>(), s);
    HSS_HIP_CHECK(hipGetLastError());
    HSS_HIP_CHECK(hipStreamSynchronize(s));
    return HSS_OK;
  });
}

hss_status hss_random_normal(int64_t n, int32_t c0, int32_t ncols, uint64_t seed, double* R, int64_t ldr,
                             void* stream) {
  return guarded([&]() -> hss_status {
    if (n < 1 || c0 < 0 || ncols < 0 || (ncols > 0 && !R) || ldr < n)
      throw Error(HSS_ERR_INVALID_ARG, "bad arguments (n >= 1, c0 >= 0, ncols >= 0, ldr >= n)");
    launch_randn(R, ldr, n, c0, ncols, seed, (hipStream_t)stream);
    HSS_HIP_CHECK(hipGetLastError());
    return HSS_OK;
  });
}

hss_status hss_random_words(int64_t n, int32_t c0, int32_t ncols, uint64_t seed, uint64_t* W, int64_t ldw,
                            void* stream) {
  return guarded([&]() -> hss_status {
    if (n < 1 || c0 < 0 || ncols < 0 || (ncols > 0 && !W) || ldw < n)
      throw Error(HSS_ERR_INVALID_ARG, "bad arguments (n >= 1, c0 >= 0, ncols >= 0, ldw >= n)");
    launch_rand_words(W, ldw, n, c0, ncols, seed, (hipStream_t)stream);
    HSS_HIP_CHECK(hipGetLastError());
    return HSS_OK;
  });
}

hss_status hss_extract(const hss_generator* gen, const int64_t* perm, int32_t nI, const int64_t* I, int32_t nJ,
                       const int64_t* Jx, double* out, int64_t ldo, void* stream) {
  return guarded([&]() -> hss_status {
    if (!gen || nI < 0 || nJ < 0 || (nI && !I) || (nJ && !Jx) || !out || ldo < std::max(nI, 1))
      throw Error(HSS_ERR_INVALID_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    if (gen->family == HSS_FAM_CALLBACK) {
      if (!gen->extract) throw Error(HSS_ERR_INVALID_ARG, "callback family needs an extract routine");
      if ((int64_t)nI * nJ > 0) {
        const hss_block b{nI, nJ, I, Jx, out, ldo};
        const int32_t rc = gen->extract(gen->ctx, 1, &b, s);
        if (rc != 0) throw Error(HSS_ERR_CALLBACK, "extract routine returned " + std::to_string(rc));
      }
      HSS_HIP_CHECK(hipStreamSynchronize(s));
      return HSS_OK;
    }
    check_device_perm(perm, gen->n);
    check_device_index(I, nI, gen->n, "I");
    check_device_index(Jx, nJ, gen->n, "J");
    GenHolder G(*gen, perm, s);
    launch_extract(G.g, nI, I, nJ, Jx, out, ldo, s);
    HSS_HIP_CHECK(hipGetLastError());
    HSS_HIP_CHECK(hipStreamSynchronize(s));
    return HSS_OK;
  });
}

hss_status hss_interpolative_batched(int32_t count, const int32_t* m, const int32_t* d, const int64_t* ld,
                                     const double* S, const int64_t* s_off, double eps_r, double eps_a,
                                     int32_t* piv, const int64_t* piv_off, double* E, const int64_t* e_off,
                                     int32_t* rank_host) {
  return guarded([&]() -> hss_status {
    if (count < 0 || (count && (!m || !d || !ld || !S || !s_off || !piv || !piv_off || !E || !e_off || !rank_host)))
      throw Error(HSS_ERR_INVALID_ARG, "NULL argument");
    if (count == 0) return HSS_OK;
    if (!(eps_r >= 0.0) || !(eps_a >= 0.0)) throw Error(HSS_ERR_INVALID_ARG, "need eps >= 0");
    for (int32_t k = 0; k < count; ++k)
      if (d[k] > HSS_MAX_D) throw Error(HSS_ERR_INVALID_ARG, "d above HSS_MAX_D (the pivot step's LDS vector)");
    int32_t mmax = 1, dmax = 1;
    std::vector<int64_t> woff(count), soff(count);
    int64_t wtot = 0, stot = 0;
    for (int32_t k = 0; k < count; ++k) {
      if (m[k] < 0 || d[k] < 0 || ld[k] < std::max(d[k], 1)) throw Error(HSS_ERR_INVALID_ARG, "bad matrix shape");
      mmax = std::max(mmax, m[k]);
      dmax = std::max(dmax, d[k]);
      woff[k] = wtot;
      wtot += (int64_t)std::max(m[k], 1) * ld[k];
      soff[k] = stot;
      stot += 16 + 2 * (int64_t)std::max(m[k], 1) + std::max(d[k], 1);
    }
    DevBuf W(sizeof(double) * std::max<int64_t>(wtot, 1)), scr(sizeof(double) * stot);
    DevBuf drk(sizeof(int32_t) * count), flag(sizeof(int32_t) * 4);
    DevBuf dt(sizeof(QrcpTask) * count), gt(sizeof(GemmTask) * count);
    std::vector<QrcpTask> tasks(count);
    std::vector<int32_t> mc(count);
    for (int32_t k = 0; k < count; ++k) {
      QrcpTask& q = tasks[k];
      std::memset(&q, 0, sizeof(q));
      q.S = S + s_off[k];
      q.lds = ld[k];
      q.W = W.as<double>() + woff[k];
      q.ldw = ld[k];
      q.scr = scr.as<double>() + soff[k];
      q.J = piv + piv_off[k];
      q.E = E + e_off[k];
      q.lde = std::max(m[k], 1);
      q.rank_out = drk.as<int32_t>() + k;
      q.er = eps_r;
      q.ea = eps_a;
      q.hmt_mn = 0.0;
      q.m = m[k];
      q.d = d[k];
      q.mcap = std::max(m[k], 1);
      q.active = 1;
      q.nopivot = 0;
      mc[k] = q.mcap;
    }
    QrcpPlan plan = make_qrcp_plan(mc);
    DevBuf wc(sizeof(int2) * qrcp_work_entries(count)), wm(2 * sizeof(int32_t)),
        wt(sizeof(int2) * plan.trsm.size());
    HSS_HIP_CHECK(hipMemcpy(dt.p, tasks.data(), sizeof(QrcpTask) * count, hipMemcpyHostToDevice));
    HSS_HIP_CHECK(hipMemcpy(wt.p, plan.trsm.data(), sizeof(int2) * plan.trsm.size(), hipMemcpyHostToDevice));
    const QrcpWork wk{wc.as<int2>(), wm.as<int32_t>(), count};
    run_qrcp(dt.as<QrcpTask>(), count, wk, wt.as<int2>(), (int32_t)plan.trsm.size(), std::min(mmax, dmax), dmax,
             mmax, flag.as<int32_t>(), gt.as<GemmTask>(), mmax, nullptr);
    HSS_HIP_CHECK(hipStreamSynchronize(nullptr));
    HSS_HIP_CHECK(hipMemcpy(rank_host, drk.p, sizeof(int32_t) * count, hipMemcpyDeviceToHost));
    return HSS_OK;
  });
}

hss_status hss_release_cache(void) {
  return guarded([&]() -> hss_status {
    arena_release_idle();
    return HSS_OK;
  });
}

hss_status hss_mlp_num_params(const hss_mlp* net, int64_t* out) {
  return guarded([&]() -> hss_status {
    need(net, "net");
    need(out, "out");
    *out = mlp_shape(*net).np;
    return HSS_OK;
  });
}

hss_status hss_mlp_forward(const hss_mlp* net, const float* params, const float* X, int64_t n, float* Y,
                           void* stream) {
  return guarded([&]() -> hss_status {
    need(net, "net");
    const MlpShape S = mlp_shape(*net);
    if (n < 0 || n >= (int64_t(1) << 31)) throw Error(HSS_ERR_INVALID_ARG, "n must be in [0, 2^31)");
    if (n == 0) return HSS_OK;
    need(params, "params");
    need(X, "X");
    need(Y, "Y");
    launch_mlp_tile(S, params, X, nullptr, nullptr, 0, n, 1, 0, n, Y, nullptr, nullptr, 0, (hipStream_t)stream);
    HSS_HIP_CHECK(hipGetLastError());
    return HSS_OK;
  });
}

hss_status hss_mlp_gradient(const hss_mlp* net, const float* params, const float* X, const float* T,
                            const float* M, int64_t n, float* grad, float* loss_dev, void* stream) {
  return guarded([&]() -> hss_status {
    need(net, "net");
    const MlpShape S = mlp_shape(*net);
    if (n < 0 || n >= (int64_t(1) << 31)) throw Error(HSS_ERR_INVALID_ARG, "n must be in [0, 2^31)");
    need(params, "params");
    need(grad, "grad");
    if (n > 0) {
      need(X, "X");
      need(T, "T");
      need(M, "M");
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t nblk = mlp_tiles(n);
    StreamBuf part(sizeof(float) * nblk * S.np, s), cl(sizeof(float) * 2 * nblk, s);
    launch_mlp_tile(S, params, X, T, M, 0, n, 1, 0, std::max<int64_t>(n, 1), nullptr, part.as<float>(),
                    cl.as<float>(), 1, s);
    launch_mlp_reduce(S.np, (int32_t)nblk, part.as<float>(), cl.as<float>(), grad, loss_dev, nullptr, nullptr,
                      nullptr, MlpAdam{}, 0, s);
    HSS_HIP_CHECK(hipGetLastError());
    return HSS_OK;
  });
}

hss_status hss_mlp_adam(int64_t np, float* params, const float* grad, float* m, float* v, float lr, float beta1,
                        float beta2, float eps, int64_t step, void* stream) {
  return guarded([&]() -> hss_status {
    if (np < 0) throw Error(HSS_ERR_INVALID_ARG, "np must be >= 0");
    if (step < 1) throw Error(HSS_ERR_INVALID_ARG, "step must be >= 1");
    if (np == 0) return HSS_OK;
    need(params, "params");
    need(grad, "grad");
    need(m, "m");
    need(v, "v");
    launch_mlp_adam(np, params, grad, m, v, adam_consts(lr, beta1, beta2, eps, step), (hipStream_t)stream);
    HSS_HIP_CHECK(hipGetLastError());
    return HSS_OK;
  });
}

hss_status hss_mlp_train(const hss_mlp* net, float* params, float* m, float* v, int64_t* step, const float* X,
                         const float* T, const float* M, int64_t n, int32_t batch, int32_t epochs, float lr,
                         uint64_t seed, float* loss_host, void* stream) {
  return guarded([&]() -> hss_status {
    need(net, "net");
    const MlpShape S = mlp_shape(*net);
    if (n < 1 || n >= (int64_t(1) << 31)) throw Error(HSS_ERR_INVALID_ARG, "n must be in [1, 2^31)");
    if (batch < 1 || epochs < 0) throw Error(HSS_ERR_INVALID_ARG, "batch must be >= 1 and epochs >= 0");
    need(step, "step");
    if (*step < 0) throw Error(HSS_ERR_INVALID_ARG, "*step must be >= 0");
    need(params, "params");
    need(m, "m");
    need(v, "v");
    need(X, "X");
    need(T, "T");
    need(M, "M");
    hipStream_t s = (hipStream_t)stream;
    const int64_t B = std::min<int64_t>(batch, n);
    const int64_t nbatch = (n + B - 1) / B;
    const int64_t nblk = mlp_tiles(B);
    StreamBuf part(sizeof(float) * nblk * S.np, s), cl(sizeof(float) * 2 * nblk, s);
    StreamBuf losses(sizeof(float) * std::max<int64_t>(1, (int64_t)epochs * nbatch), s);
    for (int32_t e = 0; e < epochs; ++e) {
      int64_t a, c;
      epoch_order(seed, e, n, a, c);
      for (int64_t b = 0; b < nbatch; ++b) {
        const int64_t p0 = b * B, p1 = std::min(n, p0 + B);
        launch_mlp_tile(S, params, X, T, M, p0, p1, a, c, n, nullptr, part.as<float>(), cl.as<float>(), 1, s);
        ++*step;
        launch_mlp_reduce(S.np, (int32_t)mlp_tiles(p1 - p0), part.as<float>(), cl.as<float>(), nullptr,
                          losses.as<float>() + (int64_t)e * nbatch + b, params, m, v,
                          adam_consts(lr, 0.9f, 0.999f, 1e-8f, *step), 1, s);
      }
    }
    HSS_HIP_CHECK(hipGetLastError());
    std::vector<float> lh((size_t)std::max<int64_t>(1, (int64_t)epochs * nbatch));
    if (epochs > 0)
      HSS_HIP_CHECK(hipMemcpyAsync(lh.data(), losses.p, sizeof(float) * epochs * nbatch, hipMemcpyDeviceToHost, s));
    HSS_HIP_CHECK(hipStreamSynchronize(s));
    if (loss_host)
      for (int32_t e = 0; e < epochs; ++e) {
        double q = 0.0;
        for (int64_t b = 0; b < nbatch; ++b) q += lh[(size_t)(e * nbatch + b)];
        loss_host[e] = (float)(q / (double)nbatch);
      }
    return HSS_OK;
  });
}

}  // extern "C"
