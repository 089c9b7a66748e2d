// Host-side job state of libhss (see driver.cpp).
#pragma once

#include <memory>
#include <vector>

#include "hss_internal.h"

namespace hss {

hss_tree* tree_build(int64_t n, const double* pts, int32_t leaf, int32_t method);
void tree_free(hss_tree* t);

struct Problem {
  hss_generator gen;
  hss_options opt;
  int64_t n = 0;
  int32_t nn = 0;
  int32_t sym = 1;
  int32_t dcap = 0;
  int32_t node0 = 0;
  std::vector<int64_t> perm;
  int64_t sglob[2] = {0, 0};
  int64_t rglob = -1;          // offset of the library-drawn R in the transient pool (-1: caller's R)
  ProbDev dev;
  int32_t d = 0, b = 0, force = 0, done = 0, rounds = 0;
  hss_status status = HSS_OK;
  std::vector<int32_t> sched;
  int32_t* sched_d = nullptr;
  int64_t* pos_d = nullptr;   // caller operators: device 0..n-1 (leaf index lists)
  double d_pred = 0.0;        // the learned predictor's final sample count (0: none)
};

struct LevelInfo {
  std::vector<int32_t> nodes;
  int32_t off = 0;
  int32_t mcap = 0, rcap = 0, qcap = 0, dcap = 0;
  int2* wg_trsm = nullptr;   // back-substitution workgroup map (device)
  int32_t ntrsm = 0;
  int2* wg_test = nullptr;   // explicit-Q workgroup map for test_ncap columns
  int32_t ntest = 0, test_ncap = 0;
  IdBlockWork idb;           // block-pivoted ID slots of the level's nodes
};

// The IDs of the compression use the block-pivoted factorization
// (k_idblock.hip); the one-step kernels still factor the stopping test's blocks.
constexpr bool kBlockId = true;

size_t arena_idle_bytes();   // idle cached transient memory on the current device
void arena_release_idle();   // free it

// The factorization of one compressed problem (ulv.cpp, k_ulv.hip).
struct UlvFactor {
  struct Node {
    int32_t g = -1;                       // global node id
    int32_t m = 0, k = 0, r = 0;          // local size, redundant count, rank
    int32_t level = 0, leaf = 0, lo = 0;
    int32_t left = -1, right = -1;        // local ids of the children
    int32_t rl = 0;                       // left child's rank
    int64_t F = 0, inv = 0, piv = 0, Y = 0;   // offsets: block, inverses, pivots, solve rows
    const int32_t *Jr = nullptr, *Jc = nullptr;
    const double *Er = nullptr, *Ec = nullptr;   // r x k, column-major
    int32_t eldr = 1, eldc = 1;
  };
  std::vector<Node> nodes;                // local ids in the tree's order (root 0)
  int32_t maxlevel = 0;
  double* fpool = nullptr;                // the nodes' blocks
  double* ipool = nullptr;                // diagonal-block inverses
  int32_t* ppool = nullptr;               // pivots
  int64_t ytot = 0;                       // rows of the solve's per-node buffers
  int64_t fbytes = 0;                     // device bytes held
  double factor_ms = 0.0;
};

struct Job {
  std::vector<Problem> probs;
  std::vector<std::unique_ptr<UlvFactor>> ulv;   // per problem, once hss_factor ran
  std::vector<NodeDesc> desc;
  std::vector<NodeState> st_h;
  std::vector<LevelInfo> levels;
  int32_t maxlevel = 0;
  int32_t strategy = 0;
  bool all_sym = true;
  bool has_callback = false;   // some problem has caller routines (HSS_FAM_CALLBACK)
  int32_t max_block = 0;   // widest sampling block so far
  hipStream_t stream = nullptr;
  hss_allocator ualloc{};          // caller's device memory (alloc = NULL: the library's own)
  std::vector<void*> allocs;       // live until the job is destroyed
  std::vector<void*> transients;   // freed when the compression ends
  double *dpool = nullptr, *tpool = nullptr, *wsa = nullptr, *wsb = nullptr, *partial = nullptr;
  double* epool = nullptr;         // compacted E (after compression)
  double* gemm_ws = nullptr;       // split-K partial tiles (transient)
  int32_t* ipool = nullptr;
  int64_t* lpool = nullptr;
  NodeDesc* desc_d = nullptr;
  NodeState* st_d = nullptr;
  ProbDev* prob_d = nullptr;
  GemmTask* tasks_d = nullptr;
  // [0] non-finite entry seen, [1] largest block count of a level, [2] a
  // node passed in a level whose ID was skipped, [3] the stopping test's
  // factorization scratch, [4] the ID's, [5] and [6] largest column count
  // and local-sample row count of a level's active nodes
  int32_t* flags_d = nullptr;
  int32_t* nodes_d = nullptr;
  QrcpTask* qtasks_d = nullptr;
  QrcpWork qwork{nullptr, nullptr, 0};   // device work map of every factorization call
  QrcpGraphs qgraphs;                    // replayed pivot-step segments
  double* idb_dpool = nullptr;           // block-ID slots (transient)
  int32_t* idb_ipool = nullptr;
  GemmTask* idb_gt = nullptr;            // block-ID GEMM tasks, 3 per node of a level
  QformTask* qform_d = nullptr;
  CholTask* chol_d = nullptr;
  int64_t* mvoff_d = nullptr;   // per node: prefix sum of rcap (matvec slots)
  int64_t mvtot = 0;
  int64_t* mvws_d = nullptr;    // per node: prefix sum of mcap (matvec workspace)
  int64_t mvwstot = 0;
  GemmTask* mvtasks_d = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t ev_flag = nullptr;    // marks a read-back of flags into hflags
  int32_t* sched_all_d = nullptr;  // sampling schedules, sched_stride int32 per problem
  int32_t* sched_h = nullptr;      // their pinned staging copy
  int64_t sched_stride = 0;
  int32_t* hflags = nullptr;       // pinned host words for read-backs
  double sample_ms = 0.0, sample_flops = 0.0, total_ms = 0.0;
  double alloc_ms = 0.0;           // host time spent in device allocations (setup statistics)
  Prof prof;
  unsigned long long* kcnt_d = nullptr;     // device algorithmic counters
  hss_kernel_stats kstats[HSS_K_COUNT] = {};
  double host_bytes[HSS_K_COUNT] = {}, host_flops[HSS_K_COUNT] = {};

  ~Job();
  void* dalloc(size_t bytes, bool transient = false);
  void dfree(void* p);                 // a block from dalloc, stream-ordered
  void drop(void* p);                  // dfree of a dalloc block the job no longer tracks
  void* arena_acquire(size_t bytes);   // transient block (see driver.cpp)
  void arena_return();
  int arena_dev = -1;                  // device whose cached block this job holds
  void release_transients();
  void compact_e();
  void setup(int32_t count, const hss_generator* gens, const hss_tree* const* trees,
             const hss_options* opts);
  // Device bytes of one problem in a job; *shared: bytes of the buffers one
  // job keeps for all of its problems, sized by this problem (the job
  // allocates their maximum once).
  static size_t estimate_bytes(const hss_generator& g, const hss_tree* t, const hss_options& o, size_t* shared);
  // Host-only checks of one problem's arguments (no HIP call): throws
  // HSS_ERR_INVALID_ARG naming problem k.
  static void validate(const hss_generator& g, const hss_tree* t, const hss_options& o, int k);
  void compress();
  void sample(Problem& P, int32_t c0, int32_t ncols);
  void sample_begin();
  void sample_end();
  void run_level(int lev, int32_t ncap);
  void extract_callbacks(int lev);
  void require_finite(const char* who);
};

}  // namespace hss

// One compressed problem; `job` is shared by the problems of a batched call.
struct hss_matrix {
  std::shared_ptr<hss::Job> job;
  int32_t k = 0;
};

namespace hss {
// Yp = H Xp in the tree's permuted order, both n x nrhs with leading
// dimension n; xh, yh hold Job::mvtot * nrhs doubles, ws Job::mvwstot * nrhs
// (written before they are read).  Asynchronous on s; allocates nothing.
void matvec_permuted(const hss_matrix* h, int32_t nrhs, const double* Xp, double* Yp, double* xh,
                     double* yh, double* ws, hipStream_t s);
// Factorization of problem h->k (hss_factor) and X = H^{-1} B in the
// tree's permuted order (hss_solve; Bp, Xp: n x nrhs, ld n; asynchronous on s).
void ulv_factor(hss_matrix* h);
void ulv_solve_permuted(const hss_matrix* h, int32_t nrhs, const double* Bp, double* Xp, hipStream_t s);
// Sets the thread's hss_last_error() message and returns code.
hss_status record_error(hss_status code, const std::string& msg);
}  // namespace hss
