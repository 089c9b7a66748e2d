// Internal definitions shared by the host driver and the HIP kernels of
// libhss.  Device data of one compression job lives in a few pools; every
// node of every problem of the job has a NodeDesc (static: capacities and
// pool offsets) and a NodeState (mutable, updated by the kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hss.h"

namespace hss {

enum NodeStateCode : int32_t { UNTOUCHED = 0, PARTIAL = 1, COMPRESSED = 2 };

// Generator as seen by the kernels (entries of the PERMUTED operator).
struct GenDev {
  int32_t family;
  int32_t symmetric;
  int64_t n;
  double t0;          // Toeplitz t(0)
  double inv2s2;      // Gaussian 1/(2 sigma^2)
  double diag;        // Laplace A_ii, Gaussian diagonal shift
  const double* tcol; // Toeplitz t(0..n-1), library owned
  const double* pts;  // points in permuted order, n x 3, library owned
  const int64_t* perm;
  const double* dense;
  int64_t ld;
  const int32_t* leaf_lo;  // per permuted index: range of its leaf (reduced-precision
  const int32_t* leaf_hi;  // sampling skips these diagonal blocks when offdiag = 1)
  int32_t offdiag;
  int32_t perm_id;    // 1: perm is the identity (Toeplitz entries from an LDS window)
};

// The generated families are symmetric; dense and caller operators say
// whether they are.
inline bool gen_symmetric(const hss_generator& g) {
  return (g.family != HSS_FAM_DENSE && g.family != HSS_FAM_CALLBACK) || g.symmetric != 0;
}
// Families whose entries the kernels compute from a formula.
inline bool gen_formula(int32_t family) {
  return family == HSS_FAM_TOEPLITZ || family == HSS_FAM_LAPLACE || family == HSS_FAM_GAUSS;
}

// Static per-node description.  Offsets are in elements of the pool of the
// matching type (double pool, int32 pool, int64 pool).  Side 0 is the row
// side (S^r, U, J^r, I^r, R^c = U^T R), side 1 the column side (S^c, V,
// J^c, I^c, R^r = V^T R); for symmetric problems side 1 aliases side 0.
struct NodeDesc {
  int32_t prob;
  int32_t level;
  int32_t leaf;
  int32_t parent, left, right;  // global node ids, -1 if none
  int32_t lo, hi;               // permuted index range within the problem
  int32_t mcap;                 // capacity of local-sample rows
  int32_t rcap;                 // capacity of the rank
  int32_t qcap;                 // capacity of the test basis Q
  int32_t eld[2];               // leading dimension of E per side (rcap while compressing,
                                // the rank once E is compacted into its own pool)
  int32_t b12ld, b21ld;         // leading dimensions of B12 / B21 (likewise)
  int64_t S[2];    // (tpool) local samples, mcap x dcap, row-major (ld = dcap)
  int64_t RR[2];   // (tpool) reduced random matrix from side s's basis: rcap x dcap row-major
  int64_t Q[2];    // (tpool) stopping-test basis, mcap x qcap column-major
  int64_t E[2];    // interpolation matrix E, column-major with leading dimension eld:
                   // rcap x mcap in the transient pool while compressing, then
                   // rank x (m - rank) in the E pool
  int64_t J[2];    // int32 pool: mcap pivot order
  int64_t I[2];    // int64 pool: rcap skeleton indices
  int64_t D;       // leaf: size x size column-major
  int64_t B12;     // B12 column-major with leading dimension b12ld (transient pool
  int64_t B21;     // while compressing, then compacted like E)
  int64_t ws;      // offset of this node's slot in the level workspace A (mcap x dcap)
  int64_t wsq;     // offset in the level workspace B (qcap x dcap)
};

struct NodeState {
  int32_t state;
  int32_t active;   // local samples are computed this round
  int32_t fresh;    // was UNTOUCHED when the round reached it
  int32_t extract;  // needs D / B extraction this round
  int32_t c0, nc;   // new columns [c0, c0 + nc) of this round
  int32_t go;       // compress (ID) this round
  int32_t test;     // not yet compressed: evaluate the stopping test
  int32_t m[2];     // rows of the local samples per side
  int32_t rank[2];
  int32_t passed[2];
  int32_t need[2];  // F-norm test must run its projections this round
  int32_t q[2];     // columns of Q per side
  int32_t tb;       // first sampling block to test this round
  int32_t nblk;     // number of blocks to test this round
  int32_t run[2];   // the current test iteration runs its QR on this side
  int32_t bc0, bnc; // columns of the block under test
  int32_t qrank;    // columns the QR of the projected block reached
  int32_t reo;      // HMT-lemma test: the block appended to Q on side reo - 1 awaits re-orthogonalization
  double rho[2];
};

// Per-problem device parameters (rewritten by the host every round).
struct ProbDev {
  int32_t d;        // columns sampled so far
  int32_t b;        // columns added in the last sampling step
  int32_t force;    // accept every open node
  int32_t done;     // root compressed: skip all work
  int32_t dcap;
  int32_t strategy;
  int32_t p;        // HMT oversampling
  int32_t symmetric;
  int64_t n;
  double eps_r, eps_a;   // eta * tol (divided by level(tau) in the kernels)
  int64_t sglob[2];      // offsets of the global samples (n x dcap col-major) in the transient pool
  const double* R;
  int64_t ldr;
  const int32_t* sched;  // d after every sampling step (block edges), nsched entries
  int32_t nsched;
  int32_t pad1;
  double eps_floor;      // lower bound of eps_r / level(tau) (sampling precision floor)
  double hmt_alpha;      // alpha of the HMT-lemma test (HSS_INC_HMT)
  GenDev gen;
};

// C(i,j) = alpha * sum_k A(i,k) B(k,j) + beta * C(i,j) with arbitrary strides.
// a_cols, when set, maps column k of A to the physical column a_cols[k];
// b_cols and c_cols map column j of B and of C to physical columns.
struct GemmTask {
  const double* A;
  const double* B;
  double* C;
  int64_t a_rs, a_cs, b_rs, b_cs, c_rs, c_cs;
  int32_t M, N, K, pad;
  double alpha, beta;
  const int32_t* a_cols = nullptr;
  const int32_t* b_cols = nullptr;
  const int32_t* c_cols = nullptr;
};

// One matrix of a batched interpolative decomposition (k_qrcp.hip).
// S: m rows of length d (row j at S + j * lds); W: panel, column j at
// W + j * ldw; scr: 16 + 2 * mcap + min(m, d) doubles of scratch; J: m
// int32; E: rank x (m - rank), column-major with leading dimension lde.
struct QrcpTask {
  const double* S;
  int64_t lds;
  double* W;
  int64_t ldw;
  double* scr;
  int32_t* J;
  double* E;
  int64_t lde;
  int32_t* rank_out;
  double er, ea;     // stop when nu_k <= max(ea, er * nu_1) (/ HMT factor)
  double hmt_mn;     // > 0: HMT factor with sqrt(hmt_mn); 0: plain threshold
  int32_t m, d, mcap, active;
  int32_t nopivot;   // 1: plain Householder QR (column k is the k-th pivot)
};

// Explicit Q of a Householder QR done by run_qrcp in nopivot mode:
// Q(:, 0:nc) = H_0 ... H_{nc-1} [I; 0], reflectors rebuilt from the panel
// columns W(k:m, k) and the diagonal rdiag[k].  With a workspace wk of
// 2 nc^2 + 8 doubles, Q is formed in compact WY form and W is overwritten
// by V; without (wk == nullptr) column by column.
struct QformTask {
  double* W;
  int64_t ldw;
  const double* rdiag;
  double* Q;
  int64_t ldq;
  double* wk;
  int32_t m, nc, active, pad;
};

constexpr int QCPW = 16;  // panel columns owned by one workgroup of the ID

struct QrcpPlan {
  std::vector<int2> step;   // (task, first column) per workgroup of a pivot step
  std::vector<int2> trsm;   // (task, first column of E) per workgroup of the solve
};
QrcpPlan make_qrcp_plan(const std::vector<int32_t>& mcaps, int cpw = QCPW);
// Busy workgroups aimed at by every pivot-step launch (5 per compute unit:
// more waves keep more column loads in flight; 4 and 7 per unit were slower).
// The plan kernel doubles it for steps that would give a workgroup 16 or
// more columns (large batches of panels).
constexpr int kQrcpTarget = 1280;   // default; the active tunables' qrcp_wg (<= HSS_QRCP_WG_MAX) is used
// Panels of at most this many cells (rows x columns, by capacity) are
// factored by one workgroup each in a single launch.
constexpr int64_t kQrcpWgCells = 64 * 1024;
// Device work map of run_qrcp: chunks holds 2 kQrcpTarget + max_tasks
// entries (the target doubles for large steps), meta two int32.
struct QrcpWork;
// Instantiated graphs of kSegSteps back-to-back pivot steps, per (grid,
// LDS bytes), owned by a compression job.
constexpr int kSegSteps = 32;
struct QrcpGraphs {
  std::map<std::pair<int, size_t>, hipGraphExec_t> execs;
  hipGraphExec_t segment(const QrcpTask* tasks, const QrcpWork& wk, int nwg, size_t lds, unsigned long long* kcnt);
  ~QrcpGraphs();
};
struct QrcpWork {
  int2* chunks;
  int32_t* meta;
  int32_t max_tasks;
  int32_t* kbuf = nullptr;        // 2 int32: step counter of the graph replays (nullptr: no graphs)
  QrcpGraphs* graphs = nullptr;   // graph cache (nullptr: plain launches)
};
inline size_t qrcp_work_entries(int32_t max_tasks) { return (size_t)2 * HSS_QRCP_WG_MAX + (size_t)std::max(max_tasks, 1); }

// Launch-shape tunables of the calling thread's compression (the defaults
// outside one); TuneScope makes a table entry active for a compression.
const hss_tunables& tune();
struct TuneScope {
  explicit TuneScope(const hss_tunables& t);
  ~TuneScope();
  const hss_tunables* saved;
};
hss_tunables tunables_for(int32_t family, int32_t precision, int64_t n);   // device 0 of the current context
// Block-pivoted ID (k_idblock.hip): per task, a slot of workspace sized
// from its capacities (panel rows dcap, columns mcap).
constexpr int kIdbCmax = 256;   // candidate columns per block
constexpr int kIdbLmax = 32;    // pivots per block at most
constexpr int kIdbMaxM = 16384; // panel columns the selection kernel stages in LDS (larger: one-step path)
constexpr int kIdbRows = 256;   // panel rows per workgroup of the block's row kernels
// per row workgroup: the upper 4 x 4 blocks of its share of Q1^T Q1
constexpr int kIdbPart = (kIdbLmax / 4) * (kIdbLmax / 4 + 1) / 2 * 16;
struct IdBlk {
  int32_t* cand;     // kIdbCmax candidate columns, ascending
  int32_t* rest;     // mcap columns left after the block, ascending
  int32_t* piv;      // kIdbLmax: the block's pivots (indices into cand), in order
  double* C;         // ldc x kIdbCmax: the candidates' rows k .. d
  int64_t ldc;
  double* G;         // kIdbCmax x kIdbCmax Gram matrix
  double* V;         // ldv x kIdbLmax: Q1 of the pivot columns, then the block's reflectors
  double* U;         // ldv x kIdbLmax: V T^T
  int64_t ldv;
  double* Y;         // kIdbLmax x mcap: V^T times the remaining columns
  double* F;         // 4 kIdbLmax x kIdbLmax, row-major: R1, M, T, Y_1
  double* P;         // ceil(ldv / kIdbRows) x kIdbPart: partial sums of Q1^T Q1
  double bound;      // largest residual norm among the non-candidates
  int32_t k;         // first panel row of the next block
  int32_t kb;        // first panel row of the last block factored
  int32_t ncand, nrest;
  int32_t L;         // pivots of the last block (0: none)
  int32_t lc;        // pivots the block's Cholesky step took
  int32_t stop;      // the threshold ended the Cholesky step
  int32_t cmax;
};
// Doubles and int32 of one task's slot.
inline int64_t idblk_doubles(int64_t dcap, int64_t mcap) {
  const auto a8 = [](int64_t x) { return (x + 7) & ~int64_t(7); };
  return a8(dcap * kIdbCmax) + a8((int64_t)kIdbCmax * kIdbCmax) + 2 * a8(dcap * kIdbLmax) + a8(kIdbLmax * mcap) +
         a8(4 * (int64_t)kIdbLmax * kIdbLmax) + a8((dcap + kIdbRows - 1) / kIdbRows * kIdbPart);
}
inline int64_t idblk_ints(int64_t mcap) { return ((kIdbCmax + kIdbLmax + mcap) + 7) & ~int64_t(7); }
struct IdBlockWork {
  IdBlk* blk = nullptr;      // device, one per task
  GemmTask* gt = nullptr;    // device, 3 per task (Gram, V^T A, update)
  int32_t max_tasks = 0;
};
// The block pivot steps of one factorization call, after the panels and
// their norms are in place (k_qrcp_init); hw_dev / hw: a mapped
// host word for the liveness polls.
void run_id_blocks(QrcpTask* tasks, int32_t ntasks, const IdBlockWork& bw, int32_t dmax, int32_t mmax,
                   int32_t* hw_dev, const int32_t* hw, double* gws, hipStream_t s, unsigned long long* kcnt);
// Factor the panels of `tasks` (dmax rows and at most ncols_max columns
// each, by capacity): for an ID with a block workspace, the block-pivoted
// factorization (k_idblock.hip); otherwise one workgroup per matrix for
// small panels, or one launch per pivot step over a device-built work map.
// `flag` points at one int32 of device scratch.
void run_qrcp(QrcpTask* tasks, int32_t ntasks, const QrcpWork& wk, const int2* wg_trsm, int32_t ntrsm,
              int32_t kmax, int32_t dmax, int32_t ncols_max, int32_t* flag, GemmTask* gtasks, int32_t mcap_max,
              hipStream_t s, unsigned long long* kcnt = nullptr, bool solve_e = true, double* gws = nullptr,
              const IdBlockWork* bw = nullptr);
// Host-synchronous count of the active panels of a factorization call.
int32_t count_active_panels(const QrcpTask* tasks, int32_t ntasks, hipStream_t s);
void run_qform(QformTask* tasks, int32_t count, const int2* wg, int32_t nwg, int32_t cpw, int32_t ncmax,
               int32_t mmax, GemmTask* gt, double* gws, hipStream_t s, unsigned long long* kcnt);

// ------------------------------------------------------------------ global views
// Device pointers read from task structures are generic (flat) to the
// compiler, and a flat access is counted both as a vector-memory and as an
// LDS operation: every wait for an LDS result then also waits for all flat
// loads in flight, which serializes loops that mix the two.  Accesses
// through these views are global-memory instructions instead.
#define HSS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const HSS_GLOBAL T* gview(const T* p) {
  return (const HSS_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ HSS_GLOBAL T* gview_w(T* p) {
  return (HSS_GLOBAL T*)p;
}

// ------------------------------------------------------------------ profiling
// Launch counts and (in profile mode) HIP-event time per kernel class; the
// algorithmic bytes / flops are accumulated on the device in kcnt[2 * class
// + {0, 1}] (unsigned 64-bit).
struct Prof {
  bool on = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double ms[HSS_K_COUNT] = {};
  int64_t launches[HSS_K_COUNT] = {};
};
extern thread_local Prof* g_prof;
void prof_begin(hipStream_t s);
// Closes the interval opened by prof_begin and charges it to class cls;
// nlaunch kernels were launched back to back inside it.
void prof_end(int cls, hipStream_t s, int nlaunch = 1);
// Counts n units of class cls without timing (classes that only total work).
void prof_count(int cls, int n);

__device__ __forceinline__ void kcount(unsigned long long* kc, int cls, double bytes, double flops) {
  if (!kc) return;
  atomicAdd(kc + 2 * cls, (unsigned long long)bytes);
  atomicAdd(kc + 2 * cls + 1, (unsigned long long)flops);
}

// ------------------------------------------------------------------ launchers
void launch_toeplitz_table(double* t, int64_t n, double h, hipStream_t s);
void launch_permute_points(const double* pts, const int64_t* perm, int64_t n, double* out,
                           hipStream_t s);
// Sampling: S(:, 0:ncols) = op(A_hat) R(:, 0:ncols); `partial` is workspace of
// partial_cap doubles for the split-K partial sums.
size_t sample_partial_elems(int64_t n, int32_t ncols);
void launch_sample(const GenDev& g, int32_t transpose, int32_t precision, const double* R,
                   int64_t ldr, double* S, int64_t lds, int32_t ncols, double* partial,
                   hipStream_t s, unsigned long long* kcnt = nullptr);
void launch_extract(const GenDev& g, int32_t nI, const int64_t* I, int32_t nJ, const int64_t* J,
                    double* out, int64_t ldo, hipStream_t s);
// Grouped GEMM over tasks of at most mcap x ncap outputs; with a workspace
// of ws_elems doubles and kcap (largest K) long enough, K is split into
// slices summed in fixed order (k_gemm.hip).
void launch_gemm(const GemmTask* tasks, int32_t ntasks, int32_t mcap, int32_t ncap,
                 hipStream_t s, unsigned long long* kcnt = nullptr, int32_t kcap = 0,
                 double* ws = nullptr, int64_t ws_elems = 0, int cls = HSS_K_GEMM);
// Split-K workspace of a compression job (doubles).
constexpr int64_t kGemmSplitElems = int64_t(16) << 20;

struct LevelArgs {
  const NodeDesc* desc;
  NodeState* st;
  const ProbDev* prob;
  const int32_t* nodes;  // global ids of this level's nodes
  int32_t count;
  double* dpool;         // persistent doubles: D, B12, B21, E
  double* tpool;         // compression-time doubles: S, RR, Q, global samples
  int32_t* ipool;
  int64_t* lpool;
  double* wsA;
  double* wsB;
  GemmTask* tasks;       // scratch task array, capacity >= 2 * count
  int32_t* flags;        // device error flags
  unsigned long long* kcnt;  // algorithmic byte / flop counters
  double* gws;           // split-K partial tiles, kGemmSplitElems doubles
};

void launch_plan(const LevelArgs& a, hipStream_t s);
void launch_extract_nodes(const LevelArgs& a, hipStream_t s);
void launch_local_samples(const LevelArgs& a, int side, int32_t mcap_max, int32_t rcap_max,
                          int32_t dcap_max, hipStream_t s);
// One iteration of the Alg. 5 test on side `side`: copy + CGS2 (GEMMs),
// norms and the F-norm tests, Householder QR of the projected block on
// many workgroups (run_qrcp, nopivot), the R-diagonal tests, explicit Q_k.
// Cholesky QR (two passes) of a projected block S_hat (m x nc, nc <=
// kCholMaxB): Q1 = S_hat R1^{-1}, Q = Q1 R2^{-1}, Rbar = R2 R1, used to
// decide a clearly failing stopping test without the Householder QR.
constexpr int kCholMaxB = 128;
struct CholTask {
  const double* S;   // S_hat, column-major, leading dimension lds
  int64_t lds;
  double* Q1;        // m x nc, leading dimension lds
  double* G;         // nc x nc Gram matrix
  double* X;         // nc x nc inverse triangular factor
  double* d1;        // nc: diagonal of R1
  int32_t m, nc, active, pad;
};
struct TestScratch {
  QrcpTask* qt;        // count entries
  QformTask* qf;       // count entries
  CholTask* ct;        // count entries
  const int2* wg;      // (task, first column) pairs for cpw-column workgroups (explicit Q)
  int32_t nwg;
  int32_t cpw;
  int32_t* flag;
  GemmTask* gt;
  QrcpWork wk;         // device work map of the Householder QR
};
// One iteration of the stopping test on one side: the F-norm test of
// Alg. 5, or with `hmt` the test of eq. HMT_IQQH (HSS_INC_HMT), whose
// appended blocks are re-orthogonalized against the earlier basis.
void launch_fnorm_test(const LevelArgs& a, int side, int32_t iter, int32_t mcap_max,
                       int32_t qcap_max, int32_t ncap, const TestScratch& ts, hipStream_t s, bool hmt);
void launch_decide_fnorm(const LevelArgs& a, hipStream_t s, int32_t* unexpected = nullptr);
void launch_build_qrcp(const LevelArgs& a, int side, int32_t hmt, QrcpTask* out, hipStream_t s);
void launch_decide_hmt(const LevelArgs& a, hipStream_t s);
void launch_reduce(const LevelArgs& a, int side, int32_t mcap_max, int32_t rcap_max,
                   int32_t dcap_max, hipStream_t s);
void launch_finalize(const LevelArgs& a, hipStream_t s);


// Matvec pieces (one workgroup per node of a level).
// Tasks of the HSS factorization and solve (k_ulv.hip), one per node.
// F: the node's m x m block in [redundant; skeleton] order (column-major,
// ld m); k = m - r redundant unknowns (the root: k = m, no basis, J null).
struct UlvBuild {
  double* F;
  const double* D;              // leaf: m x m in local order (else null)
  const double *Fl, *Fr;        // children's blocks (their trailing r x r blocks are read)
  const double *B12, *B21;
  const int32_t *Jr, *Jc;       // the node's row / column ID order (null at the root)
  int32_t m, k, r;
  int32_t rl, kl, ml, kr, mr;   // left rank; children's k and m
  int32_t ld12, ld21;
};
struct UlvPanel {
  double* F;
  double* inv;     // Linv then Uinv, 32 x 32 each, column-major
  int32_t* piv;    // the node's pivot rows (k entries)
  int32_t m, k, jb, nb;
};
struct UlvSwap {   // the row swaps of one panel on columns [c0, c1) of X
  double* X;
  const int32_t* piv;
  int64_t ld, c0, c1;
  int32_t jb, nb;
};
struct UlvMove {   // right-hand sides into / solutions out of a node's Y
  double* Y;                    // m x nrhs, ld m, [R; S] order
  double* ext;                  // leaf: permuted B or X (n rows, ld ldext); else null
  double *Yl, *Yr;              // children's Y (their rows k.. hold the skeleton)
  const int32_t* J;             // the node's row (in) or column (out) ID order; null at the root
  int64_t ldext;
  int32_t m, k, r, lo, rl, kl, ml, kr, mr;
};
struct UlvSubst {   // a node's whole forward or backward block substitution
  double* Y;                    // m x nrhs, ld m
  const double* F;
  const double* inv;            // the node's diagonal-block inverses
  const int32_t* piv;
  int32_t m, k;
};
constexpr int UST_MAXR = 16;    // right-hand sides up to which the fused substitutions run
void launch_ulv_subst(const UlvSubst* t, int32_t count, int32_t nrhs, int32_t backward, hipStream_t s);
void launch_ulv_build(const UlvBuild* t, int32_t count, int64_t maxelems, hipStream_t s);
void launch_ulv_panel(const UlvPanel* t, int32_t count, int32_t* flag, hipStream_t s);
void launch_ulv_swap(const UlvSwap* t, int32_t count, int64_t maxcols, hipStream_t s);
void launch_ulv_rhs_in(const UlvMove* t, int32_t count, int32_t nrhs, int64_t maxelems, hipStream_t s);
void launch_ulv_x_out(const UlvMove* t, int32_t count, int32_t nrhs, int64_t maxelems, hipStream_t s);

struct MvArgs {
  const NodeDesc* desc;
  const NodeState* st;
  const int32_t* nodes;
  int32_t count;
  const double* dpool;
  const double* epool;  // compacted E
  const int32_t* ipool;
  double* xh;           // per node: rcap x nrhs (column-major, ld = rcap)
  double* yh;
  const int64_t* xh_off;  // per global node offset into xh / yh
  const double* X;      // permuted input, n x nrhs (ld = n)
  double* Y;
  int64_t n;
  int32_t nrhs;
  double* ws;           // per node: mcap x nrhs workspace (column-major, ld = mcap)
  const int64_t* ws_off;
};
void launch_mv_up(const MvArgs& a, GemmTask* tasks, int32_t mcap, hipStream_t s);
void launch_mv_down(const MvArgs& a, GemmTask* tasks, int32_t mcap, hipStream_t s);
void launch_gather_rows(const double* X, int64_t ldx, const int64_t* perm, int64_t n, int32_t nrhs,
                        double* out, int64_t ldo, int32_t inverse, hipStream_t s);
void launch_eye_block(double* X, int64_t n, int64_t j0, int32_t nb, hipStream_t s);
// dst(i,j) = src(i,j) for rows x cols blocks, one workgroup per block
struct Copy2D {
  const double* src;
  int64_t lds;
  double* dst;
  int64_t ldd;
  int32_t rows, cols;
};
void launch_copy2d(const Copy2D* tasks, int32_t count, hipStream_t s);
void launch_err_block(const GenDev& g, const double* Hc, int64_t ldh, int64_t j0, int32_t nb,
                      double* accum, hipStream_t s);
void launch_err_cols(const double* Ac, int64_t lda, const double* Hc, int64_t ldh, int64_t n, int32_t nb,
                     double* accum, hipStream_t s);
void launch_check_finite(const double* p, int64_t rows, int32_t cols, int64_t ld, int32_t* flag, hipStream_t s);
// Columns c0 .. c0+ncols-1 of the counter-based Gaussian R (k_rng.hip),
// written to R (n x ncols, leading dimension ldr), or their raw Philox words.
void launch_randn(double* R, int64_t ldr, int64_t n, int32_t c0, int32_t ncols, uint64_t seed, hipStream_t s);
void launch_rand_words(uint64_t* W, int64_t ldw, int64_t n, int32_t c0, int32_t ncols, uint64_t seed,
                       hipStream_t s);

// ---- learned predictor network (k_mlp.hip) ----
struct MlpShape {
  int32_t nl;
  int32_t sz[HSS_MLP_MAX_LAYERS + 1];
  int32_t ald[HSS_MLP_MAX_LAYERS + 1];   // LDS leading dimension of each activation tile
  int32_t aoff[HSS_MLP_MAX_LAYERS + 1];  // LDS offset (floats) of each activation tile
  int64_t woff[HSS_MLP_MAX_LAYERS];
  int64_t boff[HSS_MLP_MAX_LAYERS];
  int64_t np;
  int32_t lds_floats;
};
struct MlpAdam {
  float lr, b1, b2, eps, bc1, bc2;  // bc = 1 - beta^step
};
MlpShape mlp_shape(const hss_mlp& net);
int64_t mlp_tiles(int64_t rows);
void launch_mlp_tile(const MlpShape& S, const float* P, const float* X, const float* T, const float* M,
                     int64_t pos0, int64_t pos1, int64_t pa, int64_t pc, int64_t nd, float* Y, float* part,
                     float* cl, int mode, hipStream_t s);
void launch_mlp_reduce(int64_t np, int32_t nblk, const float* part, const float* cl, float* grad, float* loss,
                       float* params, float* am, float* av, const MlpAdam& a, int adam, hipStream_t s);
void launch_mlp_adam(int64_t np, float* params, const float* grad, float* am, float* av, const MlpAdam& a,
                     hipStream_t s);

}  // namespace hss

#define HSS_HIP_CHECK(expr)                                                        \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) throw hss::Error(HSS_ERR_DEVICE, std::string(#expr) + ": " + \
                                           hipGetErrorString(_e));                 \
  } while (0)

namespace hss {
struct Error {
  hss_status code;
  std::string msg;
  Error(hss_status c, std::string m) : code(c), msg(std::move(m)) {}
};
}  // namespace hss
