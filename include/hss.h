/*
 * hss.h - adaptive randomized HSS compression on AMD MI355X (gfx950).
 *
 * C ABI of libhss.so.  The method is the one of Gorman, Chavez, Ghysels,
 * Mary, Rouet and Li, "Matrix-free construction of HSS representation
 * using adaptive randomized sampling" (arXiv 1810.04125):
 *   - random sampling S^r = A R, S^c = A^T R and element extraction
 *     A(I,J) (Sec. 2.2 eq. sample_off_diag; Sec. 4.1 partially matrix-free
 *     interface): entries generated on the GPU for the built-in operator
 *     families, or caller routines for both (HSS_FAM_CALLBACK);
 *   - bottom-up interpolative decompositions of the local samples
 *     (eqs. ID, QRCPSr; Alg. 1 and 2);
 *   - the adaptive driver (Alg. 3) with the doubling (Alg. 4, with the
 *     HMT-scaled RRQR of eq. RRQRHMTstop) and incrementing (Alg. 5, block
 *     Gram-Schmidt with eq. stopping_criteria) strategies.
 *
 * Conventions for every call:
 *   - every function returns hss_status; HSS_OK = 0, positive values are
 *     warnings with valid outputs, negative values are errors after which
 *     no output is valid and every resource of the call has been freed;
 *     hss_last_error() gives a thread-local message for the last non-OK
 *     status;
 *   - "device" pointers are HIP device memory of the current device,
 *     "host" pointers are ordinary host memory; ownership of every pointer
 *     argument stays with the caller, which must keep it valid for the
 *     duration of the call (asynchronous calls: until the stream reaches
 *     the work);
 *   - matrices are column-major with an explicit leading dimension unless
 *     stated otherwise; indices are 0-based;
 *   - real arithmetic only: the paper's conjugate transpose is the
 *     transpose.
 */
#ifndef HSS_H
#define HSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HSS_OK = 0,
  HSS_NOT_CONVERGED = 1,               /* d reached d_max; open nodes were accepted as they stood */
  HSS_TOL_BELOW_SAMPLING_PRECISION = 2,/* thresholds raised to the sampling precision floor */
  HSS_ERR_INVALID_ARG = -1,
  HSS_ERR_OUT_OF_MEMORY = -2,
  HSS_ERR_DEVICE = -3,                 /* a HIP runtime call failed */
  HSS_ERR_CALLBACK = -4,               /* a caller routine of HSS_FAM_CALLBACK returned non-zero */
  HSS_ERR_NONFINITE = -5,              /* a non-finite sample or entry was met */
  HSS_ERR_INTERNAL = -6,
  HSS_ERR_SINGULAR = -7                /* hss_factor met a zero pivot */
} hss_status;

/* Operator families whose entries the kernels generate on the fly. */
typedef enum {
  HSS_FAM_TOEPLITZ = 0, /* symmetric Toeplitz: t(0)=pi^2/(6h^2), t(k)=(-1)^k/(k^2 h^2) */
  HSS_FAM_LAPLACE = 1,  /* 1/(4 pi |x_i-x_j|) for i != j, `diag` on the diagonal */
  HSS_FAM_GAUSS = 2,    /* exp(-|x_i-x_j|^2/(2 sigma^2)) + diag * delta_ij */
  HSS_FAM_DENSE = 3,    /* explicit n x n matrix in device memory (read from HBM) */
  HSS_FAM_CALLBACK = 4  /* caller routines for the products and the entries (below) */
} hss_family;

/* Partially matrix-free operator (Sec. 4.1): the method needs only the
 * products with random blocks and selected sub-blocks of A, so a caller
 * with a fast product (sparse, low-rank, FFT-based, another hierarchical
 * matrix) supplies two routines instead of the entries.
 *
 * Both routines work in the PERMUTED order of the tree (A_hat(i, j) =
 * a(perm[i], perm[j])), on device memory of the current device, with
 * column-major blocks.  They are called from the thread that called the
 * library, with `stream` the stream of the call: they may enqueue their
 * work asynchronously on it (the library orders its own work behind
 * theirs on that stream) or finish it before they return.  A non-zero
 * return aborts the call with HSS_ERR_CALLBACK; nothing they wrote is
 * used.  `ctx` is the generator's ctx, passed through.
 *
 * hss_sample_fn: Sr = A_hat R and Sc = A_hat^T R for the n x ncols block
 *   R (leading dimension ldr); Sr and Sc have leading dimension lds.
 *   Either output may be NULL and is then not wanted (Sc is always NULL
 *   when the generator is symmetric).  Called once per sampling step with
 *   the new columns only.
 *
 * hss_extract_fn: out_k(a, b) = A_hat(I_k[a], J_k[b]) for every block k
 *   of `blocks` (a host array of nblocks entries, valid during the call).
 *   The blocks of one call are all the sub-blocks one tree level needs in
 *   a sampling round (the diagonal blocks D of its leaves and the
 *   couplings B12, B21 of its nodes whose children have just compressed),
 *   gathered so that the caller can serve them together (Sec. 4.2:
 *   extraction synchronized per level). */
typedef struct {
  int32_t nI, nJ;
  const int64_t* I;   /* device, nI permuted row positions */
  const int64_t* J;   /* device, nJ permuted column positions */
  double* out;        /* device, nI x nJ, column-major */
  int64_t ldo;        /* leading dimension of out, >= max(nI, 1) */
} hss_block;

typedef int32_t (*hss_sample_fn)(void* ctx, int64_t n, int32_t ncols, const double* R, int64_t ldr,
                                 double* Sr, double* Sc, int64_t lds, void* stream);
typedef int32_t (*hss_extract_fn)(void* ctx, int32_t nblocks, const hss_block* blocks, void* stream);

/* Sample-growth strategy and stopping test (Alg. 3-5). */
typedef enum {
  HSS_DBL_FNORM = 0, /* doubling, block Gram-Schmidt F-norm test (eq. stopping_criteria) */
  HSS_INC_FNORM = 1, /* incrementing by delta_d, same test (Alg. 5) */
  HSS_DBL_HMT = 2,   /* doubling, RRQR with the HMT factor, accept iff r < d - p (Alg. 4) */
  HSS_INC_HMT = 3    /* incrementing by delta_d, test of eq. HMT_IQQH (Sec. 3.1, Lemma 4.1 of
                        Halko, Martinsson and Tropp): a side passes when hmt_alpha sqrt(2/pi)
                        times the largest 2-norm of the newest block's columns projected off
                        the basis of the earlier blocks is <= eta*atol/level; absolute
                        tolerance only (rtol is not used, by the test or by the ID) */
} hss_strategy;

/* Arithmetic of the sampling product A R (the ID and the tests stay FP64). */
typedef enum {
  HSS_SAMPLE_FP64 = 0,
  HSS_SAMPLE_FP32 = 1,   /* FP32 MFMA, FP32 accumulation per K chunk, FP64 chunk sums */
  HSS_SAMPLE_BF16X3 = 2  /* bf16 hi/lo split, three bf16 MFMA products, FP32 accumulation */
} hss_precision;

/* Operator description.  All pointers are device pointers in the ORIGINAL
 * (unpermuted) index order; the library applies the tree permutation.
 *   toeplitz: h (grid step)
 *   laplace : points (n x 3, xyz interleaved, row-major), diag (A_ii)
 *   gauss   : points, sigma, diag
 *   dense   : dense (column-major, leading dimension ld >= n); symmetric
 *             tells whether A = A^T may be assumed (then S^c = S^r)
 *   callback: sample, extract, ctx; symmetric as for dense.  The
 *             routines receive PERMUTED positions, so the tree's
 *             permutation is the caller's to apply. */
typedef struct {
  int32_t family;
  int32_t symmetric;
  int64_t n;
  double h;
  double sigma;
  double diag;
  const double* points;
  const double* dense;
  int64_t ld;
  hss_sample_fn sample;
  hss_extract_fn extract;
  void* ctx;
} hss_generator;

/* Cluster tree (Sec. 2.1): binary, numbered level by level top-down from
 * 0 at the root, every node owns the contiguous permuted range [lo, hi),
 * children partition their parent.  Host memory; leaves have
 * left = right = -1, the root has parent = -1.  perm[i] is the original
 * index at permuted position i. */
typedef struct {
  int64_t n;
  int32_t num_nodes;
  int64_t* perm;
  int32_t* lo;
  int32_t* hi;
  int32_t* left;
  int32_t* right;
  int32_t* parent;
  int32_t* level;
} hss_tree;

/* Build a cluster tree on the host.  points_host: n x 3 row-major, or
 * NULL for index bisection.  method: 0 index bisection, 1 recursive
 * coordinate bisection (split the axis of largest extent), 2 kd (axis =
 * depth mod 3).  A node with m > leaf_size indices splits into floor(m/2)
 * and the rest, points ordered by (coordinate, original index); indices
 * inside a leaf ascend.  The tree is owned by the caller: free it with
 * hss_tree_free. */
hss_status hss_tree_build(int64_t n, const double* points_host, int32_t leaf_size,
                          int32_t method, hss_tree** out);
void hss_tree_free(hss_tree* tree);

/* Learned start of the incrementing strategy (not part of the paper's
 * method; see the predictor network calls below).  With
 * options.predictor set, hss_compress first runs the network on one
 * feature row per tree level of the problem (family one-hot; 0.5 log2 of
 * the kernel parameter, h for Toeplitz or sigma for the Gaussian kernel,
 * 0 for Laplace; (log2 n - 14)/3; level/8; (log2 of the level's mean node
 * size - 10)/4; (-log10 rtol - 6)/2) and takes d0 = the predicted final
 * sample count 2^y (output 1 of the root row) rounded to the nearest
 * multiple of delta_d, within [delta_d, min(d_max, n)].  The stopping tests still
 * decide every node: a low prediction costs rounds, a high one samples.
 * The prediction also sizes the compression's sample capacity (its
 * device memory grows with it): twice the predicted count rounded up to a
 * multiple of delta_d, at least d0 + 4 delta_d, at most d_max.  A run
 * that reaches that capacity with its root still open is restarted from
 * scratch with options.d_max, starting from the capacity it reached (its
 * statistics are those of the restarted run).
 * Only for HSS_FAM_TOEPLITZ, HSS_FAM_LAPLACE and HSS_FAM_GAUSS with the
 * incrementing strategies; options.d0 is then ignored. */
#define HSS_MLP_MAX_LAYERS 6
#define HSS_MLP_MAX_WIDTH 128
typedef struct {
  int32_t n_layers;                        /* 1 .. HSS_MLP_MAX_LAYERS */
  int32_t sizes[HSS_MLP_MAX_LAYERS + 1];   /* each 1 .. HSS_MLP_MAX_WIDTH */
} hss_mlp;
typedef struct {
  hss_mlp net;             /* sizes[0] = 8 inputs, sizes[n_layers] = 2 outputs */
  const float* params;     /* device, hss_mlp_num_params floats (layout below) */
} hss_predictor;

/* Device memory from the caller (e.g. a framework's caching allocator).
 * alloc returns `bytes` of device memory usable on `stream`, or NULL when
 * it cannot (the call then fails with HSS_ERR_OUT_OF_MEMORY and frees
 * what it took); free gives back a block alloc returned, on the stream it
 * was used on.  Both run on the calling thread, during hss_compress /
 * hss_compress_batched (the compression's working memory, freed when it
 * ends) and during hss_matvec (its temporaries) and hss_destroy (the
 * generators the handle keeps).  The functions and ctx must stay valid
 * until the handle is destroyed.  alloc = NULL: the library allocates
 * itself (hipMallocAsync, plus one cached block per device for the
 * compression's working memory; see hss_release_cache). */
typedef struct {
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* p, void* stream);
  void* ctx;
} hss_allocator;

/* Launch-shape tunables (not part of the method): the workgroup counts
 * the grouped GEMMs (gemm_wg, at most gemm_max_split K slices) and the
 * sampling product (sample_wg) split K to reach, and the workgroup target
 * of the one-step pivot kernels (qrcp_wg, 64 .. HSS_QRCP_WG_MAX).  Results
 * depend on them only through the order of floating-point sums. */
#define HSS_QRCP_WG_MAX 4096
typedef struct {
  int32_t gemm_wg;
  int32_t gemm_max_split;
  int32_t sample_wg;
  int32_t qrcp_wg;
} hss_tunables;

/* The built-in tunables. */
hss_status hss_default_tunables(hss_tunables* out);
/* Load a tunables table (the autotuner, python -m
 * paper_1810_04125_amd.autotune, writes one): text lines
 *   arch family precision n_lo n_hi gemm_wg gemm_max_split sample_wg qrcp_wg
 * (arch as the device reports it, e.g. gfx950; family and precision as
 * the hss_family / hss_precision numbers; '#' starts a comment).  A
 * compression takes the first line that matches its device, the family
 * and precision of its first problem and n_lo <= n < n_hi of that
 * problem, else the defaults.  path NULL or "" clears the table.  Without a
 * call, the first compression loads the file named by the environment
 * variable HSS_TUNE_FILE, if set.  Host only; errors in the file return
 * HSS_ERR_INVALID_ARG and leave the table unchanged. */
hss_status hss_load_tunables(const char* path);
/* The tunables a compression with this key would take. */
hss_status hss_lookup_tunables(const char* arch, int32_t family, int32_t precision, int64_t n,
                               hss_tunables* out);

/* Options of one compression (Alg. 3).
 *   rtol, atol : relative / absolute tolerance; every node tau uses
 *                eta*rtol/level(tau) and eta*atol/level(tau)
 *   eta        : global safety factor on the per-node tolerance (1 = literal)
 *   d0         : initial number of random vectors
 *   delta_d    : increment (HSS_INC_FNORM, HSS_INC_HMT)
 *   oversample_p : p of the HMT acceptance r < d - p (HSS_DBL_HMT)
 *   hmt_alpha  : alpha of eq. HMT_IQQH (HSS_INC_HMT; 0 = 10): the bound holds
 *                except with probability alpha^-p, p = delta_d
 *   d_max      : cap on the number of random vectors; min(d_max, n) <= HSS_MAX_D,
 *                <= ncols_R when R is given
 *   R, ldr, ncols_R : device, the n x ncols_R Gaussian matrix the method
 *                draws from, rows in PERMUTED order; columns are consumed
 *                left to right and never regenerated.  R = NULL: the
 *                library draws the columns itself on the device, each
 *                round only the new ones, from the counter-based generator
 *                of hss_random_normal with `seed` (ldr and ncols_R unused)
 *   stream     : hipStream_t for all work (NULL = default stream)
 *   seed       : key of the generated R (used only when R is NULL)
 *   predictor  : learned d0 (hss_predictor above), or NULL
 *   allocator  : device memory from the caller (hss_allocator above); all
 *                problems of a batched call take the first one's */
typedef struct {
  double rtol;
  double atol;
  double eta;
  int32_t strategy;
  int32_t d0;
  int32_t delta_d;
  int32_t oversample_p;
  int32_t d_max;
  int32_t sample_precision;
  const double* R;
  int64_t ldr;
  int32_t ncols_R;
  int32_t profile;   /* 1: time every kernel launch with HIP events (slower; see hss_get_kernel_stats) */
  void* stream;
  double hmt_alpha;
  uint64_t seed;
  const hss_predictor* predictor;   /* host struct, NULL = off: learned d0 (above) */
  hss_allocator allocator;          /* alloc = NULL: the library's own */
} hss_options;

/* Largest sample count of a compression: a pivot step of the ID keeps its
 * Householder vector (one double per sample) in the 160 KB of LDS of a
 * compute unit. */
#define HSS_MAX_D 16384

typedef struct hss_matrix hss_matrix;

/* Adaptive HSS compression (Alg. 3): returns the generators D, U, V
 * (as skeleton indices J and interpolation matrices E), B12, B21 of every
 * node.  Host-synchronous: one small device-to-host copy per sampling
 * round decides whether to sample more.  Returns HSS_NOT_CONVERGED
 * (a warning) when d reached d_max before the root compressed. */
hss_status hss_compress(const hss_generator* gen, const hss_tree* tree,
                        const hss_options* opt, hss_matrix** out);

/* `count` independent compressions run together: every kernel launch
 * covers the same tree level of all problems of a group, and each round
 * samples every open problem before the tree pass (Sec. 4,
 * level-synchronised traversal).  Problems are taken in order into groups
 * whose estimated device memory fits in min(60% of the free HBM, 80 GiB); groups run
 * one after the other.  gens, trees, opts and out are arrays of length
 * count; all options must use the same strategy and the same stream.
 * The sampling time in hss_info is that of the problem's group. */
hss_status hss_compress_batched(int32_t count, const hss_generator* gens,
                                const hss_tree* const* trees, const hss_options* opts,
                                hss_matrix** out);

void hss_destroy(hss_matrix* h);

/* Y = H X for nrhs right-hand sides, X and Y device, ORIGINAL ordering,
 * asynchronous on `stream`: the call returns once the work is queued; its
 * temporaries are stream-ordered allocations freed behind it on `stream`.
 * Upward pass x_hat = V^T x, top-down sibling couplings through B12/B21 and
 * the nested bases (eq. nestedUV).  Calls on one hss_matrix share its task
 * arrays: issue them on one stream (calls on different streams race). */
hss_status hss_matvec(const hss_matrix* h, int32_t nrhs, const double* X, int64_t ldx,
                      double* Y, int64_t ldy, void* stream);

/* Direct factorization of the compressed matrix for hss_solve (the ULV
 * factorization column of the paper's table sixdrivers; the paper gives no
 * algorithm, this one follows from the interpolative bases of Sec. 2.2).
 * Per node, in the order [redundant; skeleton] of its local rows and
 * columns, the transforms [[I, -E^T], [0, I]] of its row and column bases
 * leave the redundant unknowns coupled to the node's own block only; an LU
 * with partial pivoting (pivots among the redundant rows) eliminates them,
 * and the skeleton Schur complements join into the parent's block with
 * B12 and B21; the root's block is factored whole.  Needs equal row and
 * column ranks at every node (every symmetric family gives them):
 * HSS_ERR_INVALID_ARG otherwise; HSS_ERR_SINGULAR on a zero pivot.  The
 * factor (about 8 (sum over nodes of m^2) bytes, m = a leaf's size or the
 * children's summed ranks) stays with h until hss_destroy; a second call
 * returns at once.  Runs on the stream h was compressed on and returns when
 * it is done. */
hss_status hss_factor(hss_matrix* h);

/* X = H^{-1} B for nrhs right-hand sides, B and X device (n x nrhs,
 * column-major, leading dimensions >= n), ORIGINAL ordering, after
 * hss_factor (HSS_ERR_INVALID_ARG before).  Bottom-up the row transforms
 * and the forward substitutions with each node's pivots and L pass the
 * skeleton part of the right-hand side to the parent; top-down the
 * skeleton unknowns from the parent give the redundant ones (back
 * substitution with U) and x = T_c^T xhat.  The call waits for the work
 * already queued on `stream`, uploads its task arrays, and returns with the
 * solve queued on `stream`; its temporaries are stream-ordered. */
hss_status hss_solve(const hss_matrix* h, int32_t nrhs, const double* B, int64_t ldb, double* X,
                     int64_t ldx, void* stream);

/* hss_matvec for callers that cannot allocate device memory during the call
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the same product, Y = H X in ORIGINAL ordering, asynchronous
 * on `stream`, with every temporary in one fixed device array of
 * HSS_NOALLOC_SCRATCH_BYTES that the library holds per GPU until the
 * process ends (the caller still passes X and Y).  The temporaries need
 * 8 (2 n + 2 S_r + S_m) nrhs bytes, each part rounded up to 256 bytes,
 * where S_r and S_m are the matrix's summed rank and row capacities
 * (about 7.6 MB per right-hand side for n = 32768, leaf 128): calls that
 * need more return HSS_ERR_INVALID_ARG with the size in the message.
 * Every call on one GPU shares that GPU's array and overwrites it: calls
 * that overlap on one GPU (different streams, or threads) race; serialize
 * them, e.g. on one stream.  Call it with the device that holds h current. */
#define HSS_NOALLOC_SCRATCH_BYTES (64u << 20)
hss_status hss_matvec_noalloc(const hss_matrix* h, int32_t nrhs, const double* X, int64_t ldx,
                              double* Y, int64_t ldy, void* stream);

/* ||A - H||_F / ||A||_F over all n^2 entries (the error measure of
 * table HMT), in FP64, by column blocks of H and generated blocks of A.
 * gen may be NULL for the built-in families (the compression keeps their
 * tables); for HSS_FAM_CALLBACK it must describe the compressed operator,
 * whose sample routine then yields the column blocks A_hat [e_j ...].
 * Host-synchronous. */
hss_status hss_rel_error(const hss_matrix* h, const hss_generator* gen, double* rel_err);

typedef struct {
  int64_t n;
  int32_t num_nodes;
  int32_t rounds;      /* passes over the tree */
  int32_t d_final;     /* random vectors used */
  int32_t hss_rank;    /* max node rank */
  int32_t status;      /* hss_status of the compression */
  int32_t symmetric;   /* 1 if only S^r was computed (S^c = S^r) */
  double sample_ms;    /* summed HIP-event time of the sampling launches */
  double total_ms;     /* wall time of hss_compress */
  double sample_flops; /* 2 n^2 d_final per product computed */
  int32_t d0;          /* initial sample count used (the predictor's when one was given) */
  int32_t pad;
  double d_predicted;  /* the predictor's final sample count (0 without one) */
} hss_info;

hss_status hss_get_info(const hss_matrix* h, hss_info* out);

/* Per kernel class of the job that produced h: launches, GPU time
 * (summed HIP-event time around each launch, only when the compression
 * ran with options.profile = 1, else 0) and the algorithmic bytes and
 * flops the launches had to move / perform by their definition:
 *   SAMPLE       k_sample_f64 / k_sample_lp: 2 n^2 c flops, 16 n c + 24 n bytes
 *                per c sampled columns
 *   SAMPLE_REDUCE  fixed-order sum of split-K sampling partials
 *   EXTRACT      k_extract_nodes: 8 bytes per generated entry
 *   GATHER       copies of local samples / reduced random matrices: 16 bytes per entry
 *   GEMM         k_gemm_grouped (+ its split-K sum): 2 M N K flops,
 *                8 (MK + KN + MN [+ MN if accumulating]) bytes
 *   TEST_NORMS   k_fn_norms, k_cq_chol, k_fn_rtest: F-norm tests of the
 *                projected block (m x b, 16 m b bytes, 4 m b flops), its
 *                Cholesky factors and the R-diagonal tests
 *   QRCP_STEP    k_qrcp_step, one Householder step (pivoted for the ID, plain
 *                for the stopping test) on the (d-k) x (m-k-1) trailing
 *                panel: 16 (d-k)(m-k-1) bytes, 4 (d-k)(m-k-1) flops
 *   QRCP_OTHER   plan, copy-in, liveness and finish kernels of the factorizations
 *   TRSM         k_trsm_diag: diagonal blocks of the back substitution for E
 *   MISC         per-level bookkeeping kernels
 *   QRCP_WG      k_qrcp_wg: whole factorizations of small panels, per step as
 *                QRCP_STEP
 *   QFORM        k_qf_prep, k_qf_solve, k_qform: explicit Q_k of the stopping
 *                test (compact WY form; its GEMMs count as GEMM)
 *   RNG          k_randn: the new columns of R when the library draws them
 *                (8 bytes written per entry)
 *   TEST_QR      Householder steps of the stopping test's QR of the projected
 *                block (no pivoting), counted as QRCP_STEP; QRCP_STEP then
 *                holds the pivot steps of the ID only
 *   ID           totals of the interpolative decompositions as the method
 *                defines their work, whatever kernels ran them: per factored
 *                d x m panel of rank r, 8 d m + 8 r (m - r) bytes (the panel
 *                read once, E written) and 4 d m r flops; launches = ID calls
 *                (one per level and side with a node to factor), ms = 0 */
enum {
  HSS_K_SAMPLE = 0, HSS_K_SAMPLE_REDUCE = 1, HSS_K_EXTRACT = 2, HSS_K_GATHER = 3, HSS_K_GEMM = 4,
  HSS_K_TEST_NORMS = 5, HSS_K_QRCP_STEP = 6, HSS_K_QRCP_OTHER = 7, HSS_K_TRSM = 8, HSS_K_MISC = 9,
  HSS_K_QRCP_WG = 10, HSS_K_QFORM = 11, HSS_K_RNG = 12, HSS_K_TEST_QR = 13, HSS_K_ID = 14,
  HSS_K_COUNT = 15
};
typedef struct {
  int64_t launches;
  double ms;
  double bytes;
  double flops;
} hss_kernel_stats;
hss_status hss_get_kernel_stats(const hss_matrix* h, int32_t kclass, hss_kernel_stats* out);

typedef struct {
  int32_t state;   /* 0 UNTOUCHED, 1 PARTIALLY_COMPRESSED, 2 COMPRESSED */
  int32_t is_leaf;
  int32_t lo, hi;
  int32_t m_r, m_c;       /* rows of the local samples tau.S^r, tau.S^c */
  int32_t rank_r, rank_c; /* columns of U_tau, V_tau */
  int32_t b_rows, b_cols; /* B12 is b_rows x b_cols (non-leaf); B21 is b_cols' x b_rows' */
} hss_node_info;

hss_status hss_get_node_info(const hss_matrix* h, int32_t node, hss_node_info* out);

/* Copy one generator of a node to host memory.  Layouts:
 *   HSS_NODE_D    : leaf, (hi-lo)^2 doubles, column-major
 *   HSS_NODE_B12  : rank_r(left) x rank_c(right), column-major
 *   HSS_NODE_B21  : rank_r(right) x rank_c(left), column-major
 *   HSS_NODE_JR / HSS_NODE_JC : m int32, pivot order: the first rank
 *                   entries are J, the rest ascend (U(J,:) = I)
 *   HSS_NODE_ER / HSS_NODE_EC : rank x (m - rank), column-major; U(rest,:) = E^T
 *   HSS_NODE_IR / HSS_NODE_IC : rank int64 skeleton indices (permuted)
 * bytes must be at least the size of the object. */
enum {
  HSS_NODE_D = 0, HSS_NODE_B12 = 1, HSS_NODE_B21 = 2, HSS_NODE_JR = 3, HSS_NODE_JC = 4,
  HSS_NODE_ER = 5, HSS_NODE_EC = 6, HSS_NODE_IR = 7, HSS_NODE_IC = 8
};
hss_status hss_copy_node(const hss_matrix* h, int32_t node, int32_t what, void* host_dst,
                         size_t bytes);

/* --- individual hot-path steps, for testing and for callers that build
 *     their own driver --------------------------------------------------- */

/* S = op(A_hat) R for ncols columns, A_hat(i,j) = a(perm[i], perm[j]),
 * op = identity (transpose = 0, S^r) or transpose (1, S^c) (Sec. 2.2
 * eq. sample_off_diag).  perm: device int64[n], checked on the host to be a
 * permutation of [0, n) (HSS_ERR_INVALID_ARG otherwise).  R, S: device, n x ncols,
 * column-major.  precision: hss_precision.  Host-synchronous (the call
 * returns when S is complete).  HSS_FAM_CALLBACK forwards to gen->sample
 * (FP64 only; perm is not used, the routine works in permuted order). */
hss_status hss_sample(const hss_generator* gen, const int64_t* perm, int32_t ncols,
                      const double* R, int64_t ldr, double* S, int64_t lds, int32_t transpose,
                      int32_t precision, void* stream);

/* out = A_hat(I, J), nI x nJ column-major (ldo >= nI); I, J device int64
 * permuted indices (Sec. 4.1: B = A(J^r, J^c) is a sub-block of A).  perm,
 * I and J are checked on the host (a permutation; indices in [0, n)).
 * HSS_FAM_CALLBACK forwards one block to gen->extract (perm not used). */
hss_status hss_extract(const hss_generator* gen, const int64_t* perm, int32_t nI,
                       const int64_t* I, int32_t nJ, const int64_t* J, double* out,
                       int64_t ldo, void* stream);

/* Batched interpolative decomposition (eqs. ID, QRCPSr): for each of
 * `count` matrices S_k (m_k x d_k, device, ROW-major with leading
 * dimension ld_k, i.e. S_k^T column-major), QR with column pivoting of
 * S_k^T that stops before the first pivot with residual norm
 * <= max(eps_a, eps_r * nu_1).  Outputs per matrix: rank[k];
 * piv_k (int32[m_k], pivot order then the rest ascending);
 * E_k (rank x (m_k - rank), column-major, leading dimension m_k).
 * Host arrays: m, d, ld, offsets (in elements) into S, piv, E.
 * Host-synchronous (ranks are returned in host memory). */
hss_status hss_interpolative_batched(int32_t count, const int32_t* m, const int32_t* d,
                                     const int64_t* ld, const double* S, const int64_t* s_off,
                                     double eps_r, double eps_a, int32_t* piv,
                                     const int64_t* piv_off, double* E, const int64_t* e_off,
                                     int32_t* rank_host);

/* Columns c0 .. c0+ncols-1 of the Gaussian matrix R that hss_compress draws
 * when options.R is NULL (Alg. 3: R-bar = randn(N, delta_d) in every
 * round), into R (device, n x ncols column-major, leading dimension
 * ldr >= n; output column t holds column c0 + t).  Entry (i, j), i a
 * PERMUTED row, depends on (seed, i, j) only:
 *   - Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011) of the counter
 *     (i >> 2, j, 0, 0) under the key (seed, 0) gives words w0..w3 for the
 *     rows 4q .. 4q+3, q = i >> 2;
 *   - u_t = ((w_t >> 11) + 1) 2^-53 in (0, 1];
 *   - Box-Muller in FP64: rows 4q, 4q+1 get sqrt(-2 log u0) cos(2 pi u1) and
 *     sqrt(-2 log u0) sin(2 pi u1), rows 4q+2, 4q+3 the same of (u2, u3),
 *     with 2 pi the nearest double, multiplied into u before cos and sin.
 * Asynchronous on `stream`.  n >= 1, c0 >= 0, ncols >= 0. */
hss_status hss_random_normal(int64_t n, int32_t c0, int32_t ncols, uint64_t seed, double* R, int64_t ldr,
                             void* stream);

/* The raw Philox words behind hss_random_normal: W(i, t) = word (i & 3) of
 * the counter (i >> 2, c0 + t, 0, 0) (device, n x ncols column-major,
 * leading dimension ldw >= n).  Asynchronous on `stream`. */
hss_status hss_random_words(int64_t n, int32_t c0, int32_t ncols, uint64_t seed, uint64_t* W, int64_t ldw,
                            void* stream);

/* Free the device memory the library keeps between compressions on the
 * current device.  The transient buffers of a compression (local samples,
 * bases, level workspaces; sized from d_max) come from one block per
 * device that is kept after the call and reused by the next compression
 * that fits in it; hss_compress_batched counts it as free memory when it
 * forms groups.  Call this to give that memory back (for example before
 * allocating elsewhere).  Blocks held by a running compression stay. */
hss_status hss_release_cache(void);

/* --- learned rank / d0 predictor ----------------------------------------
 * Not part of the paper's method: the adaptive driver (Alg. 3) needs an
 * initial sample count d0 and, with the incrementing strategy (Alg. 5),
 * pays one round of sampling, stopping tests and IDs per increment between
 * d0 and the final d.  A small network fed with features that are known
 * before any sampling (family, kernel parameter, n, tree level, node size,
 * tolerance) predicts per-level node ranks and the final d, so d0 can start
 * close to it.  The stopping tests of the compression still decide: a low
 * prediction only costs extra rounds, a high one extra sample columns.
 *
 * The network is a fully connected ReLU net in FP32: layer l maps
 * sizes[l] -> sizes[l+1], ReLU after every layer but the last.  Parameters
 * are one device float array, for each layer W_l (sizes[l+1] x sizes[l],
 * ROW-major) followed by b_l (sizes[l+1]).  Samples are ROW-major: X is
 * n x sizes[0], Y, T (targets) and M (0/1 masks) are n x sizes[n_layers].
 * Loss: sum(M (Y - T)^2) / max(1, sum M); Adam as Kingma and Ba (2015). */
/* (hss_mlp and HSS_MLP_MAX_* are defined above, with hss_predictor.) */

/* Number of parameters (floats) of the network, to host *out. */
hss_status hss_mlp_num_params(const hss_mlp* net, int64_t* out);

/* Y = net(X) for n samples; device pointers; asynchronous on `stream`. */
hss_status hss_mlp_forward(const hss_mlp* net, const float* params, const float* X, int64_t n,
                           float* Y, void* stream);

/* grad (device, num_params floats) = dLoss/dparams over the n samples, and
 * the loss to *loss_dev (device float, may be NULL).  Partial gradients of
 * 32-sample tiles are summed in tile order, so the result is deterministic.
 * Allocates a stream-ordered workspace of about (n/32) * num_params floats;
 * asynchronous on `stream`. */
hss_status hss_mlp_gradient(const hss_mlp* net, const float* params, const float* X,
                            const float* T, const float* M, int64_t n, float* grad,
                            float* loss_dev, void* stream);

/* One Adam step, in place on params, m, v (device, np floats each); step is
 * the 1-based step count used in the bias corrections. */
hss_status hss_mlp_adam(int64_t np, float* params, const float* grad, float* m, float* v,
                        float lr, float beta1, float beta2, float eps, int64_t step,
                        void* stream);

/* Mini-batch Adam training, all on the device: `epochs` passes over the n
 * samples, each in an order given by the affine permutation
 * i -> (a i + c) mod n with a coprime to n, a and c drawn from `seed` and
 * the epoch number; batches of `batch` consecutive positions (the last one
 * ragged).  *step (host, in/out) is the Adam step count.  loss_host (host,
 * `epochs` floats, may be NULL) receives the mean batch loss of each
 * epoch.  Host-synchronous. */
hss_status hss_mlp_train(const hss_mlp* net, float* params, float* m, float* v, int64_t* step,
                         const float* X, const float* T, const float* M, int64_t n,
                         int32_t batch, int32_t epochs, float lr, uint64_t seed,
                         float* loss_host, void* stream);

const char* hss_last_error(void);
const char* hss_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HSS_H */
