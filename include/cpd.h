/*
 * cpd.h -- C ABI of libcpd: CSF-MTTKRP and sparse CP-ALS on one MI355X (gfx950).
 *
 * The operations follow "Parallel Sparse Tensor Decomposition in Chapel"
 * (Rolinger, Simon, Krieger; arXiv:1812.05961): CP-ALS of Algorithm 1
 * (Section III), whose MTTKRP is computed on one compressed sparse fiber (CSF)
 * tree per mode order (Section III), after the one-time sort of the nonzeros
 * (the "Sort" routine of Section V-B / Table III).
 *
 * Conventions for every entry point
 *   - Pointers documented as "device" are HIP device pointers (for example
 *     torch.Tensor.data_ptr() of a CUDA tensor); "host" pointers are CPU memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     GPU work of a call is ordered on that stream.  A call returns once its
 *     work is queued unless stated otherwise.
 *   - Calls return a cpd_status and never abort or throw.  On failure
 *     cpd_last_error() gives a message for the calling thread.
 *   - The caller owns every buffer it passes; the library never frees them.
 *     Objects the library creates (cpd_csf) are freed by their *_free call.
 *   - Tensors have 2..5 modes (CSF trees, MTTKRP, CP-ALS; the dense steps
 *     take up to CPD_MAX_MODES = 8 Gram matrices), each of length
 *     1..2^31-1, and 1..2^31-1 nonzeros; ranks are 1..64.  Indices are
 *     0-based int32.
 *   - Factor matrices are row-major: element (i, r) at ptr[i * ld + r].
 */
#ifndef CPD_H
#define CPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CPD_OK = 0,
    CPD_EINVAL = 1,        /* bad argument: sizes, ranges, indices, null pointers */
    CPD_ENOMEM = 2,        /* a device or host allocation failed */
    CPD_EHIP = 3,          /* a HIP runtime call failed */
    CPD_EUNSUPPORTED = 4   /* valid request this build does not handle */
} cpd_status;

/* Gather precision of the MTTKRP (factor rows read from HBM). */
enum { CPD_FP32 = 0, CPD_BF16_GATHER = 1 };

/* Conflict handling where output rows collide (Section V-D2: locks versus
 * privatised buffers).  On the GPU "atomic" replaces the paper's mutex pool.
 * PRIVATE (non-root modes only): every block keeps a copy of the output in LDS
 * when it fits 64 KiB, else each of the chip's eight XCDs adds into its own
 * HBM copy and the copies are summed into the output afterwards.  AUTO: no
 * copies at the root; below it the LDS copy iff
 * rows * 1024 <= 0.02 * nnz and it fits, else atomics (with the most frequent
 * output rows accumulated in LDS at levels >= 2). */
enum { CPD_VARIANT_AUTO = 0, CPD_VARIANT_ATOMIC = 1, CPD_VARIANT_PRIVATE = 2 };

/* Kernel family: AUTO picks (ROW above the leaf level, TILED at the leaf
 * level, LANE otherwise, each where eligible -- see cpd_mttkrp_plan -- and,
 * with CPD_VARIANT_AUTO, TILED at an internal level); ROW = groups of
 * lanes each holding 16-byte chunks of the factor rows, several leaves per
 * wave step (root and internal levels; tile widths in multiples of 32);
 * LANE = the rank spread over the lanes, one leaf per wave step (any level);
 * ROUND = leaf level only: a wave takes its leaves in rounds of 64, gathers
 * the rows of the round's fibers into LDS, then adds one row per leaf with
 * atomics issued back to back (tile widths rounded up to multiples of 64;
 * no privatised variant: CPD_VARIANT_PRIVATE with AUTO runs LANE);
 * TILED = any level below the root: the leaves regrouped by tiles of the
 * output mode's indices (the level's mode tiling, built on the first such
 * call and kept with the tree: 16 bytes per nonzero for 2..3 modes, 32 for
 * 4..5; inside a tile tree order at the leaf level, at an internal level
 * ordered by the other levels' indices, the largest dimension first); each
 * wave adds one row per leaf, the Hadamard product of the leaf's rows at the
 * other levels (gathered once per run of leaves that share them) scaled by
 * its value, into a private LDS copy of its tile's output rows and adds the
 * copy to the output once per tile; tile_nnz = the tile height in output
 * rows (0 = what 5 KiB of LDS per wave hold, at least 16), capped by the
 * LDS; no privatised variant, as ROUND. */
enum { CPD_KERNEL_AUTO = 0, CPD_KERNEL_ROW = 1, CPD_KERNEL_LANE = 2, CPD_KERNEL_ROUND = 3, CPD_KERNEL_TILED = 4 };

#define CPD_MAX_MODES 8
#define CPD_MAX_RANK 64

/* Last error message of the calling thread ("" if none). */
const char *cpd_last_error(void);

/* Test hook for the allocation-failure paths: from now on every device
 * allocation request of the library larger than `bytes` fails with
 * CPD_ENOMEM (cached scratch blocks included), as if the device were out of
 * memory; bytes < 0 removes the limit (the default).  Process-wide; always
 * CPD_OK. */
cpd_status cpd_set_alloc_limit(int64_t bytes);

/* ABI version of this library (incremented on incompatible changes). */
int32_t cpd_abi_version(void);

/* ---------------------------------------------------------------------------
 * CSF construction (Section III's compressed sparse fiber; the paper's "Sort"
 * preprocessing, Section V-C).
 *
 * Opaque handle to one CSF tree held in device memory owned by the library.
 * Level l (0 = root) of a tree with mode order `order` holds one node per
 * distinct index prefix (i_order[0], ..., i_order[l]) of the sorted nonzeros:
 *   fids[l]  int32, count[l] entries: index i_order[l] of each node;
 *   fptr[l]  int32, count[l]+1 entries (l < N-1): first child of each node at
 *            level l+1, and fptr[l][count[l]] = count[l+1];
 *   vals     float, count[N-1] entries: leaf values.
 * Nonzeros with equal coordinates are merged into one whose value is the
 * float32 sum of the duplicates in input order.
 */
typedef struct cpd_csf_s *cpd_csf;

/* Build a CSF from COO.
 *   nmodes  N in [2, 5] (CPD_EUNSUPPORTED for 6..8, CPD_EINVAL otherwise);
 *           dims: host, N lengths;  nnz in [1, 2^31-1].
 *   inds    host array of N device pointers, each nnz int32 indices.
 *   vals    device, nnz floats.
 *   order   host, a permutation of 0..N-1 (root first), or NULL for modes by
 *           ascending length, ties to the lower mode.
 *   out     receives the handle (NULL on failure).
 * Checks every index against its dim on the device (one 4-byte read back) and
 * reads the level counts back: the call waits for `stream` before returning.
 * CPD_EUNSUPPORTED when sum of ceil(log2 dims) exceeds 128 bits.
 * The input arrays are not modified and may be freed after the call. */
cpd_status cpd_csf_build(int32_t nmodes, const int64_t *dims, int64_t nnz,
                         const int32_t *const *inds, const float *vals, const int32_t *order,
                         void *stream, cpd_csf *out);

/* One tree rooted at each mode (the layout CP-ALS reads, every MTTKRP at the
 * root level, Section III): out[m] (host array of N handles) holds the tree
 * with order (m, then the other modes by descending length, ties to the lower
 * mode).  Each tree equals cpd_csf_build with that order.  The tree of the
 * longest mode is sorted on every key field; each other tree re-sorts those
 * sorted, merged nonzeros on its root field only (the order of the other
 * fields is already right for keys that share a root index).  Arguments and
 * checks as cpd_csf_build; on failure every out[m] is NULL. */
cpd_status cpd_csf_build_rooted(int32_t nmodes, const int64_t *dims, int64_t nnz,
                                const int32_t *const *inds, const float *vals, void *stream, cpd_csf *out);

/* Mode count, mode order (host, N entries) and level counts (host, N
 * entries; count[N-1] = nonzeros after merging).  Null outputs are skipped. */
cpd_status cpd_csf_info(cpd_csf csf, int32_t *nmodes, int32_t *order, int64_t *counts);

/* Copy level `level` to caller device buffers: fids (count[level] int32),
 * fptr (count[level]+1 int32, levels < N-1 only) and vals (count[N-1]
 * floats, leaf level only).  Null outputs are skipped. */
cpd_status cpd_csf_export(cpd_csf csf, int32_t level, int32_t *fids, int32_t *fptr, float *vals,
                          void *stream);

/* Work split of the MTTKRP kernels: the leaves are cut into tiles of
 * tile_nnz consecutive nonzeros, and for each tile t the node holding leaf
 * t*tile_nnz is found at every level l < N-1.  Writes starts[l * ntiles + t]
 * (device, (N-1) * ntiles int32, or NULL to only query) and *ntiles (host). */
cpd_status cpd_csf_tiles(cpd_csf csf, int32_t tile_nnz, int32_t *starts, int64_t *ntiles,
                         void *stream);

/* Free the handle and its device arrays (waits for work queued on them). */
void cpd_csf_free(cpd_csf csf);

/* ---------------------------------------------------------------------------
 * MTTKRP (the MTTKRP step of Algorithm 1: Y = X_(n) times the Khatri-Rao product
 * of the other factors), computed on the CSF tree, element-wise:
 *     Y(i, r) = sum over nonzeros with i_mode = i of x * prod_{m != mode} A_m(i_m, r).
 * `mode` may sit at any level of the tree (root, internal or leaf). */
typedef struct {
    int32_t precision;   /* CPD_FP32 or CPD_BF16_GATHER */
    int32_t variant;     /* CPD_VARIANT_* */
    int32_t kernel;      /* CPD_KERNEL_* */
    int32_t tile_nnz;    /* leaves per work unit; 0 = automatic */
} cpd_mttkrp_opts;

/* factors: host array of N device pointers (the entry for `mode` is not
 *          read); float rows for CPD_FP32, bfloat16 bits (uint16) for
 *          CPD_BF16_GATHER; row stride ld elements (ld >= rank).
 * out:     device, dims[mode] x rank floats with row stride ldo >= rank;
 *          overwritten (columns >= rank untouched).
 * opts:    NULL for defaults.
 * Uses a library-allocated workspace for CPD_VARIANT_PRIVATE with per-XCD
 * copies and for the first call with a new tile width. */
cpd_status cpd_mttkrp(cpd_csf csf, const void *const *factors, int32_t ld, int32_t rank,
                      int32_t mode, float *out, int32_t ldo, const cpd_mttkrp_opts *opts,
                      void *stream);

/* The allocation-free form of cpd_mttkrp, for callers that cannot allocate
 * device memory: code under stream capture, tight serving loops, hosts that
 * forbid hipMalloc.  Same arguments, result and kernels as cpd_mttkrp; every
 * temporary of the call (a tile table the tree has not cached for the width,
 * the leaf factor in frequency-rank order, the per-XCD output copies of
 * CPD_VARIANT_PRIVATE) is carved from one fixed device array of the library
 * (cpd_mttkrp_noalloc_workspace_bytes() bytes, 64 MiB), one copy per device,
 * held until the process ends; its device address is looked up once per
 * device, on the first call with that device current.  Internal-level hot-row
 * tables are used only when the tree already holds the level's ranking (a
 * cpd_mttkrp call has built it); otherwise that level runs with atomics alone.
 * Errors: as cpd_mttkrp, plus CPD_EUNSUPPORTED ("... workspace") when the
 * call's temporaries exceed the array; nothing is allocated either way.
 * Every call on a device shares that device's array and it keeps the last
 * call's contents (what must start at zero is cleared by a kernel in the
 * call): calls that overlap in time on one device, from several streams or
 * host threads, race and give wrong results; serialise them. */
size_t cpd_mttkrp_noalloc_workspace_bytes(void);
cpd_status cpd_mttkrp_noalloc(cpd_csf csf, const void *const *factors, int32_t ld, int32_t rank,
                              int32_t mode, float *out, int32_t ldo, const cpd_mttkrp_opts *opts,
                              void *stream);

/* The kernel family cpd_mttkrp runs for a request, by the rule it applies,
 * decided on the host without touching the device.
 *   nmodes         N (MTTKRP kernels exist for 2..5);
 *   dims_by_level  host, N lengths in tree order (dims[order[l]]);
 *   depth          level of the output mode (0 = root);
 *   ld, rank, precision, kernel: as for cpd_mttkrp (kernel = the request);
 *   rows_aligned   nonzero when every non-output factor starts 16-byte aligned;
 *   leaf_words     nonzero when the tree has leaf words (every leaf length
 *                  below 2^29, always so for trees cpd_csf_build makes).
 * ROW is eligible for 3..5 modes at non-leaf levels, when the padded rank
 * fits in ld and rows are 16-byte multiples below 16 MiB, and every gathered
 * level (all but `depth`) has fewer than 2^24 rows with rows * row bytes
 * <= 2^32 (its rows are addressed by 32-bit byte offsets).  ROUND is eligible
 * at the leaf level (depth N-1) when the tree has leaf words, ld is a multiple
 * of 4 and at least the rank rounded up to 4, and the factors are 16-byte
 * aligned; TILED under the same conditions at every level below the root.
 * AUTO picks ROW above the leaf level and TILED at the leaf level, each when
 * eligible, LANE otherwise (cpd_mttkrp runs LANE instead of ROUND or TILED
 * for CPD_VARIANT_PRIVATE, and TILED at an internal level with
 * CPD_VARIANT_AUTO; cpd_mttkrp_noalloc runs ROUND at the leaf level and the
 * shape rule's kernel at an internal level when the tree holds no tiling of
 * that height yet, and so does cpd_mttkrp with CPD_KERNEL_AUTO when the
 * device has no room for the tiling; TILED requested explicitly returns
 * CPD_ENOMEM then).
 * *kernel_out (host) = CPD_KERNEL_ROW, CPD_KERNEL_LANE, CPD_KERNEL_ROUND or
 * CPD_KERNEL_TILED; CPD_EUNSUPPORTED when ROW, ROUND or TILED is requested and
 * not eligible, or N is outside 2..5. */
cpd_status cpd_mttkrp_plan(int32_t nmodes, const int64_t *dims_by_level, int32_t depth, int32_t ld,
                           int32_t rank, int32_t precision, int32_t kernel, int32_t rows_aligned,
                           int32_t leaf_words, int32_t *kernel_out);

/* ---------------------------------------------------------------------------
 * Dense steps of Algorithm 1 (FP64 on the GPU). */

/* G = A^T A (the A^T A terms of Algorithm 1).
 * A: device, rows x rank floats, stride ld.  G: device, rank x rank doubles. */
cpd_status cpd_gram(const float *A, int64_t rows, int32_t rank, int32_t ld, double *G,
                    void *stream);

/* One mode update after its MTTKRP (the per-mode steps of Algorithm 1: V, solve, normalise):
 *   V = Hadamard product of grams[m] over m != mode;
 *   A = Y V^+, with V^+ = V^{-1} by symmetric Gauss-Jordan elimination when
 *       every pivot (the square of Cholesky's diagonal) exceeds
 *       rank*eps*max(diag V), else the Moore-Penrose inverse from a Jacobi
 *       eigendecomposition dropping eigenvalues <= rank*eps*max eigenvalue;
 *   lambda_r = 2-norm of column r of A; A(:, r) /= lambda_r when > 0.
 * grams:    host array of nmodes device pointers to rank x rank doubles.
 * Y:        device, rows x rank floats (stride ldy).
 * A:        device, rows x rank floats written (stride lda).
 * A_bf16:   device or NULL, rows x rank bfloat16 copy of A (stride ldb),
 *           round-to-nearest-even of the float values.
 * lambda:   device, rank doubles written.
 * G_new:    device or NULL, rank x rank doubles: A^T A of the written A.
 * used_pinv: device or NULL, one int32 set to 1 when the fallback ran, else 0. */
cpd_status cpd_solve_normalize(const double *const *grams, int32_t nmodes, int32_t mode,
                               const float *Y, int64_t rows, int32_t rank, int32_t ldy,
                               float *A, int32_t lda, uint16_t *A_bf16, int32_t ldb,
                               double *lambda, double *G_new, int32_t *used_pinv,
                               void *stream);

/* Fit of K = [[lambda; A_0..A_{N-1}]] (the fit step of Algorithm 1):
 *   fit = 1 - sqrt(max(0, normX2 - 2 <X,K> + ||K||^2)) / sqrt(normX2), with
 *   <X,K> = sum_r lambda_r sum_i A_last(i, r) Y_last(i, r) (Y_last = MTTKRP of
 *   the last mode with the other final factors) and
 *   ||K||^2 = lambda^T (Hadamard of all grams) lambda.
 * All pointers device except `grams` (host array of nmodes device pointers);
 * fit: one double written on the device. */
cpd_status cpd_fit(double normX2, const double *lambda, const float *A_last, int32_t lda,
                   const float *Y_last, int32_t ldy, int64_t rows, int32_t rank,
                   const double *const *grams, int32_t nmodes, double *fit, void *stream);

/* out (device, one double) = sum of squares of vals (device, n floats). */
cpd_status cpd_sumsq(const float *vals, int64_t n, double *out, void *stream);

/* ---------------------------------------------------------------------------
 * CP-ALS (Algorithm 1) from COO. */
typedef struct {
    int32_t precision;       /* CPD_FP32 or CPD_BF16_GATHER (MTTKRP gathers only;
                                the solve, norms and fit stay FP64) */
    int32_t variant;         /* CPD_VARIANT_* for every MTTKRP */
    int32_t kernel;          /* CPD_KERNEL_* */
    int32_t tile_nnz;        /* 0 = automatic */
    int32_t single_csf;      /* 0: one CSF per mode, rooted at that mode, the
                                other modes by descending length (the default:
                                every MTTKRP is a root-level one);
                                1: one CSF in `order` (or ascending lengths) */
    int32_t fast_fit;        /* 0 (default): after the last sweep the reported
                                fit is evaluated from one more MTTKRP of the last
                                mode with the final FP32 factors, FP64 products
                                and FP64 sums, so it is the fit of the returned
                                model to ~1e-8 also as the fit nears 1;
                                1: no extra pass with FP32 gathers (the last
                                sweep's fit, from its FP32 MTTKRP; near fit 1 it
                                is good to about sqrt(rel. error of that MTTKRP),
                                ~1e-3); with BF16 gathers the extra pass then uses
                                FP32 rows and FP32 sums */
    const int32_t *order;    /* host, N entries, or NULL (used with single_csf) */
    const float *const *init;/* host array of N device pointers to I_m x rank
                                floats (stride rank), or NULL: seeded U(0,1) */
    uint64_t seed;           /* seed of the U(0,1) initialisation */
    double *fit_trace;       /* host, max_iters doubles, or NULL */
    double *timing_ms;       /* host, 4 + max_iters*(N+1) doubles, or NULL:
                                [0] CSF build (with the selection, if any),
                                [1] all iterations, [2] final fit, [3] total;
                                then per iteration: N MTTKRP times and the
                                iteration time */
    int32_t select;          /* 0: as above; 1: per mode, the CSF order and
                                MTTKRP options cpd_select picks with the
                                network `selector_params`; 2: cpd_select's
                                fallback rule (one shared ascending tree).
                                With 1 or 2 the variant, kernel, tile_nnz,
                                single_csf and order fields are not used;
                                3..5 modes. */
    int32_t selector_hidden; /* hidden width of the network (select = 1) */
    const float *selector_params; /* device, the network's parameters (select = 1) */
} cpd_als_opts;

/* Run CP-ALS with `rank` components for at most max_iters sweeps; when tol > 0
 * stop from the second sweep on once |fit - previous fit| < tol (the per-sweep
 * fit, from that sweep's MTTKRP of the last mode; fit_trace holds these).
 * fit_out: the fit of the returned model (see fast_fit).
 * factors_out: host array of N device pointers, I_m x rank floats (stride
 *              rank), written with unit-norm columns.
 * lambda_out:  host, rank doubles.  fit_out, iters_out: host.
 * Waits for `stream` before returning. */
cpd_status cpd_als(int32_t nmodes, const int64_t *dims, int64_t nnz, const int32_t *const *inds,
                   const float *vals, int32_t rank, int32_t max_iters, double tol,
                   const cpd_als_opts *opts, float *const *factors_out, double *lambda_out,
                   double *fit_out, int32_t *iters_out, void *stream);

/* ---------------------------------------------------------------------------
 * CP with missing values (tensor completion; the paper lists it next to
 * least-squares CP among the CPD library's decompositions, Section III):
 * the nonzeros are the observed entries, every other entry is unknown.  Mode
 * by mode, row i of A_n solves (G_i + reg I) a = y_i with
 * G_i = sum over observed entries of row i of h h^T and y_i = sum of x h
 * (h: the Hadamard product of the other modes' rows of the entry; y is the
 * MTTKRP of the observed entries), and after each sweep the RMSE over the
 * observed entries is sqrt((sum x^2 - 2 sum_i a_i.y_i + sum_i a_i^T G_i a_i)
 * / n_obs) from the last mode.  No column weights; rows without observations
 * become zero.  reg must be > 0 (every row system is then positive definite).
 * ------------------------------------------------------------------------- */

/* Row Grams of `mode`, which must be the root of the tree (e.g. a tree of
 * cpd_csf_build_rooted): G (device, dims[mode] x rank x rank doubles,
 * row-major per row) is zeroed, then G[i][r][c] for r <= c receives
 * sum over row i's entries of h_r h_c, products formed in FP64 from the FP32
 * factors (host array of N device pointers, row stride ld >= rank; the
 * root's entry is not read).  Entries below the diagonal are left zero.
 * FP64 atomics: the summation order varies between calls.  3..5 modes, leaf
 * indices below 2^29. */
cpd_status cpd_row_gram(cpd_csf csf, const float *const *factors, int64_t ld, int32_t rank, int32_t mode,
                        double *G, void *stream);

/* For each of `rows` rows: solve (G_i + reg I) a = y_i (G as cpd_row_gram
 * writes it, only r <= c read; Y device rows x ldy floats) by Gauss-Jordan in
 * FP64 and write a to A (device rows x lda floats, columns < rank).  terms:
 * device, 2 doubles receiving sum_i a_i.y_i and sum_i a_i^T G_i a_i, or NULL.
 * CPD_EINVAL unless reg > 0. */
cpd_status cpd_row_solve(const double *G, const float *Y, int64_t ldy, int64_t rows, int32_t rank, double reg,
                         float *A, int64_t lda, double *terms, void *stream);

/* Completion ALS from COO (arguments of cpd_csf_build; duplicates are merged
 * by summing), `rank` components, at most max_iters sweeps (stop from the
 * second on once the RMSE changes by less than tol > 0).  factors: host array
 * of N device pointers to I_m x rank floats (stride rank): the initial values
 * (factor 0 is not read: mode 0 is solved first), overwritten with the
 * result.  rmse: host, max_iters doubles (the RMSE after each sweep; the last
 * one evaluated once more for the returned factors from an MTTKRP of the last
 * mode with FP64 products and sums, accurate to ~1e-8 of the data's scale also
 * as the RMSE nears 0), or NULL.
 * iters: host, sweeps run.  3..5 modes.  Waits for `stream`. */
cpd_status cpd_complete(int32_t nmodes, const int64_t *dims, int64_t nnz, const int32_t *const *inds,
                        const float *vals, int32_t rank, int32_t max_iters, double tol, double reg,
                        float *const *factors, double *rmse, int32_t *iters, void *stream);

/* ---------------------------------------------------------------------------
 * Variant selector.  Section V-D2 of the paper settles the lock-or-privatise
 * question by a rule on the output length, the thread count and the nonzero
 * count, and observes that the better choice depends on the tensor.  Here a
 * small network predicts the MTTKRP time of every candidate (CSF mode order,
 * conflict handling, tile width) from tensor statistics, and the candidate
 * with the smallest prediction is taken.  Without a network the fallback is
 * that rule on the tree in ascending-length order. */

/* Per-mode statistics of a COO tensor from a strided sample of its nonzeros. */
typedef struct {
    int32_t nmodes;
    int32_t reserved;
    int64_t nnz;
    int64_t sample;                   /* nonzeros in the sample (<= 2^20) */
    int64_t dims[CPD_MAX_MODES];
    double top1[CPD_MAX_MODES];       /* share of the sample at the most frequent index */
    double distinct[CPD_MAX_MODES];   /* distinct sampled indices / min(dim, sample) */
    double alpha[CPD_MAX_MODES];      /* cpd_zipf_alpha(top1, dim) */
} cpd_stats;

/* Fill *out for a COO tensor (arguments as in cpd_csf_build; indices are not
 * range-checked here).  Sorts a sample of each mode's indices on the device;
 * waits for `stream` before returning. */
cpd_status cpd_tensor_stats(int32_t nmodes, const int64_t *dims, int64_t nnz,
                            const int32_t *const *inds, void *stream, cpd_stats *out);

/* The exponent a >= 0 of a Zipf law p_k proportional to k^-a over dim items
 * whose largest probability 1/sum_k k^-a equals top1 (0 when top1 <= 1/dim;
 * capped at 8).  Host only. */
double cpd_zipf_alpha(double top1, int64_t dim);

/* CSF mode orders a candidate can use for MTTKRP of mode n: all modes by
 * ascending length (ties to the lower mode); n first then the rest ascending;
 * the rest ascending then n last; all by descending length; n first then the
 * rest by descending length (the trees cpd_als builds by default). */
enum { CPD_ORDER_ASC = 0, CPD_ORDER_FIRST = 1, CPD_ORDER_LAST = 2, CPD_ORDER_DESC = 3, CPD_ORDER_ROOTED = 4,
       CPD_ORDER_KINDS = 5 };

typedef struct {
    int32_t order_kind;              /* CPD_ORDER_* */
    int32_t depth;                   /* level of the mode in `order` */
    int32_t order[CPD_MAX_MODES];    /* the CSF mode order (nmodes entries) */
    cpd_mttkrp_opts opts;            /* precision CPD_FP32; variant, kernel, tile */
} cpd_choice;

#define CPD_SEL_MAX_CAND 24
#define CPD_SEL_NFEAT 43

/* Candidates for MTTKRP of `mode` at `rank` (3..5 modes): every distinct
 * order of the five kinds; at the root the ROW kernel with tile widths 32,
 * 128, 512 (or atomic LANE with 64, 256, 1024 when the tree exceeds the ROW
 * kernels' index limits); at internal levels ROW without and with the LDS
 * table of hot rows (atomic, private) and atomic LANE, tile 256, and TILED
 * (default tile height); at the leaf
 * level TILED (default tile height), ROUND with tile widths 64, 256, 1024 and
 * atomic LANE, tile 256; below the root also privatised LANE (tile 256) when
 * dims[mode] * rank * 4 <= 64 KiB.
 * out: host, CPD_SEL_MAX_CAND entries; *n receives the count.
 * Factor rows are assumed padded as cpd_als pads them (stride a multiple of
 * 4 floats, at least the rank rounded up to 8/16/32/36/64). */
cpd_status cpd_select_candidates(const cpd_stats *st, int32_t rank, int32_t mode,
                                 cpd_choice *out, int32_t *n);

/* Network inputs of n candidates: feat (host, n x CPD_SEL_NFEAT floats,
 * row-major) from the statistics, the rank, the mode and each candidate. */
cpd_status cpd_select_features(const cpd_stats *st, int32_t rank, int32_t mode,
                               const cpd_choice *cand, int32_t n, float *feat);

/* The fallback: ascending-length order; below the root privatised LANE iff
 * dims[mode] * 1024 (the private copies) <= 0.02 * nnz and the copy fits in
 * 64 KiB of LDS (the rule of Section V-D2), else atomics with the level's
 * default kernel (ROW at internal levels, TILED at the leaf level); default
 * tile widths (root 128, internal 256, TILED its default).  Always one of
 * the candidates. */
cpd_status cpd_select_heuristic(const cpd_stats *st, int32_t rank, int32_t mode, cpd_choice *out);

/* Pick the candidate with the smallest predicted time.
 * params: device, cpd_mlp_param_count(CPD_SEL_NFEAT, hidden) floats of a
 *         trained network, or NULL for the fallback.
 * out:    host, the choice.  pred (host, CPD_SEL_MAX_CAND floats) and ncand
 *         (host) receive the predictions and the candidate count when not
 *         NULL (ncand = 0 for the fallback).
 * Waits for `stream` before returning. */
cpd_status cpd_select(const cpd_stats *st, int32_t rank, int32_t mode, const float *params,
                      int32_t hidden, cpd_choice *out, float *pred, int32_t *ncand, void *stream);

/* ---------------------------------------------------------------------------
 * The selector's network: in -> hidden -> hidden -> 1 with ReLU after the
 * first two layers (hidden <= 64, in <= 4096), float32, mean squared error,
 * Adam updates (Kingma and Ba, ICLR 2015).  Parameters are one flat device
 * array: W1 (hidden x in, row-major), b1 (hidden), W2 (hidden x hidden), b2
 * (hidden), W3 (hidden), b3 (1). */

/* Number of parameters (0 for a bad shape). */
int64_t cpd_mlp_param_count(int32_t n_in, int32_t hidden);

/* He-normal weights (standard deviation sqrt(2 / fan-in)) from a seeded
 * counter-based generator, zero biases.  params: device. */
cpd_status cpd_mlp_init(float *params, int32_t n_in, int32_t hidden, uint64_t seed, void *stream);

/* out[b] = f(X[b]) for batch rows of X (device, batch x n_in). out: device. */
cpd_status cpd_mlp_forward(const float *params, int32_t n_in, int32_t hidden, const float *X,
                           int64_t batch, float *out, void *stream);

/* loss = mean_b (f(X[b]) - y[b])^2 and its gradient with respect to every
 * parameter (back-propagation; batch sums in batch order).  All device:
 * X batch x n_in, y batch, loss one float (or NULL), grad param_count floats. */
cpd_status cpd_mlp_loss_grad(const float *params, int32_t n_in, int32_t hidden, const float *X,
                             const float *y, int64_t batch, float *loss, float *grad, void *stream);

/* One Adam step (step >= 1) on count parameters: m and v (device, count
 * floats each) are the moment estimates, updated in place. */
cpd_status cpd_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t count,
                        float lr, float beta1, float beta2, float eps, int32_t step, void *stream);

/* Mini-batch training for `epochs` passes over n samples (X device n x n_in,
 * y device n), shuffled each epoch by a seeded host generator, Adam with
 * beta1 0.9, beta2 0.999, eps 1e-8 from zero moments.  loss_trace: host,
 * epochs floats (mean batch loss per epoch), or NULL.  Waits for `stream`. */
cpd_status cpd_mlp_train(float *params, int32_t n_in, int32_t hidden, const float *X,
                         const float *y, int64_t n, int32_t epochs, int32_t batch, float lr,
                         uint64_t seed, float *loss_trace, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CPD_H */
