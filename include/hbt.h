/*
 * hbt.h - C ABI of the Householder-aligned permutation test on AMD MI355X.
 *
 * The test compares the dispersion ("semantic breadth") of two clouds of
 * l2-normalised vectors X (n x d) and Y (m x d) (paper Sec. 3.1, "Problem
 * setting"; Algorithm 1 inputs).  It
 *   1. computes the sample mean directions mu_x, mu_y in FP64 (Sec. 3.1,
 *      "Householder mean-direction alignment"; Algorithm 1, Step 1);
 *   2. reflects X with H = I - 2 v v^T / (v^T v), v = mu_x - mu_y, so that
 *      H mu_x = mu_y, leaving Y unchanged (Eq. for u and H; eq:householder_fast);
 *   3. computes T_obs = log v(X') - log v(Y) with v = 1 / g_d(r) and r the
 *      mean resultant length (Sec. 3.1, "Dispersion proxy"; eq:tobs);
 *   4. pools Z = [X'; Y], draws B random splits into sizes (n, m), and
 *      counts splits with T_b >= T_obs (Sec. 3.1, "Permutation procedure";
 *      Algorithm 1, Step 5; Algorithm 2 for the group sums as one product);
 *   5. returns p = (1 + count) / (B + 1) (eq:pvalue).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers on the current HIP device unless
 *     stated otherwise, row-major, owned by the caller.  The library never
 *     allocates device memory: scratch space is the caller's workspace
 *     (`ws`, `ws_bytes`), sized by the matching *_workspace_size call.
 *   - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued on
 *     it and the call returns without synchronising; results are valid once
 *     the stream reaches that point.
 *   - Host-detectable errors return a non-zero hbt_status BEFORE anything is
 *     enqueued.  Conditions found on the device (degenerate clouds, bad
 *     explicit masks) are reported per pair in hbt_result.status.  HIP
 *     failures return HBT_ERR_DEVICE.  hbt_last_error() gives a thread-local
 *     message for the last non-OK return.  No C++ exception crosses the ABI.
 *   - Inputs must have unit-norm rows (the paper normalises every embedding,
 *     Sec. 3.1 Eq. 2).  They are not renormalised: every call tests each row
 *     as it sums the columns, and a pair with a row whose norm is off by more
 *     than 1e-4 gets the per-pair status HBT_ERR_NOT_UNIT (a pair whose mean
 *     resultant length is outside (0, 1) gets HBT_ERR_DEGENERATE first).
 *
 * Random splits.  Split b (a global index, perm_offset <= b < perm_offset+B)
 * of pair `pair_index` under `seed` puts in group 1 the n items that come
 * first in the order (P_i, S_i, i), where P_i is byte (i mod 4) of word
 * (i mod 16)/4 of Philox4x32-10(counter (i/16, b, pair_index, 0), key seed)
 * and S_i is word (i mod 4) of Philox4x32-10(counter (i/4, b, pair_index, 1),
 * key seed); the key is (seed mod 2^32, seed >> 32).  Masks store bit
 * (i mod 32) of word i/32 for item i, ceil(N/32) words per split.
 */
#ifndef HBT_H_
#define HBT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HBT_ABI_VERSION 2
#define HBT_MAX_N 65536     /* largest pooled size n + m */
#define HBT_MAX_D 8192      /* largest dimension */

typedef enum hbt_status {
    HBT_OK = 0,
    HBT_ERR_ARG = 1,          /* NULL pointer, bad enum, offset overflow */
    HBT_ERR_SIZE = 2,         /* n < 2, m < 2, d < 1, B < 1, or above the limits */
    HBT_ERR_DTYPE = 3,        /* unsupported input dtype / precision combination */
    HBT_ERR_WORKSPACE = 4,    /* ws NULL or ws_bytes below the required size */
    HBT_ERR_DEGENERATE = 5,   /* per pair: r_X or r_Y outside (0, 1); H = I used */
    HBT_ERR_MASK = 6,         /* per pair: an explicit mask row does not hold n items */
    HBT_ERR_DEVICE = 7,       /* a HIP call failed */
    HBT_ERR_UNSUPPORTED = 8,  /* option not built */
    HBT_ERR_INTERNAL = 9,     /* per pair: split selection overflowed its bucket buffer */
    HBT_ERR_NOT_UNIT = 10     /* per pair: some row of X or Y has | |x| - 1 | > 1e-4 (or is
                                 NaN); the test assumes l2-normalised rows (Sec. 3.1, Eq. 2),
                                 and the pair's other results are not meaningful */
} hbt_status;

typedef enum hbt_precision {
    HBT_F64 = 0,      /* group sums on FP64 MFMA */
    HBT_F32 = 1,      /* group sums on FP32 MFMA */
    HBT_BF16X2 = 2,   /* z = hi + lo split into two BF16 planes, FP32 accumulation */
    HBT_I8X3 = 3,     /* z rounded to 21-bit fixed point (z * 2^20), three balanced
                         int8 digit planes on the int8 MFMA: exact integer group
                         sums, FP64 epilogue; the 8-bit-operand variant of the
                         group-sum product (route 0 only) */
    HBT_BF16_E4M3 = 4, /* the split-BF16 hi plane plus lo = z - hi as FP8 e4m3 (of
                         lo * 2^17, round to nearest even): bf16 MFMA for hi, the
                         E8M0-scaled fp8 MFMA for lo, one FP32 accumulator; the
                         mask stays exact (route 0, split rows of FP32 or FP64) */
    HBT_BF16_LAZY = 5 /* the split-BF16 planes, with the lo plane multiplied only
                         where it can change a decision: the group sums of every
                         split from the hi plane alone (one BF16 product, the
                         half-precision GEMM of Sec. 3.2, practical note 1);
                         splits whose T_b lies within that product's error band
                         of the threshold (every split of a pair with
                         min(n, m) < 16) get the split-BF16 product of both
                         planes, then the FP64 recheck as usual.  Counts and p
                         are those of the FP64 statistic, as for the other
                         precisions; T_b (and t_mean, t_sd) carry the hi plane's
                         error outside the band.  hbt_perm_test,
                         hbt_perm_test_static and hbt_perm_test_batched; route 0 */
} hbt_precision;

typedef enum hbt_dtype { HBT_IN_F32 = 0, HBT_IN_F64 = 1 } hbt_dtype;

/* g_d of Sec. 3.1 ("Dispersion proxy"): the paper uses "the same estimator as
 * in prior work" without writing it; BANERJEE is the vMF concentration
 * estimate kappa = r (d - r^2) / (1 - r^2) (Banerjee et al., JMLR 2005). */
typedef enum hbt_gd { HBT_GD_BANERJEE = 0, HBT_GD_IDENTITY = 1 } hbt_gd;

/* GREATER: count T_b >= T_obs ("u broader than k", Sec. 3.1).
 * TWO_SIDED: count |T_b| >= |T_obs| (Table 5 reports two-sided values). */
typedef enum hbt_alternative { HBT_ALT_GREATER = 0, HBT_ALT_TWO_SIDED = 1 } hbt_alternative;

/* Per-pair result, written to DEVICE memory (112 bytes). */
typedef struct hbt_result {
    double t_obs;        /* log v(X') - log v(Y), FP64 (eq:tobs) */
    double r_x;          /* mean resultant length of X (= of X', H orthogonal) */
    double r_y;          /* mean resultant length of Y */
    double p;            /* (1 + count) / (B + 1) (eq:pvalue) */
    double tau;          /* tie tolerance: T_b counts if T_b >= T_obs - tau */
    double mu_cos;       /* cosine of the angle between the unit mean directions,
                            1 - |mu_x - mu_y|^2 / 2 (Sec. 3.1) */
    double t_mean;       /* mean of the B permuted statistics T_b */
    double t_sd;         /* their standard deviation (divisor B); both use the final
                            T_b (FP64 for rechecked splits) and are NaN if any T_b is */
    int64_t count;       /* exceedances among the B splits */
    int64_t B;           /* splits evaluated */
    int64_t n_recheck;   /* splits re-evaluated in FP64 because T_b was near T_obs */
    int64_t n, m;        /* group sizes of the pair */
    int32_t status;      /* hbt_status of this pair */
    int32_t h_identity;  /* 1 when H = I (alignment off, or |v| <= 1e-12) */
} hbt_result;            /* 112 bytes */

/* Parameters of one test (96 bytes; host memory). */
typedef struct hbt_perm_params {
    int64_t n, m, d;        /* group sizes and dimension */
    int64_t B;              /* number of random splits */
    uint64_t seed;          /* Philox key */
    uint64_t perm_offset;   /* global index of the first split (resume / sharding);
                               perm_offset + B <= 2^32, else HBT_ERR_ARG */
    uint32_t pair_index;    /* Philox counter word 2 */
    int32_t precision;      /* hbt_precision */
    int32_t input_dtype;    /* hbt_dtype of X and Y */
    int32_t gd;             /* hbt_gd */
    int32_t alternative;    /* hbt_alternative */
    int32_t align;          /* 1 = Householder alignment (the paper), 0 = naive test */
    int32_t stat_route;     /* 0 = norms of the group sums; 1 = point-to-centroid products */
    int32_t flags;          /* HBT_FLAG_* bits */
    int64_t block_perms;    /* splits per block (B0 of Algorithm 2); 0 = automatic.
                               Results do not depend on it. */
    const uint32_t* masks;  /* optional DEVICE B x ceil((n+m)/32) group-1 masks replacing
                               the Philox splits; each row must hold exactly n items. */
} hbt_perm_params;

/* flags: skip the FP64 recheck (counts then follow the chosen precision alone) */
#define HBT_FLAG_NO_RECHECK 1
/* flags: T_out of hbt_perm_test is a double array (B doubles) instead of floats */
#define HBT_FLAG_T_OUT_F64 2
/* flags: T_out of hbt_perm_test holds 3 doubles per split: T_b and the squared
 * norms |sigma_1|^2, |sigma_2|^2 of the two group sums it came from (the
 * output of the group-sum product, before any FP64 recheck; a diagnostic of
 * each stage's error) */
#define HBT_FLAG_T_OUT_NORMS 4

int32_t hbt_abi_version(void);
const char* hbt_status_string(int32_t status);
const char* hbt_last_error(void);

/* hbt_align: Steps 1-4 of Algorithm 1 (mean directions in FP64, Householder
 * reflection of X onto Y's mean direction, T_obs).
 *   X (n x d), Y (m x d): unit rows, dtype input_dtype.
 *   X_out (n x d, same dtype): receives H x_i; may alias X.
 *   v_out (d doubles, nullable): receives v = mu_x - mu_y.
 *   result (device, one hbt_result): t_obs, r_x, r_y, tau, mu_cos, n, m,
 *   status, h_identity; p, t_mean, t_sd, count, B and n_recheck are set to 0.
 * Errors: HBT_ERR_ARG (NULL X/Y/X_out/result, bad enum), HBT_ERR_SIZE,
 * HBT_ERR_WORKSPACE, HBT_ERR_DEVICE. */
size_t hbt_align_workspace_size(int64_t n, int64_t m, int64_t d);
hbt_status hbt_align(int32_t input_dtype, const void* X, int64_t n, const void* Y, int64_t m,
                     int64_t d, int32_t align, int32_t gd, void* X_out, double* v_out,
                     hbt_result* result, void* ws, size_t ws_bytes, void* stream);

/* hbt_perm_test: the whole test for one pair (Algorithm 1; the group sums of
 * all splits of a block are one product of the 0/1 split masks with Z, as in
 * Algorithm 2 and eq:gemm).
 *   X (n x d), Y (m x d): unit rows, dtype prm->input_dtype.
 *   result: one device hbt_result.
 *   T_out (nullable, device, B floats; B doubles with HBT_FLAG_T_OUT_F64;
 *     B x 3 doubles (T_b, |sigma_1|^2, |sigma_2|^2) with HBT_FLAG_T_OUT_NORMS):
 *     T_b as computed by the chosen precision (before any FP64 recheck;
 *     HBT_BF16_LAZY: by the hi plane, or by split BF16 for the splits its
 *     first pass could not decide).
 *   mask_out (nullable, device, B x ceil((n+m)/32) words): the splits used.
 * Errors: as hbt_align, plus HBT_ERR_DTYPE and HBT_ERR_UNSUPPORTED;
 * HBT_ERR_SIZE when one block of splits (block_perms) would need more
 * group-sum tiles than 32-bit tile numbers hold (blocks of billions of
 * splits at a large d). */
size_t hbt_perm_test_workspace_size(const hbt_perm_params* prm);
hbt_status hbt_perm_test(const void* X, const void* Y, const hbt_perm_params* prm,
                         hbt_result* result, float* T_out, uint32_t* mask_out, void* ws,
                         size_t ws_bytes, void* stream);

/* hbt_perm_test_batched: many independent pairs in one sequence of launches.
 *   Z_all (device, FP32 or FP64 per common->input_dtype): rows X_0, Y_0,
 *     X_1, Y_1, ..., each d wide; pair p's X starts at row row_offset[p] and
 *     its Y at row_offset[p] + n[p].  The call cannot see Z_all's length:
 *     the caller guarantees row_offset[p] + n[p] + m[p] <= its row count
 *     (the Python binding checks it); a negative offset is HBT_ERR_ARG.
 *   row_offset, n, m, B: HOST arrays of npairs int64 (row_offset may have
 *     npairs + 1 entries; only the first npairs are read).
 *   pair_index: HOST array of npairs Philox counter words, or NULL for
 *     common->pair_index + p.  Pairs with equal n, m, B and pair index get
 *     identical splits (the reuse of one block of random splits across pairs
 *     of equal sizes, Sec. 3.2 practical notes): the call draws them once and
 *     those pairs share the masks.  Distinct indices give independent splits.
 *     hbt_perm_test_batched_workspace_size takes no indices and returns the
 *     size for distinct ones, which also covers shared ones.
 *   common: precision, input_dtype, gd, alternative, align, seed,
 *     perm_offset, flags (n, m, d, B, masks and block_perms are ignored).
 *   results: DEVICE array of npairs hbt_result.
 * Errors: as hbt_perm_test; a pair with bad sizes fails the whole call;
 * HBT_ERR_SIZE also when the call's group-sum tiles would not fit 32-bit
 * tile numbers (only near the size limits, e.g. thousands of pairs of 2^20
 * splits at d = 8192; split the batch). */
size_t hbt_perm_test_batched_workspace_size(int64_t npairs, const int64_t* n, const int64_t* m,
                                            const int64_t* B, int64_t d,
                                            const hbt_perm_params* common);
hbt_status hbt_perm_test_batched(int64_t npairs, const void* Z_all, const int64_t* row_offset,
                                 const int64_t* n, const int64_t* m, const int64_t* B,
                                 const uint32_t* pair_index, int64_t d,
                                 const hbt_perm_params* common, hbt_result* results, void* ws,
                                 size_t ws_bytes, void* stream);

/* hbt_perm_test_clouds: many pairs over a set of clouds that pairs share
 * (e.g. every pair of one word with others: the word's cloud is one of
 * them), each cloud stored once.  The permutation test of Algorithm 1 for
 * every pair, as hbt_perm_test_batched computes it, with the Householder
 * reflection (eq:householder_fast) folded into the statistic instead of
 * applied to the stored rows: the group-sum product runs on the unreflected
 * rows of both clouds, and per split the reflected group sums follow as
 *   sigma' = sigma - c v,  c = sum over the smaller group's X rows of
 *   2 (v . x_i) / (v . v)  (FP64, from the split mask),
 *   |sigma'|^2 = |sigma|^2 - 2 c (v . sigma) + c^2 (v . v),
 *   |t - sigma'|^2 = |t - sigma|^2 + 2 c (v . t - v . sigma) + c^2 (v . v),
 * whose error is 2 sigma' . E + |E|^2 for the product's error E, as without
 * the fold, whatever v . v is.
 *   Z_all (device, FP32): the clouds' rows; cloud c is cloud_rows[c] rows
 *     from row cloud_offset[c] (host arrays of nclouds int64), every cloud
 *     starting on a 16-byte boundary.  The caller guarantees the rows exist.
 *   pair_x, pair_y (host, npairs int64): the clouds of pair p (X, Y); B, and
 *     pair_index (nullable), as in hbt_perm_test_batched.
 *   common: precision must be HBT_BF16X2, input_dtype HBT_IN_F32,
 *     stat_route 0; gd, alternative, align, seed, perm_offset, flags apply.
 *   d: a multiple of 4, at most 1024.
 *   results: DEVICE array of npairs hbt_result.
 * The splits, counts and p-values are those of the same pairs in
 * hbt_perm_test_batched (counts follow the FP64 statistic through the same
 * recheck band).
 * Errors: HBT_ERR_ARG (NULL, cloud index out of range, negative offset),
 * HBT_ERR_SIZE, HBT_ERR_UNSUPPORTED (other precisions, dtypes, routes, d or
 * alignment), HBT_ERR_WORKSPACE, HBT_ERR_DEVICE. */
size_t hbt_perm_test_clouds_workspace_size(int64_t nclouds, const int64_t* cloud_rows, int64_t npairs,
                                           const int64_t* pair_x, const int64_t* pair_y, const int64_t* B,
                                           int64_t d, const hbt_perm_params* common);
hbt_status hbt_perm_test_clouds(int64_t nclouds, const void* Z_all, const int64_t* cloud_offset,
                                const int64_t* cloud_rows, int64_t npairs, const int64_t* pair_x,
                                const int64_t* pair_y, const int64_t* B, const uint32_t* pair_index, int64_t d,
                                const hbt_perm_params* common, hbt_result* results, void* ws, size_t ws_bytes,
                                void* stream);

/* hbt_pipeline_chunks: how many chunks of pairs the batched call pipelines
 * (the product of one chunk runs while the next is aligned and split, on
 * three streams joined by events; split BF16 and int8 planes with FP32 rows,
 * d a multiple of 4 and at most 1024, 16-byte aligned rows; other calls run
 * as one chunk).  chunks = 1 turns the pipeline off, 0 returns to the tuned
 * value (default 1); *previous (nullable) receives the setting it replaces.  Process-wide,
 * for later calls, overriding the tuned value; results do not depend on it.
 * Errors: HBT_ERR_ARG (chunks outside [0, 64]). */
hbt_status hbt_pipeline_chunks(int32_t chunks, int32_t* previous);

/* The FP64 recheck spreads its work in one of two ways, with the same bits:
 * the flags of a pair whose segment sums fit the workspace's slots become
 * one work item per flag and 512-row segment, the others one work item per
 * flag over all segments.  The environment variable
 * HBT_RECHECK_SLOTS (a count, read by every call) caps the slots a call
 * uses, 0 sending every flag down the second way; results do not depend on
 * it. */

/* hbt_recheck_band: the half-width *eps (host double) of the band around the
 * decision threshold inside which a split's T_b, computed by `precision` and
 * `stat_route`, is re-evaluated in FP64 (the count follows the FP64 statistic
 * of Algorithm 1 Step 5 that way), for a split whose groups of n and m items
 * have mean resultant lengths r1 and r2 (Sec. 3.1, "Dispersion proxy").  For
 * HBT_BF16_LAZY it is the band of the first, hi-plane product, inside which a
 * split goes to the split-BF16 product (whose band is HBT_BF16X2's).  The
 * band bounds |T_b - T_b(FP64)|: the storage error of the rows, which may add
 * up coherently over repeated rows, the accumulation error of the product,
 * and for stat_route 1 the FP32 point-to-centroid products.  Host function,
 * nothing is enqueued.
 * Errors: HBT_ERR_ARG (NULL eps, bad enum), HBT_ERR_SIZE (n, m < 1, d outside
 * [1, HBT_MAX_D]). */
hbt_status hbt_recheck_band(int32_t precision, int32_t stat_route, int32_t gd, int64_t n, int64_t m,
                            int64_t d, double r1, double r2, double* eps);

/* hbt_perm_test_static: hbt_perm_test for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and results as hbt_perm_test
 * without ws / ws_bytes: the workspace is a static device array inside the
 * library, HBT_STATIC_SCRATCH_BYTES per device (64 MiB; enough for one pair
 * of n + m = 5000 at d = 1024 with B = 20,000), held by every device the
 * library runs on until the process ends.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine); the first call on a
 * device looks up that device's scratch address.  Calls on one device share
 * the scratch: calls that overlap in time on one device (two streams, two
 * host threads) race and must be serialised by the caller; each call
 * initialises what it reads from the scratch.
 * Errors: as hbt_perm_test; HBT_ERR_WORKSPACE when the test needs more than
 * HBT_STATIC_SCRATCH_BYTES (hbt_perm_test_workspace_size tells). */
#define HBT_STATIC_SCRATCH_BYTES (64u << 20)
hbt_status hbt_perm_test_static(const void* X, const void* Y, const hbt_perm_params* prm,
                                hbt_result* result, float* T_out, uint32_t* mask_out, void* stream);

/* Stage timing, a profiling aid.  hbt_stage_timing(1) clears the record and
 * makes every later call record a pair of HIP events around each of its
 * stages on its stream; hbt_stage_timing(0) stops recording.
 * hbt_stage_times() waits for the recorded events, writes the summed
 * milliseconds (ms) and the number of timed launches (launches) of each stage
 * (HBT_NUM_STAGES entries each, host memory) and clears the record.
 * Errors: HBT_ERR_ARG (NULL outputs), HBT_ERR_DEVICE. */
typedef enum hbt_stage {
    HBT_STAGE_ALIGN = 0,     /* column sums, finalize, reflection + storage */
    HBT_STAGE_SPLIT = 1,     /* Philox split masks */
    HBT_STAGE_GROUPSUM = 2,  /* group-sum product (eq:gemm) with norm epilogue */
    HBT_STAGE_STAT = 3,      /* permuted statistics and exceedance counts */
    HBT_STAGE_RECHECK = 4,   /* FP64 re-evaluation near the threshold */
    HBT_STAGE_OTHER = 5,     /* table uploads, zero fills, p-values */
    HBT_STAGE_CENTROID = 6,  /* point-to-centroid products (statistic route 1) */
    HBT_NUM_STAGES = 7
} hbt_stage;
hbt_status hbt_stage_timing(int32_t enable);
hbt_status hbt_stage_times(double* ms, int64_t* launches);

/* Tuned launch parameters (the batching of Sec. 3.2's practical notes over
 * many pairs), one entry per (precision, d padded to 64):
 *   cost[2]     per-split costs of the two tile widths of the split-BF16
 *               product: a work-group covers 64 columns of Z and 1024
 *               splits of one pair (eight waves) or 256 (four waves).  Every
 *               call picks, per pair (per block for hbt_perm_test), the
 *               width w minimising cost_w * round_up(B, w); until tuned
 *               cost_1024 = 1 and cost_256 = 1.15.  A single-pair call takes
 *               the narrow width when its block's wide tiles would number
 *               fewer than two per compute unit (one pair must fill the GPU).
 *   grid_wide   work-groups per compute unit of the persistent 1024-split
 *               launch (default 16);
 *   grid_narrow the same for the 256-split split-BF16 launch (default 32) or
 *               the int8-plane launch (default 16);
 *   split_cap   split-stage work-groups per compute unit while it runs
 *               beside the alignment (default 6);
 *   chunks      pipeline chunks of the batched call (default 1; see
 *               hbt_pipeline_chunks).
 * No result depends on any of them.
 *   hbt_tune_batched: measures them on the caller's workload (split BF16,
 *     BF16 + e4m3 or int8 planes, common->precision; the lazy split-BF16
 *     precision uses the split-BF16 entry) with HIP events, every candidate
 *     twice keeping the faster: the widths (every pair forced to each;
 *     cost_w = product time / sum_p round_up(B_p, w) round_up(n_p + m_p,
 *     128)), then the grids of the launches the workload uses (wide 4, 8,
 *     16, 32; narrow 8, 16, 32, 64; by product time), then split_cap (4, 5,
 *     6, 8) and chunks (1, 2, 4) by whole-call time.  About 30 calls of
 *     hbt_perm_test_batched on its arguments; it synchronises the stream,
 *     clears the stage-timing record, installs the entry and leaves the
 *     results of a last call with the chosen parameters in `results`.  When
 *     the environment variable HBT_TUNE_CACHE names a file, the tuned
 *     entries are written to it (JSON), and the library reads it on first
 *     use in every process.
 *   hbt_tune_entry_get / hbt_tune_entry_set: one entry (tuned = 1 once
 *     measured, set or loaded).  HBT_BF16_LAZY has no entry of its own (it
 *     runs on the HBT_BF16X2 one) and is refused with HBT_ERR_ARG.
 *   hbt_tune_get / hbt_tune_set: only the split-BF16 costs of dimension d
 *     (costs[0] for width 1024, costs[1] for 256).
 *   hbt_tune_save / hbt_tune_load: every tuned entry to / from a JSON file
 *     (the format HBT_TUNE_CACHE uses); a malformed file changes nothing.
 *   hbt_tile_widths: the split-BF16 widths (host, npairs entries) a call
 *     with these per-pair B would use at dimension d.
 * Errors: HBT_ERR_ARG (bad pointer, precision, value or file), HBT_ERR_SIZE,
 * and those of hbt_perm_test_batched. */
typedef struct hbt_tune_entry {
    double cost[2];
    int32_t grid_wide, grid_narrow, split_cap, chunks;
    int32_t tuned, _pad;
} hbt_tune_entry;  /* 40 bytes */
hbt_status hbt_tune_batched(int64_t npairs, const void* Z_all, const int64_t* row_offset,
                            const int64_t* n, const int64_t* m, const int64_t* B,
                            const uint32_t* pair_index, int64_t d, const hbt_perm_params* common,
                            hbt_result* results, void* ws, size_t ws_bytes, void* stream);
hbt_status hbt_tune_entry_get(int32_t precision, int64_t d, hbt_tune_entry* entry);
hbt_status hbt_tune_entry_set(int32_t precision, int64_t d, const hbt_tune_entry* entry);
hbt_status hbt_tune_get(int64_t d, double* costs, int32_t* tuned);
hbt_status hbt_tune_set(int64_t d, const double* costs);
hbt_status hbt_tune_save(const char* path);
hbt_status hbt_tune_load(const char* path);
hbt_status hbt_tile_widths(int64_t npairs, const int64_t* B, int64_t d, int32_t* widths);

/* ------------------------------------------------------------------------
 * Learned permutation-budget allocator.  The paper gives every pair the same
 * number of splits; here a small network estimates, from quantities of
 * Algorithm 1 Steps 1-4, the mean and log standard deviation of a pair's
 * permuted statistics T_b (Algorithm 1 Step 5), and the normal approximation
 * p^ = 1 - Phi((T_obs - mean) / sd) sets how many splits the pair gets.  The
 * permutation p-value of eq:pvalue stays the decision.
 *
 * Network: 12 -> 64 -> 64 -> 2, ReLU, FP32, parameters theta (HBT_MLP_PARAMS
 * floats, device): shift[12], scale[12] (inputs enter as (x - shift) *
 * scale), oshift[2], oscale[2] (outputs leave as oshift + oscale * y~), these
 * 28 not trained; then W1[64][12], b1[64], W2[64][64], b2[64], W3[2][64],
 * b3[2], row-major, y~ = W3 relu(W2 relu(W1 x~ + b1) + b2) + b3.  Outputs per
 * row: (mean, log sd).
 * ------------------------------------------------------------------------ */
#define HBT_MLP_FEATURES 12
#define HBT_MLP_PARAMS 5150
#define HBT_MLP_TRAINABLE_OFFSET 28   /* theta[28:] is trained */

/* features (device, npairs x 12 floats) of each pair from its results (device,
 * from hbt_perm_test or hbt_perm_test_batched; any B >= 1): log n, log m,
 * r_X, r_Y, the pooled MRL after alignment (n r_X + m r_Y) / (n + m) (the
 * appendix's alignment optimum), mu_cos, log g_d(r_X), log g_d(r_Y), T_obs,
 * n / (n + m), log(1 - r_X^2), log(1 - r_Y^2); computed in FP64.
 * Errors: HBT_ERR_ARG (NULL pointer, bad gd), HBT_ERR_SIZE (npairs < 1, d
 * outside [1, HBT_MAX_D]), HBT_ERR_DEVICE. */
hbt_status hbt_budget_features(int64_t npairs, const hbt_result* results, int64_t d, int32_t gd,
                               float* features, void* stream);

/* targets (device, npairs x 2 floats) = (t_mean, log t_sd) of each result:
 * the network's training targets, from runs with many splits.
 * Errors: HBT_ERR_ARG, HBT_ERR_SIZE (npairs < 1), HBT_ERR_DEVICE. */
hbt_status hbt_null_targets(int64_t npairs, const hbt_result* results, float* targets, void* stream);

/* theta[0:24] = per-feature mean and 1 / standard deviation over `rows`
 * feature rows (FP64 reductions; a constant feature gets scale 1).
 * Errors: HBT_ERR_ARG, HBT_ERR_SIZE (rows < 1), HBT_ERR_DEVICE. */
hbt_status hbt_feature_norm(int64_t rows, const float* features, float* theta, void* stream);

/* theta[24:28] = per-output mean and standard deviation of `rows` targets
 * (rows x 2 floats), so the network fits standardised targets.
 * Errors: HBT_ERR_ARG, HBT_ERR_SIZE (rows < 1), HBT_ERR_DEVICE. */
hbt_status hbt_target_norm(int64_t rows, const float* targets, float* theta, void* stream);

/* out (device, rows x 2 floats) = network(features).
 * Errors: HBT_ERR_ARG, HBT_ERR_SIZE (rows < 1), HBT_ERR_DEVICE. */
hbt_status hbt_mlp_forward(int64_t rows, const float* features, const float* theta, float* out,
                           void* stream);

/* grad (device, HBT_MLP_PARAMS floats; entries below the trainable offset are
 * left untouched) = gradient of L = (1/rows) sum_r (1/2) |(out_r - target_r) /
 * oscale|^2 with targets (device, rows x 2); loss (device double, nullable) = L.  The
 * sum over rows runs in a fixed order in FP64, so results are reproducible.
 * Errors: HBT_ERR_ARG, HBT_ERR_SIZE, HBT_ERR_WORKSPACE, HBT_ERR_DEVICE. */
size_t hbt_mlp_grad_workspace_size(int64_t rows);
hbt_status hbt_mlp_grad(int64_t rows, const float* features, const float* targets,
                        const float* theta, float* grad, double* loss, void* ws, size_t ws_bytes,
                        void* stream);

/* One Adam step (Kingma & Ba 2015, Algorithm 1, bias-corrected; step >= 1)
 * on theta[28:], with first and second moments adam_m, adam_v (device,
 * HBT_MLP_PARAMS floats each, zero before step 1).
 * Errors: HBT_ERR_ARG (NULL pointer, step < 1, lr <= 0, betas outside
 * [0, 1)), HBT_ERR_DEVICE. */
hbt_status hbt_mlp_adam(float* theta, const float* grad, float* adam_m, float* adam_v, int64_t step,
                        float lr, float beta1, float beta2, float eps, void* stream);

/* budgets (device, npairs int64) from the network outputs (device, npairs x 2)
 * and the pairs' T_obs (results): with p^ as above, pairs with p^ in the
 * fallback band [p_lo, p_hi] get b_max; the others get
 * ceil(zq^2 p^ (1 - p^) / (p^ - e)^2), e the nearer band edge, clamped to
 * [b_min, b_max] (the splits that put zq standard errors of the estimated p
 * between p^ and the band).  p_lo = p_hi = alpha gives the plain rule.
 * Errors: HBT_ERR_ARG (NULL pointer, 0 > p_lo > p_hi > 1, zq <= 0),
 * HBT_ERR_SIZE (npairs < 1, b_min < 1, b_max < b_min), HBT_ERR_DEVICE. */
hbt_status hbt_budgets(int64_t npairs, const float* mlp_out, const hbt_result* results,
                       double p_lo, double p_hi, int64_t b_min, int64_t b_max, double zq,
                       int64_t* budgets, void* stream);

/* budgets (device, npairs int64) by expected cost, from the network outputs
 * and the pairs' T_obs as in hbt_budgets: a pair whose p^ lies in the
 * fallback band [p_lo, p_hi] gets b_max (it would be rerun with b_max
 * splits anyway); any other pair gets the B among b_min, 2 b_min, 4 b_min,
 * ... (below b_max) and b_max that minimises the expected number of splits
 * B + b_max * P(its permutation p after B splits lands in the band), the
 * p-value (1 + count) / (B + 1) taken as normal with mean (1 + B p^) / (B + 1)
 * and standard deviation sqrt(B p^ (1 - p^)) / (B + 1) (ties: the smaller
 * B).  A pair far from the band thus gets b_min, one near an edge as many
 * splits as keep a rerun unlikely, unless a rerun is the cheaper risk.
 * Errors: HBT_ERR_ARG (NULL pointer, 0 > p_lo > p_hi > 1), HBT_ERR_SIZE
 * (npairs < 1, b_min < 1, b_max < b_min), HBT_ERR_DEVICE. */
hbt_status hbt_budgets_min_cost(int64_t npairs, const float* mlp_out, const hbt_result* results,
                                double p_lo, double p_hi, int64_t b_min, int64_t b_max,
                                int64_t* budgets, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HBT_H_ */
