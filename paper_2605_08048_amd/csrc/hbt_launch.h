// Host-side launchers of the HIP kernels (one translation unit per stage).
// Every launcher enqueues on `s` and returns the HIP status of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hbt_internal.h"

namespace hbt {

// Copy `bytes` (<= 3072 per launch, split internally) of host data into
// device memory through kernel arguments: stream-ordered, no host buffer
// outlives the call, capturable in a graph.
hipError_t upload(void* dst, const void* src, size_t bytes, hipStream_t s);

// Zero `bytes` (a multiple of 8) of device memory with a fill kernel.
hipError_t zero(void* dst, size_t bytes, hipStream_t s);

// --- alignment (Algorithm 1, Steps 1-4) ---------------------------------
// FP64 column sums of every chunk: partial[chunk][d].
// chunk_bad[chunk] = 1 when a row of the chunk is not a unit vector
// (| |x| - 1 | > 1e-4 or NaN), else 0; every launcher below writes it.
hipError_t launch_colsum(int input_dtype, const PairDesc* pairs, int npairs,
                         int nchunks, int d, double* partial, int32_t* chunk_bad, hipStream_t s);
// Per pair: sums, r, mean directions, v, v.v, identity, T_obs, tau, the pooled
// total t (FP64 and FP32), the hbt_result header.
hipError_t launch_finalize(const PairDesc* pairs, int npairs, const double* partial,
                           const int32_t* chunk_bad, int d,
                           int d_pad, int align, int gd, double* sxy, PairState* st, double* v,
                           double* t64, float* t32, PairCount* cnt, hbt_result* res,
                           hipStream_t s, int p0 = 0,  // pairs [p0, p0 + npairs)
                           float* v32 = nullptr);      // FP32 copy of v (d_pad per pair), nullable
// coef[coef0 + i] = 2 (v . x_i) / (v . v) (0 when H = I) for the X rows of
// every pair (FP32 rows), total = sum of n.
hipError_t launch_fold_coef(const PairDesc* pairs, int npairs, const PairState* st, const double* v, int d,
                            int d_pad, int64_t total, double* coef, hipStream_t s);
// Reflect X rows, write Z in the precision's storage format, the FP64
// coefficients 2 (v.x_i) / (v.v) and zero padding.
// 16-byte-load variants for FP32 rows with d % 4 == 0 and d_pad <= 1024 (the
// caller also checks that every X, Y is 16-byte aligned).
bool vector_rows_ok(int input_dtype, int d, int d_pad);
hipError_t launch_colsum_vec(const PairDesc* pairs, int npairs, int nchunks, int d,
                             int d_pad, double* partial, int32_t* chunk_bad, hipStream_t s);
// Column sums plus the storage of the 32-row groups that hold no X rows (the
// 16-byte path of the group-sum calls); launch_reflect_vec then takes the
// x_octets(n) octets of each pair (total_octets = their sum over pairs).
hipError_t launch_colsum_store_vec(int precision, const PairDesc* pairs, int npairs, int nchunks,
                                   int d, int d_pad, double* partial, void* zstore,
                                   int64_t zplane_elems, float* z32, int32_t* chunk_bad,
                                   hipStream_t s, int c0 = 0);  // chunks [c0, c0 + nchunks)
hipError_t launch_reflect_vec(int precision, const PairDesc* pairs, int npairs,
                              int64_t total_octets, const PairState* st, const double* v, int d,
                              int d_pad, double* coef, void* zstore, int64_t zplane_elems,
                              float* z32, hipStream_t s,
                              int64_t oct0 = 0  /* octets [oct0, total_octets) */);
hipError_t launch_reflect(int input_dtype, int precision, const PairDesc* pairs, int npairs,
                          int64_t total_octets, const PairState* st, const double* v, int d,
                          int d_pad, double* coef, void* zstore, int64_t zplane_elems,
                          float* z32, hipStream_t s);
// hbt_align's output: X' in the input dtype (may alias X).
hipError_t launch_reflect_out(int input_dtype, const PairDesc* pair, const PairState* st,
                              const double* v, int n, int d, void* X_out, double* v_out,
                              hipStream_t s);

// --- random splits ------------------------------------------------------
// LDS bytes a work-group of the split kernel (four split rows) needs for
// pairs of up to max_np pooled rows, and the device's limit per work-group.
size_t split_lds_per_block(int max_np);
size_t split_lds_limit();
// Per-pair problems found while drawing or copying splits go to sstat (one
// int32 per pair, zeroed by the caller), apart from the pair state that the
// alignment writes, so that the split stage may run beside the alignment.
// wg_per_cu > 0 pads each work-group's LDS so that at most that many share a
// CU: beside the alignment kernels, an uncapped split kernel takes every wave
// slot and the two stages run one after the other.  The split kernel reads
// only the block table (bp): sizes, mask row width and pair index are copied
// there, and rows of pairs that share another pair's splits are skipped.
constexpr int kSplitWgPerCuBesideAlign = 6;
hipError_t launch_split_masks(const BlockPair* bp, int npairs,
                              int64_t rows, int max_np, uint64_t seed, uint32_t* mask,
                              int32_t* sstat, int wg_per_cu, hipStream_t s,
                              int64_t row0 = 0  /* split rows [row0, rows) */);
// Explicit masks: copy rows of ceil(N/32) words into the workspace layout and
// check that each holds exactly n items.
hipError_t launch_copy_masks(const uint32_t* user, int64_t user_row0, int64_t rows, int N, int n,
                             int Wp, uint32_t* mask, int32_t* sstat, hipStream_t s);
// Copy workspace masks back to a caller buffer of ceil(N/32) words per row.
hipError_t launch_export_masks(const uint32_t* mask, int64_t rows, int Wp, int W, uint32_t* out,
                               hipStream_t s);

// --- group sums (eq:gemm) -----------------------------------------------
// Splits per group-sum tile (the tile list steps b0 by this).
int groupsum_tile_splits(int precision);
// partial[slot][row] = (|sigma_small|^2, |t - sigma_small|^2) over the slot's
// kDSlot columns, sigma_small = mask_small . Z; slot-major with prow rows per
// slot (the block's split rows).
// FP32 / FP64 use the tile list; split BF16 uses the per-pair groups: ngw
// groups of kTileWide-split tiles (ntw tiles), then ng256 of kTileNarrow.
// Split-BF16 tile widths: kTileWide splits per work-group of eight waves, or
// kTileNarrow per work-group of four.
constexpr int kTileWide = 1024, kTileNarrow = 256;
// Compute units of the current device (cached per device).
int device_cus();
hipError_t launch_groupsum(int precision, const PairDesc* pairs, const BlockPair* bp,
                           const GemmTile* tiles, int ntiles, const GemmGroup* groups, int ngw,
                           int ntw, int ng256, int nt256, int d_pad, const void* zstore,
                           int64_t zplane_elems, const uint32_t* mask, const float* t32,
                           const double* t64, double* partial, int64_t prow, float* sig,
                           hipStream_t s, int grid_wide = 16, int grid_narrow = 0,
                           const float* v32 = nullptr, double* pv = nullptr, bool hi_only = false);
// grid_wide / grid_narrow: persistent work-groups per CU of the 1024-split
// launch and of the 256-split (or int8) launch (0: 32 for the 256-split
// split-BF16 kernel, 16 for int8).  pv (split BF16 only, nullable): also
// v . sigma per split and slot (v32 the pairs' FP32 Householder vectors),
// for pairs whose rows are stored unreflected.  hi_only (split BF16, no pv):
// the products of the hi plane alone (the lazy precision's first pass).

// The lazy precision's second pass: rlist holds, for each pair p, rcnt[p]
// split rows from rlist[mrow0 of p] (the splits its first pass could not
// decide).  launch_refine_tiles builds their 256-split tile table (one group
// per entry of `groups`, the first pass's table, in its order) and the tile
// count on the device; launch_groupsum_refine runs the split-BF16 product on
// those splits and writes their partial rows in place.
hipError_t launch_refine_tiles(const GemmGroup* groups, int ngroups, const uint32_t* rcnt, int d_pad,
                               GemmGroup* out, int64_t* ntile, hipStream_t s);
hipError_t launch_groupsum_refine(const PairDesc* pairs, const BlockPair* bp, const GemmGroup* rgroups,
                                  int ngroups, const int64_t* ntile, int d_pad, const void* zstore,
                                  int64_t zplane_elems, const uint32_t* mask, const float* t32, double* partial,
                                  int64_t prow, const uint32_t* rlist, const uint32_t* rcnt, int grid_narrow,
                                  hipStream_t s);
hipError_t launch_groupsum_refine(const PairDesc* pairs, const BlockPair* bp, const GemmGroup* rgroups,
                                  int ngroups, const int64_t* ntile, int d_pad, const void* zstore,
                                  int64_t zplane_elems, const uint32_t* mask, const float* t32, double* partial,
                                  int64_t prow, const uint32_t* rlist, const uint32_t* rcnt, int grid_wide,
                                  int grid_narrow, hipStream_t s);

// --- point-to-centroid route (statistic route 2) -------------------------
// z_i . t per pooled row; then Q = Z S^T with the masked column sums
// partial[row tile][row] = (|sigma_small|^2 part, |t - sigma_small|^2 part),
// prow rows per tile.
hipError_t launch_row_dot_t(const PairDesc* pairs, int npairs, const float* z32,
                            const double* t64, int d_pad, int64_t total_rows, double* zt,
                            hipStream_t s);
hipError_t launch_centroid(bool bf16x3, const PairDesc* pairs, const BlockPair* bp, const CTile* tiles,
                           int ntiles, int d_pad, const float* z32, const float* sig,
                           const uint32_t* mask, const double* zt, double* partial,
                           int64_t prow, hipStream_t s);

// --- statistic, exceedances, recheck, p ---------------------------------
// Fold sums of shared clouds: mask words per segment of a split's X items
// (each segment is summed by its own wave), and the segments of a pair.
constexpr int kFoldSegWords = 16;
__host__ __device__ inline int fold_segments(int n) { return ((n + 31) / 32 + kFoldSegWords - 1) / kFoldSegWords; }
hipError_t launch_stat(const PairDesc* pairs, const BlockPair* bp, int npairs, int64_t rows,
                       const PairState* st, const double* partial, int nslot, int64_t prow, int d, int gd,
                       int alternative, const RecheckBand& band, int no_recheck, void* T_out,
                       int T_mode, double* Tw,
                       PairCount* cnt, uint32_t* flags, uint32_t* nflag, hipStream_t s, const double* pv = nullptr,
                       const uint32_t* mask = nullptr, const double* coef = nullptr,
                       double* fpart = nullptr, int fold_segs = 0);
// A split whose T_b is within `band` of the threshold is flagged: it joins
// its pair's recheck list (flags from the pair's first block row, nflag[pair]
// counting them; the counts are zeroed by the caller) and is not counted.
// launch_stat with pv (v . sigma per slot), mask, coef and fpart non-null
// reflects the group sums of pairs stored unreflected (the Householder fold):
// a first kernel writes each split's fold sums per segment into fpart
// (fold_segs x rows doubles, segment-major; fold_segs = the largest pair's
// fold_segments(n)), which the statistic kernel adds in segment order.
// The lazy precision's statistic.  First pass (refined = false), on the hi
// plane's sums: splits within `band` of the threshold, NaN, or of a pair with
// min(n, m) < kLazyMinGroup go to their pair's list (rlist / rcnt, zeroed
// counts) and are not counted; the others are decided.  Second pass (refined
// = true), on the listed splits' split-BF16 sums: decided, or flagged for the
// FP64 recheck.  Tw (and T_out, nullable, as in launch_stat) holds each
// split's latest T_b.
constexpr int kLazyMinGroup = 16;
hipError_t launch_stat_lazy(bool refined, const PairDesc* pairs, const BlockPair* bp, int npairs, int64_t rows,
                            const PairState* st, const double* partial, int nslot, int64_t prow, int d, int gd,
                            int alternative, const RecheckBand& band, int no_recheck, double* Tw, PairCount* cnt,
                            uint32_t* flags, uint32_t* nflag, uint32_t* rlist, uint32_t* rcnt, hipStream_t s,
                            void* T_out = nullptr, int T_mode = 0);
// FP64 recheck of the flagged splits.  flags: per pair, from the pair's
// first block row, the split rows k_stat flagged; nflag: their number per
// pair.  plan: 4 (npairs + 1) int64 of work plan (written here).  rseg:
// `slots` vectors of d_pad doubles (per flag and segment sums; nullptr when
// no pair has more than one segment); the value of each flag's sums does not
// depend on it.
constexpr int kRecheckSlotsSingle = 2048;
inline int64_t recheck_plan_words(int npairs) { return 4 * ((int64_t)npairs + 1); }
int recheck_segments(int max_np);
int64_t recheck_slots(int npairs, int d_pad);
hipError_t launch_recheck(int input_dtype, const PairDesc* pairs, const BlockPair* bp, int npairs,
                          const PairState* st, const double* v, const double* t64, const double* coef,
                          const uint32_t* mask, const uint32_t* flags, const uint32_t* nflag, int64_t* plan,
                          int64_t max_flags, int max_np, double* rseg, int64_t slots, int d, int gd,
                          int alternative, PairCount* cnt, double* Tw, hipStream_t s);
// Sums of T_b - T_obs and its square per pair over the current block (Tw
// holds the block's final T_b, recheck applied).
hipError_t launch_moments(int npairs, const BlockPair* bp, const PairState* st, const double* Tw,
                          PairCount* cnt, hipStream_t s);
// --- permutation-budget allocator ---------------------------------------
size_t mlp_train_ws_bytes(int64_t rows);
hipError_t launch_features(int64_t npairs, const hbt_result* res, int d, int gd, float* feat,
                           hipStream_t s);
hipError_t launch_null_targets(int64_t npairs, const hbt_result* res, float* target, hipStream_t s);
hipError_t launch_feature_norm(int64_t rows, const float* feat, float* theta, hipStream_t s);
hipError_t launch_target_norm(int64_t rows, const float* target, float* theta, hipStream_t s);
hipError_t launch_mlp_forward(int64_t rows, const float* feat, const float* theta, float* out,
                              hipStream_t s);
hipError_t launch_mlp_grad(int64_t rows, const float* feat, const float* target, const float* theta,
                           float* grad, double* loss, void* ws, hipStream_t s);
hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_budgets(int64_t npairs, const float* out, const hbt_result* res, double lo,
                          double hi, int64_t bmin, int64_t bmax, double zq, int64_t* budget,
                          hipStream_t s);
hipError_t launch_budgets_cost(int64_t npairs, const float* out, const hbt_result* res, double lo,
                               double hi, int64_t bmin, int64_t bmax, int64_t* budget, hipStream_t s);

// Per pair: count, B, p, null moments and status (the alignment's, else that
// of the split rows that drew its masks).
hipError_t launch_final(int npairs, const BlockPair* bp, const PairState* st, const int32_t* sstat,
                        const PairCount* cnt, const int64_t* Btot, hbt_result* res, hipStream_t s);

}  // namespace hbt
