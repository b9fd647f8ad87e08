// Permuted statistics, exceedance counts and the p-value (Algorithm 1,
// Steps 5-6; Algorithm 2's r_1, r_2, T^(b) and streaming count; eq:pvalue).
//
// The scalar math per split (norms, g_d, T_b) is FP64.  A split whose T_b,
// computed from FP32 / split-BF16 group sums, lies within the precision's
// error bound of the decision threshold is not counted here: it goes to a
// list and is re-evaluated from the input rows in FP64 (recheck), so the
// final counts follow the FP64 statistic.
#include "hbt_launch.h"

namespace hbt {

// Householder fold: c = sum over the smaller group's X rows of 2 (v . x_i) /
// (v . v) per split row, in segments of kFoldSegWords mask words (512 X
// items): work-group (x, y) takes the 256 split rows of block x and segment y
// of each row's pair, and writes the segment's sum (FP64; four running sums,
// over the indices i % 4 = 0, 1, 2, 3, added at the end) to
// fpart[y][row]; segments past a pair's fold_segments(n) are not written.
// Large pairs thus spread over as many waves as they have segments.  In a
// wave of one pair (consecutive split rows, Wp words apart) the segment's
// words of the 64 rows pass through LDS, read as 64-byte runs of each row so
// that every fetched line is used whole; the 32 coefficients of a word are
// wave-uniform (scalar loads) and a lane adds the ones its bits select, the
// selection made with sign-extended one-bit masks rather than branches.  A
// wave across a pair boundary takes each lane's own pair.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
void k_fold_c(const PairDesc* __restrict__ pairs, const BlockPair* __restrict__ bp, int npairs,
              int64_t rows, const uint32_t* __restrict__ mask, const double* __restrict__ coef,
              double* __restrict__ fpart) {
    constexpr int kW = kFoldSegWords;
    // 64 rows x 16 words per wave; a row takes 20 words so that the lanes'
    // 16-byte reads of their own rows fall on distinct banks
    __shared__ uint4 stg[4][64][kW / 4 + 1];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int seg = blockIdx.y, w0 = kW * seg;
    const int64_t row0 = (int64_t)blockIdx.x * 256 + 64 * wave;
    const int64_t row = row0 + lane;
    const bool active = row < rows;
    if (row0 >= rows) return;  // the whole wave
    int p = 0;
    if (active) p = upper_index(npairs, row, [&](int k) { return bp[k].mrow0; });
    const int p0 = __shfl(p, 0, 64);  // lane 0 is active
    const bool one_pair = __ballot(!active || p == p0) == ~0ull;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (one_pair) {
        const int pu = __builtin_amdgcn_readfirstlane(p0);
        const int nu = pairs[pu].n, Wp = pairs[pu].Wp;
        const int nw = (nu + 31) >> 5;  // X words of a row (nw <= Wp, Wp % 4 == 0)
        if (w0 >= nw) return;           // wave-uniform: no such segment
        const uint32_t flip = pairs[pu].flip ? 0xffffffffu : 0u;
        const double* cf = coef + pairs[pu].coef0;
        const uint32_t* mk0 = mask_row(mask, bp[pu], row0, Wp);  // 16-byte aligned rows
#pragma unroll
        for (int i = 0; i < kW / 4; ++i) {
            const int idx = 64 * i + lane, r = idx >> 2, q = idx & 3, wq = w0 + 4 * q;
            uint4 val = make_uint4(0u, 0u, 0u, 0u);
            if (row0 + r < rows && wq < nw) val = *(const uint4*)(mk0 + (int64_t)r * Wp + wq);
            stg[wave][r][q] = val;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int kend = min(kW, nw - w0);
        for (int k = 0; k < kend; ++k) {
            const int w = w0 + k;
            const uint4 u = stg[wave][lane][k >> 2];
            const uint32_t word = (k & 3) == 0 ? u.x : (k & 3) == 1 ? u.y : (k & 3) == 2 ? u.z : u.w;
            const uint32_t bits = (word ^ flip) & range_bits(w, 0, nu);
            const double* cw = cf + 32 * w;  // the array has 32 spare entries at its end
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                const uint32_t sel = (uint32_t)__builtin_amdgcn_sbfe((int)bits, j, 1);
                const uint64_t cb = (uint64_t)__double_as_longlong(cw[j]);
                const uint64_t m = ((uint64_t)sel << 32) | sel;
                acc[j & 3] += __longlong_as_double((long long)(cb & m));
            }
        }
    } else if (active) {
        const PairDesc pd = pairs[p];
        const int nw = (pd.n + 31) >> 5;
        if (w0 >= nw) return;
        const uint32_t* mk = mask_row(mask, bp[p], row, pd.Wp);
        const uint32_t flip = pd.flip ? 0xffffffffu : 0u;
        const double* cf = coef + pd.coef0;
        for (int w = w0; w < min(nw, w0 + kW); ++w) {
            const uint32_t bits = (mk[w] ^ flip) & range_bits(w, 0, pd.n);
#pragma unroll 4
            for (int j = 0; j < 32; ++j) acc[j & 3] += (bits >> j) & 1u ? cf[32 * w + j] : 0.0;
        }
    }
    if (active) fpart[(int64_t)seg * rows + row] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// MODE kStatLazyFirst (the lazy precision's first pass, hi-plane sums): a
// split whose T_b lies within the band, is NaN, or belongs to a pair with
// min(n, m) < kLazyMinGroup joins its pair's refinement list (rlist from the
// pair's first row, rcnt the length) instead of being decided.  MODE
// kStatRefined: thread i takes list entry i (entry k of pair p is thread
// mrow0 of p + k, for k < rcnt[p]) and decides that split from its
// split-BF16 sums, with the usual FP64-recheck flags.
//
// A split row joins a list of its pair (the recheck flags, or the lazy
// precision's refinement list) at list[first block row of the pair + k], k
// from the pair's counter: one atomic per wave when all its rows belong to
// one pair.
__device__ __forceinline__ void list_append(bool want, bool one_pair, int p0, int p, int64_t row,
                                            const BlockPair* bp, uint32_t* list, uint32_t* count) {
    const uint64_t wm = __ballot(want);
    if (one_pair) {
        uint32_t base = 0;
        if (lane_id() == 0 && wm) base = atomicAdd(&count[p0], (uint32_t)__popcll(wm));
        base = (uint32_t)__shfl((int)base, 0, 64);
        if (want) list[bp[p0].mrow0 + base + mbcnt64(wm)] = (uint32_t)row;
    } else if (want) {
        const uint32_t k = atomicAdd(&count[p], 1u);
        list[bp[p].mrow0 + k] = (uint32_t)row;
    }
}

enum StatMode { kStatPlain = 0, kStatLazyFirst = 1, kStatRefined = 2 };
template <int MODE>
__global__ __launch_bounds__(256) void k_stat(const PairDesc* __restrict__ pairs,
                                              const BlockPair* __restrict__ bp, int npairs,
                                              int64_t rows, const PairState* __restrict__ st,
                                              const double* __restrict__ partial, int nslot,
                                              int64_t prow, int d,
                                              int gd, int alternative, RecheckBand band,
                                              int no_recheck, void* T_out,
                                              int T_mode, double* __restrict__ Tw,
                                              PairCount* cnt, uint32_t* flags, uint32_t* nflag,
                                              const double* __restrict__ pv,
                                              const double* __restrict__ fpart,
                                              uint32_t* __restrict__ rlist, uint32_t* __restrict__ rcnt) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool in_range = i < rows;
    int p = 0;
    bool exceed = false;
    if (in_range) p = upper_index(npairs, i, [&](int k) { return bp[k].mrow0; });
    // a wave's first lane is in range whenever any of its lanes is
    const int p0 = __shfl(p, 0, 64);
    bool active = in_range;
    bool refine = false;  // kStatLazyFirst: the split goes to its pair's list
    bool flag = false;    // the split goes to its pair's FP64-recheck list
    int64_t row = i;
    if (MODE == kStatRefined && in_range) {
        active = i - bp[p].mrow0 < (int64_t)rcnt[p];
        if (active) row = rlist[i];
    }
    const bool one_pair = __ballot(!in_range || p == p0) == ~0ull;
    if (active) {
        const PairDesc pd = pairs[p];
        const PairState q = st[p];
        // partials are slot-major (slot k of all rows, then slot k + 1), so
        // the lanes of a wave read consecutive rows
        const double2* pr = (const double2*)partial + row;
        double ss_small = 0.0, ss_large = 0.0;
        const int ns = nslot > 0 ? nslot : pd.Np / 64;  // 0: the point-to-centroid row tiles of the pair
        for (int k = 0; k < ns; ++k) {
            const double2 v = pr[k * prow];
            ss_small += v.x;
            ss_large += v.y;
        }
        if (pv) {
            // Householder fold: the product summed the unreflected rows, so
            // sigma' = sigma - c v with c = sum over the smaller group's X rows
            // of 2 (v . x_i) / (v . v) (k_fold_c's segment sums), and
            //   |sigma'|^2     = |sigma|^2 - 2 c (v . sigma) + c^2 (v . v),
            //   |t - sigma'|^2 = |t - sigma|^2 + 2 c (v . t - v . sigma) + c^2 (v . v)
            // (t the pooled total of the reflected rows).
            double sv = 0.0;
            for (int k = 0; k < ns; ++k) sv += pv[k * prow + row];
            double c = 0.0;  // k_fold_c's segments, in order
            for (int k = 0; k < fold_segments(pd.n); ++k) c += fpart[k * rows + row];
            const double cvv = c * c * q.vv;
            ss_small = ss_small - 2.0 * c * sv + cvv;
            ss_large = ss_large + 2.0 * c * (q.vt - sv) + cvv;
        }
        // group 1 has n items, group 2 has m; the product ran on the smaller one
        const double ss1 = pd.flip ? ss_large : ss_small;
        const double ss2 = pd.flip ? ss_small : ss_large;
        const double n = (double)pd.n, m = (double)pd.m, dd = (double)d;
        const double r1 = sqrt(ss1) / n, r2 = sqrt(ss2) / m;
        const double T = log_g(r2, dd, gd) - log_g(r1, dd, gd);  // log v(X^(b)) - log v(Y^(b))
        if (T_out) {
            if (T_mode == 2) {  // T_b and both squared group-sum norms
                double* o = (double*)T_out + 3 * row;
                o[0] = T;
                o[1] = ss1;
                o[2] = ss2;
            } else if (T_mode == 1) {
                ((double*)T_out)[row] = T;
            } else {
                ((float*)T_out)[row] = (float)T;
            }
        }
        Tw[row] = T;
        const bool two = alternative == HBT_ALT_TWO_SIDED;
        const double val = two ? fabs(T) : T;
        const double thr = (two ? fabs(q.t_obs) : q.t_obs) - q.tau;
        const double eps = recheck_eps(band, n, m, dd, r1, r2, gd);
        const bool nan = T != T;
        if (MODE == kStatLazyFirst) {
            refine = nan || fabs(val - thr) <= eps || (pd.n < pd.m ? pd.n : pd.m) < kLazyMinGroup;
            if (!refine) exceed = val >= thr;
        } else {
            flag = !no_recheck && !nan && fabs(val - thr) <= eps;
            if (!flag) exceed = nan || val >= thr;
        }
    }
    if (MODE == kStatLazyFirst)
        list_append(refine, one_pair, p0, p, row, bp, rlist, rcnt);
    else
        list_append(flag, one_pair, p0, p, row, bp, flags, nflag);
    // count: one atomic per wave when all its rows belong to one pair
    const uint64_t ex = __ballot(exceed);
    if (one_pair) {
        if (lane_id() == 0 && ex) atomicAdd(&cnt[p0].count, (unsigned long long)__popcll(ex));
    } else if (exceed) {
        atomicAdd(&cnt[p].count, 1ull);
    }
}

hipError_t launch_stat(const PairDesc* pairs, const BlockPair* bp, int npairs, int64_t rows,
                       const PairState* st, const double* partial, int nslot, int64_t prow, int d, int gd,
                       int alternative, const RecheckBand& band, int no_recheck, void* T_out,
                       int T_mode, double* Tw, PairCount* cnt, uint32_t* flags, uint32_t* nflag,
                       hipStream_t s, const double* pv, const uint32_t* mask, const double* coef,
                       double* fpart, int fold_segs) {
    if (rows <= 0) return hipSuccess;
    const dim3 grid((unsigned)((rows + 255) / 256));
    if (pv) {
        if (!mask || !coef || !fpart || fold_segs < 1 || fold_segs > 65535) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_fold_c, dim3(grid.x, (unsigned)fold_segs), dim3(256), 0, s, pairs, bp, npairs,
                           rows, mask, coef, fpart);
    }
    hipLaunchKernelGGL(k_stat<kStatPlain>, grid, dim3(256), 0, s, pairs, bp, npairs, rows, st, partial, nslot,
                       prow, d, gd, alternative, band, no_recheck, T_out, T_mode, Tw, cnt, flags, nflag, pv, fpart,
                       nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_stat_lazy(bool refined, const PairDesc* pairs, const BlockPair* bp, int npairs, int64_t rows,
                            const PairState* st, const double* partial, int nslot, int64_t prow, int d, int gd,
                            int alternative, const RecheckBand& band, int no_recheck, double* Tw, PairCount* cnt,
                            uint32_t* flags, uint32_t* nflag, uint32_t* rlist, uint32_t* rcnt, hipStream_t s,
                            void* T_out, int T_mode) {
    if (rows <= 0) return hipSuccess;
    if (!rlist || !rcnt) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((rows + 255) / 256));
    if (refined)
        hipLaunchKernelGGL(k_stat<kStatRefined>, grid, dim3(256), 0, s, pairs, bp, npairs, rows, st, partial,
                           nslot, prow, d, gd, alternative, band, no_recheck, T_out, T_mode, Tw, cnt, flags, nflag,
                           nullptr, nullptr, rlist, rcnt);
    else
        hipLaunchKernelGGL(k_stat<kStatLazyFirst>, grid, dim3(256), 0, s, pairs, bp, npairs, rows, st, partial,
                           nslot, prow, d, gd, alternative, band, no_recheck, T_out, T_mode, Tw, cnt, flags, nflag,
                           nullptr, nullptr, rlist, rcnt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 recheck of the flagged splits.  The smaller group's sum is gathered
// from the input rows, each rebuilt in FP64 as the aligned row
// x_i - coef_i v (X, one rounding: fma(-coef_i, v, x_i)) or y_j (Y); the
// other group's sum is t - sigma_small with the FP64 pooled total t.
//
// k_stat lists the flags of each pair from the pair's first block row.  The
// rows of a pair are cut into segments of kSegWords mask words (512 pooled
// rows); wave w of a work-group takes words w, w + 4, w + 8 and w + 12 of a
// segment, and each lane columns c0 + 64 u + lane (u < 12) of each pass of
// kRecheckPass columns.  For each flag and column, sigma_small is formed in
// one order: per wave, its rows of the segment in ascending order; the
// segment's sum is the 4 wave sums added in wave order; then the segment
// sums are added in segment order.  For the squares, thread t of the
// work-group holds columns c0 + t, c0 + t + 256 and c0 + t + 512 of each
// pass (passes in order, then in that order); the work-group adds its
// threads' squares in a fixed tree.  How the work is
// spread never changes a bit:
//   * a pair whose flag segments fit the workspace slots has one work item
//     per flag and segment, whose sums go to the slots and are added by
//     k_recheck_finish; every other pair has one item per flag that walks
//     all segments with running totals (k_recheck_plan lays the items out on
//     the device, from the per-pair flag counts).
// ---------------------------------------------------------------------------
constexpr int kRecheckWaves = 4;
constexpr int kRecheckThreads = 64 * kRecheckWaves;
constexpr int kRecheckPass = 768;  // columns per pass (12 per lane)
constexpr int kRecheckCols = kRecheckPass / kRecheckThreads;  // columns per thread in the sums
static_assert(kRecheckPass % kRecheckThreads == 0, "a pass is whole columns per thread");
constexpr int kSegWords = 16;
constexpr int kRecheckRows = 8;    // rows in flight per wave (4 for FP64 rows)

// Segments of a pair's pooled mask positions.
__device__ __forceinline__ int pair_words(const PairDesc& pd) { return (pd.n + pd.m + pd.ygap + 31) >> 5; }
__device__ __forceinline__ int pair_segs(const PairDesc& pd) { return (pair_words(pd) + kSegWords - 1) / kSegWords; }

// Sum over the threads of a work-group in a fixed order (a butterfly in each
// wave, then the waves in order); every thread gets the sum.
__device__ __forceinline__ double block_sum(double x, double* red) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    __syncthreads();  // the previous sum's readers are done with red
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kRecheckWaves; ++q) s += red[q];
    return s;
}

// The squares of one column's sums (thread-local, in the order above).
__device__ __forceinline__ void add_squares(double sm, double tcol, double& ss_small, double& ss_large) {
    const double l = tcol - sm;
    ss_small = fma(sm, sm, ss_small);
    ss_large = fma(l, l, ss_large);
}

// The flag's FP64 statistic, decision and T_b (one thread).
__device__ void recheck_decide(const PairDesc& pd, const PairState& q, int p, int64_t row, double ss_small,
                               double ss_large, int d, int gd, int alternative, PairCount* cnt, double* Tw) {
    const double dd = (double)d;
    const double ss1 = pd.flip ? ss_large : ss_small;
    const double ss2 = pd.flip ? ss_small : ss_large;
    const double r1 = sqrt(ss1) / (double)pd.n, r2 = sqrt(ss2) / (double)pd.m;
    const double T = log_g(r2, dd, gd) - log_g(r1, dd, gd);
    const bool two = alternative == HBT_ALT_TWO_SIDED;
    const double val = two ? fabs(T) : T;
    const double thr = (two ? fabs(q.t_obs) : q.t_obs) - q.tau;
    if (T != T || val >= thr) atomicAdd(&cnt[p].count, 1ull);
    atomicAdd(&cnt[p].n_recheck, 1ull);
    Tw[row] = T;
}

// The work plan (one work-group), four arrays of npairs + 1 int64 in `plan`:
//   [0] whole items, [1] segmented items, [2] slots, [3] segmented flags:
//       exclusive prefixes over the pairs, totals at index npairs.
// A pair is segmented when it has more than one segment and its flag
// segments, added to those of the pairs before it, fit `slots`.
template <int NT>
__device__ __forceinline__ int64_t block_scan(int64_t x, int64_t* sh, int64_t* total) {
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int o = 1; o < NT; o <<= 1) {
        const int64_t y = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    const int64_t r = sh[t];
    *total = sh[NT - 1];
    __syncthreads();
    return r;
}

// NT threads: 64 for calls of at most 64 pairs (a single pair), else 1024
template <int NT>
__global__ __launch_bounds__(NT) void k_recheck_plan(const PairDesc* __restrict__ pairs, int npairs,
                                                     const uint32_t* __restrict__ nflag, int64_t slots,
                                                     int64_t* __restrict__ plan) {
    __shared__ int64_t sh[NT];
    const int t = threadIdx.x;
    const int np1 = npairs + 1;
    int64_t bw = 0, bs = 0, bc = 0, bf = 0;
    for (int p0 = 0; p0 < npairs; p0 += NT) {
        const int p = p0 + t;
        int64_t F = 0, G = 0;
        if (p < npairs) {
            F = nflag[p];
            G = pair_segs(pairs[p]);
        }
        const int64_t cand = (G > 1 && F > 0) ? F * G : 0;
        int64_t tc, tw, ts, tf;
        const int64_t ic = block_scan<NT>(cand, sh, &tc);
        const bool seg = cand > 0 && bc + ic <= slots;
        const int64_t wi = seg ? 0 : F, si = seg ? F * G : 0, fi = seg ? F : 0;
        const int64_t iw = block_scan<NT>(wi, sh, &tw);
        const int64_t is = block_scan<NT>(si, sh, &ts);
        const int64_t jf = block_scan<NT>(fi, sh, &tf);
        if (p < npairs) {
            plan[p] = bw + iw - wi;
            plan[np1 + p] = bs + is - si;
            plan[2 * np1 + p] = bc + ic - cand;
            plan[3 * np1 + p] = bf + jf - fi;
        }
        bw += tw;
        bs += ts;
        bc += tc;
        bf += tf;
    }
    if (t == 0) {
        plan[npairs] = bw;
        plan[np1 + npairs] = bs;
        plan[2 * np1 + npairs] = bc;
        plan[3 * np1 + npairs] = bf;
    }
}

struct RecheckArgs {
    const PairDesc* pairs;
    const BlockPair* bp;
    int npairs;
    const PairState* st;
    const double* v;
    const double* t64;
    const double* coef;
    const uint32_t* mask;
    const uint32_t* flags;
    const uint32_t* nflag;
    const int64_t* plan;
    int d, d_pad, gd, alternative;
    double* rseg;
    PairCount* cnt;
    double* Tw;
};

// One work item: flag j of pair p over segments [sg0, sg1).  Segmented items
// write the flag's segment sums to its slots; whole items keep running
// totals over every segment and decide the flag.
template <typename Tin>
__device__ void recheck_item(const RecheckArgs& A, int p, int64_t j, int sg0, int sg1, bool whole,
                             double (*part)[kRecheckPass], double* red) {
    constexpr int kU = kRecheckPass / 64;  // columns per lane per pass
    // rows in flight per wave (FP64 rows: half as many, for the registers;
    // the order in which rows are added does not depend on it)
    constexpr int kRows = sizeof(Tin) == 4 ? kRecheckRows : kRecheckRows / 2;
    const int t = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63;
    const PairDesc pd = A.pairs[p];
    const BlockPair bq = A.bp[p];
    const int d = A.d;
    const int W = pair_words(pd), G = pair_segs(pd);
    const uint32_t flip = pd.flip ? 0xffffffffu : 0u;
    const Tin* X = (const Tin*)pd.X;
    const Tin* Y = (const Tin*)pd.Y;
    const double* vp = A.v + (int64_t)p * A.d_pad;
    const double* tp = A.t64 + (int64_t)p * A.d_pad;
    const double* cf = A.coef + pd.coef0;
    const int64_t slot = whole ? 0 : A.plan[2 * (A.npairs + 1) + p] + j * G;
    const int64_t row = A.flags[bq.mrow0 + j];
    const uint32_t* mk = mask_row(A.mask, bq, row, pd.Wp);
    double ssS = 0.0, ssL = 0.0;
    for (int c0 = 0; c0 < d; c0 += kRecheckPass) {
        double vc[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int col = c0 + 64 * u + lane;
            vc[u] = col < d ? vp[col] : 0.0;
        }
        double tot[kRecheckCols];
#pragma unroll
        for (int k = 0; k < kRecheckCols; ++k) tot[k] = 0.0;
        for (int sg = sg0; sg < sg1; ++sg) {
            double acc[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) acc[u] = 0.0;
            // this wave's words of the segment: w0, w0 + 4, w0 + 8, w0 + 12
            const int w0 = sg * kSegWords + wave, we = min(W, (sg + 1) * kSegWords);
            int w = w0;
            auto word_bits = [&](int ww) -> uint32_t {
                return ww < we ? (mk[ww] ^ flip) & item_bits(ww, pd.n, pd.m, pd.ygap) : 0u;
            };
            uint32_t U = word_bits(w);
            for (;;) {
                int rows[kRows];
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    while (!U && w + kRecheckWaves < we) U = word_bits(w += kRecheckWaves);
                    if (U) {
                        rows[k] = 32 * w + __builtin_ctz(U);
                        U &= U - 1u;
                    } else {
                        rows[k] = -1;
                    }
                }
                if (rows[0] < 0) break;
                // columns are clamped to the row (no branch around a load)
                Tin z[kRows][kU];
                double kc[kRows];
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    int i = rows[k] < 0 ? 0 : rows[k];
                    if (i >= pd.n) i -= pd.ygap;  // Y's mask positions to pooled items
                    const bool isx = i < pd.n;
                    kc[k] = isx ? cf[i] : 0.0;
                    const Tin* src = isx ? X + (int64_t)i * d : Y + (int64_t)(i - pd.n) * d;
#pragma unroll
                    for (int u = 0; u < kU; ++u) {
                        const int col = c0 + 64 * u + lane;
                        z[k][u] = src[col < d ? col : d - 1];
                    }
                }
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    if (rows[k] < 0) continue;
#pragma unroll
                    for (int u = 0; u < kU; ++u) acc[u] += fma(-kc[k], vc[u], (double)z[k][u]);
                }
            }
            // the segment's sum: the wave sums in wave order
#pragma unroll
            for (int u = 0; u < kU; ++u) part[wave][64 * u + lane] = acc[u];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kRecheckCols; ++k) {
                const int cc = t + kRecheckThreads * k;
                double sm = 0.0;
#pragma unroll
                for (int q = 0; q < kRecheckWaves; ++q) sm += part[q][cc];
                if (whole)
                    tot[k] += sm;
                else if (c0 + cc < d)
                    A.rseg[(slot + sg) * A.d_pad + c0 + cc] = sm;
            }
            __syncthreads();
        }
        if (whole) {
#pragma unroll
            for (int k = 0; k < kRecheckCols; ++k) {
                const int cc = t + kRecheckThreads * k;
                if (c0 + cc < d) add_squares(tot[k], tp[c0 + cc], ssS, ssL);
            }
        }
    }
    if (whole) {
        const double s1 = block_sum(ssS, red), s2 = block_sum(ssL, red);
        if (t == 0) recheck_decide(pd, A.st[p], p, row, s1, s2, d, A.gd, A.alternative, A.cnt, A.Tw);
    }
}

template <typename Tin>
__global__ __launch_bounds__(kRecheckThreads) void k_recheck(RecheckArgs A) {
    __shared__ double part[kRecheckWaves][kRecheckPass];  // per-wave sums of a segment
    __shared__ double red[kRecheckWaves];
    const int np1 = A.npairs + 1;
    const int64_t* wpre = A.plan;
    const int64_t* spre = A.plan + np1;
    const int64_t NW = wpre[A.npairs], NS = spre[A.npairs];
    for (int64_t it = blockIdx.x; it < NW + NS; it += gridDim.x) {
        if (it < NW) {  // one flag, every segment
            const int p = upper_index(A.npairs, it, [&](int k) { return wpre[k]; });
            recheck_item<Tin>(A, p, it - wpre[p], 0, pair_segs(A.pairs[p]), true, part, red);
        } else {  // one flag, one segment
            const int64_t x = it - NW;
            const int p = upper_index(A.npairs, x, [&](int k) { return spre[k]; });
            const int64_t r = x - spre[p];
            const int G = pair_segs(A.pairs[p]);
            const int sg = (int)(r % G);
            recheck_item<Tin>(A, p, r / G, sg, sg + 1, false, part, red);
        }
    }
}

// The segmented flags: sigma_small from the segment sums in segment order,
// then the same squares, statistic and decision as a whole item.
__global__ __launch_bounds__(kRecheckThreads) void k_recheck_finish(RecheckArgs A) {
    __shared__ double red[kRecheckWaves];
    const int np1 = A.npairs + 1;
    const int64_t* spl = A.plan + 2 * np1;
    const int64_t* fpre = A.plan + 3 * np1;
    const int64_t NF = fpre[A.npairs];
    const int t = threadIdx.x, d = A.d;
    for (int64_t qf = blockIdx.x; qf < NF; qf += gridDim.x) {
        const int p = upper_index(A.npairs, qf, [&](int k) { return fpre[k]; });
        const int64_t j = qf - fpre[p];
        const PairDesc pd = A.pairs[p];
        const int G = pair_segs(pd);
        const int64_t row = A.flags[A.bp[p].mrow0 + j];
        const double* src = A.rseg + (spl[p] + j * G) * A.d_pad;
        const double* tp = A.t64 + (int64_t)p * A.d_pad;
        double ssS = 0.0, ssL = 0.0;
        for (int c0 = 0; c0 < d; c0 += kRecheckPass)
#pragma unroll
            for (int k = 0; k < kRecheckCols; ++k) {
                const int cc = t + kRecheckThreads * k;
                const int col = c0 + cc;
                if (col < d) {
                    double sm = 0.0;
                    for (int sg = 0; sg < G; ++sg) sm += src[(int64_t)sg * A.d_pad + col];
                    add_squares(sm, tp[col], ssS, ssL);
                }
            }
        const double s1 = block_sum(ssS, red), s2 = block_sum(ssL, red);
        if (t == 0) recheck_decide(pd, A.st[p], p, row, s1, s2, d, A.gd, A.alternative, A.cnt, A.Tw);
    }
}

int recheck_segments(int max_np) { return ((max_np + 31) / 32 + kSegWords - 1) / kSegWords; }

int64_t recheck_slots(int npairs, int d_pad) {
    // a single pair has few flags; a batch gets up to 8192 slots within 128 MiB
    if (npairs <= 1) return kRecheckSlotsSingle;
    const int64_t fit = ((int64_t)128 << 20) / ((int64_t)8 * d_pad);
    return fit < kRecheckSlotsSingle ? kRecheckSlotsSingle : fit > 8192 ? 8192 : fit;
}

hipError_t launch_recheck(int input_dtype, const PairDesc* pairs, const BlockPair* bp, int npairs,
                          const PairState* st, const double* v, const double* t64, const double* coef,
                          const uint32_t* mask, const uint32_t* flags, const uint32_t* nflag, int64_t* plan,
                          int64_t max_flags, int max_np, double* rseg, int64_t slots, int d, int gd,
                          int alternative, PairCount* cnt, double* Tw, hipStream_t s) {
    if (max_flags <= 0) return hipSuccess;
    if (!plan || npairs < 1) return hipErrorInvalidValue;
    const int d_pad = (d + kDPad - 1) / kDPad * kDPad;
    if (npairs <= 64)
        hipLaunchKernelGGL(k_recheck_plan<64>, dim3(1), dim3(64), 0, s, pairs, npairs, nflag,
                           rseg ? slots : (int64_t)0, plan);
    else
        hipLaunchKernelGGL(k_recheck_plan<1024>, dim3(1), dim3(1024), 0, s, pairs, npairs, nflag,
                           rseg ? slots : (int64_t)0, plan);
    const RecheckArgs A{pairs, bp, npairs, st, v, t64, coef, mask, flags, nflag, plan,
                        d, d_pad, gd, alternative, rseg, cnt, Tw};
    // the item count is known on the device only: a grid for the largest
    // count, whose work-groups without an item return at once (a single
    // pair, whose flags are few, gets at most 1024; the work-groups loop over
    // the items when there are more)
    const int64_t gmax_grid = npairs == 1 ? 1024 : 4096;
    const int64_t want = max_flags * (int64_t)recheck_segments(max_np);
    const unsigned g = (unsigned)(want < gmax_grid ? want : gmax_grid);
    if (input_dtype == HBT_IN_F64)
        hipLaunchKernelGGL(k_recheck<double>, dim3(g), dim3(kRecheckThreads), 0, s, A);
    else
        hipLaunchKernelGGL(k_recheck<float>, dim3(g), dim3(kRecheckThreads), 0, s, A);
    if (rseg) {
        // a segmented flag takes at least two slots
        int64_t fw = slots / 2 < max_flags ? slots / 2 : max_flags;
        if (fw > gmax_grid) fw = gmax_grid;
        if (fw > 0)
            hipLaunchKernelGGL(k_recheck_finish, dim3((unsigned)fw), dim3(kRecheckThreads), 0, s, A);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// null moments: sums of T_b - T_obs and (T_b - T_obs)^2 over a block's splits,
// one work-group per pair, in a fixed order; blocks add in stream order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_moments(const BlockPair* __restrict__ bp,
                                                 const PairState* __restrict__ st,
                                                 const double* __restrict__ Tw, PairCount* cnt) {
    __shared__ double r1[256], r2[256];
    const int p = blockIdx.x;
    const BlockPair q = bp[p];
    const double c = st[p].t_obs;
    double a = 0.0, b = 0.0;
    for (int64_t k = threadIdx.x; k < q.nb; k += 256) {
        const double x = Tw[q.mrow0 + k] - c;
        a += x;
        b += x * x;
    }
    r1[threadIdx.x] = a;
    r2[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            r1[threadIdx.x] += r1[threadIdx.x + o];
            r2[threadIdx.x] += r2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cnt[p].sum_dt += r1[0];
        cnt[p].sum_dt2 += r2[0];
    }
}

hipError_t launch_moments(int npairs, const BlockPair* bp, const PairState* st, const double* Tw,
                          PairCount* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_moments, dim3(npairs), dim3(256), 0, s, bp, st, Tw, cnt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// p = (1 + count) / (B + 1)  (eq:pvalue)
// ---------------------------------------------------------------------------
__global__ void k_final(int npairs, const BlockPair* __restrict__ bp, const PairState* __restrict__ st,
                        const int32_t* __restrict__ sstat,
                        const PairCount* __restrict__ cnt, const int64_t* __restrict__ Btot,
                        hbt_result* res) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const PairState q = st[p];
    hbt_result r = res[p];
    r.count = (int64_t)cnt[p].count;
    r.n_recheck = (int64_t)cnt[p].n_recheck;
    r.B = Btot[p];
    r.p = (1.0 + (double)r.count) / ((double)r.B + 1.0);
    const double mean = cnt[p].sum_dt / (double)r.B;
    const double var = cnt[p].sum_dt2 / (double)r.B - mean * mean;
    r.t_mean = q.t_obs + mean;
    r.t_sd = var != var ? var : sqrt(var > 0.0 ? var : 0.0);
    r.status = q.status != HBT_OK ? q.status : sstat[bp[p].owner];  // the alignment's status first
    res[p] = r;
}

hipError_t launch_final(int npairs, const BlockPair* bp, const PairState* st, const int32_t* sstat,
                        const PairCount* cnt, const int64_t* Btot, hbt_result* res, hipStream_t s) {
    hipLaunchKernelGGL(k_final, dim3((npairs + 255) / 256), dim3(256), 0, s, npairs, bp, st, sstat,
                       cnt, Btot, res);
    return hipGetLastError();
}

}  // namespace hbt
