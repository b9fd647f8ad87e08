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
            const bool border = !no_recheck && !nan && fabs(val - thr) <= eps;
            if (border) {
                const uint32_t k = atomicAdd(nflag, 1u);
                flags[k] = (uint32_t)row;
            } else {
                exceed = nan || val >= thr;
            }
        }
    }
    if (MODE == kStatLazyFirst) {
        // list appends: one atomic per wave when all its rows belong to one pair
        const uint64_t rm = __ballot(refine);
        if (one_pair) {
            uint32_t base = 0;
            if (lane_id() == 0 && rm) base = atomicAdd(&rcnt[p0], (uint32_t)__popcll(rm));
            base = (uint32_t)__shfl((int)base, 0, 64);
            if (refine) rlist[bp[p0].mrow0 + base + mbcnt64(rm)] = (uint32_t)row;
        } else if (refine) {
            const uint32_t k = atomicAdd(&rcnt[p], 1u);
            rlist[bp[p].mrow0 + k] = (uint32_t)row;
        }
    }
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
// x_i - coef_i v (X) or y_j (Y); the other group's sum is t - sigma_small
// with the FP64 pooled total t.
//
// The gather over a split's mask words is cut into segments of kSegWords
// words (512 pooled rows); wave w of a work-group walks words w, w + 8, ...
// of a segment.  sigma_small is always formed in one order: per wave, its
// segment sums added in segment order; then the 8 waves' totals added in
// wave order.  The first f_seg flags of the list (when segments are enabled)
// are split into one work item per segment, whose per-wave sums go to
// workspace slots that k_recheck_finish adds in that order; this puts many
// work-groups on a call with few flags.  Every other flag is done whole by
// one work-group whose waves keep their running totals in registers.  The
// value of a flag's sums therefore does not depend on how the work is
// spread.  512 threads, columns in passes of 768.
// ---------------------------------------------------------------------------
constexpr int kRecheckWaves = kRecheckSegRows;  // 8
constexpr int kRecheckThreads = 64 * kRecheckWaves;
constexpr int kRecheckPass = 768;        // columns per pass (12 per lane)
constexpr int kSegWords = 16;

struct FlagCtx {
    int64_t row;
    int p, N, W, G;
    PairDesc pd;
    PairState q;
    const uint32_t* mk;
};

__device__ __forceinline__ FlagCtx flag_ctx(const PairDesc* pairs, const BlockPair* bp, int npairs,
                                            const PairState* st, const uint32_t* mask,
                                            const uint32_t* flags, uint32_t f) {
    FlagCtx c;
    c.row = flags[f];
    c.p = upper_index(npairs, c.row, [&](int k) { return bp[k].mrow0; });
    c.pd = pairs[c.p];
    c.q = st[c.p];
    c.mk = mask_row(mask, bp[c.p], c.row, c.pd.Wp);
    c.N = c.pd.n + c.pd.m;
    c.W = (c.N + c.pd.ygap + 31) >> 5;  // mask words that hold items (Y's start ygap further on)
    c.G = (c.W + kSegWords - 1) / kSegWords;
    return c;
}

// The flag's statistic from the per-thread sums of squares (thread t holds
// the columns c0 + t + 512 k of every pass, in that order), its decision and
// its FP64 T_b.
__device__ void recheck_finish_flag(const FlagCtx& c, double ss_small, double ss_large, int d,
                                    int gd, int alternative, PairCount* cnt, double* Tw,
                                    double* red1, double* red2) {
    red1[threadIdx.x] = ss_small;
    red2[threadIdx.x] = ss_large;
    __syncthreads();
    for (int o = kRecheckThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            red1[threadIdx.x] += red1[threadIdx.x + o];
            red2[threadIdx.x] += red2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double dd = (double)d;
        const double ss1 = c.pd.flip ? red2[0] : red1[0];
        const double ss2 = c.pd.flip ? red1[0] : red2[0];
        const double r1 = sqrt(ss1) / (double)c.pd.n, r2 = sqrt(ss2) / (double)c.pd.m;
        const double T = log_g(r2, dd, gd) - log_g(r1, dd, gd);
        const bool two = alternative == HBT_ALT_TWO_SIDED;
        const double val = two ? fabs(T) : T;
        const double thr = (two ? fabs(c.q.t_obs) : c.q.t_obs) - c.q.tau;
        if (T != T || val >= thr) atomicAdd(&cnt[c.p].count, 1ull);
        atomicAdd(&cnt[c.p].n_recheck, 1ull);
        Tw[c.row] = T;
    }
    __syncthreads();
}

template <typename Tin>
__global__ __launch_bounds__(kRecheckThreads) void k_recheck(
    const PairDesc* __restrict__ pairs, const BlockPair* __restrict__ bp, int npairs,
    const PairState* __restrict__ st, const double* __restrict__ v,
    const double* __restrict__ t64, const double* __restrict__ coef,
    const uint32_t* __restrict__ mask, const uint32_t* __restrict__ flags,
    const uint32_t* __restrict__ nflag, int d, int d_pad, int gd, int alternative,
    double* __restrict__ rseg, int f_seg, int g_max, PairCount* cnt, double* __restrict__ Tw) {
    constexpr int kU = kRecheckPass / 64;  // columns per lane per pass
    constexpr int kRows = 4;               // rows in flight per wave
    __shared__ double part[kRecheckWaves][kRecheckPass];  // per-wave partial group sums
    __shared__ double red1[kRecheckThreads], red2[kRecheckThreads];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const uint32_t total = *nflag;
    const int64_t nseg = total < (uint32_t)f_seg ? (int64_t)total : (int64_t)f_seg;
    const int64_t nitems = nseg * g_max + ((int64_t)total - nseg);
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const bool whole = it >= nseg * g_max;
        const uint32_t f = whole ? (uint32_t)(nseg + (it - nseg * g_max)) : (uint32_t)(it / g_max);
        const int sg = whole ? 0 : (int)(it % g_max);
        const FlagCtx c = flag_ctx(pairs, bp, npairs, st, mask, flags, f);
        if (!whole && sg >= c.G) continue;  // work-group-uniform
        const int s0 = sg, s1 = whole ? c.G : sg + 1;
        const PairDesc& pd = c.pd;
        const double* vp = v + (int64_t)c.p * d_pad;
        const double* tp = t64 + (int64_t)c.p * d_pad;
        const double* cf = coef + pd.coef0;
        const uint32_t flip = pd.flip ? 0xffffffffu : 0u;
        const Tin* X = (const Tin*)pd.X;
        const Tin* Y = (const Tin*)pd.Y;
        const int W = c.W;
        // members of the smaller group in mask word w
        auto word_bits = [&](int w, int wend) -> uint32_t {
            if (w >= wend) return 0u;
            return (c.mk[w] ^ flip) & item_bits(w, pd.n, pd.m, pd.ygap);
        };
        double ss_small = 0.0, ss_large = 0.0;
        for (int c0 = 0; c0 < d; c0 += kRecheckPass) {
            double vc[kU], tot[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int col = c0 + 64 * u + lane;
                vc[u] = col < d ? vp[col] : 0.0;
                tot[u] = 0.0;
            }
            for (int sgi = s0; sgi < s1; ++sgi) {
                const int wend = min(W, (sgi + 1) * kSegWords);
                double acc[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) acc[u] = 0.0;
                // kRows rows at a time, all loads issued before the adds
                int w = sgi * kSegWords + wave;
                uint32_t bits = word_bits(w, wend);
                for (;;) {
                    int rows[kRows];
#pragma unroll
                    for (int t = 0; t < kRows; ++t) {
                        while (!bits && w < wend) {
                            w += kRecheckWaves;
                            bits = word_bits(w, wend);
                        }
                        if (bits) {
                            rows[t] = 32 * w + __builtin_ctz(bits);
                            bits &= bits - 1u;
                        } else {
                            rows[t] = -1;
                        }
                    }
                    if (rows[0] < 0) break;
                    // columns are clamped to the row (no branch around a load);
                    // absent rows and clamped columns are weighted by 0
                    Tin z[kRows][kU];
                    double kc[kRows], wt[kRows];
#pragma unroll
                    for (int t = 0; t < kRows; ++t) {
                        int i = rows[t] < 0 ? 0 : rows[t];
                        if (i >= pd.n) i -= pd.ygap;  // Y's mask positions to pooled items
                        const bool isx = i < pd.n;
                        kc[t] = (rows[t] >= 0 && isx) ? cf[i] : 0.0;
                        wt[t] = rows[t] >= 0 ? 1.0 : 0.0;
                        const Tin* src = isx ? X + (int64_t)i * d : Y + (int64_t)(i - pd.n) * d;
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int col = c0 + 64 * u + lane;
                            z[t][u] = src[col < d ? col : d - 1];
                        }
                    }
#pragma unroll
                    for (int t = 0; t < kRows; ++t)
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const double cm = (c0 + 64 * u + lane) < d ? wt[t] : 0.0;
                            acc[u] += cm * ((double)z[t][u] - kc[t] * vc[u]);
                        }
                }
                if (whole) {
#pragma unroll
                    for (int u = 0; u < kU; ++u) tot[u] += acc[u];
                } else {
                    double* dst = rseg + (((int64_t)f * g_max + sgi) * kRecheckWaves + wave) * d_pad + c0;
#pragma unroll
                    for (int u = 0; u < kU; ++u)
                        if (c0 + 64 * u + lane < d) dst[64 * u + lane] = acc[u];
                }
            }
            if (whole) {
#pragma unroll
                for (int u = 0; u < kU; ++u) part[wave][64 * u + lane] = tot[u];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int cc = threadIdx.x + kRecheckThreads * k;
                    if (cc < kRecheckPass && c0 + cc < d) {
                        double sm = 0.0;
#pragma unroll
                        for (int q = 0; q < kRecheckWaves; ++q) sm += part[q][cc];
                        const double l = tp[c0 + cc] - sm;
                        ss_small += sm * sm;
                        ss_large += l * l;
                    }
                }
                __syncthreads();
            }
        }
        if (whole) recheck_finish_flag(c, ss_small, ss_large, d, gd, alternative, cnt, Tw, red1, red2);
    }
}

// The segmented flags: sigma_small from the per-wave segment sums in the
// order above, then the same statistic and decision as a whole flag.
__global__ __launch_bounds__(kRecheckThreads) void k_recheck_finish(
    const PairDesc* __restrict__ pairs, const BlockPair* __restrict__ bp, int npairs,
    const PairState* __restrict__ st, const double* __restrict__ t64,
    const uint32_t* __restrict__ mask, const uint32_t* __restrict__ flags,
    const uint32_t* __restrict__ nflag, int d, int d_pad, int gd, int alternative,
    const double* __restrict__ rseg, int f_seg, int g_max, PairCount* cnt, double* __restrict__ Tw) {
    __shared__ double red1[kRecheckThreads], red2[kRecheckThreads];
    const uint32_t total = *nflag;
    const uint32_t f = blockIdx.x;
    if (f >= total || f >= (uint32_t)f_seg) return;
    const FlagCtx c = flag_ctx(pairs, bp, npairs, st, mask, flags, f);
    const double* tp = t64 + (int64_t)c.p * d_pad;
    double ss_small = 0.0, ss_large = 0.0;
    for (int c0 = 0; c0 < d; c0 += kRecheckPass)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int cc = threadIdx.x + kRecheckThreads * k;
            if (cc < kRecheckPass && c0 + cc < d) {
                // the 8 wave totals are independent chains: each segment's 8
                // loads are issued together
                double t[kRecheckWaves];
#pragma unroll
                for (int q = 0; q < kRecheckWaves; ++q) t[q] = 0.0;
                const double* src = rseg + (int64_t)f * g_max * kRecheckWaves * d_pad + c0 + cc;
                for (int sgi = 0; sgi < c.G; ++sgi) {
                    double x[kRecheckWaves];
#pragma unroll
                    for (int q = 0; q < kRecheckWaves; ++q) x[q] = src[((int64_t)sgi * kRecheckWaves + q) * d_pad];
#pragma unroll
                    for (int q = 0; q < kRecheckWaves; ++q) t[q] += x[q];
                }
                double sm = 0.0;
#pragma unroll
                for (int q = 0; q < kRecheckWaves; ++q) sm += t[q];
                const double l = tp[c0 + cc] - sm;
                ss_small += sm * sm;
                ss_large += l * l;
            }
        }
    recheck_finish_flag(c, ss_small, ss_large, d, gd, alternative, cnt, Tw, red1, red2);
}

int recheck_segments(int max_np) { return ((max_np + 31) / 32 + kSegWords - 1) / kSegWords; }

int recheck_seg_flags(int max_np) {
    const int g = recheck_segments(max_np);
    return g > 1 ? kRecheckSegSlots / g : 0;
}

hipError_t launch_recheck(int input_dtype, const PairDesc* pairs, const BlockPair* bp,
                          int npairs, const PairState* st, const double* v, const double* t64,
                          const double* coef, const uint32_t* mask, const uint32_t* flags,
                          const uint32_t* nflag, int64_t max_flags, int max_np, double* rseg, int d,
                          int gd, int alternative, PairCount* cnt, double* Tw, hipStream_t s) {
    if (max_flags <= 0) return hipSuccess;
    const int d_pad = (d + kDPad - 1) / kDPad * kDPad;
    const int g_max = recheck_segments(max_np);
    int f_seg = rseg ? recheck_seg_flags(max_np) : 0;
    if (f_seg > max_flags) f_seg = (int)max_flags;
    // enough work-groups for every segment of the segmented flags
    const int64_t want = max_flags + (int64_t)f_seg * (g_max - 1);
    const unsigned g = (unsigned)(want < 4096 ? want : 4096);
    if (input_dtype == HBT_IN_F64)
        hipLaunchKernelGGL(k_recheck<double>, dim3(g), dim3(kRecheckThreads), 0, s, pairs, bp, npairs,
                           st, v, t64, coef, mask, flags, nflag, d, d_pad, gd, alternative, rseg, f_seg,
                           g_max, cnt, Tw);
    else
        hipLaunchKernelGGL(k_recheck<float>, dim3(g), dim3(kRecheckThreads), 0, s, pairs, bp, npairs,
                           st, v, t64, coef, mask, flags, nflag, d, d_pad, gd, alternative, rseg, f_seg,
                           g_max, cnt, Tw);
    if (f_seg > 0)
        hipLaunchKernelGGL(k_recheck_finish, dim3((unsigned)f_seg), dim3(kRecheckThreads), 0, s, pairs, bp,
                           npairs, st, t64, mask, flags, nflag, d, d_pad, gd, alternative, rseg, f_seg,
                           g_max, cnt, Tw);
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
