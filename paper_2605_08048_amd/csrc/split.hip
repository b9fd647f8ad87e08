// Random splits of the pooled set into groups of sizes (n, m): the "randomly
// partition Z" step of Algorithm 1 / the sign-matrix rows of Algorithm 2,
// stored as a 0/1 bit mask of group 1.
//
// Split b of a pair puts in group 1 the n items first in the order
// (P_i, S_i, i): P_i an 8-bit primary key, S_i a 32-bit secondary key, both
// from Philox4x32-10 (counter (i/16, b, pair, 0) and (i/4, b, pair, 1)).
// Selection without a sort: a 256-bin histogram of P finds the byte theta
// holding rank n-1; items with P < theta are in; the ~N/256 items with
// P == theta are ranked by (S_i, i) and the first n - #{P < theta} join.
// Only those bucket items ever need a secondary key.
//
// One wavefront per split row; waves of a work-group are independent and
// synchronise only within themselves.
#include "hbt_launch.h"

namespace hbt {

__device__ __forceinline__ uint32_t word_of(uint4 w, int k) {
    return k == 0 ? w.x : k == 1 ? w.y : k == 2 ? w.z : w.w;
}

// Per-wave LDS carve-up (bytes), for pairs with up to max_np pooled rows.
struct SplitLds {
    int keys, hist, mlds, cidx, ckey, total;
    __host__ __device__ SplitLds(int max_np) {
        keys = 0;
        hist = max_np;
        mlds = hist + 1024;
        cidx = mlds + max_np / 8;
        ckey = cidx + 4 * kCandCap;
        total = ckey + 4 * kCandCap;
    }
};

__global__ __launch_bounds__(256) void k_split_masks(const PairDesc* __restrict__ pairs,
                                                     const BlockPair* __restrict__ bp, int npairs,
                                                     int64_t rows, int max_np, uint32_t key0,
                                                     uint32_t key1, uint32_t* __restrict__ mask,
                                                     PairState* st) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const SplitLds L(max_np);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (row >= rows) return;
    unsigned char* base = smem + wave * L.total;
    unsigned char* keys = base + L.keys;
    uint32_t* hist = (uint32_t*)(base + L.hist);
    uint32_t* mlds = (uint32_t*)(base + L.mlds);
    uint32_t* cidx = (uint32_t*)(base + L.cidx);
    uint32_t* ckey = (uint32_t*)(base + L.ckey);

    const int p = upper_index(npairs, row, [&](int k) { return bp[k].mrow0; });
    const PairDesc pd = pairs[p];
    const uint32_t b = bp[p].perm_base + (uint32_t)(row - bp[p].mrow0);
    const int N = pd.n + pd.m, n = pd.n;

    for (int j = lane; j < 256; j += 64) hist[j] = 0;
    wave_sync();
    // 1. primary keys: 16 per Philox block; histogram of their values
    const int nc = (N + 15) >> 4;
    for (int c = lane; c < nc; c += 64) {
        const uint4 w = philox4x32_10(make_uint4((uint32_t)c, b, pd.pair_index, 0u), key0, key1);
        ((uint4*)keys)[c] = w;
        const int lim = N - 16 * c;
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < lim) atomicAdd(&hist[(word_of(w, j >> 2) >> (8 * (j & 3))) & 0xffu], 1u);
    }
    wave_sync();
    // 2. theta = the byte value holding rank n-1 (0-based); below = #{P < theta}
    uint32_t h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = hist[4 * lane + j];
    const uint32_t sum = h[0] + h[1] + h[2] + h[3];
    const uint32_t incl = wave_incl_scan(sum);
    const uint32_t excl = incl - sum;
    const bool owner = excl < (uint32_t)n && (uint32_t)n <= incl;
    uint32_t theta = 0, below = 0;
    if (owner) {
        // the first bin (from the left) where the running count reaches n
        uint32_t acc = excl;
        bool found = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!found && acc + h[j] >= (uint32_t)n) {
                theta = 4 * lane + j;
                below = acc;
                found = true;
            }
            acc += h[j];
        }
    }
    const uint64_t own = __ballot(owner);
    const int src = __ffsll((unsigned long long)own) - 1;
    theta = __shfl(theta, src, 64);
    below = __shfl(below, src, 64);
    const uint32_t need = (uint32_t)n - below;
    // 3. one pass over the keys: bits of P < theta, and the bucket P == theta.
    //    Four independent byte reads per lane per iteration (items i0 + l + 64 t)
    //    keep several LDS reads in flight; each ballot is one 64-item mask slice.
    uint32_t cnt = 0;
    for (int i0 = 0; i0 < pd.Np; i0 += 256) {
        uint32_t P[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int i = i0 + 64 * t + lane;
            P[t] = i < pd.Np ? (uint32_t)keys[i] : 0u;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ib = i0 + 64 * t;
            if (ib >= pd.Np) break;
            const int i = ib + lane;
            const bool in = i < N;
            const uint64_t lt = __ballot(in && P[t] < theta);
            const uint64_t eq = __ballot(in && P[t] == theta);
            if (lane == 0) {
                mlds[ib >> 5] = (uint32_t)lt;
                mlds[(ib >> 5) + 1] = (uint32_t)(lt >> 32);
            }
            if (in && P[t] == theta) {
                const uint32_t pos = cnt + mbcnt64(eq);
                if (pos < (uint32_t)kCandCap) cidx[pos] = (uint32_t)i;
            }
            cnt += (uint32_t)__popcll((unsigned long long)eq);
        }
    }
    if (cnt > (uint32_t)kCandCap) {
        if (lane == 0) atomicExch(&st[p].status, (int)HBT_ERR_INTERNAL);
        cnt = kCandCap;
    }
    wave_sync();
    // 4. secondary keys of the bucket items; 5. the `need` bucket items first in
    //    (S, i) order join group 1.  With at most 64 bucket items (the usual
    //    case: about N / 256) each lane holds one and ranks it against the
    //    others through lane broadcasts; larger buckets rank through LDS.
    if (cnt <= 64) {
        uint32_t sk = 0xffffffffu, ik = 0xffffffffu;
        if ((uint32_t)lane < cnt) {
            ik = cidx[lane];
            const uint4 w = philox4x32_10(make_uint4(ik >> 2, b, pd.pair_index, 1u), key0, key1);
            sk = word_of(w, ik & 3);
        }
        uint32_t rank = 0;
        for (uint32_t q = 0; q < cnt; ++q) {
            const uint32_t s2 = __builtin_amdgcn_readlane(sk, q);
            const uint32_t i2 = __builtin_amdgcn_readlane(ik, q);
            rank += (s2 < sk) || (s2 == sk && i2 < ik);
        }
        if ((uint32_t)lane < cnt && rank < need) atomicOr(&mlds[ik >> 5], 1u << (ik & 31));
    } else {
        for (uint32_t k = lane; k < cnt; k += 64) {
            const uint32_t i = cidx[k];
            const uint4 w = philox4x32_10(make_uint4(i >> 2, b, pd.pair_index, 1u), key0, key1);
            ckey[k] = word_of(w, i & 3);
        }
        wave_sync();
        for (uint32_t k = lane; k < cnt; k += 64) {
            const uint32_t sk = ckey[k], ik = cidx[k];
            uint32_t rank = 0;
            for (uint32_t q = 0; q < cnt; ++q) {
                const uint32_t s2 = ckey[q], i2 = cidx[q];
                rank += (s2 < sk) || (s2 == sk && i2 < ik);
            }
            if (rank < need) atomicOr(&mlds[ik >> 5], 1u << (ik & 31));
        }
    }
    wave_sync();
    uint32_t* out = const_cast<uint32_t*>(mask_row(mask, bp[p], row, pd.Wp));
    for (int w = lane; w < pd.Wp; w += 64) out[w] = mlds[w];
}

size_t split_lds_limit() {
    static size_t lim = 0;
    if (!lim) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            lim = (size_t)v;
        else
            lim = 65536;
    }
    return lim;
}

size_t split_lds_per_wave(int max_np) { return (size_t)SplitLds(max_np).total; }

hipError_t launch_split_masks(const PairDesc* pairs, const BlockPair* bp, int npairs,
                              int64_t rows, int max_np, uint64_t seed, uint32_t* mask,
                              PairState* st, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const SplitLds L(max_np);
    // at most 64 KB of LDS per work-group
    const size_t cap = split_lds_limit() < 65536 ? split_lds_limit() : 65536;
    int waves = (int)(cap / (size_t)L.total);
    if (waves > 4) waves = 4;
    if (waves < 1) return hipErrorInvalidValue;
    const size_t lds = (size_t)waves * L.total;
    hipLaunchKernelGGL(k_split_masks, dim3((unsigned)((rows + waves - 1) / waves)), dim3(64 * waves),
                       lds, s, pairs,
                       bp, npairs, rows, max_np, (uint32_t)seed, (uint32_t)(seed >> 32), mask, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// explicit masks: copy + validate (exactly n items, no bits at or beyond N)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_copy_masks(const uint32_t* __restrict__ user,
                                                    int64_t rows, int N, int n, int Wp,
                                                    uint32_t* __restrict__ mask, PairState* st) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + wave;
    if (row >= rows) return;
    const int W = (N + 31) >> 5;
    int pc = 0;
    bool bad = false;
    for (int w = lane; w < Wp; w += 64) {
        uint32_t x = w < W ? user[row * W + w] : 0u;
        if (w == W - 1 && (N & 31)) {
            bad |= (x >> (N & 31)) != 0u;
        }
        pc += __popc(x);
        mask[row * Wp + w] = x;
    }
    for (int o = 32; o > 0; o >>= 1) pc += __shfl_xor(pc, o, 64);
    const bool anybad = __ballot(bad) != 0;
    if (lane == 0 && (pc != n || anybad)) atomicExch(&st->status, (int)HBT_ERR_MASK);
}

hipError_t launch_copy_masks(const uint32_t* user, int64_t user_row0, int64_t rows, int N, int n,
                             int Wp, uint32_t* mask, PairState* st, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const int W = (N + 31) >> 5;
    hipLaunchKernelGGL(k_copy_masks, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s,
                       user + user_row0 * W, rows, N, n, Wp, mask, st);
    return hipGetLastError();
}

__global__ void k_export_masks(const uint32_t* __restrict__ mask, int64_t rows, int Wp, int W,
                               uint32_t* __restrict__ out) {
    const int64_t total = rows * W;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = k / W;
        out[k] = mask[r * Wp + (k - r * W)];
    }
}

hipError_t launch_export_masks(const uint32_t* mask, int64_t rows, int Wp, int W, uint32_t* out,
                               hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    int64_t g = (rows * W + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_export_masks, dim3((unsigned)g), dim3(256), 0, s, mask, rows, Wp, W, out);
    return hipGetLastError();
}

}  // namespace hbt
