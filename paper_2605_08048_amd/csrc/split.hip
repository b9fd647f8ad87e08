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
#include <atomic>

#include "hbt_launch.h"

namespace hbt {

__device__ __forceinline__ uint32_t word_of(uint4 w, int k) {
    return k == 0 ? w.x : k == 1 ? w.y : k == 2 ? w.z : w.w;
}

// Per-wave LDS carve-up (bytes), for pairs with up to max_np pooled rows:
// the 256-bin histogram, the bucket items (index, secondary key) and the
// split's mask row.
// (The 256-bin histograms live in a static array, one per wave, so that a
// bin's LDS address is the key times 4 plus a constant.)
struct SplitLds {
    int cidx, ckey, mlds, total;
    __host__ __device__ SplitLds(int max_np) {
        cidx = 0;
        ckey = cidx + 4 * kCandCap;
        mlds = ckey + 4 * kCandCap;
        total = mlds + max_np / 8;
    }
};
constexpr int kSplitWaves = 4;          // waves (split rows) per work-group
constexpr int kSplitStaticLds = kSplitWaves * 1024;

// hist[W][key] += 1 for the 16 keys of a block.  The wave's histogram offset
// W * 1024 goes into the LDS instruction's immediate offset, so that a key
// costs one VALU operation (its byte times 4) besides the LDS add.  (Written
// as inline asm: with plain atomics the compiler merges the four waves' code
// paths and adds the offset in a register.  An add without return writes no
// register, and one wave's LDS operations complete in issue order, so the
// later reads of the histogram see every add.)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
template <int OFF>
__device__ __forceinline__ void lds_inc(uint32_t addr, uint32_t one) {
    asm volatile("ds_add_u32 %0, %1 offset:%2" : : "v"(addr), "v"(one), "i"(OFF) : "memory");
}
#pragma clang diagnostic pop
template <int W>
__device__ __forceinline__ void count_block(uint32_t (*hist)[256], uint4 w) {
    const uint32_t base = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)&hist[0][0];
    const uint32_t one = 1u;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        lds_inc<W * 1024>(base + (((word_of(w, j >> 2) >> (8 * (j & 3))) & 0xffu) << 2), one);
}

// Bit j of the result = [byte j % 4 of word j / 4 < theta] for the 16 keys of
// a block (item j's primary key, below the bucket byte theta), with four
// bytes compared at once: for each byte x and t = theta,
//   x < t  <=>  (x7 = 0 and t7 = 1) or (x7 = t7 and (x & 127) < (t & 127)),
// where (x & 127) + (128 - (t & 127)) has bit 7 set exactly when
// (x & 127) >= (t & 127) (no carry leaves the byte); one three-input logic
// operation combines the three conditions in bit 7.  The 16 flags are then
// gathered: bit 8 b + q <- byte b of word q, packed to bit 4 b + q, and the
// 4 x 4 bit matrix transposed (two delta swaps) to bit 4 q + b.
__device__ __forceinline__ uint32_t below_theta(uint4 w, uint32_t theta4) {
    const uint32_t k = 0x80808080u - (theta4 & 0x7f7f7f7fu);  // per byte 128 - (t & 127)
    // truth table of (~x & t) | (~(x ^ t) & ~s) over the operands (x, t, s)
    constexpr unsigned kTT = ((~0xF0u & 0xCCu) | (~(0xF0u ^ 0xCCu) & ~0xAAu)) & 0xffu;
    auto lt7 = [&](uint32_t x) {
        return __builtin_amdgcn_bitop3_b32(x, theta4, (x & 0x7f7f7f7fu) + k, (unsigned char)kTT);
    };
    uint32_t u = (lt7(w.x) >> 7) & 0x01010101u;
    u |= (lt7(w.y) >> 6) & 0x02020202u;
    u |= (lt7(w.z) >> 5) & 0x04040404u;
    u |= (lt7(w.w) >> 4) & 0x08080808u;
    uint32_t v = (u | (u >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0xffffu;
    uint32_t t = (v ^ (v >> 3)) & 0x0A0Au;
    v ^= t ^ (t << 3);
    t = (v ^ (v >> 6)) & 0x00CCu;
    v ^= t ^ (t << 6);
    return v;
}

// Philox block c of split b: the primary keys of items 16c .. 16c+15 as 16
// little-endian bytes.  Items at or past N get the key 0xFF; they are removed
// from the histogram's top bin afterwards and never enter group 1.
__device__ __forceinline__ uint4 primary_block(int c, int N, uint32_t b, uint32_t pair,
                                               uint32_t k0, uint32_t k1) {
    uint4 w = philox4x32_10(make_uint4((uint32_t)c, b, pair, 0u), k0, k1);
    const int lim = N - 16 * c;
    if (lim < 16) {
        auto fill = [&](uint32_t x, int base) {
            const int v = lim - base;
            return v >= 4 ? x : v <= 0 ? 0xffffffffu : x | (0xffffffffu << (8 * v));
        };
        w = make_uint4(fill(w.x, 0), fill(w.y, 4), fill(w.z, 8), fill(w.w, 12));
    }
    return w;
}

// One wave per split row.  R > 0: each lane keeps its (at most R) Philox
// blocks in registers between the histogram and the classification pass
// (pairs with N <= 1024 R); R == 0: the blocks are generated again.
template <int R>
__global__ __launch_bounds__(256) void k_split_masks(const BlockPair* __restrict__ bp, int npairs,
                                                     int64_t rows, int max_np, uint32_t key0,
                                                     uint32_t key1, uint32_t* __restrict__ mask,
                                                     int32_t* sstat, int64_t row0) {
    __shared__ uint32_t hist_all[kSplitWaves][256];
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const SplitLds L(max_np);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * kSplitWaves + wave + row0;
    if (row >= rows) return;
    unsigned char* base = smem + wave * L.total;
    uint32_t* hist = hist_all[wave];
    uint32_t* cidx = (uint32_t*)(base + L.cidx);
    uint32_t* ckey = (uint32_t*)(base + L.ckey);
    uint32_t* mlds = (uint32_t*)(base + L.mlds);

    const int p = upper_index(npairs, row, [&](int k) { return bp[k].mrow0; });
    const BlockPair pd = bp[p];   // the pair's sizes, mask row width and index (not a PairDesc)
    if (pd.owner != p) return;    // another pair's rows draw these masks (wave-uniform)
    const uint32_t b = bp[p].perm_base + (uint32_t)(row - bp[p].mrow0);
    const int N = pd.n + pd.m, n = pd.n;
    const int nc = (N + 15) >> 4;       // Philox blocks holding items
    const int nw = pd.Wp * 2;           // blocks covering the padded mask row (Np / 16)
    const int niter = (nw + 63) >> 6;   // wave-uniform

    ((uint4*)hist)[lane] = make_uint4(0u, 0u, 0u, 0u);
    wave_sync();
    // 1. primary keys and their histogram
    constexpr int RK = R > 0 ? R : 1;
    uint4 key[RK];
    auto gen_count = [&](int k) {
        const int c = 64 * k + lane;
        uint4 w = make_uint4(0u, 0u, 0u, 0u);
        if (c < nc) {
            w = primary_block(c, N, b, pd.pair_index, key0, key1);
            switch (wave) {  // wave-uniform
                case 0: count_block<0>(hist_all, w); break;
                case 1: count_block<1>(hist_all, w); break;
                case 2: count_block<2>(hist_all, w); break;
                default: count_block<3>(hist_all, w); break;
            }
        }
        return w;
    };
    if constexpr (R > 0) {
#pragma unroll
        for (int k = 0; k < R; ++k) key[k] = k < niter ? gen_count(k) : make_uint4(0u, 0u, 0u, 0u);
    } else {
        for (int k = 0; k < niter; ++k) (void)gen_count(k);
    }
    wave_sync();
    // 2. theta = the byte value holding rank n-1 (0-based); below = #{P < theta};
    //    the padding keys are taken out of bin 255 first
    uint32_t h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = hist[4 * lane + j];
    if (lane == 63) h[3] -= (uint32_t)(16 * nc - N);
    const uint32_t sum = h[0] + h[1] + h[2] + h[3];
    const uint32_t incl = wave_incl_scan(sum);
    const uint32_t excl = incl - sum;
    const bool owner = excl < (uint32_t)n && (uint32_t)n <= incl;
    uint32_t theta = 0, below = 0, bucket = 0;
    if (owner) {
        uint32_t acc = excl;
        bool found = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!found && acc + h[j] >= (uint32_t)n) {
                theta = 4 * lane + j;
                below = acc;
                bucket = h[j];
                found = true;
            }
            acc += h[j];
        }
    }
    const uint64_t own = __ballot(owner);
    const int src = __ffsll((unsigned long long)own) - 1;
    theta = __builtin_amdgcn_readlane(theta, src);
    below = __builtin_amdgcn_readlane(below, src);
    bucket = __builtin_amdgcn_readlane(bucket, src);
    const uint32_t need = (uint32_t)n - below;
    if (bucket > (uint32_t)kCandCap) {  // not seen in practice (expected size N / 256)
        if (lane == 0) atomicExch(&sstat[p], (int)HBT_ERR_INTERNAL);
        uint32_t* out = const_cast<uint32_t*>(mask_row(mask, bp[p], row, pd.Wp));
        for (int w = lane; w < pd.Wp; w += 64) out[w] = 0u;  // an empty group: nothing to gather
        return;
    }
    // 3. classification: each lane builds the 16 bits "P < theta" of its
    //    block, two neighbouring lanes form one 32-bit mask word; blocks that
    //    hold a byte equal to theta (a few per split) list those items
    const uint32_t theta4 = theta * 0x01010101u;
    uint32_t cbase = 0;  // bucket items listed so far (wave-uniform)
    auto classify = [&](int k, uint4 w) {
        const int c = 64 * k + lane;
        uint32_t lt = below_theta(w, theta4);
        // bit 7 of each byte equal to theta (exact), gathered into one word:
        // bit 8 b + q marks item 4 q + b of the block
        uint32_t eq = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t x = word_of(w, q) ^ theta4;
            const uint32_t z = ~(((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u;
            eq |= z >> (7 - q);
        }
        if (c >= nc) {
            lt = 0u;
            eq = 0u;
        } else if (16 * c + 16 > N) {  // tail block: drop the padding items (keys 0xFF)
            for (int j = N - 16 * c; j < 16; ++j) eq &= ~(1u << (8 * (j & 3) + (j >> 2)));
        }
        const uint32_t ne = (uint32_t)__popc(eq);
        const uint32_t incl = wave_incl_scan(ne);
        uint32_t pos = cbase + incl - ne;
        cbase += __builtin_amdgcn_readlane(incl, 63);
        while (eq) {
            const int t = __ffs(eq) - 1;
            cidx[pos++] = (uint32_t)(16 * c + 4 * (t & 7) + (t >> 3));
            eq &= eq - 1u;
        }
        // lane ^ 1's bits (quad_perm [1,0,3,2])
        const uint32_t nb = (uint32_t)__builtin_amdgcn_mov_dpp((int)lt, 0xB1, 0xF, 0xF, false);
        if (!(lane & 1) && c < nw) mlds[c >> 1] = lt | (nb << 16);
    };
    if constexpr (R > 0) {
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (k < niter) classify(k, key[k]);  // wave-uniform
    } else {
        for (int k = 0; k < niter; ++k) {
            const int c = 64 * k + lane;
            classify(k, c < nc ? primary_block(c, N, b, pd.pair_index, key0, key1) : make_uint4(0u, 0u, 0u, 0u));
        }
    }
    wave_sync();
    const uint32_t cnt = bucket;
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
        // (S, i) order as one 64-bit key
        const uint64_t key = ((uint64_t)sk << 32) | ik;
        uint32_t rank = 0;
        for (uint32_t q = 0; q < cnt; ++q) {
            const uint64_t k2 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(sk, q) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane(ik, q);
            rank += k2 < key;
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
    if (pd.ygap == 0) {
        for (int w = lane; w < pd.Wp; w += 64) out[w] = mlds[w];
    } else {
        // two-run storage: X's items keep their positions, Y's move ygap
        // positions on (X's padding in between); n + ygap is a multiple of 128
        const int ys = n + pd.ygap;
        for (int w = lane; w < pd.Wp; w += 64) {
            uint32_t x;
            if (32 * w < ys) {
                x = mlds[w] & range_bits(w, 0, n);
            } else {
                const int p0 = 32 * w - pd.ygap, q = p0 >> 5, sh = p0 & 31;
                const uint32_t a = mlds[q], b = q + 1 < pd.Wp ? mlds[q + 1] : 0u;
                x = sh ? (a >> sh) | (b << (32 - sh)) : a;
                x &= range_bits(w, ys, ys + pd.m);
            }
            out[w] = x;
        }
    }
}

// LDS of one CU (160 KB on MI355X), from the device.
static size_t lds_per_cu() {
    static std::atomic<size_t> v{0};
    size_t x = v.load(std::memory_order_relaxed);
    if (!x) {
        int dev = 0, a = 0;
        x = (hipGetDevice(&dev) == hipSuccess &&
             hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
             a > 0) ? (size_t)a : 163840;
        v.store(x, std::memory_order_relaxed);
    }
    return x;
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

size_t split_lds_per_block(int max_np) { return (size_t)kSplitWaves * SplitLds(max_np).total + kSplitStaticLds; }

hipError_t launch_split_masks(const BlockPair* bp, int npairs,
                              int64_t rows, int max_np, uint64_t seed, uint32_t* mask,
                              int32_t* sstat, int wg_per_cu, hipStream_t s, int64_t row0) {
    if (rows <= row0) return hipSuccess;
    const SplitLds L(max_np);
    // four split rows per work-group; at most 64 KB of LDS per work-group
    size_t lds = (size_t)kSplitWaves * L.total;
    if (wg_per_cu > 0) {
        const size_t share = lds_per_cu() / (size_t)wg_per_cu;
        if (share > lds + kSplitStaticLds) lds = share - kSplitStaticLds;
    }
    if (lds + kSplitStaticLds > 65536 || lds + kSplitStaticLds > split_lds_limit()) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((rows - row0 + kSplitWaves - 1) / kSplitWaves)), block(64 * kSplitWaves);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    // registers for the keys of the largest pair: R blocks of 16 per lane
    const int r = (max_np + 1023) / 1024;
#define HBT_SPLIT(RR) hipLaunchKernelGGL(k_split_masks<RR>, grid, block, lds, s, bp, npairs, rows, max_np, k0, k1, mask, sstat, row0)
    if (r <= 1) HBT_SPLIT(1);
    else if (r <= 2) HBT_SPLIT(2);
    else if (r <= 4) HBT_SPLIT(4);
    else if (r <= 8) HBT_SPLIT(8);
    else if (r <= 12) HBT_SPLIT(12);
    else if (r <= 16) HBT_SPLIT(16);
    else HBT_SPLIT(0);
#undef HBT_SPLIT
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// explicit masks: copy + validate (exactly n items, no bits at or beyond N)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_copy_masks(const uint32_t* __restrict__ user,
                                                    int64_t rows, int N, int n, int Wp,
                                                    uint32_t* __restrict__ mask, int32_t* sstat) {
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
    if (lane == 0 && (pc != n || anybad)) atomicExch(sstat, (int)HBT_ERR_MASK);
}

hipError_t launch_copy_masks(const uint32_t* user, int64_t user_row0, int64_t rows, int N, int n,
                             int Wp, uint32_t* mask, int32_t* sstat, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const int W = (N + 31) >> 5;
    hipLaunchKernelGGL(k_copy_masks, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s,
                       user + user_row0 * W, rows, N, n, Wp, mask, sstat);
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
