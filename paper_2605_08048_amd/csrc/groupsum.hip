// Group sums of all splits of a block as one matrix product (eq:gemm,
// Algorithm 2), on MFMA, with the squared norms of both groups reduced in
// the epilogue so the B0 x d sums are never stored.
//
// With M_small the 0/1 mask of the smaller group (B0 x Np) and Z (Np x d):
//   sigma_small = M_small . Z,   sigma_large = t - sigma_small   (t = 1^T Z)
// (the paper's U = S X with S = 2 M - 1 carries the same information; the
// 0/1 form on the smaller group keeps t - sigma well conditioned and is exact
// in BF16).  The product is computed transposed, C = Z^T M_small^T (d x B0),
// so that each lane of an MFMA result holds one split (column) and several
// columns of d (rows): the per-split norm reduction is then mostly in-lane.
//
// Output per split row and per slot of kDSlot columns, slot-major (prow rows
// per slot, so a tile's stores and the statistic's loads are contiguous):
//   partial[slot][row] = (sum_c sigma_small[c]^2, sum_c (t[c] - sigma_small[c])^2)
//
// Tile = kDSlot columns x (1024 splits for split BF16 with eight waves, or
// 256 with four; 256 for FP32 / FP64 and the int8 digit planes).
#include <atomic>
#include <type_traits>

#include "hbt_launch.h"

namespace hbt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

// ---------------------------------------------------------------------------
// split BF16: z = hi + lo, C += Z_hi^T M + Z_lo^T M, FP32 accumulation
// v_mfma_f32_32x32x16_bf16: A (32 x 16) lane l -> row l%32, k 8(l/32)..+7;
// B (16 x 32) lane l -> k 8(l/32)..+7, col l%32; D lane l -> col l%32,
// rows 8(v/4) + 4(l/32) + v%4.
//
// Work-group tile: 64 columns x 1024 splits (kTileWide); 8 waves, wave w owns
// splits [128 w, 128 w + 128) as 4 blocks of 32 and the 64 columns as 2
// blocks of 32 (accumulators 2 x 4 x 16 floats per lane).  The narrow width
// (256 splits) has 4 waves of 64 splits.
//  * Z streams through LDS in chunks of 128 pooled rows (16 octets; both
//    planes of the 64-column slice = 32 KB) with direct global -> LDS loads,
//    one chunk ahead, into two buffers; each chunk feeds all waves of the
//    work-group, so the wide tile reads each Z slice once per 1024 splits.
//  * Mask words become bf16 operands with one AND per register: a set bit
//    lands in the exponent field (a power of two, not 1), and the stored
//    planes hold each row divided by the power its bit meets, in the row
//    order that makes this work (bf16_plane_row); no table, no LDS traffic.
//  * Operands of K-step s+1 are read while the MFMAs of K-step s run.
//  * Tiles are numbered so that the b-tiles of one (pair, column slice) go to
//    one XCD (work-groups are dealt to the 8 XCDs round-robin), and the pair
//    order is longest-first.
// ---------------------------------------------------------------------------
constexpr int kChunk = 128;                      // pooled rows per chunk
constexpr int kOct = kChunk / 8;                 // octets per chunk
constexpr int kChunkVec = 2 * kOct * kDSlot;     // uint4 per chunk (both planes)
constexpr int kXcd = 8;                          // XCDs of an MI355X

// One 16-byte-per-lane direct load from global memory into LDS: lane l's
// 16 bytes land at LDS address lds + 16 l (M0 holds the wave's base).  Issued
// as inline asm so that the compiler inserts no waits of its own for these
// LDS writes: the kernel waits for them explicitly (vmcnt) before a barrier.
// M0 is declared clobbered; no code generated for this kernel reads M0
// otherwise, so nothing of the compiler's lives there across the statement.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void dma16(const void* src, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(src), "s"(lds)
                 : "memory", "m0");
}
#pragma clang diagnostic pop

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// Work-group barrier without a memory fence.  __syncthreads() would also
// drain every outstanding global load, including the direct-to-LDS loads of
// the chunks still in flight; the explicit s_waitcnt before each barrier
// orders exactly the loads that must have landed, and every LDS read of the
// previous chunk has been consumed by an MFMA before the barrier.  The empty
// asm statements keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Work-group g -> logical tile: within each block of 32 consecutive
// work-groups, XCD x (= g mod 8) receives the 4 consecutive logical tiles
// 4x .. 4x+3.  A permutation of [0, round_up(T, 32)).
__device__ __forceinline__ int xcd_remap(int g) {
    return 32 * (g / 32) + 4 * (g % kXcd) + (g / kXcd) % 4;
}

// s_waitcnt operand: at most `loads` vector-memory operations outstanding (one
// chunk's direct-to-LDS loads of a wave), no wait on export or LDS counters
// (gfx9 encoding: vmcnt [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8])
constexpr int wait_vmcnt(int loads) { return (loads & 0xf) | ((loads >> 4) << 14) | (0x7 << 4) | (0xf << 8); }

// JB split blocks of 32 per wave, NW waves: a work-group covers 32 JB NW
// splits (JB = 4, NW = 8: 1024; JB = 2, NW = 4: 256; the tile width the plan
// picks per pair).  Each wave loads 32 / NW of the chunk's 32 octet rows.
//
// Persistent launch: work-group b walks the tiles b, b + G, b + 2G, ...
// (G = gridDim.x; tiles are numbered longest pair first), and the chunk
// loader runs one chunk ahead of the multiplication across tile boundaries,
// so the first chunk of the next tile streams in during the last step and
// the epilogue of the current one.  Chunk g of a work-group's sequence goes to
// LDS buffer g mod 2; the step that multiplies chunk g issues chunk g + 1 into
// the other buffer, which every wave finished reading in the previous step.
// Two waves per SIMD (at most 256 registers per lane): the wide tile is one
// work-group of 8 waves per CU (two buffers, 96 KB of LDS), the narrow one
// two work-groups of 4 (72 KB each), so that a wave's barriers, waits and
// epilogue overlap the other waves' MFMAs.  On 512 pairs, d = 768: 4 waves x
// 512 splits with two work-groups per CU 4.18 ms (11.1 GB fetched), 8 waves x
// 1024 splits 4.02 ms; one work-group per CU of 4 waves 4.7 ms.
//
// FOLD (pairs of shared clouds, stored unreflected): the epilogue also sums
// v . sigma per split and slot into pv (v the pair's FP32 Householder vector
// v32), from which the statistic reflects the group sums (Householder fold).
//
// LO8 (BF16 hi + E4M3 lo): the lo plane is one e4m3 byte per value,
// round(lo 2^17), in 16-row units (the int8 planes' layout: unit h of a
// 32-row group, byte 4 s + b, holds group row s + 4 h + 8 b).  A chunk holds
// the 16 hi octets and the 8 lo units; the hi product runs as above on one
// plane, and the lo product on v_mfma_scale_f32_32x32x64_f8f6f4, one 64-row
// K-step per two mask words: lane half h takes the 32 bytes of group 2 s + h
// (its two units) as the A operand, and register v of the B operand is
// (w >> v) & 0x01010101 for the group's mask word w, a byte 0x01 (e4m3
// 2^-9) per member.  E8M0 scales 2^-17 (A) and 2^9 (B) make the product
// sum_i m_i lo_i exactly as stored, into the same FP32 accumulators.  The
// fp8 MFMA forms each 64-term dot product to about 2^-13 of the sum of the
// terms' magnitudes (measured), far below the e4m3 rounding of lo itself.
//
// HI (the lazy precision's first pass): the hi plane alone; a chunk holds its
// 16 octets.  REFINE (its second pass): both planes as split BF16, for the
// splits listed per pair in rlist (pair p's rcnt[p] split rows from
// rlist[mrow0 of p]), with the tile table and its length (ntile_dev) built on
// the device; each listed split's sums are those the split-BF16 kernel gives
// it (same instructions, same order), written to its own partial row.
enum GroupsumMode { kModeSplit = 0, kModeLo8 = 1, kModeHi = 2, kModeRefine = 3 };
template <int JB, int NW, bool FOLD, int MODE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_groupsum_bf16x2(
    const PairDesc* __restrict__ pairs, const BlockPair* __restrict__ bp,
    const GemmGroup* __restrict__ groups, int ngroups, int ntile_arg, int nslot, int d_pad,
    const uint4* __restrict__ zhi, const uint4* __restrict__ zlo,
    const uint32_t* __restrict__ mask, const float* __restrict__ t32,
    double* __restrict__ partial, int64_t prow, float* __restrict__ sig,
    const float* __restrict__ v32, double* __restrict__ pv, int scale_lo, int scale_mask,
    const uint32_t* __restrict__ rlist, const uint32_t* __restrict__ rcnt,
    const int64_t* __restrict__ ntile_dev) {
    constexpr bool LO8 = MODE == kModeLo8, HI = MODE == kModeHi, IND = MODE == kModeRefine;
    constexpr int kWS = 32 * JB;
    constexpr int kTile = NW * kWS;
    constexpr int kMaskVec = kTile;
    constexpr int kMaskLoads = kWS / 64;
    // LDS rows (64 uint4 each) of a chunk: 16 octets of each bf16 plane, or
    // 16 hi octets and 8 lo units; each wave loads an equal share
    constexpr int kChunkRows = LO8 ? kOct + kOct / 2 : HI ? kOct : 2 * kOct;
    constexpr int kRowsW = kChunkRows / NW;
    static_assert(kRowsW * NW == kChunkRows, "waves split a chunk evenly");
    static_assert(!FOLD || MODE == kModeSplit, "the fold runs on split BF16 only");
    static_assert(!IND || JB == 2, "the refinement skips blocks of 32 splits: 0, 1 or 2 per wave");
    const int ntile_total = IND ? (int)*ntile_dev : ntile_arg;
    __shared__ uint4 zbuf[2][kChunkVec];
    __shared__ uint4 mbuf[2][kMaskVec];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int h = lane >> 5, c = lane & 31;
    const uint32_t rot = 8u * h;
    const int nlogical = (ntile_total + 31) / 32 * 32;
    auto next_valid = [&](int it) {  // the padding of the last 32 logical tiles is skipped
        while (it < nlogical && xcd_remap(it) >= ntile_total) it += gridDim.x;
        return it;
    };
    struct Tile {
        int pair, slot, b0;
    };
    auto tile_of = [&](int it) {
        const int L = xcd_remap(it);
        const GemmGroup grp = groups[upper_index(ngroups, L, [&](int k) { return groups[k].tile0; })];
        const int local = L - (int)grp.tile0;
        return Tile{grp.pair, local / grp.nbt, (local % grp.nbt) * kTile};
    };

    // loader cursor: tile l_it, chunk l_ch (one chunk ahead of the multiplication)
    int l_it = next_valid(blockIdx.x);
    if (l_it >= nlogical) return;  // work-group-uniform
    int l_ch = 0, l_nchunk = 0, l_nxc = 0;
    const uint4* l_zsrc = nullptr;
    const uint4* l_zsrc_y = nullptr;
    const uint4* l_lo8 = nullptr;  // LO8: the pair's first lo unit in this column slice
    const uint4* l_mload[kMaskLoads];
    auto l_setup = [&]() {
        const Tile t = tile_of(l_it);
        const PairDesc pd = pairs[t.pair];
        const BlockPair bq = bp[t.pair];
        l_nchunk = pd.Np / kChunk;
        l_nxc = pd.nxc;
        if constexpr (LO8) {
            l_zsrc = zhi + (pd.zrow0 >> 3) * d_pad + t.slot * kDSlot;
            l_lo8 = zlo + (pd.zrow0 >> 4) * d_pad + t.slot * kDSlot;
        } else {
            const uint4* plane = (kRowsW * wave) / kOct ? zlo : zhi;
            const int64_t off = (kRowsW * wave) % kOct;
            l_zsrc = plane + ((pd.zrow0 >> 3) + off) * d_pad + t.slot * kDSlot;
            l_zsrc_y = plane + ((pd.zrow_y >> 3) + off) * d_pad + t.slot * kDSlot;
        }
#pragma unroll
        for (int k = 0; k < kMaskLoads; ++k) {
            const int r = t.b0 + wave * kWS + 64 * k + lane;
            int64_t mrow;
            if constexpr (IND) mrow = rlist[bq.mrow0 + (r < (int)rcnt[t.pair] ? r : 0)];
            else mrow = bq.mrow0 + (r < bq.nb ? r : 0);
            l_mload[k] = (const uint4*)mask_row(mask, bq, mrow, pd.Wp);
        }
    };
    l_setup();
    const int64_t chunk_stride = (int64_t)kOct * d_pad;
    // one chunk at the cursor into buffer b, then advance the cursor (past the
    // work-group's last chunk it stays there: a harmless reload into a free buffer)
    auto issue_next = [&](int b) {
        const uint32_t zl = __builtin_amdgcn_readfirstlane(lds_addr(&zbuf[b][kRowsW * wave * kDSlot]));
        const uint32_t ml = __builtin_amdgcn_readfirstlane(lds_addr(&mbuf[b][wave * kWS]));
        if constexpr (LO8) {
#pragma unroll
            for (int k = 0; k < kRowsW; ++k) {
                const int r = kRowsW * wave + k;  // wave-uniform
                const uint4* src = r < kOct ? l_zsrc + ((int64_t)kOct * l_ch + r) * d_pad
                                            : l_lo8 + ((int64_t)(kOct / 2) * l_ch + (r - kOct)) * d_pad;
                dma16(src + lane, zl + 16 * kDSlot * k);
            }
        } else {
            const uint4* base = l_ch < l_nxc ? l_zsrc + l_ch * chunk_stride : l_zsrc_y + (l_ch - l_nxc) * chunk_stride;
#pragma unroll
            for (int k = 0; k < kRowsW; ++k) dma16(base + k * d_pad + lane, zl + 16 * kDSlot * k);
        }
#pragma unroll
        for (int k = 0; k < kMaskLoads; ++k) dma16(l_mload[k] + l_ch, ml + 16 * 64 * k);
        if (l_ch + 1 < l_nchunk) {
            ++l_ch;
        } else {
            const int nit = next_valid(l_it + gridDim.x);
            if (nit < nlogical) {
                l_it = nit;
                l_ch = 0;
                l_setup();
            }
        }
    };

    int g = 0;  // global step: buffer g % 2
    issue_next(0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    for (int c_it = next_valid(blockIdx.x); c_it < nlogical; c_it = next_valid(c_it + gridDim.x)) {
        const Tile t = tile_of(c_it);
        const PairDesc pd = pairs[t.pair];
        const BlockPair bq = bp[t.pair];
        const int nchunk = pd.Np / kChunk;
        const uint32_t flip = pd.flip ? 0xffffffffu : 0u;
        const int d0 = t.slot * kDSlot;
        int brow[JB];
        uint32_t keep[JB];
#pragma unroll
        for (int j = 0; j < JB; ++j) {
            brow[j] = t.b0 + wave * kWS + j * 32 + c;
            if constexpr (IND) {  // the listed split's row in the block (relative to the pair's first)
                const bool in = brow[j] < (int)rcnt[t.pair];
                keep[j] = in ? 0xffffffffu : 0u;
                brow[j] = in ? (int)((int64_t)rlist[bq.mrow0 + brow[j]] - bq.mrow0) : 0;
            } else {
                keep[j] = brow[j] < bq.nb ? 0xffffffffu : 0u;
            }
        }
        // REFINE: the wave's leading blocks of 32 splits that hold listed
        // splits (wave-uniform, 0 to JB)
        int jlive = JB;
        if constexpr (IND) {
            const int rem = (int)rcnt[t.pair] - (t.b0 + wave * kWS);
            jlive = __builtin_amdgcn_readfirstlane(rem <= 0 ? 0 : rem >= kWS ? JB : (rem + 31) / 32);
        }
        f32x16 acc[2][JB];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < JB; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

        for (int ch = 0; ch < nchunk; ++ch, ++g) {
            const int b = g & 1;
            issue_next(b ^ 1);  // chunk g + 1 into the buffer read in step g - 1
            const uint4* cur = zbuf[b];
            const uint4* mcur = mbuf[b];
            uint4 mw[JB];
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                const uint4 x = mcur[wave * kWS + 32 * j + c];
                auto prep = [&](uint32_t u) {
                    const uint32_t y = (u ^ flip) & keep[j];
                    return __builtin_amdgcn_alignbit(y, y, rot);
                };
                mw[j] = make_uint4(prep(x.x), prep(x.y), prep(x.z), prep(x.w));
            }
            // the bf16 products of the wave's first NJ blocks of 32 splits
            auto products = [&](auto nj_) {
                constexpr int NJ = decltype(nj_)::value;
                auto fetch = [&](int s, bf16x8 (&a)[2][2], bf16x8 (&bm)[JB]) {
                    const int o = 2 * s + h;
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        a[0][i] = as_bf16x8(cur[o * kDSlot + 32 * i + c]);
                        if (!LO8 && !HI) a[1][i] = as_bf16x8(cur[(kOct + o) * kDSlot + 32 * i + c]);
                    }
                    const uint32_t kBit = 0x00800080u << (4 * (s & 1));
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        const uint32_t word = s < 2 ? mw[j].x : s < 4 ? mw[j].y : s < 6 ? mw[j].z : mw[j].w;
                        bm[j] = as_bf16x8(make_uint4(word & kBit, word & (kBit << 1), word & (kBit << 2),
                                                     word & (kBit << 3)));
                    }
                };
                bf16x8 a[2][2][2], bm[2][JB];
                fetch(0, a[0], bm[0]);
#pragma unroll
                for (int s = 0; s < kChunk / 16; ++s) {
                    if (s + 1 < kChunk / 16) fetch(s + 1, a[(s + 1) & 1], bm[(s + 1) & 1]);
#pragma unroll
                    for (int pl = 0; pl < (LO8 || HI ? 1 : 2); ++pl)
#pragma unroll
                        for (int i = 0; i < 2; ++i)
#pragma unroll
                            for (int j = 0; j < NJ; ++j)
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[s & 1][pl][i], bm[s & 1][j],
                                                                                    acc[i][j], 0, 0, 0);
                }
            };
            if constexpr (IND) {  // blocks past the pair's list have no split to multiply
                if (jlive == JB) products(std::integral_constant<int, JB>{});
                else if (jlive > 0) products(std::integral_constant<int, 1>{});
            } else {
                products(std::integral_constant<int, JB>{});
            }
            if constexpr (LO8) {
                // the lo plane: two 64-row K-steps; group g = 2 s2 + h of the
                // chunk is mask word g, and the words were rotated right by
                // 8 h for the bf16 operands (rotate back)
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    const int g = 2 * s2 + h;
                    i32x8 a8[2];
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const uint4 u0 = cur[(kOct + 2 * g) * kDSlot + 32 * i + c];
                        const uint4 u1 = cur[(kOct + 2 * g + 1) * kDSlot + 32 * i + c];
                        a8[i] = i32x8{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w,
                                      (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
                    }
#pragma unroll
                    for (int j = 0; j < JB; ++j) {
                        const uint32_t wr = s2 == 0 ? (h ? mw[j].y : mw[j].x) : (h ? mw[j].w : mw[j].z);
                        const uint32_t w = __builtin_amdgcn_alignbit(wr, wr, 32u - rot);
                        i32x8 b8;
#pragma unroll
                        for (int v = 0; v < 8; ++v) b8[v] = (int)((w >> v) & 0x01010101u);
#pragma unroll
                        for (int i = 0; i < 2; ++i)
                            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                                a8[i], b8, acc[i][j], 0, 0, 0, scale_lo, 0, scale_mask);
                    }
                }
            }
            // chunk g + 1 has landed (this wave's loads, then every wave's
            // through the barrier); every wave is done reading buffer b
            __builtin_amdgcn_s_waitcnt(0);
            lds_barrier();
        }

        const float* tp = t32 + (int64_t)t.pair * d_pad + d0;
        float tv[2][16];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) tv[i][v] = tp[32 * i + 8 * (v >> 2) + 4 * h + (v & 3)];
        float vr[2][16];
        if constexpr (FOLD) {
            const float* vq = v32 + (int64_t)t.pair * d_pad + d0;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int v = 0; v < 16; ++v) vr[i][v] = vq[32 * i + 8 * (v >> 2) + 4 * h + (v & 3)];
        }
#pragma unroll
        for (int j = 0; j < JB; ++j) {
            float ss = 0.0f, sl = 0.0f, sd = 0.0f;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const float sv = acc[i][j][v];
                    const float lv = tv[i][v] - sv;
                    ss += sv * sv;
                    sl += lv * lv;
                    if (FOLD) sd += vr[i][v] * sv;
                }
            ss += __shfl_xor(ss, 32, 64);
            sl += __shfl_xor(sl, 32, 64);
            if (FOLD) sd += __shfl_xor(sd, 32, 64);
            if (h == 0 && keep[j]) {
                double2* out = (double2*)partial + t.slot * prow + bq.mrow0 + brow[j];
                *out = make_double2((double)ss, (double)sl);
                if (FOLD) pv[t.slot * prow + bq.mrow0 + brow[j]] = (double)sd;
            }
            if (sig && keep[j]) {
                float* sr = sig + (bq.mrow0 + brow[j]) * (int64_t)d_pad + d0;
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int v = 0; v < 16; ++v) sr[32 * i + 8 * (v >> 2) + 4 * h + (v & 3)] = acc[i][j][v];
            }
        }
        // loads and stores may complete out of order: drain the stores (and
        // the chunks in flight) so that the next steps' counts see loads only
        __builtin_amdgcn_s_waitcnt(0);
    }
    __builtin_amdgcn_s_waitcnt(0);  // the reloads past the end
}

// ---------------------------------------------------------------------------
// int8 digit planes: z 2^20 = q0 2^14 + q1 2^7 + q2, stored as the planes
// (q0, -q1, q2).  Two exact int32 sums per output on v_mfma_i32_32x32x32_i8:
//   S_hi = Q0^T M,   S_lo = (-Q1)^T (-128 M) + Q2^T M = 128 Q1^T M + Q2^T M
// (the mask byte -128 is 0x80), so sigma = (S_hi 2^14 + S_lo) 2^-20 in FP64.
// A (32 x 32) lane l -> row l%32, k 16(l/32)..+15; B (32 x 32) lane l ->
// k 16(l/32)..+15, col l%32; D lane l -> col l%32, rows 8(v/4) + 4(l/32) + v%4.
//
// Work-group tile: 64 columns x kTileI8 (512) splits of eight waves; wave w
// owns splits [64 w, 64 w + 64) as 2 blocks of 32 and the 64 columns as 2
// blocks of 32 (accumulators 2 sums x 2 x 2 x 16 int32 per lane; 224
// registers per lane, 2 waves per SIMD).  One work-group per CU (64 KB of
// LDS) shares each Z chunk between all eight waves, as the wide split-BF16
// tile does (on 512 pairs, d = 768: 3.77 ms with 256 splits of four waves
// and two work-groups per CU, 3.6-3.7 ms this way).
// A K-step is 32 pooled rows, one mask word: operand register s of lane
// half h is (word >> (s + 4 h)) & 0x01010101 (the planes' row order makes
// those the lane's rows), and that shifted left by 7 for the middle plane.
// Z streams through LDS in chunks of 128 rows (three planes of the 64
// columns = 24 KB, mask words 4 KB), two buffers, with the persistent launch
// of the split-BF16 kernel.  Splits past the block's end take the
// mask of its first split and are not written.
// ---------------------------------------------------------------------------
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
constexpr int kHex = kChunk / 16;                  // 16-row units per chunk
constexpr int kChunkVecI8 = 3 * kHex * kDSlot;     // uint4 per chunk (three planes)
// |S_lo| <= 64 N (2^7 + 1) and |S_hi| <= 64 N must stay int32 for every pooled size
static_assert(64LL * HBT_MAX_N * 129 < (1LL << 31), "int8 digit sums overflow int32");

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_groupsum_i8x3(
    const PairDesc* __restrict__ pairs, const BlockPair* __restrict__ bp,
    const GemmGroup* __restrict__ groups, int ngroups, int ntile_total, int nslot, int d_pad,
    const uint4* __restrict__ zq, int64_t plane_vec, const uint32_t* __restrict__ mask,
    const double* __restrict__ t64, double* __restrict__ partial, int64_t prow) {
    constexpr int JB = 2, kWS = 32 * JB;        // splits per wave
    constexpr int kRowsPerWave = 3 * kHex / 8;  // LDS rows of Z each wave loads (3)
    constexpr int kMaskLoads = kWS / 64;        // mask loads per wave per chunk
    constexpr int kWaitOneChunk = wait_vmcnt(0);  // the one chunk in flight
    static_assert(kTileI8 == 8 * kWS && kRowsPerWave * 8 == 3 * kHex, "eight waves");
    __shared__ uint4 zbuf[2][kChunkVecI8];
    __shared__ uint4 mbuf[2][kTileI8];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int h = lane >> 5, c = lane & 31;
    const uint32_t rsh = 4u * h;
    const int nlogical = (ntile_total + 31) / 32 * 32;
    auto next_valid = [&](int it) {
        while (it < nlogical && xcd_remap(it) >= ntile_total) it += gridDim.x;
        return it;
    };
    struct Tile {
        int pair, slot, b0;
    };
    auto tile_of = [&](int it) {
        const int L = xcd_remap(it);
        const GemmGroup grp = groups[upper_index(ngroups, L, [&](int k) { return groups[k].tile0; })];
        const int local = L - (int)grp.tile0;
        return Tile{grp.pair, local / grp.nbt, (local % grp.nbt) * kTileI8};
    };

    // loader cursor (one chunk ahead of the multiplication, across tiles)
    int l_it = next_valid(blockIdx.x);
    if (l_it >= nlogical) return;  // work-group-uniform
    int l_ch = 0, l_nchunk = 0;
    int64_t l_unit0 = 0;  // first 16-row unit of the pair's column slice
    int l_d0 = 0;
    const uint4* l_mload[kMaskLoads];
    auto l_setup = [&]() {
        const Tile t = tile_of(l_it);
        const PairDesc pd = pairs[t.pair];
        const BlockPair bq = bp[t.pair];
        l_nchunk = pd.Np / kChunk;
        l_unit0 = pd.zrow0 >> 4;
        l_d0 = t.slot * kDSlot;
#pragma unroll
        for (int k = 0; k < kMaskLoads; ++k) {
            const int r = t.b0 + kWS * wave + 64 * k + lane;
            l_mload[k] = (const uint4*)mask_row(mask, bq, bq.mrow0 + (r < bq.nb ? r : 0), pd.Wp);
        }
    };
    l_setup();
    // chunk at the cursor: LDS rows (plane, unit) 3 w .. 3 w + 2, lane l moving
    // column l; then the wave's mask words; then advance the cursor (it stays
    // on the work-group's last chunk at the end: harmless reloads)
    auto issue_next = [&](int b) {
#pragma unroll
        for (int k = 0; k < kRowsPerWave; ++k) {
            const int r = kRowsPerWave * wave + k;  // wave-uniform
            const uint4* src = zq + (r / kHex) * plane_vec + (l_unit0 + (int64_t)kHex * l_ch + r % kHex) * d_pad + l_d0;
            dma16(src + lane, __builtin_amdgcn_readfirstlane(lds_addr(&zbuf[b][r * kDSlot])));
        }
        const uint32_t ml = __builtin_amdgcn_readfirstlane(lds_addr(&mbuf[b][kWS * wave]));
#pragma unroll
        for (int k = 0; k < kMaskLoads; ++k) dma16(l_mload[k] + l_ch, ml + 16 * 64 * k);
        if (l_ch + 1 < l_nchunk) {
            ++l_ch;
        } else {
            const int nit = next_valid(l_it + gridDim.x);
            if (nit < nlogical) {
                l_it = nit;
                l_ch = 0;
                l_setup();
            }
        }
    };

    int g = 0;  // global step: buffer g % 2
    issue_next(0);
    __builtin_amdgcn_s_waitcnt(kWaitOneChunk);
    __syncthreads();

    for (int c_it = next_valid(blockIdx.x); c_it < nlogical; c_it = next_valid(c_it + gridDim.x)) {
        const Tile t = tile_of(c_it);
        const PairDesc pd = pairs[t.pair];
        const BlockPair bq = bp[t.pair];
        const int nchunk = pd.Np / kChunk;
        const uint32_t flip = pd.flip ? 0xffffffffu : 0u;
        const int d0 = t.slot * kDSlot;
        i32x16 acc[2][2][JB];  // [S_hi, S_lo][column block][split block]
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < JB; ++j)
#pragma unroll
                    for (int v = 0; v < 16; ++v) acc[q][i][j][v] = 0;

        for (int ch = 0; ch < nchunk; ++ch, ++g) {
            const int b = g & 1;
            issue_next(b ^ 1);
            const uint4* cur = zbuf[b];
            const uint4* mcur = mbuf[b];
            // the chunk's mask words of the lane's splits: group flip, lane-half shift
            uint4 mw[JB];
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                const uint4 x = mcur[kWS * wave + 32 * j + c];
                mw[j] = make_uint4((x.x ^ flip) >> rsh, (x.y ^ flip) >> rsh, (x.z ^ flip) >> rsh, (x.w ^ flip) >> rsh);
            }
            auto fetch = [&](int s, i32x4 (&a)[3][2], i32x4 (&bm)[JB]) {
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const uint4 u = cur[(q * kHex + 2 * s + h) * kDSlot + 32 * i + c];
                        a[q][i] = i32x4{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
                    }
#pragma unroll
                for (int j = 0; j < JB; ++j) {
                    const uint32_t w = s == 0 ? mw[j].x : s == 1 ? mw[j].y : s == 2 ? mw[j].z : mw[j].w;
                    bm[j] = i32x4{(int)(w & 0x01010101u), (int)((w >> 1) & 0x01010101u),
                                  (int)((w >> 2) & 0x01010101u), (int)((w >> 3) & 0x01010101u)};
                }
            };
            i32x4 a[2][3][2], bm[2][JB];
            fetch(0, a[0], bm[0]);
#pragma unroll
            for (int s = 0; s < kChunk / 32; ++s) {  // K-steps of 32 pooled rows
                if (s + 1 < kChunk / 32) fetch(s + 1, a[(s + 1) & 1], bm[(s + 1) & 1]);
                const int bb = s & 1;
                // middle plane first, then the high plane, then the low plane into
                // the same sum as the middle one: 16 MFMAs between dependent ones
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < JB; ++j) {
                        const i32x4 m128 = bm[bb][j] << 7;  // bytes 0x80 = -128 where the mask is set
                        acc[1][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[bb][1][i], m128, acc[1][i][j], 0, 0, 0);
                    }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < JB; ++j)
                        acc[0][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[bb][0][i], bm[bb][j], acc[0][i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < JB; ++j)
                        acc[1][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[bb][2][i], bm[bb][j], acc[1][i][j], 0, 0, 0);
            }
            __builtin_amdgcn_s_waitcnt(kWaitOneChunk);
            lds_barrier();
        }

        // epilogue: sigma_small in FP64, squared norms of sigma_small and
        // t - sigma_small over the slot's 64 columns
        const double* tp = t64 + (int64_t)t.pair * d_pad + d0;
        double tv[2][16];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) tv[i][v] = tp[32 * i + 8 * (v >> 2) + 4 * h + (v & 3)];
#pragma unroll
        for (int j = 0; j < JB; ++j) {
            const int brow = t.b0 + wave * kWS + j * 32 + c;
            double ss = 0.0, sl = 0.0;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const double sv = __builtin_fma((double)acc[0][i][j][v], 16384.0, (double)acc[1][i][j][v]) *
                                      (1.0 / 1048576.0);
                    const double lv = tv[i][v] - sv;
                    ss += sv * sv;
                    sl += lv * lv;
                }
            ss += __shfl_xor(ss, 32, 64);
            sl += __shfl_xor(sl, 32, 64);
            if (h == 0 && brow < bq.nb) {
                double2* out = (double2*)partial + t.slot * prow + bq.mrow0 + brow;
                *out = make_double2(ss, sl);
            }
        }
        // loads and stores may complete out of order: drain the stores (and
        // the chunks in flight) so that the next steps' counts see loads only
        __builtin_amdgcn_s_waitcnt(0);
    }
    __builtin_amdgcn_s_waitcnt(0);  // the reloads past the end
}

// ---------------------------------------------------------------------------
// FP32 / FP64: v_mfma_{f32_16x16x4f32, f64_16x16x4f64}
// A (16 x 4) lane l -> row l%16, k l/16; B (4 x 16) lane l -> k l/16, col l%16;
// D lane l -> col l%16, register v -> row 4(l/16) + v (f32) or 4v + l/16 (f64).
// Wave tile: 64 columns (4 blocks) x 64 splits (4 blocks).
// ---------------------------------------------------------------------------
template <typename T>
struct MfmaFp;
template <>
struct MfmaFp<float> {
    typedef f32x4 acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
};
template <>
struct MfmaFp<double> {
    typedef f64x4 acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int v) { return 4 * v + q; }
};

template <typename T>
__global__ __launch_bounds__(256) void k_groupsum_fp(const PairDesc* __restrict__ pairs,
                                                     const BlockPair* __restrict__ bp,
                                                     const GemmTile* __restrict__ tiles,
                                                     int nslot, int d_pad, const T* __restrict__ z,
                                                     const uint32_t* __restrict__ mask,
                                                     const T* __restrict__ tvec,
                                                     double* __restrict__ partial, int64_t prow,
                                                     float* __restrict__ sig) {
    typedef typename MfmaFp<T>::acc_t acc_t;
    const GemmTile tile = tiles[blockIdx.x / nslot];
    const int slot = blockIdx.x % nslot;
    const PairDesc pd = pairs[tile.pair];
    const BlockPair bq = bp[tile.pair];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane >> 4, c = lane & 15;
    const int d0 = slot * kDSlot;
    int brow[4];
    bool valid[4];
    const uint32_t* mrow[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        brow[j] = tile.b0 + wave * 64 + j * 16 + c;
        valid[j] = brow[j] < bq.nb;
        mrow[j] = mask_row(mask, bq, bq.mrow0 + (valid[j] ? brow[j] : 0), pd.Wp);
    }
    const uint32_t flip = pd.flip ? 0xffffffffu : 0u;
    const T* za = z + pd.zrow0 * d_pad + d0 + c;
    acc_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;

    for (int kw = 0; kw < pd.Wp; ++kw) {
        uint32_t mw[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) mw[j] = valid[j] ? (mrow[j][kw] ^ flip) : 0u;
#pragma unroll 2
        for (int s = 0; s < 8; ++s) {  // K-steps of 4 pooled rows
            const int64_t rowz = (int64_t)(32 * kw + 4 * s + q) * d_pad;
            T a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = za[rowz + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = ((mw[j] >> (4 * s + q)) & 1u) ? (T)1 : (T)0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = MfmaFp<T>::mma(a[i], b[j], acc[i][j]);
        }
    }
    const T* tp = tvec + (int64_t)tile.pair * d_pad + d0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        T ss = 0, sl = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const T sv = acc[i][j][v];
                const T lv = tp[16 * i + MfmaFp<T>::row(q, v)] - sv;
                ss += sv * sv;
                sl += lv * lv;
            }
        ss += __shfl_xor(ss, 16, 64);
        sl += __shfl_xor(sl, 16, 64);
        ss += __shfl_xor(ss, 32, 64);
        sl += __shfl_xor(sl, 32, 64);
        if (q == 0 && valid[j]) {
            double2* out = (double2*)partial + slot * prow + bq.mrow0 + brow[j];
            *out = make_double2((double)ss, (double)sl);
        }
        if (sig && valid[j]) {  // the group sums themselves, for the point-to-centroid route
            float* sr = sig + (bq.mrow0 + brow[j]) * (int64_t)d_pad + d0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) sr[16 * i + MfmaFp<T>::row(q, v)] = (float)acc[i][j][v];
        }
    }
}

// Work-groups of a persistent launch over `tiles` tiles: per_cu per CU, a
// multiple of 32 so that the XCD numbering holds.  Measured on MI355X (512
// pairs, d = 768): with one resident work-group per CU (int8 planes), 1 per
// CU leaves the tail unbalanced and one per tile loses the cross-tile
// prefetch, 4 is best; with two resident (split BF16), 2 / 4 / 8 / 16 / 32 /
// 64 per CU give 4.80 / 4.70 / 4.62 / 4.60 / 4.52 / 4.50 ms and one per tile
// 4.51 ms: the co-resident work-group already hides a tile's start.  The
// eight-wave wide tile (one work-group per CU): 8 or 16 per CU, within noise.
static std::atomic<int> g_cus[64];
int device_cus() {
    int dev = 0;
    int cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
        cus = g_cus[dev].load(std::memory_order_relaxed);
        if (!cus && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            g_cus[dev].store(cus, std::memory_order_relaxed);
    }
    return cus > 0 ? cus : 256;
}

static unsigned persistent_grid(int64_t tiles, int per_cu) {
    const int cus = device_cus();
    const int64_t want = (int64_t)(cus * per_cu + 31) / 32 * 32;
    const int64_t all = (tiles + 31) / 32 * 32;
    return (unsigned)(all < want ? all : want);
}

int groupsum_tile_splits(int precision) {
    return precision == HBT_BF16X2 || precision == HBT_BF16_E4M3 ? kTileWide : kTileB;
}

hipError_t launch_groupsum(int precision, const PairDesc* pairs, const BlockPair* bp,
                           const GemmTile* tiles, int ntiles, const GemmGroup* groups, int ngw,
                           int ntw, int ng256, int nt256, int d_pad, const void* zstore,
                           int64_t zplane_elems, const uint32_t* mask, const float* t32,
                           const double* t64, double* partial, int64_t prow, float* sig, hipStream_t s,
                           int grid_wide, int grid_narrow, const float* v32, double* pv, bool hi_only) {
    const int nslot = d_pad / kDSlot;
    if (grid_wide <= 0) grid_wide = 16;
    if (grid_narrow <= 0) grid_narrow = precision == HBT_I8X3 ? 16 : 32;
    dim3 block(256);
    if (hi_only && (precision != HBT_BF16X2 || pv)) return hipErrorInvalidValue;
    switch (precision) {
        case HBT_BF16X2: {
            const uint4* zhi = (const uint4*)zstore;
            const uint4* zlo = (const uint4*)zstore + zplane_elems / 8;
            static_assert(32 * 4 * 8 == kTileWide && 32 * 2 * 4 == kTileNarrow, "tile widths");
            if (hi_only) {
                if (ntw > 0)
                    hipLaunchKernelGGL((k_groupsum_bf16x2<4, 8, false, kModeHi>), dim3(persistent_grid(ntw, grid_wide)),
                                       dim3(512), 0, s, pairs, bp, groups, ngw, ntw, nslot, d_pad, zhi, zlo, mask,
                                       t32, partial, prow, sig, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr);
                if (nt256 > 0)
                    hipLaunchKernelGGL((k_groupsum_bf16x2<2, 4, false, kModeHi>), dim3(persistent_grid(nt256, grid_narrow)),
                                       block, 0, s, pairs, bp, groups + ngw, ng256, nt256, nslot, d_pad, zhi, zlo,
                                       mask, t32, partial, prow, sig, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr);
                break;
            }
            if (ntw > 0) {
                if (pv)
                    hipLaunchKernelGGL((k_groupsum_bf16x2<4, 8, true, kModeSplit>), dim3(persistent_grid(ntw, grid_wide)),
                                       dim3(512), 0, s, pairs, bp, groups, ngw, ntw, nslot, d_pad, zhi, zlo, mask,
                                       t32, partial, prow, sig, v32, pv, 0, 0, nullptr, nullptr, nullptr);
                else
                    hipLaunchKernelGGL((k_groupsum_bf16x2<4, 8, false, kModeSplit>), dim3(persistent_grid(ntw, grid_wide)),
                                       dim3(512), 0, s, pairs, bp, groups, ngw, ntw, nslot, d_pad, zhi, zlo, mask,
                                       t32, partial, prow, sig, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr);
            }
            if (nt256 > 0) {
                if (pv)
                    hipLaunchKernelGGL((k_groupsum_bf16x2<2, 4, true, kModeSplit>), dim3(persistent_grid(nt256, grid_narrow)),
                                       block, 0, s, pairs, bp, groups + ngw, ng256, nt256, nslot, d_pad, zhi, zlo,
                                       mask, t32, partial, prow, sig, v32, pv, 0, 0, nullptr, nullptr, nullptr);
                else
                    hipLaunchKernelGGL((k_groupsum_bf16x2<2, 4, false, kModeSplit>), dim3(persistent_grid(nt256, grid_narrow)),
                                       block, 0, s, pairs, bp, groups + ngw, ng256, nt256, nslot, d_pad, zhi, zlo,
                                       mask, t32, partial, prow, sig, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr);
            }
            break;
        }
        case HBT_BF16_E4M3: {
            // hi plane: bf16 [rows/8][d_pad][8]; lo plane at byte 2 zplane_elems:
            // e4m3 [rows/16][d_pad][16]
            const uint4* zhi = (const uint4*)zstore;
            const uint4* zlo = (const uint4*)((const char*)zstore + 2 * zplane_elems);
            const int sa = 127 - kE4m3LoShift, sb = 127 + 9;  // E8M0: 2^-17 on lo, 2^9 on the 0x01 mask bytes
            if (ntw > 0)
                hipLaunchKernelGGL((k_groupsum_bf16x2<4, 8, false, kModeLo8>), dim3(persistent_grid(ntw, grid_wide)),
                                   dim3(512), 0, s, pairs, bp, groups, ngw, ntw, nslot, d_pad, zhi, zlo, mask,
                                   t32, partial, prow, sig, nullptr, nullptr, sa, sb, nullptr, nullptr, nullptr);
            if (nt256 > 0)
                hipLaunchKernelGGL((k_groupsum_bf16x2<2, 4, false, kModeLo8>), dim3(persistent_grid(nt256, grid_narrow)),
                                   block, 0, s, pairs, bp, groups + ngw, ng256, nt256, nslot, d_pad, zhi, zlo,
                                   mask, t32, partial, prow, sig, nullptr, nullptr, sa, sb, nullptr, nullptr, nullptr);
            break;
        }
        case HBT_I8X3:
            if (nt256 > 0)
                hipLaunchKernelGGL(k_groupsum_i8x3, dim3(persistent_grid(nt256, grid_narrow)), dim3(512), 0, s,
                                   pairs, bp, groups + ngw, ng256, nt256, nslot, d_pad, (const uint4*)zstore,
                                   zplane_elems / 16, mask, t64, partial, prow);
            break;
        case HBT_F32:
            if (ntiles <= 0) return hipSuccess;
            hipLaunchKernelGGL(k_groupsum_fp<float>, dim3((unsigned)(ntiles * nslot)), block, 0, s,
                               pairs, bp, tiles, nslot, d_pad, (const float*)zstore, mask, t32,
                               partial, prow, sig);
            break;
        default:
            if (ntiles <= 0) return hipSuccess;
            hipLaunchKernelGGL(k_groupsum_fp<double>, dim3((unsigned)(ntiles * nslot)), block, 0, s,
                               pairs, bp, tiles, nslot, d_pad, (const double*)zstore, mask, t64,
                               partial, prow, sig);
            break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The lazy precision's second pass.  Tile table: group g of the product's
// table (one per pair, longest pair first) gets ceil(rcnt / 256) b-tiles of
// the listed splits per column slot, tile0 the running sum; one work-group
// scans the groups 256 at a time and writes the total to ntile.  (Tiles of
// kTileWide splits for pairs with long lists, a quarter of the Z reads per
// split, were measured slower on 512 pairs at d = 768: 0.88 against 0.78 ms,
// with a quarter as many tiles and one work-group per CU instead of two.)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_refine_tiles(const GemmGroup* __restrict__ groups, int ngroups,
                                                      const uint32_t* __restrict__ rcnt, int nslot,
                                                      GemmGroup* __restrict__ out, int64_t* __restrict__ ntile) {
    __shared__ int64_t sh[256];
    const int t = threadIdx.x;
    int64_t base = 0;
    for (int g0 = 0; g0 < ngroups; g0 += 256) {
        const int g = g0 + t;
        int pair = 0, nbt = 0;
        if (g < ngroups) {
            pair = groups[g].pair;
            nbt = (int)((rcnt[pair] + kTileNarrow - 1) / kTileNarrow);
        }
        const int64_t tiles = (int64_t)nbt * nslot;
        sh[t] = tiles;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {  // inclusive scan
            const int64_t v = t >= o ? sh[t - o] : 0;
            __syncthreads();
            sh[t] += v;
            __syncthreads();
        }
        if (g < ngroups) out[g] = GemmGroup{pair, nbt, base + sh[t] - tiles};
        base += sh[255];
        __syncthreads();  // every thread has read sh[255] before the next chunk writes sh
    }
    if (t == 0) *ntile = base;
}

hipError_t launch_refine_tiles(const GemmGroup* groups, int ngroups, const uint32_t* rcnt, int d_pad,
                               GemmGroup* out, int64_t* ntile, hipStream_t s) {
    if (ngroups <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_refine_tiles, dim3(1), dim3(256), 0, s, groups, ngroups, rcnt, d_pad / kDSlot, out,
                       ntile);
    return hipGetLastError();
}

hipError_t launch_groupsum_refine(const PairDesc* pairs, const BlockPair* bp, const GemmGroup* rgroups,
                                  int ngroups, const int64_t* ntile, int d_pad, const void* zstore,
                                  int64_t zplane_elems, const uint32_t* mask, const float* t32, double* partial,
                                  int64_t prow, const uint32_t* rlist, const uint32_t* rcnt, int grid_narrow,
                                  hipStream_t s) {
    if (ngroups <= 0) return hipErrorInvalidValue;
    if (grid_narrow <= 0) grid_narrow = 32;
    const uint4* zhi = (const uint4*)zstore;
    const uint4* zlo = (const uint4*)zstore + zplane_elems / 8;
    // the tile count is known on the device only: a full persistent grid,
    // whose work-groups without a tile return at once
    const unsigned grid = (unsigned)((device_cus() * grid_narrow + 31) / 32 * 32);
    hipLaunchKernelGGL((k_groupsum_bf16x2<2, 4, false, kModeRefine>), dim3(grid), dim3(256), 0, s, pairs, bp,
                       rgroups, ngroups, 0, d_pad / kDSlot, d_pad, zhi, zlo, mask, t32, partial, prow, nullptr,
                       nullptr, nullptr, 0, 0, rlist, rcnt, ntile);
    return hipGetLastError();
}

}  // namespace hbt
