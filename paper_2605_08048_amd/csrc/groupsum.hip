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
// Output per split row and per slot of kDSlot columns:
//   partial[row][slot] = (sum_c sigma_small[c]^2, sum_c (t[c] - sigma_small[c])^2)
//
// Work-group = 4 waves; tile = kDSlot columns x (512 splits for split BF16,
// 256 for FP32 / FP64).
#include "hbt_launch.h"

namespace hbt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// 8 mask bits -> 8 bf16 values 0.0 / 1.0 (bf16 1.0 = 0x3F80).
__device__ __forceinline__ bf16x8 expand_bits_bf16(uint32_t byte) {
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t two = (byte >> (2 * j)) & 3u;          // tokens 2j, 2j+1
        const uint32_t spread = (two | (two << 15)) & 0x10001u; // bit0 -> bit0, bit1 -> bit16
        w[j] = spread * 0x3F80u;
    }
    uint4 u = make_uint4(w[0], w[1], w[2], w[3]);
    return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

// ---------------------------------------------------------------------------
// split BF16: z = hi + lo, C += Z_hi^T M + Z_lo^T M, FP32 accumulation
// v_mfma_f32_32x32x16_bf16: A (32 x 16) lane l -> row l%32, k 8(l/32)..+7;
// B (16 x 32) lane l -> k 8(l/32)..+7, col l%32; D lane l -> col l%32,
// rows 8(v/4) + 4(l/32) + v%4.
//
// Work-group tile: kDSlot (64) columns x kTileBF16 (512) splits; 4 waves,
// wave w owns splits [128 w, 128 w + 128) as 4 blocks of 32 and all 64
// columns as 2 blocks of 32 (accumulators: 2 x 4 x 16 floats per lane).
// The pooled rows are consumed in chunks of 64 (8 octets): the chunk's
// 64-column slice of both planes (16 KB) is staged in LDS once and read by
// all four waves; the next chunk is loaded into registers while the current
// one is multiplied (two LDS buffers).
// ---------------------------------------------------------------------------
constexpr int kTileBF16 = 512;
constexpr int kChunk = 64;                        // pooled rows per chunk
constexpr int kChunkVec = 2 * (kChunk / 8) * kDSlot;  // uint4 per chunk (both planes)

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_groupsum_bf16x2(
    const PairDesc* __restrict__ pairs, const BlockPair* __restrict__ bp,
    const GemmTile* __restrict__ tiles, int nslot, int d_pad, const uint4* __restrict__ zhi,
    const uint4* __restrict__ zlo, const uint32_t* __restrict__ mask,
    const float* __restrict__ t32, double* __restrict__ partial) {
    // two separate LDS objects ([plane][octet][column] each), so the compiler
    // can see that a direct load into one never feeds a read of the other
    __shared__ uint4 lds0[kChunkVec];
    __shared__ uint4 lds1[kChunkVec];
    const GemmTile tile = tiles[blockIdx.x / nslot];
    const int slot = blockIdx.x % nslot;
    const PairDesc pd = pairs[tile.pair];
    const BlockPair bq = bp[tile.pair];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int h = lane >> 5, c = lane & 31;
    const int d0 = slot * kDSlot;
    const int nchunk = pd.Np / kChunk;

    // mask rows of this lane's four split blocks; rows past the pair's splits
    // read its first row and are zeroed by keep[] (no branch around the load)
    int brow[4];
    uint32_t keep[4];
    const uint2* mrow[4];
    const uint32_t flip = pd.flip ? 0xffffffffu : 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        brow[j] = tile.b0 + wave * 128 + j * 32 + c;
        const bool valid = brow[j] < bq.nb;
        keep[j] = valid ? 0xffffffffu : 0u;
        mrow[j] = (const uint2*)mask_row(mask, bq, bq.mrow0 + (valid ? brow[j] : 0), pd.Wp);
    }

    // chunk loader: the chunk tile is 16 rows (plane x octet) of kDSlot uint4;
    // wave w fills rows 4w .. 4w+3 with direct global -> LDS loads (lane l
    // moves column l of a row, 1 KB per wave per load)
    const int64_t oct0 = pd.zrow0 >> 3;
    const uint4* gsrc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = 4 * wave + k;
        const int plane = r / (kChunk / 8), oct = r % (kChunk / 8);
        gsrc[k] = (plane ? zlo : zhi) + (oct0 + oct) * d_pad + d0 + lane;
    }
    const int64_t chunk_stride = (int64_t)(kChunk / 8) * d_pad;
    auto issue = [&](int ch, uint4* dst) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void*)(gsrc[k] + ch * chunk_stride),
                (__attribute__((address_space(3))) void*)(dst + (4 * wave + k) * kDSlot), 16, 0, 0);
    };

    uint2 mw_next[4];
    issue(0, lds0);
#pragma unroll
    for (int j = 0; j < 4; ++j) mw_next[j] = mrow[j][0];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    f32x16 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    // one chunk: stream chunk ch+1 into `nxt` while multiplying `cur`
    auto step = [&](int ch, const uint4* cur, uint4* nxt) {
        uint2 mw[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            mw[j].x = (mw_next[j].x ^ flip) & keep[j];
            mw[j].y = (mw_next[j].y ^ flip) & keep[j];
        }
        if (ch + 1 < nchunk) {
            issue(ch + 1, nxt);
#pragma unroll
            for (int j = 0; j < 4; ++j) mw_next[j] = mrow[j][ch + 1];
        }
#pragma unroll
        for (int s = 0; s < kChunk / 16; ++s) {  // K-steps of 16 pooled rows
            const int o = 2 * s + h;             // octet of this lane's 8 rows
            bf16x8 a_hi[2], a_lo[2], bm[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a_hi[i] = as_bf16x8(cur[o * kDSlot + 32 * i + c]);
                a_lo[i] = as_bf16x8(cur[(kChunk / 8 + o) * kDSlot + 32 * i + c]);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t word = s < 2 ? mw[j].x : mw[j].y;
                bm[j] = expand_bits_bf16((word >> (8 * (2 * (s & 1) + h))) & 0xffu);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_hi[i], bm[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_lo[i], bm[j], acc[i][j], 0, 0, 0);
        }
        // the next chunk's LDS writes and mask loads have landed; every wave is
        // done reading `cur` before it is refilled
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };
    for (int ch = 0; ch < nchunk; ch += 2) {
        step(ch, lds0, lds1);
        if (ch + 1 < nchunk) step(ch + 1, lds1, lds0);
    }
    // epilogue: squared norms of sigma_small and t - sigma_small over the 64 columns
    const float* tp = t32 + (int64_t)tile.pair * d_pad + d0;
    float tv[2][16];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) tv[i][v] = tp[32 * i + 8 * (v >> 2) + 4 * h + (v & 3)];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float ss = 0.0f, sl = 0.0f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const float sv = acc[i][j][v];
                const float lv = tv[i][v] - sv;
                ss += sv * sv;
                sl += lv * lv;
            }
        ss += __shfl_xor(ss, 32, 64);
        sl += __shfl_xor(sl, 32, 64);
        if (h == 0 && keep[j]) {
            double2* out = (double2*)partial + (bq.mrow0 + brow[j]) * nslot + slot;
            *out = make_double2((double)ss, (double)sl);
        }
    }
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
                                                     double* __restrict__ partial) {
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
            double2* out = (double2*)partial + (bq.mrow0 + brow[j]) * nslot + slot;
            *out = make_double2((double)ss, (double)sl);
        }
    }
}

int groupsum_tile_splits(int precision) { return precision == HBT_BF16X2 ? kTileBF16 : kTileB; }

hipError_t launch_groupsum(int precision, const PairDesc* pairs, const BlockPair* bp,
                           const GemmTile* tiles, int ntiles, int d_pad, const void* zstore,
                           int64_t zplane_elems, const uint32_t* mask, const float* t32,
                           const double* t64, double* partial, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    const int nslot = d_pad / kDSlot;
    dim3 grid((unsigned)(ntiles * nslot)), block(256);
    switch (precision) {
        case HBT_BF16X2:
            hipLaunchKernelGGL(k_groupsum_bf16x2, grid, block, 0, s, pairs, bp, tiles, nslot, d_pad,
                               (const uint4*)zstore, (const uint4*)zstore + zplane_elems / 8, mask,
                               t32, partial);
            break;
        case HBT_F32:
            hipLaunchKernelGGL(k_groupsum_fp<float>, grid, block, 0, s, pairs, bp, tiles, nslot,
                               d_pad, (const float*)zstore, mask, t32, partial);
            break;
        default:
            hipLaunchKernelGGL(k_groupsum_fp<double>, grid, block, 0, s, pairs, bp, tiles, nslot,
                               d_pad, (const double*)zstore, mask, t64, partial);
            break;
    }
    return hipGetLastError();
}

}  // namespace hbt
