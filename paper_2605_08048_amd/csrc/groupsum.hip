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
// Work-group = 4 waves; tile = kDSlot columns x kTileB (=256) splits; each
// wave owns 64 columns x 64 splits.
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
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_groupsum_bf16x2(
    const PairDesc* __restrict__ pairs, const BlockPair* __restrict__ bp,
    const GemmTile* __restrict__ tiles, int nslot, int d_pad, const uint4* __restrict__ zhi,
    const uint4* __restrict__ zlo, const uint32_t* __restrict__ mask,
    const float* __restrict__ t32, double* __restrict__ partial) {
    const GemmTile tile = tiles[blockIdx.x / nslot];
    const int slot = blockIdx.x % nslot;
    const PairDesc pd = pairs[tile.pair];
    const BlockPair bq = bp[tile.pair];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int h = lane >> 5, c = lane & 31;
    const int d0 = slot * kDSlot;
    // the two 32-split column blocks of this wave
    int brow[2];
    bool valid[2];
    const uint32_t* mrow[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        brow[j] = tile.b0 + wave * 64 + j * 32 + c;
        valid[j] = brow[j] < bq.nb;
        mrow[j] = mask_row(mask, bq, bq.mrow0 + (valid[j] ? brow[j] : 0), pd.Wp);
    }
    const uint32_t flip = pd.flip ? 0xffffffffu : 0u;
    // Z planes: [octet][col] of uint4 (8 bf16 of one column, 8 rows)
    const int64_t oct0 = pd.zrow0 >> 3;
    const uint4* ah = zhi + oct0 * d_pad + d0 + c;
    const uint4* al = zlo + oct0 * d_pad + d0 + c;

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    for (int kw = 0; kw < pd.Wp; ++kw) {  // 32 pooled rows per mask word
        uint32_t mw[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) mw[j] = valid[j] ? (mrow[j][kw] ^ flip) : 0u;
#pragma unroll
        for (int s = 0; s < 2; ++s) {  // two K-steps of 16 rows
            const int64_t o = (int64_t)(4 * kw + 2 * s + h) * d_pad;
            bf16x8 a_hi[2], a_lo[2], bm[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a_hi[i] = as_bf16x8(ah[o + 32 * i]);
                a_lo[i] = as_bf16x8(al[o + 32 * i]);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) bm[j] = expand_bits_bf16((mw[j] >> (8 * (2 * s + h))) & 0xffu);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_hi[i], bm[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_lo[i], bm[j], acc[i][j], 0, 0, 0);
                }
        }
    }
    // epilogue: squared norms of sigma_small and t - sigma_small over 64 columns
    const float* tp = t32 + (int64_t)tile.pair * d_pad + d0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        float ss = 0.0f, sl = 0.0f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
                const float sv = acc[i][j][v];
                const float lv = tp[r] - sv;
                ss += sv * sv;
                sl += lv * lv;
            }
        ss += __shfl_xor(ss, 32, 64);
        sl += __shfl_xor(sl, 32, 64);
        if (h == 0 && valid[j]) {
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
