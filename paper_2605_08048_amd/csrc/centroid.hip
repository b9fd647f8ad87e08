// Point-to-centroid route to the permuted mean resultant lengths.
//
// For unit vectors the squared norm of a group sum equals the sum of the
// group's point-to-centroid products: |sigma|^2 = sum_{i in G} z_i . sigma
// (Sec. 3.1, MRL definition).  With S the stacked group sums of the smaller
// group (one row per split, from the group-sum kernel) the products of every
// pooled row with every split's centroid direction form one product
//   Q = Z S^T   (pooled rows x splits),
// and two masked column sums give both squared norms:
//   |sigma_small|^2 = sum_i M_bi Q_ib,
//   |t - sigma_small|^2 = sum_{i not in the small group, i < N} (z_i . t - Q_ib).
// This is a second, independent reduction of the same quantities (route 2 of
// the statistic); it runs on FP32 MFMA (v_mfma_f32_16x16x4f32) when the first
// product is FP32 or FP64, and on split-BF16 MFMA (three terms) when it is
// split BF16.
#include <type_traits>

#include "hbt_launch.h"

namespace hbt {

typedef float f32x4c __attribute__((ext_vector_type(4)));

// z_i . t for every pooled row (FP64 accumulation of the stored FP32 row):
// one wave per row, each lane four consecutive columns per 16-byte load
// (d_pad is a multiple of 64, so rows of z32 and t64 are 16-byte aligned).
__global__ __launch_bounds__(256) void k_row_dot_t(const PairDesc* __restrict__ pairs, int npairs,
                                                   const float* __restrict__ z32,
                                                   const double* __restrict__ t64, int d_pad,
                                                   int64_t total_rows, double* __restrict__ zt) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + wave;
    if (r >= total_rows) return;
    const int p = upper_index(npairs, r, [&](int k) { return pairs[k].zrow0; });
    const float4* zr = (const float4*)(z32 + r * d_pad);
    const double2* tp = (const double2*)(t64 + (int64_t)p * d_pad);
    double s = 0.0;
    for (int c = lane; 4 * c < d_pad; c += 64) {
        const float4 z = zr[c];
        const double2 t0 = tp[2 * c], t1 = tp[2 * c + 1];
        s += (double)z.x * t0.x + (double)z.y * t0.y + (double)z.z * t1.x + (double)z.w * t1.y;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) zt[r] = s;
}

hipError_t launch_row_dot_t(const PairDesc* pairs, int npairs, const float* z32,
                            const double* t64, int d_pad, int64_t total_rows, double* zt,
                            hipStream_t s) {
    if (total_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_dot_t, dim3((unsigned)((total_rows + 3) / 4)), dim3(256), 0, s, pairs,
                       npairs, z32, t64, d_pad, total_rows, zt);
    return hipGetLastError();
}

// Work-group tile: 128 pooled rows x 256 splits of one pair (CTile), eight
// waves, wave w owning rows [64 (w / 4), +64) and splits [64 (w % 4), +64).
// K = d runs in chunks of 32 columns staged through LDS: each thread loads its
// share of the next chunk (Z: 128 rows x 32 columns, 2 coalesced 16-byte
// loads; S: 256 split rows x 32 columns, 4 loads) into registers while the
// current chunk is multiplied from LDS, then stores it after a barrier.  Both
// row halves share each staged chunk of S, so a split's centroid is read
// once per 128 pooled rows (with 64-row tiles the re-reads of S from L2
// bounded the kernel).  Two products:
//  * FP32 (v_mfma_f32_16x16x4f32): the wave tile is 4 x 4 blocks of 16 x 16;
//    K is taken four at a time per lane (lane l holds k = 4(l/16) .. +3 of a
//    16-wide step as one 16-byte LDS read), each of the four MFMAs of a step
//    consuming one of them (A lane l -> row l%16, k slot l/16; B the same k
//    slot, col l%16; D lane l -> col l%16, rows 4(l/16) + v).
//  * split BF16, three terms (v_mfma_f32_32x32x16_bf16): z = zh + zl and
//    s = sh + sl split (round to nearest even) once, as the chunk is staged
//    into LDS as bf16 planes, Q += zh sh + zh sl + zl sh (the zl sl term, below
//    2^-16 |z| |s|, is dropped); the wave tile is 2 x 2 blocks of 32 x 32
//    (A lane l -> row l%32, k 8(l/32) .. +7; D lane l -> col l%32, rows
//    8(v/4) + 4(l/32) + v%4).
// Epilogue: per split, the masked sums of Q over the tile's rows,
// partial[row tile][split row] = (sum_small Q, sum_{other, i < N} (z_i . t - Q)).
constexpr int kCK = 32;       // K columns per staged chunk
constexpr int kCStride = 36;  // LDS row stride in floats (chunk + 4 padding)

typedef __bf16 bf16x8c __attribute__((ext_vector_type(8)));
typedef float f32x16c __attribute__((ext_vector_type(16)));

// hi = bf16(x), lo = bf16(x - hi) of 8 floats
__device__ __forceinline__ void split8(const float4& u, const float4& v, bf16x8c& hi, bf16x8c& lo) {
    const float x[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 h = (__bf16)x[e];
        hi[e] = h;
        lo[e] = (__bf16)(x[e] - (float)h);
    }
}

template <bool BF>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(BF ? 4 : 3))) void k_centroid(const PairDesc* __restrict__ pairs,
                                                  const BlockPair* __restrict__ bp,
                                                  const CTile* __restrict__ tiles, int d_pad,
                                                  const float* __restrict__ z32,
                                                  const float* __restrict__ sig,
                                                  const uint32_t* __restrict__ mask,
                                                  const double* __restrict__ zt,
                                                  double* __restrict__ partial, int64_t prow) {
    // FP32 mode: the chunk as floats; split-BF16 mode: its hi and lo parts as
    // bf16, split once when staged
    constexpr int kBStride = kCK + 8;  // bf16 row stride (80 bytes)
    constexpr int kSL = kTileB * kCK / 4 / 512;  // 16-byte loads of S per thread and chunk (4)
    __shared__ __attribute__((aligned(16))) float Zs[BF ? 1 : kCTileRows][kCStride];
    __shared__ __attribute__((aligned(16))) float Ss[BF ? 1 : kTileB][kCStride];
    __shared__ __attribute__((aligned(16))) __bf16 Zb[BF ? 2 : 1][BF ? kCTileRows : 1][kBStride];
    __shared__ __attribute__((aligned(16))) __bf16 Sb[BF ? 2 : 1][BF ? kTileB : 1][kBStride];
    const CTile tile = tiles[blockIdx.x];
    const PairDesc pd = pairs[tile.pair];
    const BlockPair bq = bp[tile.pair];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int wr = wave >> 2, ws = wave & 3;  // the wave's row half and split quarter
    const int i0 = tile.i0, b0 = tile.b0;
    const int N = pd.n + pd.m;
    // this thread's loads of a chunk
    const float* zsrc = z32 + (pd.zrow0 + i0 + (t >> 2)) * (int64_t)d_pad + 8 * (t & 3);
    // split rows b0 + (t >> 3) + 64 j; those past the block read nothing
    const float* ssrc = sig + (bq.mrow0 + b0 + (t >> 3)) * (int64_t)d_pad + 4 * (t & 7);
    const int nval = bq.nb - b0 - (t >> 3);  // j < ceil(nval / 64) are valid
    float4 zr[2], sr[kSL];
    auto fetch = [&](int k0) {
        zr[0] = *(const float4*)(zsrc + k0);
        zr[1] = *(const float4*)(zsrc + k0 + 4);
#pragma unroll
        for (int j = 0; j < kSL; ++j)
            sr[j] = 64 * j < nval ? *(const float4*)(ssrc + (int64_t)64 * j * d_pad + k0)
                                  : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    auto stage = [&]() {
        if constexpr (BF) {
            bf16x8c h, l;
            split8(zr[0], zr[1], h, l);
            *(bf16x8c*)&Zb[0][t >> 2][8 * (t & 3)] = h;
            *(bf16x8c*)&Zb[1][t >> 2][8 * (t & 3)] = l;
#pragma unroll
            for (int j = 0; j < kSL; ++j) {
                const uint2 hl0 = split_bf16x2(sr[j].x, sr[j].y), hl1 = split_bf16x2(sr[j].z, sr[j].w);
                *(uint2*)&Sb[0][(t >> 3) + 64 * j][4 * (t & 7)] = make_uint2(hl0.x, hl1.x);
                *(uint2*)&Sb[1][(t >> 3) + 64 * j][4 * (t & 7)] = make_uint2(hl0.y, hl1.y);
            }
        } else {
            *(float4*)&Zs[t >> 2][8 * (t & 3)] = zr[0];
            *(float4*)&Zs[t >> 2][8 * (t & 3) + 4] = zr[1];
#pragma unroll
            for (int j = 0; j < kSL; ++j) *(float4*)&Ss[(t >> 3) + 64 * j][4 * (t & 7)] = sr[j];
        }
    };
    constexpr int NA = BF ? 2 : 4;   // row blocks per wave
    constexpr int NB = BF ? 2 : 4;   // split blocks per wave
    constexpr int NV = BF ? 16 : 4;  // accumulator floats per block
    using Acc = typename std::conditional<BF, f32x16c, f32x4c>::type;
    Acc acc[NA][NB];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[a][b][v] = 0.0f;
    fetch(0);
    for (int k0 = 0; k0 < d_pad; k0 += kCK) {
        __syncthreads();  // the previous chunk has been read
        stage();
        __syncthreads();
        if (k0 + kCK < d_pad) fetch(k0 + kCK);  // in flight during this chunk's products
#pragma unroll
        for (int kk = 0; kk < kCK; kk += 16) {
            if constexpr (BF) {
                bf16x8c ah[2], al[2], bh[2], bl[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int r = 64 * wr + 32 * a + (lane & 31), k = kk + 8 * (lane >> 5);
                    ah[a] = *(const bf16x8c*)&Zb[0][r][k];
                    al[a] = *(const bf16x8c*)&Zb[1][r][k];
                }
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int r = 64 * ws + 32 * b + (lane & 31), k = kk + 8 * (lane >> 5);
                    bh[b] = *(const bf16x8c*)&Sb[0][r][k];
                    bl[b] = *(const bf16x8c*)&Sb[1][r][k];
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                    }
            } else {
                float4 av[4], bv[4];
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    av[a] = *(const float4*)&Zs[64 * wr + 16 * a + (lane & 15)][kk + 4 * (lane >> 4)];
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    bv[b] = *(const float4*)&Ss[64 * ws + 16 * b + (lane & 15)][kk + 4 * (lane >> 4)];
                const float* af = (const float*)av;
                const float* bf = (const float*)bv;
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[4 * a + q], bf[4 * b + q], acc[a][b],
                                                                             0, 0, 0);
            }
        }
    }
    // epilogue: masked sums per split column
    const uint32_t flip = pd.flip ? 0xffffffffu : 0u;
    const int iw = i0 + 64 * wr;  // the wave's 64 rows
    const double* ztp = zt + pd.zrow0 + iw;
    constexpr int CW = BF ? 32 : 16;  // columns per block
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int brow = b0 + 64 * ws + CW * b + (lane % CW);
        const bool valid = brow < bq.nb;
        const uint32_t* mk = mask_row(mask, bq, bq.mrow0 + (valid ? brow : 0), pd.Wp);
        const uint2 w = *(const uint2*)(mk + (iw >> 5));  // rows iw .. iw + 63 of this split
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int r = BF ? 32 * a + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)
                                 : 16 * a + 4 * (lane >> 4) + v;  // row within the wave's 64
                const int i = iw + r;
                const uint32_t word = r < 32 ? w.x : w.y;
                const bool small = (((word ^ flip) >> (r & 31)) & 1u) && i < N;
                const double Q = (double)acc[a][b][v];
                if (small) s1 += Q;
                else if (i < N) s2 += ztp[r] - Q;
            }
        if (!BF) {
            s1 += __shfl_xor(s1, 16, 64);
            s2 += __shfl_xor(s2, 16, 64);
        }
        s1 += __shfl_xor(s1, 32, 64);
        s2 += __shfl_xor(s2, 32, 64);
        if (lane < CW && valid) {
            double2* out = (double2*)partial + (int64_t)(iw / 64) * prow + bq.mrow0 + brow;
            *out = make_double2(s1, s2);
        }
    }
}

hipError_t launch_centroid(bool bf16x3, const PairDesc* pairs, const BlockPair* bp, const CTile* tiles,
                           int ntiles, int d_pad, const float* z32, const float* sig,
                           const uint32_t* mask, const double* zt, double* partial,
                           int64_t prow, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (bf16x3)
        hipLaunchKernelGGL(k_centroid<true>, dim3((unsigned)ntiles), dim3(512), 0, s, pairs, bp, tiles, d_pad,
                           z32, sig, mask, zt, partial, prow);
    else
        hipLaunchKernelGGL(k_centroid<false>, dim3((unsigned)ntiles), dim3(512), 0, s, pairs, bp, tiles, d_pad,
                           z32, sig, mask, zt, partial, prow);
    return hipGetLastError();
}

}  // namespace hbt
