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
// the statistic); it runs on FP32 MFMA (v_mfma_f32_16x16x4f32) for every
// precision of the first product.
#include "hbt_launch.h"

namespace hbt {

typedef float f32x4c __attribute__((ext_vector_type(4)));

// z_i . t for every pooled row (FP64 accumulation of the stored FP32 row).
__global__ __launch_bounds__(256) void k_row_dot_t(const PairDesc* __restrict__ pairs, int npairs,
                                                   const float* __restrict__ z32,
                                                   const double* __restrict__ t64, int d_pad,
                                                   int64_t total_rows, double* __restrict__ zt) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + wave;
    if (r >= total_rows) return;
    const int p = upper_index(npairs, r, [&](int k) { return pairs[k].zrow0; });
    const float* zr = z32 + r * d_pad;
    const double* tp = t64 + (int64_t)p * d_pad;
    double s = 0.0;
    for (int c = lane; c < d_pad; c += 64) s += (double)zr[c] * tp[c];
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

// Work-group tile: 64 pooled rows x 256 splits (4 waves along the splits,
// each 64 x 64 as 4 x 4 blocks of 16 x 16); K = d in steps of 4.
// A (16 x 4) lane l -> row l%16, k l/16; B (4 x 16) lane l -> k l/16, col
// l%16; D lane l -> col (split) l%16, rows (pooled) 4(l/16) + v.
// Output: partial[split row][row tile] = (sum M Q, sum (1 - M)(z.t - Q)).
__global__ __launch_bounds__(256) void k_centroid(const PairDesc* __restrict__ pairs,
                                                  const BlockPair* __restrict__ bp,
                                                  const GemmTile* __restrict__ tiles,
                                                  int ntile_i, int d_pad,
                                                  const float* __restrict__ z32,
                                                  const float* __restrict__ sig,
                                                  const uint32_t* __restrict__ mask,
                                                  const double* __restrict__ zt,
                                                  double* __restrict__ partial, int64_t prow) {
    const GemmTile tile = tiles[blockIdx.x / ntile_i];
    const int itile = blockIdx.x % ntile_i;
    const PairDesc pd = pairs[tile.pair];
    const BlockPair bq = bp[tile.pair];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane >> 4, c = lane & 15;
    const int i0 = itile * 64;
    const int N = pd.n + pd.m;
    if (i0 >= pd.Np) return;  // row tiles past this pair's rows (pairs differ in size)
    int brow[4];
    bool valid[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        brow[j] = tile.b0 + wave * 64 + 16 * j + c;
        valid[j] = brow[j] < bq.nb;
    }
    const float* za = z32 + (pd.zrow0 + i0 + c) * (int64_t)d_pad + q;
    const float* sb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        sb[j] = sig + (bq.mrow0 + (valid[j] ? brow[j] : 0)) * (int64_t)d_pad + q;
    f32x4c acc[4][4];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[ii][j][v] = 0.0f;
    for (int k = 0; k < d_pad; k += 4) {
        float a[4], b[4];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) a[ii] = za[(int64_t)16 * ii * d_pad + k];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = valid[j] ? sb[j][k] : 0.0f;
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[ii][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ii], b[j], acc[ii][j], 0, 0, 0);
    }
    const uint32_t flip = pd.flip ? 0xffffffffu : 0u;
    const double* ztp = zt + pd.zrow0 + i0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t* mk = mask_row(mask, bq, bq.mrow0 + (valid[j] ? brow[j] : 0), pd.Wp);
        const uint2 w = *(const uint2*)(mk + (i0 >> 5));  // rows i0 .. i0+63 of this split
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * ii + 4 * q + v;  // row within the tile
                const int i = i0 + r;
                const uint32_t word = r < 32 ? w.x : w.y;
                const bool small = (((word ^ flip) >> (r & 31)) & 1u) && i < N;
                const double Q = (double)acc[ii][j][v];
                if (small) s1 += Q;
                else if (i < N) s2 += ztp[r] - Q;
            }
        s1 += __shfl_xor(s1, 16, 64);
        s2 += __shfl_xor(s2, 16, 64);
        s1 += __shfl_xor(s1, 32, 64);
        s2 += __shfl_xor(s2, 32, 64);
        if (q == 0 && valid[j]) {
            double2* out = (double2*)partial + itile * prow + bq.mrow0 + brow[j];
            *out = make_double2(s1, s2);
        }
    }
}

hipError_t launch_centroid(const PairDesc* pairs, const BlockPair* bp, const GemmTile* tiles,
                           int ntiles, int ntile_i, int d_pad, const float* z32, const float* sig,
                           const uint32_t* mask, const double* zt, double* partial,
                           int64_t prow, hipStream_t s) {
    if (ntiles <= 0 || ntile_i <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_centroid, dim3((unsigned)(ntiles * ntile_i)), dim3(256), 0, s, pairs, bp,
                       tiles, ntile_i, d_pad, z32, sig, mask, zt, partial, prow);
    return hipGetLastError();
}

}  // namespace hbt
