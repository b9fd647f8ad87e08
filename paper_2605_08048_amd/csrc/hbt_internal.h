// Internal plan structures and device helpers of the HIP path (gfx950).
// Host and device code of the library include this header; it is not part of
// the public ABI (include/hbt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hbt.h"

namespace hbt {

// Pooled rows of a pair are padded to a multiple of kRowPad in the Z
// storage (zero rows), columns to a multiple of kDPad (zero columns).
constexpr int kRowPad = 128;
constexpr int kDPad = 64;
// Each group-sum tile reduces its squared norms over kDSlot columns; the
// statistic kernel adds the d_pad / kDSlot slots of a split row in FP64.
constexpr int kDSlot = 64;
// Splits per work-group of the int8 digit-plane kernel (one tile width).
constexpr int kTileI8 = 512;
// Split rows per group-sum tile (4 waves x 64 rows).
constexpr int kTileB = 256;
// Capacity of the boundary bucket of the split selection (items whose
// primary key equals the selected byte; about N / 256 of them).
constexpr int kCandCap = 512;

// One pair of clouds (device table entry, 96 bytes).
struct PairDesc {
    const void* X;       // n rows of d values (input dtype)
    const void* Y;       // m rows
    int32_t n, m;
    int32_t Np;          // n + m rounded up to kRowPad
    int32_t Wp;          // mask words per split row in the workspace (Np / 32)
    int64_t zrow0;       // first row of this pair in the Z storage
    int64_t coef0;       // first of its n reflection coefficients
    uint32_t pair_index; // Philox counter word 2
    int32_t flip;        // 1 when m < n: group sums run on the group-2 mask
    int32_t cx0, cx1;    // column-sum chunks of X: [cx0, cx1); of Y: [cy0, cy1)
    int32_t cy1;
    int32_t cy0;         // (= cx1 when X and Y are stored as one pooled run)
    int64_t xoct0;       // first of its x_octets(n) octets in the numbering of the storage
                         // octets that hold X rows (the reflection's work items)
    // Two-run storage (pairs of shared clouds): the pooled rows [0, Np) are
    // nxc 128-row chunks of X's storage from zrow0, then Y's storage from
    // zrow_y; in the pooled (and mask) order Y's rows start at n + ygap, the
    // ygap rows between being X's padding.  One run: nxc = Np / 128, ygap = 0.
    int64_t zrow_y;
    int32_t nxc;
    int32_t ygap;
};
static_assert(sizeof(PairDesc) == 96, "PairDesc layout");

// Splits of one pair inside the current block (device table entry).
struct BlockPair {
    int64_t mrow0;       // first split row of the pair in the block buffers
    int64_t mword0;      // first mask word of that row (rows hold Wp words)
    uint32_t perm_base;  // global index of that split
    int32_t nb;          // splits of the pair in this block
    int32_t owner;       // the pair whose split rows draw these masks: itself, or
                         // the first pair with the same n, m, B and pair index
                         // (identical splits), whose mask words mword0 points at
    // copies of the pair's PairDesc fields that the split stage reads, so that
    // it needs this table only
    int32_t n, m;
    int32_t Wp;          // mask words per split row (Np / 32)
    uint32_t pair_index; // Philox counter word 2
    int32_t ygap;        // PairDesc::ygap: Y's items sit ygap positions further in the mask
};
static_assert(sizeof(BlockPair) == 48, "BlockPair layout");

#ifdef __HIPCC__
// The bits of mask word w that stand for items (not padding): positions
// [0, n) (X) and [n + ygap, n + m + ygap) (Y).
__device__ __forceinline__ uint32_t range_bits(int w, int lo, int hi) {
    const int a = lo > 32 * w ? lo - 32 * w : 0, b = hi < 32 * w + 32 ? hi - 32 * w : 32;
    if (a >= b) return 0u;
    const uint32_t upto_b = b == 32 ? 0xffffffffu : (1u << b) - 1u;
    return upto_b & ~((1u << a) - 1u);
}
__device__ __forceinline__ uint32_t item_bits(int w, int n, int m, int ygap) {
    return range_bits(w, 0, n) | range_bits(w, n + ygap, n + m + ygap);
}
#endif

#ifdef __HIPCC__
// Mask words of split row `row` (a block row of pair bq).
__device__ __forceinline__ const uint32_t* mask_row(const uint32_t* mask, const BlockPair& bq,
                                                    int64_t row, int Wp) {
    return mask + bq.mword0 + (row - bq.mrow0) * (int64_t)Wp;
}
#endif

// A run of rows of one cloud for the column sums.
struct SumChunk {
    int32_t pair, side;  // side 0 = X, 1 = Y
    int32_t r0, r1;
};
constexpr int kSumChunk = 128;  // X rows per column-sum chunk
constexpr int kSumChunkY = 32;  // pooled rows per Y chunk: one 32-row group of the Z storage
// Storage octets of a pair that hold X rows: the 32-row groups that hold any.
__host__ __device__ constexpr int64_t x_octets(int64_t n) { return 4 * ((n + 31) / 32); }

// A group-sum tile of the FP32 / FP64 kernels: kTileB split rows of one pair
// (the grid covers all column slots).
struct GemmTile {
    int32_t pair;
    int32_t b0;          // first split of the tile, relative to the pair's block rows
};

// A point-to-centroid tile: kCTileRows pooled rows [i0, i0 + kCTileRows) x
// kTileB split rows [b0, b0 + kTileB) of one pair's block rows.  Its partial
// sums are written per 64 rows (pooled sizes are padded to 128).
constexpr int kCTileRows = 128;
struct CTile {
    int32_t pair;
    int32_t b0;
    int32_t i0;
    int32_t _pad;
};

// The split-BF16 kernel's tiles of one pair: nbt split tiles x (d_pad / 64)
// column slices, numbered from tile0 (slice-major, split tile fastest).
struct GemmGroup {
    int32_t pair;
    int32_t nbt;
    int64_t tile0;
};

// FP64 per-pair state written by the finalize kernel.
struct PairState {
    double r_x, r_y, t_obs, tau, vv, f_x, f_y;
    double vt;           // v . t (t the pooled total of the aligned rows)
    int32_t identity, status;
    int32_t _pad2[2];
};

// Device-side counters of a pair (zeroed at the start of a call).
struct PairCount {
    unsigned long long count;
    unsigned long long n_recheck;
    double sum_dt, sum_dt2;  // sums of T_b - T_obs and of its square, block by block
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
#ifdef __HIPCC__

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products, Weyl key schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        // each three-way XOR as one v_bitop3 (truth table 0x96 = a ^ b ^ c)
        c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, (unsigned char)0x96),
                       (uint32_t)p1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, (unsigned char)0x96),
                       (uint32_t)p0);
    }
    return c;
}

// Memory fence + scheduling barrier among the lanes of one wave, for LDS
// data written by one lane and read by another.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Inclusive prefix sum over the 64 lanes of a wave (all lanes active): a
// Kogge-Stone scan inside each row of 16 lanes by DPP row shifts, then the
// row totals carried across rows by row broadcasts of lanes 15 and 31.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    int v = (int)x;
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 -> rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 -> rows 2, 3
    return (uint32_t)v;
}

// Split of two floats into BF16 hi + lo parts: hi = bf16(a), lo =
// bf16(a - hi), both round-to-nearest-even (the gfx950 packed conversion
// v_cvt_pk_bf16_f32); returns the packed hi pair and lo pair (element a in
// the low 16 bits).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint2 split_bf16x2(float a, float b) {
    const f32x2_t f = {a, b};
    const bf16x2_t hi = __builtin_convertvector(f, bf16x2_t);
    const bf16x2_t lo = __builtin_convertvector(f - __builtin_convertvector(hi, f32x2_t), bf16x2_t);
    return make_uint2(__builtin_bit_cast(uint32_t, hi), __builtin_bit_cast(uint32_t, lo));
}

// Split-BF16 row order and scaling.  The group-sum kernel turns a 32-bit
// mask word (32 pooled rows) into its bf16 operand with one AND per register:
// register e (0..7) of a lane is w & (0x00800080 << e), w the word rotated
// right by 8 in the upper half of the wave.  A set bit thus becomes a bf16
// whose only set bit is exponent bit e, the power of two 2^(2^e - 127)
// instead of 1, and the rows that meet exponent bit e are stored divided by
// it, so every product is the row value itself (scaling by a power of two is
// exact, and |z| <= 1 keeps z * 2^126 finite).  Storage octet o4 = 2 s + h
// (0..3) of a 32-row group, position k (0..7), holds group row
// bf16_plane_row(o4, k), multiplied by bf16_plane_scale(o4, k).
__host__ __device__ constexpr int bf16_plane_row(int o4, int k) {
    return ((k & 1 ? 23 : 7) + 4 * (o4 >> 1) + (k >> 1) + 8 * (o4 & 1)) & 31;
}
constexpr bool bf16_plane_rows_ok() {  // a permutation of the 32 rows
    uint32_t seen = 0;
    for (int o = 0; o < 4; ++o)
        for (int k = 0; k < 8; ++k) seen |= 1u << bf16_plane_row(o, k);
    return seen == 0xffffffffu;
}
static_assert(bf16_plane_rows_ok(), "split-BF16 row order must be a permutation");
__device__ __forceinline__ float bf16_plane_scale(int o4, int k) {
    const int e = 4 * (o4 >> 1) + (k >> 1);
    return __uint_as_float((uint32_t)(254 - (1 << e)) << 23);  // 2^(127 - 2^e)
}

__device__ __forceinline__ float bf16_plane_inv_scale(int o4, int k) {
    const int e = 4 * (o4 >> 1) + (k >> 1);
    return __uint_as_float((uint32_t)(1 << e) << 23);  // 2^(2^e - 127)
}

// BF16 hi + E4M3 lo: the hi plane is the split-BF16 hi plane; the lo plane
// holds e4m3(lo 2^kE4m3LoShift), lo = z - hi exact in FP32 (|lo| <= 2^-9 |z|,
// so a unit row's values stay below e4m3's largest finite 448), one byte per
// value in 16-row units [rows/16][d_pad][16]: unit f8_unit(r) of a 32-row
// group, byte f8_byte(r), holds group row r (the int8 planes' order).
constexpr int kE4m3LoShift = 17;
__host__ __device__ constexpr int f8_unit(int r) { return (r & 7) >> 2; }
__host__ __device__ constexpr int f8_byte(int r) { return 4 * (r & 3) + (r >> 3); }

// Int8 digit planes.  z is rounded to Q = round(z 2^20) and written as three
// balanced base-128 digits, Q = q0 2^14 + q1 2^7 + q2 (q1, q2 in [-64, 63],
// |q0| <= 64 for |z| <= 1), stored as the int8 planes q0, -q1, q2 (the
// group-sum kernel multiplies the middle plane by the mask byte -128, which
// folds 2^7 q1 into the sum of q2 exactly).  Storage unit: 16 rows of one column
// (16 bytes, the int8 MFMA operand of one lane); unit h (0, 1) of a 32-row
// group, byte p = 4 s + b, holds group row s + 4 h + 8 b, so that the group-sum
// kernel makes operand register s of lane half h as (w >> (s + 4 h)) &
// 0x01010101 from the group's mask word w.  A wave of the reflection writes
// half a unit: storage octet o4 (0..3) of a group = unit o4 / 2, bytes
// 8 (o4 & 1) .. +7, position k (0..7) holding group row i8_plane_row(o4, k).
__host__ __device__ constexpr int i8_plane_row(int o4, int k) {
    return 2 * (o4 & 1) + (k >> 2) + 4 * (o4 >> 1) + 8 * (k & 3);
}
constexpr bool i8_plane_rows_ok() {
    uint32_t seen = 0;
    for (int o = 0; o < 4; ++o)
        for (int k = 0; k < 8; ++k) seen |= 1u << i8_plane_row(o, k);
    return seen == 0xffffffffu;
}
static_assert(i8_plane_rows_ok(), "int8 row order must be a permutation");
// the three plane bytes of z: q0, -q1, q2
__device__ __forceinline__ void i8_digits(double z, uint32_t& q0, uint32_t& q1, uint32_t& q2) {
    const int Q = __double2int_rn(z * 1048576.0);
    const int d2 = ((Q + 64) & 127) - 64;
    const int Q1 = (Q - d2) >> 7;  // exact: Q - d2 is a multiple of 128
    const int d1 = ((Q1 + 64) & 127) - 64;
    const int d0 = (Q1 - d1) >> 7;
    q0 = (uint32_t)d0 & 0xffu;
    q1 = (uint32_t)(-d1) & 0xffu;  // stored negated
    q2 = (uint32_t)d2 & 0xffu;
}

// log g_d(r) of Sec. 3.1 ("Dispersion proxy"), in FP64.
__host__ __device__ inline double log_g(double r, double d, int gd) {
    if (gd == HBT_GD_IDENTITY) return log(r);
    const double rr = r * r;
    return log(r * (d - rr) / ((1.0 - r) * (1.0 + r)));
}

// |s * d/ds log g_d(sqrt(s))| for s = r^2: the factor by which a relative
// error of s moves log g_d.
__host__ __device__ inline double log_g_sensitivity(double s, double d, int gd) {
    if (gd == HBT_GD_IDENTITY) return 0.5;
    return fabs(0.5 - s / (d - s) + s / (1.0 - s));
}

// Recheck band: how far a reduced-precision T_b may lie from the FP64 value.
// The product runs over the smaller group (k = min(n, m) items) and the
// larger group's sum is t - sigma_small with an FP64 t, so both squared norms
// carry the one error vector E of sigma_small:
//   |sigma_g + E|^2 - |sigma_g|^2 = 2 sigma_g . E + |E|^2   (group g = 1, 2).
// Per coordinate the stored rows are off by at most e_row (a unit row's RMS
// coordinate scale times the storage format's bound).  Rows may repeat (the
// same sentence twice gives the same vectors), so the k errors in E can add
// coherently: |E| is not assumed to shrink as 1/sqrt(k).  Across the d
// coordinates the rounding errors are taken as unrelated to the direction of
// sigma_g, which gives, relative to |sigma_g|^2 = (n_g r_g)^2,
//   rel_g = e_acc + a_g / r_g + a_g^2 d / r_g^2,   a_g = s_store e_row k / n_g,
// with e_acc the accumulation error of the product (relative to the sums).
// The point-to-centroid route adds the error of its K = d dot products
// z_i . sigma (FP32, or split BF16 in three terms): up to e_q sqrt(d)
// |sigma_small| each, summed over k (small group) or the N - k others
// (large group).  A relative error rel of r^2
// moves log g_d(r) by rel * sensitivity(r^2).
struct RecheckBand {
    double e_acc;    // relative accumulation error of the group sums
    double e_row;    // per-coordinate storage error scale of a unit row
    double s_store;  // safety factor on the storage term
    double e_q;      // point-to-centroid dot-product error (0: route 0)
};
__host__ __device__ inline double recheck_eps(const RecheckBand& b, double n, double m, double d,
                                              double r1, double r2, int gd) {
    const double k = n < m ? n : m;
    const double a1 = b.s_store * b.e_row * (k / n), a2 = b.s_store * b.e_row * (k / m);
    double rel1 = b.e_acc + a1 / r1 + a1 * a1 * d / (r1 * r1);
    double rel2 = b.e_acc + a2 / r2 + a2 * a2 * d / (r2 * r2);
    if (b.e_q > 0.0) {
        const bool small1 = n <= m;
        const double rs = small1 ? r1 : r2, rl = small1 ? r2 : r1;
        const double ql = b.e_q * sqrt(d) * (k / (n + m - k)) * rs / (rl * rl);
        const double qs = b.e_q * sqrt(d) / rs;
        rel1 += small1 ? qs : ql;
        rel2 += small1 ? ql : qs;
    }
    const double fs = fabs(log_g(r1, d, gd)) + fabs(log_g(r2, d, gd));
    return rel1 * log_g_sensitivity(r1 * r1, d, gd) + rel2 * log_g_sensitivity(r2 * r2, d, gd) +
           1e-13 * fs;
}

// Binary search: last index k in [0, count) with key(k) <= x, for an
// ascending sequence of keys.
template <typename F>
__device__ __forceinline__ int upper_index(int count, int64_t x, F key) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (key(mid) <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Column-sum chunk c: chunks are numbered pair by pair, the X chunks of a
// pair ([cx0, cx1)) before its Y chunks ([cx1, cy1)).  X chunk k holds X rows
// [kSumChunk k, kSumChunk (k + 1)) (clipped to n).  The Y chunks are the
// 32-row groups of the Z storage from the one holding row n to the padded
// end Np: Y chunk k holds pooled rows [max(n, 32 j), min(n + m, 32 (j + 1)))
// (none for the groups of padding only), j = n / 32 + k.
__device__ __forceinline__ SumChunk chunk_of(const PairDesc* pairs, int npairs, int c) {
    const int p = upper_index(npairs, c, [&](int k) { return pairs[k].cx0; });
    const int cx0 = pairs[p].cx0, cx1 = pairs[p].cx1;
    const int n = pairs[p].n, N = n + pairs[p].m;
    SumChunk ch;
    ch.pair = p;
    ch.side = c < cx1 ? 0 : 1;
    if (!ch.side) {
        ch.r0 = (c - cx0) * kSumChunk;
        ch.r1 = ch.r0 + kSumChunk < n ? ch.r0 + kSumChunk : n;
    } else {
        const int j = n / kSumChunkY + (c - cx1);
        ch.r0 = (kSumChunkY * j > n ? kSumChunkY * j : n) - n;
        ch.r1 = (kSumChunkY * (j + 1) < N ? kSumChunkY * (j + 1) : N) - n;
    }
    return ch;
}

#endif  // __HIPCC__

}  // namespace hbt
