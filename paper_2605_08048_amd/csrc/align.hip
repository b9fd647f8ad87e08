// Mean directions, Householder reflection and observed statistic on the GPU
// (Sec. 3.1 "Householder mean-direction alignment", eq:householder_fast,
// eq:tobs; Algorithm 1, Steps 1-4).  All reductions are FP64 and run in a
// fixed order, so results do not depend on timing.
#include <string.h>

#include "hbt_launch.h"

namespace hbt {

// ---------------------------------------------------------------------------
// small utilities: table upload through kernel arguments, zero fill
// ---------------------------------------------------------------------------
struct UploadChunk {
    unsigned char b[3072];
};

__global__ void k_upload(unsigned char* dst, UploadChunk c, int bytes) {
    for (int i = threadIdx.x; i < bytes; i += blockDim.x) dst[i] = c.b[i];
}

hipError_t upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const unsigned char* p = (const unsigned char*)src;
    unsigned char* q = (unsigned char*)dst;
    while (bytes) {
        const size_t k = bytes < sizeof(UploadChunk) ? bytes : sizeof(UploadChunk);
        UploadChunk c;
        memcpy(c.b, p, k);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, q, c, (int)k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        p += k;
        q += k;
        bytes -= k;
    }
    return hipSuccess;
}

__global__ void k_zero(uint64_t* dst, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = 0;
}

hipError_t zero(void* dst, size_t bytes, hipStream_t s) {
    const int64_t words = (int64_t)(bytes / 8);
    if (!words) return hipSuccess;
    int64_t g = (words + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)g), dim3(256), 0, s, (uint64_t*)dst, words);
    return hipGetLastError();
}

// Unit-row check of the inputs (Sec. 3.1, Eq. 2: every embedding is
// l2-normalised before the test): a row fails when | |x| - 1 | > 1e-4,
// i.e. |x|^2 outside [(1 - 1e-4)^2, (1 + 1e-4)^2]; NaN fails too.  The
// column-sum pass reads every row once, so it tests them there and writes one
// flag per chunk (1 = some row of the chunk failed); the finalize step turns
// a pair's flags into the status HBT_ERR_NOT_UNIT.
__device__ __forceinline__ bool not_unit(double ss) {
    return !(ss >= 0.99980001 && ss <= 1.00020001);
}

// Sum of x over the 64 lanes of a wave, returned to every lane: an inclusive
// scan by DPP row shifts and row broadcasts (lane 63 ends with the total),
// then a read of lane 63.
__device__ __forceinline__ float wave_total_f32(float x) {
    float v = x;
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// ---------------------------------------------------------------------------
// column sums: one work-group = 64 columns x one chunk of rows, 4 row phases
// ---------------------------------------------------------------------------
template <typename Tin>
__global__ __launch_bounds__(256) void k_colsum(const PairDesc* __restrict__ pairs,
                                                int npairs, int d,
                                                double* __restrict__ partial,
                                                int32_t* __restrict__ chunk_bad) {
    const SumChunk ch = chunk_of(pairs, npairs, blockIdx.x);
    const PairDesc pd = pairs[ch.pair];
    const Tin* base = (const Tin*)(ch.side ? pd.Y : pd.X);
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    if (blockIdx.y == 0) {  // the first column tile also tests whole rows (wave ty: rows ty, ty + 4, ...)
        bool bad = false;
        for (int r = ch.r0 + ty; r < ch.r1; r += 4) {
            double ss = 0.0;
            for (int cc = tx; cc < d; cc += 64) {
                const double a = (double)base[(int64_t)r * d + cc];
                ss += a * a;
            }
            for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
            bad |= not_unit(ss);
        }
        bad = __syncthreads_or(bad);
        if (threadIdx.x == 0) chunk_bad[blockIdx.x] = bad ? 1 : 0;
    }
    const int c = blockIdx.y * 64 + tx;
    double s0 = 0.0, s1 = 0.0;
    if (c < d) {
        int r = ch.r0 + ty;
        for (; r + 4 < ch.r1; r += 8) {
            const double a = (double)base[(int64_t)r * d + c];
            const double b = (double)base[(int64_t)(r + 4) * d + c];
            s0 += a;
            s1 += b;
        }
        if (r < ch.r1) s0 += (double)base[(int64_t)r * d + c];
    }
    __shared__ double red[4][64];
    red[ty][tx] = s0 + s1;
    __syncthreads();
    if (ty == 0 && c < d)
        partial[(int64_t)blockIdx.x * d + c] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

hipError_t launch_colsum(int input_dtype, const PairDesc* pairs, int npairs,
                         int nchunks, int d, double* partial, int32_t* chunk_bad, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    dim3 grid(nchunks, (d + 63) / 64);
    if (input_dtype == HBT_IN_F64)
        hipLaunchKernelGGL(k_colsum<double>, grid, dim3(256), 0, s, pairs, npairs, d, partial, chunk_bad);
    else
        hipLaunchKernelGGL(k_colsum<float>, grid, dim3(256), 0, s, pairs, npairs, d, partial, chunk_bad);
    return hipGetLastError();
}

// FP32 rows with d a multiple of 4 and 16-byte aligned rows: one
// work-group = one chunk of rows x all columns; wave w sums rows w, w+4, ...
// of the chunk with 16-byte loads (lane l: columns 4(l + 64 j) .. +3), the
// four waves' sums are added in a fixed order through LDS.
// Row loads through a buffer resource: the hardware returns 0 for every
// byte offset at or past the resource's size without touching memory, so a
// row that does not exist (size 0) or a column at or past d reads zero with
// no branch and no select, and the loads of several rows are all in flight
// before the first wait.  Word 3 is the gfx9 raw-buffer format (32-bit data).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}

// This lane's J x 4 columns 256 j + 64 e + lane of one FP32 row of d values
// (all zero when the row is not valid).
template <int J>
__device__ __forceinline__ void load_cols(float (&x)[J][4], const float* row, int d, bool valid) {
    const int lane = threadIdx.x & 63;
    const __amdgpu_buffer_rsrc_t rs = row_rsrc(row, valid ? 4 * d : 0);
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            x[j][e] = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(rs, 4 * (256 * j + 64 * e + lane), 0, 0));
}

// (red: at least 3 rows of 256 J doubles)
template <int J>
__device__ __forceinline__ void colsum4_chunk(const SumChunk& ch, const PairDesc& pd, int d,
                                              double* __restrict__ partial_row,
                                              double (*red)[256 * J], int32_t* bad_out) {
    const float* base = (const float*)(ch.side ? pd.Y : pd.X);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    double acc[J][4];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[j][e] = 0.0;
    bool bad = false;
    // rows r, r + 4, r + 8, r + 12 per step, all loads issued first (rows past
    // the chunk read zero, see load_cols); the additions keep the row order
    for (int r = ch.r0 + wave; r < ch.r1; r += 16) {
        float4 x[4][J];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rr = r + 4 * q;
            const __amdgpu_buffer_rsrc_t rs =
                row_rsrc(base + (int64_t)(rr < ch.r1 ? rr : r) * d, rr < ch.r1 ? 4 * d : 0);
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * (lane + 64 * j), 0, 0);
                x[q][j] = make_float4(__uint_as_float(u.x), __uint_as_float(u.y),
                                      __uint_as_float(u.z), __uint_as_float(u.w));
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (r + 4 * q >= ch.r1) continue;  // wave-uniform: nothing added past the chunk
            float ss = 0.0f;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                acc[j][0] += (double)x[q][j].x;
                acc[j][1] += (double)x[q][j].y;
                acc[j][2] += (double)x[q][j].z;
                acc[j][3] += (double)x[q][j].w;
                ss += x[q][j].x * x[q][j].x + x[q][j].y * x[q][j].y + x[q][j].z * x[q][j].z +
                      x[q][j].w * x[q][j].w;
            }
            bad |= not_unit((double)wave_total_f32(ss));
        }
    }
    if (wave > 0)
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) red[wave - 1][4 * (lane + 64 * j) + e] = acc[j][e];
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) *bad_out = bad ? 1 : 0;
    if (wave == 0)
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = 4 * (lane + 64 * j) + e;
                if (c < d) partial_row[c] = (acc[j][e] + red[0][c]) + (red[1][c] + red[2][c]);
            }
}

template <int J>
__global__ __launch_bounds__(256) void k_colsum4(const PairDesc* __restrict__ pairs,
                                                 int npairs, int d,
                                                 double* __restrict__ partial,
                                                 int32_t* __restrict__ chunk_bad) {
    __shared__ double red[3][256 * J];
    const SumChunk ch = chunk_of(pairs, npairs, blockIdx.x);
    colsum4_chunk<J>(ch, pairs[ch.pair], d, partial + (int64_t)blockIdx.x * d, red, chunk_bad + blockIdx.x);
}

bool vector_rows_ok(int input_dtype, int d, int d_pad) {
    return input_dtype == HBT_IN_F32 && d % 4 == 0 && d_pad <= 1024;
}

hipError_t launch_colsum_vec(const PairDesc* pairs, int npairs, int nchunks, int d,
                             int d_pad, double* partial, int32_t* chunk_bad, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    const int J = (d_pad + 255) / 256;
    const dim3 g(nchunks), b(256);
    switch (J) {
        case 1: hipLaunchKernelGGL(k_colsum4<1>, g, b, 0, s, pairs, npairs, d, partial, chunk_bad); break;
        case 2: hipLaunchKernelGGL(k_colsum4<2>, g, b, 0, s, pairs, npairs, d, partial, chunk_bad); break;
        case 3: hipLaunchKernelGGL(k_colsum4<3>, g, b, 0, s, pairs, npairs, d, partial, chunk_bad); break;
        case 4: hipLaunchKernelGGL(k_colsum4<4>, g, b, 0, s, pairs, npairs, d, partial, chunk_bad); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Householder coefficients 2 (v . x_i) / (v . v) of every X row, for pairs
// whose rows are stored unreflected (eq:householder_fast folded into the
// statistic): one wave per row, FP64 dot product of the FP32 row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fold_coef(const PairDesc* __restrict__ pairs, int npairs,
                                                   const PairState* __restrict__ st,
                                                   const double* __restrict__ v, int d, int d_pad,
                                                   int64_t total, double* __restrict__ coef) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + wave;
    if (r >= total) return;
    const int p = upper_index(npairs, r, [&](int k) { return pairs[k].coef0; });
    const PairDesc pd = pairs[p];
    const int identity = st[p].identity;
    double w = 0.0;
    if (!identity) {  // wave-uniform
        const float* x = (const float*)pd.X + (r - pd.coef0) * d;
        const double* vp = v + (int64_t)p * d_pad;
        for (int c = lane; c < d; c += 64) w += vp[c] * (double)x[c];
        for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
    }
    if (lane == 0) coef[r] = identity ? 0.0 : 2.0 * w / st[p].vv;
}

hipError_t launch_fold_coef(const PairDesc* pairs, int npairs, const PairState* st, const double* v, int d,
                            int d_pad, int64_t total, double* coef, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold_coef, dim3((unsigned)((total + 3) / 4)), dim3(256), 0, s, pairs, npairs, st, v,
                       d, d_pad, total, coef);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// finalize: one work-group per pair
// ---------------------------------------------------------------------------
// Deterministic block sum of per-thread values (256 threads).
__device__ double block_sum(double x, double* red) {
    const int t = threadIdx.x;
    red[t] = x;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_finalize(const PairDesc* __restrict__ pairs,
                                                  const double* __restrict__ partial,
                                                  const int32_t* __restrict__ chunk_bad, int d,
                                                  int d_pad, int align, int gd, double* sxy,
                                                  PairState* st, double* v, double* t64,
                                                  float* t32, PairCount* cnt, hbt_result* res,
                                                  int p0, float* __restrict__ v32) {
    __shared__ double red[256];
    const int p = blockIdx.x + p0;
    const PairDesc pd = pairs[p];
    double* sx = sxy + (int64_t)p * 2 * d_pad;
    double* sy = sx + d_pad;
    double* vp = v + (int64_t)p * d_pad;
    double* tp = t64 + (int64_t)p * d_pad;
    float* tq = t32 + (int64_t)p * d_pad;
    // Step 1: sums of X and Y, chunk partials added in chunk order (eight
    // loads in flight at a time; the additions keep that order)
    auto chunk_sum = [&](int k0, int k1, int c) {
        double acc = 0.0;
        int k = k0;
        for (; k + 8 <= k1; k += 8) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = partial[(int64_t)(k + u) * d + c];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += t[u];
        }
        for (; k < k1; ++k) acc += partial[(int64_t)k * d + c];
        return acc;
    };
    int bad = 0;
    for (int k = pd.cx0 + threadIdx.x; k < pd.cx1; k += 256) bad |= chunk_bad[k];
    for (int k = pd.cy0 + threadIdx.x; k < pd.cy1; k += 256) bad |= chunk_bad[k];
    bad = __syncthreads_or(bad);
    double ssx = 0.0, ssy = 0.0;
    for (int c = threadIdx.x; c < d_pad; c += 256) {
        double a = 0.0, b = 0.0;
        if (c < d) {
            a = chunk_sum(pd.cx0, pd.cx1, c);
            b = chunk_sum(pd.cy0, pd.cy1, c);
        }
        sx[c] = a;
        sy[c] = b;
        ssx += a * a;
        ssy += b * b;
    }
    ssx = block_sum(ssx, red);
    ssy = block_sum(ssy, red);
    const double nx = sqrt(ssx), ny = sqrt(ssy);
    const double r_x = nx / (double)pd.n, r_y = ny / (double)pd.m;
    // mean directions and v = mu_x - mu_y (Eq. for u, before normalisation)
    double vv = 0.0;
    for (int c = threadIdx.x; c < d_pad; c += 256) {
        const double mx = nx > 0.0 ? sx[c] / nx : 0.0;
        const double my = ny > 0.0 ? sy[c] / ny : 0.0;
        const double vc = mx - my;
        vp[c] = vc;
        vv += vc * vc;
    }
    vv = block_sum(vv, red);
    const int identity = (!align) || !(sqrt(vv) > 1e-12) || !(r_x > 0.0) || !(r_y > 0.0);
    // t = H s_x + s_y: the pooled total of Z = [X'; Y]
    double w = 0.0;
    for (int c = threadIdx.x; c < d_pad; c += 256) w += vp[c] * sx[c];
    w = block_sum(w, red);
    const double coef = identity ? 0.0 : 2.0 * w / vv;
    double vt = 0.0;
    for (int c = threadIdx.x; c < d_pad; c += 256) {
        const double tc = (sx[c] - coef * vp[c]) + sy[c];
        tp[c] = tc;
        tq[c] = (float)tc;
        vt += vp[c] * tc;
        if (v32) v32[(int64_t)p * d_pad + c] = (float)vp[c];
    }
    vt = block_sum(vt, red);
    if (threadIdx.x == 0) {
        const double dd = (double)d;
        const double fx = log_g(r_x, dd, gd), fy = log_g(r_y, dd, gd);
        const double scale = fabs(fx) + fabs(fy);
        PairState q;
        q.r_x = r_x;
        q.r_y = r_y;
        q.t_obs = fy - fx;  // log v(X') - log v(Y), v = 1/g_d(r)
        q.tau = 1e-10 * (scale > 1.0 ? scale : 1.0);
        q.vv = vv;
        q.f_x = fx;
        q.f_y = fy;
        q.vt = vt;
        q.identity = identity;
        q.status = (r_x > 0.0 && r_x < 1.0 && r_y > 0.0 && r_y < 1.0)
                       ? (bad ? HBT_ERR_NOT_UNIT : HBT_OK)
                       : HBT_ERR_DEGENERATE;
        q._pad2[0] = q._pad2[1] = 0;
        st[p] = q;
        cnt[p].count = 0;
        cnt[p].n_recheck = 0;
        cnt[p].sum_dt = 0.0;
        cnt[p].sum_dt2 = 0.0;
        hbt_result r;
        r.t_obs = q.t_obs;
        r.r_x = r_x;
        r.r_y = r_y;
        r.p = 0.0;
        r.tau = q.tau;
        r.mu_cos = 1.0 - 0.5 * vv;  // |mu_x - mu_y|^2 = 2 - 2 cos
        r.t_mean = 0.0;
        r.t_sd = 0.0;
        r.count = 0;
        r.B = 0;
        r.n_recheck = 0;
        r.n = pd.n;
        r.m = pd.m;
        r.status = q.status;
        r.h_identity = identity;
        res[p] = r;
    }
}

hipError_t launch_finalize(const PairDesc* pairs, int npairs, const double* partial,
                           const int32_t* chunk_bad, int d,
                           int d_pad, int align, int gd, double* sxy, PairState* st, double* v,
                           double* t64, float* t32, PairCount* cnt, hbt_result* res,
                           hipStream_t s, int p0, float* v32) {
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(npairs), dim3(256), 0, s, pairs, partial, chunk_bad, d, d_pad, align,
                       gd, sxy, st, v, t64, t32, cnt, res, p0, v32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reflection + storage: one work-group per octet of 8 pooled rows
// Two values' e4m3 lo bytes: lo = z - hi (hi the stored, scaled bf16 of each,
// times inv to undo the plane scale; exact in FP32), rounded to nearest even
// as e4m3 of lo 2^kE4m3LoShift, at group rows ra, rb of the 32-row group whose
// first lo unit (of this column) plo points at.
__device__ __forceinline__ void store_e4m3_lo2(unsigned char* plo, int d_pad, int ra, int rb, float za,
                                               float zb, uint32_t hi2, float inva, float invb) {
    const float ha = __uint_as_float(hi2 << 16) * inva;
    const float hb = __uint_as_float(hi2 & 0xffff0000u) * invb;
    constexpr float up = (float)(1 << kE4m3LoShift);
    const uint32_t q = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32((za - ha) * up, (zb - hb) * up, 0, false);
    plo[(int64_t)f8_unit(ra) * d_pad * 16 + f8_byte(ra)] = (unsigned char)(q & 0xffu);
    plo[(int64_t)f8_unit(rb) * d_pad * 16 + f8_byte(rb)] = (unsigned char)((q >> 8) & 0xffu);
}

// ---------------------------------------------------------------------------
// Z storage formats:
//   HBT_F64    : double [Np][d_pad]
//   HBT_F32    : float  [Np][d_pad]
//   HBT_BF16X2 : two planes (hi, then lo at +zplane_elems) of bf16
//                [Np/8][d_pad][8]: the 8 values of a storage octet are
//                contiguous per column, the operand layout of the bf16 MFMA;
//                storage octet 4 g + o4 holds rows 32 g + bf16_plane_row(o4, k)
//                of the pair, scaled by bf16_plane_scale(o4, k) (k = 0..7).
//   HBT_BF16_E4M3: the HBT_BF16X2 hi plane, then at byte 2 zplane_elems the
//                e4m3 lo plane [Np/16][d_pad][16] (f8_unit, f8_byte).
//   HBT_I8X3   : three planes (q0, q1, q2 at +zplane_elems bytes each) of
//                int8 digits [Np/16][d_pad][16]; storage octet 4 g + o4
//                fills bytes 8 (o4 & 1) .. +7 of unit 2 g + o4 / 2 with rows
//                32 g + i8_plane_row(o4, k).
// A work-group (or wave) handles the 8 rows of one storage octet for every
// format; the row-major formats simply write each row in its place.
template <typename Tin, int PREC>
__global__ __launch_bounds__(256) void k_reflect(const PairDesc* __restrict__ pairs, int npairs,
                                                 const PairState* __restrict__ st,
                                                 const double* __restrict__ v, int d, int d_pad,
                                                 double* __restrict__ coef, void* zstore,
                                                 int64_t zplane_elems, float* __restrict__ z32) {
    __shared__ double cf[8];
    const int64_t oct = blockIdx.x;
    const int p = upper_index(npairs, oct * 8, [&](int k) { return pairs[k].zrow0; });
    const PairDesc pd = pairs[p];
    const int identity = st[p].identity;
    const double vv = st[p].vv;
    const double* vp = v + (int64_t)p * d_pad;
    const int lo8 = (int)(oct - pd.zrow0 / 8);  // storage octet within the pair
    const int g0 = 32 * (lo8 >> 2), o4 = lo8 & 3;
    const int N = pd.n + pd.m;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // coefficients 2 (v . x_i) / (v . v) of the X rows (eq:householder_fast)
    for (int r = wave; r < 8; r += 4) {
        const int i = g0 + (PREC == HBT_I8X3 ? i8_plane_row(o4, r) : bf16_plane_row(o4, r));
        double w = 0.0;
        if (!identity && i < pd.n) {
            const Tin* x = (const Tin*)pd.X + (int64_t)i * d;
            for (int c = lane; c < d; c += 64) w += vp[c] * (double)x[c];
            for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
        }
        if (lane == 0) {
            const double k = (!identity && i < pd.n) ? 2.0 * w / vv : 0.0;
            cf[r] = k;
            if (i < pd.n) coef[pd.coef0 + i] = k;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < d_pad; c += 256) {
        double z[8];
        const double vc = c < d ? vp[c] : 0.0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = g0 + (PREC == HBT_I8X3 ? i8_plane_row(o4, r) : bf16_plane_row(o4, r));
            double val = 0.0;
            if (c < d) {
                if (i < pd.n)
                    val = (double)((const Tin*)pd.X)[(int64_t)i * d + c] - cf[r] * vc;
                else if (i < N)
                    val = (double)((const Tin*)pd.Y)[(int64_t)(i - pd.n) * d + c];
            }
            z[r] = val;
        }
        if (z32) {  // row-major FP32 copy for the point-to-centroid route
#pragma unroll
            for (int r = 0; r < 8; ++r)
                z32[(pd.zrow0 + g0 + bf16_plane_row(o4, r)) * (int64_t)d_pad + c] = (float)z[r];
        }
        if (PREC == HBT_I8X3) {
            uint32_t w[3][2] = {{0u, 0u}, {0u, 0u}, {0u, 0u}};
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                uint32_t q[3];
                i8_digits(z[r], q[0], q[1], q[2]);
#pragma unroll
                for (int k = 0; k < 3; ++k) w[k][r >> 2] |= q[k] << (8 * (r & 3));
            }
            uint2* dst = (uint2*)((char*)zstore + ((oct >> 1) * d_pad + c) * 16 + 8 * (oct & 1));
#pragma unroll
            for (int k = 0; k < 3; ++k)
                *(uint2*)((char*)dst + k * zplane_elems) = make_uint2(w[k][0], w[k][1]);
        } else if (PREC == HBT_BF16X2) {
            uint32_t hi[4], lo[4];
#pragma unroll
            for (int r = 0; r < 8; r += 2) {
                const float a = (float)z[r] * bf16_plane_scale(o4, r);
                const float b = (float)z[r + 1] * bf16_plane_scale(o4, r + 1);
                const uint2 hl = split_bf16x2(a, b);
                hi[r / 2] = hl.x;
                lo[r / 2] = hl.y;
            }
            uint4* ph = (uint4*)zstore + oct * d_pad + c;
            *ph = make_uint4(hi[0], hi[1], hi[2], hi[3]);
            *(ph + zplane_elems / 8) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
        } else if (PREC == HBT_BF16_E4M3) {
            uint32_t hi[4];
            unsigned char* plo = (unsigned char*)zstore + 2 * zplane_elems + (((oct >> 2) * 2) * d_pad + c) * 16;
#pragma unroll
            for (int r = 0; r < 8; r += 2) {
                const float a = (float)z[r], b = (float)z[r + 1];
                hi[r / 2] = split_bf16x2(a * bf16_plane_scale(o4, r), b * bf16_plane_scale(o4, r + 1)).x;
                store_e4m3_lo2(plo, d_pad, bf16_plane_row(o4, r), bf16_plane_row(o4, r + 1), a, b, hi[r / 2],
                               bf16_plane_inv_scale(o4, r), bf16_plane_inv_scale(o4, r + 1));
            }
            *((uint4*)zstore + oct * d_pad + c) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        } else if (PREC == HBT_F32) {
#pragma unroll
            for (int r = 0; r < 8; ++r)
                ((float*)zstore)[(pd.zrow0 + g0 + bf16_plane_row(o4, r)) * (int64_t)d_pad + c] = (float)z[r];
        } else {
#pragma unroll
            for (int r = 0; r < 8; ++r)
                ((double*)zstore)[(pd.zrow0 + g0 + bf16_plane_row(o4, r)) * (int64_t)d_pad + c] = z[r];
        }
    }
}

template <typename Tin>
static hipError_t launch_reflect_t(int precision, const PairDesc* pairs, int npairs,
                                   int64_t total_octets, const PairState* st, const double* v,
                                   int d, int d_pad, double* coef, void* z, int64_t ze, float* z32,
                                   hipStream_t s) {
    dim3 g((unsigned)total_octets), b(256);
    switch (precision) {
        case HBT_F64:
            hipLaunchKernelGGL((k_reflect<Tin, HBT_F64>), g, b, 0, s, pairs, npairs, st, v, d, d_pad,
                               coef, z, ze, z32);
            break;
        case HBT_F32:
            hipLaunchKernelGGL((k_reflect<Tin, HBT_F32>), g, b, 0, s, pairs, npairs, st, v, d, d_pad,
                               coef, z, ze, z32);
            break;
        case HBT_I8X3:
            hipLaunchKernelGGL((k_reflect<Tin, HBT_I8X3>), g, b, 0, s, pairs, npairs, st, v, d,
                               d_pad, coef, z, ze, z32);
            break;
        case HBT_BF16_E4M3:
            hipLaunchKernelGGL((k_reflect<Tin, HBT_BF16_E4M3>), g, b, 0, s, pairs, npairs, st, v, d,
                               d_pad, coef, z, ze, z32);
            break;
        default:
            hipLaunchKernelGGL((k_reflect<Tin, HBT_BF16X2>), g, b, 0, s, pairs, npairs, st, v, d,
                               d_pad, coef, z, ze, z32);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_reflect(int input_dtype, int precision, const PairDesc* pairs, int npairs,
                          int64_t total_octets, const PairState* st, const double* v, int d,
                          int d_pad, double* coef, void* zstore, int64_t zplane_elems,
                          float* z32, hipStream_t s) {
    if (total_octets <= 0) return hipSuccess;
    if (input_dtype == HBT_IN_F64)
        return launch_reflect_t<double>(precision, pairs, npairs, total_octets, st, v, d, d_pad,
                                        coef, zstore, zplane_elems, z32, s);
    return launch_reflect_t<float>(precision, pairs, npairs, total_octets, st, v, d, d_pad, coef,
                                   zstore, zplane_elems, z32, s);
}

// The same reflection and storage for FP32 rows with d a multiple of 4 and
// 16-byte aligned rows (the condition shared with the vector column sums):
// one wave per octet, the octet's 8 rows held in registers (lane l: columns
// 256 j + 64 e + l, j < J, e < 4, each load instruction reading 256
// contiguous bytes of a row); the coefficients are FP64 wave reductions, and
// every store instruction then writes one contiguous run of columns (1 KB per
// plane for split BF16).
__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Stores one storage octet of a pair: this lane's J x 4 columns of the 8
// rows row_of(0..7) (pair-relative pooled rows), z_r = x_r - k_r vc in FP64,
// in the precision's format.  soct is the octet's index in the whole storage.
template <int PREC, int J, typename RowOf>
__device__ __forceinline__ void store_octet(const float (&x)[8][J][4], const double (&k)[8],
                                            const double (&vc)[J][4], int64_t soct, int64_t zrow0,
                                            RowOf row_of, int o4, int d_pad, void* zstore,
                                            int64_t zplane_elems, float* __restrict__ z32) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = 256 * j + 64 * e + lane;
            if (256 * j + 64 * e >= d_pad) continue;  // wave-uniform: d_pad is a multiple of 64
            if (PREC == HBT_F64) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int64_t zr = zrow0 + row_of(r);
                    const double z = (double)x[r][j][e] - k[r] * vc[j][e];
                    ((double*)zstore)[zr * d_pad + c] = z;
                    if (z32) z32[zr * d_pad + c] = (float)z;
                }
                continue;
            }
            if (PREC == HBT_I8X3) {  // digits of the FP64 update
                uint32_t w[3][2] = {{0u, 0u}, {0u, 0u}, {0u, 0u}};
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    uint32_t q[3];
                    i8_digits((double)x[r][j][e] - k[r] * vc[j][e], q[0], q[1], q[2]);
#pragma unroll
                    for (int t = 0; t < 3; ++t) w[t][r >> 2] |= q[t] << (8 * (r & 3));
                }
                char* dst = (char*)zstore + ((soct >> 1) * d_pad + c) * 16 + 8 * (soct & 1);
#pragma unroll
                for (int t = 0; t < 3; ++t) *(uint2*)(dst + t * zplane_elems) = make_uint2(w[t][0], w[t][1]);
                continue;
            }
            // FP64 update, rounded to FP32 at once (the storage is FP32 or BF16 hi+lo)
            float zf[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) zf[r] = (float)((double)x[r][j][e] - k[r] * vc[j][e]);
            if (PREC == HBT_F32 || z32) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int64_t zr = zrow0 + row_of(r);
                    if (PREC == HBT_F32) ((float*)zstore)[zr * d_pad + c] = zf[r];
                    if (z32) z32[zr * d_pad + c] = zf[r];
                }
            }
            if (PREC == HBT_BF16X2) {
                uint32_t hi[4], lo[4];
#pragma unroll
                for (int r = 0; r < 8; r += 2) {
                    const uint2 hl = split_bf16x2(zf[r] * bf16_plane_scale(o4, r), zf[r + 1] * bf16_plane_scale(o4, r + 1));
                    hi[r / 2] = hl.x;
                    lo[r / 2] = hl.y;
                }
                uint4* ph = (uint4*)zstore + soct * d_pad + c;
                *ph = make_uint4(hi[0], hi[1], hi[2], hi[3]);
                *(ph + zplane_elems / 8) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
            }
            if (PREC == HBT_BF16_E4M3) {
                uint32_t hi[4];
                unsigned char* plo = (unsigned char*)zstore + 2 * zplane_elems + (((soct >> 2) * 2) * d_pad + c) * 16;
#pragma unroll
                for (int r = 0; r < 8; r += 2) {
                    hi[r / 2] = split_bf16x2(zf[r] * bf16_plane_scale(o4, r), zf[r + 1] * bf16_plane_scale(o4, r + 1)).x;
                    store_e4m3_lo2(plo, d_pad, row_of(r) & 31, row_of(r + 1) & 31, zf[r], zf[r + 1], hi[r / 2],
                                   bf16_plane_inv_scale(o4, r), bf16_plane_inv_scale(o4, r + 1));
                }
                *((uint4*)zstore + soct * d_pad + c) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
            }
        }
}

template <int PREC>
__device__ __forceinline__ int plane_row(int o4, int k) {
    return PREC == HBT_I8X3 ? i8_plane_row(o4, k) : bf16_plane_row(o4, k);
}

// The reflection on the 16-byte path: one wave per storage octet of the
// 32-row groups that hold X rows (x_octets(n) per pair, numbered from
// PairDesc::xoct0); the groups that hold only Y rows or padding are stored by
// k_colsum_store4.
template <int PREC, int J>
__global__ __launch_bounds__(256) void k_reflect4(const PairDesc* __restrict__ pairs, int npairs,
                                                  int64_t total_octets,
                                                  const PairState* __restrict__ st,
                                                  const double* __restrict__ v, int d, int d_pad,
                                                  double* __restrict__ coef, void* zstore,
                                                  int64_t zplane_elems, float* __restrict__ z32,
                                                  int64_t oct0) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t oct = (int64_t)blockIdx.x * 4 + wave + oct0;
    if (oct >= total_octets) return;
    const int p = upper_index(npairs, oct, [&](int k) { return pairs[k].xoct0; });
    const PairDesc pd = pairs[p];
    const int identity = st[p].identity;
    const double vv = st[p].vv;
    const double* vp = v + (int64_t)p * d_pad;
    const int lo8 = (int)(oct - pd.xoct0);  // storage octet within the pair
    const int g0 = 32 * (lo8 >> 2), o4 = lo8 & 3;
    const int N = pd.n + pd.m;
    auto row_of = [&](int r) { return g0 + plane_row<PREC>(o4, r); };
    auto col = [&](int j, int e) { return 256 * j + 64 * e + lane; };
    float x[8][J][4];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = row_of(r);  // wave-uniform; a padding row reads Y's last row and keeps zeros
        const float* row = i < pd.n ? (const float*)pd.X + (int64_t)i * d
                                    : (const float*)pd.Y + (int64_t)((i < N ? i : N - 1) - pd.n) * d;
        load_cols<J>(x[r], row, d, i < N);
    }
    double vc[J][4];
    const __amdgpu_buffer_rsrc_t vrs = row_rsrc(vp, 8 * d);  // columns past d read 0
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            vc[j][e] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(vrs, 8 * col(j, e), 0, 0));
    // coefficients 2 (v . x_i) / (v . v) of the X rows (eq:householder_fast)
    double k[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = row_of(r);
        k[r] = 0.0;
        if (!identity && i < pd.n) {  // wave-uniform
            double w = 0.0;
#pragma unroll
            for (int j = 0; j < J; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) w += vc[j][e] * (double)x[r][j][e];
            k[r] = 2.0 * wave_sum_f64(w) / vv;
        }
    }
    // the update below converts the rows to FP64 again instead of keeping the
    // dot product's FP64 copies alive (twice the registers)
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int j = 0; j < J; ++j)
            asm volatile("" : "+v"(x[r][j][0]), "+v"(x[r][j][1]), "+v"(x[r][j][2]), "+v"(x[r][j][3]));
    if (lane < 8) {
        double kr = k[0];
#pragma unroll
        for (int r = 1; r < 8; ++r) kr = lane == r ? k[r] : kr;
        const int i = row_of(lane);
        if (i < pd.n) coef[pd.coef0 + i] = kr;
    }
    store_octet<PREC, J>(x, k, vc, pd.zrow0 / 8 + lo8, pd.zrow0, row_of, o4, d_pad, zstore,
                         zplane_elems, z32);
}

hipError_t launch_reflect_vec(int precision, const PairDesc* pairs, int npairs,
                              int64_t total_octets, const PairState* st, const double* v, int d,
                              int d_pad, double* coef, void* zstore, int64_t zplane_elems,
                              float* z32, hipStream_t s, int64_t oct0) {
    if (total_octets <= oct0) return hipSuccess;
    const int J = (d_pad + 255) / 256;
    const dim3 g((unsigned)((total_octets - oct0 + 3) / 4)), b(256);
#define HBT_R4(PR, JJ)                                                                         \
    hipLaunchKernelGGL((k_reflect4<PR, JJ>), g, b, 0, s, pairs, npairs, total_octets, st, v, d, \
                       d_pad, coef, zstore, zplane_elems, z32, oct0)
#define HBT_R4J(PR)                            \
    switch (J) {                               \
        case 1: HBT_R4(PR, 1); break;          \
        case 2: HBT_R4(PR, 2); break;          \
        case 3: HBT_R4(PR, 3); break;          \
        case 4: HBT_R4(PR, 4); break;          \
        default: return hipErrorInvalidValue;  \
    }
    switch (precision) {
        case HBT_F64: HBT_R4J(HBT_F64); break;
        case HBT_F32: HBT_R4J(HBT_F32); break;
        case HBT_I8X3: HBT_R4J(HBT_I8X3); break;
        case HBT_BF16_E4M3: HBT_R4J(HBT_BF16_E4M3); break;
        default: HBT_R4J(HBT_BF16X2); break;
    }
#undef HBT_R4J
#undef HBT_R4
    return hipGetLastError();
}

// Column sums and, in the same pass, the Z storage of the Y rows (16-byte
// path, group-sum calls).  X chunks are summed as in k_colsum4.  A Y chunk is
// one 32-row group of the storage: wave w loads octet w (the 8 rows
// plane_row(w, .) of the group), adds its Y rows to the sums and stores the
// octet as it is (H leaves Y unchanged; rows past n + m are the zero
// padding), except in the group that also holds X rows, which the reflection
// stores.  Y's rows are then read once for both purposes.
template <int PREC, int J>
__global__ __launch_bounds__(256) void k_colsum_store4(const PairDesc* __restrict__ pairs,
                                                       int npairs, int d, int d_pad,
                                                       double* __restrict__ partial, void* zstore,
                                                       int64_t zplane_elems,
                                                       float* __restrict__ z32,
                                                       int32_t* __restrict__ chunk_bad, int c0) {
    __shared__ double red[4][256 * J];
    const int c = blockIdx.x + c0;
    const SumChunk ch = chunk_of(pairs, npairs, c);
    const PairDesc pd = pairs[ch.pair];
    double* prow = partial + (int64_t)c * d;
    if (!ch.side) {  // work-group-uniform
        colsum4_chunk<J>(ch, pd, d, prow, red, chunk_bad + c);
        return;
    }
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int n = pd.n, N = n + pd.m;
    const int g0 = (n + ch.r0) & ~31;  // the chunk's group
    auto row_of = [&](int r) { return g0 + plane_row<PREC>(wave, r); };
    auto col = [&](int j, int e) { return 256 * j + 64 * e + lane; };
    float x[8][J][4];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = row_of(r);
        const bool y = i >= n && i < N;  // wave-uniform; other rows read Y's first row and keep zeros
        load_cols<J>(x[r], (const float*)pd.Y + (int64_t)(y ? i - n : 0) * d, d, y);
    }
    // each wave's sums go to LDS at once, so they are not live across the stores
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            double t = 0.0;
#pragma unroll
            for (int r = 0; r < 8; ++r) t += (double)x[r][j][e];
            red[wave][col(j, e)] = t;
        }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = row_of(r);
        if (i < n || i >= N) continue;  // wave-uniform: only this group's Y rows
        float ss = 0.0f;
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) ss += x[r][j][e] * x[r][j][e];
        bad |= not_unit((double)wave_total_f32(ss));
    }
    // the stores convert the rows to FP64 again instead of keeping the sums'
    // FP64 copies alive (twice the registers)
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int j = 0; j < J; ++j)
            asm volatile("" : "+v"(x[r][j][0]), "+v"(x[r][j][1]), "+v"(x[r][j][2]), "+v"(x[r][j][3]));
    if (g0 >= n) {  // wave-uniform
        double k0[8], v0[J][4];
#pragma unroll
        for (int r = 0; r < 8; ++r) k0[r] = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) v0[j][e] = 0.0;
        store_octet<PREC, J>(x, k0, v0, pd.zrow0 / 8 + g0 / 8 + wave, pd.zrow0, row_of, wave, d_pad,
                             zstore, zplane_elems, z32);
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) chunk_bad[c] = bad ? 1 : 0;
    for (int cc = threadIdx.x; cc < d; cc += 256)
        prow[cc] = (red[0][cc] + red[1][cc]) + (red[2][cc] + red[3][cc]);
}

hipError_t launch_colsum_store_vec(int precision, const PairDesc* pairs, int npairs, int nchunks,
                                   int d, int d_pad, double* partial, void* zstore,
                                   int64_t zplane_elems, float* z32, int32_t* chunk_bad,
                                   hipStream_t s, int c0) {
    if (nchunks <= 0) return hipSuccess;
    const int J = (d_pad + 255) / 256;
    const dim3 g(nchunks), b(256);
#define HBT_C4(PR, JJ)                                                                         \
    hipLaunchKernelGGL((k_colsum_store4<PR, JJ>), g, b, 0, s, pairs, npairs, d, d_pad, partial, \
                       zstore, zplane_elems, z32, chunk_bad, c0)
#define HBT_C4J(PR)                            \
    switch (J) {                               \
        case 1: HBT_C4(PR, 1); break;          \
        case 2: HBT_C4(PR, 2); break;          \
        case 3: HBT_C4(PR, 3); break;          \
        case 4: HBT_C4(PR, 4); break;          \
        default: return hipErrorInvalidValue;  \
    }
    switch (precision) {
        case HBT_F64: HBT_C4J(HBT_F64); break;
        case HBT_F32: HBT_C4J(HBT_F32); break;
        case HBT_I8X3: HBT_C4J(HBT_I8X3); break;
        case HBT_BF16_E4M3: HBT_C4J(HBT_BF16_E4M3); break;
        default: HBT_C4J(HBT_BF16X2); break;
    }
#undef HBT_C4J
#undef HBT_C4
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// hbt_align's output: X' = H X in the input dtype, one wave per row
// ---------------------------------------------------------------------------
template <typename Tin>
__global__ __launch_bounds__(256) void k_reflect_out(const PairDesc* __restrict__ pair,
                                                     const PairState* __restrict__ st,
                                                     const double* __restrict__ v, int n, int d,
                                                     Tin* X_out) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + wave;
    if (i >= n) return;
    const Tin* x = (const Tin*)pair->X + (int64_t)i * d;
    Tin* y = X_out + (int64_t)i * d;
    const int identity = st->identity;
    double w = 0.0;
    if (!identity) {
        for (int c = lane; c < d; c += 64) w += v[c] * (double)x[c];
        for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
    }
    const double k = identity ? 0.0 : 2.0 * w / st->vv;
    // every lane has read its share of the row (inside the dot product) before
    // any write, so X_out may alias X
    for (int c = lane; c < d; c += 64) y[c] = (Tin)((double)x[c] - k * v[c]);
}

__global__ void k_copy_v(const double* v, int d, double* out) {
    for (int c = threadIdx.x; c < d; c += blockDim.x) out[c] = v[c];
}

hipError_t launch_reflect_out(int input_dtype, const PairDesc* pair, const PairState* st,
                              const double* v, int n, int d, void* X_out, double* v_out,
                              hipStream_t s) {
    dim3 g((n + 3) / 4), b(256);
    if (input_dtype == HBT_IN_F64)
        hipLaunchKernelGGL(k_reflect_out<double>, g, b, 0, s, pair, st, v, n, d, (double*)X_out);
    else
        hipLaunchKernelGGL(k_reflect_out<float>, g, b, 0, s, pair, st, v, n, d, (float*)X_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !v_out) return e;
    hipLaunchKernelGGL(k_copy_v, dim3(1), dim3(256), 0, s, v, d, v_out);
    return hipGetLastError();
}

}  // namespace hbt
