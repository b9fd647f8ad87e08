// Learned permutation-budget allocator: features of a pair from its
// alignment results, a 12 -> 64 -> 64 -> 2 ReLU network (forward, gradient,
// Adam), and the number of permutations implied by the network's estimate
// of the pair's permutation null distribution.
//
// The network predicts (mean, log sd) of the permuted statistics T_b of a
// pair (Sec. 3.1, Algorithm 1 Step 5) from quantities of Algorithm 1 Steps
// 1-4.  The exact permutation p-value (eq:pvalue) remains the decision: the
// prediction only sets how many splits a pair gets.
//
// Parameter vector theta (float), row-major blocks in this order:
//   shift[12], scale[12]      input standardisation x~ = (x - shift) * scale
//   oshift[2], oscale[2]      output standardisation out = oshift + oscale * y~
//   W1[64][12], b1[64]        hidden layer 1 (ReLU)
//   W2[64][64], b2[64]        hidden layer 2 (ReLU)
//   W3[2][64],  b3[2]         y~ (standardised (mean, log sd))
#include "hbt_launch.h"

namespace hbt {

constexpr int kF = HBT_MLP_FEATURES, kH = 64, kO = 2;
constexpr int oShift = 0, oScale = kF, oOShift = 2 * kF, oOScale = oOShift + kO, oW1 = oOScale + kO,
              oB1 = oW1 + kH * kF, oW2 = oB1 + kH,
              oB2 = oW2 + kH * kH, oW3 = oB2 + kH, oB3 = oW3 + kO * kH, kP = oB3 + kO;
static_assert(kP == HBT_MLP_PARAMS, "parameter layout");
static_assert(oW1 == HBT_MLP_TRAINABLE_OFFSET, "trainable offset");

// ---------------------------------------------------------------------------
// features (FP64 arithmetic, stored as float)
// ---------------------------------------------------------------------------
__global__ void k_features(int64_t npairs, const hbt_result* __restrict__ res, double d, int gd,
                           float* __restrict__ feat) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const hbt_result r = res[p];
    const double n = (double)r.n, m = (double)r.m, N = n + m;
    const double f[kF] = {log(n),
                          log(m),
                          r.r_x,
                          r.r_y,
                          (n * r.r_x + m * r.r_y) / N,  // pooled MRL after alignment
                          r.mu_cos,
                          log_g(r.r_x, d, gd),
                          log_g(r.r_y, d, gd),
                          r.t_obs,
                          n / N,
                          log1p(-r.r_x * r.r_x),
                          log1p(-r.r_y * r.r_y)};
#pragma unroll
    for (int k = 0; k < kF; ++k) feat[p * kF + k] = (float)f[k];
}

// training targets of a pair: (mean, log sd) of its permuted statistics
__global__ void k_null_targets(int64_t npairs, const hbt_result* __restrict__ res,
                               float* __restrict__ target) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    target[p * kO] = (float)res[p].t_mean;
    target[p * kO + 1] = (float)log(res[p].t_sd);
}

hipError_t launch_null_targets(int64_t npairs, const hbt_result* res, float* target, hipStream_t s) {
    hipLaunchKernelGGL(k_null_targets, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, npairs,
                       res, target);
    return hipGetLastError();
}

// Column statistics of a rows x cols matrix: shift[k] = mean, scale[k] =
// 1 / sd (invert) or sd (population sd); one work-group per column,
// fixed-order FP64 reductions.  A constant column gets scale 1.
__global__ __launch_bounds__(256) void k_col_norm(int64_t rows, int cols, const float* __restrict__ feat,
                                                  float* __restrict__ shift, float* __restrict__ scale,
                                                  int invert) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    auto block_sum = [&](double x) {
        red[threadIdx.x] = x;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        const double s = red[0];
        __syncthreads();
        return s;
    };
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += 256) s += (double)feat[r * cols + k];
    const double mean = block_sum(s) / (double)rows;
    double q = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += 256) {
        const double x = (double)feat[r * cols + k] - mean;
        q += x * x;
    }
    const double sd = sqrt(block_sum(q) / (double)rows);
    if (threadIdx.x == 0) {
        shift[k] = (float)mean;
        scale[k] = sd > 0.0 ? (float)(invert ? 1.0 / sd : sd) : 1.0f;
    }
}

// ---------------------------------------------------------------------------
// network: one thread per row, parameters in LDS (read as broadcasts)
// ---------------------------------------------------------------------------
// Layer 1 of one row: x~ and z1 = relu(W1 x~ + b1), held in registers.
__device__ __forceinline__ void layer1(const float* th, const float* x, float (&xs)[kF], float (&z1)[kH]) {
#pragma unroll
    for (int i = 0; i < kF; ++i) xs[i] = (x[i] - th[oShift + i]) * th[oScale + i];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float s = th[oB1 + j];
#pragma unroll
        for (int i = 0; i < kF; ++i) s = fmaf(th[oW1 + j * kF + i], xs[i], s);
        z1[j] = s > 0.0f ? s : 0.0f;
    }
}

// Unit j of layer 2: relu(W2[j] . z1 + b2[j]).
__device__ __forceinline__ float unit2(const float* th, const float (&z1)[kH], int j) {
    float s = th[oB2 + j];
#pragma unroll
    for (int i = 0; i < kH; ++i) s = fmaf(th[oW2 + j * kH + i], z1[i], s);
    return s > 0.0f ? s : 0.0f;
}

__device__ __forceinline__ void load_theta(float* lds, const float* theta) {
    for (int k = threadIdx.x; k < kP; k += blockDim.x) lds[k] = theta[k];
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_forward(int64_t rows, const float* __restrict__ feat,
                                                     const float* __restrict__ theta,
                                                     float* __restrict__ out) {
    __shared__ float th[kP];
    load_theta(th, theta);
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float xs[kF], z1[kH];
    layer1(th, feat + r * kF, xs, z1);
    float o0 = th[oB3], o1 = th[oB3 + 1];
    for (int j = 0; j < kH; ++j) {  // the output layer accumulates unit by unit
        const float z = unit2(th, z1, j);
        o0 = fmaf(th[oW3 + j], z, o0);
        o1 = fmaf(th[oW3 + kH + j], z, o1);
    }
    out[r * kO + 0] = fmaf(th[oOScale], o0, th[oOShift]);
    out[r * kO + 1] = fmaf(th[oOScale + 1], o1, th[oOShift + 1]);
}

// Per-row pass of the gradient of L = (1/R) sum_r (1/2) |(out_r - target_r) / oscale|^2
// (the squared error of y~ against standardised targets):
// forward, then the error signals at the pre-activations of the three layers
// (dout, d2, d1).  Writes what the per-parameter reduction needs: x~, z1, z2,
// d1, d2, dout, and the row's loss.
struct TrainWs {
    float *xs, *z1, *z2, *d1, *d2, *dout;
    double* loss;
};

__global__ __launch_bounds__(256) void k_mlp_rows(int64_t rows, const float* __restrict__ feat,
                                                  const float* __restrict__ target,
                                                  const float* __restrict__ theta, TrainWs w) {
    __shared__ float th[kP];
    load_theta(th, theta);
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float xs[kF], z1[kH];
    layer1(th, feat + r * kF, xs, z1);
    float* z2 = w.z2 + r * kH;
    float o0 = th[oB3], o1 = th[oB3 + 1];
    for (int j = 0; j < kH; ++j) {
        const float z = unit2(th, z1, j);
        z2[j] = z;
        o0 = fmaf(th[oW3 + j], z, o0);
        o1 = fmaf(th[oW3 + kH + j], z, o1);
    }
    const float inv = 1.0f / (float)rows;
    // error of y~ against the standardised target (t - oshift) / oscale
    const float e0 = o0 - (target[r * kO] - th[oOShift]) / th[oOScale];
    const float e1 = o1 - (target[r * kO + 1] - th[oOShift + 1]) / th[oOScale + 1];
    const float g0 = e0 * inv, g1 = e1 * inv;
    // d2_j = relu'(a2_j) (W3^T dout)_j, and d1 = relu'(a1) o (W2^T d2), the
    // latter accumulated unit by unit of layer 2
    float d1[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) d1[i] = 0.0f;
    for (int j = 0; j < kH; ++j) {
        const float d2 = z2[j] > 0.0f ? fmaf(th[oW3 + j], g0, th[oW3 + kH + j] * g1) : 0.0f;
        w.d2[r * kH + j] = d2;
#pragma unroll
        for (int i = 0; i < kH; ++i) d1[i] = fmaf(th[oW2 + j * kH + i], d2, d1[i]);
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) {
        w.d1[r * kH + i] = z1[i] > 0.0f ? d1[i] : 0.0f;
        w.z1[r * kH + i] = z1[i];
    }
#pragma unroll
    for (int i = 0; i < kF; ++i) w.xs[r * kF + i] = xs[i];
    w.dout[r * kO] = g0;
    w.dout[r * kO + 1] = g1;
    w.loss[r] = 0.5 * ((double)e0 * (double)e0 + (double)e1 * (double)e1);
}

// One thread per trainable parameter: the sum over rows, in row order, of
// its gradient terms (outer products of error signals and inputs), FP64.
// Thread kP - oW1 (one past the last parameter) sums the loss.
__global__ __launch_bounds__(256) void k_mlp_reduce(int64_t rows, TrainWs w, float* __restrict__ grad,
                                                    double* __restrict__ loss_out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = oW1 + t;
    if (k > kP) return;
    if (k == kP) {
        if (loss_out) {
            double s = 0.0;
            for (int64_t r = 0; r < rows; ++r) s += w.loss[r];
            *loss_out = s / (double)rows;
        }
        return;
    }
    const float *a, *b;  // the two factors; b == nullptr for a bias
    int sa, sb;
    if (k < oB1) {
        const int j = (k - oW1) / kF, i = (k - oW1) % kF;
        a = w.d1 + j, sa = kH, b = w.xs + i, sb = kF;
    } else if (k < oW2) {
        a = w.d1 + (k - oB1), sa = kH, b = nullptr, sb = 0;
    } else if (k < oB2) {
        const int j = (k - oW2) / kH, i = (k - oW2) % kH;
        a = w.d2 + j, sa = kH, b = w.z1 + i, sb = kH;
    } else if (k < oW3) {
        a = w.d2 + (k - oB2), sa = kH, b = nullptr, sb = 0;
    } else if (k < oB3) {
        const int j = (k - oW3) / kH, i = (k - oW3) % kH;
        a = w.dout + j, sa = kO, b = w.z2 + i, sb = kH;
    } else {
        a = w.dout + (k - oB3), sa = kO, b = nullptr, sb = 0;
    }
    double s = 0.0;
    if (b) {
        for (int64_t r = 0; r < rows; ++r) s += (double)a[r * sa] * (double)b[r * sb];
    } else {
        for (int64_t r = 0; r < rows; ++r) s += (double)a[r * sa];
    }
    grad[k] = (float)s;
}

// Adam (Kingma & Ba, Algorithm 1) on theta[oW1:]; c1 = 1 - beta1^t and
// c2 = 1 - beta2^t come from the host.
__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ grad,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int k = oW1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kP) return;
    const float g = grad[k];
    const float mk = b1 * m[k] + (1.0f - b1) * g;
    const float vk = b2 * v[k] + (1.0f - b2) * g * g;
    m[k] = mk;
    v[k] = vk;
    theta[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// ---------------------------------------------------------------------------
// budgets: p^ = 1 - Phi((T_obs - mean) / sd); outside the fallback band
// [p_lo, p_hi] the number of splits that separates p^ from the nearer edge by
// zq standard errors, clamped to [b_min, b_max]; inside it, b_max.
// ---------------------------------------------------------------------------
__global__ void k_budgets(int64_t npairs, const float* __restrict__ out,
                          const hbt_result* __restrict__ res, double lo, double hi, int64_t bmin,
                          int64_t bmax, double zq, int64_t* __restrict__ budget) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const double mu = (double)out[p * kO], sd = exp((double)out[p * kO + 1]);
    const double ph = 0.5 * erfc((res[p].t_obs - mu) / sd * 0.70710678118654752440);
    int64_t B = bmax;
    if (ph < lo || ph > hi) {
        const double edge = ph < lo ? lo : hi;
        const double gap = (ph - edge) * (ph - edge);
        const double need = zq * zq * ph * (1.0 - ph) / gap;
        if (need < (double)bmax) {
            const int64_t c = (int64_t)ceil(need);
            B = c < bmin ? bmin : c;
        }
    }
    budget[p] = B;
}

// Expected-cost rule: a pair whose p^ lies in the fallback band gets bmax
// (it would be rerun there anyway); any other pair gets the B among bmin,
// 2 bmin, 4 bmin, ... (below bmax) and bmax that minimises the expected
// splits B + bmax * P(its p lands in [lo, hi] after B splits) (a landing
// is rerun with bmax splits), the estimate (1 + count) / (B + 1) taken as
// normal with mean (1 + B p^) / (B + 1) and sd sqrt(B p^ (1 - p^)) / (B + 1);
// ties go to the smaller B.
__device__ double land_prob(double ph, double B, double lo, double hi) {
    const double mean = (1.0 + B * ph) / (B + 1.0);
    const double sd = sqrt(B * ph * (1.0 - ph)) / (B + 1.0);
    if (!(sd > 0.0)) return (mean >= lo && mean <= hi) ? 1.0 : 0.0;
    const double k = 0.70710678118654752440 / sd;
    // Phi((hi - mean) / sd) - Phi((lo - mean) / sd)
    return 0.5 * erfc((lo - mean) * k) - 0.5 * erfc((hi - mean) * k);
}

__global__ void k_budgets_cost(int64_t npairs, const float* __restrict__ out,
                               const hbt_result* __restrict__ res, double lo, double hi, int64_t bmin,
                               int64_t bmax, int64_t* __restrict__ budget) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const double mu = (double)out[p * kO], sd = exp((double)out[p * kO + 1]);
    const double ph = 0.5 * erfc((res[p].t_obs - mu) / sd * 0.70710678118654752440);
    int64_t B = bmax;
    if (ph < lo || ph > hi) {
        double best = (double)bmax;
        for (int64_t c = bmin; c < bmax; c *= 2) {
            const double cost = (double)c + (double)bmax * land_prob(ph, (double)c, lo, hi);
            if (cost < best) {
                best = cost;
                B = c;
            }
        }
    }
    budget[p] = B;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t mlp_train_ws_bytes(int64_t rows) {
    return (size_t)rows * (kF + 4 * kH + kO) * sizeof(float) + (size_t)rows * sizeof(double) + 256;
}

static TrainWs carve_train(void* ws, int64_t rows) {
    TrainWs w;
    char* p = (char*)ws;
    w.loss = (double*)p;
    p += rows * sizeof(double);
    auto take = [&](int k) {
        float* q = (float*)p;
        p += rows * k * sizeof(float);
        return q;
    };
    w.xs = take(kF);
    w.z1 = take(kH);
    w.z2 = take(kH);
    w.d1 = take(kH);
    w.d2 = take(kH);
    w.dout = take(kO);
    return w;
}

hipError_t launch_features(int64_t npairs, const hbt_result* res, int d, int gd, float* feat,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_features, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, npairs,
                       res, (double)d, gd, feat);
    return hipGetLastError();
}

hipError_t launch_feature_norm(int64_t rows, const float* feat, float* theta, hipStream_t s) {
    hipLaunchKernelGGL(k_col_norm, dim3(kF), dim3(256), 0, s, rows, kF, feat, theta + oShift,
                       theta + oScale, 1);
    return hipGetLastError();
}

hipError_t launch_target_norm(int64_t rows, const float* target, float* theta, hipStream_t s) {
    hipLaunchKernelGGL(k_col_norm, dim3(kO), dim3(256), 0, s, rows, kO, target, theta + oOShift,
                       theta + oOScale, 0);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(int64_t rows, const float* feat, const float* theta, float* out,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, rows,
                       feat, theta, out);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(int64_t rows, const float* feat, const float* target, const float* theta,
                           float* grad, double* loss, void* ws, hipStream_t s) {
    const TrainWs w = carve_train(ws, rows);
    hipLaunchKernelGGL(k_mlp_rows, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, rows, feat,
                       target, theta, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nt = kP - oW1 + 1;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((nt + 255) / 256), dim3(256), 0, s, rows, w, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s) {
    const int nt = kP - oW1;
    hipLaunchKernelGGL(k_adam, dim3((nt + 255) / 256), dim3(256), 0, s, theta, grad, m, v, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_budgets(int64_t npairs, const float* out, const hbt_result* res, double lo,
                          double hi, int64_t bmin, int64_t bmax, double zq, int64_t* budget,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_budgets, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, npairs, out,
                       res, lo, hi, bmin, bmax, zq, budget);
    return hipGetLastError();
}

hipError_t launch_budgets_cost(int64_t npairs, const float* out, const hbt_result* res, double lo,
                               double hi, int64_t bmin, int64_t bmax, int64_t* budget, hipStream_t s) {
    hipLaunchKernelGGL(k_budgets_cost, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, npairs,
                       out, res, lo, hi, bmin, bmax, budget);
    return hipGetLastError();
}

}  // namespace hbt
