/*
 * FP64 CPU oracle for the Householder-aligned permutation test.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into its own shared
 * library and is loaded by the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg.  The product library never includes, links
 * or calls it, and it shares no code with the GPU path: it has its own
 * Philox, its own selection (a full sort) and its own arithmetic.
 *
 * Everything is plain and sequential per permutation: double precision,
 * direct loops, no blocking or reordering beyond what the paper's
 * definitions state.  OpenMP only spreads independent permutations over
 * threads; each permutation's arithmetic is the same sequential loop.
 *
 * The method (Householder-Aligned Permutation Test, Sec. 3.1 and
 * Algorithm 1 of the paper):
 *   1. sample means and mean directions of X and Y;
 *   2. Householder vector v = mu_x - mu_y (the axis u = v/|v|, Eq. for u);
 *   3. align X:  x' = x - 2 v (v.x) / (v.v)      (eq:householder_fast);
 *   4. observed statistic T_obs = log v(X') - log v(Y), v = 1/g_d(r)  (eq:tobs);
 *   5. pool Z = X' u Y, B random splits into sizes (n, m), statistic per split;
 *   6. p = (1 + #{T_b >= T_obs}) / (B + 1)                           (eq:pvalue).
 *
 * Readings where the paper is silent or ambiguous:
 *   - g_d is the Banerjee et al. (2005) vMF concentration estimate
 *     r (d - r^2) / (1 - r^2); g_d(r) = r is offered as the alternative.
 *   - H = I when |v| <= 1e-12 or when alignment is switched off.
 *   - T_obs uses r of the unaligned X (equal to r(X') since H is orthogonal),
 *     so identical groups give exactly 0.
 *   - random split b: item i gets an 8-bit primary key and a 32-bit
 *     secondary key from Philox4x32-10; group 1 is the n items that come
 *     first in the order (primary, secondary, i).
 *   - a permuted statistic counts as an exceedance when T_b >= T_obs - tau
 *     or T_b is NaN, tau = 1e-10 * max(1, |f(r_X)| + |f(r_Y)|).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_SIZE 2
#define ORC_ERR_DEGENERATE 5
#define ORC_ERR_MASK 6
#define ORC_ERR_NOT_UNIT 10

#define ORC_GD_BANERJEE 0
#define ORC_GD_IDENTITY 1
#define ORC_ALT_GREATER 0
#define ORC_ALT_TWO_SIDED 1

/* ------------------------------------------------------------------------
 * Philox-4xW-R (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11, Sec. 4).  One round: two W x W -> 2W products of
 * the even counter words with the multipliers; the new words are
 * (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0).  The key is bumped by the Weyl
 * constants before every round but the first.  The macro is instantiated for
 * W = 32 (used by the method) and W = 64 (checked against numpy's
 * independent Philox4x64-10), so both widths share one round structure.
 * ---------------------------------------------------------------------- */
static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}
static inline void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

#define PHILOX4_DEFINE(NAME, W, MULHILO, M0, M1, WEYL0, WEYL1)               \
    void NAME(const W ctr[4], const W key[2], int rounds, W out[4]) {         \
        W x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];                 \
        W k0 = key[0], k1 = key[1];                                           \
        for (int r = 0; r < rounds; ++r) {                                    \
            if (r > 0) { k0 += (W)(WEYL0); k1 += (W)(WEYL1); }                \
            W hi0, lo0, hi1, lo1;                                             \
            MULHILO((W)(M0), x0, &hi0, &lo0);                                 \
            MULHILO((W)(M1), x2, &hi1, &lo1);                                 \
            W y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;                         \
            x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;                             \
        }                                                                     \
        out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;                   \
    }

PHILOX4_DEFINE(oracle_philox4x32, uint32_t, mulhilo32, 0xD2511F53u, 0xCD9E8D57u,
               0x9E3779B9u, 0xBB67AE85u)
PHILOX4_DEFINE(oracle_philox4x64, uint64_t, mulhilo64, 0xD2E7470EE14C6C93ull,
               0xCA5A826395121157ull, 0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)

/* ------------------------------------------------------------------------
 * Random split b of N items (the "randomly partition Z" step of
 * Algorithm 1, with exactly n items in group 1).
 *   primary key   P_i = byte (i mod 4) of word ((i mod 16) / 4) of
 *                       Philox4x32-10(ctr = (i / 16, b, pair, 0), key = seed)
 *   secondary key S_i = word (i mod 4) of
 *                       Philox4x32-10(ctr = (i / 4, b, pair, 1), key = seed)
 * The 64-bit seed is the key (low word, high word).  Group 1 is the n items
 * that come first when all N items are sorted by (P_i, S_i, i).
 * ---------------------------------------------------------------------- */
static void block4(uint64_t seed, uint32_t pair, uint32_t b, uint32_t c0, uint32_t stream,
                   uint32_t out[4]) {
    uint32_t ctr[4] = {c0, b, pair, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32(ctr, key, 10, out);
}

void oracle_split_keys(uint64_t seed, uint32_t pair, uint32_t b, int64_t N,
                       uint8_t* primary, uint32_t* secondary) {
    for (int64_t i = 0; i < N; ++i) {
        uint32_t w[4];
        block4(seed, pair, b, (uint32_t)(i / 16), 0, w);
        primary[i] = (uint8_t)(w[(i % 16) / 4] >> (8 * (i % 4)));
        block4(seed, pair, b, (uint32_t)(i / 4), 1, w);
        secondary[i] = w[i % 4];
    }
}

typedef struct { uint8_t p; uint32_t s; int64_t i; } split_item;

static int item_cmp(const void* a, const void* b) {
    const split_item* x = (const split_item*)a;
    const split_item* y = (const split_item*)b;
    if (x->p != y->p) return x->p < y->p ? -1 : 1;
    if (x->s != y->s) return x->s < y->s ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

/* Group-1 mask of split b: bit (i mod 32) of word i/32 is set iff item i is in
 * group 1.  W = ceil(N/32) words; bits at positions >= N are zero. */
void oracle_split_mask(uint64_t seed, uint32_t pair, uint32_t b, int64_t N, int64_t n,
                       uint32_t* mask) {
    uint8_t* P = (uint8_t*)malloc((size_t)N);
    uint32_t* S = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    split_item* it = (split_item*)malloc((size_t)N * sizeof(split_item));
    oracle_split_keys(seed, pair, b, N, P, S);
    for (int64_t i = 0; i < N; ++i) { it[i].p = P[i]; it[i].s = S[i]; it[i].i = i; }
    qsort(it, (size_t)N, sizeof(split_item), item_cmp);
    int64_t W = (N + 31) / 32;
    memset(mask, 0, (size_t)W * sizeof(uint32_t));
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = it[k].i;
        mask[i / 32] |= 1u << (i % 32);
    }
    free(it); free(S); free(P);
}

/* ------------------------------------------------------------------------
 * Concentration map and breadth (Sec. 3.1, "Dispersion proxy"): kappa =
 * g_d(r), v = 1/g_d(r).  log_g returns log g_d(r), so log v = -log_g.
 * ---------------------------------------------------------------------- */
double oracle_log_g(double r, int64_t d, int gd) {
    if (gd == ORC_GD_IDENTITY) return log(r);
    /* Banerjee, Dhillon, Ghosh, Sra (JMLR 6, 2005): kappa ~ r (d - r^2) / (1 - r^2) */
    double rr = r * r;
    return log(r * ((double)d - rr) / (1.0 - rr));
}

/* Mean resultant length of a set of rows (Sec. 3.1, MRL definition). */
double oracle_mrl(const double* A, int64_t n, int64_t d) {
    double ss = 0.0;
    for (int64_t c = 0; c < d; ++c) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += A[i * d + c];
        ss += (s / (double)n) * (s / (double)n);
    }
    return sqrt(ss);
}

/* ------------------------------------------------------------------------
 * Steps 1-4 of Algorithm 1: means, directions, Householder vector, aligned
 * X, observed statistic.
 *   info[0] = r_X   info[1] = r_Y   info[2] = T_obs   info[3] = h_identity
 *   info[4] = v.v   info[5] = tau   info[6] = f(r_X)  info[7] = f(r_Y)
 * mu_x, mu_y, v are d-vectors; Xp (n x d) receives the aligned X.
 * Returns ORC_OK, ORC_ERR_DEGENERATE (r outside (0, 1); H = I is used then)
 * or ORC_ERR_NOT_UNIT (a row of X or Y is not l2-normalised as Sec. 3.1, Eq. 2
 * assumes: | |x| - 1 | > 1e-4, or NaN; the computation goes on).
 * ---------------------------------------------------------------------- */
int oracle_align(const double* X, int64_t n, const double* Y, int64_t m, int64_t d,
                 int align, int gd, double* Xp, double* mu_x, double* mu_y, double* v,
                 double* info) {
    if (n < 2 || m < 2 || d < 1) return ORC_ERR_SIZE;
    int status = ORC_OK;
    /* Step 1: x_bar = (1/n) sum_i x_i, y_bar = (1/m) sum_j y_j, sequential sums */
    double* xbar = (double*)calloc((size_t)d, sizeof(double));
    double* ybar = (double*)calloc((size_t)d, sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < d; ++c) xbar[c] += X[i * d + c];
    for (int64_t j = 0; j < m; ++j)
        for (int64_t c = 0; c < d; ++c) ybar[c] += Y[j * d + c];
    for (int64_t c = 0; c < d; ++c) { xbar[c] /= (double)n; ybar[c] /= (double)m; }
    double rx = 0.0, ry = 0.0;
    for (int64_t c = 0; c < d; ++c) { rx += xbar[c] * xbar[c]; ry += ybar[c] * ybar[c]; }
    rx = sqrt(rx);
    ry = sqrt(ry);
    if (!(rx > 0.0 && rx < 1.0 && ry > 0.0 && ry < 1.0)) status = ORC_ERR_DEGENERATE;
    /* precondition of Eq. 2: unit rows, | |x| - 1 | <= 1e-4 */
    for (int64_t i = 0; i < n + m && status == ORC_OK; ++i) {
        const double* row = i < n ? X + i * d : Y + (i - n) * d;
        double ss = 0.0;
        for (int64_t c = 0; c < d; ++c) ss += row[c] * row[c];
        if (!(fabs(sqrt(ss) - 1.0) <= 1e-4)) status = ORC_ERR_NOT_UNIT;
    }
    /* mean directions mu = x_bar / |x_bar| */
    for (int64_t c = 0; c < d; ++c) {
        mu_x[c] = rx > 0.0 ? xbar[c] / rx : 0.0;
        mu_y[c] = ry > 0.0 ? ybar[c] / ry : 0.0;
    }
    /* Step 2: Householder vector v = mu_x - mu_y (u = v / |v|) */
    double vv = 0.0;
    for (int64_t c = 0; c < d; ++c) { v[c] = mu_x[c] - mu_y[c]; vv += v[c] * v[c]; }
    int identity = (!align) || !(sqrt(vv) > 1e-12) || !(rx > 0.0) || !(ry > 0.0);
    /* Step 3: x'_i = x_i - 2 v (v . x_i) / (v . v)   (X' = H X, Y unchanged) */
    for (int64_t i = 0; i < n; ++i) {
        double w = 0.0;
        if (!identity)
            for (int64_t c = 0; c < d; ++c) w += v[c] * X[i * d + c];
        double coef = identity ? 0.0 : 2.0 * w / vv;
        for (int64_t c = 0; c < d; ++c) Xp[i * d + c] = X[i * d + c] - coef * v[c];
    }
    /* Step 4: T_obs = log v(X') - log v(Y) = log g(r_Y) - log g(r_X) */
    double fx = oracle_log_g(rx, d, gd), fy = oracle_log_g(ry, d, gd);
    double tobs = fy - fx;
    double scale = fabs(fx) + fabs(fy);
    info[0] = rx; info[1] = ry; info[2] = tobs; info[3] = identity ? 1.0 : 0.0;
    info[4] = vv; info[5] = 1e-10 * (scale > 1.0 ? scale : 1.0); info[6] = fx; info[7] = fy;
    free(xbar); free(ybar);
    return status;
}

/* Permuted statistic for one split (Algorithm 1, Step 5): group sums by
 * direct summation over the pooled rows Z (N x d) in ascending row order. */
double oracle_split_stat(const double* Z, int64_t n, int64_t m, int64_t d, const uint32_t* mask,
                         int gd, double* r1_out, double* r2_out) {
    int64_t N = n + m;
    double* s1 = (double*)calloc((size_t)d, sizeof(double));
    double* s2 = (double*)calloc((size_t)d, sizeof(double));
    for (int64_t i = 0; i < N; ++i) {
        double* s = ((mask[i / 32] >> (i % 32)) & 1u) ? s1 : s2;
        for (int64_t c = 0; c < d; ++c) s[c] += Z[i * d + c];
    }
    double q1 = 0.0, q2 = 0.0;
    for (int64_t c = 0; c < d; ++c) {
        double a = s1[c] / (double)n, b = s2[c] / (double)m;
        q1 += a * a;
        q2 += b * b;
    }
    double r1 = sqrt(q1), r2 = sqrt(q2);
    free(s1); free(s2);
    if (r1_out) *r1_out = r1;
    if (r2_out) *r2_out = r2;
    /* T_b = log(1/g(r1)) - log(1/g(r2)) */
    return oracle_log_g(r2, d, gd) - oracle_log_g(r1, d, gd);
}

static int exceeds(double T, double tobs, double tau, int alternative) {
    if (isnan(T)) return 1;
    if (alternative == ORC_ALT_TWO_SIDED) return fabs(T) >= fabs(tobs) - tau;
    return T >= tobs - tau;
}

static int popcount32(uint32_t x) {
    int c = 0;
    while (x) { x &= x - 1; ++c; }
    return c;
}

/* ------------------------------------------------------------------------
 * The whole test (Algorithm 1).  Permutation indices are global:
 * b = perm_offset + k for k in [0, B).  masks (optional, B x ceil(N/32))
 * replace the Philox splits.
 *   out[0] = T_obs  out[1] = r_X  out[2] = r_Y  out[3] = p  out[4] = count
 *   out[5] = h_identity  out[6] = tau  out[7] = v.v
 * T_out (optional, B) receives T_b; mask_out (optional) the splits used.
 * ---------------------------------------------------------------------- */
int oracle_perm_test(const double* X, int64_t n, const double* Y, int64_t m, int64_t d,
                     int64_t B, uint64_t seed, uint32_t pair, uint64_t perm_offset, int align,
                     int gd, int alternative, const uint32_t* masks, double* out, double* T_out,
                     uint32_t* mask_out, int nthreads) {
    if (n < 2 || m < 2 || d < 1 || B < 1) return ORC_ERR_SIZE;
    if (perm_offset + (uint64_t)B > 0x100000000ull) return ORC_ERR_ARG;
    int64_t N = n + m, W = (N + 31) / 32;
    double* Z = (double*)malloc((size_t)(N * d) * sizeof(double));
    double* mux = (double*)malloc((size_t)d * sizeof(double));
    double* muy = (double*)malloc((size_t)d * sizeof(double));
    double* v = (double*)malloc((size_t)d * sizeof(double));
    double info[8];
    /* Steps 1-4; Step 5 pools Z = [X'; Y] */
    int status = oracle_align(X, n, Y, m, d, align, gd, Z, mux, muy, v, info);
    memcpy(Z + n * d, Y, (size_t)(m * d) * sizeof(double));
    double tobs = info[2], tau = info[5];
    if (masks) {
        for (int64_t k = 0; k < B; ++k) {
            int pc = 0;
            for (int64_t w = 0; w < W; ++w) pc += popcount32(masks[k * W + w]);
            uint32_t tail = (N % 32) ? (masks[k * W + W - 1] >> (N % 32)) : 0u;
            if (pc != n || tail) { status = ORC_ERR_MASK; break; }
        }
    }
    int64_t count = 0;
    if (status != ORC_ERR_MASK) {
#ifdef _OPENMP
        if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : count)
#endif
        for (int64_t k = 0; k < B; ++k) {
            uint32_t* mk = (uint32_t*)malloc((size_t)W * sizeof(uint32_t));
            if (masks)
                memcpy(mk, masks + k * W, (size_t)W * sizeof(uint32_t));
            else
                oracle_split_mask(seed, pair, (uint32_t)(perm_offset + (uint64_t)k), N, n, mk);
            double T = oracle_split_stat(Z, n, m, d, mk, gd, NULL, NULL);
            if (T_out) T_out[k] = T;
            if (mask_out) memcpy(mask_out + k * W, mk, (size_t)W * sizeof(uint32_t));
            count += exceeds(T, tobs, tau, alternative);
            free(mk);
        }
    }
    /* Step 6: p = (1 + count) / (B + 1)  (eq:pvalue) */
    out[0] = tobs; out[1] = info[0]; out[2] = info[1];
    out[3] = (1.0 + (double)count) / ((double)B + 1.0);
    out[4] = (double)count; out[5] = info[3]; out[6] = tau; out[7] = info[4];
    free(Z); free(mux); free(muy); free(v);
    return status;
}

/* T_b for an arbitrary list of global permutation indices (for sampled
 * comparisons at full size). */
int oracle_perm_stats_at(const double* X, int64_t n, const double* Y, int64_t m, int64_t d,
                         uint64_t seed, uint32_t pair, int align, int gd, const uint64_t* blist,
                         int64_t nb, double* T_out, double* r1_out, double* r2_out,
                         uint32_t* mask_out, int nthreads) {
    if (n < 2 || m < 2 || d < 1) return ORC_ERR_SIZE;
    int64_t N = n + m, W = (N + 31) / 32;
    double* Z = (double*)malloc((size_t)(N * d) * sizeof(double));
    double* mux = (double*)malloc((size_t)d * sizeof(double));
    double* muy = (double*)malloc((size_t)d * sizeof(double));
    double* v = (double*)malloc((size_t)d * sizeof(double));
    double info[8];
    int status = oracle_align(X, n, Y, m, d, align, gd, Z, mux, muy, v, info);
    memcpy(Z + n * d, Y, (size_t)(m * d) * sizeof(double));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t k = 0; k < nb; ++k) {
        uint32_t* mk = (uint32_t*)malloc((size_t)W * sizeof(uint32_t));
        oracle_split_mask(seed, pair, (uint32_t)blist[k], N, n, mk);
        double r1, r2;
        T_out[k] = oracle_split_stat(Z, n, m, d, mk, gd, &r1, &r2);
        if (r1_out) r1_out[k] = r1;
        if (r2_out) r2_out[k] = r2;
        if (mask_out) memcpy(mask_out + k * W, mk, (size_t)W * sizeof(uint32_t));
        free(mk);
    }
    free(Z); free(mux); free(muy); free(v);
    return status;
}

/* ------------------------------------------------------------------------
 * Exhaustive enumeration: every n-subset of {0..N-1} (lexicographic order)
 * is group 1 once.  The observed split is among them, so the exact p-value
 * is count / C(N, n) with no +1.  out as in oracle_perm_test; out[3] is the
 * exact p and out[8] = C(N, n).
 * ---------------------------------------------------------------------- */
int oracle_exhaustive(const double* X, int64_t n, const double* Y, int64_t m, int64_t d,
                      int align, int gd, int alternative, double* out, double* T_out,
                      int64_t T_cap) {
    if (n < 2 || m < 2 || d < 1) return ORC_ERR_SIZE;
    int64_t N = n + m, W = (N + 31) / 32;
    if (N > 40) return ORC_ERR_SIZE;
    double* Z = (double*)malloc((size_t)(N * d) * sizeof(double));
    double* mux = (double*)malloc((size_t)d * sizeof(double));
    double* muy = (double*)malloc((size_t)d * sizeof(double));
    double* v = (double*)malloc((size_t)d * sizeof(double));
    double info[8];
    int status = oracle_align(X, n, Y, m, d, align, gd, Z, mux, muy, v, info);
    memcpy(Z + n * d, Y, (size_t)(m * d) * sizeof(double));
    double tobs = info[2], tau = info[5];
    int64_t* idx = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    uint32_t* mk = (uint32_t*)malloc((size_t)W * sizeof(uint32_t));
    for (int64_t k = 0; k < n; ++k) idx[k] = k;
    int64_t count = 0, total = 0;
    for (;;) {
        memset(mk, 0, (size_t)W * sizeof(uint32_t));
        for (int64_t k = 0; k < n; ++k) mk[idx[k] / 32] |= 1u << (idx[k] % 32);
        double T = oracle_split_stat(Z, n, m, d, mk, gd, NULL, NULL);
        if (T_out && total < T_cap) T_out[total] = T;
        count += exceeds(T, tobs, tau, alternative);
        ++total;
        /* next combination in lexicographic order */
        int64_t k = n - 1;
        while (k >= 0 && idx[k] == N - n + k) --k;
        if (k < 0) break;
        ++idx[k];
        for (int64_t j = k + 1; j < n; ++j) idx[j] = idx[j - 1] + 1;
    }
    out[0] = tobs; out[1] = info[0]; out[2] = info[1];
    out[3] = (double)count / (double)total;
    out[4] = (double)count; out[5] = info[3]; out[6] = tau; out[7] = info[4];
    out[8] = (double)total;
    free(idx); free(mk); free(Z); free(mux); free(muy); free(v);
    return status;
}
