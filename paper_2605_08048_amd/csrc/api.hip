// Host side of the C ABI (include/hbt.h): argument checks, workspace carving,
// plan tables and the launch sequence of a test.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hbt_launch.h"

// Device scratch of hbt_perm_test_static: the workspace of a single-pair test
// for callers that cannot allocate.  Each device the library runs on holds its
// own copy until the process ends.  Host code must never pass this name to a
// kernel or a copy (in host code it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, once per device.
__device__ __align__(256) unsigned char scratch[HBT_STATIC_SCRATCH_BYTES];

namespace {

using namespace hbt;

thread_local std::string g_err;

hbt_status fail(hbt_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
hbt_status fail(hbt_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(HBT_ERR_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                        __FILE__, __LINE__);                                              \
    } while (0)

// --- stage timing ------------------------------------------------------
struct StageRecord {
    int stage;
    hipEvent_t start, stop;
};
std::mutex g_timing_mu;
bool g_timing = false;
std::vector<StageRecord> g_records;

// Records a start event at construction and a stop event at destruction on
// the stream, when timing is enabled.
struct StageTimer {
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    int stage;
    StageTimer(int st, hipStream_t str) : s(str), stage(st) {
        std::lock_guard<std::mutex> g(g_timing_mu);
        if (!g_timing) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess ||
            hipEventRecord(a, s) != hipSuccess) {
            a = b = nullptr;
        }
    }
    ~StageTimer() {
        if (!a) return;
        if (hipEventRecord(b, s) != hipSuccess) return;
        std::lock_guard<std::mutex> g(g_timing_mu);
        g_records.push_back(StageRecord{stage, a, b});
    }
};

constexpr int64_t kAutoBlock = 32768;  // splits per block when block_perms == 0

int64_t round_up(int64_t x, int64_t k) { return (x + k - 1) / k * k; }

// Recheck band of each precision (recheck_eps; terms in hbt_internal.h).
// Storage bounds per coordinate of a unit row, scaled to the RMS coordinate
// 1/sqrt(d) where the format is relative: FP32 2^-24, split BF16 2^-16 (hi
// rounds to 8 significant bits, lo the remainder to 8 more), int8 digit
// planes an absolute 2^-21 (z rounded to a multiple of 2^-20).  e_acc is the
// measured FP32 accumulation error (worst 2.5e-7 for FP32, 1.6e-6 for split
// BF16 over 35 shapes with n, m from 2 to 5000, d = 64 ... 1024, r up to
// 0.997); the int8 sums are exact.  The safety factors keep the worst error
// of an exact emulation of the stored rows (duplicated rows repeated up to
// 1000 times, clouds with r from 0.02 to 1, a group of 2) below a quarter of
// the band.  The point-to-centroid route reads an FP32 copy of the rows and
// the centroids as floats, so its band is at least the FP32 one, plus the
// dot-product term of its products (FP32, or split BF16 in three terms).
RecheckBand precision_band(int precision, int d, bool route2) {
    const double rd = 1.0 / std::sqrt((double)d);
    RecheckBand b;
    switch (precision) {
        case HBT_F64: b = RecheckBand{1e-12, 0x1p-53 * rd, 4.0, 0.0}; break;
        case HBT_F32: b = RecheckBand{4e-6, 0x1p-24 * rd, 4.0, 0.0}; break;
        case HBT_I8X3: b = RecheckBand{1e-10, 0x1p-21, 12.0, 0.0}; break;
        // e4m3 keeps 4 significant bits: |lo - e4m3(lo)| <= 2^-4 |lo| <= 2^-12 |z|
        // (lo the bf16 remainder, |lo| <= 2^-8 |z|); plus the fp8 MFMA's own
        // rounding of its 64-term dot products (2^-13 of the lo terms, i.e.
        // 2^-21 |z|) and the subnormal spacing of the scaled lo (2^-27 absolute)
        case HBT_BF16_E4M3: b = RecheckBand{4e-6, (0x1p-12 + 0x1p-21) * rd + 0x1p-27, 4.0, 0.0}; break;
        // the lazy precision's first pass: the bf16 hi plane alone keeps 8
        // significant bits, |z - hi| <= 2^-8 |z| (the second pass has the
        // split-BF16 band; pairs with a group under kLazyMinGroup skip the
        // first pass's decisions)
        case HBT_BF16_LAZY: b = RecheckBand{4e-6, 0x1p-8 * rd, 4.0, 0.0}; break;
        default: b = RecheckBand{4e-6, 0x1p-16 * rd, 4.0, 0.0}; break;
    }
    if (route2) {
        b.e_acc = std::max(b.e_acc, 4e-6);
        b.e_row = std::max(b.e_row, 0x1p-24 * rd);
        // FP32 products: accumulation over K = d; split BF16 (three terms):
        // besides, each product z_c s_c is off by up to 2^-15 |z_c s_c| (the
        // two splits' remainders and the dropped lo x lo term)
        b.e_q = 8.0 * 0x1p-24 + (precision == HBT_BF16X2 ? 0x1p-15 * rd : 0.0);
    }
    return b;
}

size_t zstore_bytes(int precision, int64_t rows, int64_t d_pad) {
    const int bytes = precision == HBT_F64 ? 8 : precision == HBT_I8X3 || precision == HBT_BF16_E4M3 ? 3 : 4;
    return (size_t)rows * d_pad * bytes;
}

// Bump allocator over the caller's workspace (256-byte aligned slices).
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base((char*)b) {}
    template <typename T>
    T* take(size_t count) {
        off = (size_t)round_up((int64_t)off, 256);
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Everything a call needs in device memory, carved in one fixed order so that
// the *_workspace_size functions and the calls agree.
struct Workspace {
    PairDesc* pairs;
    BlockPair* bp;
    GemmTile* tiles;
    GemmGroup* groups;
    int64_t* Btot;
    double* partial_sum;
    int32_t* chunk_bad;  // per column-sum chunk: a row is not a unit vector
    double* sxy;
    PairState* st;
    double* v;
    double* t64;
    float* t32;
    PairCount* cnt;
    double* coef;
    void* zstore;
    uint32_t* mask;
    double* partial;
    uint32_t* flags;
    double* tw;         // final T_b of the current block (moments)
    double* rseg;       // recheck segment sums (nullptr when no pair has more than one segment)
    int64_t* rplan;     // recheck work plan
    uint32_t* nflag;    // per pair: its recheck flags
    int32_t* sstat;     // per pair: problems of the split stage (merged into the result status)
    // point-to-centroid route
    float* sig;         // group sums of the smaller group, block rows x d_pad
    float* z32;         // row-major FP32 Z when the main storage is not FP32
    double* zt;         // z_i . t per pooled row
    double* partial2;   // block rows x row tiles x 2
    CTile* ctiles;      // its tile list (64 rows x 256 splits per tile)
    // pairs of shared clouds (rows stored unreflected, the Householder fold)
    PairDesc* cdesc;    // one run of storage per cloud (the column-sum table)
    float* v32;         // FP32 copy of each pair's v
    double* pv;         // v . sigma per split row and slot (slot-major)
    double* fpart;      // fold sums per segment of X items and split row (segment-major)
    // the lazy precision's refinement lists and their tile table
    uint32_t* rlist;    // per pair, from its first block row: the split rows to refine
    uint32_t* rcnt;     // per pair: their number
    GemmGroup* rgroups; // tile table of the refinement product (one group per product group)
    int64_t* rtiles;    // its tile count
    size_t bytes;
};

// Tuned launch parameters (see tile_cost).
struct TileCost {
    double c[2];      // [0]: kTileWide-split tiles, [1]: 256-split tiles
    int grid_wide;    // persistent work-groups per CU, 1024-split launch
    int grid_narrow;  // ... 256-split split-BF16 or int8 launch
    int split_cap;    // split work-groups per CU beside the alignment
    int chunks;       // pipeline chunks of the batched call
    bool tuned;
};
TileCost default_tune(int precision) {
    return TileCost{{1.0, 1.15}, 16, precision == HBT_I8X3 ? 16 : 32, kSplitWgPerCuBesideAlign, 1, false};
}
struct Plan {
    int npairs = 0;
    int d = 0, d_pad = 0, nslot = 0;
    int precision = HBT_F32;
    int input_dtype = HBT_IN_F32;
    int max_np = 0;
    std::vector<PairDesc> pairs;
    std::vector<BlockPair> bp;
    std::vector<SumChunk> chunks;
    std::vector<GemmTile> tiles;
    std::vector<GemmGroup> groups; // split BF16: the kTileWide groups, then the 256-wide ones
    int64_t ntile_total = 0;      // tiles of the split-BF16 kernel over all groups
    int ngw = 0, ng256 = 0;       // groups of each tile width
    int64_t ntw = 0, nt256 = 0;   // their tiles (tile0 counts from 0 in each segment)
    std::vector<int64_t> Btot;
    int64_t zrows = 0, ncoef = 0;
    int64_t xoct = 0;             // storage octets that hold X rows (all pairs)
    int64_t block_rows = 0;       // split rows of the largest block
    int64_t block_mask_words = 0; // mask words of the largest block
    bool need_store = true;       // group-sum path (false for hbt_align)
    bool route2 = false;          // point-to-centroid statistic route
    bool aligned16 = true;        // every X, Y starts on a 16-byte boundary
    int ntile_i = 0;              // its row tiles (of 64) per split, largest pair
    std::vector<CTile> ctiles;    // b-tile major, then row tiles (per pair)
    // Pipeline chunks of the batched call: pairs [pa, pb), their groups from
    // g0 (the wide ones, then the narrow ones, tiles numbered from 0 in each)
    struct Chunk {
        int pa, pb, g0, ngw, ng256;
        int64_t ntw, nt256;
    };
    std::vector<Chunk> cplan;
    TileCost tune = default_tune(HBT_BF16X2);  // launch parameters of (precision, d_pad)
    bool lazy = false;             // HBT_BF16_LAZY: split-BF16 storage (precision), hi-plane first pass
    bool fold = false;             // pairs of shared clouds, stored unreflected
    int fold_segs = 0;             // the largest pair's fold_segments(n)
    std::vector<PairDesc> cdesc;   // their clouds
};

// The product kernels number their tiles with 32-bit integers.  A plan whose
// tile list would not fit (possible only near the size limits: many pairs at
// a large d, or very large split blocks) is refused before anything is
// enqueued; the lazy precision is checked for the refinement tiles it would
// need if every split went to its second product.
hbt_status check_tiles(const Plan& P) {
    constexpr int64_t kMaxTiles = INT32_MAX - 64;
    int64_t worst = std::max<int64_t>(P.ntile_total, (int64_t)P.tiles.size() * P.nslot);
    worst = std::max<int64_t>(worst, (int64_t)P.ctiles.size());
    if (P.lazy) {
        int64_t t = 0;
        for (const BlockPair& b : P.bp) t += (b.nb + kTileNarrow - 1) / kTileNarrow;
        worst = std::max<int64_t>(worst, t * P.nslot);
    }
    if (worst > kMaxTiles)
        return fail(HBT_ERR_SIZE, "%lld product tiles in one call, at most %lld: split the batch or the block",
                    (long long)worst, (long long)kMaxTiles);
    return HBT_OK;
}

Workspace carve(const Plan& P, void* ws) {
    Carve c(ws);
    Workspace w;
    const int np = std::max(P.npairs, 1);
    w.pairs = c.take<PairDesc>(np);
    w.bp = c.take<BlockPair>(np);
    w.tiles = c.take<GemmTile>(std::max<size_t>(P.tiles.size(), 1));
    w.groups = c.take<GemmGroup>(std::max<size_t>(P.groups.size(), 1));
    w.Btot = c.take<int64_t>(np);
    w.partial_sum = c.take<double>(std::max<size_t>(P.chunks.size(), 1) * P.d);
    w.chunk_bad = c.take<int32_t>(std::max<size_t>(P.chunks.size(), 1));
    w.sxy = c.take<double>((size_t)np * 2 * P.d_pad);
    w.st = c.take<PairState>(np);
    w.v = c.take<double>((size_t)np * P.d_pad);
    w.t64 = c.take<double>((size_t)np * P.d_pad);
    w.t32 = c.take<float>((size_t)np * P.d_pad);
    w.cnt = c.take<PairCount>(np);
    if (P.need_store) {
        w.coef = c.take<double>(std::max<int64_t>(P.ncoef, 1) + 32);  // 32 spare: whole mask words read
        const size_t zb = zstore_bytes(P.precision, P.zrows, P.d_pad);
        w.zstore = c.take<char>(zb);
        w.mask = c.take<uint32_t>(std::max<int64_t>(P.block_mask_words, 1));
        w.partial = c.take<double>((size_t)std::max<int64_t>(P.block_rows, 1) * P.nslot * 2);
        w.flags = c.take<uint32_t>(std::max<int64_t>(P.block_rows, 1));
        w.tw = c.take<double>(std::max<int64_t>(P.block_rows, 1));
        w.rseg = recheck_segments(P.max_np) > 1
                     ? c.take<double>((size_t)recheck_slots(P.npairs, P.d_pad) * P.d_pad) : nullptr;
        w.rplan = c.take<int64_t>(recheck_plan_words(np));
        w.nflag = c.take<uint32_t>((size_t)(np + 1) / 2 * 2);
        w.sstat = c.take<int32_t>((size_t)(np + 1) / 2 * 2);
        if (P.route2) {
            w.sig = c.take<float>((size_t)std::max<int64_t>(P.block_rows, 1) * P.d_pad);
            w.z32 = P.precision == HBT_F32 ? nullptr : c.take<float>((size_t)P.zrows * P.d_pad);
            w.zt = c.take<double>(std::max<int64_t>(P.zrows, 1));
            w.partial2 = c.take<double>((size_t)std::max<int64_t>(P.block_rows, 1) * P.ntile_i * 2);
            w.ctiles = c.take<CTile>(std::max<size_t>(P.ctiles.size(), 1));
        } else {
            w.sig = nullptr;
            w.z32 = nullptr;
            w.zt = nullptr;
            w.partial2 = nullptr;
            w.ctiles = nullptr;
        }
    } else {
        w.sig = nullptr;
        w.z32 = nullptr;
        w.zt = nullptr;
        w.partial2 = nullptr;
        w.ctiles = nullptr;
        w.coef = nullptr;
        w.zstore = nullptr;
        w.mask = nullptr;
        w.partial = nullptr;
        w.flags = nullptr;
        w.tw = nullptr;
        w.rseg = nullptr;
        w.rplan = nullptr;
        w.nflag = nullptr;
        w.sstat = nullptr;
    }
    if (P.fold) {
        w.cdesc = c.take<PairDesc>(std::max<size_t>(P.cdesc.size(), 1));
        w.v32 = c.take<float>((size_t)np * P.d_pad);
        w.pv = c.take<double>((size_t)std::max<int64_t>(P.block_rows, 1) * P.nslot);
        w.fpart = c.take<double>((size_t)std::max<int64_t>(P.block_rows, 1) * std::max(P.fold_segs, 1));
    } else {
        w.cdesc = nullptr;
        w.v32 = nullptr;
        w.pv = nullptr;
        w.fpart = nullptr;
    }
    if (P.lazy) {
        w.rlist = c.take<uint32_t>((size_t)std::max<int64_t>(P.block_rows, 1));
        w.rcnt = c.take<uint32_t>((size_t)(np + 1) / 2 * 2);
        w.rgroups = c.take<GemmGroup>(std::max<size_t>(P.groups.size(), 1));
        w.rtiles = c.take<int64_t>(1);
    } else {
        w.rlist = nullptr;
        w.rcnt = nullptr;
        w.rgroups = nullptr;
        w.rtiles = nullptr;
    }
    w.bytes = c.off + 256;
    return w;
}

void add_pair(Plan& P, const void* X, const void* Y, int64_t n, int64_t m, uint32_t pair_index) {
    P.aligned16 = P.aligned16 && ((uintptr_t)X % 16 == 0) && ((uintptr_t)Y % 16 == 0);
    PairDesc pd;
    memset(&pd, 0, sizeof pd);
    pd.X = X;
    pd.Y = Y;
    pd.n = (int32_t)n;
    pd.m = (int32_t)m;
    pd.Np = (int32_t)round_up(n + m, kRowPad);
    pd.Wp = pd.Np / 32;
    pd.zrow0 = P.zrows;
    pd.coef0 = P.ncoef;
    pd.pair_index = pair_index;
    pd.flip = m < n ? 1 : 0;
    const int p = (int)P.pairs.size();
    pd.cx0 = (int32_t)P.chunks.size();
    for (int64_t r = 0; r < n; r += kSumChunk)
        P.chunks.push_back(SumChunk{p, 0, (int32_t)r, (int32_t)std::min<int64_t>(n, r + kSumChunk)});
    pd.cx1 = (int32_t)P.chunks.size();
    for (int64_t j = n / kSumChunkY; kSumChunkY * j < pd.Np; ++j)  // groups from row n to Np
        P.chunks.push_back(SumChunk{p, 1, (int32_t)(std::max<int64_t>(n, kSumChunkY * j) - n),
                                    (int32_t)(std::min<int64_t>(n + m, kSumChunkY * (j + 1)) - n)});
    pd.cy1 = (int32_t)P.chunks.size();
    pd.cy0 = pd.cx1;
    pd.zrow_y = P.zrows;
    pd.nxc = pd.Np / kRowPad;
    pd.ygap = 0;
    pd.xoct0 = P.xoct;
    P.xoct += x_octets(n);
    P.zrows += pd.Np;
    P.ncoef += n;
    P.max_np = std::max(P.max_np, (int)pd.Np);
    P.pairs.push_back(pd);
    P.npairs = (int)P.pairs.size();
}

hbt_status check_enums(const hbt_perm_params* prm) {
    if (prm->precision < HBT_F64 || prm->precision > HBT_BF16_LAZY)
        return fail(HBT_ERR_ARG, "unknown precision %d", prm->precision);
    if (prm->input_dtype != HBT_IN_F32 && prm->input_dtype != HBT_IN_F64)
        return fail(HBT_ERR_DTYPE, "unknown input dtype %d", prm->input_dtype);
    if (prm->gd != HBT_GD_BANERJEE && prm->gd != HBT_GD_IDENTITY)
        return fail(HBT_ERR_ARG, "unknown g_d %d", prm->gd);
    if (prm->alternative != HBT_ALT_GREATER && prm->alternative != HBT_ALT_TWO_SIDED)
        return fail(HBT_ERR_ARG, "unknown alternative %d", prm->alternative);
    if (prm->align != 0 && prm->align != 1) return fail(HBT_ERR_ARG, "align must be 0 or 1");
    if (prm->stat_route != 0 && prm->stat_route != 1)
        return fail(HBT_ERR_ARG, "unknown stat_route %d", prm->stat_route);
    if (prm->stat_route == 1 &&
        (prm->precision == HBT_I8X3 || prm->precision == HBT_BF16_E4M3 || prm->precision == HBT_BF16_LAZY))
        return fail(HBT_ERR_UNSUPPORTED,
                    "the int8, BF16 + e4m3 and lazy split-BF16 products compute the statistic by route 0 only");
    if (prm->flags & ~(HBT_FLAG_NO_RECHECK | HBT_FLAG_T_OUT_F64 | HBT_FLAG_T_OUT_NORMS))
        return fail(HBT_ERR_ARG, "unknown flags 0x%x", prm->flags);
    return HBT_OK;
}

hbt_status check_sizes(int64_t n, int64_t m, int64_t d, int64_t B, uint64_t perm_offset) {
    if (n < 2 || m < 2) return fail(HBT_ERR_SIZE, "n and m must be >= 2 (got %lld, %lld)", (long long)n, (long long)m);
    if (d < 1 || d > HBT_MAX_D) return fail(HBT_ERR_SIZE, "d = %lld outside [1, %d]", (long long)d, HBT_MAX_D);
    if (n + m > HBT_MAX_N) return fail(HBT_ERR_SIZE, "n + m = %lld above %d", (long long)(n + m), HBT_MAX_N);
    if (B < 1) return fail(HBT_ERR_SIZE, "B must be >= 1");
    if (perm_offset > 0x100000000ull || (uint64_t)B > 0x100000000ull - perm_offset)
        return fail(HBT_ERR_ARG, "perm_offset + B exceeds 2^32 split indices");
    return HBT_OK;
}

TileCost tile_cost(int d_pad, int precision);

void finish_plan(Plan& P, int64_t d, int precision, int input_dtype) {
    P.d = (int)d;
    P.d_pad = (int)round_up(d, kDPad);
    P.nslot = P.d_pad / kDSlot;
    // the lazy precision stores and tunes as split BF16; only its product
    // and statistic stages differ
    P.lazy = precision == HBT_BF16_LAZY;
    P.precision = P.lazy ? HBT_BF16X2 : precision;
    P.input_dtype = input_dtype;
    P.tune = tile_cost(P.d_pad, P.precision);
}

// ---------------------------------------------------------------------------
// Tuned launch parameters, per (precision, d_pad): the per-split costs of the
// two tile widths of the split-BF16 product (per pair, or per block of one
// pair, the width w in {kTileWide, 256} minimising cost_w * round_up(B, w)),
// the persistent grids of the product launches, the split stage's
// work-groups per CU beside the alignment and the pipeline chunks of the
// batched call.  hbt_tune_batched measures them on the caller's workload;
// HBT_TUNE_CACHE names a JSON file that is read on first use and written
// after each tuning.
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::pair<int, int>, TileCost> g_tune;  // (precision, d_pad)
thread_local int g_force_width = 0;  // 0: choose; kTileWide or 256: every pair (tuning runs)
int tune_load_locked(const char* path);
void tune_cache_once_locked() {
    static bool done = false;
    if (done) return;
    done = true;
    const char* path = getenv("HBT_TUNE_CACHE");
    if (path && *path) (void)tune_load_locked(path);
}

TileCost tile_cost(int d_pad, int precision) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache_once_locked();
    auto it = g_tune.find({precision, d_pad});
    return it != g_tune.end() ? it->second : default_tune(precision);
}

// JSON cache: {"hbt_tune_version": 1, "entries": [{"precision": p, "d_pad":
// D, "cost": [c0, c1], "grid_wide": g, "grid_narrow": g, "split_cap": s,
// "chunks": k}, ...]}, one entry per line.
int tune_save_locked(const char* path) {
    FILE* f = fopen(path, "w");
    if (!f) return -1;
    fprintf(f, "{\"hbt_tune_version\": 1, \"entries\": [");
    bool first = true;
    for (const auto& kv : g_tune) {
        const TileCost& t = kv.second;
        if (!t.tuned) continue;
        fprintf(f, "%s\n {\"precision\": %d, \"d_pad\": %d, \"cost\": [%.17g, %.17g], \"grid_wide\": %d, "
                   "\"grid_narrow\": %d, \"split_cap\": %d, \"chunks\": %d}",
                first ? "" : ",", kv.first.first, kv.first.second, t.c[0], t.c[1], t.grid_wide, t.grid_narrow,
                t.split_cap, t.chunks);
        first = false;
    }
    fprintf(f, "\n]}\n");
    return fclose(f) == 0 ? 0 : -1;
}

bool tune_valid(const TileCost& t) {
    return t.c[0] > 0.0 && t.c[1] > 0.0 && t.grid_wide >= 1 && t.grid_wide <= 256 && t.grid_narrow >= 1 &&
           t.grid_narrow <= 256 && t.split_cap >= 1 && t.split_cap <= 16 && t.chunks >= 1 && t.chunks <= 64;
}

// Reads the entries of a file written by tune_save_locked; returns the number
// read, or -1 when the file cannot be read or holds a malformed entry (then
// nothing is changed).
int tune_load_locked(const char* path) {
    FILE* f = fopen(path, "r");
    if (!f) return -1;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
    fclose(f);
    if (text.find("\"hbt_tune_version\": 1") == std::string::npos) return -1;
    std::vector<std::pair<std::pair<int, int>, TileCost>> got;
    size_t pos = text.find('[');
    while (pos != std::string::npos && (pos = text.find('{', pos + 1)) != std::string::npos) {
        const size_t end = text.find('}', pos);
        if (end == std::string::npos) return -1;
        const std::string e = text.substr(pos, end - pos + 1);
        int prec, dp;
        TileCost t{};
        t.tuned = true;
        if (sscanf(e.c_str(),
                   "{\"precision\": %d, \"d_pad\": %d, \"cost\": [%lf, %lf], \"grid_wide\": %d, "
                   "\"grid_narrow\": %d, \"split_cap\": %d, \"chunks\": %d}",
                   &prec, &dp, &t.c[0], &t.c[1], &t.grid_wide, &t.grid_narrow, &t.split_cap, &t.chunks) != 8)
            return -1;
        if (prec < HBT_F64 || prec > HBT_BF16_E4M3 || dp < kDPad || dp > HBT_MAX_D || dp % kDPad || !tune_valid(t))
            return -1;
        got.push_back({{prec, dp}, t});
        pos = end;
    }
    for (const auto& kv : got) g_tune[kv.first] = kv.second;
    return (int)got.size();
}

int choose_width(int64_t B, const TileCost& tc) {
    if (g_force_width) return g_force_width;
    const double tw = tc.c[0] * (double)round_up(B, kTileWide), t256 = tc.c[1] * (double)round_up(B, 256);
    return t256 < tw ? 256 : kTileWide;
}

// Groups of split-BF16 tiles, pairs in the given order, segmented by width.
// The product's groups of the pairs [pa, pb) (in `order`, largest first), as
// one pipeline chunk: its wide groups, then its narrow ones, tiles numbered
// from 0 within each width.
void add_groups(Plan& P, const std::vector<int>& order, const int64_t* B, int pa, int pb) {
    const TileCost& tc = P.tune;
    Plan::Chunk c{pa, pb, (int)P.groups.size(), 0, 0, 0, 0};
    std::vector<GemmGroup> g2;
    for (int p : order) {
        const int w = P.precision == HBT_I8X3 ? kTileI8 : choose_width(B[p], tc);
        const int nbt = (int)((B[p] + w - 1) / w);
        if (w == kTileWide) {
            P.groups.push_back(GemmGroup{p, nbt, c.ntw});
            c.ntw += (int64_t)nbt * P.nslot;
        } else {
            g2.push_back(GemmGroup{p, nbt, c.nt256});
            c.nt256 += (int64_t)nbt * P.nslot;
        }
    }
    c.ngw = (int)P.groups.size() - c.g0;
    c.ng256 = (int)g2.size();
    P.groups.insert(P.groups.end(), g2.begin(), g2.end());
    P.ngw += c.ngw;
    P.ng256 += c.ng256;
    P.ntw += c.ntw;
    P.nt256 += c.nt256;
    P.ntile_total = P.ntw + P.nt256;
    P.cplan.push_back(c);
}

// The block-table entry of a pair's splits [perm_base, perm_base + nb).
BlockPair block_pair(int64_t mrow0, int64_t mword0, uint64_t perm_base, int64_t nb, int owner,
                     const PairDesc& pd) {
    BlockPair b;
    memset(&b, 0, sizeof b);
    b.mrow0 = mrow0;
    b.mword0 = mword0;
    b.perm_base = (uint32_t)perm_base;
    b.nb = (int32_t)nb;
    b.owner = owner;
    b.n = pd.n;
    b.m = pd.m;
    b.Wp = pd.Wp;
    b.pair_index = pd.pair_index;
    b.ygap = pd.ygap;
    return b;
}

// Point-to-centroid tiles of pair p's first nb block rows: every 256-split
// tile times every 64-row tile of its padded rows.
void add_ctiles(Plan& P, int p, int64_t nb) {
    for (int64_t b = 0; b < nb; b += kTileB)
        for (int i0 = 0; i0 < P.pairs[p].Np; i0 += kCTileRows) P.ctiles.push_back(CTile{p, (int32_t)b, i0, 0});
}

// Single-pair plan with blocks of B0 splits.
Plan plan_single(const hbt_perm_params* prm, const void* X, const void* Y, int64_t* B0_out) {
    Plan P;
    add_pair(P, X, Y, prm->n, prm->m, prm->pair_index);
    finish_plan(P, prm->d, prm->precision, prm->input_dtype);
    int64_t B0 = prm->block_perms > 0 ? prm->block_perms : kAutoBlock;
    B0 = std::min<int64_t>(B0, prm->B);
    *B0_out = B0;
    P.bp.push_back(block_pair(0, 0, prm->perm_offset, B0, 0, P.pairs[0]));
    const int tb = groupsum_tile_splits(prm->precision);
    for (int64_t b = 0; b < B0; b += tb) P.tiles.push_back(GemmTile{0, (int32_t)b});
    P.groups.push_back(GemmGroup{0, (int32_t)((B0 + 255) / 256), 0});  // room for the narrower width
    P.ntile_total = (int64_t)P.groups[0].nbt * P.nslot;
    if (prm->stat_route == 1) {
        P.route2 = true;
        P.ntile_i = P.pairs[0].Np / 64;
        add_ctiles(P, 0, B0);
    }
    P.Btot.push_back(prm->B);
    P.block_rows = B0;
    P.block_mask_words = B0 * P.pairs[0].Wp;
    return P;
}

// 16-byte row loads apply: FP32 rows, d a multiple of 4, aligned bases.
bool vector_rows(const Plan& P) { return P.aligned16 && vector_rows_ok(P.input_dtype, P.d, P.d_pad); }

// Householder reflection of every pair and the precision's Z storage.  On the
// 16-byte-load path the column-sum pass has already stored the 32-row groups
// that hold only Y rows or padding, so the reflection covers the groups that
// hold X rows.
hipError_t reflect(const Plan& P, const Workspace& w, float* z32, hipStream_t s) {
    if (vector_rows(P))
        return launch_reflect_vec(P.precision, w.pairs, P.npairs, P.xoct, w.st, w.v, P.d, P.d_pad,
                                  w.coef, w.zstore, P.zrows * P.d_pad, z32, s);
    return launch_reflect(P.input_dtype, P.precision, w.pairs, P.npairs, P.zrows / 8, w.st, w.v, P.d,
                          P.d_pad, w.coef, w.zstore, P.zrows * P.d_pad, z32, s);
}

hbt_status enqueue_prologue(const Plan& P, const Workspace& w, int align, int gd, hbt_result* res,
                            hipStream_t s, bool upload_pairs = true) {
    if (upload_pairs) {
        StageTimer t(HBT_STAGE_OTHER, s);
        HIP_TRY(upload(w.pairs, P.pairs.data(), P.pairs.size() * sizeof(PairDesc), s));
    }
    StageTimer t(HBT_STAGE_ALIGN, s);
    if (vector_rows(P) && P.need_store)
        HIP_TRY(launch_colsum_store_vec(P.precision, w.pairs, P.npairs, (int)P.chunks.size(), P.d,
                                        P.d_pad, w.partial_sum, w.zstore, P.zrows * P.d_pad, w.z32,
                                        w.chunk_bad, s));
    else if (vector_rows(P))
        HIP_TRY(launch_colsum_vec(w.pairs, P.npairs, (int)P.chunks.size(), P.d, P.d_pad, w.partial_sum,
                                  w.chunk_bad, s));
    else
        HIP_TRY(launch_colsum(P.input_dtype, w.pairs, P.npairs, (int)P.chunks.size(), P.d,
                              w.partial_sum, w.chunk_bad, s));
    HIP_TRY(launch_finalize(w.pairs, P.npairs, w.partial_sum, w.chunk_bad, P.d, P.d_pad, align, gd, w.sxy, w.st,
                            w.v, w.t64, w.t32, w.cnt, res, s));
    return HBT_OK;
}

// A second stream per device for work that runs beside the caller's stream
// within one call (default priority, created on first use and kept), and the
// events that fork it from the caller's stream and join it back.  Both are
// stream-ordered, so a captured call records them as graph edges.
std::mutex g_side_mu;
hipStream_t g_side[2][64];

hipError_t side_stream(hipStream_t* out, int which = 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_side_mu);
    hipStream_t& q = g_side[which][dev];
    if (!q && (e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking)) != hipSuccess) return e;
    *out = q;
    return hipSuccess;
}

// Events of one call (created and destroyed by the call; their records and
// waits are stream-ordered, so a captured call records them as graph edges).
struct Events {
    std::vector<hipEvent_t> ev;
    ~Events() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    hipError_t record(hipStream_t s, hipEvent_t* out) {
        hipEvent_t e;
        hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r != hipSuccess) return r;
        ev.push_back(e);
        *out = e;
        return hipEventRecord(e, s);
    }
};

struct Fork {
    hipStream_t main, side = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    explicit Fork(hipStream_t s) : main(s) {}
    ~Fork() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    hipError_t begin() {
        hipError_t e;
        if ((e = side_stream(&side)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&a, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&b, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventRecord(a, main)) != hipSuccess) return e;
        return hipStreamWaitEvent(side, a, 0);
    }
    hipError_t join() {
        hipError_t e;
        if ((e = hipEventRecord(b, side)) != hipSuccess) return e;
        return hipStreamWaitEvent(main, b, 0);
    }
};

// Segment slots of the recheck: what the workspace holds, or fewer when the
// environment variable HBT_RECHECK_SLOTS asks for fewer (0: every flag is
// done whole by one work-group).  The results do not depend on it; it exists
// to exercise both ways of spreading the work.
int64_t recheck_slot_budget(int npairs, int d_pad) {
    const int64_t held = recheck_slots(npairs, d_pad);
    const char* e = getenv("HBT_RECHECK_SLOTS");
    if (!e || !*e) return held;
    char* end = nullptr;
    const long long v = strtoll(e, &end, 10);
    if (end == e || v < 0) return held;
    return v < held ? (int64_t)v : held;
}

// The stages after the group sums: statistic and counts, recheck, null
// moments, p-values.
hbt_status batched_epilogue(const Plan& P, const Workspace& w, const hbt_perm_params* common,
                            hbt_result* results, hipStream_t s) {
    const int np = P.npairs;
    const int no_recheck = common->flags & HBT_FLAG_NO_RECHECK;
    if (P.lazy) {
        // first pass: decide from the hi-plane sums what they can decide,
        // list the rest; second pass: split-BF16 sums of the listed splits
        { StageTimer t_(HBT_STAGE_STAT, s); HIP_TRY(launch_stat_lazy(false, w.pairs, w.bp, np, P.block_rows, w.st,
                          w.partial, P.nslot, P.block_rows, P.d, common->gd, common->alternative,
                          precision_band(HBT_BF16_LAZY, P.d, false), no_recheck, w.tw, w.cnt, w.flags, w.nflag,
                          w.rlist, w.rcnt, s)); }
        { StageTimer t_(HBT_STAGE_OTHER, s); HIP_TRY(launch_refine_tiles(w.groups, (int)P.groups.size(), w.rcnt,
                          P.d_pad, w.rgroups, w.rtiles, s)); }
        { StageTimer t_(HBT_STAGE_GROUPSUM, s); HIP_TRY(launch_groupsum_refine(w.pairs, w.bp, w.rgroups,
                          (int)P.groups.size(), w.rtiles, P.d_pad, w.zstore, P.zrows * P.d_pad, w.mask, w.t32,
                          w.partial, P.block_rows, w.rlist, w.rcnt, P.tune.grid_narrow, s)); }
        { StageTimer t_(HBT_STAGE_STAT, s); HIP_TRY(launch_stat_lazy(true, w.pairs, w.bp, np, P.block_rows, w.st,
                          w.partial, P.nslot, P.block_rows, P.d, common->gd, common->alternative,
                          precision_band(HBT_BF16X2, P.d, false), no_recheck, w.tw, w.cnt, w.flags, w.nflag,
                          w.rlist, w.rcnt, s)); }
    } else { StageTimer t_(HBT_STAGE_STAT, s); HIP_TRY(launch_stat(w.pairs, w.bp, np, P.block_rows, w.st,
                        P.route2 ? w.partial2 : w.partial, P.route2 ? 0 : P.nslot,
                        P.block_rows, P.d, common->gd,
                        common->alternative, precision_band(P.precision, P.d, P.route2), no_recheck, nullptr,
                        0, w.tw, w.cnt, w.flags, w.nflag, s, w.pv, w.mask, w.coef, w.fpart, P.fold_segs)); }
    if (!no_recheck) {
        StageTimer t_(HBT_STAGE_RECHECK, s);
        HIP_TRY(launch_recheck(P.input_dtype, w.pairs, w.bp, np, w.st, w.v, w.t64, w.coef, w.mask, w.flags,
                               w.nflag, w.rplan, P.block_rows, P.max_np, w.rseg, recheck_slot_budget(np, P.d_pad),
                               P.d, common->gd, common->alternative,
                               w.cnt, w.tw, s));
    }
    { StageTimer t_(HBT_STAGE_OTHER, s); HIP_TRY(launch_moments(np, w.bp, w.st, w.tw, w.cnt, s)); }
    { StageTimer t_(HBT_STAGE_OTHER, s); HIP_TRY(launch_final(np, w.bp, w.st, w.sstat, w.cnt, w.Btot, results, s)); }
    return HBT_OK;
}

// The batched call as a pipeline over chunks of pairs (Plan::cplan): the
// caller's stream aligns chunk k (column sums, finalize, reflection and
// storage), a second stream draws its splits, and a third runs its group-sum
// product once both are done, so that the product of chunk k overlaps the
// alignment and the splits of chunk k + 1.  Events order the streams (a
// captured call records them as graph edges); the streams join before the
// statistic.  Every stage computes what it does without the pipeline, so the
// results do not depend on the chunking.
hbt_status batched_pipelined(const Plan& P, const Workspace& w, const hbt_perm_params* common,
                             hbt_result* results, hipStream_t s) {
    const int np = P.npairs;
    hipStream_t qs, qg;  // splits, group sums
    HIP_TRY(side_stream(&qs, 0));
    HIP_TRY(side_stream(&qg, 1));
    Events ev;
    hipEvent_t e0;
    {
        StageTimer t_(HBT_STAGE_OTHER, s);
        HIP_TRY(upload(w.bp, P.bp.data(), P.bp.size() * sizeof(BlockPair), s));
    }
    HIP_TRY(ev.record(s, &e0));
    HIP_TRY(hipStreamWaitEvent(qs, e0, 0));
    {
        StageTimer t_(HBT_STAGE_SPLIT, qs);
        HIP_TRY(zero(w.sstat, (size_t)(np + 1) / 2 * 8, qs));
    }
    {
        StageTimer t_(HBT_STAGE_OTHER, s);
        HIP_TRY(upload(w.pairs, P.pairs.data(), P.pairs.size() * sizeof(PairDesc), s));
        HIP_TRY(upload(w.groups, P.groups.data(), P.groups.size() * sizeof(GemmGroup), s));
        HIP_TRY(upload(w.Btot, P.Btot.data(), P.Btot.size() * sizeof(int64_t), s));
        HIP_TRY(zero(w.nflag, (size_t)(np + 1) / 2 * 8, s));
        if (P.lazy) HIP_TRY(zero(w.rcnt, (size_t)(np + 1) / 2 * 8, s));
    }
    HIP_TRY(ev.record(s, &e0));
    HIP_TRY(hipStreamWaitEvent(qg, e0, 0));
    for (const Plan::Chunk& c : P.cplan) {
        const bool last = c.pb == np;
        const int64_t r0 = P.bp[c.pa].mrow0, r1 = last ? P.block_rows : P.bp[c.pb].mrow0;
        const int c0 = P.pairs[c.pa].cx0, c1 = P.pairs[c.pb - 1].cy1;
        const int64_t o0 = P.pairs[c.pa].xoct0, o1 = last ? P.xoct : P.pairs[c.pb].xoct0;
        hipEvent_t es, ea;
        {
            StageTimer t_(HBT_STAGE_SPLIT, qs);
            HIP_TRY(launch_split_masks(w.bp, np, r1, P.max_np, common->seed, w.mask, w.sstat,
                                       P.tune.split_cap, qs, r0));
        }
        HIP_TRY(ev.record(qs, &es));
        {
            StageTimer t_(HBT_STAGE_ALIGN, s);
            HIP_TRY(launch_colsum_store_vec(P.precision, w.pairs, np, c1 - c0, P.d, P.d_pad, w.partial_sum,
                                            w.zstore, P.zrows * P.d_pad, w.z32, w.chunk_bad, s, c0));
            HIP_TRY(launch_finalize(w.pairs, c.pb - c.pa, w.partial_sum, w.chunk_bad, P.d, P.d_pad,
                                    common->align, common->gd, w.sxy, w.st, w.v, w.t64, w.t32, w.cnt,
                                    results, s, c.pa));
            HIP_TRY(launch_reflect_vec(P.precision, w.pairs, np, o1, w.st, w.v, P.d, P.d_pad, w.coef,
                                       w.zstore, P.zrows * P.d_pad, nullptr, s, o0));
        }
        HIP_TRY(ev.record(s, &ea));
        HIP_TRY(hipStreamWaitEvent(qg, es, 0));
        HIP_TRY(hipStreamWaitEvent(qg, ea, 0));
        {
            StageTimer t_(HBT_STAGE_GROUPSUM, qg);
            HIP_TRY(launch_groupsum(P.precision, w.pairs, w.bp, w.tiles, 0, w.groups + c.g0, c.ngw,
                                    (int)c.ntw, c.ng256, (int)c.nt256, P.d_pad, w.zstore,
                                    P.zrows * P.d_pad, w.mask, w.t32, w.t64, w.partial, P.block_rows,
                                    nullptr, qg, P.tune.grid_wide, P.tune.grid_narrow, nullptr, nullptr, P.lazy));
        }
    }
    hipEvent_t ej;
    HIP_TRY(ev.record(qs, &ej));
    HIP_TRY(hipStreamWaitEvent(s, ej, 0));
    HIP_TRY(ev.record(qg, &ej));
    HIP_TRY(hipStreamWaitEvent(s, ej, 0));
    return batched_epilogue(P, w, common, results, s);
}

}  // namespace

extern "C" {

int32_t hbt_abi_version(void) { return HBT_ABI_VERSION; }

const char* hbt_status_string(int32_t status) {
    switch (status) {
        case HBT_OK: return "ok";
        case HBT_ERR_ARG: return "invalid argument";
        case HBT_ERR_SIZE: return "invalid size";
        case HBT_ERR_DTYPE: return "unsupported dtype";
        case HBT_ERR_WORKSPACE: return "workspace too small";
        case HBT_ERR_DEGENERATE: return "degenerate cloud (r outside (0,1))";
        case HBT_ERR_MASK: return "explicit mask row does not hold n items";
        case HBT_ERR_DEVICE: return "HIP error";
        case HBT_ERR_UNSUPPORTED: return "unsupported option";
        case HBT_ERR_INTERNAL: return "split selection bucket overflow";
        case HBT_ERR_NOT_UNIT: return "a row is not a unit vector (| |x| - 1 | > 1e-4)";
        default: return "unknown status";
    }
}

const char* hbt_last_error(void) { return g_err.c_str(); }

hbt_status hbt_stage_timing(int32_t enable) {
    std::vector<StageRecord> old;
    {
        std::lock_guard<std::mutex> g(g_timing_mu);
        g_timing = enable != 0;
        old.swap(g_records);
    }
    for (auto& r : old) {
        (void)hipEventSynchronize(r.stop);
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    return HBT_OK;
}

hbt_status hbt_stage_times(double* ms, int64_t* launches) {
    g_err.clear();
    if (!ms || !launches) return fail(HBT_ERR_ARG, "NULL output");
    std::vector<StageRecord> recs;
    {
        std::lock_guard<std::mutex> g(g_timing_mu);
        recs.swap(g_records);
    }
    for (int k = 0; k < HBT_NUM_STAGES; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    hbt_status st = HBT_OK;
    for (auto& r : recs) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
        if (e != hipSuccess && st == HBT_OK)
            st = fail(HBT_ERR_DEVICE, "stage timing: %s", hipGetErrorString(e));
        ms[r.stage] += t;
        launches[r.stage] += 1;
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    return st;
}

// ---------------------------------------------------------------------------
size_t hbt_align_workspace_size(int64_t n, int64_t m, int64_t d) {
    if (n < 2 || m < 2 || d < 1 || d > HBT_MAX_D || n + m > HBT_MAX_N) return 0;
    Plan P;
    P.need_store = false;
    add_pair(P, nullptr, nullptr, n, m, 0);
    finish_plan(P, d, HBT_F64, HBT_IN_F32);
    return carve(P, nullptr).bytes;
}

hbt_status hbt_align(int32_t input_dtype, const void* X, int64_t n, const void* Y, int64_t m,
                     int64_t d, int32_t align, int32_t gd, void* X_out, double* v_out,
                     hbt_result* result, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!X || !Y || !X_out || !result) return fail(HBT_ERR_ARG, "NULL X, Y, X_out or result");
    if (input_dtype != HBT_IN_F32 && input_dtype != HBT_IN_F64)
        return fail(HBT_ERR_DTYPE, "unknown input dtype %d", input_dtype);
    if (gd != HBT_GD_BANERJEE && gd != HBT_GD_IDENTITY) return fail(HBT_ERR_ARG, "unknown g_d %d", gd);
    if (align != 0 && align != 1) return fail(HBT_ERR_ARG, "align must be 0 or 1");
    hbt_status st = check_sizes(n, m, d, 1, 0);
    if (st) return st;
    Plan P;
    P.need_store = false;
    add_pair(P, X, Y, n, m, 0);
    finish_plan(P, d, HBT_F64, input_dtype);
    const size_t need = carve(P, nullptr).bytes;
    if (!ws || ws_bytes < need)
        return fail(HBT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    hipStream_t s = (hipStream_t)stream;
    Workspace w = carve(P, ws);
    st = enqueue_prologue(P, w, align, gd, result, s);
    if (st) return st;
    HIP_TRY(launch_reflect_out(input_dtype, w.pairs, w.st, w.v, (int)n, (int)d, X_out, v_out, s));
    return HBT_OK;
}

// ---------------------------------------------------------------------------
size_t hbt_perm_test_workspace_size(const hbt_perm_params* prm) {
    if (!prm || check_sizes(prm->n, prm->m, prm->d, prm->B, prm->perm_offset) ||
        prm->precision < HBT_F64 || prm->precision > HBT_BF16_LAZY) {
        return 0;
    }
    int64_t B0;
    Plan P = plan_single(prm, nullptr, nullptr, &B0);
    if (check_tiles(P)) return 0;
    return carve(P, nullptr).bytes;
}

hbt_status hbt_perm_test(const void* X, const void* Y, const hbt_perm_params* prm,
                         hbt_result* result, float* T_out, uint32_t* mask_out, void* ws,
                         size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!prm) return fail(HBT_ERR_ARG, "NULL params");
    if (!X || !Y || !result) return fail(HBT_ERR_ARG, "NULL X, Y or result");
    hbt_status st = check_sizes(prm->n, prm->m, prm->d, prm->B, prm->perm_offset);
    if (st) return st;
    if ((st = check_enums(prm))) return st;
    if (prm->block_perms < 0) return fail(HBT_ERR_ARG, "block_perms must be >= 0");
    int64_t B0;
    Plan P = plan_single(prm, X, Y, &B0);
    if ((st = check_tiles(P))) return st;
    const size_t need = carve(P, nullptr).bytes;
    if (!ws || ws_bytes < need)
        return fail(HBT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (!prm->masks && split_lds_per_block(P.max_np) > std::min<size_t>(split_lds_limit(), 65536))
        return fail(HBT_ERR_SIZE, "n + m too large for the split kernel's LDS");
    hipStream_t s = (hipStream_t)stream;
    Workspace w = carve(P, ws);
    const PairDesc& pd = P.pairs[0];
    const int N = (int)(prm->n + prm->m);
    const int W = (N + 31) / 32;

    const RecheckBand band = precision_band(P.precision, P.d, P.route2);
    const int no_recheck = prm->flags & HBT_FLAG_NO_RECHECK;
    const int t_mode = (prm->flags & HBT_FLAG_T_OUT_NORMS) ? 2 : (prm->flags & HBT_FLAG_T_OUT_F64) ? 1 : 0;
    const int64_t t_size = t_mode == 2 ? 24 : t_mode == 1 ? 8 : 4;
    // the tables of split block b0 (nb splits) and its tile width
    // One pair alone fills the GPU only with enough tiles: the narrow width
    // when the wide one would not give two tiles per CU (the width never
    // changes a result).
    auto block_width = [&](int64_t nb) {
        if (P.precision == HBT_I8X3) return kTileI8;
        const int w = choose_width(nb, P.tune);
        if (w == kTileWide && !g_force_width &&
            (nb + kTileWide - 1) / kTileWide * P.nslot < 2 * (int64_t)device_cus())
            return kTileNarrow;
        return w;
    };
    auto block_tables = [&](int64_t b0, int64_t nb) -> hipError_t {
        const BlockPair bq = block_pair(0, 0, prm->perm_offset + (uint64_t)b0, nb, 0, pd);
        const int wdt = block_width(nb);
        const GemmGroup grp{0, (int32_t)((nb + wdt - 1) / wdt), 0};
        hipError_t e;
        if ((e = upload(w.bp, &bq, sizeof bq, s)) != hipSuccess) return e;
        if ((e = upload(w.groups, &grp, sizeof grp, s)) != hipSuccess) return e;
        return zero(w.nflag, 8, s);
    };
    auto block_splits = [&](int64_t b0, int64_t nb, hipStream_t q) -> hipError_t {
        if (prm->masks) return launch_copy_masks(prm->masks, b0, nb, N, (int)prm->n, pd.Wp, w.mask, w.sstat, q);
        return launch_split_masks(w.bp, 1, nb, P.max_np, prm->seed, w.mask, w.sstat,
                                  P.tune.split_cap, q);
    };
    {
        // The plan tables and block 0's tables sit next to each other at the
        // start of the workspace (pairs, bp, tiles, groups, Btot): one image,
        // one upload.  The recheck counter and the split status are adjacent
        // too: one fill.
        StageTimer t_(HBT_STAGE_OTHER, s);
        const int64_t nb0 = std::min<int64_t>(B0, prm->B);
        const BlockPair bq = block_pair(0, 0, prm->perm_offset, nb0, 0, pd);
        const int wdt = block_width(nb0);
        const GemmGroup grp{0, (int32_t)((nb0 + wdt - 1) / wdt), 0};
        std::vector<unsigned char> img((size_t)((const char*)(w.Btot + 1) - (const char*)w.pairs), 0);
        auto put = [&](const void* dst, const void* src, size_t bytes) {
            memcpy(img.data() + ((const char*)dst - (const char*)w.pairs), src, bytes);
        };
        put(w.pairs, P.pairs.data(), sizeof(PairDesc));
        put(w.bp, &bq, sizeof bq);
        put(w.tiles, P.tiles.data(), P.tiles.size() * sizeof(GemmTile));
        put(w.groups, &grp, sizeof grp);
        put(w.Btot, P.Btot.data(), sizeof(int64_t));
        HIP_TRY(upload(w.pairs, img.data(), img.size(), s));
        HIP_TRY(zero(w.nflag, (size_t)((const char*)(w.sstat + 2) - (const char*)w.nflag), s));
    }
    // The first block's splits depend only on the seed and the sizes: they are
    // drawn on a second stream beside the alignment and joined before the
    // group sums (as in the batched call); later blocks follow in order.
    Fork fork(s);
    HIP_TRY(fork.begin());
    {
        StageTimer t_(HBT_STAGE_SPLIT, fork.side);
        HIP_TRY(block_splits(0, std::min<int64_t>(B0, prm->B), fork.side));
    }
    st = enqueue_prologue(P, w, prm->align, prm->gd, result, s, false);
    if (st) return st;
    const float* z32 = P.precision == HBT_F32 ? (const float*)w.zstore : w.z32;
    {
        StageTimer t_(HBT_STAGE_ALIGN, s);
        HIP_TRY(reflect(P, w, w.z32, s));
        if (P.route2) {
            HIP_TRY(upload(w.ctiles, P.ctiles.data(), P.ctiles.size() * sizeof(CTile), s));
            HIP_TRY(launch_row_dot_t(w.pairs, 1, z32, w.t64, P.d_pad, P.zrows, w.zt, s));
        }
    }
    HIP_TRY(fork.join());
    for (int64_t b0 = 0; b0 < prm->B; b0 += B0) {
        const int64_t nb = std::min<int64_t>(B0, prm->B - b0);
        const int wdt = block_width(nb);
        const GemmGroup grp{0, (int32_t)((nb + wdt - 1) / wdt), 0};
        if (b0 > 0) {
            {
                StageTimer t_(HBT_STAGE_OTHER, s);
                HIP_TRY(block_tables(b0, nb));
            }
            StageTimer t_(HBT_STAGE_SPLIT, s);
            HIP_TRY(block_splits(b0, nb, s));
        }
        const int ntiles = (int)((nb + groupsum_tile_splits(P.precision) - 1) / groupsum_tile_splits(P.precision));
        {
            StageTimer t_(HBT_STAGE_GROUPSUM, s);
            const int nt = grp.nbt * P.nslot;
            if (P.lazy) HIP_TRY(zero(w.rcnt, 8, s));  // the block's refinement list
            // the wide segment, or the other one (the narrow split-BF16 width, int8 planes)
            HIP_TRY(launch_groupsum(P.precision, w.pairs, w.bp, w.tiles, ntiles, w.groups, wdt == kTileWide,
                                    wdt == kTileWide ? nt : 0, wdt != kTileWide, wdt != kTileWide ? nt : 0, P.d_pad,
                                    w.zstore, P.zrows * P.d_pad, w.mask, w.t32, w.t64, w.partial,
                                    P.block_rows, w.sig, s, P.tune.grid_wide, P.tune.grid_narrow, nullptr, nullptr,
                                    P.lazy));
        }
        if (P.route2) {
            StageTimer t_(HBT_STAGE_CENTROID, s);
            HIP_TRY(launch_centroid(P.precision == HBT_BF16X2, w.pairs, w.bp, w.ctiles,
                                    (int)((nb + kTileB - 1) / kTileB) * (P.pairs[0].Np / kCTileRows), P.d_pad,
                                    z32, w.sig,
                                    w.mask, w.zt, w.partial2, P.block_rows, s));
        }
        void* T_blk = T_out ? (char*)T_out + b0 * t_size : nullptr;
        if (P.lazy) {
            // decide what the hi plane can, refine the rest with both planes
            { StageTimer t_(HBT_STAGE_STAT, s); HIP_TRY(launch_stat_lazy(false, w.pairs, w.bp, 1, nb, w.st,
                              w.partial, P.nslot, P.block_rows, P.d, prm->gd, prm->alternative,
                              precision_band(HBT_BF16_LAZY, P.d, false), no_recheck, w.tw, w.cnt, w.flags,
                              w.nflag, w.rlist, w.rcnt, s, T_blk, t_mode)); }
            { StageTimer t_(HBT_STAGE_OTHER, s); HIP_TRY(launch_refine_tiles(w.groups, 1, w.rcnt, P.d_pad,
                              w.rgroups, w.rtiles, s)); }
            { StageTimer t_(HBT_STAGE_GROUPSUM, s); HIP_TRY(launch_groupsum_refine(w.pairs, w.bp, w.rgroups, 1,
                              w.rtiles, P.d_pad, w.zstore, P.zrows * P.d_pad, w.mask, w.t32, w.partial,
                              P.block_rows, w.rlist, w.rcnt, P.tune.grid_narrow, s)); }
            { StageTimer t_(HBT_STAGE_STAT, s); HIP_TRY(launch_stat_lazy(true, w.pairs, w.bp, 1, nb, w.st,
                              w.partial, P.nslot, P.block_rows, P.d, prm->gd, prm->alternative,
                              precision_band(HBT_BF16X2, P.d, false), no_recheck, w.tw, w.cnt, w.flags,
                              w.nflag, w.rlist, w.rcnt, s, T_blk, t_mode)); }
        } else { StageTimer t_(HBT_STAGE_STAT, s); HIP_TRY(launch_stat(w.pairs, w.bp, 1, nb, w.st,
                            P.route2 ? w.partial2 : w.partial, P.route2 ? 0 : P.nslot,
                            P.block_rows, P.d, prm->gd,
                            prm->alternative, band, no_recheck, T_blk, t_mode, w.tw,
                            w.cnt, w.flags, w.nflag, s)); }
        if (!no_recheck) {
            StageTimer t_(HBT_STAGE_RECHECK, s);
            HIP_TRY(launch_recheck(P.input_dtype, w.pairs, w.bp, 1, w.st, w.v, w.t64, w.coef, w.mask,
                                   w.flags, w.nflag, w.rplan, nb, P.max_np, w.rseg, recheck_slot_budget(1, P.d_pad),
                                   P.d, prm->gd, prm->alternative, w.cnt, w.tw, s));
        }
        { StageTimer t_(HBT_STAGE_OTHER, s); HIP_TRY(launch_moments(1, w.bp, w.st, w.tw, w.cnt, s)); }
        if (mask_out)
            HIP_TRY(launch_export_masks(w.mask, nb, pd.Wp, W, mask_out + b0 * W, s));
    }
    { StageTimer t_(HBT_STAGE_OTHER, s); HIP_TRY(launch_final(1, w.bp, w.st, w.sstat, w.cnt, w.Btot, result, s)); }
    return HBT_OK;
}

// ---------------------------------------------------------------------------
// Pairs of shared clouds: every cloud is stored once, unreflected, in one run
// padded to kRowPad rows (its 32-row groups stored by the column-sum pass as
// they are summed); pair p pools cloud pair_x[p] (X) and cloud pair_y[p] (Y)
// as two runs, X's padding between them in the mask order.
static bool plan_clouds(Plan& P, int64_t nclouds, const void* Z_all, const int64_t* cloud_offset,
                        const int64_t* cloud_rows, int64_t npairs, const int64_t* pair_x,
                        const int64_t* pair_y, const int64_t* B, const uint32_t* pair_index, int64_t d,
                        const hbt_perm_params* common) {
    P.fold = true;
    for (int64_t c = 0; c < nclouds; ++c) {
        const char* base = Z_all ? (const char*)Z_all + (size_t)cloud_offset[c] * d * 4 : nullptr;
        P.aligned16 = P.aligned16 && ((uintptr_t)base % 16 == 0);
        PairDesc cd;
        memset(&cd, 0, sizeof cd);
        cd.X = base;
        cd.Y = base;
        cd.n = 0;
        cd.m = (int32_t)cloud_rows[c];
        cd.Np = (int32_t)round_up(cloud_rows[c], kRowPad);
        cd.Wp = cd.Np / 32;
        cd.zrow0 = P.zrows;
        cd.zrow_y = P.zrows;
        cd.nxc = cd.Np / kRowPad;
        cd.cx0 = cd.cx1 = cd.cy0 = (int32_t)P.chunks.size();
        for (int64_t j = 0; kSumChunkY * j < cd.Np; ++j)
            P.chunks.push_back(SumChunk{(int32_t)c, 1, (int32_t)(kSumChunkY * j),
                                        (int32_t)std::min<int64_t>(cd.m, kSumChunkY * (j + 1))});
        cd.cy1 = (int32_t)P.chunks.size();
        P.zrows += cd.Np;
        P.cdesc.push_back(cd);
    }
    int64_t rows = 0, words = 0;
    std::map<std::tuple<int64_t, int64_t, int64_t, uint32_t>, int> first;
    for (int64_t p = 0; p < npairs; ++p) {
        const PairDesc& cx = P.cdesc[(size_t)pair_x[p]];
        const PairDesc& cy = P.cdesc[(size_t)pair_y[p]];
        PairDesc pd;
        memset(&pd, 0, sizeof pd);
        pd.X = cx.X;
        pd.Y = cy.X;
        pd.n = cx.m;
        pd.m = cy.m;
        pd.Np = cx.Np + cy.Np;
        pd.Wp = pd.Np / 32;
        pd.zrow0 = cx.zrow0;
        pd.zrow_y = cy.zrow0;
        pd.nxc = cx.Np / kRowPad;
        pd.ygap = cx.Np - cx.m;
        pd.coef0 = P.ncoef;
        pd.pair_index = pair_index ? pair_index[p] : common->pair_index + (uint32_t)p;
        pd.flip = pd.m < pd.n ? 1 : 0;
        pd.cx0 = cx.cx1;
        pd.cx1 = cx.cy1;
        pd.cy0 = cy.cx1;
        pd.cy1 = cy.cy1;
        P.ncoef += pd.n;
        P.max_np = std::max(P.max_np, (int)pd.Np);
        P.fold_segs = std::max(P.fold_segs, fold_segments(pd.n));
        P.pairs.push_back(pd);
        const auto key = std::make_tuple((int64_t)pd.n, (int64_t)pd.m, B[p], pd.pair_index);
        const auto hit = first.find(key);
        if (hit == first.end()) {
            first.emplace(key, (int)p);
            P.bp.push_back(block_pair(rows, words, common->perm_offset, B[p], (int)p, pd));
            words += B[p] * pd.Wp;
        } else {
            const BlockPair& o = P.bp[(size_t)hit->second];
            P.bp.push_back(block_pair(rows, o.mword0, common->perm_offset, B[p], hit->second, pd));
        }
        P.Btot.push_back(B[p]);
        rows += B[p];
    }
    P.npairs = (int)npairs;
    finish_plan(P, d, common->precision, common->input_dtype);
    std::vector<int> order((size_t)npairs);
    for (int64_t p = 0; p < npairs; ++p) order[(size_t)p] = (int)p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P.pairs[a].Np > P.pairs[b].Np; });
    add_groups(P, order, B, 0, (int)npairs);
    P.block_rows = rows;
    P.block_mask_words = words;
    return true;
}

// Number of pipeline chunks of a batched call (1 = no pipeline).
int g_pipeline_chunks = 0;  // process-wide override (hbt_pipeline_chunks); 0: the tuned value
int pipeline_chunks(const Plan& P, int64_t npairs) {
    if (!(P.precision == HBT_BF16X2 || P.precision == HBT_I8X3 || P.precision == HBT_BF16_E4M3) || !vector_rows(P) ||
        !P.need_store || P.route2)
        return 1;
    const int c = g_pipeline_chunks > 0 ? g_pipeline_chunks : P.tune.chunks;
    return (int)std::max<int64_t>(1, std::min<int64_t>(c, npairs));
}

static bool plan_batched(Plan& P, int64_t npairs, const void* Z_all, const int64_t* row_offset,
                         const int64_t* n, const int64_t* m, const int64_t* B,
                         const uint32_t* pair_index, int64_t d, const hbt_perm_params* common) {
    const size_t es = common->input_dtype == HBT_IN_F64 ? 8 : 4;
    int64_t rows = 0, words = 0;
    // Pairs with equal n, m, B and pair index get identical splits (the
    // counters and the key are the same): the first of them draws the masks
    // and the others read its mask words.
    std::map<std::tuple<int64_t, int64_t, int64_t, uint32_t>, int> first;
    for (int64_t p = 0; p < npairs; ++p) {
        const char* X = Z_all ? (const char*)Z_all + (size_t)row_offset[p] * d * es : nullptr;
        const char* Y = X ? X + (size_t)n[p] * d * es : nullptr;
        const uint32_t idx = pair_index ? pair_index[p] : common->pair_index + (uint32_t)p;
        add_pair(P, X, Y, n[p], m[p], idx);
        const auto key = std::make_tuple(n[p], m[p], B[p], idx);
        const auto hit = first.find(key);
        if (hit == first.end()) {
            first.emplace(key, (int)p);
            P.bp.push_back(block_pair(rows, words, common->perm_offset, B[p], (int)p, P.pairs.back()));
            words += B[p] * P.pairs.back().Wp;
        } else {
            const BlockPair& o = P.bp[(size_t)hit->second];
            P.bp.push_back(block_pair(rows, o.mword0, common->perm_offset, B[p], hit->second, P.pairs.back()));
        }
        P.Btot.push_back(B[p]);
        rows += B[p];
    }
    finish_plan(P, d, common->precision, common->input_dtype);
    // tiles, largest pooled size first (longest-processing-time order)
    auto by_size = [&](int pa, int pb) {
        std::vector<int> order;
        for (int p = pa; p < pb; ++p) order.push_back(p);
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return P.pairs[a].Np > P.pairs[b].Np; });
        return order;
    };
    const std::vector<int> order = by_size(0, (int)npairs);
    // the tile list of the FP32 / FP64 products (the others use the groups)
    const int tb = groupsum_tile_splits(P.precision);
    if (P.precision == HBT_F32 || P.precision == HBT_F64)
        for (int p : order)
            for (int64_t b = 0; b < B[p]; b += tb) P.tiles.push_back(GemmTile{p, (int32_t)b});
    // Pipeline chunks: consecutive pair ranges of about equal product work
    // (B N), so that the product of one chunk runs while the next chunk is
    // aligned and split.  Only for the persistent product kernels on the
    // 16-byte-load path; otherwise one chunk.
    const int nchunk = pipeline_chunks(P, npairs);
    if (nchunk <= 1) {
        add_groups(P, order, B, 0, (int)npairs);
    } else {
        double total = 0.0;
        for (int64_t p = 0; p < npairs; ++p) total += (double)B[p] * P.pairs[p].Np;
        double acc = 0.0;
        int pa = 0;
        for (int64_t p = 0; p < npairs; ++p) {
            acc += (double)B[p] * P.pairs[p].Np;
            const int k = (int)P.cplan.size();
            if (p + 1 == npairs || (acc >= total * (k + 1) / nchunk && k + 1 < nchunk)) {
                add_groups(P, by_size(pa, (int)p + 1), B, pa, (int)p + 1);
                pa = (int)p + 1;
            }
        }
    }
    if (common->stat_route == 1) {
        P.route2 = true;
        P.ntile_i = P.max_np / 64;
        for (int64_t p = 0; p < npairs; ++p) add_ctiles(P, (int)p, B[p]);
    }
    P.block_rows = rows;
    P.block_mask_words = words;
    return true;
}

size_t hbt_perm_test_batched_workspace_size(int64_t npairs, const int64_t* n, const int64_t* m,
                                            const int64_t* B, int64_t d,
                                            const hbt_perm_params* common) {
    if (npairs < 1 || !n || !m || !B || !common) return 0;
    if (common->precision < HBT_F64 || common->precision > HBT_BF16_LAZY) return 0;
    for (int64_t p = 0; p < npairs; ++p)
        if (check_sizes(n[p], m[p], d, B[p], common->perm_offset)) return 0;
    std::vector<int64_t> off((size_t)npairs + 1, 0);
    Plan P;
    plan_batched(P, npairs, nullptr, off.data(), n, m, B, nullptr, d, common);
    if (check_tiles(P)) return 0;
    return carve(P, nullptr).bytes;
}

hbt_status hbt_perm_test_batched(int64_t npairs, const void* Z_all, const int64_t* row_offset,
                                 const int64_t* n, const int64_t* m, const int64_t* B,
                                 const uint32_t* pair_index, int64_t d,
                                 const hbt_perm_params* common, hbt_result* results, void* ws,
                                 size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!common || !Z_all || !row_offset || !n || !m || !B || !results)
        return fail(HBT_ERR_ARG, "NULL argument");
    if (npairs < 1 || npairs > (1 << 24)) return fail(HBT_ERR_SIZE, "npairs = %lld", (long long)npairs);
    hbt_status st = check_enums(common);
    if (st) return st;
    int64_t total_rows = 0;
    for (int64_t p = 0; p < npairs; ++p) {
        if ((st = check_sizes(n[p], m[p], d, B[p], common->perm_offset)))
            return fail(st, "pair %lld: %s", (long long)p, g_err.c_str());
        if (row_offset[p] < 0) return fail(HBT_ERR_ARG, "pair %lld: negative row offset", (long long)p);
        total_rows += B[p];
    }
    if (total_rows >= (int64_t)1 << 32) return fail(HBT_ERR_SIZE, "too many splits in one call");
    Plan P;
    plan_batched(P, npairs, Z_all, row_offset, n, m, B, pair_index, d, common);
    if ((st = check_tiles(P))) return st;
    const size_t need = carve(P, nullptr).bytes;
    if (!ws || ws_bytes < need)
        return fail(HBT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (split_lds_per_block(P.max_np) > std::min<size_t>(split_lds_limit(), 65536))
        return fail(HBT_ERR_SIZE, "n + m too large for the split kernel's LDS");
    hipStream_t s = (hipStream_t)stream;
    Workspace w = carve(P, ws);
    const int np = P.npairs;
    if (P.cplan.size() > 1) return batched_pipelined(P, w, common, results, s);
    // Three streams until the group sums: the caller's uploads the pair table
    // and aligns; a second one uploads the block table (all the split stage
    // reads) and draws the splits, which depend only on the seeds and the
    // group sizes (integer VALU work beside HBM-bound work); a third uploads
    // the tables only the later stages read.  The table uploads are chains of
    // small kernels (a few microseconds each), so no chain waits for another.
    // At most 6 split work-groups per CU (the default split_cap) leave
    // wave slots to the alignment kernels (measured on 512 pairs, d = 768,
    // split BF16: 8.03 ms per call at 8 or uncapped, where the alignment
    // then waits for wave slots; 7.25 ms at 6, the two stages 2.1 ms each;
    // 7.56 ms at 5, 7.63 ms at 4).
    hipStream_t qs, qt;
    HIP_TRY(side_stream(&qs, 0));
    HIP_TRY(side_stream(&qt, 1));
    Events ev;
    hipEvent_t e0;
    HIP_TRY(ev.record(s, &e0));
    HIP_TRY(hipStreamWaitEvent(qs, e0, 0));
    HIP_TRY(hipStreamWaitEvent(qt, e0, 0));
    {
        StageTimer t_(HBT_STAGE_SPLIT, qs);
        HIP_TRY(upload(w.bp, P.bp.data(), P.bp.size() * sizeof(BlockPair), qs));
        HIP_TRY(zero(w.sstat, (size_t)(np + 1) / 2 * 8, qs));
        HIP_TRY(launch_split_masks(w.bp, np, P.block_rows, P.max_np, common->seed, w.mask, w.sstat,
                                   P.tune.split_cap, qs));
    }
    {
        StageTimer t_(HBT_STAGE_OTHER, qt);
        if (P.precision == HBT_BF16X2 || P.precision == HBT_I8X3 || P.precision == HBT_BF16_E4M3)
            HIP_TRY(upload(w.groups, P.groups.data(), P.groups.size() * sizeof(GemmGroup), qt));
        else
            HIP_TRY(upload(w.tiles, P.tiles.data(), P.tiles.size() * sizeof(GemmTile), qt));
        HIP_TRY(upload(w.Btot, P.Btot.data(), P.Btot.size() * sizeof(int64_t), qt));
        HIP_TRY(zero(w.nflag, (size_t)(np + 1) / 2 * 8, qt));
        if (P.lazy) HIP_TRY(zero(w.rcnt, (size_t)(np + 1) / 2 * 8, qt));
        if (P.route2) HIP_TRY(upload(w.ctiles, P.ctiles.data(), P.ctiles.size() * sizeof(CTile), qt));
    }
    {
        StageTimer t_(HBT_STAGE_OTHER, s);
        HIP_TRY(upload(w.pairs, P.pairs.data(), P.pairs.size() * sizeof(PairDesc), s));
    }
    st = enqueue_prologue(P, w, common->align, common->gd, results, s, false);
    if (st) return st;
    {
        StageTimer t_(HBT_STAGE_ALIGN, s);
        HIP_TRY(reflect(P, w, P.route2 ? w.z32 : nullptr, s));
    }
    HIP_TRY(ev.record(qs, &e0));
    HIP_TRY(hipStreamWaitEvent(s, e0, 0));
    HIP_TRY(ev.record(qt, &e0));
    HIP_TRY(hipStreamWaitEvent(s, e0, 0));
    {
        StageTimer t_(HBT_STAGE_GROUPSUM, s);
        HIP_TRY(launch_groupsum(P.precision, w.pairs, w.bp, w.tiles, (int)P.tiles.size(), w.groups,
                                P.ngw, (int)P.ntw, P.ng256, (int)P.nt256, P.d_pad, w.zstore,
                                P.zrows * P.d_pad, w.mask, w.t32, w.t64, w.partial, P.block_rows,
                                P.route2 ? w.sig : nullptr, s, P.tune.grid_wide, P.tune.grid_narrow, nullptr,
                                nullptr, P.lazy));
    }
    if (P.route2) {
        StageTimer t_(HBT_STAGE_CENTROID, s);
        const float* z32 = P.precision == HBT_F32 ? (const float*)w.zstore : w.z32;
        HIP_TRY(launch_row_dot_t(w.pairs, np, z32, w.t64, P.d_pad, P.zrows, w.zt, s));
        HIP_TRY(launch_centroid(P.precision == HBT_BF16X2, w.pairs, w.bp, w.ctiles, (int)P.ctiles.size(),
                                P.d_pad, z32, w.sig, w.mask, w.zt, w.partial2, P.block_rows, s));
    }
    return batched_epilogue(P, w, common, results, s);
}


// ---------------------------------------------------------------------------
// permutation-budget allocator
// ---------------------------------------------------------------------------
hbt_status hbt_budget_features(int64_t npairs, const hbt_result* results, int64_t d, int32_t gd,
                               float* features, void* stream) {
    g_err.clear();
    if (!results || !features) return fail(HBT_ERR_ARG, "NULL pointer");
    if (gd != HBT_GD_BANERJEE && gd != HBT_GD_IDENTITY) return fail(HBT_ERR_ARG, "unknown g_d %d", gd);
    if (npairs < 1) return fail(HBT_ERR_SIZE, "npairs = %lld", (long long)npairs);
    if (d < 1 || d > HBT_MAX_D) return fail(HBT_ERR_SIZE, "d = %lld", (long long)d);
    HIP_TRY(launch_features(npairs, results, (int)d, gd, features, (hipStream_t)stream));
    return HBT_OK;
}

hbt_status hbt_null_targets(int64_t npairs, const hbt_result* results, float* targets, void* stream) {
    g_err.clear();
    if (!results || !targets) return fail(HBT_ERR_ARG, "NULL pointer");
    if (npairs < 1) return fail(HBT_ERR_SIZE, "npairs = %lld", (long long)npairs);
    HIP_TRY(launch_null_targets(npairs, results, targets, (hipStream_t)stream));
    return HBT_OK;
}

hbt_status hbt_feature_norm(int64_t rows, const float* features, float* theta, void* stream) {
    g_err.clear();
    if (!features || !theta) return fail(HBT_ERR_ARG, "NULL pointer");
    if (rows < 1) return fail(HBT_ERR_SIZE, "rows = %lld", (long long)rows);
    HIP_TRY(launch_feature_norm(rows, features, theta, (hipStream_t)stream));
    return HBT_OK;
}

hbt_status hbt_target_norm(int64_t rows, const float* targets, float* theta, void* stream) {
    g_err.clear();
    if (!targets || !theta) return fail(HBT_ERR_ARG, "NULL pointer");
    if (rows < 1) return fail(HBT_ERR_SIZE, "rows = %lld", (long long)rows);
    HIP_TRY(launch_target_norm(rows, targets, theta, (hipStream_t)stream));
    return HBT_OK;
}

hbt_status hbt_mlp_forward(int64_t rows, const float* features, const float* theta, float* out,
                           void* stream) {
    g_err.clear();
    if (!features || !theta || !out) return fail(HBT_ERR_ARG, "NULL pointer");
    if (rows < 1 || rows > ((int64_t)1 << 31) - 256) return fail(HBT_ERR_SIZE, "rows = %lld", (long long)rows);
    HIP_TRY(launch_mlp_forward(rows, features, theta, out, (hipStream_t)stream));
    return HBT_OK;
}

size_t hbt_mlp_grad_workspace_size(int64_t rows) {
    return rows < 1 ? 0 : mlp_train_ws_bytes(rows);
}

hbt_status hbt_mlp_grad(int64_t rows, const float* features, const float* targets,
                        const float* theta, float* grad, double* loss, void* ws, size_t ws_bytes,
                        void* stream) {
    g_err.clear();
    if (!features || !targets || !theta || !grad) return fail(HBT_ERR_ARG, "NULL pointer");
    if (rows < 1 || rows > ((int64_t)1 << 31) - 256) return fail(HBT_ERR_SIZE, "rows = %lld", (long long)rows);
    if (!ws || ws_bytes < mlp_train_ws_bytes(rows))
        return fail(HBT_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, mlp_train_ws_bytes(rows));
    HIP_TRY(launch_mlp_grad(rows, features, targets, theta, grad, loss, ws, (hipStream_t)stream));
    return HBT_OK;
}

hbt_status hbt_mlp_adam(float* theta, const float* grad, float* adam_m, float* adam_v, int64_t step,
                        float lr, float beta1, float beta2, float eps, void* stream) {
    g_err.clear();
    if (!theta || !grad || !adam_m || !adam_v) return fail(HBT_ERR_ARG, "NULL pointer");
    if (step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps >= 0.0f))
        return fail(HBT_ERR_ARG, "bad Adam settings (step %lld, lr %g, betas %g %g, eps %g)",
                    (long long)step, lr, beta1, beta2, eps);
    const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
    HIP_TRY(launch_adam(theta, grad, adam_m, adam_v, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream));
    return HBT_OK;
}

hbt_status hbt_budgets(int64_t npairs, const float* mlp_out, const hbt_result* results,
                       double p_lo, double p_hi, int64_t b_min, int64_t b_max, double zq,
                       int64_t* budgets, void* stream) {
    g_err.clear();
    if (!mlp_out || !results || !budgets) return fail(HBT_ERR_ARG, "NULL pointer");
    if (!(p_lo >= 0.0 && p_lo <= p_hi && p_hi <= 1.0) || !(zq > 0.0))
        return fail(HBT_ERR_ARG, "band [%g, %g], zq %g", p_lo, p_hi, zq);
    if (npairs < 1 || b_min < 1 || b_max < b_min)
        return fail(HBT_ERR_SIZE, "npairs %lld, budgets [%lld, %lld]", (long long)npairs,
                    (long long)b_min, (long long)b_max);
    HIP_TRY(launch_budgets(npairs, mlp_out, results, p_lo, p_hi, b_min, b_max, zq, budgets,
                           (hipStream_t)stream));
    return HBT_OK;
}

hbt_status hbt_budgets_min_cost(int64_t npairs, const float* mlp_out, const hbt_result* results,
                                double p_lo, double p_hi, int64_t b_min, int64_t b_max, int64_t* budgets,
                                void* stream) {
    g_err.clear();
    if (!mlp_out || !results || !budgets) return fail(HBT_ERR_ARG, "NULL pointer");
    if (!(p_lo >= 0.0 && p_lo <= p_hi && p_hi <= 1.0)) return fail(HBT_ERR_ARG, "band [%g, %g]", p_lo, p_hi);
    if (npairs < 1 || b_min < 1 || b_max < b_min)
        return fail(HBT_ERR_SIZE, "npairs %lld, budgets [%lld, %lld]", (long long)npairs,
                    (long long)b_min, (long long)b_max);
    HIP_TRY(launch_budgets_cost(npairs, mlp_out, results, p_lo, p_hi, b_min, b_max, budgets,
                                (hipStream_t)stream));
    return HBT_OK;
}

// ---------------------------------------------------------------------------
// tile widths of the split-BF16 product
// ---------------------------------------------------------------------------
hbt_status hbt_tile_widths(int64_t npairs, const int64_t* B, int64_t d, int32_t* widths) {
    g_err.clear();
    if (!B || !widths) return fail(HBT_ERR_ARG, "NULL pointer");
    if (npairs < 1 || d < 1 || d > HBT_MAX_D) return fail(HBT_ERR_SIZE, "npairs %lld, d %lld", (long long)npairs, (long long)d);
    const TileCost tc = tile_cost((int)round_up(d, kDPad), HBT_BF16X2);
    for (int64_t p = 0; p < npairs; ++p) {
        if (B[p] < 1) return fail(HBT_ERR_SIZE, "B[%lld] = %lld", (long long)p, (long long)B[p]);
        widths[p] = choose_width(B[p], tc);
    }
    return HBT_OK;
}

// The checks of the shared-clouds call that need no device memory.
static hbt_status check_clouds(int64_t nclouds, const int64_t* cloud_rows, int64_t npairs,
                               const int64_t* pair_x, const int64_t* pair_y, const int64_t* B, int64_t d,
                               const hbt_perm_params* common) {
    if (!common || !cloud_rows || !pair_x || !pair_y || !B) return fail(HBT_ERR_ARG, "NULL argument");
    if (nclouds < 1 || nclouds > (1 << 24) || npairs < 1 || npairs > (1 << 24))
        return fail(HBT_ERR_SIZE, "nclouds %lld, npairs %lld", (long long)nclouds, (long long)npairs);
    hbt_status st = check_enums(common);
    if (st) return st;
    if (common->precision != HBT_BF16X2 || common->input_dtype != HBT_IN_F32 || common->stat_route != 0)
        return fail(HBT_ERR_UNSUPPORTED, "shared clouds: split BF16 from FP32 rows, statistic route 0");
    if (d < 1 || d > 1024 || d % 4)
        return fail(HBT_ERR_UNSUPPORTED, "shared clouds: d a multiple of 4 up to 1024 (got %lld)", (long long)d);
    for (int64_t c = 0; c < nclouds; ++c)
        if (cloud_rows[c] < 2 || cloud_rows[c] > HBT_MAX_N)
            return fail(HBT_ERR_SIZE, "cloud %lld has %lld rows", (long long)c, (long long)cloud_rows[c]);
    int64_t total = 0;
    for (int64_t p = 0; p < npairs; ++p) {
        if (pair_x[p] < 0 || pair_x[p] >= nclouds || pair_y[p] < 0 || pair_y[p] >= nclouds)
            return fail(HBT_ERR_ARG, "pair %lld: cloud index out of range", (long long)p);
        const int64_t n = cloud_rows[pair_x[p]], m = cloud_rows[pair_y[p]];
        if (round_up(n, kRowPad) + round_up(m, kRowPad) > HBT_MAX_N + kRowPad)
            return fail(HBT_ERR_SIZE, "pair %lld: n + m too large", (long long)p);
        if ((st = check_sizes(n, m, d, B[p], common->perm_offset)))
            return fail(st, "pair %lld: %s", (long long)p, g_err.c_str());
        total += B[p];
    }
    if (total >= (int64_t)1 << 32) return fail(HBT_ERR_SIZE, "too many splits in one call");
    return HBT_OK;
}

size_t hbt_perm_test_clouds_workspace_size(int64_t nclouds, const int64_t* cloud_rows, int64_t npairs,
                                           const int64_t* pair_x, const int64_t* pair_y, const int64_t* B,
                                           int64_t d, const hbt_perm_params* common) {
    if (check_clouds(nclouds, cloud_rows, npairs, pair_x, pair_y, B, d, common)) return 0;
    std::vector<int64_t> off((size_t)nclouds, 0);
    Plan P;
    plan_clouds(P, nclouds, nullptr, off.data(), cloud_rows, npairs, pair_x, pair_y, B, nullptr, d, common);
    if (check_tiles(P)) return 0;
    return carve(P, nullptr).bytes;
}

hbt_status hbt_perm_test_clouds(int64_t nclouds, const void* Z_all, const int64_t* cloud_offset,
                                const int64_t* cloud_rows, int64_t npairs, const int64_t* pair_x,
                                const int64_t* pair_y, const int64_t* B, const uint32_t* pair_index, int64_t d,
                                const hbt_perm_params* common, hbt_result* results, void* ws, size_t ws_bytes,
                                void* stream) {
    g_err.clear();
    if (!Z_all || !cloud_offset || !results) return fail(HBT_ERR_ARG, "NULL argument");
    hbt_status st = check_clouds(nclouds, cloud_rows, npairs, pair_x, pair_y, B, d, common);
    if (st) return st;
    for (int64_t c = 0; c < nclouds; ++c)
        if (cloud_offset[c] < 0) return fail(HBT_ERR_ARG, "cloud %lld: negative row offset", (long long)c);
    Plan P;
    plan_clouds(P, nclouds, Z_all, cloud_offset, cloud_rows, npairs, pair_x, pair_y, B, pair_index, d, common);
    if (!vector_rows(P)) return fail(HBT_ERR_UNSUPPORTED, "shared clouds: every cloud must start on 16 bytes");
    if ((st = check_tiles(P))) return st;
    const size_t need = carve(P, nullptr).bytes;
    if (!ws || ws_bytes < need)
        return fail(HBT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (split_lds_per_block(P.max_np) > std::min<size_t>(split_lds_limit(), 65536))
        return fail(HBT_ERR_SIZE, "n + m too large for the split kernel's LDS");
    hipStream_t s = (hipStream_t)stream;
    Workspace w = carve(P, ws);
    const int np = P.npairs;
    hipStream_t qs, qt;
    HIP_TRY(side_stream(&qs, 0));
    HIP_TRY(side_stream(&qt, 1));
    Events ev;
    hipEvent_t e0;
    HIP_TRY(ev.record(s, &e0));
    HIP_TRY(hipStreamWaitEvent(qs, e0, 0));
    HIP_TRY(hipStreamWaitEvent(qt, e0, 0));
    {
        StageTimer t_(HBT_STAGE_SPLIT, qs);
        HIP_TRY(upload(w.bp, P.bp.data(), P.bp.size() * sizeof(BlockPair), qs));
        HIP_TRY(zero(w.sstat, (size_t)(np + 1) / 2 * 8, qs));
        HIP_TRY(launch_split_masks(w.bp, np, P.block_rows, P.max_np, common->seed, w.mask, w.sstat,
                                   P.tune.split_cap, qs));
    }
    {
        StageTimer t_(HBT_STAGE_OTHER, qt);
        HIP_TRY(upload(w.groups, P.groups.data(), P.groups.size() * sizeof(GemmGroup), qt));
        HIP_TRY(upload(w.Btot, P.Btot.data(), P.Btot.size() * sizeof(int64_t), qt));
        HIP_TRY(zero(w.nflag, (size_t)(np + 1) / 2 * 8, qt));
    }
    {
        StageTimer t_(HBT_STAGE_OTHER, s);
        HIP_TRY(upload(w.cdesc, P.cdesc.data(), P.cdesc.size() * sizeof(PairDesc), s));
        HIP_TRY(upload(w.pairs, P.pairs.data(), P.pairs.size() * sizeof(PairDesc), s));
    }
    {
        // every cloud summed and stored once; per pair the directions, v, T_obs
        // and the reflected total; then the pairs' coefficients 2 (v . x_i) / (v . v)
        StageTimer t_(HBT_STAGE_ALIGN, s);
        HIP_TRY(launch_colsum_store_vec(P.precision, w.cdesc, (int)P.cdesc.size(), (int)P.chunks.size(), P.d,
                                        P.d_pad, w.partial_sum, w.zstore, P.zrows * P.d_pad, nullptr,
                                        w.chunk_bad, s));
        HIP_TRY(launch_finalize(w.pairs, np, w.partial_sum, w.chunk_bad, P.d, P.d_pad, common->align, common->gd,
                                w.sxy, w.st, w.v, w.t64, w.t32, w.cnt, results, s, 0, w.v32));
        HIP_TRY(launch_fold_coef(w.pairs, np, w.st, w.v, P.d, P.d_pad, P.ncoef, w.coef, s));
    }
    HIP_TRY(ev.record(qs, &e0));
    HIP_TRY(hipStreamWaitEvent(s, e0, 0));
    HIP_TRY(ev.record(qt, &e0));
    HIP_TRY(hipStreamWaitEvent(s, e0, 0));
    {
        StageTimer t_(HBT_STAGE_GROUPSUM, s);
        HIP_TRY(launch_groupsum(P.precision, w.pairs, w.bp, w.tiles, 0, w.groups, P.ngw, (int)P.ntw, P.ng256,
                                (int)P.nt256, P.d_pad, w.zstore, P.zrows * P.d_pad, w.mask, w.t32, w.t64,
                                w.partial, P.block_rows, nullptr, s, P.tune.grid_wide, P.tune.grid_narrow,
                                w.v32, w.pv));
    }
    return batched_epilogue(P, w, common, results, s);
}

hbt_status hbt_pipeline_chunks(int32_t chunks, int32_t* previous) {
    g_err.clear();
    if (chunks < 0 || chunks > 64) return fail(HBT_ERR_ARG, "chunks = %d (0 ... 64)", chunks);
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (previous) *previous = g_pipeline_chunks;
    g_pipeline_chunks = chunks;
    return HBT_OK;
}

hbt_status hbt_recheck_band(int32_t precision, int32_t stat_route, int32_t gd, int64_t n, int64_t m,
                            int64_t d, double r1, double r2, double* eps) {
    g_err.clear();
    if (!eps) return fail(HBT_ERR_ARG, "NULL pointer");
    if (precision < HBT_F64 || precision > HBT_BF16_LAZY) return fail(HBT_ERR_ARG, "unknown precision %d", precision);
    if (stat_route != 0 && stat_route != 1) return fail(HBT_ERR_ARG, "unknown stat_route %d", stat_route);
    if (gd != HBT_GD_BANERJEE && gd != HBT_GD_IDENTITY) return fail(HBT_ERR_ARG, "unknown g_d %d", gd);
    if (n < 1 || m < 1 || d < 1 || d > HBT_MAX_D)
        return fail(HBT_ERR_SIZE, "n %lld, m %lld, d %lld", (long long)n, (long long)m, (long long)d);
    *eps = recheck_eps(precision_band(precision, (int)d, stat_route == 1), (double)n, (double)m,
                       (double)d, r1, r2, gd);
    return HBT_OK;
}

hbt_status hbt_tune_get(int64_t d, double* costs, int32_t* tuned) {
    g_err.clear();
    if (!costs) return fail(HBT_ERR_ARG, "NULL pointer");
    if (d < 1 || d > HBT_MAX_D) return fail(HBT_ERR_SIZE, "d = %lld", (long long)d);
    const TileCost tc = tile_cost((int)round_up(d, kDPad), HBT_BF16X2);
    costs[0] = tc.c[0];
    costs[1] = tc.c[1];
    if (tuned) *tuned = tc.tuned ? 1 : 0;
    return HBT_OK;
}

hbt_status hbt_tune_set(int64_t d, const double* costs) {
    g_err.clear();
    if (!costs) return fail(HBT_ERR_ARG, "NULL pointer");
    if (d < 1 || d > HBT_MAX_D) return fail(HBT_ERR_SIZE, "d = %lld", (long long)d);
    if (!(costs[0] > 0.0) || !(costs[1] > 0.0)) return fail(HBT_ERR_ARG, "costs must be positive");
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache_once_locked();
    const std::pair<int, int> key{HBT_BF16X2, (int)round_up(d, kDPad)};
    auto it = g_tune.find(key);
    TileCost t = it != g_tune.end() ? it->second : default_tune(HBT_BF16X2);
    t.c[0] = costs[0];
    t.c[1] = costs[1];
    t.tuned = true;
    g_tune[key] = t;
    return HBT_OK;
}

hbt_status hbt_tune_entry_get(int32_t precision, int64_t d, hbt_tune_entry* e) {
    g_err.clear();
    if (!e) return fail(HBT_ERR_ARG, "NULL pointer");
    if (precision == HBT_BF16_LAZY)
        return fail(HBT_ERR_ARG, "the lazy split-BF16 precision uses the split-BF16 entry (HBT_BF16X2)");
    if (precision < HBT_F64 || precision > HBT_BF16_E4M3) return fail(HBT_ERR_ARG, "unknown precision %d", precision);
    if (d < 1 || d > HBT_MAX_D) return fail(HBT_ERR_SIZE, "d = %lld", (long long)d);
    const TileCost t = tile_cost((int)round_up(d, kDPad), precision);
    memset(e, 0, sizeof *e);
    e->cost[0] = t.c[0];
    e->cost[1] = t.c[1];
    e->grid_wide = t.grid_wide;
    e->grid_narrow = t.grid_narrow;
    e->split_cap = t.split_cap;
    e->chunks = t.chunks;
    e->tuned = t.tuned ? 1 : 0;
    return HBT_OK;
}

hbt_status hbt_tune_entry_set(int32_t precision, int64_t d, const hbt_tune_entry* e) {
    g_err.clear();
    if (!e) return fail(HBT_ERR_ARG, "NULL pointer");
    if (precision == HBT_BF16_LAZY)
        return fail(HBT_ERR_ARG, "the lazy split-BF16 precision uses the split-BF16 entry (HBT_BF16X2)");
    if (precision < HBT_F64 || precision > HBT_BF16_E4M3) return fail(HBT_ERR_ARG, "unknown precision %d", precision);
    if (d < 1 || d > HBT_MAX_D) return fail(HBT_ERR_SIZE, "d = %lld", (long long)d);
    const TileCost t{{e->cost[0], e->cost[1]}, e->grid_wide, e->grid_narrow, e->split_cap, e->chunks, true};
    if (!tune_valid(t))
        return fail(HBT_ERR_ARG, "costs must be positive, grids in [1, 256], split_cap in [1, 16], chunks in [1, 64]");
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache_once_locked();
    g_tune[{precision, (int)round_up(d, kDPad)}] = t;
    return HBT_OK;
}

hbt_status hbt_tune_save(const char* path) {
    g_err.clear();
    if (!path) return fail(HBT_ERR_ARG, "NULL path");
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache_once_locked();
    if (tune_save_locked(path) != 0) return fail(HBT_ERR_ARG, "cannot write %s", path);
    return HBT_OK;
}

hbt_status hbt_tune_load(const char* path) {
    g_err.clear();
    if (!path) return fail(HBT_ERR_ARG, "NULL path");
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache_once_locked();
    if (tune_load_locked(path) < 0) return fail(HBT_ERR_ARG, "cannot read %s or it is malformed", path);
    return HBT_OK;
}

hbt_status hbt_tune_batched(int64_t npairs, const void* Z_all, const int64_t* row_offset,
                            const int64_t* n, const int64_t* m, const int64_t* B,
                            const uint32_t* pair_index, int64_t d, const hbt_perm_params* common,
                            hbt_result* results, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!common || !B || !n || !m) return fail(HBT_ERR_ARG, "NULL argument");
    const int prec = common->precision;
    if (prec != HBT_BF16X2 && prec != HBT_I8X3 && prec != HBT_BF16_E4M3)
        return fail(HBT_ERR_ARG, "tuning covers the split-BF16, BF16 + e4m3 and int8-plane products only");
    if (npairs < 1 || d < 1 || d > HBT_MAX_D) return fail(HBT_ERR_SIZE, "npairs %lld, d %lld", (long long)npairs, (long long)d);
    const int d_pad = (int)round_up(d, kDPad);
    hipStream_t s = (hipStream_t)stream;
    TileCost best = tile_cost(d_pad, prec);
    auto install = [&](const TileCost& t) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[{prec, d_pad}] = t;
    };
    auto call = [&]() {
        return hbt_perm_test_batched(npairs, Z_all, row_offset, n, m, B, pair_index, d, common, results, ws,
                                     ws_bytes, stream);
    };
    // one measured call: the product's time (stage events) and the whole call's
    auto measure = [&](double* product_ms, double* call_ms) -> hbt_status {
        hbt_status st = hbt_stage_timing(1);
        if (st) return st;
        hipEvent_t a, b;
        HIP_TRY(hipEventCreate(&a));
        HIP_TRY(hipEventCreate(&b));
        HIP_TRY(hipEventRecord(a, s));
        st = call();
        HIP_TRY(hipEventRecord(b, s));
        double ms[HBT_NUM_STAGES];
        int64_t launches[HBT_NUM_STAGES];
        const hbt_status st2 = hbt_stage_times(ms, launches);
        hbt_stage_timing(0);
        HIP_TRY(hipEventSynchronize(b));
        float total = 0.0f;
        HIP_TRY(hipEventElapsedTime(&total, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (st) return st;
        if (st2) return st2;
        if (!(ms[HBT_STAGE_GROUPSUM] > 0.0)) return fail(HBT_ERR_DEVICE, "no timing of the product");
        *product_ms = ms[HBT_STAGE_GROUPSUM];
        *call_ms = total;
        return HBT_OK;
    };
    // every candidate twice, keeping the faster call (the first call of a
    // setting may pay first-touch or clock ramp-up)
    auto best_of_two = [&](const TileCost& t, double* product_ms, double* call_ms) -> hbt_status {
        install(t);
        double p0, c0, p1, c1;
        hbt_status st = measure(&p0, &c0);
        if (!st) st = measure(&p1, &c1);
        if (st) return st;
        *product_ms = std::min(p0, p1);
        *call_ms = std::min(c0, c1);
        return HBT_OK;
    };
    const int saved_chunks = g_pipeline_chunks;
    g_pipeline_chunks = 0;
    hbt_status st = HBT_OK;
    // 1. tile widths (split BF16, BF16 + e4m3): per-split costs of each width
    // with every pair forced to it
    const bool widths_tuned = prec == HBT_BF16X2 || prec == HBT_BF16_E4M3;
    if (widths_tuned) {
        const int widths[2] = {kTileWide, 256};
        for (int k = 0; k < 2 && !st; ++k) {
            double units = 0.0;  // padded splits times pooled rows
            for (int64_t p = 0; p < npairs; ++p)
                units += (double)round_up(B[p], widths[k]) * (double)round_up(n[p] + m[p], kRowPad);
            g_force_width = widths[k];
            double pm, cm;
            st = best_of_two(best, &pm, &cm);
            g_force_width = 0;
            if (!st) best.c[k] = pm / units;
        }
    }
    // 2. persistent grids of the product launches this workload uses
    {
        double pm, cm;
        if (!st) st = best_of_two(best, &pm, &cm);
        double best_ms = pm;
        const int wide[] = {4, 8, 16, 32};
        const int narrow[] = {8, 16, 32, 64};
        bool any_wide = false, any_narrow = prec == HBT_I8X3;
        for (int64_t p = 0; p < npairs && widths_tuned; ++p) {
            const int w = choose_width(B[p], best);
            any_wide |= w == kTileWide;
            any_narrow |= w != kTileWide;
        }
        for (int g : wide) {
            if (st || !any_wide) break;
            TileCost t = best;
            t.grid_wide = g;
            st = best_of_two(t, &pm, &cm);
            if (!st && pm < best_ms) { best_ms = pm; best = t; }
        }
        for (int g : narrow) {
            if (st || !any_narrow) break;
            TileCost t = best;
            t.grid_narrow = g;
            st = best_of_two(t, &pm, &cm);
            if (!st && pm < best_ms) { best_ms = pm; best = t; }
        }
    }
    // 3. split work-groups per CU beside the alignment, then 4. pipeline
    // chunks: whole-call time
    {
        double pm, cm;
        if (!st) st = best_of_two(best, &pm, &cm);
        double best_call = cm;
        for (int c : {4, 5, 6, 8}) {
            if (st) break;
            TileCost t = best;
            t.split_cap = c;
            st = best_of_two(t, &pm, &cm);
            if (!st && cm < best_call) { best_call = cm; best = t; }
        }
        for (int k : {1, 2, 4}) {
            if (st) break;
            TileCost t = best;
            t.chunks = k;
            st = best_of_two(t, &pm, &cm);
            if (!st && cm < best_call) { best_call = cm; best = t; }
        }
    }
    g_pipeline_chunks = saved_chunks;
    if (st) return st;
    best.tuned = true;
    install(best);
    // a last call with the chosen parameters leaves its results in `results`
    st = call();
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(s));
    const char* path = getenv("HBT_TUNE_CACHE");
    if (path && *path) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        if (tune_save_locked(path) != 0) return fail(HBT_ERR_ARG, "cannot write the tuning cache %s", path);
    }
    return HBT_OK;
}

// hbt_perm_test on the library's own scratch.  The scratch address of each
// device is looked up once, with that device current, and kept.
hbt_status hbt_perm_test_static(const void* X, const void* Y, const hbt_perm_params* prm,
                                hbt_result* result, float* T_out, uint32_t* mask_out, void* stream) {
    static std::mutex mu;
    static void* ptr[64] = {};
    g_err.clear();
    if (!prm) return fail(HBT_ERR_ARG, "NULL params");
    if (!X || !Y || !result) return fail(HBT_ERR_ARG, "NULL X, Y or result");
    hbt_status st = check_sizes(prm->n, prm->m, prm->d, prm->B, prm->perm_offset);
    if (st) return st;
    if ((st = check_enums(prm))) return st;
    const size_t need = hbt_perm_test_workspace_size(prm);
    if (need > (size_t)HBT_STATIC_SCRATCH_BYTES)
        return fail(HBT_ERR_WORKSPACE,
                    "this test needs %zu bytes of scratch; the static scratch holds %zu "
                    "(use hbt_perm_test with a caller workspace)",
                    need, (size_t)HBT_STATIC_SCRATCH_BYTES);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(HBT_ERR_DEVICE, "device %d out of range", dev);
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> g(mu);
        if (!ptr[dev]) HIP_TRY(hipGetSymbolAddress(&ptr[dev], HIP_SYMBOL(scratch)));
        ws = ptr[dev];
    }
    return hbt_perm_test(X, Y, prm, result, T_out, mask_out, ws, (size_t)HBT_STATIC_SCRATCH_BYTES,
                         stream);
}

}  // extern "C"
