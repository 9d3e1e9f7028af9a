// Host side of the C ABI: argument validation, context and scratch, the
// entropy key table, and the orchestration of the per-level kernels.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "fic_internal.h"

namespace fic {

struct Timer {
    struct Rec {
        int kind, slot;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;
    int open = -1;
};

// Captured encodes.  A graph bakes in every pointer of its encode (caller
// buffers, scratch slots, its own copy of the level tables), so it is keyed by
// the exact arguments and dropped whenever a scratch slot is reallocated.
struct GraphEntry {
    std::vector<uint8_t> key;
    hipGraphExec_t exec = nullptr;
    void *tables = nullptr;   // device copy of the level tables the graph reads
    uint64_t last_use = 0;
};

struct GraphCache {
    int max = 0;
    uint64_t tick = 0;
    hipStream_t cap = nullptr;   // capture stream (the legacy stream cannot be captured)
    std::vector<GraphEntry> e;
};

static void free_graph(GraphEntry &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.tables) (void)hipFree(g.tables);
    g.exec = nullptr;
    g.tables = nullptr;
}

void drop_graphs(GraphCache *gc) {
    if (!gc) return;
    for (auto &g : gc->e) free_graph(g);
    gc->e.clear();
}

// ---------------------------------------------------------------- fixed decoder scratch
// The second image of fic_decode_noalloc's double buffer.  Every GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  On the host the array's name is only a stand-in: host code uses
// the per-device address that hipGetSymbolAddress returned, never the name.
static __device__ __align__(256) uint8_t scratch[FIC_DECODE_NOALLOC_MAX_PIXELS];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Takes the array's address on `device` (which must be current) once per
// device; fic_ctx_create calls it.
static int scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return FIC_OK;   // the entry point then refuses this device
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return FIC_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return FIC_E_HIP;
    g_scratch_ptr[device] = ptr;
    return FIC_OK;
}

static void *scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace fic

using namespace fic;
using std::max;
using std::min;

namespace {

// ---------------------------------------------------------------- entropy table
// Natural logarithms of primes to ~100 bits with double-double arithmetic:
// ln p = e ln 2 + 2 atanh(z), z = (m - 1)/(m + 1) for p = 2^e m, m in [1, 2).
struct dd { double hi, lo; };

dd two_sum(double a, double b) {
    const double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
dd quick_two_sum(double a, double b) {
    const double s = a + b;
    return {s, b - (s - a)};
}
dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    const dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
dd dd_mul(dd a, dd b) {
    const double p = a.hi * b.hi;
    const double e = fma(a.hi, b.hi, -p) + (a.hi * b.lo + a.lo * b.hi);
    return quick_two_sum(p, e);
}
dd dd_div_d(dd a, double b) {  // a / b, b an exact double
    const double q1 = a.hi / b;
    const double p = q1 * b, pe = fma(q1, b, -p);
    const dd r = dd_add(a, dd{-p, -pe});
    const double q2 = r.hi / b;
    return quick_two_sum(q1, q2);
}
dd dd_atanh2(double num, double den) {  // 2 atanh(num/den) for 0 <= num/den <= 1/3
    const dd z = dd_div_d(dd{num, 0.0}, den);
    const dd z2 = dd_mul(z, z);
    dd term = z, sum = {0.0, 0.0};
    for (int i = 0; i < 60; ++i) {
        sum = dd_add(sum, dd_div_d(term, 2.0 * i + 1.0));
        term = dd_mul(term, z2);
        if (fabs(term.hi) < 1e-40) break;
    }
    return dd_add(sum, sum);
}
int64_t round_scaled(dd v) {  // round-half-even(v * 2^32)
    const double hi = ldexp(v.hi, 32), lo = ldexp(v.lo, 32);
    double r = nearbyint(hi);
    const double f = (hi - r) + lo;
    if (f > 0.5) r += 1.0;
    else if (f < -0.5) r -= 1.0;
    return (int64_t)r;
}

int64_t g_table[kTableSize];
bool g_table_ready = false;

void build_table() {
    if (g_table_ready) return;
    const dd ln2 = dd_atanh2(1.0, 3.0);
    static int64_t lam[kTableSize];
    static bool composite[kTableSize];
    memset(lam, 0, sizeof(lam));
    memset(composite, 0, sizeof(composite));
    for (int p = 2; p < kTableSize; ++p) {
        if (composite[p]) continue;
        for (int m = p * p; m < kTableSize; m += p) composite[m] = true;
        int e = 0;
        double m = p;
        while (m >= 2.0) {
            m *= 0.5;
            ++e;
        }
        dd l = dd_atanh2(m - 1.0, m + 1.0);
        l = dd_add(l, dd_mul(ln2, dd{(double)e, 0.0}));
        lam[p] = round_scaled(l);
    }
    g_table[0] = g_table[1] = 0;
    for (int q = 2; q < kTableSize; ++q) {
        int rest = q;
        int64_t acc = 0;
        for (int p = 2; rest > 1; ++p)
            while (rest % p == 0) {
                rest /= p;
                acc += lam[p];
            }
        g_table[q] = (int64_t)q * acc;
    }
    g_table_ready = true;
}

// ---------------------------------------------------------------- validation
bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

bool engine_ok(int e) { return e >= FIC_ENGINE_MFMA && e <= FIC_ENGINE_MFMA_F16_16X16; }

// The engine that searches a level of block size B: the matrix engine
// measured fastest per block size for MFMA (f16 32x32 tiles at B = 2 and 4,
// where it needs no replicated operands; f16 16x16 tiles at B = 8; int8 hi/lo
// planes at B = 16 and 32, where f32 accumulation of f16 products would no
// longer be exact above B = 16), FP32 where the requested matrix engine has
// no form.
int engine_for(int engine, int B) {
    if (engine == FIC_ENGINE_MFMA)
        return (B == 2 || B == 4) ? E_F16 : B == 8 ? E_H16 : mfma_supported(B) ? E_I8 : E_FP32;
    if (engine == FIC_ENGINE_MFMA_I8) return mfma_supported(B) ? E_I8 : E_FP32;
    if (engine == FIC_ENGINE_MFMA_F16) return f16_supported(B) ? E_F16 : E_FP32;
    if (engine == FIC_ENGINE_MFMA_F16_16X16) return B <= 16 ? E_H16 : E_FP32;
    return E_FP32;
}

// floor(log2 v) for v in 1..32: the slot of block size v
int log2i(int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v && l < 5) ++l;
    return l;
}

int check_sset(const int32_t *num, int count, int den) {
    if (!num || count < 1 || count > kMaxS || den < 1 || den > 1024) return FIC_E_INVALID;
    for (int k = 0; k < count; ++k) {
        if (num[k] < 0 || num[k] > den) return FIC_E_INVALID;
        if (k > 0 && num[k] <= num[k - 1]) return FIC_E_INVALID;
    }
    return FIC_OK;
}

int check_rms(fic_ratio r) { return (r.num < 0 || r.num > 65535 || r.den < 1 || r.den > 16) ? FIC_E_INVALID : FIC_OK; }

int check_pct(fic_ratio p) { return (p.den < 1 || p.num < 0 || p.num >= p.den) ? FIC_E_INVALID : FIC_OK; }

bool image_ok(const fic_image *img, int B) {
    return img && img->pix && img->width >= 2 * B && img->height >= 2 * B && img->width <= 65535 &&
           img->height <= 65535 && (int64_t)img->width * img->height <= (1 << 28) && img->pitch >= img->width;
}

int64_t n_candidates(int W, int H, int B, int L) {
    return (int64_t)((W - 2 * B) / L + 1) * ((H - 2 * B) / L + 1);
}

SSet make_sset(const int32_t *num, int count, int den) {
    SSet s;
    memset(&s, 0, sizeof(s));
    s.count = count;
    s.den = den;
    for (int k = 0; k < count; ++k) s.num[k] = num[k];
    return s;
}


#define FIC_TRY(expr)                              \
    do {                                           \
        const hipError_t e_ = (expr);              \
        if (e_ != hipSuccess) return hip_status(e_); \
    } while (0)

// ---------------------------------------------------------------- batched level plans
size_t al(size_t v) { return (v + 255) / 256 * 256; }

long cdiv(long a, long b) { return (a + b - 1) / b; }

// One image's share of one level: what the caller hands over.
struct ImgIn {
    const fic_image *img;
    int B, L, pct_num, pct_den, pool_max;
    fic_pool *pool;
    const uint32_t *rxy;
    const int32_t *nr;
    int range_cap;
    fic_level_codes *codes;     // NULL for a pool-only plan
    uint32_t *children;
    int32_t *nchildren;
    int pool_expect;            // > 0: the pool size to plan chunks for (else from the candidates)
};

struct LevelPlan {
    std::vector<ImgLvl> h;
    std::vector<int> pre;       // K_NUM x (n + 1)
    size_t slot_bytes[S_NUM_SLOTS];
    size_t table_off;           // offset of this plan's tables in S_TABLES
    BatchHost bh;
};

// Fills geometry, block counts and scratch offsets (as byte offsets cast to
// pointers; bind() rebases them once the slots are allocated).
// build_integ: this plan computes the images' summed-area tables (every plan
// of one encode lays them out identically, so later levels reuse them).
// Returns false when a launch of the batch would need 2^31 or more workgroups.
bool plan_level(LevelPlan &pl, const std::vector<ImgIn> &in, bool do_search, int engine, int level0,
                bool build_integ, int pool_key, const int8_t (*tune)[6]) {
    bool fits = true;
    const int n = (int)in.size();
    pl.h.assign(n, ImgLvl());
    pl.pre.assign((size_t)K_NUM * (n + 1), 0);
    memset(pl.slot_bytes, 0, sizeof(pl.slot_bytes));
    memset(&pl.bh, 0, sizeof(pl.bh));
    const int B = in[0].B;
    const int KS = B * B / 16;
    const int eng = do_search ? engine_for(engine, B) : E_FP32;
    pl.bh.B = B;
    pl.bh.eng = eng;
    const int form = form_of_engine(eng);
    if (form >= 0) pl.bh.shape = pick_shape(form, B, tune ? tune[form][log2i(B)] : -1);
    pl.bh.pool_key = pool_key;
    pl.bh.L = in[0].L;
    pl.bh.KS = KS;
    size_t off[S_NUM_SLOTS] = {0};
    // entropy-key strip length, one per level: strips of candidate rows as long
    // as possible (sliding windows reuse work) while the whole batch still
    // gives ~1024 waves
    long strip_rows = 0;
    for (const ImgIn &x : in) {
        const int nx = (x.img->width - 2 * x.B) / x.L + 1, ny = (x.img->height - 2 * x.B) / x.L + 1;
        strip_rows += (long)cdiv(nx, 64) * ny;
    }
    const int strip = (int)max(1L, min(16L, strip_rows / 1024));
    pl.bh.fused_sel = 1;
    for (const ImgIn &x : in)
        if (n_candidates(x.img->width, x.img->height, x.B, x.L) > kFusedSelMax) pl.bh.fused_sel = 0;
    for (int i = 0; i < n; ++i) {
        const ImgIn &x = in[i];
        ImgLvl &d = pl.h[i];
        memset(&d, 0, sizeof(d));
        d.pix = x.img->pix;
        d.W = x.img->width;
        d.H = x.img->height;
        d.pitch = x.img->pitch;
        d.B = x.B;
        d.L = x.L;
        d.nx = (d.W - 2 * d.B) / d.L + 1;
        d.ny = (d.H - 2 * d.B) / d.L + 1;
        d.nd = d.nx * d.ny;
        d.c = ((long long)x.pct_num * d.nd + x.pct_den - 1) / x.pct_den;
        d.pool_max = x.pool_max;
        d.pool_cap = x.pool->capacity;
        d.range_cap = x.range_cap;
        d.pcount = x.pool->count;
        d.pxy = x.pool->xy;
        d.pkey = x.pool->key;
        d.psum4 = x.pool->sum4;
        d.pa = x.pool->a;
        d.rxy = x.rxy;
        d.nr = x.nr;
        if (x.codes) {
            d.ccount = x.codes->count;
            d.cxy = x.codes->xy;
            d.csplit = x.codes->split;
            d.cdom = x.codes->domain;
            d.ciso = x.codes->iso;
            d.csidx = x.codes->s_idx;
            d.coff = x.codes->offset;
            d.cerr = x.codes->err;
        }
        d.children = x.children;
        d.nchildren = x.nchildren;
        d.eng = eng;
        pl.bh.any_cap |= x.pool_max > 0;
        // block counts
        long blk[K_NUM] = {0};
        if (level0) blk[K_LEVEL0] = cdiv((long)(d.W / d.B) * (d.H / d.B), 256);
        // entropy: one wave per strip of candidate rows, the strip as long as
        // possible (sliding windows reuse work) while still giving ~1024 waves;
        // variance: one thread per candidate
        d.strip = strip;
        blk[K_KEYS] = pool_key == FIC_POOL_VARIANCE ? cdiv(d.nd, 256) : cdiv(d.nx, 64) * cdiv(d.ny, d.strip);
        blk[K_HIST] = max(1, min(256, cdiv(d.nd, 256)));
        blk[K_PCMP] = cdiv(d.nd, kScanBlock);
        blk[K_MOM] = cdiv(d.pool_cap, 256);
        if (build_integ) {
            blk[K_IROW] = cdiv(d.H + 1, 4);
            blk[K_ICOL] = cdiv(integ_col_items(d.W, d.H), 256);
            blk[K_ICSCAN] = cdiv(integ_scan_items(d.W, d.H), 256);
        }
        // pool scratch
        auto take = [&](Slot s, size_t bytes) {
            const size_t o = off[s];
            off[s] += al(bytes);
            return o;
        };
        d.integ = (uint32_t *)take(S_INTEG, sizeof(uint32_t) * integ_words(d.W, d.H));
        d.itmp = (uint32_t *)take(S_ITMP, sizeof(uint32_t) * (size_t)integ_col_items(d.W, d.H));
        d.keys = (int64_t *)take(S_KEYS, sizeof(int64_t) * (size_t)d.nd);
        d.sel = (PoolSel *)take(S_SEL, sizeof(PoolSel));
        d.pblocksum = (int *)take(S_PBLOCK, sizeof(int) * (size_t)(blk[K_PCMP] + 1));
        d.pblockoff = (int *)take(S_PBLOCK, sizeof(int) * (size_t)(blk[K_PCMP] + 1));
        if (do_search) {
            const int n2 = d.B * d.B;
            blk[K_RANGE] = cdiv(d.range_cap, 256);
            blk[K_FINAL] = cdiv(d.range_cap, 4);
            blk[K_CCMP] = cdiv(d.range_cap, kScanBlock);
            d.ri = (RInfo *)take(S_RINFO, sizeof(RInfo) * (size_t)(d.range_cap + 1));
            d.sidx = (int32_t *)take(S_RINFO, sizeof(int32_t) * (size_t)(d.range_cap + 1));
            d.cblocksum = (int *)take(S_CBLOCK, sizeof(int) * (size_t)(blk[K_CCMP] + 1));
            d.cblockoff = (int *)take(S_CBLOCK, sizeof(int) * (size_t)(blk[K_CCMP] + 1));
            if (eng != E_FP32) {
                // int8: A fragments per quad and half; f16: per quad (32 rows)
                const bool f16 = eng == E_F16;
                // chunks are counted for the pool size the percentile and the cap
                // leave (the capacity may hold every candidate); the kernels split
                // the actual pool evenly over them
                long long pexp = x.pool_expect > 0 ? x.pool_expect : d.nd - d.c;
                if (d.pool_max > 0) pexp = min(pexp, (long long)d.pool_max);
                pexp = max(1LL, min(pexp, (long long)d.pool_cap));
                d.geo = f16 ? f16_geometry(d.B, d.range_cap, (int)pexp, pl.bh.shape)
                            : mfma_geometry(d.B, d.range_cap, (int)pexp, pl.bh.shape);
                const int nquads = d.geo.nrg * (d.geo.rpw / 4);
                const int tile = f16 ? kDomTile32 : kDomTile;
                // a search stage may read up to a stage past a chunk's end: the
                // operands carry that many zero tiles
                const int ntiles = f16 ? f16_tiles(d.pool_cap) : mfma_tiles(d.pool_cap);
                // ... and a chunk is addressed with 32-bit offsets
                if (((long)cdiv(ntiles, d.geo.nchunk) + kF16PadTiles) * d.geo.kt * 1024 >= (1L << 31)) fits = false;
                const long afr = (long)nquads * (f16 ? 1 : 2) * d.geo.ka;   // 1 KiB fragments
                blk[K_AFRAG] = cdiv(afr * 64, 256);
                // int8 planes: one thread writes both planes of a K-step
                blk[K_BFRAG] = cdiv((long)ntiles * (d.geo.pl == 2 ? d.geo.ka : d.geo.kt) * 64, 256);
                blk[K_SEARCH] = cdiv(d.geo.nwg, 8) * 8;  // image blocks start at multiples of 8
                d.nslot = d.geo.nslot;
                d.afrag = (uint4 *)take(S_AFRAG, (size_t)afr * 1024);
                // the f16 form at B <= 4 keeps a second, exact copy of the tiles
                d.bfrag = (uint4 *)take(S_BFRAG, (size_t)ntiles * d.geo.kt * 1024 * (f16 && d.B <= 4 ? 2 : 1));
                // f16: Sd4 and sqrt(A), then the exact (A, Sd4); int8: the first two
                d.dinfo = (float2 *)take(S_DINFO, (size_t)ntiles * tile * sizeof(float2) * (f16 ? 2 : 1));
            } else {
                fp32_geometry(d.B, d.range_cap, d.pool_cap, &d.fnchunk, &d.ftpc);
                d.rpad = fp32_rpad(d.range_cap);
                d.ppad = fp32_ppad(d.pool_cap);
                blk[K_VIEWS] = cdiv((long)n2 * d.rpad, 256);
                blk[K_DOMS] = cdiv((long)n2 * d.ppad, 256);
                blk[K_SEARCH] = fp32_blocks(d.B, d.range_cap, d.pool_cap);
                d.nslot = d.fnchunk;
                d.vf = (float *)take(S_VF32, (size_t)n2 * d.rpad * 8 * sizeof(float));
                d.df = (float *)take(S_DF32, (size_t)n2 * d.ppad * sizeof(float));
                d.dinfo = (float2 *)take(S_DINFO, (size_t)d.ppad * sizeof(float2));
            }
            d.part = (Partial *)take(S_PARTIAL, sizeof(Partial) * (size_t)d.range_cap * d.nslot);
        }
        for (int k = 0; k < K_NUM; ++k) {
            const long v = (long)pl.pre[(size_t)k * (n + 1) + i] + blk[k];
            if (v > INT32_MAX) fits = false;
            pl.pre[(size_t)k * (n + 1) + i + 1] = (int)std::min(v, (long)INT32_MAX);
        }
    }
    for (int k = 0; k < K_NUM; ++k) pl.bh.blocks[k] = pl.pre[(size_t)k * (n + 1) + n];
    if (do_search && eng != E_FP32) off[S_QUEUE] = al(sizeof(int) * queue_ints(n));
    for (int s = 0; s < S_NUM_SLOTS; ++s) pl.slot_bytes[s] = off[s];
    pl.bh.dev.n = n;
    return fits;
}

size_t table_bytes(const LevelPlan &pl) {
    return al(sizeof(ImgLvl) * pl.h.size()) + al(sizeof(int) * pl.pre.size());
}

// Rebase the scratch offsets onto the allocated slots and point the device
// table at its place in S_TABLES.
template <class T>
void rebase(fic_ctx *ctx, T *&p, Slot s) {
    p = (T *)((char *)ctx->slot[s].ptr + (size_t)p);
}

void bind(fic_ctx *ctx, LevelPlan &pl, void *tables = nullptr) {
    auto rb = [&](auto &p, Slot s) { rebase(ctx, p, s); };
    for (auto &d : pl.h) {
        rb(d.integ, S_INTEG);
        rb(d.itmp, S_ITMP);
        rb(d.keys, S_KEYS);
        rb(d.sel, S_SEL);
        rb(d.pblocksum, S_PBLOCK);
        rb(d.pblockoff, S_PBLOCK);
        if (d.nslot > 0) {  // planned with a search
            rb(d.ri, S_RINFO);
            rb(d.sidx, S_RINFO);
            d.ns = d.sidx + d.range_cap;
            rb(d.cblocksum, S_CBLOCK);
            rb(d.cblockoff, S_CBLOCK);
            rb(d.part, S_PARTIAL);
            rb(d.dinfo, S_DINFO);
            if (d.eng != E_FP32) {
                rb(d.afrag, S_AFRAG);
                rb(d.bfrag, S_BFRAG);
            } else {
                rb(d.vf, S_VF32);
                rb(d.df, S_DF32);
            }
        } else {
            d.ri = nullptr;
            d.sidx = d.ns = nullptr;
        }
    }
    char *base = (char *)(tables ? tables : ctx->slot[S_TABLES].ptr) + pl.table_off;
    pl.bh.dev.queue = pl.slot_bytes[S_QUEUE] ? (int *)ctx->slot[S_QUEUE].ptr : nullptr;
    pl.bh.dev.d = (const ImgLvl *)base;
    pl.bh.dev.pre = (const int *)(base + al(sizeof(ImgLvl) * pl.h.size()));
}

// Copies every plan's tables to S_TABLES with one async copy from pinned
// memory; the staging buffer is reused once the previous copy has finished.
int upload(fic_ctx *ctx, std::vector<LevelPlan> &plans, hipStream_t st, void *tables = nullptr) {
    size_t total = 0;
    for (auto &pl : plans) total += table_bytes(pl);
    if (ctx->staging_event) {
        if (hipEventSynchronize(ctx->staging_event) != hipSuccess) return FIC_E_HIP;
    }
    if (ctx->staging_bytes < total) {
        if (ctx->staging) (void)hipHostFree(ctx->staging);
        ctx->staging = nullptr;
        ctx->staging_bytes = 0;
        if (hipHostMalloc(&ctx->staging, total) != hipSuccess) return FIC_E_NOMEM;
        ctx->staging_bytes = total;
    }
    if (!ctx->staging_event && hipEventCreateWithFlags(&ctx->staging_event, hipEventDisableTiming) != hipSuccess)
        return FIC_E_HIP;
    for (auto &pl : plans) {
        char *dst = (char *)ctx->staging + pl.table_off;
        memcpy(dst, pl.h.data(), sizeof(ImgLvl) * pl.h.size());
        memcpy(dst + al(sizeof(ImgLvl) * pl.h.size()), pl.pre.data(), sizeof(int) * pl.pre.size());
    }
    if (hipMemcpyAsync(tables ? tables : ctx->slot[S_TABLES].ptr, ctx->staging, total, hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return FIC_E_HIP;
    if (hipEventRecord(ctx->staging_event, st) != hipSuccess) return FIC_E_HIP;
    return FIC_OK;
}

// Reserve the largest per-slot need over all plans (levels run one after the
// other on the stream) plus room for every table.
int reserve_plans(fic_ctx *ctx, std::vector<LevelPlan> &plans, size_t extra_dec0) {
    size_t need[S_NUM_SLOTS] = {0};
    size_t tables = 0;
    for (auto &pl : plans) {
        for (int s = 0; s < S_NUM_SLOTS; ++s) need[s] = max(need[s], pl.slot_bytes[s]);
        pl.table_off = tables;
        tables += table_bytes(pl);
    }
    need[S_TABLES] = tables;
    need[S_DEC0] = max(need[S_DEC0], extra_dec0);
    return reserve(ctx, need);
}

int run_integ(fic_ctx *ctx, LevelPlan &pl, hipStream_t st) {
    mark(ctx, FIC_T_POOL, pl.bh.B, st);
    FIC_TRY(launch_integ_b(pl.bh, st));
    mark(ctx, -1, 0, st);
    return FIC_OK;
}

int run_pool(fic_ctx *ctx, LevelPlan &pl, hipStream_t st) {
    mark(ctx, FIC_T_POOL, pl.bh.B, st);
    FIC_TRY(launch_pool_b(pl.bh, ctx->table, st));
    mark(ctx, -1, 0, st);
    return FIC_OK;
}

int run_search(fic_ctx *ctx, LevelPlan &pl, hipStream_t st) {
    const BatchHost &b = pl.bh;
    mark(ctx, FIC_T_PREP, b.B, st);
    FIC_TRY(launch_range_info_b(b, st));
    if (b.eng == E_F16) FIC_TRY(launch_f16_prep_b(b, st));
    else if (b.eng == E_I8 || b.eng == E_H16) FIC_TRY(launch_mfma_prep_b(b, st));
    else FIC_TRY(launch_fp32_prep_b(b, st));
    if (b.eng != E_FP32) FIC_TRY(launch_search_plan_b(b, st));
    mark(ctx, FIC_T_SEARCH, b.B, st);
    if (b.eng == E_F16) FIC_TRY(launch_f16_search_b(b, st));
    else if (b.eng == E_I8 || b.eng == E_H16) FIC_TRY(launch_mfma_search_b(b, st));
    else FIC_TRY(launch_fp32_search_b(b, st));
    mark(ctx, FIC_T_FINAL, b.B, st);
    FIC_TRY(launch_finalize_b(b, st));
    if (!b.is_last) FIC_TRY(launch_children_b(b, st));
    mark(ctx, -1, 0, st);
    return FIC_OK;
}

// Every launch of one encode, in order.
int run_encode(fic_ctx *ctx, std::vector<LevelPlan> &plans, hipStream_t s) {
    FIC_TRY(launch_level0_b(plans[0].bh, s));
    int st = run_integ(ctx, plans[0], s);
    if (st != FIC_OK) return st;
    for (auto &pl : plans) {
        st = run_pool(ctx, pl, s);
        if (st != FIC_OK) return st;
        st = run_search(ctx, pl, s);
        if (st != FIC_OK) return st;
    }
    return FIC_OK;
}

template <class T>
void put(std::vector<uint8_t> &k, const T &v) {
    const uint8_t *b = (const uint8_t *)&v;
    k.insert(k.end(), b, b + sizeof(T));
}

// Every argument of an encode, field by field (no struct padding).
std::vector<uint8_t> encode_key(const fic_image *imgs, int n, const fic_params *p, const fic_pool *pools,
                                const fic_level_codes *codes) {
    std::vector<uint8_t> k;
    put(k, n);
    put(k, *p);   // int32 fields only
    for (int i = 0; i < n; ++i) {
        put(k, imgs[i].pix);
        put(k, imgs[i].width);
        put(k, imgs[i].height);
        put(k, imgs[i].pitch);
    }
    for (int i = 0; i < n * p->levels; ++i) {
        const fic_pool &q = pools[i];
        put(k, q.capacity);
        put(k, q.count);
        put(k, q.xy);
        put(k, q.key);
        put(k, q.sum4);
        put(k, q.a);
        const fic_level_codes &c = codes[i];
        put(k, c.capacity);
        put(k, c.count);
        put(k, c.xy);
        put(k, c.split);
        put(k, c.domain);
        put(k, c.iso);
        put(k, c.s_idx);
        put(k, c.offset);
        put(k, c.err);
    }
    return k;
}

// Records the encode's launches into a graph (on the capture stream), keeps
// it with its own copy of the level tables, and launches it on s.
int capture_encode(fic_ctx *ctx, std::vector<LevelPlan> &plans, std::vector<uint8_t> key, hipStream_t s) {
    GraphCache *gc = ctx->graphs;
    size_t total = 0;
    for (auto &pl : plans) total += table_bytes(pl);
    GraphEntry g;
    g.key = std::move(key);
    if (hipMalloc(&g.tables, total) != hipSuccess) return FIC_E_NOMEM;
    for (auto &pl : plans) bind(ctx, pl, g.tables);
    int st = upload(ctx, plans, s, g.tables);
    if (st != FIC_OK) {
        free_graph(g);
        return st;
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(gc->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        free_graph(g);
        return FIC_E_HIP;
    }
    st = run_encode(ctx, plans, gc->cap);
    const hipError_t ec = hipStreamEndCapture(gc->cap, &graph);
    if (st == FIC_OK && ec != hipSuccess) st = FIC_E_HIP;
    if (st == FIC_OK && hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) st = FIC_E_HIP;
    if (graph) (void)hipGraphDestroy(graph);
    if (st != FIC_OK) {
        free_graph(g);
        return st;
    }
    if ((int)gc->e.size() >= gc->max) {  // evict the least recently used
        size_t lru = 0;
        for (size_t i = 1; i < gc->e.size(); ++i)
            if (gc->e[i].last_use < gc->e[lru].last_use) lru = i;
        free_graph(gc->e[lru]);
        gc->e.erase(gc->e.begin() + lru);
    }
    g.last_use = ++gc->tick;
    gc->e.push_back(g);
    FIC_TRY(hipGraphLaunch(gc->e.back().exec, s));
    return FIC_OK;
}

bool pool_ok(const fic_pool *p) { return p && p->count && p->xy && p->key && p->sum4 && p->a && p->capacity >= 1; }

bool codes_ok(const fic_level_codes *c) {
    return c && c->count && c->xy && c->split && c->domain && c->iso && c->s_idx && c->offset && c->err;
}


int check_decode(fic_ctx *ctx, const fic_params *p, const fic_pool *pools, const fic_level_codes *codes,
                 int32_t width, int32_t height, int32_t iterations, const uint8_t *out) {
    if (!ctx || !p || !pools || !codes || !out || iterations < 0) return FIC_E_INVALID;
    const int st = fic_validate_params(p, width, height);
    if (st != FIC_OK) return st;
    for (int l = 0; l < p->levels; ++l)
        if (!pool_ok(&pools[l]) || !codes_ok(&codes[l])) return FIC_E_INVALID;
    return FIC_OK;
}

// X0 then `iterations` synchronous updates, alternating between out and
// `other` (a width x height buffer, pitch width) so that the last lands in
// out.  X0 covers every pixel (the accepted ranges tile the image), so
// nothing is read from `other` before this call writes it.
int run_decode(fic_ctx *ctx, const fic_params *p, const fic_pool *pools, const fic_level_codes *codes, int width,
               int iterations, uint8_t *out, uint8_t *other, bool timed, hipStream_t s) {
    uint8_t *buf0 = (iterations % 2 == 0) ? out : other;
    uint8_t *buf1 = (iterations % 2 == 0) ? other : out;
    for (int l = 0; l < p->levels; ++l)
        FIC_TRY(launch_decode_init(p->block0 >> l, &codes[l], codes[l].capacity, buf0, width, s));
    for (int it = 0; it < iterations; ++it) {
        const uint8_t *cur = (it % 2 == 0) ? buf0 : buf1;
        uint8_t *nxt = (it % 2 == 0) ? buf1 : buf0;
        if (timed) mark(ctx, FIC_T_DECODE, 1, s);
        for (int l = 0; l < p->levels; ++l)
            FIC_TRY(launch_decode_iter(p->block0 >> l, &codes[l], codes[l].capacity, &pools[l],
                                       make_sset(p->s_num[l], p->s_count[l], p->s_den[l]), cur, nxt, width, s));
    }
    if (timed) mark(ctx, -1, 0, s);
    return FIC_OK;
}

}  // namespace

namespace fic {

int hip_status(hipError_t e) { return e == hipSuccess ? FIC_OK : (e == hipErrorOutOfMemory ? FIC_E_NOMEM : FIC_E_HIP); }

int persistent_grid(const void *kernel, int static_blocks) {
    static std::mutex mu;
    static std::vector<std::pair<const void *, int>> per_cu;   // resident workgroups per CU, per kernel
    static int cus[kMaxDevices];
    int dev = 0;
    (void)hipGetDevice(&dev);
    int resident = 0, ncu = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (auto &e : per_cu)
            if (e.first == kernel) resident = e.second;
        if (resident == 0) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kernel, 256, 0) != hipSuccess || resident < 1)
                resident = 1;
            per_cu.push_back({kernel, resident});
        }
        if (dev >= 0 && dev < kMaxDevices) {
            if (cus[dev] == 0 && hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                cus[dev] = 0;
            ncu = cus[dev];
        }
    }
    if (ncu < 1) ncu = 256;
    const long cap = max(8L, (long)resident * ncu / 8 * 8);
    return (int)min((long)static_blocks, cap);
}

int enter(fic_ctx *ctx) {
    if (!ctx) return FIC_E_INVALID;
    return hip_status(hipSetDevice(ctx->device));
}

int reserve(fic_ctx *ctx, const size_t *bytes) {
    int64_t total = 0;
    for (int i = 0; i < S_NUM_SLOTS; ++i)
        total += (int64_t)(bytes[i] > ctx->slot[i].bytes ? bytes[i] : ctx->slot[i].bytes);
    if (ctx->limit > 0 && total > ctx->limit) return FIC_E_NOMEM;
    bool synced = false;
    for (int i = 0; i < S_NUM_SLOTS; ++i) {
        if (bytes[i] <= ctx->slot[i].bytes) continue;
        if (ctx->slot[i].ptr) {
            if (!synced) {
                if (hipDeviceSynchronize() != hipSuccess) return FIC_E_HIP;
                synced = true;
                drop_graphs(ctx->graphs);  // they point into the slot being freed
            }
            (void)hipFree(ctx->slot[i].ptr);
            ctx->slot[i].ptr = nullptr;
            ctx->slot[i].bytes = 0;
        }
        const size_t want = (bytes[i] + 255) / 256 * 256;
        if (hipMalloc(&ctx->slot[i].ptr, want) != hipSuccess) {
            ctx->slot[i].ptr = nullptr;
            return FIC_E_NOMEM;
        }
        ctx->slot[i].bytes = want;
    }
    return FIC_OK;
}

static hipEvent_t take_event(Timer *t) {
    if (!t->spare.empty()) {
        hipEvent_t e = t->spare.back();
        t->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void mark(fic_ctx *ctx, int kind, int B, hipStream_t st) {
    Timer *t = ctx->timer;
    if (!t) return;
    if (t->open >= 0) {
        (void)hipEventRecord(t->recs[t->open].b, st);
        t->open = -1;
    }
    if (kind < 0 || t->recs.size() >= (1u << 16)) return;
    Timer::Rec r;
    r.kind = kind;
    r.slot = log2i(B);
    r.a = take_event(t);
    r.b = take_event(t);
    if (!r.a || !r.b) return;
    (void)hipEventRecord(r.a, st);
    t->recs.push_back(r);
    t->open = (int)t->recs.size() - 1;
}

static void recycle(Timer *t) {
    for (auto &r : t->recs) {
        t->spare.push_back(r.a);
        t->spare.push_back(r.b);
    }
    t->recs.clear();
    t->open = -1;
}

static void destroy_timer(Timer *t) {
    if (!t) return;
    recycle(t);
    for (hipEvent_t e : t->spare) (void)hipEventDestroy(e);
    delete t;
}

// ---------------------------------------------------------------- tile shapes
int mfma_shape_count(int B, bool f16);
bool mfma_shape_at(int B, bool f16, int index, TileShape &out);
TileShape mfma_pick(int B, bool f16, int choice);
int f16_shape_count(int B);
bool f16_shape_at(int B, int index, TileShape &out);
TileShape f16_pick(int B, int choice);

int form_of_engine(int eng) { return eng == E_I8 ? F_I8 : eng == E_H16 ? F_H16 : eng == E_F16 ? F_F16 : -1; }

int shape_count(int form, int B) {
    if (form == F_I8) return mfma_supported(B) ? mfma_shape_count(B, false) : 0;
    if (form == F_H16) return mfma_shape_count(B, true);
    if (form == F_F16) return f16_supported(B) ? f16_shape_count(B) : 0;
    return 0;
}

bool shape_at(int form, int B, int index, TileShape &out) {
    if (form == F_I8 || form == F_H16) return mfma_shape_at(B, form == F_H16, index, out);
    if (form == F_F16) return f16_shape_at(B, index, out);
    return false;
}

TileShape pick_shape(int form, int B, int choice) {
    return form == F_F16 ? f16_pick(B, choice) : mfma_pick(B, form == F_H16, choice);
}

}  // namespace fic

// ==================================================================== C ABI
extern "C" {

const char *fic_strerror(int status) {
    switch (status) {
        case FIC_OK: return "ok";
        case FIC_E_INVALID: return "invalid argument";
        case FIC_E_NOMEM: return "out of device memory or over the scratch limit";
        case FIC_E_HIP: return "HIP runtime error";
        case FIC_E_CAPACITY: return "caller buffer too small";
        case FIC_E_ARCH: return "device is not gfx950";
        case FIC_E_LIMIT: return "input larger than the fixed scratch of the allocation-free entry point";
        default: return "unknown status";
    }
}

int fic_entropy_table(int64_t *out, int32_t n) {
    if (!out || n < 0 || n > kTableSize) return FIC_E_INVALID;
    build_table();
    memcpy(out, g_table, sizeof(int64_t) * (size_t)n);
    return FIC_OK;
}

int fic_validate_params(const fic_params *p, int32_t width, int32_t height) {
    if (!p) return FIC_E_INVALID;
    if (p->levels < 1 || p->levels > kMaxLevels) return FIC_E_INVALID;
    if (!pow2(p->block0) || p->block0 > 32 || (p->block0 >> (p->levels - 1)) < 2) return FIC_E_INVALID;
    if (width < 2 * p->block0 || height < 2 * p->block0 || width % p->block0 || height % p->block0) return FIC_E_INVALID;
    if (width > 65535 || height > 65535 || (int64_t)width * height > (1 << 28)) return FIC_E_INVALID;
    if (check_pct(p->pool_pct) != FIC_OK || p->pool_max < 0) return FIC_E_INVALID;
    if (p->pool_key != FIC_POOL_ENTROPY && p->pool_key != FIC_POOL_VARIANCE) return FIC_E_INVALID;
    if (!engine_ok(p->engine)) return FIC_E_INVALID;
    for (int l = 0; l < p->levels; ++l) {
        if (p->step[l] < 1) return FIC_E_INVALID;
        if (check_sset(p->s_num[l], p->s_count[l], p->s_den[l]) != FIC_OK) return FIC_E_INVALID;
        if (check_rms(p->split_rms[l]) != FIC_OK) return FIC_E_INVALID;
    }
    return FIC_OK;
}

int fic_level_engine(int32_t engine, int32_t B) {
    if (!engine_ok(engine) || B < 2 || B > 32 || !pow2(B)) return FIC_E_INVALID;
    const int e = engine_for(engine, B);
    return e == E_F16 ? FIC_ENGINE_MFMA_F16 : e == E_I8 ? FIC_ENGINE_MFMA_I8
         : e == E_H16 ? FIC_ENGINE_MFMA_F16_16X16 : FIC_ENGINE_FP32;
}

int fic_query_capacity(const fic_params *p, int32_t width, int32_t height, int64_t *pool_cap, int64_t *range_cap) {
    const int st = fic_validate_params(p, width, height);
    if (st != FIC_OK) return st;
    if (!pool_cap || !range_cap) return FIC_E_INVALID;
    for (int l = 0; l < kMaxLevels; ++l) {
        pool_cap[l] = range_cap[l] = 0;
        if (l >= p->levels) continue;
        const int B = p->block0 >> l;
        const int64_t nd = n_candidates(width, height, B, p->step[l]);
        pool_cap[l] = (p->pool_max > 0 && p->pool_max < nd) ? p->pool_max : nd;
        range_cap[l] = (int64_t)(width / B) * (height / B);
    }
    return FIC_OK;
}

int fic_ctx_create(fic_ctx **out, int device) {
    if (!out) return FIC_E_INVALID;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return FIC_E_HIP;
    if (device < 0 || device >= ndev) return FIC_E_INVALID;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return FIC_E_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FIC_E_ARCH;
    if (hipSetDevice(device) != hipSuccess) return FIC_E_HIP;
    if (scratch_setup(device) != FIC_OK) return FIC_E_HIP;
    fic_ctx *ctx = new fic_ctx;
    memset(ctx, 0, sizeof(*ctx));
    ctx->device = device;
    memset(ctx->tune, -1, sizeof(ctx->tune));
    build_table();
    if (hipMalloc(&ctx->table, sizeof(g_table)) != hipSuccess) {
        delete ctx;
        return FIC_E_NOMEM;
    }
    if (hipMemcpy(ctx->table, g_table, sizeof(g_table), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(ctx->table);
        delete ctx;
        return FIC_E_HIP;
    }
    *out = ctx;
    return FIC_OK;
}

void fic_ctx_destroy(fic_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    destroy_timer(ctx->timer);
    if (ctx->graphs) {
        drop_graphs(ctx->graphs);
        if (ctx->graphs->cap) (void)hipStreamDestroy(ctx->graphs->cap);
        delete ctx->graphs;
    }
    if (ctx->staging_event) (void)hipEventDestroy(ctx->staging_event);
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    for (int i = 0; i < S_NUM_SLOTS; ++i)
        if (ctx->slot[i].ptr) (void)hipFree(ctx->slot[i].ptr);
    if (ctx->table) (void)hipFree(ctx->table);
    delete ctx;
}

int fic_ctx_set_scratch_limit(fic_ctx *ctx, int64_t bytes) {
    if (!ctx || bytes < 0) return FIC_E_INVALID;
    ctx->limit = bytes;
    return FIC_OK;
}

int fic_ctx_set_graphs(fic_ctx *ctx, int32_t max_graphs) {
    if (!ctx || max_graphs < 0 || max_graphs > 1024) return FIC_E_INVALID;
    int st = enter(ctx);
    if (st != FIC_OK) return st;
    if (!ctx->graphs) {
        if (max_graphs == 0) return FIC_OK;
        ctx->graphs = new GraphCache;
        if (hipStreamCreateWithFlags(&ctx->graphs->cap, hipStreamNonBlocking) != hipSuccess) {
            delete ctx->graphs;
            ctx->graphs = nullptr;
            return FIC_E_HIP;
        }
    }
    if (hipDeviceSynchronize() != hipSuccess) return FIC_E_HIP;
    if (max_graphs < (int)ctx->graphs->e.size()) drop_graphs(ctx->graphs);
    ctx->graphs->max = max_graphs;
    return FIC_OK;
}

int fic_ctx_graph_count(fic_ctx *ctx) { return ctx && ctx->graphs ? (int)ctx->graphs->e.size() : 0; }

int fic_shape_count(int32_t form, int32_t B) {
    if (form < 0 || form >= F_NUM || B < 1 || B > 32 || !pow2(B)) return 0;
    return shape_count(form, B);
}

int fic_shape_describe(int32_t form, int32_t B, int32_t index, int32_t *out) {
    if (!out || fic_shape_count(form, B) <= index || index < 0) return FIC_E_INVALID;
    TileShape t;
    if (!shape_at(form, B, index, t)) return FIC_E_INVALID;
    out[0] = t.pl;
    out[1] = t.rq;
    out[2] = t.dt;
    out[3] = t.wpe;
    return FIC_OK;
}

int fic_ctx_get_tuning(fic_ctx *ctx, fic_tuning *out) {
    if (!ctx || !out) return FIC_E_INVALID;
    for (int f = 0; f < F_NUM; ++f)
        for (int l = 0; l < 6; ++l) out->choice[f][l] = ctx->tune[f][l];
    return FIC_OK;
}

int fic_ctx_set_tuning(fic_ctx *ctx, const fic_tuning *in) {
    if (!ctx || !in) return FIC_E_INVALID;
    for (int f = 0; f < F_NUM; ++f)
        for (int l = 0; l < 6; ++l) {
            const int c = in->choice[f][l];
            if (c < -1 || c >= fic_shape_count(f, 1 << l)) return FIC_E_INVALID;
        }
    for (int f = 0; f < F_NUM; ++f)
        for (int l = 0; l < 6; ++l) ctx->tune[f][l] = (int8_t)in->choice[f][l];
    if (ctx->graphs) drop_graphs(ctx->graphs);
    return FIC_OK;
}

int fic_autotune(fic_ctx *ctx, const fic_image *imgs, int32_t n_images, const fic_params *p, fic_pool *pools,
                 fic_level_codes *codes, int32_t reps, fic_stream stream, fic_tuning *out) {
    if (!ctx || !p || reps < 1 || reps > 100 || ctx->timer) return FIC_E_INVALID;
    // first an ordinary encode: validates everything and warms the scratch
    int st = fic_encode(ctx, imgs, n_images, p, pools, codes, stream);
    if (st != FIC_OK) return st;
    struct Entry { int form, slot, count, best; double best_ms; };
    std::vector<Entry> ent;
    int maxc = 0;
    for (int l = 0; l < p->levels; ++l) {
        const int B = p->block0 >> l, form = form_of_engine(engine_for(p->engine, B));
        const int c = form >= 0 ? shape_count(form, B) : 0;
        if (c > 1) {
            ent.push_back(Entry{form, log2i(B), c, 0, 1e300});
            maxc = std::max(maxc, c);
        }
    }
    int8_t saved[3][6];
    memcpy(saved, ctx->tune, sizeof(saved));
    for (int i = 0; i < maxc && st == FIC_OK; ++i) {
        // levels with fewer candidates run their best so far meanwhile
        for (const Entry &e : ent) ctx->tune[e.form][e.slot] = (int8_t)(i < e.count ? i : e.best);
        st = fic_encode(ctx, imgs, n_images, p, pools, codes, stream);   // warm-up of this candidate
        if (st != FIC_OK) break;
        st = fic_ctx_set_timing(ctx, 1);
        for (int r = 0; r < reps && st == FIC_OK; ++r) st = fic_encode(ctx, imgs, n_images, p, pools, codes, stream);
        fic_timing t;
        const int st2 = st == FIC_OK ? fic_ctx_read_timing(ctx, &t) : FIC_OK;
        fic_ctx_set_timing(ctx, 0);
        if (st == FIC_OK) st = st2;
        if (st != FIC_OK) break;
        for (Entry &e : ent) {
            if (i >= e.count) continue;
            const double ms = t.ms[FIC_T_PREP][e.slot] + t.ms[FIC_T_SEARCH][e.slot] + t.ms[FIC_T_FINAL][e.slot];
            // another candidate replaces the current best only when clearly
            // faster (3 %), so run-to-run noise keeps the measured default
            if (i == 0 || ms < 0.97 * e.best_ms) {
                e.best_ms = ms;
                e.best = i;
            }
        }
    }
    if (st != FIC_OK) {
        memcpy(ctx->tune, saved, sizeof(saved));
        return st;
    }
    for (const Entry &e : ent) ctx->tune[e.form][e.slot] = (int8_t)e.best;
    if (ctx->graphs) drop_graphs(ctx->graphs);
    // leave the buffers holding an encode with the chosen shapes
    st = fic_encode(ctx, imgs, n_images, p, pools, codes, stream);
    if (st == FIC_OK && out) fic_ctx_get_tuning(ctx, out);
    return st;
}

int fic_ctx_set_timing(fic_ctx *ctx, int enable) {
    if (!ctx) return FIC_E_INVALID;
    int st = enter(ctx);
    if (st != FIC_OK) return st;
    if (enable) {
        if (!ctx->timer) ctx->timer = new Timer;
        else recycle(ctx->timer);
    } else {
        (void)hipDeviceSynchronize();
        destroy_timer(ctx->timer);
        ctx->timer = nullptr;
    }
    return FIC_OK;
}

int fic_ctx_read_timing(fic_ctx *ctx, fic_timing *out) {
    if (!ctx || !out) return FIC_E_INVALID;
    memset(out, 0, sizeof(*out));
    Timer *t = ctx->timer;
    if (!t) return FIC_OK;
    int st = enter(ctx);
    if (st != FIC_OK) return st;
    for (auto &r : t->recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return FIC_E_HIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return FIC_E_HIP;
        out->ms[r.kind][r.slot] += ms;
        out->launches[r.kind][r.slot] += 1;
    }
    recycle(t);
    return FIC_OK;
}

int fic_build_domain_pool(fic_ctx *ctx, const fic_image *img, int32_t B, int32_t L, fic_ratio pct,
                          int32_t pool_max, int32_t pool_key, fic_pool *out, fic_stream stream) {
    if (!ctx || B < 2 || B > 32 || L < 1 || !image_ok(img, B) || check_pct(pct) != FIC_OK || pool_max < 0 ||
        !pool_ok(out) || (pool_key != FIC_POOL_ENTROPY && pool_key != FIC_POOL_VARIANCE))
        return FIC_E_INVALID;
    const int64_t nd = n_candidates(img->width, img->height, B, L);
    const int64_t need = (pool_max > 0 && pool_max < nd) ? pool_max : nd;
    if (out->capacity < need) return FIC_E_CAPACITY;
    int st = enter(ctx);
    if (st != FIC_OK) return st;
    std::vector<ImgIn> in(1);
    in[0] = ImgIn{img, B, L, pct.num, pct.den, pool_max, out, nullptr, nullptr, 0, nullptr, nullptr, nullptr};
    std::vector<LevelPlan> plans(1);
    if (!plan_level(plans[0], in, false, FIC_ENGINE_MFMA, 0, true, pool_key, ctx->tune)) return FIC_E_NOMEM;
    st = reserve_plans(ctx, plans, 0);
    if (st != FIC_OK) return st;
    bind(ctx, plans[0]);
    hipStream_t s = (hipStream_t)stream;
    st = upload(ctx, plans, s);
    if (st != FIC_OK) return st;
    st = run_integ(ctx, plans[0], s);
    if (st != FIC_OK) return st;
    return run_pool(ctx, plans[0], s);
}

int fic_encode_level(fic_ctx *ctx, const fic_image *img, const fic_pool *pool, const uint32_t *ranges_xy,
                     const int32_t *n_ranges, int32_t range_capacity, int32_t B, const int32_t *s_num,
                     int32_t s_count, int32_t s_den, fic_ratio split_rms, int32_t is_last, int32_t engine,
                     fic_level_codes *out, uint32_t *children_xy, int32_t *n_children, fic_stream stream) {
    if (!ctx || !pow2(B) || B < 2 || B > 32 || !image_ok(img, B) || !pool_ok(pool) || !ranges_xy || !n_ranges ||
        range_capacity < 0 || check_sset(s_num, s_count, s_den) != FIC_OK || check_rms(split_rms) != FIC_OK ||
        !codes_ok(out) || !engine_ok(engine) ||
        (!is_last && (!children_xy || !n_children)))
        return FIC_E_INVALID;
    if (out->capacity < range_capacity) return FIC_E_CAPACITY;
    int st = enter(ctx);
    if (st != FIC_OK) return st;
    // the search needs no pool scratch: the coarsest step keeps the unused key
    // buffer small, and the chunks are planned for the caller's pool capacity
    std::vector<ImgIn> in(1);
    in[0] = ImgIn{img, B, B, 0, 1, 0, const_cast<fic_pool *>(pool), ranges_xy, n_ranges, range_capacity, out,
                  children_xy, n_children, pool->capacity};
    std::vector<LevelPlan> plans(1);
    if (!plan_level(plans[0], in, true, engine, 0, true, FIC_POOL_ENTROPY, ctx->tune)) return FIC_E_NOMEM;
    plans[0].bh.ss = make_sset(s_num, s_count, s_den);
    plans[0].bh.rms = split_rms;
    plans[0].bh.is_last = is_last ? 1 : 0;
    st = reserve_plans(ctx, plans, 0);
    if (st != FIC_OK) return st;
    bind(ctx, plans[0]);
    hipStream_t s = (hipStream_t)stream;
    st = upload(ctx, plans, s);
    if (st != FIC_OK) return st;
    st = run_integ(ctx, plans[0], s);
    if (st != FIC_OK) return st;
    return run_search(ctx, plans[0], s);
}

int fic_encode(fic_ctx *ctx, const fic_image *imgs, int32_t n_images, const fic_params *p, fic_pool *pools,
               fic_level_codes *codes, fic_stream stream) {
    if (!ctx || !imgs || n_images < 0 || !p || !pools || !codes) return FIC_E_INVALID;
    const int NL = p->levels;
    // validate everything before the first launch
    for (int i = 0; i < n_images; ++i) {
        const fic_image *img = &imgs[i];
        if (!img->pix || img->pitch < img->width) return FIC_E_INVALID;
        int st = fic_validate_params(p, img->width, img->height);
        if (st != FIC_OK) return st;
        int64_t pcap[kMaxLevels], rcap[kMaxLevels];
        fic_query_capacity(p, img->width, img->height, pcap, rcap);
        for (int l = 0; l < NL; ++l) {
            fic_pool *pl = &pools[i * NL + l];
            fic_level_codes *cl = &codes[i * NL + l];
            if (!pool_ok(pl) || !codes_ok(cl)) return FIC_E_INVALID;
            if (pl->capacity < pcap[l] || cl->capacity < rcap[l]) return FIC_E_CAPACITY;
        }
    }
    if (n_images == 0) return FIC_OK;
    int st = enter(ctx);
    if (st != FIC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    GraphCache *gc = ctx->graphs;
    const bool use_graph = gc && gc->max > 0 && !ctx->timer;
    std::vector<uint8_t> key;
    if (use_graph) {
        key = encode_key(imgs, n_images, p, pools, codes);
        for (auto &g : gc->e)
            if (g.key == key) {
                g.last_use = ++gc->tick;
                FIC_TRY(hipGraphLaunch(g.exec, s));
                return FIC_OK;
            }
    }
    std::vector<LevelPlan> plans(NL);
    for (int l = 0; l < NL; ++l) {
        const int B = p->block0 >> l;
        const bool last = l == NL - 1;
        std::vector<ImgIn> in(n_images);
        for (int i = 0; i < n_images; ++i) {
            const fic_image *img = &imgs[i];
            fic_level_codes *cl = &codes[i * NL + l];
            in[i] = ImgIn{img, B, p->step[l], p->pool_pct.num, p->pool_pct.den, p->pool_max, &pools[i * NL + l],
                          cl->xy, cl->count, (img->width / B) * (img->height / B), cl,
                          last ? nullptr : codes[i * NL + l + 1].xy, last ? nullptr : codes[i * NL + l + 1].count};
        }
        if (!plan_level(plans[l], in, true, p->engine, l == 0, l == 0, p->pool_key, ctx->tune)) return FIC_E_NOMEM;
        plans[l].bh.ss = make_sset(p->s_num[l], p->s_count[l], p->s_den[l]);
        plans[l].bh.rms = p->split_rms[l];
        plans[l].bh.is_last = last ? 1 : 0;
    }
    st = reserve_plans(ctx, plans, 0);
    if (st != FIC_OK) return st;
    if (use_graph) return capture_encode(ctx, plans, std::move(key), s);
    for (auto &pl : plans) bind(ctx, pl);
    st = upload(ctx, plans, s);
    if (st != FIC_OK) return st;
    return run_encode(ctx, plans, s);
}

int fic_decode(fic_ctx *ctx, const fic_params *p, const fic_pool *pools, const fic_level_codes *codes, int32_t width,
               int32_t height, int32_t iterations, uint8_t *out, fic_stream stream) {
    int st = check_decode(ctx, p, pools, codes, width, height, iterations, out);
    if (st != FIC_OK) return st;
    st = enter(ctx);
    if (st != FIC_OK) return st;
    size_t b[S_NUM_SLOTS] = {0};
    b[S_DEC0] = (size_t)width * height;
    st = reserve(ctx, b);
    if (st != FIC_OK) return st;
    return run_decode(ctx, p, pools, codes, width, iterations, out, (uint8_t *)sp(ctx, S_DEC0), true,
                      (hipStream_t)stream);
}

int fic_decode_noalloc(fic_ctx *ctx, const fic_params *p, const fic_pool *pools, const fic_level_codes *codes,
                       int32_t width, int32_t height, int32_t iterations, uint8_t *out, fic_stream stream) {
    int st = check_decode(ctx, p, pools, codes, width, height, iterations, out);
    if (st != FIC_OK) return st;
    if ((int64_t)width * height > FIC_DECODE_NOALLOC_MAX_PIXELS) return FIC_E_LIMIT;
    st = enter(ctx);
    if (st != FIC_OK) return st;
    uint8_t *fixed = (uint8_t *)scratch_of(ctx->device);
    if (!fixed) return FIC_E_HIP;
    return run_decode(ctx, p, pools, codes, width, iterations, out, fixed, false, (hipStream_t)stream);
}

}  // extern "C"
