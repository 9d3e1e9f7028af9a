// Host side of the C ABI: argument validation, context and scratch, the
// entropy key table, and the orchestration of the per-level kernels.
#include <math.h>
#include <string.h>

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

}  // namespace fic

using namespace fic;

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

int hip_status(hipError_t e) { return e == hipSuccess ? FIC_OK : (e == hipErrorOutOfMemory ? FIC_E_NOMEM : FIC_E_HIP); }

#define FIC_TRY(expr)                              \
    do {                                           \
        const hipError_t e_ = (expr);              \
        if (e_ != hipSuccess) return hip_status(e_); \
    } while (0)

// ---------------------------------------------------------------- scratch sizing
void max_into(size_t *dst, const size_t *src) {
    for (int i = 0; i < S_NUM_SLOTS; ++i)
        if (src[i] > dst[i]) dst[i] = src[i];
}

void pool_bytes(int64_t nd, size_t *b) {
    const size_t nb = (size_t)((nd + kScanBlock - 1) / kScanBlock);
    b[S_KEYS] = sizeof(int64_t) * (size_t)nd;
    b[S_SEL] = sizeof(PoolSel);
    b[S_BLOCKSUM] = b[S_BLOCKOFF] = sizeof(int) * (nb + 1);
}

void level_bytes(int B, int range_cap, int pool_cap, bool mfma, size_t *b) {
    const size_t nb = (size_t)((range_cap + kScanBlock - 1) / kScanBlock);
    b[S_BLOCKSUM] = b[S_BLOCKOFF] = sizeof(int) * (nb + 1);
    b[S_RINFO] = sizeof(RInfo) * (size_t)(range_cap + 1);
    int nchunk, tpc;
    if (mfma) {
        nchunk = mfma_geometry(B, range_cap, pool_cap).nslot;
        const size_t KS = (size_t)B * B / 16;
        const size_t ntiles = (size_t)(pool_cap + kDomTile - 1) / kDomTile;
        b[S_AFRAG] = (size_t)mfma_quads_padded(B, range_cap) * 2 * KS * 1024;
        b[S_BFRAG] = ntiles * KS * 1024;
        b[S_DINFO] = ntiles * kDomTile * sizeof(float2);
    } else {
        fp32_geometry(B, range_cap, pool_cap, &nchunk, &tpc);
        const size_t n = (size_t)B * B;
        b[S_VF32] = n * (size_t)fp32_rpad(range_cap) * 8 * sizeof(float);
        b[S_DF32] = n * (size_t)fp32_ppad(pool_cap) * sizeof(float);
        b[S_DINFO] = (size_t)fp32_ppad(pool_cap) * sizeof(float2);
    }
    b[S_PARTIAL] = sizeof(Partial) * (size_t)range_cap * nchunk;
}

// ---------------------------------------------------------------- launch bodies
int do_pool(fic_ctx *ctx, const fic_image *img, int B, int L, fic_ratio pct, int pool_max, fic_pool *out,
            hipStream_t st) {
    const int W = img->width, H = img->height;
    const int nx = (W - 2 * B) / L + 1;
    const int64_t nd = n_candidates(W, H, B, L);
    const int64_t c = ((int64_t)pct.num * nd + pct.den - 1) / pct.den;
    PoolSel *sel = (PoolSel *)sp(ctx, S_SEL);
    int64_t *keys = (int64_t *)sp(ctx, S_KEYS);
    mark(ctx, FIC_T_POOL, B, st);
    FIC_TRY(launch_sel_init(sel, c, pool_max, st));
    FIC_TRY(launch_pool_keys(img->pix, img->pitch, nx, (int)nd, L, 2 * B, ctx->table, keys, sel, st));
    FIC_TRY(launch_pool_select(keys, (int)nd, c, pool_max, sel, st));
    FIC_TRY(launch_pool_compact(keys, (int)nd, nx, L, c, pool_max, sel, (int *)sp(ctx, S_BLOCKSUM),
                                (int *)sp(ctx, S_BLOCKOFF), out, st));
    const int cap = (int)(pool_max > 0 && pool_max < nd ? pool_max : nd);
    FIC_TRY(launch_pool_moments(img->pix, img->pitch, B, cap, out, st));
    mark(ctx, -1, 0, st);
    return FIC_OK;
}

int do_level(fic_ctx *ctx, const fic_image *img, const fic_pool *pool, const uint32_t *rxy, const int32_t *nr,
             int range_cap, int B, SSet ss, fic_ratio rms, int is_last, bool mfma, fic_level_codes *out,
             uint32_t *children, int32_t *n_children, hipStream_t st) {
    const int pool_cap = pool->capacity;
    RInfo *ri = (RInfo *)sp(ctx, S_RINFO);
    Partial *part = (Partial *)sp(ctx, S_PARTIAL);
    float2 *dinfo = (float2 *)sp(ctx, S_DINFO);
    int nchunk, tpc;
    mark(ctx, FIC_T_PREP, B, st);
    FIC_TRY(launch_range_info(img->pix, img->pitch, B, rxy, nr, range_cap, ri, st));
    if (mfma) {
        nchunk = mfma_geometry(B, range_cap, pool_cap).nslot;
        FIC_TRY(launch_mfma_prep(img->pix, img->pitch, B, rxy, nr, range_cap, pool, pool_cap, sp(ctx, S_AFRAG),
                                 sp(ctx, S_BFRAG), dinfo, st));
        mark(ctx, FIC_T_SEARCH, B, st);
        FIC_TRY(launch_mfma_search(B, sp(ctx, S_AFRAG), sp(ctx, S_BFRAG), dinfo, ri, nr, range_cap, pool, pool_cap,
                                   ss, part, st));
    } else {
        fp32_geometry(B, range_cap, pool_cap, &nchunk, &tpc);
        FIC_TRY(launch_fp32_prep(img->pix, img->pitch, B, rxy, nr, range_cap, pool, pool_cap,
                                 (float *)sp(ctx, S_VF32), (float *)sp(ctx, S_DF32), dinfo, st));
        mark(ctx, FIC_T_SEARCH, B, st);
        FIC_TRY(launch_fp32_search(B, (const float *)sp(ctx, S_VF32), (const float *)sp(ctx, S_DF32), dinfo, ri, nr,
                                   range_cap, pool, pool_cap, ss, part, st));
    }
    mark(ctx, FIC_T_FINAL, B, st);
    FIC_TRY(launch_finalize(img->pix, img->pitch, B, rxy, nr, range_cap, pool, part, nchunk, ss, rms, is_last, out,
                            st));
    if (!is_last)
        FIC_TRY(launch_children(out, range_cap, B, (int *)sp(ctx, S_BLOCKSUM), (int *)sp(ctx, S_BLOCKOFF), children,
                                n_children, st));
    mark(ctx, -1, 0, st);
    return FIC_OK;
}

bool pool_ok(const fic_pool *p) { return p && p->count && p->xy && p->key && p->sum4 && p->a && p->capacity >= 1; }

bool codes_ok(const fic_level_codes *c) {
    return c && c->count && c->xy && c->split && c->domain && c->iso && c->s_idx && c->offset && c->err;
}

int enter(fic_ctx *ctx) {
    if (!ctx) return FIC_E_INVALID;
    return hip_status(hipSetDevice(ctx->device));
}

}  // namespace

namespace fic {

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

static int log2i(int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v && l < 5) ++l;
    return l;
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
    if (p->engine != FIC_ENGINE_MFMA && p->engine != FIC_ENGINE_FP32) return FIC_E_INVALID;
    for (int l = 0; l < p->levels; ++l) {
        if (p->step[l] < 1) return FIC_E_INVALID;
        if (check_sset(p->s_num[l], p->s_count[l], p->s_den[l]) != FIC_OK) return FIC_E_INVALID;
        if (check_rms(p->split_rms[l]) != FIC_OK) return FIC_E_INVALID;
    }
    return FIC_OK;
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
    fic_ctx *ctx = new fic_ctx;
    memset(ctx, 0, sizeof(*ctx));
    ctx->device = device;
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
                          int32_t pool_max, fic_pool *out, fic_stream stream) {
    if (!ctx || B < 2 || B > 32 || L < 1 || !image_ok(img, B) || check_pct(pct) != FIC_OK || pool_max < 0 ||
        !pool_ok(out))
        return FIC_E_INVALID;
    const int64_t nd = n_candidates(img->width, img->height, B, L);
    const int64_t need = (pool_max > 0 && pool_max < nd) ? pool_max : nd;
    if (out->capacity < need) return FIC_E_CAPACITY;
    int st = enter(ctx);
    if (st != FIC_OK) return st;
    size_t b[S_NUM_SLOTS] = {0};
    pool_bytes(nd, b);
    st = reserve(ctx, b);
    if (st != FIC_OK) return st;
    return do_pool(ctx, img, B, L, pct, pool_max, out, (hipStream_t)stream);
}

int fic_encode_level(fic_ctx *ctx, const fic_image *img, const fic_pool *pool, const uint32_t *ranges_xy,
                     const int32_t *n_ranges, int32_t range_capacity, int32_t B, const int32_t *s_num,
                     int32_t s_count, int32_t s_den, fic_ratio split_rms, int32_t is_last, int32_t engine,
                     fic_level_codes *out, uint32_t *children_xy, int32_t *n_children, fic_stream stream) {
    if (!ctx || !pow2(B) || B < 2 || B > 32 || !image_ok(img, B) || !pool_ok(pool) || !ranges_xy || !n_ranges ||
        range_capacity < 0 || check_sset(s_num, s_count, s_den) != FIC_OK || check_rms(split_rms) != FIC_OK ||
        !codes_ok(out) || (engine != FIC_ENGINE_MFMA && engine != FIC_ENGINE_FP32) ||
        (!is_last && (!children_xy || !n_children)))
        return FIC_E_INVALID;
    if (out->capacity < range_capacity) return FIC_E_CAPACITY;
    int st = enter(ctx);
    if (st != FIC_OK) return st;
    const bool mfma = engine == FIC_ENGINE_MFMA && mfma_supported(B);
    size_t b[S_NUM_SLOTS] = {0};
    level_bytes(B, range_capacity, pool->capacity, mfma, b);
    st = reserve(ctx, b);
    if (st != FIC_OK) return st;
    return do_level(ctx, img, pool, ranges_xy, n_ranges, range_capacity, B, make_sset(s_num, s_count, s_den),
                    split_rms, is_last ? 1 : 0, mfma, out, children_xy, n_children, (hipStream_t)stream);
}

int fic_encode(fic_ctx *ctx, const fic_image *imgs, int32_t n_images, const fic_params *p, fic_pool *pools,
               fic_level_codes *codes, fic_stream stream) {
    if (!ctx || !imgs || n_images < 0 || !p || !pools || !codes) return FIC_E_INVALID;
    const int NL = p->levels;
    size_t need[S_NUM_SLOTS] = {0};
    // validate everything before the first launch
    for (int i = 0; i < n_images; ++i) {
        const fic_image *img = &imgs[i];
        if (!img->pix || img->pitch < img->width) return FIC_E_INVALID;
        int st = fic_validate_params(p, img->width, img->height);
        if (st != FIC_OK) return st;
        int64_t pcap[kMaxLevels], rcap[kMaxLevels];
        fic_query_capacity(p, img->width, img->height, pcap, rcap);
        for (int l = 0; l < NL; ++l) {
            const int B = p->block0 >> l;
            fic_pool *pl = &pools[i * NL + l];
            fic_level_codes *cl = &codes[i * NL + l];
            if (!pool_ok(pl) || !codes_ok(cl)) return FIC_E_INVALID;
            if (pl->capacity < pcap[l] || cl->capacity < rcap[l]) return FIC_E_CAPACITY;
            size_t b[S_NUM_SLOTS] = {0};
            pool_bytes(n_candidates(img->width, img->height, B, p->step[l]), b);
            max_into(need, b);
            memset(b, 0, sizeof(b));
            level_bytes(B, (int)rcap[l], pl->capacity, p->engine == FIC_ENGINE_MFMA && mfma_supported(B), b);
            max_into(need, b);
        }
    }
    int st = enter(ctx);
    if (st != FIC_OK) return st;
    st = reserve(ctx, need);
    if (st != FIC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < n_images; ++i) {
        const fic_image *img = &imgs[i];
        const int W = img->width, H = img->height;
        FIC_TRY(launch_level0(W / p->block0, H / p->block0, p->block0, codes[i * NL].xy, codes[i * NL].count, s));
        for (int l = 0; l < NL; ++l) {
            const int B = p->block0 >> l;
            fic_pool *pl = &pools[i * NL + l];
            fic_level_codes *cl = &codes[i * NL + l];
            st = do_pool(ctx, img, B, p->step[l], p->pool_pct, p->pool_max, pl, s);
            if (st != FIC_OK) return st;
            const bool last = l == NL - 1;
            const int rcap = (W / B) * (H / B);
            st = do_level(ctx, img, pl, cl->xy, cl->count, rcap, B, make_sset(p->s_num[l], p->s_count[l], p->s_den[l]),
                          p->split_rms[l], last ? 1 : 0, p->engine == FIC_ENGINE_MFMA && mfma_supported(B), cl,
                          last ? nullptr : codes[i * NL + l + 1].xy, last ? nullptr : codes[i * NL + l + 1].count, s);
            if (st != FIC_OK) return st;
        }
    }
    return FIC_OK;
}

int fic_decode(fic_ctx *ctx, const fic_params *p, const fic_pool *pools, const fic_level_codes *codes, int32_t width,
               int32_t height, int32_t iterations, uint8_t *out, fic_stream stream) {
    if (!ctx || !p || !pools || !codes || !out || iterations < 0) return FIC_E_INVALID;
    int st = fic_validate_params(p, width, height);
    if (st != FIC_OK) return st;
    for (int l = 0; l < p->levels; ++l)
        if (!pool_ok(&pools[l]) || !codes_ok(&codes[l])) return FIC_E_INVALID;
    st = enter(ctx);
    if (st != FIC_OK) return st;
    size_t b[S_NUM_SLOTS] = {0};
    b[S_DEC0] = (size_t)width * height;
    st = reserve(ctx, b);
    if (st != FIC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    uint8_t *scratch = (uint8_t *)sp(ctx, S_DEC0);
    uint8_t *buf0 = (iterations % 2 == 0) ? out : scratch;
    uint8_t *buf1 = (iterations % 2 == 0) ? scratch : out;
    for (int l = 0; l < p->levels; ++l)
        FIC_TRY(launch_decode_init(p->block0 >> l, &codes[l], codes[l].capacity, buf0, width, s));
    for (int it = 0; it < iterations; ++it) {
        const uint8_t *cur = (it % 2 == 0) ? buf0 : buf1;
        uint8_t *nxt = (it % 2 == 0) ? buf1 : buf0;
        mark(ctx, FIC_T_DECODE, 1, s);
        for (int l = 0; l < p->levels; ++l)
            FIC_TRY(launch_decode_iter(p->block0 >> l, &codes[l], codes[l].capacity, &pools[l],
                                       make_sset(p->s_num[l], p->s_count[l], p->s_den[l]), cur, nxt, width, s));
    }
    mark(ctx, -1, 0, s);
    return FIC_OK;
}

}  // extern "C"
