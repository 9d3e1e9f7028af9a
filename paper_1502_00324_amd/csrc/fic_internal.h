// Internal declarations of the gfx950 fractal encoder library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fic.h"

namespace fic {

// ---------------------------------------------------------------- constants
constexpr int kWave = 64;
constexpr int kMaxLevels = FIC_MAX_LEVELS;
constexpr int kMaxS = FIC_MAX_S;
constexpr int kTableSize = 4097;       // entropy table entries, q = 0..4096
constexpr int kScanBlock = 1024;       // items per block in stable compaction
constexpr int kDomTile = 16;           // domains per column tile of the int8 engine
constexpr int kDomTile32 = 32;         // domains per column tile of the f16 engine
constexpr int kF16PadTiles = 16;       // zero tiles after the matrix engines' operands (>= tiles per LDS stage)
constexpr int kFusedSelMax = 131072;   // candidates per image for the one-workgroup selection

// Tiles of the matrix engines' domain operands for a pool capacity, padding
// included (kF16PadTiles zero tiles: a search stage may read up to a stage
// past a chunk's end without a bound check).
__host__ __device__ inline int f16_tiles(int pool_cap) { return (pool_cap + kDomTile32 - 1) / kDomTile32 + kF16PadTiles; }
__host__ __device__ inline int mfma_tiles(int pool_cap) { return (pool_cap + kDomTile - 1) / kDomTile + kF16PadTiles; }

// ---------------------------------------------------------------- small PODs
// Contrast set of one level, passed by value to kernels.
struct SSet {
    int32_t count, den;
    int32_t num[kMaxS];
};

// Per-range values prepared for the search kernels.
// The prune test compares the isometry-max of C' = sum (view-128)(dom-128)
// with  tn*sqrtA[p] - bn*Sd4[p] - an  (see search_common.h).
struct RInfo {
    int64_t cr;      // n*sum(r^2) - (sum r)^2
    int32_t sr;      // sum r
    float bn;        // (128 n - Sr) / n
    float an;        // (512 n Sr - 65536 n^2) / n + margin
    float pad;
    int64_t gbest;   // best val found so far by any search workgroup (atomic min)
};

// One search partial: the best code of a range within one domain chunk.
struct Partial {
    int64_t val;
    int32_t p;       // -1 when the chunk held no domain
    int32_t k;
};

// Radix-select state kept in device memory.
struct SelState {
    unsigned long long key_prefix;
    uint32_t idx_prefix;
    int32_t remaining;
    int32_t all;            // 1 = fewer candidates than requested: keep every one
    int32_t pad[3];
    uint32_t hist[256];
};

// Thresholds deciding pool membership, produced on the device.
struct PoolSel {
    SelState pct;           // c-th largest key (drop threshold)
    SelState cap;           // pool_max-th smallest (key, index)
    unsigned long long gmin;
};

// ---------------------------------------------------------------- address spaces
// Buffer pointers read out of the batch descriptors carry no address space
// for the compiler, so loads through them become flat loads, and a flat load
// counts on the LDS wait counter as well: every LDS wait in a loop would then
// also wait for the global loads in flight.  All these buffers live in
// global memory; these casts say so.
template <class T>
using gptr = const __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> as_global(const T *p) {
    return (gptr<T>)p;
}

// ---------------------------------------------------------------- isometries
// out[y][x] = in[sy][sx] for isometry t = 4m + r of a B x B block:
// r clockwise quarter turns, then a left-right mirror when m = 1.
__host__ __device__ inline void iso_src(int t, int B, int y, int x, int &sy, int &sx) {
    const int e = B - 1;
    switch (t) {
        case 0: sy = y;     sx = x;     break;
        case 1: sy = e - x; sx = y;     break;
        case 2: sy = e - y; sx = e - x; break;
        case 3: sy = x;     sx = e - y; break;
        case 4: sy = y;     sx = e - x; break;
        case 5: sy = x;     sx = y;     break;
        case 6: sy = e - y; sx = x;     break;
        default: sy = e - x; sx = e - y; break;
    }
}

// Inverse isometry: quarter turns 1 and 3 swap, every other one is an involution.
__host__ __device__ inline int iso_inv(int t) { return t == 1 ? 3 : (t == 3 ? 1 : t); }

// ---------------------------------------------------------------- scratch
// Scratch slots owned by a context; each grows on demand.
enum Slot {
    S_KEYS, S_SEL, S_PBLOCK, S_CBLOCK, S_RINFO, S_AFRAG, S_BFRAG, S_DINFO, S_PARTIAL,
    S_VF32, S_DF32, S_DEC0, S_TABLES, S_INTEG, S_ITMP, S_PACK, S_QUEUE, S_NUM_SLOTS
};

struct Buf { void *ptr; size_t bytes; };

}  // namespace fic

namespace fic {
struct Timer;       // event records of the optional stage timing
struct GraphCache;  // captured encodes for replay
}

struct fic_ctx {
    int device;
    int64_t limit;               // 0 = unlimited
    fic::Buf slot[fic::S_NUM_SLOTS];
    int64_t *table;              // device entropy table
    fic::Timer *timer;           // non-null while stage timing is on
    fic::GraphCache *graphs;     // non-null once graph replay has been enabled
    void *staging;               // pinned host buffer for the level tables
    size_t staging_bytes;
    int8_t tune[3][6];           // tile-shape candidate per (form, log2 B), -1 = default
    hipEvent_t staging_event;    // last copy out of the staging buffer
};

namespace fic {

int reserve(fic_ctx *ctx, const size_t *bytes);   // bytes[S_NUM_SLOTS], 0 = untouched
int hip_status(hipError_t e);                      // FIC_OK, FIC_E_NOMEM or FIC_E_HIP
int enter(fic_ctx *ctx);                           // makes the ctx's device current

// Stage timing: mark(ctx, kind, B, st) opens a stage (closing the previous
// open one); mark(ctx, -1, 0, st) closes it.  No-ops unless timing is on.
void mark(fic_ctx *ctx, int kind, int B, hipStream_t st);
inline void *sp(fic_ctx *ctx, Slot s) { return ctx->slot[s].ptr; }

// ---------------------------------------------------------------- search geometry
// Tile shape of a matrix search kernel: operand form (16-row engine only),
// range quads per wave, domain tiles per LDS stage, waves per SIMD the
// register allocation aims at.  Each (form, B) has a list of compiled shapes;
// candidate 0 is the measured default, a context's tuning picks another.
struct TileShape { int pl, rq, dt, wpe; };
enum Form { F_I8 = 0, F_H16 = 1, F_F16 = 2, F_NUM = 3 };   // = FIC_FORM_*
int shape_count(int form, int B);
bool shape_at(int form, int B, int index, TileShape &out);
// The shape a plan uses: an FIC_MFMA_SHAPE / FIC_F16_SHAPE override if it
// names a compiled shape, else candidate `choice` (>= 0), else the default.
TileShape pick_shape(int form, int B, int choice);
int form_of_engine(int eng);   // Engine -> Form, -1 for FP32

struct MfmaGeom {
    int pl;       // operand form: 1 = raw pixels (K = 4B^2), 2 = decimated hi/lo planes (K = 2 B^2)
    int ka;       // 64-deep K-steps of a range fragment (per half)
    int kt;       // 64-deep K-steps of a domain tile (ka * pl)
    int rpw;      // ranges per workgroup
    int nrg;      // range groups
    int tpc;      // domain tiles per chunk
    int nchunk;   // chunks over the pool capacity
    int xcd;      // 1 = XCD-aware mapping (nchunk % 8 == 0)
    int G;        // chunks walked by one workgroup
    int nslot;    // partial results per range
    int nwg;      // workgroups
};
MfmaGeom mfma_geometry(int B, int range_cap, int pool_cap, const TileShape &sh);   // 16-row engine
MfmaGeom f16_geometry(int B, int range_cap, int pool_cap, const TileShape &sh);    // 32x32 f16 engine
void split_chunks(MfmaGeom &g, int range_cap, int ntiles, int tile_kib, int dt, bool rows16, int slots);

// ---------------------------------------------------------------- batched levels
// One quadtree level of a batch of images runs as one launch set whatever
// the number of images: every kernel takes the device table of per-image
// level state below, and a launch of kind k gives image i the workgroups
// [pre[k][i], pre[k][i+1]) (found by binary search on the prefix table); the
// matrix searches are persistent and take their work from device queues.
// Search engine of a level: every image of a level uses the same one.
enum Engine { E_FP32 = 0, E_I8 = 1, E_F16 = 2, E_H16 = 3 };

enum Kind {
    K_LEVEL0, K_KEYS, K_HIST, K_PCMP, K_MOM, K_RANGE, K_AFRAG, K_BFRAG, K_VIEWS, K_DOMS, K_SEARCH, K_FINAL,
    K_CCMP, K_IROW, K_ICOL, K_ICSCAN, K_NUM
};

struct ImgLvl {
    // image
    const uint8_t *pix;
    int W, H, pitch;
    // level geometry: candidates nx * ny = nd at step L, c = ceil(p nd)
    int B, L, nx, ny, nd, pool_max, pool_cap, range_cap;
    int strip;           // candidate rows per wave of the entropy key kernel
    long long c;
    // pool (caller buffers)
    int32_t *pcount;
    uint32_t *pxy;
    int64_t *pkey;
    uint32_t *psum4;
    int64_t *pa;
    // ranges in, codes and children out (caller buffers)
    const uint32_t *rxy;
    const int32_t *nr;
    int32_t *ccount;
    uint32_t *cxy;
    uint8_t *csplit;
    uint32_t *cdom;
    uint8_t *ciso, *csidx, *coff;
    int64_t *cerr;
    uint32_t *children;
    int32_t *nchildren;
    // integral images of this image (shared by every level) and the
    // column-pass chunk sums
    uint32_t *integ, *itmp;
    // scratch slices of this image
    int64_t *keys;
    PoolSel *sel;
    int *pblocksum, *pblockoff, *cblocksum, *cblockoff;
    RInfo *ri;
    // the ranges the search kernels take (search order -> range index) and
    // their count: every range but the constant ones when S holds 0, whose
    // code is fixed (range moments kernel)
    int32_t *sidx, *ns;
    Partial *part;
    uint4 *afrag, *bfrag;
    float2 *dinfo;
    float *vf, *df;
    // search geometry of the engine in use
    int eng;             // search engine of this level (Engine)
    MfmaGeom geo;        // matrix engines
    int rpad, ppad, fnchunk, ftpc;  // FP32
    int nslot;           // partial results per range
};

// Summed-area tables of one image (built by k_integ.hip): SI and SII over
// I and I^2, (H+1) x (W+1); then four parity classes q = 2 py + px of Q^2,
// Q the 2x2 sum at (2i + px, 2j + py), (H/2+1) x (W/2+1) each; uint32 mod 2^32.
struct IntegGeom {
    int W, H, ws, hs, wq, hq;   // ws = W+1, hs = H+1, wq = W/2+1, hq = H/2+1
    __device__ uint32_t *si(uint32_t *base) const { return base; }
    __device__ uint32_t *sii(uint32_t *base) const { return base + (size_t)hs * ws; }
    __device__ uint32_t *sq(uint32_t *base, int q) const { return base + 2 * (size_t)hs * ws + (size_t)q * hq * wq; }
    // table a = 0 (SI), 1 (SII), 2..5 (SQ_{a-2}): pointer, rows, columns
    __device__ void table(uint32_t *base, int a, uint32_t *&p, int &rows, int &cols) const {
        if (a < 2) {
            p = a == 0 ? si(base) : sii(base);
            rows = hs;
            cols = ws;
        } else {
            p = sq(base, a - 2);
            rows = hq;
            cols = wq;
        }
    }
};

// Sum over the w x h box at (x, y) of a summed-area table with row stride s;
// exact whenever the true sum is below 2^32.
__device__ inline uint32_t box_sum(const uint32_t *t, int s, int x, int y, int w, int h) {
    return t[(size_t)(y + h) * s + x + w] - t[(size_t)y * s + x + w] - t[(size_t)(y + h) * s + x] + t[(size_t)y * s + x];
}

struct BatchDev {
    const ImgLvl *d;     // device table, n entries
    const int *pre;      // device prefixes, K_NUM x (n + 1)
    int n;
    // work queue of the persistent search: kQueueHeads counters (one per
    // XCD), then per XCD the prefix over images of their item counts, n + 1
    // entries each (k_search_plan fills it)
    int *queue;
};
constexpr int kQueueHeads = 16;
inline size_t queue_ints(int n) { return kQueueHeads + 8 * (size_t)(n + 1); }

// Items of one image in XCD x's queue of a persistent search: the live range
// groups (those holding a range of the search list) times the partial-result
// slots, split over the XCDs as the static chunk walk splits them.
__device__ inline int search_items(const ImgLvl &d, int x) {
    const MfmaGeom &g = d.geo;
    const int R = min(*d.ns, d.range_cap);
    const int nrg = (R + g.rpw - 1) / g.rpw;
    if (g.xcd) return nrg * (g.nslot / 8);
    const long N = (long)nrg * g.nslot;
    return N > x ? (int)((N - x + 7) / 8) : 0;
}

// Range group, chunk walk and partial-result slot of item k of XCD x's queue
// within image d (R ranges in its search list).
__device__ inline void item_walk(const MfmaGeom &g, int R, int x, int k, int &rg, int &cfirst, int &cstep, int &ncs,
                                 int &slot, bool rotate = false) {
    const int nrg = (R + g.rpw - 1) / g.rpw;
    if (g.xcd) {   // XCD x owns chunks x, x + 8, ...: groups of G of them
        const int grp = k / nrg;
        // rotate: each XCD starts its pass over the range groups at a
        // different eighth, so the first walks of a group do not all start
        // at once without a shared best (the chunks an XCD reads stay the
        // same; measured faster at B = 4, slower at B = 8)
        rg = (k - grp * nrg + (rotate ? (int)((long long)x * nrg / 8) : 0)) % nrg;
        cfirst = x + 8 * grp * g.G;
        cstep = 8;
        ncs = g.G;
        slot = x + 8 * grp;
    } else {       // one chunk per item, items dealt round-robin over the queues
        const int j = 8 * k + x;
        rg = j % nrg;
        cfirst = slot = j / nrg;
        cstep = 1;
        ncs = 1;
    }
}

struct ImgLvl;
__device__ inline IntegGeom integ_geom(int W, int H) {
    IntegGeom g;
    g.W = W;
    g.H = H;
    g.ws = W + 1;
    g.hs = H + 1;
    g.wq = W / 2 + 1;
    g.hq = H / 2 + 1;
    return g;
}

__device__ inline int find_img(const int *pre, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Host view of one batched level: grid sizes per kind and the device table.
struct BatchHost {
    BatchDev dev;
    int blocks[K_NUM];   // total workgroups per kind
    int B, L, KS, any_cap, eng, pool_key;
    TileShape shape;     // matrix engines: the tile shape every image of the level uses
    int fused_sel;       // every image has <= kFusedSelMax candidates: one-workgroup selection
    SSet ss;
    fic_ratio rms;
    int is_last;
};

// Grid of a persistent search launch: the kernel's resident workgroups over
// the whole GPU (a multiple of 8, so workgroup w runs on XCD w % 8), at most
// the static count.
int persistent_grid(const void *kernel, int static_blocks);

// pool
hipError_t launch_pool_b(const BatchHost &b, const int64_t *table, hipStream_t st);
// levels
hipError_t launch_level0_b(const BatchHost &b, hipStream_t st);
hipError_t launch_range_info_b(const BatchHost &b, hipStream_t st);
hipError_t launch_finalize_b(const BatchHost &b, hipStream_t st);
hipError_t launch_search_plan_b(const BatchHost &b, hipStream_t st);
hipError_t launch_children_b(const BatchHost &b, hipStream_t st);
// MFMA engine
hipError_t launch_integ_b(const BatchHost &b, hipStream_t st);
size_t integ_words(int W, int H);
int integ_col_items(int W, int H);
int integ_scan_items(int W, int H);
bool mfma_supported(int B);   // int8 engine
bool f16_supported(int B);    // f16 engine
hipError_t launch_f16_prep_b(const BatchHost &b, hipStream_t st);
hipError_t launch_f16_search_b(const BatchHost &b, hipStream_t st);
hipError_t launch_mfma_prep_b(const BatchHost &b, hipStream_t st);
hipError_t launch_mfma_search_b(const BatchHost &b, hipStream_t st);
// FP32 engine
void fp32_geometry(int B, int range_cap, int pool_cap, int *nchunk, int *tiles_per_chunk);
int fp32_rpad(int range_cap);
int fp32_ppad(int pool_cap);
int fp32_blocks(int B, int range_cap, int pool_cap);
hipError_t launch_fp32_prep_b(const BatchHost &b, hipStream_t st);
hipError_t launch_fp32_search_b(const BatchHost &b, hipStream_t st);
// block counts per kind for one image (host)

// decoder (one image)
hipError_t launch_decode_init(int B, const fic_level_codes *codes, int cap, uint8_t *img, int pitch,
                              hipStream_t st);
hipError_t launch_decode_iter(int B, const fic_level_codes *codes, int cap, const fic_pool *pool, SSet ss,
                              const uint8_t *cur, uint8_t *nxt, int pitch, hipStream_t st);

}  // namespace fic
