// Quadtree level plumbing (Sec. 2, Fig 1; Sec. 3.3) for every image of a
// batch: level-0 ranges, range moments for the prune test, the per-range code
// (argmin merge, isometry recovery, stored offset, split rule) and the child
// list.
#include "fic_internal.h"
#include "scan_util.h"

namespace fic {

// ---------------------------------------------------------------- level 0
__global__ __launch_bounds__(256) void k_level0(BatchDev b) {
    const int *pre = b.pre + K_LEVEL0 * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int nx = d.W / d.B, ny = d.H / d.B;
    const int r = (blockIdx.x - pre[im]) * 256 + threadIdx.x;
    if (r == 0) *d.ccount = nx * ny;
    if (r >= nx * ny) return;
    const int ry = r / nx, rx = r - ry * nx;
    d.cxy[r] = ((uint32_t)(ry * d.B) << 16) | (uint32_t)(rx * d.B);
}

hipError_t launch_level0_b(const BatchHost &b, hipStream_t st) {
    if (b.blocks[K_LEVEL0] > 0) k_level0<<<b.blocks[K_LEVEL0], 256, 0, st>>>(b.dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------- range moments
// One wave per range.  The prune margin is n/4 + 4 in units of C'; the float
// rounding of the prune test is below n/16 in the same units.
// One thread per range: Sr and sum r^2 from the summed-area tables.
__global__ __launch_bounds__(256) void k_range_info(BatchDev b, int s_has_zero) {
    const int *pre = b.pre + K_RANGE * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int r = (blockIdx.x - pre[im]) * 256 + threadIdx.x;
    const bool live = r < min(*d.nr, d.range_cap);
    bool searched = false;
    if (live) {
        const int B = d.B, n = B * B;
        const uint32_t v = d.rxy[r];
        const int x0 = v & 0xffff, y0 = v >> 16;
        const IntegGeom g = integ_geom(d.W, d.H);
        const int64_t s = box_sum(g.si(d.integ), g.ws, x0, y0, B, B);
        const int64_t ss = box_sum(g.sii(d.integ), g.ws, x0, y0, B, B);
        RInfo o;
        o.cr = (int64_t)n * ss - s * s;
        o.sr = (int32_t)s;
        o.bn = (float)(128.0 - (double)s / n);
        o.an = (float)(512.0 * s - 65536.0 * n + (n / 4 + 4));
        o.pad = 0.f;
        o.gbest = INT64_MAX;
        d.ri[r] = o;
        // A constant range (Cr = 0) has Bx = n X4 - Sr Sd4 = 0 against every
        // domain, so val = num^2 A >= 0; with 0 in S the first pair in the
        // search order, domain 0, isometry 0, s index 0, already reaches
        // val 0, and nothing beats or ties it earlier.  Its code is written
        // here (one partial, the other slots empty) and the search skips it.
        if (o.cr == 0 && s_has_zero) {
            Partial* q = d.part + (size_t)r * d.nslot;
            q[0] = Partial{0, 0, 0};
            for (int j = 1; j < d.nslot; ++j) q[j] = Partial{INT64_MAX, -1, 0};
        } else {
            searched = true;
        }
    }
    // append the searched ranges to the search list, one atomic per wave
    const uint64_t m = __ballot(searched);
    if (m) {
        const int lane = threadIdx.x & 63, leader = __ffsll((unsigned long long)m) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(d.ns, __popcll(m));
        base = __shfl(base, leader, 64);
        if (searched) d.sidx[base + __popcll(m & ((1ull << lane) - 1))] = r;
    }
}

// Clears the search-list count of every image before the range moments.
__global__ void k_search_list_reset(BatchDev b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < b.n) *b.d[i].ns = 0;
}

hipError_t launch_range_info_b(const BatchHost &b, hipStream_t st) {
    if (b.blocks[K_RANGE] > 0) {
        k_search_list_reset<<<(b.dev.n + 255) / 256, 256, 0, st>>>(b.dev);
        k_range_info<<<b.blocks[K_RANGE], 256, 0, st>>>(b.dev, b.ss.num[0] == 0 ? 1 : 0);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- search queue
// The work items of a level's persistent search, from the search lists the
// range moments just built: per XCD queue x, the prefix over images of their
// item counts; every queue head back to 0.
__global__ __launch_bounds__(64) void k_search_plan(BatchDev b) {
    const int x = threadIdx.x;
    if (x >= 8) return;
    int *pre = b.queue + kQueueHeads + x * (b.n + 1);
    int acc = 0;
    pre[0] = 0;
    for (int i = 0; i < b.n; ++i) {
        acc += search_items(b.d[i], x);
        pre[i + 1] = acc;
    }
    b.queue[x] = 0;
}

hipError_t launch_search_plan_b(const BatchHost &b, hipStream_t st) {
    if (b.blocks[K_SEARCH] > 0) k_search_plan<<<1, 64, 0, st>>>(b.dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------- finalize
__device__ inline bool lex_less(int64_t va, int pa, int64_t vb, int pb) { return va < vb || (va == vb && pa < pb); }

// One wave per range: merge the partials in (val, domain) order, pick the
// isometry (the lowest t of maximal cross term, or t = 0 when the chosen
// contrast is 0 and every isometry ties), then the offset, val_q and split.
__global__ __launch_bounds__(256) void k_finalize(BatchDev b, SSet ss, fic_ratio rms, int is_last) {
    const int *pre = b.pre + K_FINAL * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int lb = blockIdx.x - pre[im];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int R = min(*d.nr, d.range_cap);
    if (lb == 0 && threadIdx.x == 0) *d.ccount = R;
    const int r = lb * 4 + w;
    if (r >= R) return;
    const int nslot = d.nslot;
    int64_t bv = INT64_MAX;
    int bp = INT32_MAX, bk = 0;
    // partials read as 16-byte words (val lo, val hi, p, k) through a
    // global-qualified pointer
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    static_assert(sizeof(Partial) == 16, "Partial is read as one 16-byte word");
    const gptr<u32x4> pq = (gptr<u32x4>)as_global(d.part);
    for (int c = lane; c < nslot; c += 64) {
        const u32x4 w = pq[(size_t)r * nslot + c];
        Partial q;
        q.val = (int64_t)(((uint64_t)w.y << 32) | w.x);
        q.p = (int32_t)w.z;
        q.k = (int32_t)w.w;
        if (q.p >= 0 && lex_less(q.val, q.p, bv, bp)) {
            bv = q.val;
            bp = q.p;
            bk = q.k;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t ov = __shfl_xor(bv, off, 64);
        const int op = __shfl_xor(bp, off, 64), ok = __shfl_xor(bk, off, 64);
        if (lex_less(ov, op, bv, bp)) {
            bv = ov;
            bp = op;
            bk = ok;
        }
    }
    const int B = d.B, n = B * B, pitch = d.pitch;
    const uint8_t *img = d.pix;
    const uint32_t v = d.rxy[r];
    const int x0 = v & 0xffff, y0 = v >> 16;
    const IntegGeom g = integ_geom(d.W, d.H);
    const int64_t sr = box_sum(g.si(d.integ), g.ws, x0, y0, B, B);
    // every lane's first domain always passes the prune test, so bp is a
    // valid pool index whenever the pool is non-empty; stay in bounds anyway
    const int P = min(*d.pcount, d.pool_cap);
    if (bp < 0 || bp >= P) {
        bp = 0;
        bk = 0;
    }
    int nk = 0;
    for (int j = 0; j < ss.count; ++j)
        if (j == bk) nk = ss.num[j];
    int t_best = 0;
    if (nk != 0) {
        const uint32_t dv = d.pxy[bp];
        const int dx0 = dv & 0xffff, dy0 = dv >> 16;
        const gptr<uint8_t> im = as_global(img);
        // X4 of every isometry: |X4| <= 1024 * 255 * 1020 < 2^31
        int32_t x4[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) x4[t] = 0;
        for (int i = lane; i < n; i += 64) {
            const int y = i / B, x = i - y * B;
            const int rv = im[(size_t)(y0 + y) * pitch + x0 + x];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                int cy, cx;
                iso_src(t, B, y, x, cy, cx);
                const gptr<uint8_t> q = im + (size_t)(dy0 + 2 * cy) * pitch + dx0 + 2 * cx;
                x4[t] += rv * (q[0] + q[1] + q[pitch] + q[pitch + 1]);
            }
        }
        // The 8 wave sums by halving exchanges: after the steps at lane
        // distances 32, 16 and 8 each lane holds one isometry's partial,
        // t = (lane >> 3) & 7, summed over 8 lanes; three more steps finish
        // the sums.  Then the largest sum, the smallest t on ties.
        const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
        int32_t y4[4], z2[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t keep = b5 ? x4[4 + k] : x4[k], give = b5 ? x4[k] : x4[4 + k];
            y4[k] = keep + __shfl_xor(give, 32, 64);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int32_t keep = b4 ? y4[2 + k] : y4[k], give = b4 ? y4[k] : y4[2 + k];
            z2[k] = keep + __shfl_xor(give, 16, 64);
        }
        int32_t w = (b3 ? z2[1] : z2[0]) + __shfl_xor(b3 ? z2[0] : z2[1], 8, 64);
        w += __shfl_xor(w, 4, 64);
        w += __shfl_xor(w, 2, 64);
        w += __shfl_xor(w, 1, 64);
        int32_t bw = w, bt = (b5 ? 4 : 0) + (b4 ? 2 : 0) + (b3 ? 1 : 0);
#pragma unroll
        for (int off = 8; off < 64; off <<= 1) {
            const int32_t ow = __shfl_xor(bw, off, 64), ot = __shfl_xor(bt, off, 64);
            if (ow > bw || (ow == bw && ot < bt)) {
                bw = ow;
                bt = ot;
            }
        }
        t_best = bt;
    }
    if (lane == 0) {
        const int64_t o = (2 * sr + n) / (2 * n);
        const int64_t dq = (int64_t)n * o - sr;
        const int64_t den = ss.den;
        const int64_t valq = bv + 16 * den * den * dq * dq;
        int split = 0;
        if (!is_last) {
            const __uint128_t lhs = (__uint128_t)(uint64_t)valq * (uint64_t)(rms.den * rms.den);
            const __uint128_t rhs = (__uint128_t)(uint64_t)(16 * den * den * (int64_t)n * n) *
                                    (uint64_t)((int64_t)rms.num * rms.num);
            split = lhs > rhs;
        }
        d.cxy[r] = v;
        d.csplit[r] = (uint8_t)split;
        d.cdom[r] = (uint32_t)bp;
        d.ciso[r] = (uint8_t)t_best;
        d.csidx[r] = (uint8_t)bk;
        d.coff[r] = (uint8_t)o;
        d.cerr[r] = valq;
    }
}

hipError_t launch_finalize_b(const BatchHost &b, hipStream_t st) {
    k_finalize<<<max(1, b.blocks[K_FINAL]), 256, 0, st>>>(b.dev, b.ss, b.rms, b.is_last);
    return hipGetLastError();
}

// ---------------------------------------------------------------- children
struct ChildOp {
    int mult = 4;
    __device__ int items(const ImgLvl &d) const { return min(*d.ccount, d.range_cap); }
    __device__ bool pred(const ImgLvl &d, int i) const { return d.csplit[i] != 0; }
    __device__ void emit(const ImgLvl &d, int i, int pos) const {
        const uint32_t v = d.cxy[i];
        const uint32_t x = v & 0xffff, y = v >> 16, h = d.B / 2;
        d.children[4 * pos + 0] = (y << 16) | x;
        d.children[4 * pos + 1] = (y << 16) | (x + h);
        d.children[4 * pos + 2] = ((y + h) << 16) | x;
        d.children[4 * pos + 3] = ((y + h) << 16) | (x + h);
    }
    __device__ int *sums(const ImgLvl &d) const { return d.cblocksum; }
    __device__ int *offs(const ImgLvl &d) const { return d.cblockoff; }
    __device__ int32_t *total(const ImgLvl &d) const { return d.nchildren; }
};

hipError_t launch_children_b(const BatchHost &b, hipStream_t st) {
    return compact_b(b.dev, K_CCMP, b.blocks[K_CCMP], ChildOp{}, st);
}

}  // namespace fic
