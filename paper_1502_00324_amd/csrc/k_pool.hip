// Domain pool (Sec. 3, Eq 5-6; Sec. 3.2.1): entropy key per candidate, radix
// selection of the thresholds on the device, stable compaction in raster order.
#include "fic_internal.h"
#include "scan_util.h"

namespace fic {

// ---------------------------------------------------------------- keys
// G = sum over gray levels of T[count]; a larger G means a lower entropy.
// One wave per strip: lane l owns candidate column cx = 64*bx + l and slides
// its window down over S candidate rows.  Each lane keeps a private 256-bin
// histogram in LDS (layout [bin][lane], no atomics) and updates G
// incrementally: adding a pixel whose bin held c adds T[c+1] - T[c].
constexpr int kStripRows = 16;

__global__ __launch_bounds__(64) void k_pool_keys(const uint8_t *__restrict__ img, int pitch, int nx, int ny, int L,
                                                  int dsz, const int64_t *__restrict__ T,
                                                  int64_t *__restrict__ keys, unsigned long long *gmin) {
    __shared__ uint16_t hist[256][64];
    __shared__ int64_t dtab[1025];
    const int lane = threadIdx.x;
    const int M = dsz * dsz;
    const bool lds_tab = M <= 1024;
    if (lds_tab)
        for (int c = lane; c < M; c += 64) dtab[c] = T[c + 1] - T[c];
    for (int v = 0; v < 256; ++v) hist[v][lane] = 0;
    __syncthreads();
    const int cx = blockIdx.x * 64 + lane;
    const int cy0 = blockIdx.y * kStripRows;
    const int cy1 = min(ny, cy0 + kStripRows);
    // inactive lanes stay for the wave reduction below
    const bool active = cx < nx && cy0 < ny;
    const uint8_t *col = img + (size_t)(active ? cx : 0) * L;
    uint16_t *h = &hist[0][lane];
    auto dlt = [&](int c) -> int64_t { return lds_tab ? dtab[c] : T[c + 1] - T[c]; };
    int64_t g = 0, gm = INT64_MAX;
    auto add_row = [&](int y) {
        const uint8_t *row = col + (size_t)y * pitch;
        for (int i = 0; i < dsz; ++i) {
            const int v = row[i];
            const int c = h[v * 64];
            g += dlt(c);
            h[v * 64] = (uint16_t)(c + 1);
        }
    };
    auto remove_row = [&](int y) {
        const uint8_t *row = col + (size_t)y * pitch;
        for (int i = 0; i < dsz; ++i) {
            const int v = row[i];
            const int c = h[v * 64];
            g -= dlt(c - 1);
            h[v * 64] = (uint16_t)(c - 1);
        }
    };
    if (active) {
        int ytop = cy0 * L;
        for (int r = 0; r < dsz; ++r) add_row(ytop + r);
        keys[(size_t)cy0 * nx + cx] = g;
        gm = g;
        for (int cy = cy0 + 1; cy < cy1; ++cy) {
            const int ynew = cy * L;
            if (L < dsz) {
                for (int r = 0; r < L; ++r) {
                    remove_row(ytop + r);
                    add_row(ytop + dsz + r);
                }
            } else {
                for (int r = 0; r < dsz; ++r) remove_row(ytop + r);
                for (int r = 0; r < dsz; ++r) add_row(ynew + r);
            }
            ytop = ynew;
            keys[(size_t)cy * nx + cx] = g;
            gm = min(gm, g);
        }
    }
    // wave minimum, then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(gm, off, 64);
        gm = min(gm, o);
    }
    if (lane == 0) atomicMin(gmin, (unsigned long long)gm);
}

// ---------------------------------------------------------------- radix select
// Passes 0..5 pick the key 8 bits at a time (keys < 2^48); passes 6..9 pick
// the candidate index (< 2^32).  largest = 1 finds the k-th largest key, 0 the
// k-th smallest (key, index) pair.  filter = 1 restricts to candidates kept by
// the percentile threshold.
__device__ inline bool pct_keep(int64_t key, const PoolSel *sel, int64_t c) {
    if (c == 0) return true;
    const unsigned long long t = sel->pct.key_prefix;
    return (unsigned long long)key < t || (t == sel->gmin && (unsigned long long)key == sel->gmin);
}

__global__ __launch_bounds__(256) void k_sel_init(PoolSel *sel, int64_t c, int pool_max) {
    const int t = threadIdx.x;
    sel->pct.hist[t] = 0;
    sel->cap.hist[t] = 0;
    if (t == 0) {
        sel->pct.key_prefix = 0;
        sel->pct.idx_prefix = 0;
        sel->pct.remaining = (int32_t)c;
        sel->pct.all = c == 0 ? 1 : 0;
        sel->cap.key_prefix = 0;
        sel->cap.idx_prefix = 0;
        sel->cap.remaining = pool_max;
        sel->cap.all = pool_max == 0 ? 1 : 0;
        sel->gmin = ~0ull;
    }
}

__global__ __launch_bounds__(256) void k_sel_hist(const int64_t *__restrict__ keys, int nd, int pass, int filter,
                                                  int64_t c, PoolSel *sel, SelState *st) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    if (st->all) return;  // uniform: every thread reads the same flag
    const unsigned long long kp = st->key_prefix;
    const uint32_t ip = st->idx_prefix;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < nd; i += gridDim.x * 256) {
        const int64_t key = keys[i];
        if (filter && !pct_keep(key, sel, c)) continue;
        uint32_t d;
        if (pass < 6) {
            const int sh = 40 - 8 * pass;
            if (((unsigned long long)key >> (sh + 8)) != (kp >> (sh + 8))) continue;
            d = (uint32_t)(((unsigned long long)key >> sh) & 255u);
        } else {
            const int sh = 24 - 8 * (pass - 6);
            if ((unsigned long long)key != kp) continue;
            if (sh < 24 && ((uint32_t)i >> (sh + 8)) != (ip >> (sh + 8))) continue;
            d = ((uint32_t)i >> sh) & 255u;
        }
        atomicAdd(&h[d], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_sel_pick(int pass, int largest, SelState *st) {
    __shared__ uint32_t cum[256];
    const int t = threadIdx.x;
    if (st->all) return;  // uniform
    // position t in the scan order: descending digits when looking for the largest
    const int d = largest ? 255 - t : t;
    const uint32_t cnt = st->hist[d];
    cum[t] = cnt;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = t >= off ? cum[t - off] : 0u;
        __syncthreads();
        cum[t] += v;
        __syncthreads();
    }
    const uint32_t incl = cum[t], excl = incl - cnt, total = cum[255];
    const int32_t rem = st->remaining;
    __syncthreads();
    st->hist[d] = 0;
    if (pass == 0 && total < (uint32_t)rem) {
        if (t == 0) st->all = 1;
        return;
    }
    if (excl < (uint32_t)rem && (uint32_t)rem <= incl) {
        st->remaining = rem - (int32_t)excl;
        if (pass < 6) st->key_prefix |= (unsigned long long)d << (40 - 8 * pass);
        else st->idx_prefix |= (uint32_t)d << (24 - 8 * (pass - 6));
    }
}

// ---------------------------------------------------------------- compaction
struct PoolPred {
    const int64_t *keys;
    const PoolSel *sel;
    int64_t c;
    int pool_max;
    __device__ bool operator()(int i) const {
        const int64_t key = keys[i];
        if (!pct_keep(key, sel, c)) return false;
        if (pool_max == 0 || sel->cap.all) return true;
        const unsigned long long tk = sel->cap.key_prefix;
        const uint32_t ti = sel->cap.idx_prefix;
        return (unsigned long long)key < tk || ((unsigned long long)key == tk && (uint32_t)i <= ti);
    }
};

struct PoolEmit {
    const int64_t *keys;
    int nx, L;
    uint32_t *xy;
    int64_t *key_out;
    __device__ void operator()(int i, int pos) const {
        const int cy = i / nx, cx = i - cy * nx;
        xy[pos] = ((uint32_t)(cy * L) << 16) | (uint32_t)(cx * L);
        key_out[pos] = keys[i];
    }
};

// Per pool entry: sum of the raw pixels and A = n*sum(D4^2) - (sum D4)^2.
__global__ __launch_bounds__(256) void k_pool_moments(const uint8_t *__restrict__ img, int pitch, int B, int cap,
                                                      const int32_t *count, const uint32_t *__restrict__ xy,
                                                      uint32_t *__restrict__ sum4, int64_t *__restrict__ a) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + w;
    if (p >= min(*count, cap)) return;
    const uint32_t v = xy[p];
    const int x0 = v & 0xffff, y0 = v >> 16;
    int64_t s = 0, ss = 0;
    for (int c = lane; c < B * B; c += 64) {
        const int cy = c / B, cx = c - cy * B;
        const uint8_t *q = img + (size_t)(y0 + 2 * cy) * pitch + x0 + 2 * cx;
        const int d4 = q[0] + q[1] + q[pitch] + q[pitch + 1];
        s += d4;
        ss += (int64_t)d4 * d4;
    }
    s = wave_sum_i64(s);
    ss = wave_sum_i64(ss);
    if (lane == 0) {
        sum4[p] = (uint32_t)s;
        a[p] = (int64_t)B * B * ss - s * s;
    }
}

// ---------------------------------------------------------------- launchers
// k_sel_init must run first on the stream: it resets gmin.
hipError_t launch_pool_keys(const uint8_t *img, int pitch, int nx, int nd, int L, int dsz, const int64_t *table,
                            int64_t *keys, PoolSel *sel, hipStream_t st) {
    const int ny = nx > 0 ? nd / nx : 0;
    const dim3 grid((nx + 63) / 64, (ny + kStripRows - 1) / kStripRows);
    if (nd > 0) k_pool_keys<<<grid, 64, 0, st>>>(img, pitch, nx, ny, L, dsz, table, keys, &sel->gmin);
    return hipGetLastError();
}

hipError_t launch_sel_init(PoolSel *sel, int64_t c, int pool_max, hipStream_t st) {
    k_sel_init<<<1, 256, 0, st>>>(sel, c, pool_max);
    return hipGetLastError();
}

hipError_t launch_pool_select(const int64_t *keys, int nd, int64_t c, int pool_max, PoolSel *sel, hipStream_t st) {
    const int blocks = max(1, min(1024, (nd + 255) / 256));
    if (c > 0)
        for (int pass = 0; pass < 6; ++pass) {
            k_sel_hist<<<blocks, 256, 0, st>>>(keys, nd, pass, 0, c, sel, &sel->pct);
            k_sel_pick<<<1, 256, 0, st>>>(pass, 1, &sel->pct);
        }
    if (pool_max > 0)
        for (int pass = 0; pass < 10; ++pass) {
            k_sel_hist<<<blocks, 256, 0, st>>>(keys, nd, pass, 1, c, sel, &sel->cap);
            k_sel_pick<<<1, 256, 0, st>>>(pass, 0, &sel->cap);
        }
    return hipGetLastError();
}

hipError_t launch_pool_compact(const int64_t *keys, int nd, int nx, int L, int64_t c, int pool_max,
                               const PoolSel *sel, int *blocksum, int *blockoff, fic_pool *pool, hipStream_t st) {
    PoolPred pred{keys, sel, c, pool_max};
    PoolEmit emit{keys, nx, L, pool->xy, pool->key};
    return compact(nd, nullptr, pred, emit, blocksum, blockoff, pool->count, 1, st);
}

hipError_t launch_pool_moments(const uint8_t *img, int pitch, int B, int cap, fic_pool *pool, hipStream_t st) {
    const int blocks = (cap + 3) / 4;
    if (blocks > 0)
        k_pool_moments<<<blocks, 256, 0, st>>>(img, pitch, B, cap, pool->count, pool->xy, pool->sum4, pool->a);
    return hipGetLastError();
}

}  // namespace fic
