// Quadtree level plumbing (Sec. 2, Fig 1; Sec. 3.3): level-0 ranges, range
// moments for the prune test, the per-range code (argmin merge, isometry
// fix-up, stored offset, split rule) and the child list.
#include "fic_internal.h"
#include "scan_util.h"

namespace fic {

__global__ __launch_bounds__(1024) void k_scan_blocks(int nb, const int *__restrict__ blocksum,
                                                      int *__restrict__ blockoff, int32_t *total_out, int mult) {
    __shared__ int wsum[16];
    __shared__ int carry_s;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int v = base + t < nb ? blocksum[base + t] : 0;
        const int incl = wave_incl_scan(v);
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int before = 0, all = 0;
        for (int i = 0; i < 16; ++i) {
            before += i < w ? wsum[i] : 0;
            all += wsum[i];
        }
        const int carry = carry_s;
        if (base + t < nb) blockoff[base + t] = carry + before + incl - v;
        __syncthreads();
        if (t == 0) carry_s = carry + all;
        __syncthreads();
    }
    if (t == 0) *total_out = carry_s * mult;
}

hipError_t launch_scan_blocks(int nb, const int *blocksum, int *blockoff, int32_t *total_out, int mult,
                              hipStream_t st) {
    k_scan_blocks<<<1, 1024, 0, st>>>(nb, blocksum, blockoff, total_out, mult);
    return hipGetLastError();
}

// ---------------------------------------------------------------- level 0
__global__ __launch_bounds__(256) void k_level0(int nx, int ny, int B, uint32_t *__restrict__ xy, int32_t *count) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r == 0) *count = nx * ny;
    if (r >= nx * ny) return;
    const int ry = r / nx, rx = r - ry * nx;
    xy[r] = ((uint32_t)(ry * B) << 16) | (uint32_t)(rx * B);
}

hipError_t launch_level0(int nx, int ny, int B, uint32_t *xy, int32_t *count, hipStream_t st) {
    k_level0<<<max(1, (nx * ny + 255) / 256), 256, 0, st>>>(nx, ny, B, xy, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------- range moments
// One wave per range.  The prune margin is n/4 + 4 in units of C'; the float
// rounding of the prune test is below n/16 in the same units.
__global__ __launch_bounds__(256) void k_range_info(const uint8_t *__restrict__ img, int pitch, int B,
                                                    const uint32_t *__restrict__ xy, const int32_t *nr, int cap,
                                                    RInfo *__restrict__ ri) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + w;
    if (r >= min(*nr, cap)) return;
    const uint32_t v = xy[r];
    const int x0 = v & 0xffff, y0 = v >> 16;
    const int n = B * B;
    int s = 0, ss = 0;
    for (int i = lane; i < n; i += 64) {
        const int y = i / B, x = i - y * B;
        const int p = img[(size_t)(y0 + y) * pitch + x0 + x];
        s += p;
        ss += p * p;
    }
    s = wave_sum_i32(s);
    ss = wave_sum_i32(ss);
    if (lane == 0) {
        RInfo o;
        o.cr = (int64_t)n * ss - (int64_t)s * s;
        o.sr = s;
        o.bn = (float)(128.0 - (double)s / n);
        o.an = (float)(512.0 * s - 65536.0 * n + (n / 4 + 4));
        o.pad = 0.f;
        ri[r] = o;
    }
}

hipError_t launch_range_info(const uint8_t *img, int pitch, int B, const uint32_t *xy, const int32_t *n, int cap,
                             RInfo *ri, hipStream_t st) {
    if (cap > 0) k_range_info<<<(cap + 3) / 4, 256, 0, st>>>(img, pitch, B, xy, n, cap, ri);
    return hipGetLastError();
}

// ---------------------------------------------------------------- finalize
__device__ inline bool lex_less(int64_t va, int pa, int64_t vb, int pb) { return va < vb || (va == vb && pa < pb); }

// One wave per range: merge the chunk partials in (val, domain) order, pick
// the isometry (the lowest t of maximal cross term, or t = 0 when the chosen
// contrast is 0 and every isometry ties), then the offset, val_q and split.
__global__ __launch_bounds__(256) void k_finalize(const uint8_t *__restrict__ img, int pitch, int B,
                                                  const uint32_t *__restrict__ xy, const int32_t *nr, int cap,
                                                  const uint32_t *__restrict__ pool_xy, const int32_t *np, int pool_cap,
                                                  const Partial *__restrict__ part,
                                                  int nchunk, SSet ss, fic_ratio rms, int is_last,
                                                  int32_t *out_count, uint32_t *out_xy, uint8_t *out_split,
                                                  uint32_t *out_dom, uint8_t *out_iso, uint8_t *out_sidx,
                                                  uint8_t *out_off, int64_t *out_err) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int R = min(*nr, cap);
    if (blockIdx.x == 0 && threadIdx.x == 0) *out_count = R;
    const int r = blockIdx.x * 4 + w;
    if (r >= R) return;
    int64_t bv = INT64_MAX;
    int bp = INT32_MAX, bk = 0;
    for (int c = lane; c < nchunk; c += 64) {
        const Partial q = part[(size_t)r * nchunk + c];
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
    const uint32_t v = xy[r];
    const int x0 = v & 0xffff, y0 = v >> 16;
    const int n = B * B;
    int64_t sr = 0;
    for (int i = lane; i < n; i += 64) {
        const int y = i / B, x = i - y * B;
        sr += img[(size_t)(y0 + y) * pitch + x0 + x];
    }
    sr = wave_sum_i64(sr);
    // every lane's first domain always passes the prune test, so bp is a
    // valid pool index whenever the pool is non-empty; stay in bounds anyway
    const int P = min(*np, pool_cap);
    if (bp < 0 || bp >= P) {
        bp = 0;
        bk = 0;
    }
    int nk = 0;
    for (int j = 0; j < ss.count; ++j)
        if (j == bk) nk = ss.num[j];
    int t_best = 0;
    if (nk != 0) {
        const uint32_t dv = pool_xy[bp];
        const int dx0 = dv & 0xffff, dy0 = dv >> 16;
        int64_t x4[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) x4[t] = 0;
        for (int i = lane; i < n; i += 64) {
            const int y = i / B, x = i - y * B;
            const int rv = img[(size_t)(y0 + y) * pitch + x0 + x];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                int cy, cx;
                iso_src(t, B, y, x, cy, cx);
                const uint8_t *q = img + (size_t)(dy0 + 2 * cy) * pitch + dx0 + 2 * cx;
                x4[t] += (int64_t)rv * (q[0] + q[1] + q[pitch] + q[pitch + 1]);
            }
        }
        int64_t best = 0;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int64_t s = wave_sum_i64(x4[t]);
            if (t == 0 || s > best) {
                best = s;
                t_best = t;
            }
        }
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
        out_xy[r] = v;
        out_split[r] = (uint8_t)split;
        out_dom[r] = (uint32_t)bp;
        out_iso[r] = (uint8_t)t_best;
        out_sidx[r] = (uint8_t)bk;
        out_off[r] = (uint8_t)o;
        out_err[r] = valq;
    }
}

hipError_t launch_finalize(const uint8_t *img, int pitch, int B, const uint32_t *xy, const int32_t *n, int cap,
                           const fic_pool *pool, const Partial *part, int nchunk, SSet ss, fic_ratio rms,
                           int is_last, fic_level_codes *out, hipStream_t st) {
    k_finalize<<<max(1, (cap + 3) / 4), 256, 0, st>>>(img, pitch, B, xy, n, cap, pool->xy, pool->count,
                                                      pool->capacity, part, nchunk, ss, rms,
                                                      is_last, out->count, out->xy, out->split, out->domain,
                                                      out->iso, out->s_idx, out->offset, out->err);
    return hipGetLastError();
}

// ---------------------------------------------------------------- children
struct SplitPred {
    const uint8_t *split;
    __device__ bool operator()(int i) const { return split[i] != 0; }
};

struct ChildEmit {
    const uint32_t *xy;
    int h;
    uint32_t *out;
    __device__ void operator()(int i, int pos) const {
        const uint32_t v = xy[i];
        const uint32_t x = v & 0xffff, y = v >> 16;
        out[4 * pos + 0] = (y << 16) | x;
        out[4 * pos + 1] = (y << 16) | (x + h);
        out[4 * pos + 2] = ((y + h) << 16) | x;
        out[4 * pos + 3] = ((y + h) << 16) | (x + h);
    }
};

hipError_t launch_children(const fic_level_codes *codes, int cap, int B, int *blocksum, int *blockoff,
                           uint32_t *children, int32_t *n_children, hipStream_t st) {
    SplitPred pred{codes->split};
    ChildEmit emit{codes->xy, B / 2, children};
    return compact(cap, codes->count, pred, emit, blocksum, blockoff, n_children, 4, st);
}

}  // namespace fic
