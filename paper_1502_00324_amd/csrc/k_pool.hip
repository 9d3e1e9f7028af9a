// Domain pool (Sec. 3, Eq 5-6; Sec. 3.2.1) for every image of a batch: entropy
// key per candidate, radix selection of the thresholds on the device, stable
// compaction in raster order, domain moments.
#include "fic_internal.h"
#include "scan_util.h"

namespace fic {

// ---------------------------------------------------------------- keys
// G = sum over gray levels of T[count]; a larger G means a lower entropy.
// One wave per strip: lane l owns candidate column cx = 64 gx + l and slides
// its window down over d.strip candidate rows (1..16, chosen per image so
// small images still give the GPU enough waves).  Each lane keeps a private
// 256-bin histogram in LDS (layout [bin][lane], no atomics) and updates G
// incrementally: adding a pixel whose bin held c adds T[c+1] - T[c].
// DSZ = 2B is the window side; the differences T[c+1] - T[c] sit in LDS up to
// 1024 pixels per window, else they are read from the table.
template <int DSZ>
__global__ __launch_bounds__(64) void k_pool_keys(BatchDev b, const int64_t *__restrict__ table) {
    constexpr int M = DSZ * DSZ, NW = DSZ / 4;   // window pixels, 4-byte words per window row
    constexpr bool LT = M <= 1024;
    __shared__ uint16_t hist[256][64];
    __shared__ int64_t dtab[LT ? M : 1];
    const gptr<int64_t> T = as_global(table);
    const int *pre = b.pre + K_KEYS * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int lb = blockIdx.x - pre[im];
    const int ngx = (d.nx + 63) / 64;
    const int gx = lb % ngx, gy = lb / ngx;
    const int lane = threadIdx.x;
    const int L = d.L, pitch = d.pitch, nx = d.nx;
    if constexpr (LT)
        for (int c = lane; c < M; c += 64) dtab[c] = T[c + 1] - T[c];
    for (int v = 0; v < 256; ++v) hist[v][lane] = 0;
    __syncthreads();
    const int cx = gx * 64 + lane;
    const int cy0 = gy * d.strip;
    const int cy1 = min(d.ny, cy0 + d.strip);
    // inactive lanes stay for the wave reduction below
    const bool active = cx < nx && cy0 < d.ny;
    const gptr<uint8_t> col = as_global(d.pix) + (size_t)(active ? cx : 0) * L;
    uint16_t *h = &hist[0][lane];
    auto dlt = [&](int c) -> int64_t {
        if constexpr (LT)
            return dtab[c];
        else
            return T[c + 1] - T[c];
    };
    int64_t g = 0, gm = INT64_MAX;
    // a window row as 4-byte words (unaligned loads)
    typedef uint32_t u32u __attribute__((aligned(1)));
    auto load_row = [&](uint32_t (&w)[NW], int y) {
        const gptr<u32u> row = (gptr<u32u>)(col + (size_t)y * pitch);
#pragma unroll
        for (int k = 0; k < NW; ++k) w[k] = row[k];
    };
    // Four pixels per step: their four counts are read together, one LDS
    // round trip instead of four.  A pixel equal to an earlier one of the
    // group takes that one's update through the equality terms, and the
    // writes, in program order, leave the last count.
    auto apply_row = [&](const uint32_t (&w)[NW], bool add) {
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const uint32_t x = w[k];
            const int v0 = x & 255, v1 = (x >> 8) & 255, v2 = (x >> 16) & 255, v3 = x >> 24;
            int c0 = h[v0 * 64], c1 = h[v1 * 64], c2 = h[v2 * 64], c3 = h[v3 * 64];
            const int e1 = v1 == v0, e2 = (v2 == v0) + (v2 == v1), e3 = (v3 == v0) + (v3 == v1) + (v3 == v2);
            if (add) {
                c1 += e1;
                c2 += e2;
                c3 += e3;
                g += dlt(c0) + dlt(c1) + dlt(c2) + dlt(c3);
                h[v0 * 64] = (uint16_t)(c0 + 1);
                h[v1 * 64] = (uint16_t)(c1 + 1);
                h[v2 * 64] = (uint16_t)(c2 + 1);
                h[v3 * 64] = (uint16_t)(c3 + 1);
            } else {
                c1 -= e1;
                c2 -= e2;
                c3 -= e3;
                g -= dlt(c0 - 1) + dlt(c1 - 1) + dlt(c2 - 1) + dlt(c3 - 1);
                h[v0 * 64] = (uint16_t)(c0 - 1);
                h[v1 * 64] = (uint16_t)(c1 - 1);
                h[v2 * 64] = (uint16_t)(c2 - 1);
                h[v3 * 64] = (uint16_t)(c3 - 1);
            }
        }
    };
    // A sequence of row operations (row of op o, add or remove), each row
    // loaded one operation ahead of its use.  Every removal follows the
    // addition of its row, so no count goes below zero.
    auto run = [&](int nops, auto row_of, auto add_of) {
        uint32_t w0[NW], w1[NW];
        load_row(w0, row_of(0));
        for (int o = 0; o < nops; o += 2) {
            if (o + 1 < nops) load_row(w1, row_of(o + 1));
            apply_row(w0, add_of(o));
            if (o + 2 < nops) load_row(w0, row_of(o + 2));
            if (o + 1 < nops) apply_row(w1, add_of(o + 1));
        }
    };
    if (active) {
        int ytop = cy0 * L;
        run(DSZ, [&](int o) { return ytop + o; }, [](int) { return true; });
        d.keys[(size_t)cy0 * nx + cx] = g;
        gm = g;
        for (int cy = cy0 + 1; cy < cy1; ++cy) {
            const int ynew = cy * L;
            if (L < DSZ) {
                // slide by L rows: remove row ytop + r, then add row ytop + DSZ + r
                run(2 * L, [&](int o) { return ytop + (o >> 1) + (o & 1) * DSZ; },
                    [](int o) { return (o & 1) != 0; });
            } else {
                run(2 * DSZ, [&](int o) { return o < DSZ ? ytop + o : ynew + o - DSZ; },
                    [](int o) { return o >= DSZ; });
            }
            ytop = ynew;
            d.keys[(size_t)cy * nx + cx] = g;
            gm = min(gm, g);
        }
    }
    // wave minimum, then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(gm, off, 64);
        gm = min(gm, o);
    }
    if (lane == 0) atomicMin(&d.sel->gmin, (unsigned long long)gm);
}

// Variance key (the alternative pool cited in Sec. 1): one thread per
// candidate, from the summed-area tables; 2^47 - (M sum p^2 - (sum p)^2), so a
// smaller key means a larger variance and the selection below is unchanged.
__global__ __launch_bounds__(256) void k_pool_keys_var(BatchDev b) {
    const int *pre = b.pre + K_KEYS * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int i = (blockIdx.x - pre[im]) * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int64_t key = INT64_MAX;
    if (i < d.nd) {
        const int cy = i / d.nx, cx = i - cy * d.nx;
        const int x = cx * d.L, y = cy * d.L, size = 2 * d.B;
        const IntegGeom g = integ_geom(d.W, d.H);
        const int64_t s = box_sum(g.si(d.integ), g.ws, x, y, size, size);
        const int64_t ss = box_sum(g.sii(d.integ), g.ws, x, y, size, size);
        key = ((int64_t)1 << 47) - ((int64_t)size * size * ss - s * s);
        d.keys[i] = key;
    }
    // wave minimum, then one atomic per wave
    int64_t gm = key;
    for (int off = 32; off > 0; off >>= 1) gm = min(gm, (int64_t)__shfl_xor(gm, off, 64));
    if (lane == 0 && gm != INT64_MAX) atomicMin(&d.sel->gmin, (unsigned long long)gm);
}

// ---------------------------------------------------------------- radix select
// Passes 0..5 pick the key 8 bits at a time (keys < 2^48); passes 6..9 pick
// the candidate index (< 2^32).  The percentile select finds the c-th largest
// key; the pool-size select the pool_max-th smallest (key, index) pair among
// the candidates the percentile keeps.
__device__ inline bool pct_keep(int64_t key, const PoolSel *sel, int64_t c) {
    if (c == 0) return true;
    const unsigned long long t = sel->pct.key_prefix;
    return (unsigned long long)key < t || (t == sel->gmin && (unsigned long long)key == sel->gmin);
}

__global__ __launch_bounds__(256) void k_sel_init(BatchDev b) {
    const ImgLvl &d = b.d[blockIdx.x];
    PoolSel *sel = d.sel;
    const int t = threadIdx.x;
    sel->pct.hist[t] = 0;
    sel->cap.hist[t] = 0;
    if (t == 0) {
        sel->pct.key_prefix = 0;
        sel->pct.idx_prefix = 0;
        sel->pct.remaining = (int32_t)d.c;
        sel->pct.all = d.c == 0 ? 1 : 0;
        sel->cap.key_prefix = 0;
        sel->cap.idx_prefix = 0;
        sel->cap.remaining = d.pool_max;
        sel->cap.all = d.pool_max == 0 ? 1 : 0;
        sel->gmin = ~0ull;
    }
}

// which = 0: percentile select (all candidates); 1: pool-size select (filtered)
__global__ __launch_bounds__(256) void k_sel_hist(BatchDev b, int pass, int which) {
    __shared__ uint32_t h[256];
    const int *pre = b.pre + K_HIST * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int lb = blockIdx.x - pre[im], nb = pre[im + 1] - pre[im];
    SelState *st = which ? &d.sel->cap : &d.sel->pct;
    h[threadIdx.x] = 0;
    __syncthreads();
    if (st->all) return;  // uniform: every thread reads the same flag
    const unsigned long long kp = st->key_prefix;
    const uint32_t ip = st->idx_prefix;
    for (int i = lb * 256 + threadIdx.x; i < d.nd; i += nb * 256) {
        const int64_t key = d.keys[i];
        if (which && !pct_keep(key, d.sel, d.c)) continue;
        uint32_t dg;
        if (pass < 6) {
            const int sh = 40 - 8 * pass;
            if (((unsigned long long)key >> (sh + 8)) != (kp >> (sh + 8))) continue;
            dg = (uint32_t)(((unsigned long long)key >> sh) & 255u);
        } else {
            const int sh = 24 - 8 * (pass - 6);
            if ((unsigned long long)key != kp) continue;
            if (sh < 24 && ((uint32_t)i >> (sh + 8)) != (ip >> (sh + 8))) continue;
            dg = ((uint32_t)i >> sh) & 255u;
        }
        atomicAdd(&h[dg], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_sel_pick(BatchDev b, int pass, int which) {
    __shared__ uint32_t cum[256];
    const ImgLvl &d = b.d[blockIdx.x];
    SelState *st = which ? &d.sel->cap : &d.sel->pct;
    const int largest = which ? 0 : 1;
    const int t = threadIdx.x;
    if (st->all) return;  // uniform
    // position t in the scan order: descending digits when looking for the largest
    const int dg = largest ? 255 - t : t;
    const uint32_t cnt = st->hist[dg];
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
    st->hist[dg] = 0;
    if (pass == 0 && total < (uint32_t)rem) {
        if (t == 0) st->all = 1;
        return;
    }
    if (excl < (uint32_t)rem && (uint32_t)rem <= incl) {
        st->remaining = rem - (int32_t)excl;
        if (pass < 6) st->key_prefix |= (unsigned long long)dg << (40 - 8 * pass);
        else st->idx_prefix |= (uint32_t)dg << (24 - 8 * (pass - 6));
    }
}

// All select passes of one image in one 1024-thread workgroup (levels whose
// images have few candidates): the same digit-by-digit selection as
// k_sel_hist / k_sel_pick, with the histogram and the selection state in LDS,
// so a level's selection is one launch instead of 12 (or 32 with a cap).
__global__ __launch_bounds__(1024) void k_sel_fused(BatchDev b) {
    __shared__ uint32_t h[256], cum[256];
    __shared__ unsigned long long kpre[2];
    __shared__ uint32_t ipre[2];
    __shared__ int32_t rem[2], all[2];
    const ImgLvl &d = b.d[blockIdx.x];
    const int t = threadIdx.x;
    const unsigned long long gmin = d.sel->gmin;
    if (t == 0) {
        kpre[0] = kpre[1] = 0;
        ipre[0] = ipre[1] = 0;
        rem[0] = (int32_t)d.c;
        all[0] = d.c == 0 ? 1 : 0;
        rem[1] = d.pool_max;
        all[1] = d.pool_max == 0 ? 1 : 0;
    }
    __syncthreads();
    for (int which = 0; which < 2; ++which) {
        const int largest = which ? 0 : 1;
        for (int pass = 0; pass < (which ? 10 : 6); ++pass) {
            if (all[which]) break;  // uniform: read after a barrier
            if (t < 256) h[t] = 0;
            const unsigned long long kp = kpre[which];
            const uint32_t ip = ipre[which];
            __syncthreads();
            for (int i = t; i < d.nd; i += 1024) {
                const int64_t key = d.keys[i];
                if (which) {   // the percentile step's survivors only
                    const unsigned long long tk = kpre[0];
                    const bool keep = d.c == 0 || (unsigned long long)key < tk ||
                                      (tk == gmin && (unsigned long long)key == gmin);
                    if (!keep) continue;
                }
                uint32_t dg;
                if (pass < 6) {
                    const int sh = 40 - 8 * pass;
                    if (((unsigned long long)key >> (sh + 8)) != (kp >> (sh + 8))) continue;
                    dg = (uint32_t)(((unsigned long long)key >> sh) & 255u);
                } else {
                    const int sh = 24 - 8 * (pass - 6);
                    if ((unsigned long long)key != kp) continue;
                    if (sh < 24 && ((uint32_t)i >> (sh + 8)) != (ip >> (sh + 8))) continue;
                    dg = ((uint32_t)i >> sh) & 255u;
                }
                atomicAdd(&h[dg], 1u);
            }
            __syncthreads();
            // scan in the order of the wanted digits (descending for the largest)
            int dgt = 0;
            uint32_t cnt = 0;
            if (t < 256) {
                dgt = largest ? 255 - t : t;
                cnt = h[dgt];
                cum[t] = cnt;
            }
            __syncthreads();
            for (int off = 1; off < 256; off <<= 1) {
                const uint32_t v = (t < 256 && t >= off) ? cum[t - off] : 0u;
                __syncthreads();
                if (t < 256) cum[t] += v;
                __syncthreads();
            }
            const int32_t r = rem[which];
            const uint32_t total = cum[255];
            __syncthreads();  // every thread has read rem before it changes
            if (t < 256) {
                const uint32_t incl = cum[t], excl = incl - cnt;
                if (pass == 0 && total < (uint32_t)r) {
                    if (t == 0) all[which] = 1;
                } else if (excl < (uint32_t)r && (uint32_t)r <= incl) {
                    rem[which] = r - (int32_t)excl;
                    if (pass < 6) kpre[which] |= (unsigned long long)dgt << (40 - 8 * pass);
                    else ipre[which] |= (uint32_t)dgt << (24 - 8 * (pass - 6));
                }
            }
            __syncthreads();
        }
    }
    if (t == 0) {
        SelState *st[2] = {&d.sel->pct, &d.sel->cap};
        for (int w = 0; w < 2; ++w) {
            st[w]->key_prefix = kpre[w];
            st[w]->idx_prefix = ipre[w];
            st[w]->remaining = rem[w];
            st[w]->all = all[w];
        }
    }
}

// ---------------------------------------------------------------- compaction
struct PoolOp {
    int mult = 1;
    __device__ int items(const ImgLvl &d) const { return d.nd; }
    __device__ bool pred(const ImgLvl &d, int i) const {
        const int64_t key = d.keys[i];
        if (!pct_keep(key, d.sel, d.c)) return false;
        if (d.pool_max == 0 || d.sel->cap.all) return true;
        const unsigned long long tk = d.sel->cap.key_prefix;
        const uint32_t ti = d.sel->cap.idx_prefix;
        return (unsigned long long)key < tk || ((unsigned long long)key == tk && (uint32_t)i <= ti);
    }
    __device__ void emit(const ImgLvl &d, int i, int pos) const {
        const int cy = i / d.nx, cx = i - cy * d.nx;
        d.pxy[pos] = ((uint32_t)(cy * d.L) << 16) | (uint32_t)(cx * d.L);
        d.pkey[pos] = d.keys[i];
    }
    __device__ int *sums(const ImgLvl &d) const { return d.pblocksum; }
    __device__ int *offs(const ImgLvl &d) const { return d.pblockoff; }
    __device__ int32_t *total(const ImgLvl &d) const { return d.pcount; }
};

// Per pool entry: Sd4 = sum of the raw pixels and A = n*sum(D4^2) - (sum D4)^2,
// each a box of the image's summed-area tables (one thread per entry).
__global__ __launch_bounds__(256) void k_pool_moments(BatchDev b) {
    const int *pre = b.pre + K_MOM * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int p = (blockIdx.x - pre[im]) * 256 + threadIdx.x;
    if (p >= min(*d.pcount, d.pool_cap)) return;
    const int B = d.B;
    const uint32_t v = d.pxy[p];
    const int x0 = v & 0xffff, y0 = v >> 16;
    const IntegGeom g = integ_geom(d.W, d.H);
    const int64_t s = box_sum(g.si(d.integ), g.ws, x0, y0, 2 * B, 2 * B);
    const int64_t ss = box_sum(g.sq(d.integ, 2 * (y0 & 1) + (x0 & 1)), g.wq, x0 >> 1, y0 >> 1, B, B);
    d.psum4[p] = (uint32_t)s;
    d.pa[p] = (int64_t)B * B * ss - s * s;
}

// ---------------------------------------------------------------- launcher
hipError_t launch_pool_b(const BatchHost &b, const int64_t *table, hipStream_t st) {
    const BatchDev &dv = b.dev;
    k_sel_init<<<dv.n, 256, 0, st>>>(dv);
    if (b.blocks[K_KEYS] > 0) {
        if (b.pool_key == FIC_POOL_VARIANCE) k_pool_keys_var<<<b.blocks[K_KEYS], 256, 0, st>>>(dv);
        else {
            switch (b.B) {
                case 2: k_pool_keys<4><<<b.blocks[K_KEYS], 64, 0, st>>>(dv, table); break;
                case 4: k_pool_keys<8><<<b.blocks[K_KEYS], 64, 0, st>>>(dv, table); break;
                case 8: k_pool_keys<16><<<b.blocks[K_KEYS], 64, 0, st>>>(dv, table); break;
                case 16: k_pool_keys<32><<<b.blocks[K_KEYS], 64, 0, st>>>(dv, table); break;
                case 32: k_pool_keys<64><<<b.blocks[K_KEYS], 64, 0, st>>>(dv, table); break;
                default: return hipErrorInvalidValue;
            }
        }
    }
    if (b.fused_sel) {
        k_sel_fused<<<dv.n, 1024, 0, st>>>(dv);
    } else {
        for (int pass = 0; pass < 6; ++pass) {
            k_sel_hist<<<b.blocks[K_HIST], 256, 0, st>>>(dv, pass, 0);
            k_sel_pick<<<dv.n, 256, 0, st>>>(dv, pass, 0);
        }
        if (b.any_cap)
            for (int pass = 0; pass < 10; ++pass) {
                k_sel_hist<<<b.blocks[K_HIST], 256, 0, st>>>(dv, pass, 1);
                k_sel_pick<<<dv.n, 256, 0, st>>>(dv, pass, 1);
            }
    }
    hipError_t e = compact_b(dv, K_PCMP, b.blocks[K_PCMP], PoolOp{}, st);
    if (e != hipSuccess) return e;
    if (b.blocks[K_MOM] > 0) k_pool_moments<<<b.blocks[K_MOM], 256, 0, st>>>(dv);
    return hipGetLastError();
}

}  // namespace fic
