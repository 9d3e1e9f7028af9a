// Plain per-pixel FP32 search engine: the baseline the MFMA engines are
// measured against, and the engine for range sizes a requested matrix engine
// has no form for.
//
// Per (range, isometry, domain) it sums (view_j - 128)(D4_j - 512) over the
// B^2 decimated cells in FP32 -- the same integer C' as the MFMA engine.
// Every product is an integer of magnitude <= 2^16 and every partial sum of
// up to 256 cells stays below 2^24, so FP32 is exact; for B = 32 the sums are
// flushed to int32 every 256 cells.  LDS-tiled: 8 ranges x 128 domains per
// 256-thread block, each thread 8 isometries x 4 domains in registers.
//
// Layouts: views vf[(j * Rpad + r) * 8 + t], domains df[j * Ppad + p], with j
// the decimated cell (row-major) and Rpad, Ppad padded to the tile sizes.
#include "fic_internal.h"
#include "search_common.h"

namespace fic {

constexpr int kF32Ranges = 8;
constexpr int kF32Doms = 128;

void fp32_geometry(int B, int range_cap, int pool_cap, int *nchunk, int *tiles_per_chunk) {
    (void)B;
    const int ntiles = (pool_cap + kF32Doms - 1) / kF32Doms;
    const int nrg = (range_cap + kF32Ranges - 1) / kF32Ranges;
    int nc = (4096 + nrg - 1) / nrg;
    nc = max(1, min(nc, max(1, ntiles / 4)));
    nc = min(nc, 4096);
    *nchunk = nc;
    *tiles_per_chunk = (ntiles + nc - 1) / nc;
}

int fp32_rpad(int range_cap) { return (range_cap + kF32Ranges - 1) / kF32Ranges * kF32Ranges; }
int fp32_ppad(int pool_cap) { return (pool_cap + kF32Doms - 1) / kF32Doms * kF32Doms; }

int fp32_blocks(int B, int range_cap, int pool_cap) {
    int nchunk, tpc;
    fp32_geometry(B, range_cap, pool_cap, &nchunk, &tpc);
    return (range_cap + kF32Ranges - 1) / kF32Ranges * nchunk;
}

__global__ __launch_bounds__(256) void k_fp32_views(BatchDev b) {
    const int *pre = b.pre + K_VIEWS * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    // 64-bit element index: B^2 x padded count passes 2^31 for large images
    const int64_t e = (int64_t)(blockIdx.x - pre[im]) * 256 + threadIdx.x;
    const int B = d.B, n = B * B, Rpad = d.rpad;
    if (e >= (int64_t)n * Rpad) return;
    // column js of the view array holds entry js of the search list
    const int j = (int)(e / Rpad), js = (int)(e - (int64_t)j * Rpad);
    const int cy = j / B, cx = j - cy * B;
    const bool valid = js < min(*d.ns, d.range_cap);
    int x0 = 0, y0 = 0;
    if (valid) {
        const uint32_t v = d.rxy[d.sidx[js]];
        x0 = v & 0xffff;
        y0 = v >> 16;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        float val = 0.f;
        if (valid) {
            int sy, sx;
            iso_src(iso_inv(t), B, cy, cx, sy, sx);
            val = (float)((int)d.pix[(size_t)(y0 + sy) * d.pitch + x0 + sx] - 128);
        }
        d.vf[(size_t)e * 8 + t] = val;
    }
}

__global__ __launch_bounds__(256) void k_fp32_doms(BatchDev b) {
    const int *pre = b.pre + K_DOMS * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    // 64-bit element index: B^2 x padded pool passes 2^31 at B = 32 on a
    // 4096^2 image (1024 x 4.07 M candidates)
    const int64_t e = (int64_t)(blockIdx.x - pre[im]) * 256 + threadIdx.x;
    const int B = d.B, n = B * B, Ppad = d.ppad, pitch = d.pitch;
    if (e >= (int64_t)n * Ppad) return;
    const int j = (int)(e / Ppad), p = (int)(e - (int64_t)j * Ppad);
    const bool valid = p < min(*d.pcount, d.pool_cap);
    float val = 0.f;
    if (valid) {
        const uint32_t v = d.pxy[p];
        const int cy = j / B, cx = j - cy * B;
        const uint8_t *q = d.pix + (size_t)((v >> 16) + 2 * cy) * pitch + (v & 0xffff) + 2 * cx;
        val = (float)(q[0] + q[1] + q[pitch] + q[pitch + 1] - 512);
    }
    d.df[e] = val;
    if (j == 0)
        d.dinfo[p] = valid ? make_float2((float)d.psum4[p], sqrt_down((double)d.pa[p])) : make_float2(0.f, 0.f);
}

template <int B>
__global__ __launch_bounds__(256) void k_fp32_search(BatchDev bt, SSet ss) {
    constexpr int n = B * B;
    constexpr int KC = n < 16 ? n : 16;
    constexpr int NKC = n / KC;
    __shared__ __align__(16) float Vs[KC][kF32Ranges * 8];
    __shared__ __align__(16) float Ds[KC][kF32Doms];
    __shared__ SLds sl;
    const int tid = threadIdx.x, tr = tid >> 5, td = tid & 31;
    load_sset(sl, ss);
    const SConst sc = make_sconst(ss);
    const float tfac = tn_factor(B * B);
    __syncthreads();
    const int *bpre = bt.pre + K_SEARCH * (bt.n + 1);
    const int im = find_img(bpre, bt.n, blockIdx.x);
    const ImgLvl &dsc = bt.d[im];
    const float *__restrict__ vf = dsc.vf;
    const float *__restrict__ df = dsc.df;
    const float2 *__restrict__ dinfo = dsc.dinfo;
    const RInfo *__restrict__ ri = dsc.ri;
    const uint32_t *__restrict__ sum4 = dsc.psum4;
    const int64_t *__restrict__ pa = dsc.pa;
    Partial *__restrict__ part = dsc.part;
    const int Rpad = dsc.rpad, Ppad = dsc.ppad, tiles_per_chunk = dsc.ftpc, nchunk = dsc.fnchunk;
    const int range_cap = dsc.range_cap, pool_cap = dsc.pool_cap;
    // R: the length of the search list (constant ranges are coded already)
    const int R = min(*dsc.ns, range_cap), P = min(*dsc.pcount, pool_cap);
    const int lb = blockIdx.x - bpre[im];
    const int nrg = (range_cap + kF32Ranges - 1) / kF32Ranges;
    const int rg = lb % nrg;
    if (lb >= nrg * nchunk || rg * kF32Ranges >= R) return;  // uniform over the block
    const int js = rg * kF32Ranges + tr;
    const bool rvalid = js < R;
    const int r = rvalid ? dsc.sidx[js] : 0;   // the range of search entry js
    const int chunk = lb / nrg;
    const int ntiles = (P + kF32Doms - 1) / kF32Doms;
    const int t0 = chunk * tiles_per_chunk, t1 = min(ntiles, t0 + tiles_per_chunk);
    const RInfo x = ri[r];
    const float bn = x.bn, an = x.an;
    float tn = -1e30f;
    int64_t best = INT64_MAX;
    int bp = INT32_MAX, bk = 0;

    for (int tile = t0; tile < t1; ++tile) {
        float acc[8][4];
        int iacc[8][4];
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[t][j] = 0.f;
                iacc[t][j] = 0;
            }
        for (int kc = 0; kc < NKC; ++kc) {
            __syncthreads();
            for (int e = tid; e < KC * 64; e += 256) {
                const int kk = e >> 6, o = e & 63;
                Vs[kk][o] = vf[((size_t)(kc * KC + kk) * Rpad + rg * kF32Ranges) * 8 + o];
            }
            for (int e = tid; e < KC * kF32Doms; e += 256) {
                const int kk = e >> 7, dd = e & 127;
                Ds[kk][dd] = df[(size_t)(kc * KC + kk) * Ppad + tile * kF32Doms + dd];
            }
            __syncthreads();
#pragma unroll 4
            for (int kk = 0; kk < KC; ++kk) {
                const float4 va = *(const float4 *)&Vs[kk][tr * 8];
                const float4 vb = *(const float4 *)&Vs[kk][tr * 8 + 4];
                const float4 d = *(const float4 *)&Ds[kk][td * 4];
                const float v[8] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};
                const float dd[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[t][j] = fmaf(v[t], dd[j], acc[t][j]);
            }
            if (n > 256 && ((kc + 1) % 16 == 0 || kc == NKC - 1)) {
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        iacc[t][j] += (int)acc[t][j];
                        acc[t][j] = 0.f;
                    }
            }
        }
        bool any = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int c[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) c[t] = n > 256 ? iacc[t][j] : (int)acc[t][j];
            const int m = max8(c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7]);
            const int p = tile * kF32Doms + td * 4 + j;
            const float2 di = dinfo[p];
            const float rhs = fmaf(tn, di.y, fmaf(-bn, di.x, -an));
            const bool pass = (p < P) & rvalid & ((float)m > rhs);
            if (pass) confirm_pair(m, p, sum4[p], pa[p], x.sr, x.cr, n, sl, sc, best, bp, bk);
            any |= pass;
        }
        if (__ballot(any)) {  // share the best of the 32 threads holding this range
            const int64_t gb = group_min_val<32>(best);
            tn = rvalid ? tn_from(gb, x.cr, sc, tfac) : -1e30f;
        }
    }
    group_min<32>(best, bp, bk);
    if (td == 0 && rvalid) {
        Partial o;
        o.val = best;
        o.p = bp == INT32_MAX ? -1 : bp;
        o.k = bk;
        part[(size_t)r * nchunk + chunk] = o;
    }
}

hipError_t launch_fp32_prep_b(const BatchHost &b, hipStream_t st) {
    if (b.blocks[K_VIEWS] > 0) k_fp32_views<<<b.blocks[K_VIEWS], 256, 0, st>>>(b.dev);
    if (b.blocks[K_DOMS] > 0) k_fp32_doms<<<b.blocks[K_DOMS], 256, 0, st>>>(b.dev);
    return hipGetLastError();
}

hipError_t launch_fp32_search_b(const BatchHost &b, hipStream_t st) {
    const int nb = b.blocks[K_SEARCH];
    if (nb == 0) return hipSuccess;
    switch (b.B) {
        case 2: k_fp32_search<2><<<nb, 256, 0, st>>>(b.dev, b.ss); break;
        case 4: k_fp32_search<4><<<nb, 256, 0, st>>>(b.dev, b.ss); break;
        case 8: k_fp32_search<8><<<nb, 256, 0, st>>>(b.dev, b.ss); break;
        case 16: k_fp32_search<16><<<nb, 256, 0, st>>>(b.dev, b.ss); break;
        case 32: k_fp32_search<32><<<nb, 256, 0, st>>>(b.dev, b.ss); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fic
