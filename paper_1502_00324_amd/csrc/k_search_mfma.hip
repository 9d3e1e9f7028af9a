// Int8 MFMA search engine (gfx950, v_mfma_i32_16x16x64_i8).
//
// The cross term of every (range, isometry) x domain pair is a dense
// contraction over the K = 4B^2 raw pixels of the 2B x 2B domain:
//   rows    = (range, isometry): the range seen through the inverse isometry,
//             each range pixel replicated over its 2x2 domain cell, minus 128;
//   columns = pool domains, raw pixels minus 128;
// both fit int8 exactly and int32 accumulation is exact (|C'| <= 4B^2 2^14).
//
// Fragment layouts (16 bytes per lane, 64 lanes per 1 KiB fragment, verified
// for this instruction: lane L feeds A row L%16 and B column L%16 with the
// 16 K-values of group L/16; result lane L holds rows 4(L/16)..+3 of column
// L%16):
//   A: quad q of 4 ranges, half h, K-step s:  afrag[((q*2 + h)*KS + s)*64 + L]
//      row i = L%16 -> range 4q + i/4, isometry 4h + i%4
//   B: tile of 16 domains, K-step s:         bfrag[(tile*KS + s)*64 + L]
//   K index k = 64 s + 16 (L/16) + byte -> raw pixel (k / 2B, k % 2B).
// With rows arranged this way the two halves give each lane all 8 isometries
// of one (range, domain) pair, so the isometry max stays in registers.
#include "fic_internal.h"
#include "search_common.h"

namespace fic {

typedef int v4i __attribute__((ext_vector_type(4)));

bool mfma_supported(int B) { return B == 4 || B == 8 || B == 16; }

static int mfma_rq(int B) { return B == 4 ? 4 : (B == 8 ? 2 : 1); }

// Quads of 4 ranges covered by the search grid (every wave reads RQ whole quads).
int mfma_quads_padded(int B, int range_cap) {
    const int rpw = 16 * mfma_rq(B);
    return (range_cap + rpw - 1) / rpw * (rpw / 4);
}

void mfma_geometry(int B, int range_cap, int pool_cap, int *ranges_per_wg, int *nchunk, int *tiles_per_chunk) {
    const int rpw = 4 * 4 * mfma_rq(B);
    const int ntiles = (pool_cap + kDomTile - 1) / kDomTile;
    const int nrg = (range_cap + rpw - 1) / rpw;
    int nc = (8192 + nrg - 1) / nrg;
    nc = max(1, min(nc, max(1, ntiles / 8)));
    nc = min(nc, 4096);
    *ranges_per_wg = rpw;
    *nchunk = nc;
    *tiles_per_chunk = (ntiles + nc - 1) / nc;
}

// ---------------------------------------------------------------- operands
__global__ __launch_bounds__(256) void k_mfma_afrag(const uint8_t *__restrict__ img, int pitch, int B, int KS,
                                                    const uint32_t *__restrict__ rxy, const int32_t *nr, int cap,
                                                    int nquads, uint4 *__restrict__ afrag) {
    const int slot = blockIdx.x * 256 + threadIdx.x;
    if (slot >= nquads * 2 * KS * 64) return;
    const int lane = slot & 63;
    int rest = slot >> 6;
    const int s = rest % KS;
    rest /= KS;
    const int h = rest & 1, q = rest >> 1;
    const int i = lane & 15, kg = lane >> 4;
    const int t = 4 * h + (i & 3);
    const int r = q * 4 + (i >> 2);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (r < min(*nr, cap)) {
        const uint32_t v = rxy[r];
        const int x0 = v & 0xffff, y0 = v >> 16;
        const int ti = iso_inv(t), D = 2 * B;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const int k = 64 * s + 16 * kg + b;
            const int dy = k / D, dx = k - dy * D;
            int sy, sx;
            iso_src(ti, B, dy >> 1, dx >> 1, sy, sx);
            const int val = (int)img[(size_t)(y0 + sy) * pitch + x0 + sx] - 128;
            w[b >> 2] |= (uint32_t)(uint8_t)(int8_t)val << (8 * (b & 3));
        }
    }
    afrag[slot] = make_uint4(w[0], w[1], w[2], w[3]);
}

__global__ __launch_bounds__(256) void k_mfma_bfrag(const uint8_t *__restrict__ img, int pitch, int B, int KS,
                                                    const uint32_t *__restrict__ pxy, const int32_t *np, int cap,
                                                    int ntiles, const uint32_t *__restrict__ sum4,
                                                    const int64_t *__restrict__ pa, uint4 *__restrict__ bfrag,
                                                    float2 *__restrict__ dinfo) {
    const int slot = blockIdx.x * 256 + threadIdx.x;
    if (slot >= ntiles * KS * 64) return;
    const int lane = slot & 63;
    const int rest = slot >> 6;
    const int s = rest % KS, tile = rest / KS;
    const int j = lane & 15, kg = lane >> 4;
    const int p = tile * kDomTile + j;
    const bool valid = p < min(*np, cap);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (valid) {
        const uint32_t v = pxy[p];
        const int x0 = v & 0xffff, y0 = v >> 16;
        const int D = 2 * B;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const int k = 64 * s + 16 * kg + b;
            const int dy = k / D, dx = k - dy * D;
            const int val = (int)img[(size_t)(y0 + dy) * pitch + x0 + dx] - 128;
            w[b >> 2] |= (uint32_t)(uint8_t)(int8_t)val << (8 * (b & 3));
        }
    }
    bfrag[slot] = make_uint4(w[0], w[1], w[2], w[3]);
    if (s == 0 && kg == 0)
        dinfo[p] = valid ? make_float2((float)sum4[p], sqrt_down((double)pa[p])) : make_float2(0.f, 0.f);
}

// ---------------------------------------------------------------- search
// One wave owns RQ quads (4 RQ ranges) and streams one chunk of domain tiles.
template <int KS, int RQ>
__global__ __launch_bounds__(256) void k_mfma_search(const v4i *__restrict__ afrag, const v4i *__restrict__ bfrag,
                                                     const float2 *__restrict__ dinfo, const RInfo *__restrict__ ri,
                                                     const int32_t *nr, int range_cap, const int32_t *np,
                                                     int pool_cap, const uint32_t *__restrict__ sum4,
                                                     const int64_t *__restrict__ pa, SSet ss, int n,
                                                     int tiles_per_chunk, int nchunk, Partial *__restrict__ part) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int R = min(*nr, range_cap), P = min(*np, pool_cap);
    const int q0 = (blockIdx.x * 4 + wave) * RQ;
    if (q0 * 4 >= R) return;  // whole wave; the kernel has no block barrier
    const int chunk = blockIdx.y;
    const int ntiles = (P + kDomTile - 1) / kDomTile;
    const int t0 = chunk * tiles_per_chunk, t1 = min(ntiles, t0 + tiles_per_chunk);
    const int g = lane >> 4;

    v4i A[RQ][2][KS];
    float tn[RQ], bn[RQ], an[RQ];
    int64_t best[RQ];
    int bp[RQ], bk[RQ], rr[RQ];
#pragma unroll
    for (int qi = 0; qi < RQ; ++qi) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int s = 0; s < KS; ++s) A[qi][h][s] = afrag[(((size_t)(q0 + qi) * 2 + h) * KS + s) * 64 + lane];
        const int r = (q0 + qi) * 4 + g;
        rr[qi] = r < R ? r : -1;
        const RInfo x = ri[r < R ? r : 0];
        bn[qi] = x.bn;
        an[qi] = x.an;
        tn[qi] = -1e30f;
        best[qi] = INT64_MAX;
        bp[qi] = INT32_MAX;
        bk[qi] = 0;
    }

    for (int tile = t0; tile < t1; ++tile) {
        v4i Bf[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) Bf[s] = bfrag[((size_t)tile * KS + s) * 64 + lane];
        const int p = tile * kDomTile + (lane & 15);
        const float2 di = dinfo[p];
        const bool pv = p < P;
#pragma unroll
        for (int qi = 0; qi < RQ; ++qi) {
            v4i cx = {0, 0, 0, 0}, cy = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                cx = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[qi][0][s], Bf[s], cx, 0, 0, 0);
                cy = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[qi][1][s], Bf[s], cy, 0, 0, 0);
            }
            const int m = max8(cx.x, cx.y, cx.z, cx.w, cy.x, cy.y, cy.z, cy.w);
            const float rhs = fmaf(tn[qi], di.y, fmaf(-bn[qi], di.x, -an[qi]));
            if (pv && rr[qi] >= 0 && (float)m > rhs)
                confirm_pair(m, p, rr[qi], n, ri, sum4, pa, ss, best[qi], bp[qi], bk[qi], tn[qi]);
        }
    }

#pragma unroll
    for (int qi = 0; qi < RQ; ++qi) {
        int64_t v = best[qi];
        int p = bp[qi], k = bk[qi];
        group_min<16>(v, p, k);
        if ((lane & 15) == 0 && rr[qi] >= 0) {
            Partial o;
            o.val = v;
            o.p = p == INT32_MAX ? -1 : p;
            o.k = k;
            part[(size_t)rr[qi] * nchunk + chunk] = o;
        }
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_mfma_prep(const uint8_t *img, int pitch, int B, const uint32_t *rxy, const int32_t *nr,
                            int range_cap, const fic_pool *pool, int pool_cap, void *afrag, void *bfrag,
                            float2 *dinfo, hipStream_t st) {
    const int KS = B * B / 16;
    const int nquads = mfma_quads_padded(B, range_cap);
    const int ntiles = (pool_cap + kDomTile - 1) / kDomTile;
    const long na = (long)nquads * 2 * KS * 64, nb = (long)ntiles * KS * 64;
    if (na > 0)
        k_mfma_afrag<<<(unsigned)((na + 255) / 256), 256, 0, st>>>(img, pitch, B, KS, rxy, nr, range_cap, nquads,
                                                                   (uint4 *)afrag);
    if (nb > 0)
        k_mfma_bfrag<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(img, pitch, B, KS, pool->xy, pool->count,
                                                                   pool_cap, ntiles, pool->sum4, pool->a,
                                                                   (uint4 *)bfrag, dinfo);
    return hipGetLastError();
}

template <int KS, int RQ>
static void launch_search_t(dim3 grid, hipStream_t st, const void *afrag, const void *bfrag, const float2 *dinfo,
                            const RInfo *ri, const int32_t *nr, int range_cap, const fic_pool *pool, int pool_cap,
                            SSet ss, int n, int tpc, int nchunk, Partial *part) {
    k_mfma_search<KS, RQ><<<grid, 256, 0, st>>>((const v4i *)afrag, (const v4i *)bfrag, dinfo, ri, nr, range_cap,
                                                pool->count, pool_cap, pool->sum4, pool->a, ss, n, tpc, nchunk,
                                                part);
}

hipError_t launch_mfma_search(int B, const void *afrag, const void *bfrag, const float2 *dinfo, const RInfo *ri,
                              const int32_t *nr, int range_cap, const fic_pool *pool, int pool_cap, SSet ss,
                              Partial *part, hipStream_t st) {
    int rpw, nchunk, tpc;
    mfma_geometry(B, range_cap, pool_cap, &rpw, &nchunk, &tpc);
    const dim3 grid((range_cap + rpw - 1) / rpw, nchunk);
    if (grid.x == 0) return hipSuccess;
    const int n = B * B;
    switch (B) {
        case 4: launch_search_t<1, 4>(grid, st, afrag, bfrag, dinfo, ri, nr, range_cap, pool, pool_cap, ss, n, tpc,
                                      nchunk, part); break;
        case 8: launch_search_t<4, 2>(grid, st, afrag, bfrag, dinfo, ri, nr, range_cap, pool, pool_cap, ss, n, tpc,
                                      nchunk, part); break;
        case 16: launch_search_t<16, 1>(grid, st, afrag, bfrag, dinfo, ri, nr, range_cap, pool, pool_cap, ss, n,
                                        tpc, nchunk, part); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fic
