// Contrast diagnostic (Sec. 3.2, Fig 5; Sec. 3.2.1, Fig 6): for the ranges
// accepted at each step, the histogram of the chosen contrast index and of
// the continuous least-squares contrast of the chosen match (Eq 2),
//   s* = (n sum r d - sum r sum d) / (n sum d^2 - (sum d)^2),  d = D4 / 4,
// i.e. s* = 4 Bx / A with Bx = n X4 - Sr Sd4 for the chosen domain and
// isometry.  s* is binned exactly in integers: bin floor(nbins 4Bx / A) for
// 0 <= 4Bx < A, an underflow bin for 4Bx < 0, an overflow bin for 4Bx >= A
// and a separate count for A = 0 (flat domain, s* undefined).
#include "fic_internal.h"
#include "scan_util.h"

namespace fic {

namespace {

struct HistLevel {
    const int32_t *ccount, *pcount;
    const uint32_t *cxy, *pxy, *cdom, *psum4;
    const int64_t *pa;
    const uint8_t *csplit, *ciso, *csidx;
    int B, last, range_cap, pool_cap;
};

// One wave per range of level l; out[l] = [under, nbins bins, over, flat, |S| s-index counts].
__global__ __launch_bounds__(256) void k_s_hist(HistLevel v, const uint8_t *__restrict__ pix, int pitch, int nbins,
                                                unsigned long long *__restrict__ out) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + w;
    if (r >= min(*v.ccount, v.range_cap)) return;
    if (!v.last && v.csplit[r]) return;
    const int B = v.B, n = B * B;
    const uint32_t rv = v.cxy[r];
    const int x0 = rv & 0xffff, y0 = rv >> 16;
    const int p = (int)min(v.cdom[r], (uint32_t)max(0, min(*v.pcount, v.pool_cap) - 1));
    const uint32_t dv = v.pxy[p];
    const int dx0 = dv & 0xffff, dy0 = dv >> 16;
    const int t = v.ciso[r];
    int64_t x4 = 0, sr = 0;
    for (int i = lane; i < n; i += 64) {
        const int y = i / B, x = i - y * B;
        const int rp = pix[(size_t)(y0 + y) * pitch + x0 + x];
        int cy, cx;
        iso_src(t, B, y, x, cy, cx);
        const uint8_t *q = pix + (size_t)(dy0 + 2 * cy) * pitch + dx0 + 2 * cx;
        x4 += (int64_t)rp * (q[0] + q[1] + q[pitch] + q[pitch + 1]);
        sr += rp;
    }
    x4 = wave_sum_i64(x4);
    sr = wave_sum_i64(sr);
    if (lane != 0) return;
    const int64_t sd4 = v.psum4[p], A = v.pa[p];
    const int64_t num4 = 4 * ((int64_t)n * x4 - sr * sd4);   // 4 Bx
    int bin;
    if (A == 0) bin = nbins + 2;
    else if (num4 < 0) bin = 0;
    else if (num4 >= A) bin = nbins + 1;
    else bin = 1 + (int)(((__int128)num4 * nbins) / A);
    atomicAdd(&out[bin], 1ull);
    atomicAdd(&out[nbins + 3 + min((int)v.csidx[r], kMaxS - 1)], 1ull);
}

__global__ void k_s_hist_zero(unsigned long long *out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = 0ull;
}

}  // namespace

}  // namespace fic

using namespace fic;

extern "C" {

int fic_s_histogram(fic_ctx *ctx, const fic_image *img, const fic_params *p, const fic_pool *pools,
                    const fic_level_codes *codes, int32_t nbins, int64_t *out, fic_stream stream) {
    if (!ctx || !img || !img->pix || !p || !pools || !codes || !out || nbins < 1 || nbins > 4096)
        return FIC_E_INVALID;
    int st = fic_validate_params(p, img->width, img->height);
    if (st != FIC_OK) return st;
    if (img->pitch < img->width) return FIC_E_INVALID;
    int64_t pcap[kMaxLevels], rcap[kMaxLevels];
    fic_query_capacity(p, img->width, img->height, pcap, rcap);
    for (int l = 0; l < p->levels; ++l) {
        const fic_pool &q = pools[l];
        const fic_level_codes &c = codes[l];
        if (!q.count || !q.xy || !q.sum4 || !q.a || !c.count || !c.xy || !c.split || !c.domain || !c.iso ||
            !c.s_idx)
            return FIC_E_INVALID;
        if (q.capacity < pcap[l] || c.capacity < rcap[l]) return FIC_E_CAPACITY;
    }
    st = enter(ctx);
    if (st != FIC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int per = nbins + 3 + kMaxS;
    const int total = per * p->levels;
    unsigned long long *o = (unsigned long long *)out;
    k_s_hist_zero<<<(total + 255) / 256, 256, 0, s>>>(o, total);
    for (int l = 0; l < p->levels; ++l) {
        HistLevel v;
        v.ccount = codes[l].count;
        v.pcount = pools[l].count;
        v.cxy = codes[l].xy;
        v.pxy = pools[l].xy;
        v.cdom = codes[l].domain;
        v.psum4 = pools[l].sum4;
        v.pa = pools[l].a;
        v.csplit = codes[l].split;
        v.ciso = codes[l].iso;
        v.csidx = codes[l].s_idx;
        v.B = p->block0 >> l;
        v.last = l == p->levels - 1;
        v.range_cap = (int)rcap[l];
        v.pool_cap = (int)pcap[l];
        if (rcap[l] > 0)
            k_s_hist<<<(unsigned)((rcap[l] + 3) / 4), 256, 0, s>>>(v, img->pix, img->pitch, nbins, o + (size_t)l * per);
    }
    return hip_status(hipGetLastError());
}

}  // extern "C"
