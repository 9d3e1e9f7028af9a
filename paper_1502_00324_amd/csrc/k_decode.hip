// Decoder (Sec. 1-2): rebuild every accepted range from its domain in the
// previous image, all ranges at once (synchronous iteration).
#include "fic_internal.h"
#include "scan_util.h"

namespace fic {

__device__ inline int64_t floor_div(int64_t a, int64_t b) {  // b > 0
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}

// X0: every accepted range filled with its stored offset.  One wave per range.
__global__ __launch_bounds__(256) void k_decode_init(int B, const int32_t *count, int cap,
                                                     const uint32_t *__restrict__ xy, const uint8_t *__restrict__ split,
                                                     const uint8_t *__restrict__ off, uint8_t *__restrict__ img,
                                                     int pitch) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + w;
    if (r >= min(*count, cap) || split[r]) return;
    const uint32_t v = xy[r];
    const int x0 = v & 0xffff, y0 = v >> 16;
    const uint8_t o = off[r];
    for (int i = lane; i < B * B; i += 64) {
        const int y = i / B, x = i - y * B;
        img[(size_t)(y0 + y) * pitch + x0 + x] = o;
    }
}

// One iteration: pixel = clamp(O + floor((2N + Q) / (2Q))), N = num*(n*D4' - Sd4'),
// Q = 4 n den, with D4' the isometry-mapped 2x2 cell sum of the domain in cur.
__global__ __launch_bounds__(256) void k_decode_iter(int B, const int32_t *count, int cap,
                                                     const uint32_t *__restrict__ xy, const uint8_t *__restrict__ split,
                                                     const uint32_t *__restrict__ dom, const uint8_t *__restrict__ iso,
                                                     const uint8_t *__restrict__ sidx, const uint8_t *__restrict__ off,
                                                     const uint32_t *__restrict__ pool_xy, SSet ss,
                                                     const uint8_t *__restrict__ cur, uint8_t *__restrict__ nxt,
                                                     int pitch) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + w;
    if (r >= min(*count, cap) || split[r]) return;
    const uint32_t v = xy[r];
    const int x0 = v & 0xffff, y0 = v >> 16;
    const uint32_t dv = pool_xy[dom[r]];
    const int dx0 = dv & 0xffff, dy0 = dv >> 16;
    const int t = iso[r], k = sidx[r];
    int64_t num = 0;
    for (int j = 0; j < ss.count; ++j)
        if (j == k) num = ss.num[j];
    const int64_t n = (int64_t)B * B;
    int64_t s4 = 0;
    for (int i = lane; i < 4 * B * B; i += 64) {
        const int y = i / (2 * B), x = i - y * (2 * B);
        s4 += cur[(size_t)(dy0 + y) * pitch + dx0 + x];
    }
    s4 = wave_sum_i64(s4);
    const int64_t q = 4 * n * ss.den;
    const int o = off[r];
    for (int i = lane; i < B * B; i += 64) {
        const int y = i / B, x = i - y * B;
        int cy, cx;
        iso_src(t, B, y, x, cy, cx);
        const uint8_t *p = cur + (size_t)(dy0 + 2 * cy) * pitch + dx0 + 2 * cx;
        const int64_t d4 = p[0] + p[1] + p[pitch] + p[pitch + 1];
        const int64_t val = o + floor_div(2 * num * (n * d4 - s4) + q, 2 * q);
        nxt[(size_t)(y0 + y) * pitch + x0 + x] = (uint8_t)(val < 0 ? 0 : (val > 255 ? 255 : val));
    }
}

hipError_t launch_decode_init(int B, const fic_level_codes *codes, int cap, uint8_t *img, int pitch,
                              hipStream_t st) {
    if (cap > 0)
        k_decode_init<<<(cap + 3) / 4, 256, 0, st>>>(B, codes->count, cap, codes->xy, codes->split, codes->offset,
                                                     img, pitch);
    return hipGetLastError();
}

hipError_t launch_decode_iter(int B, const fic_level_codes *codes, int cap, const fic_pool *pool, SSet ss,
                              const uint8_t *cur, uint8_t *nxt, int pitch, hipStream_t st) {
    if (cap > 0)
        k_decode_iter<<<(cap + 3) / 4, 256, 0, st>>>(B, codes->count, cap, codes->xy, codes->split, codes->domain,
                                                     codes->iso, codes->s_idx, codes->offset, pool->xy, ss, cur, nxt,
                                                     pitch);
    return hipGetLastError();
}

}  // namespace fic
