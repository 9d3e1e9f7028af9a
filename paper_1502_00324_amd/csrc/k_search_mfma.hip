// 16-row MFMA search engine (gfx950, v_mfma_i32_16x16x64_i8 and
// v_mfma_f32_16x16x32_f16).
//
// The cross term of every (range, isometry) x domain pair is a dense
// contraction.  Centred at 128, both operands fit int8 and the int32
// accumulators are exact.  Two operand forms give the same integer
//   C' = sum over decimated positions of (r - 128) (D4 - 512)
// (D4 the 2x2 sum of the domain, Sec. 3.1):
//   raw (pl = 1, K = 4B^2): rows hold the range, each pixel replicated over
//       its 2x2 domain cell; columns hold the raw domain pixels minus 128;
//   planes (pl = 2, K = 2B^2): D4 - 512 = 4 hi + lo with hi = floor(D4/4) - 128
//       and lo = D4 mod 4; rows hold the range once per decimated position,
//       the hi and lo planes are contracted separately and C' = 4 C_hi + C_lo.
//   f16 (pl = 3, K = B^2, v_mfma_f32_16x16x32_f16): the range minus 128 and
//       D4 - 512 as f16 (exact: integers below 2^11), f32 accumulation exact
//       (every partial sum an integer of magnitude <= B^2 2^16 <= 2^24); the
//       accumulators are floats, so the epilogue needs no conversion or
//       combination.  Same 16-row layout as the int8 forms.
//   f16 with the fused threshold (pl = 4, B = 2 and 4, one K-step of 32):
//       K-groups 0 and 1 (lanes 0..31) hold the <= 16 decimated positions,
//       centred at each block's own rounded mean: r - m_r and D4 - m_d with
//       m_r = round(Sr/n), m_d = round(Sd4/n) (magnitudes <= 255 and <= 1020,
//       exact in f16; sums <= n 2^18 <= 2^22, exact in f32), so
//         acc1 = sum (r - m_r)(D4 - m_d) = Bx/n + e_r e_d / n,
//         e_r = Sr - n m_r, e_d = Sd4 - n m_d, |e_r e_d / n| <= n/4.
//       K-group 2 (lanes 32..47) holds the prune threshold as a short dot
//       product: rows (tn_hi, tn_hi, tn_lo, 65504, K_r), columns
//       (-sA_hi, -sA_lo, -sA_hi, kill_d, 128), so the accumulator is
//         acc = acc1 - tn sA + 128 K_r + 65504 kill_d
//       up to the dropped terms (< 2^-20 tn sA), with tn = tn_hi + tn_lo and
//       sA = sqrt A = sA_hi + sA_lo as f16 pairs, 128 K_r = n/4 + 16 the
//       margin (the centring, the split and the f32 sums), kill_d = -1024
//       past the pool, and K_r = 65504 (no best yet: every pair passes) or
//       -65504 (nothing can win: no pair passes).  A pair can reach the
//       range's best only if Bx/n > tn sA, hence only if acc > 0, so the test
//       is the isometry maximum and one compare.  The threshold rows live in
//       the A registers and are rewritten whenever tn changes; passing pairs
//       recompute acc1 without them and confirm with Bx = n acc1 - e_r e_d.
// The planes form does half the MFMA work of the raw form and moves half the
// domain bytes; planes and f16 need B^2 >= 64, so B = 4 keeps the raw form in
// the int8 engine.  Up to B = 32 the int32 planes are exact (|C_hi| <= B^2
// 2^14 <= 2^24); the f16 form is exact up to B = 16 only.
//
// Fragment layouts (16 bytes per lane, 64 lanes per 1 KiB fragment, verified
// for this instruction: lane L feeds A row L%16 and B column L%16 with the
// 16 K-values of group L/16; result lane L holds rows 4(L/16)..+3 of column
// L%16):
//   A: quad q of 4 ranges, half h, K-step s < ka:  afrag[((q*2 + h)*ka + s)*64 + L]
//      row i = L%16 -> range 4q + i/4, isometry 4h + i%4
//   B: tile of 16 domains, K-step s < kt:         bfrag[(tile*kt + s)*64 + L]
//      planes form: steps [0, ka) hold hi, [ka, 2 ka) hold lo
//   K index k = 64 s + 16 (L/16) + byte -> raw pixel (k / 2B, k % 2B), or
//   decimated position (k / B, k % B) in the planes form; f16 form: 8 halves
//   per lane, k = 32 s + 8 (L/16) + e -> decimated position (k / B, k % B)
//   (the same row/column/result layout, checked for this instruction).
// With rows arranged this way the two halves give each lane all 8 isometries
// of one (range, domain) pair, so the isometry max stays in registers.
#include <stdio.h>
#include <stdlib.h>

#include <type_traits>

#include "fic_internal.h"
#include "search_common.h"

namespace fic {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ h8v as_h8(const v4i &x) {
    h8v h;
    __builtin_memcpy(&h, &x, sizeof(h));
    return h;
}

bool mfma_supported(int B) { return B == 4 || B == 8 || B == 16 || B == 32; }

// Operand form (pl), range quads per wave (RQ), domain tiles per LDS stage
// (DT) and the occupancy the register allocation aims at (waves per SIMD).
// Each range size and form class (int8: pl 1 or 2; f16: pl 3 or 4) has a
// measured default (its first entry); FIC_MFMA_SHAPE="pl,rq,dt,wpe" selects
// another compiled shape of the same class (used to tune).
struct Shape { int B, pl, rq, dt, wpe; };
static const Shape kShapes[] = {
    {4, 1, 2, 16, 3}, {4, 1, 1, 16, 3}, {4, 1, 4, 16, 2},
    {8, 2, 2, 8, 3}, {8, 2, 2, 16, 2}, {8, 2, 1, 8, 4}, {8, 2, 3, 8, 2}, {8, 2, 4, 8, 2}, {8, 1, 2, 8, 2},
    {16, 2, 2, 1, 3}, {16, 2, 2, 1, 2}, {16, 2, 1, 2, 3}, {16, 2, 2, 2, 2}, {16, 2, 1, 1, 4}, {16, 1, 1, 1, 2},
    {8, 3, 2, 12, 3}, {8, 3, 2, 8, 3}, {8, 3, 1, 8, 4}, {8, 3, 2, 16, 2}, {8, 3, 3, 8, 2}, {8, 3, 4, 8, 2},
    {16, 3, 1, 2, 3}, {16, 3, 2, 1, 2}, {16, 3, 1, 1, 4}, {16, 3, 2, 2, 2},
    {32, 2, 1, 1, 2}, {32, 2, 2, 1, 1}, {32, 2, 1, 2, 1},
    {4, 4, 2, 8, 3}, {4, 4, 2, 16, 3}, {4, 4, 1, 8, 4}, {4, 4, 2, 8, 4}, {4, 4, 3, 8, 3}, {4, 4, 4, 8, 2},
    {2, 4, 2, 8, 3},
};
// Candidates of (B, int8 or f16 class) in table order; index 0 is the default.
int mfma_shape_count(int B, bool f16) {
    int c = 0;
    for (const Shape &s : kShapes) c += s.B == B && (s.pl >= 3) == f16;
    return c;
}
bool mfma_shape_at(int B, bool f16, int index, TileShape &out) {
    int c = 0;
    for (const Shape &s : kShapes)
        if (s.B == B && (s.pl >= 3) == f16 && c++ == index) {
            out = TileShape{s.pl, s.rq, s.dt, s.wpe};
            return true;
        }
    return false;
}
TileShape mfma_pick(int B, bool f16, int choice) {
    const char *e = getenv("FIC_MFMA_SHAPE");
    int pl = 0, rq = 0, dt = 0, wpe = 0;
    if (e && sscanf(e, "%d,%d,%d,%d", &pl, &rq, &dt, &wpe) == 4)
        for (const Shape &s : kShapes)
            if (s.B == B && (s.pl >= 3) == f16 && s.pl == pl && s.rq == rq && s.dt == dt && s.wpe == wpe)
                return TileShape{s.pl, s.rq, s.dt, s.wpe};
    TileShape t{1, 1, 1, 1};
    if (choice >= 0 && mfma_shape_at(B, f16, choice, t)) return t;
    mfma_shape_at(B, f16, 0, t);
    return t;
}

// Work split (both matrix engines).  A workgroup owns rpw ranges (a range
// group) and streams domain tiles in chunks of about 1.5 MB of fragments,
// small enough to stay resident in one XCD's 4 MB L2 while every range group
// running on that XCD reads it.  With 8 or more chunks the mapping is
// XCD-aware: workgroups are dispatched round-robin (id % 8 = XCD), XCD x owns
// chunks x, x+8, x+16, ..., and consecutive workgroups of an XCD take
// consecutive range groups of the same chunks.  A workgroup walks G chunks of
// its XCD with one running best over them (about a quarter of the XCD's
// chunks, and enough to keep the partial results, one per range and slot,
// under 256 MB).  tile_kib is the fragment size of one domain tile in KiB.
// Partial-result slots per XCD and range group: measured best at 64 for
// B = 32 (a walk of two or three chunks, which the concurrent workgroups of
// an XCD share in its L2), 4 otherwise (FIC_SLOTS_PER_XCD overrides both).
static int slots_per_xcd(int dflt) {
    const char *e = getenv("FIC_SLOTS_PER_XCD");
    const int v = e ? atoi(e) : 0;
    return v >= 1 && v <= 64 ? v : dflt;
}

// Target chunk size in KiB of fragments, over the expected pool: measured
// best at 2048 for the f16 32x32 form, 1024 for the 16-row forms
// (FIC_CHUNK_KIB, FIC_MFMA_CHUNK_KIB override them).
static int chunk_kib(bool rows16) {
    const char *e = getenv(rows16 ? "FIC_MFMA_CHUNK_KIB" : "FIC_CHUNK_KIB");
    const int v = e ? atoi(e) : 0;
    return v >= 64 && v <= 16384 ? v : rows16 ? 1024 : 2048;
}

void split_chunks(MfmaGeom &g, int range_cap, int ntiles, int tile_kib, int dt, bool rows16, int slots) {
    g.nrg = (range_cap + g.rpw - 1) / g.rpw;
    g.tpc = max(8 * dt, chunk_kib(rows16) / tile_kib);
    g.nchunk = (ntiles + g.tpc - 1) / g.tpc;
    if (g.nchunk < 8) {
        // small pool: split finer only to give the GPU enough workgroups
        int nc = max(g.nchunk, min((ntiles + 8 * dt - 1) / (8 * dt), (2048 + g.nrg - 1) / max(1, g.nrg)));
        g.nchunk = max(1, min(nc, 8));
    } else {
        g.nchunk = (g.nchunk + 7) / 8 * 8;
    }
    g.tpc = max(1, (ntiles + g.nchunk - 1) / g.nchunk);
    g.xcd = g.nchunk % 8 == 0 ? 1 : 0;
    if (g.xcd) {
        const int per_xcd = g.nchunk / 8;
        const long max_slots = max(8L, (256L << 20) / 16 / max(1, range_cap));
        const int groups_max = (int)max(1L, max_slots / 8);
        const int spx = slots_per_xcd(slots);
        g.G = max((per_xcd + groups_max - 1) / groups_max, (per_xcd + spx - 1) / spx);
        g.nslot = 8 * ((per_xcd + g.G - 1) / g.G);
    } else {
        g.G = 1;
        g.nslot = g.nchunk;
    }
    g.nwg = g.nrg * g.nslot;
}

MfmaGeom mfma_geometry(int B, int range_cap, int pool_cap, const TileShape &sh) {
    MfmaGeom g;
    g.pl = sh.pl;
    g.ka = sh.pl == 2 ? B * B / 64 : sh.pl == 3 ? B * B / 32 : sh.pl == 4 ? 1 : B * B / 16;
    g.kt = sh.pl == 2 ? 2 * g.ka : g.ka;
    g.rpw = 16 * sh.rq;
    const int ntiles = (pool_cap + kDomTile - 1) / kDomTile;
    split_chunks(g, range_cap, ntiles, g.kt, sh.dt, true, B == 32 ? 64 : 4);
    return g;
}

// ---------------------------------------------------------------- operands
__device__ __forceinline__ void k_mfma_afrag(const BatchDev &b, const int bid) {
    const int *pre = b.pre + K_AFRAG * (b.n + 1);
    const int im = find_img(pre, b.n, bid);
    const ImgLvl &d = b.d[im];
    const int B = d.B, KA = d.geo.ka, planes = d.geo.pl == 2, f16 = d.geo.pl == 3, ft = d.geo.pl == 4;
    const int nquads = d.geo.nrg * (d.geo.rpw / 4);
    const int64_t slot = (int64_t)(bid - pre[im]) * 256 + threadIdx.x;
    if (slot >= (int64_t)nquads * 2 * KA * 64) return;
    const int lane = (int)(slot & 63);
    int rest = (int)(slot >> 6);
    const int s = rest % KA;
    rest /= KA;
    const int h = rest & 1, q = rest >> 1;
    const int i = lane & 15, kg = lane >> 4;
    const int t = 4 * h + (i & 3);
    // row i of quad q: entry 4q + i/4 of the search list
    const int js = q * 4 + (i >> 2);
    const int r = js < *d.ns ? d.sidx[js] : -1;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (ft) {
        // positions in K-groups 0 and 1 minus the range's rounded mean; the
        // threshold group (2) is written by the search kernel, group 3 is 0
        h8v hv = h8v{0};
        if (kg < 2 && r >= 0) {
            const uint32_t v = d.rxy[r];
            const int x0 = v & 0xffff, y0 = v >> 16, n = B * B;
            const int ti = iso_inv(t), cen = round_mean(d.ri[r].sr, n);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * kg + e;
                if (k >= n) continue;   // B = 2: 4 positions
                const int cy = k / B, cx = k - cy * B;
                int sy, sx;
                iso_src(ti, B, cy, cx, sy, sx);
                hv[e] = (_Float16)((int)d.pix[(size_t)(y0 + sy) * d.pitch + x0 + sx] - cen);
            }
        }
        __builtin_memcpy(w, &hv, sizeof(w));
    } else if (f16 && r >= 0) {
        const uint32_t v = d.rxy[r];
        const int x0 = v & 0xffff, y0 = v >> 16;
        const int ti = iso_inv(t);
        h8v hv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 32 * s + 8 * kg + e;
            const int cy = k / B, cx = k - cy * B;
            int sy, sx;
            iso_src(ti, B, cy, cx, sy, sx);
            hv[e] = (_Float16)((int)d.pix[(size_t)(y0 + sy) * d.pitch + x0 + sx] - 128);
        }
        __builtin_memcpy(w, &hv, sizeof(w));
    } else if (r >= 0) {
        const uint32_t v = d.rxy[r];
        const int x0 = v & 0xffff, y0 = v >> 16;
        const int ti = iso_inv(t), D = 2 * B;
#pragma unroll
        for (int bb = 0; bb < 16; ++bb) {
            const int k = 64 * s + 16 * kg + bb;
            int cy, cx;  // decimated position
            if (planes) {
                cy = k / B;
                cx = k - cy * B;
            } else {
                cy = (k / D) >> 1;
                cx = (k % D) >> 1;
            }
            int sy, sx;
            iso_src(ti, B, cy, cx, sy, sx);
            const int val = (int)d.pix[(size_t)(y0 + sy) * d.pitch + x0 + sx] - 128;
            w[bb >> 2] |= (uint32_t)(uint8_t)(int8_t)val << (8 * (bb & 3));
        }
    }
    d.afrag[slot] = make_uint4(w[0], w[1], w[2], w[3]);
}

// D4 of the 8 decimated positions (cy, cx0 .. cx0 + 7) of a domain at
// (x0, y0): 2x2 sums over 16 bytes of image rows y0 + 2cy and y0 + 2cy + 1,
// read as 4-byte words (unaligned); each 16-bit half of a word sum holds one
// D4 <= 1020.
__device__ __forceinline__ void d4_row8(gptr<uint8_t> pix, int pitch, int x0, int y0, int cy, int cx0, int (&d4)[8]) {
    typedef uint32_t u32u __attribute__((aligned(1)));
    const gptr<uint8_t> q = pix + (size_t)(y0 + 2 * cy) * pitch + x0 + 2 * cx0;
    const gptr<u32u> r0 = (gptr<u32u>)q, r1 = (gptr<u32u>)(q + pitch);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t a = r0[i], c = r1[i];
        const uint32_t t = (a & 0x00ff00ffu) + ((a >> 8) & 0x00ff00ffu) + (c & 0x00ff00ffu) + ((c >> 8) & 0x00ff00ffu);
        d4[2 * i] = (int)(t & 0xffffu);
        d4[2 * i + 1] = (int)(t >> 16);
    }
}

__device__ __forceinline__ void k_mfma_bfrag(const BatchDev &b, const int bid) {
    const int *pre = b.pre + K_BFRAG * (b.n + 1);
    const int im = find_img(pre, b.n, bid);
    const ImgLvl &d = b.d[im];
    const int B = d.B, KA = d.geo.ka, KT = d.geo.kt, planes = d.geo.pl == 2, f16 = d.geo.pl == 3,
              ft = d.geo.pl == 4;
    const int ntiles = mfma_tiles(d.pool_cap);
    float *dsd = (float *)d.dinfo, *dsa = dsd + (size_t)ntiles * kDomTile;
    // one thread per (tile, K-step, lane) of the output; in the planes form
    // one per K-step of the hi plane, writing both planes
    const int KS = planes ? KA : KT;
    const int64_t gid = (int64_t)(bid - pre[im]) * 256 + threadIdx.x;   // can pass 2^31
    if (gid >= (int64_t)ntiles * KS * 64) return;
    const int lane = (int)(gid & 63);
    const int rest = (int)(gid >> 6);
    const int s = rest % KS, tile = rest / KS;
    const int64_t slot = ((int64_t)tile * KT + s) * 64 + lane;
    const int j = lane & 15, kg = lane >> 4;
    const int p = tile * kDomTile + j;
    const bool valid = p < min(*d.pcount, d.pool_cap);
    if (planes) {
        // both planes of the thread's 16 positions (each D4 read once)
        uint32_t wh[4] = {0u, 0u, 0u, 0u}, wl[4] = {0u, 0u, 0u, 0u};
        if (valid) {   // B >= 8: each group of 8 positions lies in one decimated row
            const uint32_t v = d.pxy[p];
            const int x0 = v & 0xffff, y0 = v >> 16;
#pragma unroll
            for (int g8 = 0; g8 < 2; ++g8) {
                const int k = 64 * s + 16 * kg + 8 * g8;
                const int cy = k / B, cx = k - cy * B;
                int d4[8];
                d4_row8(as_global(d.pix), d.pitch, x0, y0, cy, cx, d4);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int bb = 8 * g8 + e;
                    wh[bb >> 2] |= (uint32_t)(uint8_t)(int8_t)((d4[e] >> 2) - 128) << (8 * (bb & 3));
                    wl[bb >> 2] |= (uint32_t)(d4[e] & 3) << (8 * (bb & 3));
                }
            }
        }
        d.bfrag[slot] = make_uint4(wh[0], wh[1], wh[2], wh[3]);
        d.bfrag[slot + (int64_t)KA * 64] = make_uint4(wl[0], wl[1], wl[2], wl[3]);
        if (s == 0 && kg == 0) {   // NaN past the pool: no pair there passes
            dsd[p] = valid ? (float)d.psum4[p] : __builtin_nanf("");
            dsa[p] = valid ? sqrt_down((double)d.pa[p]) : __builtin_nanf("");
        }
        return;
    }
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (ft) {
        // K-groups 0, 1: positions minus the domain's rounded mean of D4;
        // group 2: the threshold operand (-sA_hi, -sA_lo, -sA_hi, kill, 128)
        h8v hv = h8v{0};
        const int n = B * B;
        if (kg < 2 && valid) {
            const uint32_t v = d.pxy[p];
            const int x0 = v & 0xffff, y0 = v >> 16, pitch = d.pitch;
            const int cen = round_mean(d.psum4[p], n);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * kg + e;
                if (k >= n) continue;
                const int cy = k / B, cx = k - cy * B;
                const uint8_t *q = d.pix + (size_t)(y0 + 2 * cy) * pitch + x0 + 2 * cx;
                hv[e] = (_Float16)(q[0] + q[1] + q[pitch] + q[pitch + 1] - cen);
            }
        } else if (kg == 2) {
            if (valid) {
                const float sa = sqrt_down((double)d.pa[p]);
                const _Float16 hi = (_Float16)sa, lo = (_Float16)(sa - (float)hi);
                hv[0] = -hi;
                hv[1] = -lo;
                hv[2] = -hi;
            } else {
                hv[3] = (_Float16)-1024.0f;
            }
            hv[4] = (_Float16)128.0f;
        }
        __builtin_memcpy(w, &hv, sizeof(w));
    } else if (valid && f16) {   // B >= 8: the 8 positions lie in one decimated row
        const uint32_t v = d.pxy[p];
        const int x0 = v & 0xffff, y0 = v >> 16;
        const int k = 32 * s + 8 * kg;
        const int cy = k / B, cx = k - cy * B;
        int d4[8];
        d4_row8(as_global(d.pix), d.pitch, x0, y0, cy, cx, d4);
        h8v hv;
#pragma unroll
        for (int e = 0; e < 8; ++e) hv[e] = (_Float16)(d4[e] - 512);
        __builtin_memcpy(w, &hv, sizeof(w));
    } else if (valid) {   // raw form: the pixels of the 2B x 2B block
        const uint32_t v = d.pxy[p];
        const int x0 = v & 0xffff, y0 = v >> 16;
        const int D = 2 * B, pitch = d.pitch;
#pragma unroll
        for (int bb = 0; bb < 16; ++bb) {
            const int k = 64 * s + 16 * kg + bb;
            const int dy = k / D, dx = k - dy * D;
            const int val = (int)d.pix[(size_t)(y0 + dy) * pitch + x0 + dx] - 128;
            w[bb >> 2] |= (uint32_t)(uint8_t)(int8_t)val << (8 * (bb & 3));
        }
    }
    d.bfrag[slot] = make_uint4(w[0], w[1], w[2], w[3]);
    if (s == 0 && kg == 0) {   // NaN past the pool: no pair there passes
        dsd[p] = valid ? (float)d.psum4[p] : __builtin_nanf("");
        dsa[p] = valid ? sqrt_down((double)d.pa[p]) : __builtin_nanf("");
    }
}

// ---------------------------------------------------------------- search
// A workgroup of 4 waves owns 16 RQ ranges (each wave RQ quads) and the
// domain tiles of its chunks.  Domain fragments and the per-domain Sd4 and
// sqrt(A) go straight from global memory into LDS in stages of DT tiles,
// double-buffered (the loads of stage s+1 are issued before the MFMAs of
// stage s), through buffer resources based at the chunk's first tile, so a
// stage's loads differ only by a scalar offset.  A chunk's last stage may
// read up to DT - 1 tiles past its end: the next chunk's domains (evaluated
// twice, harmless: the partials merge by (val, domain)) or the zero padding
// tiles, whose NaN moments never pass.
template <int PL> struct AccOf { typedef v4i type; typedef int max_type; };   // int32 accumulators
template <> struct AccOf<3> { typedef v4f type; typedef float max_type; };  // f16 form: f32 accumulators
template <> struct AccOf<4> { typedef v4f type; typedef float max_type; };  // f16, fused threshold

template <int KA, int PL, int RQ, int DT, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_mfma_search(BatchDev bt, SSet ss) {
    typedef typename AccOf<PL>::type Acc;
    typedef typename AccOf<PL>::max_type MaxT;   // C'max: exact int, or an exact integer in a float
    constexpr bool FT = PL == 4;                 // the threshold is in the accumulators
    constexpr int NP = PL == 2 ? 2 : 1;          // accumulator planes
    constexpr int KB = KA * NP;                  // K-steps of a domain tile
    // share range bests across workgroups only when a stage is long enough
    // (>= 4 tiles, or one tile of >= 32 K-steps) to hide the coherent load of
    // the shared values
    constexpr bool SHARE = DT >= 4 || KB >= 32;
    constexpr int STAGE = DT * KB * 64;          // uint4 per stage
    constexpr int PER_T = STAGE / 256;
    static_assert(STAGE % 256 == 0, "stage must split evenly over 256 threads");
    // the two stage buffers of fragments, separate arrays: a stage's
    // direct-to-LDS loads into one are then known not to touch the other
    constexpr int ND = DT * kDomTile;            // domains per stage
    constexpr int NDL = FT ? 1 : ND;             // the fused threshold needs no per-domain values
    static_assert(DT <= kF16PadTiles, "a stage reads at most DT - 1 tiles past a chunk");
    __shared__ uint4 bl0[STAGE];
    __shared__ uint4 bl1[STAGE];
    __shared__ float sa0[NDL], sa1[NDL], sd0[NDL], sd1[NDL];   // sqrt(A) rounded down, Sd4
    __shared__ SLds sl;
    __shared__ int s_item;
    // per range (4 waves x RQ quads x 4 ranges): values only the rare paths
    // and the stage ends read (Cr, the best value the threshold reflects,
    // Sr).  The f16 form keeps them in LDS, which frees the registers its
    // 12-tile stages need; the int8 forms, whose stages are one or two tiles
    // (a stage end per tile or two), keep them in registers.
    struct RangeLds { int64_t cr, tb; int sr; };
    __shared__ RangeLds s_rng[4 * RQ * 4];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    load_sset(sl, ss);
    const SConst sc = make_sconst(ss);
    // Persistent: the workgroup takes items (image, range group, chunk walk)
    // from its XCD's queue until it is empty.  Workgroup w runs on XCD w % 8,
    // and the items of XCD x walk the chunks x, x + 8, ..., so the concurrent
    // workgroups of one XCD read the same chunks from its L2.
    const int xcd = blockIdx.x & 7;
    const int *qpre = bt.queue + kQueueHeads + xcd * (bt.n + 1);
    const int total = qpre[bt.n];
  auto run_item = [&](const int im, const int k) {
    const ImgLvl &dsc = bt.d[im];
    const MfmaGeom geo = dsc.geo;
    const gptr<v4i> afrag = as_global((const v4i *)dsc.afrag);
    RInfo *__restrict__ ri = dsc.ri;
    const gptr<int64_t> pa = as_global(dsc.pa);
    Partial *__restrict__ part = dsc.part;
    const int range_cap = dsc.range_cap, pool_cap = dsc.pool_cap, n = dsc.B * dsc.B;
    const int nalloc = mfma_tiles(pool_cap);
    const float *dsd = (const float *)dsc.dinfo, *dsa = dsd + (size_t)nalloc * kDomTile;
    const gptr<float> dsd_g = as_global(dsd);
    const float tfac = tn_factor(n);
    const int32_t *np = dsc.pcount;
    // R: the length of the search list (constant ranges are coded already)
    const int R = uniform(min(*dsc.ns, range_cap)), P = uniform(min(*np, pool_cap));
    int rg, cfirst, cstep, ncs, slot;
    item_walk(geo, R, xcd, k, rg, cfirst, cstep, ncs, slot);
    const gptr<int32_t> sidx = as_global(dsc.sidx);
    const int ntiles = (P + kDomTile - 1) / kDomTile;
    const int q0 = (rg * 4 + wave) * RQ;
    const bool wave_on = q0 * 4 < R;
    const int g = lane >> 4;

    v4i A[RQ][2][KA];
    float tn[RQ], bn[RQ], an[RQ];
    int64_t best[RQ];
    int bp[RQ], bk[RQ], rr[RQ];
    RangeLds rreg[RQ];
    const auto rng = [&](int qi) -> RangeLds & {
        if constexpr (PL == 3) return s_rng[(wave * RQ + qi) * 4 + g];
        else return rreg[qi];
    };
#pragma unroll
    for (int qi = 0; qi < RQ; ++qi) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int s = 0; s < KA; ++s) A[qi][h][s] = afrag[(((size_t)(q0 + qi) * 2 + h) * KA + s) * 64 + lane];
        const int js = (q0 + qi) * 4 + g;
        const int r = js < R ? sidx[js] : -1;
        rr[qi] = r;
        const RInfo x = ri[r >= 0 ? r : 0];
        bn[qi] = x.bn;
        an[qi] = x.an;
        // every lane of the range writes the same values (no other wave reads them)
        RangeLds &rl = rng(qi);
        rl.sr = (int)x.sr;
        rl.cr = x.cr;
        tn[qi] = r >= 0 ? -1e30f : __builtin_nanf("");  // NaN: the row never passes
        rl.tb = INT64_MAX;
        // start from the best other walks of this range have shared (a stale
        // copy only loosens the test)
        if (r >= 0 && x.gbest < INT64_MAX) {
            rl.tb = x.gbest;
            tn[qi] = tn_shared(x.gbest, x.cr, sc, tfac);
        }
        best[qi] = INT64_MAX;
        bp[qi] = INT32_MAX;
        bk[qi] = 0;
    }

    // Fused threshold: K-group 2 (lanes 32..47) of both halves' A fragment
    // holds the row's threshold; row i = lane % 16 belongs to range i / 4 of
    // the quad, whose tn lives in result lanes 16 (i / 4) .. + 15.
    const float ft_k = (float)(n / 4 + 16) / 128.0f;
    auto build_thr = [&](int qi) {
        const float t = __shfl(tn[qi], 16 * ((lane & 15) >> 2), 64);
        _Float16 th = (_Float16)0, tl = (_Float16)0, kr;
        if (__builtin_isnan(t)) {
            kr = (_Float16)-65504.0f;            // nothing can win: no pair passes
        } else if (t < -1e29f) {
            kr = (_Float16)65504.0f;             // no best yet: every pair passes
        } else {
            th = (_Float16)t;
            tl = (_Float16)(t - (float)th);
            kr = (_Float16)ft_k;
        }
        h8v hv = h8v{0};
        hv[0] = th;
        hv[1] = th;
        hv[2] = tl;
        hv[3] = (_Float16)65504.0f;              // times the domain's kill value
        hv[4] = kr;                              // times 128
        v4i w;
        __builtin_memcpy(&w, &hv, sizeof(w));
        if (lane >= 32 && lane < 48) {
            A[qi][0][0] = w;
            A[qi][1][0] = w;
        }
    };
    if constexpr (FT) {
#pragma unroll
        for (int qi = 0; qi < RQ; ++qi) build_thr(qi);
    }

    // Drain the one-time loads above now: vmcnt is in-order, so a wait for
    // them inside the tile loop would also wait for the stage prefetch.
    __builtin_amdgcn_s_waitcnt(0);

    typedef __attribute__((address_space(3))) void *lds_t;
    // the wave index as a scalar: the LDS destination of a direct load is a
    // per-wave base in M0
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    constexpr int PER_D = (ND + 255) / 256;
    int t0 = 0;  // first tile of the chunk being streamed
    __amdgpu_buffer_rsrc_t rfrag, rsa, rsd;
    // one stage of the current chunk into the LDS buffers given: fragments,
    // then per-domain values; wave w fills its own 64-slot blocks
    auto gload = [&](uint4 *fdst, float *adst, float *ddst, int stg) {
#pragma unroll
        for (int i = 0; i < PER_T; ++i)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rfrag, (lds_t)(fdst + 64 * wv + 256 * i), 16,
                                                     (unsigned)(tid + 256 * i) * 16u, (unsigned)stg * STAGE * 16u, 0,
                                                     0);
        if constexpr (!FT) {
#pragma unroll
            for (int i = 0; i < PER_D; ++i) {
                if (ND % 256 == 0 || tid + 256 * i < ND) {
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsa, (lds_t)(adst + 64 * wv + 256 * i), 4,
                                                             (unsigned)(tid + 256 * i) * 4u, (unsigned)stg * ND * 4u,
                                                             0, 0);
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsd, (lds_t)(ddst + 64 * wv + 256 * i), 4,
                                                             (unsigned)(tid + 256 * i) * 4u, (unsigned)stg * ND * 4u,
                                                             0, 0);
                }
            }
        }
    };
    // acc[qi][h][plane]: the planes are combined (4 hi + lo) at the test,
    // one tile later, so no MFMA result is waited for at issue time.
    // Up to 8 K-steps a tile's fragments are read into registers one tile
    // ahead of its MFMAs (two register sets alternate), so the LDS latency is
    // covered by the previous tile; longer tiles keep a ring of a few K-steps
    // (below), to bound registers.
    constexpr bool PREF = KB <= 8;
    constexpr int KR = PREF ? KB : NP;
    auto rd = [&](const uint4 *Bs, int dt, int s) {
        const uint4 u = Bs[(dt * KB + s) * 64 + lane];
        return v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
    };
    auto read_tile = [&](v4i (&Bf)[KR], const uint4 *Bs, int dt) {
#pragma unroll
        for (int s = 0; s < KR; ++s) Bf[s] = rd(Bs, dt, s);
    };
    // Longer tiles keep a ring of KD + 1 K-steps: step s + KD is read while
    // the MFMAs of step s issue.
    constexpr int KD = 2;
    auto mfma_tile = [&](Acc (&acc)[RQ][2][NP], const uint4 *Bs, int dt, v4i (&Bf)[KR]) {
#pragma unroll
        for (int qi = 0; qi < RQ; ++qi)
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) acc[qi][0][pl] = acc[qi][1][pl] = Acc{0, 0, 0, 0};
        v4i ring[PREF ? 1 : KD + 1][NP];
        if constexpr (!PREF) {
#pragma unroll
            for (int s = 0; s < KD; ++s)
#pragma unroll
                for (int pl = 0; pl < NP; ++pl) ring[s][pl] = rd(Bs, dt, pl * KA + s);
        }
#pragma unroll
        for (int s = 0; s < KA; ++s) {
            if constexpr (!PREF) {
                if (s + KD < KA) {
#pragma unroll
                    for (int pl = 0; pl < NP; ++pl) ring[(s + KD) % (KD + 1)][pl] = rd(Bs, dt, pl * KA + s + KD);
                }
                // keep the reads here: the scheduler would sink them next to their MFMAs
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) {
                const v4i &b = PREF ? Bf[pl * KA + s] : ring[s % (KD + 1)][pl];
#pragma unroll
                for (int qi = 0; qi < RQ; ++qi)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if constexpr (PL >= 3)
                            acc[qi][h][pl] = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(A[qi][h][s]), as_h8(b),
                                                                                    acc[qi][h][pl], 0, 0, 0);
                        else
                            acc[qi][h][pl] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[qi][h][s], b,
                                                                                   acc[qi][h][pl], 0, 0, 0);
                    }
            }
        }
    };
    auto cprime = [&](const v4i (&a)[NP]) -> v4i {
        if constexpr (PL == 2) return (a[0] << 2) + a[1];
        else return a[0];
    };
    // the largest C' over the 8 isometries of each lane's pair; in the f16
    // form the f32 accumulators hold exact integers
    auto cmax = [&](const Acc (&x)[NP], const Acc (&y)[NP]) -> MaxT {
        if constexpr (PL >= 3) {
            return max8f(x[0].x, x[0].y, x[0].z, x[0].w, y[0].x, y[0].y, y[0].z, y[0].w);
        } else {
            const v4i cx = cprime(x), cy = cprime(y);
            return max8(cx.x, cx.y, cx.z, cx.w, cy.x, cy.y, cy.z, cy.w);
        }
    };
  for (int cj = 0; cj < ncs; ++cj) {
    const int chunk = cfirst + cj * cstep;
    // the chunks split the actual pool evenly (their count is fixed by the
    // plan, the pool size only known here)
    const int tpc = (ntiles + geo.nchunk - 1) / geo.nchunk;
    t0 = chunk * tpc;
    const int t1 = min(ntiles, t0 + tpc);
    const int nstage = t1 > t0 ? (t1 - t0 + DT - 1) / DT : 0;
    if (nstage == 0) continue;   // uniform over the workgroup
    // resources over [t0, nalloc): a chunk's offsets stay below 2^31 (the plan checks)
    const int left = uniform((int)min((long)(nalloc - t0) * kDomTile * 4, (long)INT32_MAX));
    rfrag = buffer_rsrc(dsc.bfrag + (size_t)t0 * KB * 64,
                        uniform((int)min((long)(nalloc - t0) * KB * 1024, (long)INT32_MAX)));
    rsa = buffer_rsrc(dsa + (size_t)t0 * kDomTile, left);
    rsd = buffer_rsrc(dsd + (size_t)t0 * kDomTile, left);
    gload(bl0, sa0, sd0, 0);
    // the direct-to-LDS loads count on vmcnt only: every wave drains its own
    // before the barrier that publishes the stage
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // one stage on LDS buffer `buf` (a constant: each buffer is one array)
    auto stage = [&](auto bc, int stg) {
        constexpr int buf = decltype(bc)::value;
        uint4 *const Bs = buf ? bl1 : bl0;
        const float *const As = buf ? sa1 : sa0;
        const float *const Ds = buf ? sd1 : sd0;
        if (stg + 1 < nstage) {
            if constexpr (buf) gload(bl0, sa0, sd0, stg + 1);
            else gload(bl1, sa1, sd1, stg + 1);
        }
        // the range bests of other workgroups: issued after the stage prefetch
        // (so its wait does not include them) and applied at the stage end
        int64_t gl[RQ];
#pragma unroll
        for (int qi = 0; qi < RQ; ++qi) gl[qi] = SHARE && rr[qi] >= 0 ? gbest_load(&ri[rr[qi]].gbest) : INT64_MAX;
        if (wave_on) {
            const int tbase = t0 + stg * DT;
            // software pipeline: the MFMAs of tile dt+1 are issued before the
            // prune test of tile dt, in the same basic block
            Acc acc[2][RQ][2][NP];
            v4i Bq[2][KR];
            // the per-domain values are read one tile ahead of their test, so
            // the test never waits for LDS
            float sq_n = FT ? 0.f : As[lane & 15], sd_n = FT ? 0.f : Ds[lane & 15];
            if constexpr (PREF) read_tile(Bq[0], Bs, 0);
            mfma_tile(acc[0], Bs, 0, Bq[0]);
            if (PREF && DT > 1) read_tile(Bq[1], Bs, 1);
#pragma unroll
            for (int dt = 0; dt < DT; ++dt) {
                const int cur = dt & 1;
                const int col = dt * kDomTile + (lane & 15);
                const float sqa = sq_n;
                float sd4f = sd_n;
                if (dt + 1 < DT) {
                    if constexpr (!FT) {
                        sq_n = As[col + kDomTile];
                        sd_n = Ds[col + kDomTile];
                    }
                    mfma_tile(acc[cur ^ 1], Bs, dt + 1, Bq[(dt + 1) & 1]);
                    // the set of tile dt is free once tile dt's MFMAs were issued
                    if (PREF && dt + 2 < DT) read_tile(Bq[dt & 1], Bs, dt + 2);
                }
                bool pass[RQ];
                bool any = false;
                MaxT mx[RQ];
                if constexpr (FT) {
                    // the threshold is in the accumulators: max over the 8 isometries > 0
#pragma unroll
                    for (int qi = 0; qi < RQ; ++qi) {
                        mx[qi] = cmax(acc[cur][qi][0], acc[cur][qi][1]);
                        pass[qi] = mx[qi] > 0.f;
                        any |= pass[qi];
                    }
                } else {
#pragma unroll
                    for (int qi = 0; qi < RQ; ++qi) {
                        mx[qi] = cmax(acc[cur][qi][0], acc[cur][qi][1]);
                        const float rhs = fmaf(tn[qi], sqa, fmaf(-bn[qi], sd4f, -an[qi]));
                        // false on NaN: rows past the ranges, domains past the
                        // pool or the chunk, and ranges already at val 0
                        pass[qi] = (float)mx[qi] > rhs;
                        any |= pass[qi];
                    }
                }
                // f16 form: issue the next tile's MFMAs one at a time between
                // groups of 3 VALU of this test (measured ~2 % faster at B = 8)
                if (PL == 3 && dt + 1 < DT) {
#pragma unroll
                    for (int i = 0; i < RQ * 2 * KB; ++i) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
                        __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);   // VALU
                    }
                }
                if (__builtin_amdgcn_ballot_w64(any)) {  // rare: exact evaluation, then share the best
                    const int p = tbase * kDomTile + col;
                    // Sd4 < 2^24: exact in float.  A passing pair is a pool domain
                    // (p < P), except in the fused form, whose confirm runs in every
                    // lane: there a domain past the pool reads padding (NaN, no pair
                    // of it passes) and no A
                    const int64_t sd4 = (int64_t)(FT ? dsd_g[p] : sd4f);
                    const int64_t Ad = p < P ? pa[p] : 0;
                    // FT: the domain tile's fragment again, for acc1 without the threshold
                    v4i bt1 = v4i{0, 0, 0, 0};
                    int64_t ed = 0;
                    if constexpr (FT) {
                        const uint4 u = Bs[(dt * KB) * 64 + lane];
                        bt1 = v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
                        ed = sd4 - (int64_t)n * round_mean(sd4, n);
                    }
#pragma unroll
                    for (int qi = 0; qi < RQ; ++qi) {
                        bool imp = false;
                        if constexpr (FT) {
                            // all lanes: the MFMA is wave-wide
                            const v4i z = v4i{0, 0, 0, 0};
                            const v4i a0 = lane < 32 ? A[qi][0][0] : z, a1 = lane < 32 ? A[qi][1][0] : z;
                            const v4f x0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(a0), as_h8(bt1), v4f{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                            const v4f x1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h8(a1), as_h8(bt1), v4f{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                            if (pass[qi]) {
                                const float c1 = max8f(x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w);
                                const int64_t er = (int64_t)rng(qi).sr - (int64_t)n * round_mean(rng(qi).sr, n);
                                imp = confirm_bx((int64_t)n * (int64_t)c1 - er * ed, p, Ad, rng(qi).cr, sl, sc, best[qi],
                                                 bp[qi], bk[qi]);
                            }
                        } else if (pass[qi]) {
                            imp = confirm_pair((int)mx[qi], p, sd4, Ad, rng(qi).sr, rng(qi).cr, n, sl, sc, best[qi], bp[qi], bk[qi]);
                        }
                        // only a lane best that tightens the shared one is worth sharing
                        // (or a walk's own 0, which ends the walk for the range)
                        imp = imp && (best[qi] < rng(qi).tb || best[qi] == 0);
                        if (__builtin_amdgcn_ballot_w64(imp)) {
                            // the 16 lanes holding this range share their best: the
                            // threshold may use it because a pair is only rejected
                            // when it cannot even tie it
                            const int64_t gb = group_min_val_wave<16>(best[qi]);
                            if (rr[qi] >= 0 && gb <= rng(qi).tb) {
                                rng(qi).tb = gb;
                                tn[qi] = tn_from(gb, rng(qi).cr, sc, tfac);
                                if (SHARE && (lane & 15) == 0) gbest_push(&ri[rr[qi]].gbest, gb);
                            }
                            if constexpr (FT) build_thr(qi);   // uniform: inside a ballot
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int qi = 0; qi < RQ; ++qi) {
            const bool changed = gl[qi] < rng(qi).tb;
            if (changed) {
                rng(qi).tb = gl[qi];
                tn[qi] = tn_shared(gl[qi], rng(qi).cr, sc, tfac);
            }
            if (FT && __builtin_amdgcn_ballot_w64(changed)) build_thr(qi);
        }
        __builtin_amdgcn_s_waitcnt(0);   // this wave's loads of the next stage
        __syncthreads();
    };
    for (int stg = 0; stg < nstage; stg += 2) {
        stage(std::integral_constant<int, 0>{}, stg);
        if (stg + 1 < nstage) stage(std::integral_constant<int, 1>{}, stg + 1);
    }
  }

    if (!wave_on) return;
#pragma unroll
    for (int qi = 0; qi < RQ; ++qi) {
        int64_t v = best[qi];
        int p = bp[qi], kk = bk[qi];
        group_min<16>(v, p, kk);
        if ((lane & 15) == 0 && rr[qi] >= 0) {
            Partial o;
            o.val = v;
            o.p = p == INT32_MAX ? -1 : p;
            o.k = kk;
            part[(size_t)rr[qi] * geo.nslot + slot] = o;
        }
    }
  };
    for (;;) {
        __syncthreads();   // every thread is done with the previous item (LDS, s_item)
        if (tid == 0) s_item = atomicAdd(bt.queue + xcd, 1);
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_item);
        if (idx >= total) break;   // uniform: every wave leaves
        const int im = uniform(find_img(qpre, bt.n, idx));
        run_item(im, uniform(idx - qpre[im]));
    }
}

// ---------------------------------------------------------------- launchers
// Both operand builders in one launch: the range fragments' workgroups
// first, then the domain tiles'.
__global__ __launch_bounds__(256) void k_mfma_prep(BatchDev b, int na) {
    if ((int)blockIdx.x < na) k_mfma_afrag(b, blockIdx.x);
    else k_mfma_bfrag(b, blockIdx.x - na);
}

hipError_t launch_mfma_prep_b(const BatchHost &b, hipStream_t st) {
    const int na = b.blocks[K_AFRAG], nt = na + b.blocks[K_BFRAG];
    if (nt > 0) k_mfma_prep<<<nt, 256, 0, st>>>(b.dev, na);
    return hipGetLastError();
}

template <int KA, int PL, int RQ, int DT, int WPE>
static hipError_t launch_search_t(const BatchHost &b, hipStream_t st) {
    const int grid = persistent_grid((const void *)k_mfma_search<KA, PL, RQ, DT, WPE>, b.blocks[K_SEARCH]);
    k_mfma_search<KA, PL, RQ, DT, WPE><<<grid, 256, 0, st>>>(b.dev, b.ss);
    return hipGetLastError();
}

hipError_t launch_mfma_search_b(const BatchHost &b, hipStream_t st) {
    if (b.blocks[K_SEARCH] == 0) return hipSuccess;
    const int B = b.B;
    const TileShape sh = b.shape;
#define FIC_SEARCH(KA, PL, RQ, DT, WPE) \
    if (sh.pl == PL && sh.rq == RQ && sh.dt == DT && sh.wpe == WPE) return launch_search_t<KA, PL, RQ, DT, WPE>(b, st)
    if (B == 4) {
        FIC_SEARCH(1, 1, 2, 16, 3);
        FIC_SEARCH(1, 1, 1, 16, 3);
        FIC_SEARCH(1, 1, 4, 16, 2);
    } else if (B == 8) {
        FIC_SEARCH(1, 2, 2, 8, 3);
        FIC_SEARCH(1, 2, 2, 16, 2);
        FIC_SEARCH(1, 2, 1, 8, 4);
        FIC_SEARCH(1, 2, 3, 8, 2);
        FIC_SEARCH(1, 2, 4, 8, 2);
        FIC_SEARCH(4, 1, 2, 8, 2);
        FIC_SEARCH(2, 3, 2, 8, 3);
        FIC_SEARCH(2, 3, 2, 12, 3);
        FIC_SEARCH(2, 3, 1, 8, 4);
        FIC_SEARCH(2, 3, 2, 16, 2);
        FIC_SEARCH(2, 3, 3, 8, 2);
        FIC_SEARCH(2, 3, 4, 8, 2);
    } else if (B == 16) {
        FIC_SEARCH(4, 2, 2, 1, 3);
        FIC_SEARCH(4, 2, 2, 1, 2);
        FIC_SEARCH(4, 2, 1, 2, 3);
        FIC_SEARCH(4, 2, 2, 2, 2);
        FIC_SEARCH(4, 2, 1, 1, 4);
        FIC_SEARCH(16, 1, 1, 1, 2);
        FIC_SEARCH(8, 3, 1, 2, 3);
        FIC_SEARCH(8, 3, 2, 1, 2);
        FIC_SEARCH(8, 3, 1, 1, 4);
        FIC_SEARCH(8, 3, 2, 2, 2);
    } else if (B == 32) {
        FIC_SEARCH(16, 2, 1, 1, 2);
        FIC_SEARCH(16, 2, 2, 1, 1);
        FIC_SEARCH(16, 2, 1, 2, 1);
    }
    if (B == 4 || B == 2) {
        FIC_SEARCH(1, 4, 2, 8, 3);
        FIC_SEARCH(1, 4, 2, 16, 3);
        FIC_SEARCH(1, 4, 1, 8, 4);
        FIC_SEARCH(1, 4, 2, 8, 4);
        FIC_SEARCH(1, 4, 3, 8, 3);
        FIC_SEARCH(1, 4, 4, 8, 2);
    }
#undef FIC_SEARCH
    return hipErrorInvalidValue;
}

}  // namespace fic
