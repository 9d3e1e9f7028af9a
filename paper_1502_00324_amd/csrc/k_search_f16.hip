// Half-precision MFMA search engine (gfx950, v_mfma_f32_32x32x16_f16).
//
// The cross term of every (range, isometry) x domain pair is contracted over
// the K = B^2 decimated positions (Sec. 3.1) with no replicated or split
// operands:
//   rows    = (range, isometry): the range seen through the inverse isometry,
//             minus 128, in [-128, 127];
//   columns = pool domains: D4 - 512, in [-512, 508] (D4 = 2x2 sum);
//   C' = sum (r - 128)(D4 - 512), the same integer as the int8 engines.
// Every operand is an integer below 2^11, so exact in f16, and every product
// and partial sum is an integer of magnitude <= B^2 2^16 <= 2^24 for B <= 16,
// so exact in the f32 accumulator whatever the summation order.  The prune
// test and the isometry maximum then run on the float results directly.
//
// Fragment layouts (16 bytes = 8 halves per lane, 64 lanes per 1 KiB; lane L
// feeds A row L%32 and B column L%32 with K-values 8(L/32)..+7 of the
// 16-deep step; result lane L holds column L%32, rows 8j + 4(L/32) + i for
// value 4j + i):
//   A: quad q of 4 ranges, K-step s:   afrag[(q*KS + s)*64 + L]
//      row m: j = m/8, h = (m/4)%2, i = m%4 -> range 4q + 2h + j/2,
//      isometry 4(j%2) + i
//   B: tile of 32 domains, K-step s:   bfrag[(tile*KS + s)*64 + L]
//   K index k = 16 s + 8 (L/32) + e -> decimated position (k / B, k % B).
// With rows arranged this way lane L holds all 8 isometries of two ranges
// (4q + 2(L/32) and the next) against domain L%32: values 0..7 and 8..15.
//
// Up to B = 8 the operands are centred at each block's own rounded mean
// instead: r - m_r and D4 - m_d with m_r = round(Sr/n), m_d = round(Sd4/n)
// (magnitudes <= 255 and <= 1020, exact in f16; sums <= n 2^18 <= 2^24,
// exact in f32).  Then acc = Bx/n + e_r e_d / n with e_r = Sr - n m_r,
// e_d = Sd4 - n m_d and |e_r e_d / n| <= n/4, so the prune test
// Bx/n > tn sqrt(A) becomes acc > tn sqrt(A) - (n/2 + 4) (n/4 for the
// centring, n/4 + 4 of float margin as in the other engines): one FMA per
// pair instead of two, and the confirm takes Bx = n acc - e_r e_d.
#include <stdio.h>
#include <stdlib.h>

#include <type_traits>

#include "fic_internal.h"
#include "search_common.h"

namespace fic {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f16x __attribute__((ext_vector_type(16)));

bool f16_supported(int B) { return B == 2 || B == 4 || B == 8 || B == 16; }

// Mean-centred operands (the header describes them): every size up to 8.
__host__ __device__ inline bool f16_centred(int B) { return B <= 8; }
// Normalised domain operands with the threshold in the accumulator input
// (one K-step: B = 2 and 4); the exact tiles are kept beside them.
__host__ __device__ inline bool f16_normalised(int B) { return B <= 4; }

// Range quads per wave (RQ), domain tiles per LDS stage (DT) and the
// occupancy the register allocation aims at (waves per SIMD); the first entry
// per size is the measured default, FIC_F16_SHAPE="rq,dt,wpe" selects another
// compiled one.
struct F16Shape { int B, rq, dt, wpe; };
static const F16Shape kF16Shapes[] = {
    {2, 1, 8, 3},
    {4, 1, 16, 4}, {4, 1, 16, 3}, {4, 1, 8, 3}, {4, 2, 8, 2}, {4, 1, 4, 3}, {4, 1, 8, 4},
    {8, 2, 4, 2}, {8, 1, 4, 3}, {8, 1, 8, 2}, {8, 2, 2, 2},
    {16, 1, 1, 3}, {16, 1, 2, 2},
};
// Candidates of B in table order; index 0 is the default.
int f16_shape_count(int B) {
    int c = 0;
    for (const F16Shape &s : kF16Shapes) c += s.B == B;
    return c;
}
bool f16_shape_at(int B, int index, TileShape &out) {
    int c = 0;
    for (const F16Shape &s : kF16Shapes)
        if (s.B == B && c++ == index) {
            out = TileShape{0, s.rq, s.dt, s.wpe};
            return true;
        }
    return false;
}
TileShape f16_pick(int B, int choice) {
    const char *e = getenv("FIC_F16_SHAPE");
    int rq = 0, dt = 0, wpe = 0;
    if (e && sscanf(e, "%d,%d,%d", &rq, &dt, &wpe) == 3)
        for (const F16Shape &s : kF16Shapes)
            if (s.B == B && s.rq == rq && s.dt == dt && s.wpe == wpe) return TileShape{0, s.rq, s.dt, s.wpe};
    TileShape t{0, 1, 1, 1};
    if (choice >= 0 && f16_shape_at(B, choice, t)) return t;
    f16_shape_at(B, 0, t);
    return t;
}

MfmaGeom f16_geometry(int B, int range_cap, int pool_cap, const TileShape &sh) {
    MfmaGeom g;
    g.pl = 0;
    g.ka = (B * B + 15) / 16;   // B = 2: the 4 positions zero-padded to one step
    g.kt = g.ka;
    g.rpw = 16 * sh.rq;
    const int ntiles = (pool_cap + kDomTile32 - 1) / kDomTile32;
    split_chunks(g, range_cap, ntiles, g.kt, sh.dt, false, 4);
    return g;
}

// ---------------------------------------------------------------- operands
__device__ __forceinline__ void k_f16_afrag(const BatchDev &b, const int bid) {
    const int *pre = b.pre + K_AFRAG * (b.n + 1);
    const int im = find_img(pre, b.n, bid);
    const ImgLvl &d = b.d[im];
    const int B = d.B, KS = d.geo.ka;
    const int nquads = d.geo.nrg * (d.geo.rpw / 4);
    const int64_t slot = (int64_t)(bid - pre[im]) * 256 + threadIdx.x;
    if (slot >= (int64_t)nquads * KS * 64) return;
    const int lane = (int)(slot & 63);
    const int rest = (int)(slot >> 6);
    const int s = rest % KS, q = rest / KS;
    const int m = lane & 31, kb = lane >> 5;
    const int j = m >> 3, h = (m >> 2) & 1, i = m & 3;
    const int js = 4 * q + 2 * h + (j >> 1);   // entry of the search list
    const int r = js < *d.ns ? d.sidx[js] : -1;
    const int t = 4 * (j & 1) + i;
    h8 w;
    if (r >= 0) {
        const uint32_t v = d.rxy[r];
        const int x0 = v & 0xffff, y0 = v >> 16;
        const int ti = iso_inv(t);
        const int cen = f16_centred(B) ? round_mean(d.ri[r].sr, B * B) : 128;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 16 * s + 8 * kb + e;
            if (k >= B * B) {   // padding of the last step (B = 2)
                w[e] = (_Float16)0;
                continue;
            }
            const int cy = k / B, cx = k - cy * B;
            int sy, sx;
            iso_src(ti, B, cy, cx, sy, sx);
            w[e] = (_Float16)((int)d.pix[(size_t)(y0 + sy) * d.pitch + x0 + sx] - cen);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = (_Float16)0;
    }
    ((h8 *)d.afrag)[slot] = w;
}

// Domain operands: f16_tiles(pool_cap) tiles, the last kF16PadTiles of them
// zero, so that a stage may read past a chunk's end without a bound check.
// Per domain, structure of arrays in dinfo: Sd4 for all the tiles' domains,
// then sqrt(A) rounded down (NaN past the pool: no pair on them passes the
// test), then with centring the pair (A, Sd4) as 32-bit integers, which the
// exact evaluation reads from LDS (A <= n^2 1020^2 / 4 < 2^32 for B <= 8).
__device__ __forceinline__ void k_f16_bfrag(const BatchDev &b, const int bid) {
    const int *pre = b.pre + K_BFRAG * (b.n + 1);
    const int im = find_img(pre, b.n, bid);
    const ImgLvl &d = b.d[im];
    const int B = d.B, KS = d.geo.kt;
    const int ntiles = f16_tiles(d.pool_cap);
    const int64_t slot = (int64_t)(bid - pre[im]) * 256 + threadIdx.x;   // can pass 2^31
    if (slot >= (int64_t)ntiles * KS * 64) return;
    const int lane = (int)(slot & 63);
    const int rest = (int)(slot >> 6);
    const int s = rest % KS, tile = rest / KS;
    const int col = lane & 31, kb = lane >> 5;
    const int p = tile * kDomTile32 + col;
    const bool valid = p < min(*d.pcount, d.pool_cap);
    h8 w;
    if (valid) {
        const uint32_t v = d.pxy[p];
        const int x0 = v & 0xffff, y0 = v >> 16, pitch = d.pitch;
        const int cen = f16_centred(B) ? round_mean(d.psum4[p], B * B) : 512;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 16 * s + 8 * kb + e;
            if (k >= B * B) {   // padding of the last step (B = 2)
                w[e] = (_Float16)0;
                continue;
            }
            const int cy = k / B, cx = k - cy * B;
            const uint8_t *q = d.pix + (size_t)(y0 + 2 * cy) * pitch + x0 + 2 * cx;
            w[e] = (_Float16)(q[0] + q[1] + q[pitch] + q[pitch + 1] - cen);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = (_Float16)0;
    }
    if (f16_normalised(B)) {
        // the exact tile goes to the second array (the exact evaluation reads
        // it); the searched one holds 2^16 (D4 - Sd4/n) / sqrt(A): 0 when
        // A = 0, NaN past the pool (a NaN column fails every test)
        ((h8 *)d.bfrag)[(size_t)ntiles * KS * 64 + slot] = w;
        h8 z;
        if (valid) {
            const int n = B * B;
            const float mu = (float)d.psum4[p] / (float)n;   // exact: Sd4 < 2^24, n a power of 2
            const int64_t A = d.pa[p];
            const float inv = A > 0 ? 65536.0f / sqrtf((float)A) : 0.0f;
            const uint32_t v = d.pxy[p];
            const int x0 = v & 0xffff, y0 = v >> 16, pitch = d.pitch;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 16 * s + 8 * kb + e;
                if (k >= n) {
                    z[e] = (_Float16)0;
                    continue;
                }
                const int cy = k / B, cx = k - cy * B;
                const uint8_t *q = d.pix + (size_t)(y0 + 2 * cy) * pitch + x0 + 2 * cx;
                z[e] = (_Float16)(((float)(q[0] + q[1] + q[pitch] + q[pitch + 1]) - mu) * inv);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) z[e] = (_Float16)__builtin_nanf("");
        }
        w = z;
    }
    ((h8 *)d.bfrag)[slot] = w;
    if (s == 0 && kb == 0) {
        float *dsd = (float *)d.dinfo, *dsa = dsd + (size_t)ntiles * kDomTile32;
        dsd[p] = valid ? (float)d.psum4[p] : __builtin_nanf("");
        dsa[p] = valid ? sqrt_down((double)d.pa[p]) : __builtin_nanf("");
        if (f16_centred(B)) {
            uint2 *dsx = (uint2 *)(dsa + (size_t)ntiles * kDomTile32);
            dsx[p] = valid ? make_uint2((uint32_t)d.pa[p], (uint32_t)d.psum4[p]) : make_uint2(0u, 0u);
        }
    }
}

// ---------------------------------------------------------------- search
// A workgroup of 4 waves owns 16 RQ ranges (each wave RQ quads) and the
// domain tiles of its chunks.  Domain fragments and the per-domain values
// go straight from global memory into LDS in stages of DT tiles,
// double-buffered (the loads of stage s+1 are issued before the MFMAs of
// stage s), through buffer resources based at the chunk's first tile: a
// stage's loads differ only by a scalar offset, so they take no vector
// instructions.  Per domain a stage holds sqrt(A) for the prune test and,
// with centring, the exact (A, Sd4) of the exact evaluation (without it, Sd4
// for the test), so a passing pair is evaluated from LDS and registers: a
// global load there would also wait for the stage prefetch, the vector
// memory counter being in order.  The normalised form (B <= 4) stages
// fragments only: its test needs no per-domain value, and its rare exact
// evaluation reads the exact tile and the domain's values from global
// memory (staging them measured slower).  A chunk's last stage may read up to
// DT - 1 tiles past its end: the next chunk's domains (evaluated twice,
// harmless: the partials merge by (val, domain)) or the zero padding tiles,
// whose NaN sqrt(A) never passes.  The MFMAs of tile t+1 are issued before
// the prune test of tile t.
template <int KS, int RQ, int DT, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_f16_search(BatchDev bt, SSet ss) {
    constexpr bool CEN = KS <= 4;                // mean-centred operands (B <= 8)
    constexpr bool NORM = KS == 1;               // normalised domains, threshold in the accumulator (B <= 4)
    constexpr int G = NORM ? 4 : 1;              // tiles per pass test (normalised form)
    constexpr int STAGE = DT * KS * 64;          // uint4 per stage
    // domains per stage whose values are staged: none for the normalised
    // form (only its exact evaluation reads them, from global memory)
    constexpr int ND = NORM ? 1 : DT * kDomTile32;
    // share range bests across workgroups only when a stage is long enough
    // (>= 4 tiles) to hide the coherent load of the shared values
    constexpr bool SHARE = DT >= 4;
    constexpr int PER_T = STAGE / 256;
    constexpr int PER_D = (ND + 255) / 256;
    constexpr int NX = NORM ? 1 : ND / 2;        // 16-byte (A, Sd4) records of two domains
    constexpr int PER_X = (NX + 255) / 256;
    static_assert(STAGE % 256 == 0, "stage must split evenly over 256 threads");
    static_assert(DT <= kF16PadTiles, "a stage reads at most DT - 1 tiles past a chunk");
    // the two stage buffers, separate arrays: a stage's direct-to-LDS loads
    // into one are then known not to touch the other
    __shared__ uint4 bl0[STAGE];
    __shared__ uint4 bl1[STAGE];
    __shared__ float sa0[ND], sa1[ND];                          // sqrt(A) rounded down
    __shared__ float sd0[CEN ? 1 : ND], sd1[CEN ? 1 : ND];      // Sd4 (the uncentred test only)
    __shared__ uint4 sx0[CEN ? NX : 1], sx1[CEN ? NX : 1];      // exact (A, Sd4) (centred only)
    __shared__ SLds sl;
    __shared__ int s_item;
    // per range (4 waves x RQ quads x 4 ranges): values only the rare paths
    // read (Cr, the best value the threshold reflects, the centring error e_r,
    // the normalised margin), kept in LDS rather than in registers the tile
    // loop needs
    struct RangeLds { int64_t cr, tb; int er; float marg; };
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
    // the level's pointers and sizes in scalar registers (alike in every lane)
    const gptr<h8> afrag = as_global((const h8 *)uniform(dsc.afrag));
    RInfo *__restrict__ ri = uniform(dsc.ri);
    const gptr<int64_t> pa = as_global((const int64_t *)uniform(dsc.pa));
    Partial *__restrict__ part = uniform(dsc.part);
    const int range_cap = uniform(dsc.range_cap), pool_cap = uniform(dsc.pool_cap), n = uniform(dsc.B * dsc.B);
    const int nalloc = f16_tiles(pool_cap);
    const float *dsd = (const float *)uniform(dsc.dinfo), *dsa = dsd + (size_t)nalloc * kDomTile32;
    const uint2 *dsx = (const uint2 *)(dsa + (size_t)nalloc * kDomTile32);
    const gptr<float> dsa_g = as_global(dsa);
    const gptr<uint64_t> dsx_g = as_global((const uint64_t *)dsx);   // (A, Sd4): low, high word
    // the exact copy of the tiles (normalised form), after the searched ones
    const gptr<h8> bfx = as_global((const h8 *)(uniform(dsc.bfrag) + (size_t)nalloc * KS * 64));
    const float tfac = tn_factor(n);
    const float cmargin = (float)(n / 2 + 4);   // centred test: n/4 centring + n/4 + 4 float margin
    // R: the length of the search list (constant ranges are coded already)
    const int R = uniform(min(*dsc.ns, range_cap)), P = uniform(min(*dsc.pcount, pool_cap));
    int rg, cfirst, cstep, ncs, slot;
    item_walk(geo, R, xcd, k, rg, cfirst, cstep, ncs, slot, true);
    const gptr<int32_t> sidx = as_global((const int32_t *)uniform(dsc.sidx));
    const int ntiles = (P + kDomTile32 - 1) / kDomTile32;
    const int q0 = (rg * 4 + wave) * RQ;
    const bool wave_on = q0 * 4 < R;
    const int hh = lane >> 5;

    // per lane: two ranges per quad, 4 q + 2 hh + u for u = 0, 1
    h8 A[RQ][KS];
    float tn[RQ][2], bn[RQ][2], an[RQ][2];
    // normalised form: the accumulator input of every tile, -(threshold) of
    // the lane's two ranges (values 0..7 and 8..15), and its error margin
    f16x cth[NORM ? RQ : 1];
    int64_t best[RQ][2];
    int bp[RQ][2], bk[RQ][2], rr[RQ][2], sr[RQ][2];
    const auto rng = [&](int qi, int u) -> RangeLds & { return s_rng[((wave * RQ + qi) * 2 + hh) * 2 + u]; };
    const int lgn = __builtin_ctz(n);   // n = B^2, B a power of two
    // The normalised test: acc' = sum (r - m_r) 2^16 (D4 - Sd4/n)/sqrt(A) + c is
    // 2^16 Bx/(n sqrt A) + c up to the range's margin, and a pair can reach
    // the best only if Bx/(n sqrt A) > tn, so with c = margin - 2^16 tn (1 -
    // 2^-20) (the 2^-20 covers the float roundings of c and of the sum) it
    // passes only if acc' > 0.  No best yet: c = 1e30, every pair passes; a
    // row without a range, or a range whose walk found val 0: -inf, none.
    // (one range's half of the accumulator input: values 8u .. 8u + 7)
    auto build_cth_half = [&](int qi, int u) {
        const float t = tn[qi][u];
        const float c = (rr[qi][u] < 0 || __builtin_isnan(t)) ? -__builtin_inff()
                      : t < -1e29f ? 1e30f
                                   : rng(qi, u).marg - 65536.0f * t * (1.0f - 1.0f / 1048576.0f);
#pragma unroll
        for (int e = 0; e < 8; ++e) cth[NORM ? qi : 0][8 * u + e] = c;
    };
    auto build_cth = [&](int qi) {
        build_cth_half(qi, 0);
        build_cth_half(qi, 1);
    };
#pragma unroll
    for (int qi = 0; qi < RQ; ++qi) {
#pragma unroll
        for (int s = 0; s < KS; ++s) A[qi][s] = afrag[((size_t)(q0 + qi) * KS + s) * 64 + lane];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int js = (q0 + qi) * 4 + 2 * hh + u;
            const int r = js < R ? sidx[js] : -1;
            rr[qi][u] = r;
            const RInfo x = ri[r >= 0 ? r : 0];
            bn[qi][u] = x.bn;
            an[qi][u] = x.an;
            sr[qi][u] = (int)x.sr;
            // every lane of the range writes the same values (no other wave reads them)
            RangeLds &rl = rng(qi, u);
            // e_r = Sr - n round(Sr / n): the centring error of the range
            rl.er = (int)x.sr - (((int)x.sr + n / 2) >> lgn << lgn);
            rl.cr = x.cr;
            tn[qi][u] = r >= 0 ? -1e30f : __builtin_nanf("");  // NaN: the row never passes
            rl.tb = INT64_MAX;
            // start from the best other walks of this range have shared (a
            // stale copy only loosens the test)
            if (r >= 0 && x.gbest < INT64_MAX) {
                rl.tb = x.gbest;
                tn[qi][u] = tn_shared(x.gbest, x.cr, sc, tfac);
            }
            best[qi][u] = INT64_MAX;
            bp[qi][u] = INT32_MAX;
            bk[qi][u] = 0;
            // |sum a_i (w~_i - w_i)| <= 2^-10 |a| |w| with a = r - m_r and |w| = 2^16/sqrt(n):
            // |a|^2 = Cr/n + n (mean - m_r)^2 <= Cr/n + n/4 (rounded up here)
            rl.marg = NORM ? 64.0f * sqrtf((float)x.cr / (float)n + 0.25f * (float)n + 1.0f) * (1.0f + 1.0f / 1024.0f) /
                                     sqrtf((float)n)
                               : 0.f;
        }
        if constexpr (NORM) build_cth(qi);
    }
    // drain the one-time loads: vmcnt is in-order, so a wait for them inside
    // the tile loop would also wait for the stage prefetch
    __builtin_amdgcn_s_waitcnt(0);

    typedef __attribute__((address_space(3))) void *lds_t;
    // the wave index as a scalar: the LDS destination of a direct load is a
    // per-wave base in M0
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    int t0 = 0;
    __amdgpu_buffer_rsrc_t rfrag, rsa, rsd, rsx;
    // one stage of the current chunk into the LDS buffers given: fragments,
    // then per-domain values; wave w fills its own 64-slot blocks
    auto gload = [&](uint4 *fdst, float *adst, float *ddst, uint4 *xdst, int stg) {
#pragma unroll
        for (int i = 0; i < PER_T; ++i)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rfrag, (lds_t)(fdst + 64 * wv + 256 * i), 16,
                                                     (unsigned)(tid + 256 * i) * 16u, (unsigned)stg * STAGE * 16u, 0,
                                                     0);
#pragma unroll
        for (int i = 0; i < (NORM ? 0 : PER_D); ++i) {
            if (ND % 256 == 0 || tid + 256 * i < ND) {
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rsa, (lds_t)(adst + 64 * wv + 256 * i), 4,
                                                         (unsigned)(tid + 256 * i) * 4u, (unsigned)stg * ND * 4u, 0,
                                                         0);
                if constexpr (!CEN)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsd, (lds_t)(ddst + 64 * wv + 256 * i), 4,
                                                             (unsigned)(tid + 256 * i) * 4u, (unsigned)stg * ND * 4u,
                                                             0, 0);
            }
        }
        if constexpr (CEN && !NORM) {
#pragma unroll
            for (int i = 0; i < PER_X; ++i)
                if (NX % 256 == 0 || tid + 256 * i < NX)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsx, (lds_t)(xdst + 64 * wv + 256 * i), 16,
                                                             (unsigned)(tid + 256 * i) * 16u,
                                                             (unsigned)stg * ND * 8u, 0, 0);
        }
    };
    // With up to 4 K-steps a tile's fragments are read into registers ahead
    // of its MFMAs, NSET sets in rotation: the read of tile t + NSET is issued
    // right after the MFMAs of tile t + 1, so it has NSET - 1 prune tests to
    // land before its own MFMAs (three sets where the registers allow; at
    // four waves per SIMD two, the other waves covering the wait).
    // Longer tiles read them in groups of 8, so one LDS wait covers a group
    // rather than every MFMA.
    constexpr bool PREF = KS <= 4;
    constexpr int KG = PREF ? KS : 8;
    constexpr int NSET = PREF && ((KS == 1 && WPE <= 3) || WPE <= 2) ? 3 : 2;
    auto read_tile = [&](h8 (&bf)[KG], const uint4 *Bs, int dt, int s0) {
#pragma unroll
        for (int s = 0; s < KG; ++s) {
            const uint4 u = Bs[(dt * KS + s0 + s) * 64 + lane];
            __builtin_memcpy(&bf[s], &u, sizeof(h8));
        }
    };
    auto mfma_tile = [&](f16x (&acc)[RQ], const uint4 *Bs, int dt, h8 (&bq)[KG]) {
#pragma unroll
        for (int qi = 0; qi < RQ; ++qi) acc[qi] = NORM ? cth[NORM ? qi : 0] : f16x{0.f};
#pragma unroll
        for (int s0 = 0; s0 < KS; s0 += KG) {
            if constexpr (!PREF) read_tile(bq, Bs, dt, s0);
#pragma unroll
            for (int s = 0; s < KG; ++s)
#pragma unroll
                for (int qi = 0; qi < RQ; ++qi)
                    acc[qi] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[qi][s0 + s], bq[s], acc[qi], 0, 0, 0);
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
        const long dl = (long)(nalloc - t0) * kDomTile32;
        rfrag = buffer_rsrc(dsc.bfrag + (size_t)t0 * KS * 64, uniform((int)min(dl / kDomTile32 * KS * 1024, (long)INT32_MAX)));
        rsa = buffer_rsrc(dsa + (size_t)t0 * kDomTile32, uniform((int)min(dl * 4, (long)INT32_MAX)));
        rsd = buffer_rsrc(dsd + (size_t)t0 * kDomTile32, uniform((int)min(dl * 4, (long)INT32_MAX)));
        rsx = buffer_rsrc(dsx + (size_t)t0 * kDomTile32, uniform((int)min(dl * 8, (long)INT32_MAX)));
        gload(bl0, sa0, sd0, sx0, 0);
        // the direct-to-LDS loads count on vmcnt only: every wave drains its
        // own before the barrier that publishes the stage
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        // one stage on LDS buffer `buf` (a constant: each buffer is one array)
        auto stage = [&](auto bc, int stg) {
            constexpr int buf = decltype(bc)::value;
            uint4 *const Bs = buf ? bl1 : bl0;
            const float *const As = buf ? sa1 : sa0;
            const float *const Ds = buf ? sd1 : sd0;
            const uint2 *const Xs = (const uint2 *)(buf ? sx1 : sx0);
            if (stg + 1 < nstage) {
                if constexpr (buf) gload(bl0, sa0, sd0, sx0, stg + 1);
                else gload(bl1, sa1, sd1, sx1, stg + 1);
            }
            // the range bests of other workgroups: issued after the stage
            // prefetch (so its wait does not include them), applied at the end
            int64_t gl[RQ][2];
#pragma unroll
            for (int qi = 0; qi < RQ; ++qi)
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    gl[qi][u] = SHARE && rr[qi][u] >= 0 ? gbest_load(&ri[rr[qi][u]].gbest) : INT64_MAX;
            if (wave_on) {
                const int tbase = t0 + stg * DT;
                f16x acc[2][RQ];
                h8 bq[NSET][KG];
                float gmx[RQ];   // normalised form: the running maximum of the current group
                // the per-domain values are read two tiles ahead of their test
                // (a ring of two), so the test never waits for LDS
                float sqv[2] = {0.f, 0.f}, sdv[2];
                sqv[0] = NORM ? 0.f : As[lane & 31];
                sdv[0] = CEN ? 0.f : Ds[lane & 31];
                if (!NORM && DT > 1) {
                    sqv[1] = As[kDomTile32 + (lane & 31)];
                    sdv[1] = CEN ? 0.f : Ds[kDomTile32 + (lane & 31)];
                }
                if constexpr (PREF) {
#pragma unroll
                    for (int j = 0; j < NSET - 1; ++j)
                        if (j < DT) read_tile(bq[j], Bs, j, 0);
                }
                mfma_tile(acc[0], Bs, 0, bq[0]);
                if (PREF && NSET - 1 < DT) read_tile(bq[NSET - 1], Bs, NSET - 1, 0);
#pragma unroll
                for (int dt = 0; dt < DT; ++dt) {
                    const int cur = dt & 1;
                    const int col = dt * kDomTile32 + (lane & 31);
                    const float sqa = sqv[cur], sd4f = sdv[cur];
                    if (dt + 1 < DT) {
                        mfma_tile(acc[cur ^ 1], Bs, dt + 1, bq[(dt + 1) % NSET]);
                        // the set of tile dt is free once tile dt's MFMAs were issued
                        if (PREF && dt + NSET < DT) read_tile(bq[dt % NSET], Bs, dt + NSET, 0);
                        // keep the read here: the scheduler would otherwise sink it
                        // towards its use and expose the LDS latency
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    if (!NORM && dt + 2 < DT) {
                        sqv[cur] = As[col + 2 * kDomTile32];
                        if constexpr (!CEN) sdv[cur] = Ds[col + 2 * kDomTile32];
                    }
                    // the exact evaluation of tile dtj for the lanes in ps (mx: the
                    // isometry maxima of the exact cross terms, the centred form only),
                    // then the range bests shared with the other lanes and walks
                    auto exact_tile = [&](const int dtj, bool (&ps)[RQ][2], float (&mx)[RQ][2], float sd4f) {
                        const int colj = dtj * kDomTile32 + (lane & 31);
                        const int p = tbase * kDomTile32 + colj;
                        // a passing pair has a finite sqrt(A): p is a pool domain
                        int64_t Ad = 0, sd4 = (int64_t)sd4f;   // Sd4 < 2^24: exact in float
                        if constexpr (NORM) {
                            const uint64_t xv = dsx_g[p];
                            Ad = (uint32_t)xv;
                            sd4 = (int64_t)(xv >> 32);
                        } else if constexpr (CEN) {
                            const uint2 xi = Xs[colj];
                            Ad = xi.x;
                            sd4 = xi.y;
                        }
                        if constexpr (NORM) {
                            const float sqx = dsa_g[p];
                            // the exact cross terms of the tile (every lane: the MFMA is
                            // wave-wide), from the exact copy of its fragment
                            const h8 bx = bfx[(size_t)(tbase + dtj) * 64 + lane];
#pragma unroll
                            for (int qi = 0; qi < RQ; ++qi) {
                                const f16x ex = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[qi][0], bx, f16x{0.f}, 0, 0, 0);
#pragma unroll
                                for (int u = 0; u < 2; ++u) {
                                    const int o = 8 * u;
                                    mx[qi][u] = max8f(ex[o], ex[o + 1], ex[o + 2], ex[o + 3], ex[o + 4], ex[o + 5],
                                                      ex[o + 6], ex[o + 7]);
                                    // the centred test on the exact cross term: the normalised
                                    // one passes a few more pairs
                                    ps[qi][u] = ps[qi][u] && rr[qi][u] >= 0 && mx[qi][u] > fmaf(tn[qi][u], sqx, -cmargin);
                                }
                            }
                        }
#pragma unroll
                        for (int qi = 0; qi < RQ; ++qi)
#pragma unroll
                            for (int u = 0; u < 2; ++u) {
                                bool imp = false;
                                if (ps[qi][u]) {
                                    if constexpr (CEN) {
                                        // e_d = Sd4 - n round(Sd4 / n), n a power of two
                                        const int ed = (int)sd4 - (((int)sd4 + n / 2) >> lgn << lgn);
                                        imp = confirm_bx((int64_t)n * (int64_t)mx[qi][u] - (int64_t)rng(qi, u).er * ed, p, Ad,
                                                         rng(qi, u).cr, sl, sc, best[qi][u], bp[qi][u], bk[qi][u]);
                                    } else {
                                        imp = confirm_pair((int)mx[qi][u], p, sd4, pa[p], sr[qi][u], rng(qi, u).cr, n, sl,
                                                           sc, best[qi][u], bp[qi][u], bk[qi][u]);
                                    }
                                }
                                // only a lane best that tightens the shared one is worth sharing
                                // (or a walk's own 0, which ends the walk for the range)
                                imp = imp && (best[qi][u] < rng(qi, u).tb || best[qi][u] == 0);
                                if (__builtin_amdgcn_ballot_w64(imp)) {
                                    // the 32 lanes holding this range share their best: a
                                    // pair is only rejected when it cannot even tie it
                                    const int64_t gb = group_min_val_wave<32>(best[qi][u]);
                                    if (rr[qi][u] >= 0 && gb <= rng(qi, u).tb) {
                                        rng(qi, u).tb = gb;
                                        tn[qi][u] = tn_from(gb, rng(qi, u).cr, sc, tfac);
                                        if (SHARE && (lane & 31) == 0) gbest_push(&ri[rr[qi][u]].gbest, gb);
                                    }
                                    if constexpr (NORM) build_cth_half(qi, u);   // uniform: inside a ballot
                                }
                            }
                    };
                    if constexpr (NORM) {
                        // the threshold is in the accumulators: the largest of the
                        // lane's 16 values (both ranges, 8 isometries) against 0, one
                        // branch per group of G tiles.  The group's running maximum
                        // rides in the spare input of the tile's maximum tree (no extra
                        // instruction); the maximum propagates NaN (a column past the
                        // pool), so a NaN group maximum is treated as a possible pass
                        // and the rare path below tests the group's tiles one by one.
#pragma unroll
                        for (int qi = 0; qi < RQ; ++qi) {
                            const f16x &a = acc[cur][qi];
                            const float prev = dt % G == 0 ? a[7] : gmx[qi];
                            gmx[qi] = FIC_MAX3(FIC_MAX3(max9f(a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], prev),
                                                        a[8], a[9]),
                                               FIC_MAX3(a[10], a[11], a[12]), FIC_MAX3(a[13], a[14], a[15]));
                        }
                        if (dt % G == G - 1 || dt == DT - 1) {
                            const int g0 = dt - dt % G;
                            bool any = false;
#pragma unroll
                            for (int qi = 0; qi < RQ; ++qi) any |= !(gmx[qi] <= 0.f);
                            if (__builtin_expect(__builtin_amdgcn_ballot_w64(any) != 0, 0)) {  // rare
                                // which tiles of the group pass, each tested alone (its
                                // fragment is still in the stage; a tile past the pool gives
                                // NaN, which fails), with the threshold as it is now (at most
                                // tighter than when the group ran: a valid test); then the
                                // passing tiles in order, one at a time (a loop, not
                                // unrolled: one copy of the evaluation)
                                uint32_t pl[RQ], gmask = 0;
#pragma unroll
                                for (int qi = 0; qi < RQ; ++qi) pl[qi] = 0;
#pragma unroll
                                for (int j = 0; j <= dt - g0; ++j) {
                                    h8 fj;
                                    {
                                        const uint4 u = Bs[(g0 + j) * KS * 64 + lane];
                                        __builtin_memcpy(&fj, &u, sizeof(h8));
                                    }
                                    bool anyj = false;
#pragma unroll
                                    for (int qi = 0; qi < RQ; ++qi) {
                                        const f16x e = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[qi][0], fj, cth[qi], 0, 0, 0);
                                        const float m = FIC_MAX3(FIC_MAX3(max8f(e[0], e[1], e[2], e[3], e[4], e[5], e[6], e[7]),
                                                                          e[8], e[9]),
                                                                 FIC_MAX3(e[10], e[11], e[12]), FIC_MAX3(e[13], e[14], e[15]));
                                        const bool b = m > 0.f;
                                        pl[qi] |= b ? 1u << j : 0u;
                                        anyj |= b;
                                    }
                                    gmask |= __builtin_amdgcn_ballot_w64(anyj) ? 1u << j : 0u;
                                }
                                gmask = __builtin_amdgcn_readfirstlane(gmask);
                                while (gmask) {
                                    const int j = __builtin_ctz(gmask);
                                    gmask &= gmask - 1;
                                    bool ps[RQ][2];
                                    float mx[RQ][2];
#pragma unroll
                                    for (int qi = 0; qi < RQ; ++qi) ps[qi][0] = ps[qi][1] = (pl[qi] >> j) & 1u;
                                    exact_tile(g0 + j, ps, mx, 0.f);
                                }
                            }
                        }
                    } else {
                        bool ps[RQ][2];
                        float mx[RQ][2];
                        bool any = false;
#pragma unroll
                        for (int qi = 0; qi < RQ; ++qi)
#pragma unroll
                            for (int u = 0; u < 2; ++u) {
                                const f16x &a = acc[cur][qi];
                                const int o = 8 * u;
                                mx[qi][u] = max8f(a[o], a[o + 1], a[o + 2], a[o + 3], a[o + 4], a[o + 5], a[o + 6], a[o + 7]);
                                const float rhs = CEN ? fmaf(tn[qi][u], sqa, -cmargin)
                                                      : fmaf(tn[qi][u], sqa, fmaf(-bn[qi][u], sd4f, -an[qi][u]));
                                // false on NaN: rows past the ranges, domains past the
                                // pool, and ranges already at val 0
                                ps[qi][u] = mx[qi][u] > rhs;
                                any |= ps[qi][u];
                            }
                        if (__builtin_expect(__builtin_amdgcn_ballot_w64(any) != 0, 0))   // rare
                            exact_tile(dt, ps, mx, sd4f);
                    }
                }
            }
#pragma unroll
            for (int qi = 0; qi < RQ; ++qi) {
                bool changed = false;
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (gl[qi][u] < rng(qi, u).tb) {
                        rng(qi, u).tb = gl[qi][u];
                        tn[qi][u] = tn_shared(gl[qi][u], rng(qi, u).cr, sc, tfac);
                        changed = true;
                    }
                if (NORM && __builtin_amdgcn_ballot_w64(changed)) build_cth(qi);
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
    for (int qi = 0; qi < RQ; ++qi)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            int64_t v = best[qi][u];
            int p = bp[qi][u], kk = bk[qi][u];
            group_min<32>(v, p, kk);
            if ((lane & 31) == 0 && rr[qi][u] >= 0) {
                Partial o;
                o.val = v;
                o.p = p == INT32_MAX ? -1 : p;
                o.k = kk;
                part[(size_t)rr[qi][u] * geo.nslot + slot] = o;
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
__global__ __launch_bounds__(256) void k_f16_prep(BatchDev b, int na) {
    if ((int)blockIdx.x < na) k_f16_afrag(b, blockIdx.x);
    else k_f16_bfrag(b, blockIdx.x - na);
}

hipError_t launch_f16_prep_b(const BatchHost &b, hipStream_t st) {
    const int na = b.blocks[K_AFRAG], nt = na + b.blocks[K_BFRAG];
    if (nt > 0) k_f16_prep<<<nt, 256, 0, st>>>(b.dev, na);
    return hipGetLastError();
}

template <int KS, int RQ, int DT, int WPE>
static hipError_t launch_f16_t(const BatchHost &b, hipStream_t st) {
    const int grid = persistent_grid((const void *)k_f16_search<KS, RQ, DT, WPE>, b.blocks[K_SEARCH]);
    k_f16_search<KS, RQ, DT, WPE><<<grid, 256, 0, st>>>(b.dev, b.ss);
    return hipGetLastError();
}

hipError_t launch_f16_search_b(const BatchHost &b, hipStream_t st) {
    if (b.blocks[K_SEARCH] == 0) return hipSuccess;
    const int B = b.B;
    const TileShape sh = b.shape;
#define FIC_F16(KS, RQ, DT, WPE) \
    if (sh.rq == RQ && sh.dt == DT && sh.wpe == WPE) return launch_f16_t<KS, RQ, DT, WPE>(b, st)
    if (B == 2) {
        FIC_F16(1, 1, 8, 3);
    } else if (B == 4) {
        FIC_F16(1, 1, 16, 3);
        FIC_F16(1, 1, 8, 3);
        FIC_F16(1, 2, 8, 2);
        FIC_F16(1, 1, 4, 3);
        FIC_F16(1, 1, 16, 4);
        FIC_F16(1, 1, 8, 4);
    } else if (B == 8) {
        FIC_F16(4, 2, 4, 2);
        FIC_F16(4, 1, 4, 3);
        FIC_F16(4, 1, 8, 2);
        FIC_F16(4, 2, 2, 2);
    } else if (B == 16) {
        FIC_F16(16, 1, 1, 3);
        FIC_F16(16, 1, 2, 2);
    }
#undef FIC_F16
    return hipErrorInvalidValue;
}

}  // namespace fic
