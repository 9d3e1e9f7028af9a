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

// Range quads per wave (RQ), domain tiles per LDS stage (DT) and the
// occupancy the register allocation aims at (waves per SIMD); the first entry
// per size is the measured default, FIC_F16_SHAPE="rq,dt,wpe" selects another
// compiled one.
struct F16Shape { int B, rq, dt, wpe; };
static const F16Shape kF16Shapes[] = {
    {2, 1, 8, 4},
    {4, 1, 8, 4}, {4, 2, 8, 2}, {4, 1, 16, 3}, {4, 2, 4, 3}, {4, 1, 8, 3},
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
__global__ __launch_bounds__(256) void k_f16_afrag(BatchDev b) {
    const int *pre = b.pre + K_AFRAG * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int B = d.B, KS = d.geo.ka;
    const int nquads = d.geo.nrg * (d.geo.rpw / 4);
    const int64_t slot = (int64_t)(blockIdx.x - pre[im]) * 256 + threadIdx.x;
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

__global__ __launch_bounds__(256) void k_f16_bfrag(BatchDev b) {
    const int *pre = b.pre + K_BFRAG * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int B = d.B, KS = d.geo.kt;
    const int ntiles = (d.pool_cap + kDomTile32 - 1) / kDomTile32;
    const int64_t slot = (int64_t)(blockIdx.x - pre[im]) * 256 + threadIdx.x;   // can pass 2^31
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
    ((h8 *)d.bfrag)[slot] = w;
    if (s == 0 && kb == 0)
        d.dinfo[p] = valid ? make_float2((float)d.psum4[p], sqrt_down((double)d.pa[p]))
                           : make_float2(__builtin_nanf(""), __builtin_nanf(""));  // never passes
}

// ---------------------------------------------------------------- search
// A workgroup of 4 waves owns 16 RQ ranges (each wave RQ quads) and the
// domain tiles of its chunks.  Domain fragments go straight from global
// memory into LDS in stages of DT tiles, double-buffered (the loads of stage
// s+1 are issued before the MFMAs of stage s); the per-domain moments pass
// through registers.  The MFMAs of tile t+1 are issued before the prune test
// of tile t.
template <int KS, int RQ, int DT, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_f16_search(BatchDev bt, SSet ss) {
    constexpr bool CEN = KS <= 4;                // mean-centred operands (B <= 8)
    constexpr int STAGE = DT * KS * 64;          // uint4 per stage
    // share range bests across workgroups only when a stage is long enough
    // (>= 4 tiles) to hide the coherent load of the shared values
    constexpr bool SHARE = DT >= 4;
    constexpr int PER_T = STAGE / 256;
    static_assert(STAGE % 256 == 0, "stage must split evenly over 256 threads");
    // the two stage buffers of fragments, separate arrays: a stage's
    // direct-to-LDS loads into one are then known not to touch the other
    __shared__ uint4 bl0[STAGE];
    __shared__ uint4 bl1[STAGE];
    __shared__ float2 dl[2][DT * kDomTile32];     // (Sd4, sqrt A) per domain
    __shared__ int64_t dla[2][DT * kDomTile32];   // exact A per domain
    __shared__ SLds sl;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    load_sset(sl, ss);
    const SConst sc = make_sconst(ss);
    const int *bpre = bt.pre + K_SEARCH * (bt.n + 1);
    const int im = find_img(bpre, bt.n, blockIdx.x);
    const ImgLvl &dsc = bt.d[im];
    const MfmaGeom geo = dsc.geo;
    const int lb = blockIdx.x - bpre[im];   // image blocks start at multiples of 8
    if (lb >= geo.nwg) return;
    const gptr<h8> afrag = as_global((const h8 *)dsc.afrag);
    const gptr<uint4> bfrag = as_global(dsc.bfrag);
    const gptr<float2> dinfo = as_global(dsc.dinfo);
    RInfo *__restrict__ ri = dsc.ri;
    const gptr<int64_t> pa = as_global(dsc.pa);
    Partial *__restrict__ part = dsc.part;
    const int range_cap = dsc.range_cap, pool_cap = dsc.pool_cap, n = dsc.B * dsc.B;
    const float tfac = tn_factor(n);
    const float cmargin = (float)(n / 2 + 4);   // centred test: n/4 centring + n/4 + 4 float margin
    int rg, cfirst, cstep, ncs, slot;
    chunk_walk(geo, lb, rg, cfirst, cstep, ncs, slot);
    // R: the length of the search list (constant ranges are coded already)
    const int R = min(*dsc.ns, range_cap), P = min(*dsc.pcount, pool_cap);
    const gptr<int32_t> sidx = as_global(dsc.sidx);
    if (rg * 16 * RQ >= R) return;  // uniform over the workgroup, before any barrier
    const int ntiles = (P + kDomTile32 - 1) / kDomTile32;
    const int q0 = (rg * 4 + wave) * RQ;
    const bool wave_on = q0 * 4 < R;
    const int hh = lane >> 5;

    // per lane: two ranges per quad, 4 q + 2 hh + u for u = 0, 1
    h8 A[RQ][KS];
    float tn[RQ][2], bn[RQ][2], an[RQ][2];
    int64_t best[RQ][2], cr[RQ][2], tb[RQ][2];  // tb: the best value tn reflects
    int bp[RQ][2], bk[RQ][2], rr[RQ][2], sr[RQ][2];
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
            cr[qi][u] = x.cr;
            tn[qi][u] = r >= 0 ? -1e30f : __builtin_nanf("");  // NaN: the row never passes
            tb[qi][u] = INT64_MAX;
            best[qi][u] = INT64_MAX;
            bp[qi][u] = INT32_MAX;
            bk[qi][u] = 0;
        }
    }
    // drain the one-time loads: vmcnt is in-order, so a wait for them inside
    // the tile loop would also wait for the stage prefetch
    __builtin_amdgcn_s_waitcnt(0);

    // per-domain moments of a stage: DT * kDomTile32 entries over the 256 threads
    constexpr int PER_D = (DT * kDomTile32 + 255) / 256;
    float2 dpre[PER_D];
    int64_t apre[PER_D];
    int t0 = 0, t1 = 0;
    // Fragments go straight from global memory to LDS (one 16-byte load per
    // lane into 1 KiB per wave, no registers); indexes are clamped to the
    // chunk's last tile, so the tiles past its end hold copies, harmless
    // under their NaN moments.
    auto gload = [&](uint4 *dst, int stg) {
        const int tbase = t0 + stg * DT;
        const size_t fend = (size_t)t1 * KS * 64 - 1;
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const size_t e = min((size_t)tbase * KS * 64 + tid + 256 * i, fend);
            __builtin_amdgcn_global_load_lds((gptr<void>)(bfrag + e),
                                             (__attribute__((address_space(3))) void *)(dst + 64 * wave + 256 * i),
                                             16, 0, 0);
        }
        // tiles past the chunk end get NaN moments: no pair on them passes
#pragma unroll
        for (int i = 0; i < PER_D; ++i) {
            const int e = tid + 256 * i;
            if (e < DT * kDomTile32) {
                const int p = tbase * kDomTile32 + e;
                dpre[i] = tbase + e / kDomTile32 < t1 ? ldg(dinfo, p) : make_float2(__builtin_nanf(""), __builtin_nanf(""));
                apre[i] = p < P ? pa[p] : 0;
            }
        }
    };
    auto swrite = [&](int buf) {
#pragma unroll
        for (int i = 0; i < PER_D; ++i) {
            const int e = tid + 256 * i;
            if (e < DT * kDomTile32) {
                dl[buf][e] = dpre[i];
                dla[buf][e] = apre[i];
            }
        }
    };
    // the tile's fragments are read up front (in groups of up to 8 K-steps),
    // so one LDS wait covers a group rather than every MFMA
    // With up to 4 K-steps a tile's fragments are read into registers one
    // tile ahead of its MFMAs (two sets alternate), so the LDS latency is
    // covered by the previous tile; longer tiles read them in groups of 8.
    constexpr bool PREF = KS <= 4;
    constexpr int KG = PREF ? KS : 8;
    auto read_tile = [&](h8 (&bf)[KG], const uint4 *Bs, int dt, int s0) {
#pragma unroll
        for (int s = 0; s < KG; ++s) {
            const uint4 u = Bs[(dt * KS + s0 + s) * 64 + lane];
            __builtin_memcpy(&bf[s], &u, sizeof(h8));
        }
    };
    auto mfma_tile = [&](f16x (&acc)[RQ], const uint4 *Bs, int dt, h8 (&bq)[KG]) {
#pragma unroll
        for (int qi = 0; qi < RQ; ++qi) acc[qi] = f16x{0.f};
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
        t1 = min(ntiles, t0 + tpc);
        const int nstage = t1 > t0 ? (t1 - t0 + DT - 1) / DT : 0;
        if (nstage > 0) {
            gload(bl0, 0);
            swrite(0);
        }
        // the direct-to-LDS loads count on vmcnt only: every wave drains its
        // own before the barrier that publishes the stage
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        // one stage on LDS buffer `buf` (a constant: each buffer is one array)
        auto stage = [&](auto bc, int stg) {
            constexpr int buf = decltype(bc)::value;
            uint4 *const Bs = buf ? bl1 : bl0;
            if (stg + 1 < nstage) gload(buf ? bl0 : bl1, stg + 1);
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
                h8 bq[2][KG];
                if constexpr (PREF) read_tile(bq[0], Bs, 0, 0);
                mfma_tile(acc[0], Bs, 0, bq[0]);
                if (PREF && DT > 1) read_tile(bq[1], Bs, 1, 0);
#pragma unroll
                for (int dt = 0; dt < DT; ++dt) {
                    const int cur = dt & 1;
                    if (dt + 1 < DT) {
                        mfma_tile(acc[cur ^ 1], Bs, dt + 1, bq[(dt + 1) & 1]);
                        // the set of tile dt is free once tile dt's MFMAs were issued
                        if (PREF && dt + 2 < DT) read_tile(bq[dt & 1], Bs, dt + 2, 0);
                    }
                    const float2 di = dl[buf][dt * kDomTile32 + (lane & 31)];
                    bool pass[RQ][2];
                    float mx[RQ][2];
                    bool any = false;
#pragma unroll
                    for (int qi = 0; qi < RQ; ++qi)
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            const f16x &a = acc[cur][qi];
                            const int o = 8 * u;
                            mx[qi][u] = max8f(a[o], a[o + 1], a[o + 2], a[o + 3], a[o + 4], a[o + 5], a[o + 6], a[o + 7]);
                            const float rhs = CEN ? fmaf(tn[qi][u], di.y, -cmargin)
                                                  : fmaf(tn[qi][u], di.y, fmaf(-bn[qi][u], di.x, -an[qi][u]));
                            // false on NaN: rows past the ranges, domains past the
                            // pool or the chunk, and ranges already at val 0
                            pass[qi][u] = mx[qi][u] > rhs;
                            any |= pass[qi][u];
                        }
                    if (__builtin_amdgcn_ballot_w64(any)) {  // rare: exact evaluation, then share the best
                        const int col = dt * kDomTile32 + (lane & 31);
                        const int p = tbase * kDomTile32 + col;
                        const int64_t sd4 = (int64_t)di.x, A = dla[buf][col];  // Sd4 < 2^24: exact in float
#pragma unroll
                        for (int qi = 0; qi < RQ; ++qi)
#pragma unroll
                            for (int u = 0; u < 2; ++u) {
                                bool imp = false;
                                if (pass[qi][u]) {
                                    if (CEN) {
                                        const int64_t er = (int64_t)sr[qi][u] - (int64_t)n * round_mean(sr[qi][u], n);
                                        const int64_t ed = sd4 - (int64_t)n * round_mean(sd4, n);
                                        imp = confirm_bx((int64_t)n * (int64_t)mx[qi][u] - er * ed, p, A, cr[qi][u], sl,
                                                         sc, best[qi][u], bp[qi][u], bk[qi][u]);
                                    } else {
                                        imp = confirm_pair((int)mx[qi][u], p, sd4, A, sr[qi][u], cr[qi][u], n, sl, sc,
                                                           best[qi][u], bp[qi][u], bk[qi][u]);
                                    }
                                }
                                if (__builtin_amdgcn_ballot_w64(imp)) {
                                    // the 32 lanes holding this range share their best: a
                                    // pair is only rejected when it cannot even tie it
                                    const int64_t gb = group_min_val<32>(best[qi][u]);
                                    if (rr[qi][u] >= 0 && gb <= tb[qi][u]) {
                                        tb[qi][u] = gb;
                                        tn[qi][u] = tn_from(gb, cr[qi][u], sc, tfac);
                                        if (SHARE && (lane & 31) == 0) gbest_push(&ri[rr[qi][u]].gbest, gb);
                                    }
                                }
                            }
                    }
                }
            }
            if (stg + 1 < nstage) swrite(buf ^ 1);
#pragma unroll
            for (int qi = 0; qi < RQ; ++qi)
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (gl[qi][u] < tb[qi][u]) {
                        tb[qi][u] = gl[qi][u];
                        tn[qi][u] = tn_shared(gl[qi][u], cr[qi][u], sc, tfac);
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
            int p = bp[qi][u], k = bk[qi][u];
            group_min<32>(v, p, k);
            if ((lane & 31) == 0 && rr[qi][u] >= 0) {
                Partial o;
                o.val = v;
                o.p = p == INT32_MAX ? -1 : p;
                o.k = k;
                part[(size_t)rr[qi][u] * geo.nslot + slot] = o;
            }
        }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_f16_prep_b(const BatchHost &b, hipStream_t st) {
    if (b.blocks[K_AFRAG] > 0) k_f16_afrag<<<b.blocks[K_AFRAG], 256, 0, st>>>(b.dev);
    if (b.blocks[K_BFRAG] > 0) k_f16_bfrag<<<b.blocks[K_BFRAG], 256, 0, st>>>(b.dev);
    return hipGetLastError();
}

template <int KS, int RQ, int DT, int WPE>
static hipError_t launch_f16_t(const BatchHost &b, hipStream_t st) {
    k_f16_search<KS, RQ, DT, WPE><<<b.blocks[K_SEARCH], 256, 0, st>>>(b.dev, b.ss);
    return hipGetLastError();
}

hipError_t launch_f16_search_b(const BatchHost &b, hipStream_t st) {
    if (b.blocks[K_SEARCH] == 0) return hipSuccess;
    const int B = b.B;
    const TileShape sh = b.shape;
#define FIC_F16(KS, RQ, DT, WPE) \
    if (sh.rq == RQ && sh.dt == DT && sh.wpe == WPE) return launch_f16_t<KS, RQ, DT, WPE>(b, st)
    if (B == 2) {
        FIC_F16(1, 1, 8, 4);
    } else if (B == 4) {
        FIC_F16(1, 1, 8, 4);
        FIC_F16(1, 2, 8, 2);
        FIC_F16(1, 1, 16, 3);
        FIC_F16(1, 2, 4, 3);
        FIC_F16(1, 1, 8, 3);
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
