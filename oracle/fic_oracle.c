/*
 * Fractal image encoder ORACLE -- test infrastructure only.
 *
 * Only the tests, the package's smoke() check and the benchmark's CPU
 * baseline may load this library.  It is a plain, slow, exact-integer
 * statement of what the encoder computes (single-threaded unless a caller
 * splits its independent candidate keys or ranges over threads), written from the
 * paper (Salarian & Miar Naimi, "Modified Fast Fractal Image Compression
 * Algorithm in spatial domain").  It shares no code, header, table or
 * generator with the GPU library.
 *
 * Readings of the paper that this file fixes (the paper leaves them open):
 *  - decimation: a 2B x 2B domain becomes B x B cells, each the sum D4 of a
 *    2 x 2 pixel group; the decimated pixel is D4/4 (Sec. 2).
 *  - isometry t = 4m + r: r clockwise quarter turns, then a left-right
 *    mirror when m = 1 (Sec. 2: rotations by 90/180/270 degrees and the
 *    mirrored copies of all four).
 *  - entropy: natural log over the 256 gray levels of the raw 2B x 2B
 *    domain (Sec. 3, Eq 5-6), ranked through the integer key G described in
 *    gen_entropy_table.py (larger G = lower entropy).
 *  - pool: candidates in raster order of their top-left corner (Sec. 3.3
 *    keeps domain coordinates in a list and uses the list index as the
 *    address); the ceil(p*Nd) lowest-entropy candidates define a threshold
 *    and only blocks with entropy strictly above it are kept (Abstract,
 *    Sec. 3); an empty result keeps the blocks of maximal entropy; an
 *    optional cap DN keeps the DN highest-entropy ones (Sec. 3.2.1), ties
 *    to the lower list index.
 *  - search: contrast s from a predefined set instead of Eq 2 (Sec. 2-3.2);
 *    distance Eq 1 with the offset of Eq 3, which equals storing the range
 *    mean (Sec. 3.3); exhaustive over (domain, isometry, s) with the
 *    lexicographically lowest index winning ties.
 *  - stored offset O = round-half-up of the range mean (8 bits, Sec. 3.3);
 *    split when the RMS error with that O exceeds the level's threshold and
 *    the level is not the last (Sec. 2, quadtree steps, Fig 1).
 *  - decoder: start from the piecewise-constant image of the offsets and
 *    apply all range maps synchronously; each pixel is O plus s times the
 *    centred decimated domain pixel, rounded half up, clamped to 0..255.
 *
 * Integer scaling used throughout (n = B^2 range pixels, s = num/den):
 *   val = num^2*A - 8*num*den*Bx + 16*den^2*Cr = 16*den^2*n*E(s)
 * with A = n*sum(D4^2) - (sum D4)^2, Bx = n*sum(r*D4') - sum(r)*sum(D4),
 * Cr = n*sum(r^2) - sum(r)^2, D4' the isometry-permuted cells, and E(s)
 * Eq 1 with the Eq 3 offset.  For den <= 1024 and B <= 32 every |term| is
 * below 1.2e18, so int64 holds val exactly.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const int64_t ENT_T[4097] = {
#include "entropy_table.inc"
};

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

int orc_entropy_table(int64_t *out, int n)
{
    if (n < 0 || n > 4097) return ORC_EINVAL;
    memcpy(out, ENT_T, sizeof(int64_t) * (size_t)n);
    return ORC_OK;
}

/* Sec. 3, Eq 5-6: entropy key of the size x size block at (x, y). */
int64_t orc_entropy_key(const uint8_t *img, int pitch, int x, int y, int size)
{
    int hist[256];
    memset(hist, 0, sizeof(hist));
    for (int dy = 0; dy < size; ++dy)
        for (int dx = 0; dx < size; ++dx)
            hist[img[(size_t)(y + dy) * pitch + x + dx]] += 1;
    int64_t g = 0;
    for (int v = 0; v < 256; ++v) g += ENT_T[hist[v]];
    return g;
}

/* Variance pool (the alternative the paper cites in Sec. 1: domains of
 * small variance are deleted): key = 2^47 - (M sum p^2 - (sum p)^2) over the
 * M raw pixels of the block, so a smaller key means a larger variance and
 * the entropy pool's drop-the-largest-keys rule applies unchanged.
 * M sum p^2 - (sum p)^2 = M^2 var <= 4096^2 * 255^2 / 4 < 2^47. */
int64_t orc_variance_key(const uint8_t *img, int pitch, int x, int y, int size)
{
    int64_t s = 0, ss = 0;
    for (int dy = 0; dy < size; ++dy)
        for (int dx = 0; dx < size; ++dx) {
            const int64_t v = img[(size_t)(y + dy) * pitch + x + dx];
            s += v;
            ss += v * v;
        }
    const int64_t m = (int64_t)size * size;
    return ((int64_t)1 << 47) - (m * ss - s * s);
}

/* Sec. 2: all 2B x 2B blocks at integer step L, raster order. */
int orc_candidates(int W, int H, int B, int L, uint32_t *xy, int cap)
{
    if (B < 1 || L < 1 || 2 * B > W || 2 * B > H) return ORC_EINVAL;
    int nx = (W - 2 * B) / L + 1, ny = (H - 2 * B) / L + 1;
    if (xy) {
        if (cap < nx * ny) return ORC_EINVAL;
        int i = 0;
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix)
                xy[i++] = ((uint32_t)(iy * L) << 16) | (uint32_t)(ix * L);
    }
    return nx * ny;
}

static int cmp_i64_desc(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x < y) - (x > y);
}

typedef struct { int64_t g; int32_t idx; } key_idx;

static int cmp_key_idx(const void *a, const void *b)
{
    const key_idx *x = (const key_idx *)a, *y = (const key_idx *)b;
    if (x->g != y->g) return (x->g > y->g) - (x->g < y->g);
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* The decimated domain: cell (j, i) = sum of the 2x2 pixels at (x+2i, y+2j). */
static void decimate(const uint8_t *img, int pitch, int x, int y, int B, int32_t *d4)
{
    for (int j = 0; j < B; ++j)
        for (int i = 0; i < B; ++i) {
            const uint8_t *p = img + (size_t)(y + 2 * j) * pitch + x + 2 * i;
            d4[j * B + i] = p[0] + p[1] + p[pitch] + p[pitch + 1];
        }
}

/* Keys of candidates [lo, hi): independent per candidate, so the range may be
 * split over threads without changing any value. */
typedef struct {
    const uint8_t *img;
    int pitch, size, kind, lo, hi;
    const uint32_t *cxy;
    int64_t *g;
} key_job;

static void *key_range(void *arg)
{
    key_job *j = (key_job *)arg;
    for (int i = j->lo; i < j->hi; ++i) {
        int x = (int)(j->cxy[i] & 0xffff), y = (int)(j->cxy[i] >> 16);
        j->g[i] = j->kind == 0 ? orc_entropy_key(j->img, j->pitch, x, y, j->size)
                               : orc_variance_key(j->img, j->pitch, x, y, j->size);
    }
    return NULL;
}

/*
 * Domain pool for range size B (domains 2B x 2B) at step L.
 * drop fraction p = p_num/p_den of the candidates (lowest entropy first,
 * rank by nearest rank ceil(p*Nd)); pool_max > 0 caps the pool size.
 * Writes xy, key G, sum4 = sum of the raw pixels, a = n*sum(D4^2) - sum4^2.
 * threads (1..64): the candidate keys are computed by that many threads.
 * Returns the pool size, or a negative status.
 */
int orc_build_pool(const uint8_t *img, int W, int H, int pitch, int B, int L,
                   int p_num, int p_den, int pool_max, int key_kind,
                   uint32_t *xy, int64_t *key, uint32_t *sum4, int64_t *a, int cap, int threads)
{
    if (p_den < 1 || p_num < 0 || p_num >= p_den || pool_max < 0 || key_kind < 0 || key_kind > 1 ||
        threads < 1 || threads > 64)
        return ORC_EINVAL;
    int nd = orc_candidates(W, H, B, L, NULL, 0);
    if (nd < 0) return nd;
    uint32_t *cxy = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nd);
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)nd);
    int64_t *sorted = (int64_t *)malloc(sizeof(int64_t) * (size_t)nd);
    char *keep = (char *)calloc((size_t)nd, 1);
    key_idx *ki = (key_idx *)malloc(sizeof(key_idx) * (size_t)nd);
    int32_t *d4 = (int32_t *)malloc(sizeof(int32_t) * (size_t)B * B);
    if (!cxy || !g || !sorted || !keep || !ki || !d4) {
        free(cxy); free(g); free(sorted); free(keep); free(ki); free(d4);
        return ORC_ENOMEM;
    }
    orc_candidates(W, H, B, L, cxy, nd);
    key_job jobs[64];
    pthread_t tid[64];
    int started[64] = {0};
    for (int t = 0; t < threads; ++t) {
        jobs[t] = (key_job){img, pitch, 2 * B, key_kind, (int)((int64_t)nd * t / threads),
                            (int)((int64_t)nd * (t + 1) / threads), cxy, g};
        if (t + 1 < threads) started[t] = pthread_create(&tid[t], NULL, key_range, &jobs[t]) == 0;
        if (!started[t]) key_range(&jobs[t]);   /* the last part, or a thread that could not start */
    }
    for (int t = 0; t + 1 < threads; ++t)
        if (started[t]) pthread_join(tid[t], NULL);
    int64_t gmin = INT64_MAX;
    for (int i = 0; i < nd; ++i)
        if (g[i] < gmin) gmin = g[i];
    /* c = ceil(p * Nd) lowest-entropy candidates (largest G) set the threshold */
    int64_t c = ((int64_t)p_num * nd + p_den - 1) / p_den;
    int count = 0;
    if (c == 0) {
        for (int i = 0; i < nd; ++i) keep[i] = 1;
        count = nd;
    } else {
        memcpy(sorted, g, sizeof(int64_t) * (size_t)nd);
        qsort(sorted, (size_t)nd, sizeof(int64_t), cmp_i64_desc);
        int64_t t = sorted[c - 1];
        for (int i = 0; i < nd; ++i)
            if (g[i] < t) { keep[i] = 1; ++count; }
        if (count == 0)
            for (int i = 0; i < nd; ++i)
                if (g[i] == gmin) { keep[i] = 1; ++count; }
    }
    if (pool_max > 0 && count > pool_max) {
        int m = 0;
        for (int i = 0; i < nd; ++i)
            if (keep[i]) { ki[m].g = g[i]; ki[m].idx = i; ++m; }
        qsort(ki, (size_t)m, sizeof(key_idx), cmp_key_idx);
        memset(keep, 0, (size_t)nd);
        for (int j = 0; j < pool_max; ++j) keep[ki[j].idx] = 1;
        count = pool_max;
    }
    int status = count;
    if (xy) {
        if (cap < count) {
            status = ORC_EINVAL;
        } else {
            int n = B * B, o = 0;
            for (int i = 0; i < nd; ++i) {
                if (!keep[i]) continue;
                int x = (int)(cxy[i] & 0xffff), y = (int)(cxy[i] >> 16);
                decimate(img, pitch, x, y, B, d4);
                int64_t s = 0, ss = 0;
                for (int j = 0; j < n; ++j) { s += d4[j]; ss += (int64_t)d4[j] * d4[j]; }
                xy[o] = cxy[i];
                if (key) key[o] = g[i];
                if (sum4) sum4[o] = (uint32_t)s;
                if (a) a[o] = (int64_t)n * ss - s * s;
                ++o;
            }
        }
    }
    free(cxy); free(g); free(sorted); free(keep); free(ki); free(d4);
    return status;
}

/*
 * Isometry t = 4m + r of a B x B block: out[y][x] = in[*sy][*sx].
 * r clockwise quarter turns, then a left-right mirror when m = 1.
 */
void orc_iso_source(int t, int B, int y, int x, int *sy, int *sx)
{
    int r = t & 3, m = t >> 2;
    if (m) x = B - 1 - x;          /* mirror acts last, so undo it first */
    int yy = y, xx = x;
    for (int q = 0; q < r; ++q) {  /* one clockwise turn: out[y][x] = in[B-1-x][y] */
        int ny = B - 1 - xx, nx = yy;
        yy = ny; xx = nx;
    }
    *sy = yy; *sx = xx;
}

/* Shared, read-only state of one quadtree step, and the slice of ranges
 * [lo, hi) one thread searches (ranges are independent of each other). */
typedef struct {
    const uint8_t *img;
    int pitch, P, B, S, tn, td, is_last, lo, hi, status;
    const int32_t *dec, *perm, *s_num;
    const int64_t *dsum, *da;
    int64_t den;
    const uint32_t *ranges_xy;
    uint8_t *split, *iso, *s_idx, *offset;
    uint32_t *domain;
    int64_t *err;
} level_job;

static void *search_ranges(void *arg)
{
    level_job *j = (level_job *)arg;
    const int B = j->B, n = B * B, P = j->P, S = j->S, pitch = j->pitch;
    const int64_t den = j->den;
    int32_t *r = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!r) { j->status = ORC_ENOMEM; return NULL; }
    for (int ri = j->lo; ri < j->hi; ++ri) {
        int rx = (int)(j->ranges_xy[ri] & 0xffff), ry = (int)(j->ranges_xy[ri] >> 16);
        int64_t sr = 0, srr = 0;
        for (int y = 0; y < B; ++y)
            for (int x = 0; x < B; ++x) {
                int v = j->img[(size_t)(ry + y) * pitch + rx + x];
                r[y * B + x] = v;
                sr += v;
                srr += (int64_t)v * v;
            }
        int64_t cr = (int64_t)n * srr - sr * sr;
        int64_t o = (2 * sr + n) / (2 * n);
        int64_t best = INT64_MAX;
        int bp = 0, bt = 0, bk = 0;
        for (int p = 0; p < P; ++p) {
            const int32_t *d = j->dec + (size_t)p * n;
            for (int t = 0; t < 8; ++t) {
                const int32_t *pm = j->perm + t * n;
                int64_t x4 = 0;
                for (int i = 0; i < n; ++i) x4 += (int64_t)r[i] * d[pm[i]];
                int64_t bx = (int64_t)n * x4 - sr * j->dsum[p];
                for (int k = 0; k < S; ++k) {
                    int64_t num = j->s_num[k];
                    int64_t val = num * num * j->da[p] - 8 * num * den * bx + 16 * den * den * cr;
                    if (val < best) { best = val; bp = p; bt = t; bk = k; }
                }
            }
        }
        int64_t dq = (int64_t)n * o - sr;
        int64_t valq = best + 16 * den * den * dq * dq;
        int sp = 0;
        if (!j->is_last) {
            __int128 lhs = (__int128)valq * j->td * j->td;
            __int128 rhs = (__int128)16 * den * den * n * n * j->tn * j->tn;
            sp = lhs > rhs;
        }
        j->split[ri] = (uint8_t)sp;
        j->domain[ri] = (uint32_t)bp;
        j->iso[ri] = (uint8_t)bt;
        j->s_idx[ri] = (uint8_t)bk;
        j->offset[ri] = (uint8_t)o;
        j->err[ri] = valq;
    }
    free(r);
    return NULL;
}

/*
 * One quadtree step: search every range of ranges_xy (B x B, top-left xy)
 * against every pool domain (2B x 2B at pool_xy), all 8 isometries and all
 * s = s_num[k]/s_den.  Outputs per range: best domain index, isometry,
 * s index, stored offset O, val_q = 16*den^2*n*E_q (error with the stored
 * O) and the split flag.  Split iff !is_last and RMS(E_q) > tn/td.
 * threads (1..64): the ranges are split over that many threads, which share
 * the decimated pool.
 */
int orc_encode_level(const uint8_t *img, int W, int H, int pitch,
                     const uint32_t *pool_xy, int P,
                     const uint32_t *ranges_xy, int R, int B,
                     const int32_t *s_num, int S, int s_den,
                     int tn, int td, int is_last,
                     uint8_t *split, uint32_t *domain, uint8_t *iso, uint8_t *s_idx,
                     uint8_t *offset, int64_t *err, int threads)
{
    if (B < 1 || B > 32 || P < 1 || R < 0 || S < 1 || S > 32 || s_den < 1 || s_den > 1024 ||
        td < 1 || tn < 0 || threads < 1 || threads > 64)
        return ORC_EINVAL;
    for (int k = 0; k < S; ++k)
        if (s_num[k] < 0 || s_num[k] > s_den || (k > 0 && s_num[k] <= s_num[k - 1])) return ORC_EINVAL;
    (void)W; (void)H;
    const int n = B * B;
    int32_t *dec = (int32_t *)malloc(sizeof(int32_t) * (size_t)P * n);
    int64_t *dsum = (int64_t *)malloc(sizeof(int64_t) * (size_t)P);
    int64_t *da = (int64_t *)malloc(sizeof(int64_t) * (size_t)P);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * 8 * (size_t)n);
    if (!dec || !dsum || !da || !perm) {
        free(dec); free(dsum); free(da); free(perm);
        return ORC_ENOMEM;
    }
    for (int p = 0; p < P; ++p) {
        int32_t *d = dec + (size_t)p * n;
        decimate(img, pitch, (int)(pool_xy[p] & 0xffff), (int)(pool_xy[p] >> 16), B, d);
        int64_t s = 0, ss = 0;
        for (int j = 0; j < n; ++j) { s += d[j]; ss += (int64_t)d[j] * d[j]; }
        dsum[p] = s;
        da[p] = (int64_t)n * ss - s * s;
    }
    for (int t = 0; t < 8; ++t)
        for (int y = 0; y < B; ++y)
            for (int x = 0; x < B; ++x) {
                int sy, sx;
                orc_iso_source(t, B, y, x, &sy, &sx);
                perm[t * n + y * B + x] = sy * B + sx;
            }
    if (threads > R) threads = R > 0 ? R : 1;
    level_job jobs[64];
    pthread_t tid[64];
    int started[64] = {0};
    for (int t = 0; t < threads; ++t) {
        jobs[t] = (level_job){img, pitch, P, B, S, tn, td, is_last, (int)((int64_t)R * t / threads),
                              (int)((int64_t)R * (t + 1) / threads), ORC_OK, dec, perm, s_num, dsum, da,
                              (int64_t)s_den, ranges_xy, split, iso, s_idx, offset, domain, err};
        if (t + 1 < threads) started[t] = pthread_create(&tid[t], NULL, search_ranges, &jobs[t]) == 0;
        if (!started[t]) search_ranges(&jobs[t]);
    }
    int status = ORC_OK;
    for (int t = 0; t < threads; ++t) {
        if (t + 1 < threads && started[t]) pthread_join(tid[t], NULL);
        if (jobs[t].status != ORC_OK) status = jobs[t].status;
    }
    free(dec); free(dsum); free(da); free(perm);
    return status;
}

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}

/*
 * Decoder.  Leaves are the accepted ranges of every level: top-left
 * (lx, ly), size lb, domain top-left (dx, dy) in the image, isometry, s =
 * num/den and stored offset.  X0 = every leaf filled with its offset; each
 * iteration rebuilds every leaf from the previous image.  Writes X_iters.
 * A non-NULL init replaces X0 (used to check that decoding has no memory).
 */
int orc_decode(int W, int H, int nleaf,
               const int32_t *lx, const int32_t *ly, const int32_t *lb,
               const int32_t *dx, const int32_t *dy, const int32_t *liso,
               const int32_t *lnum, const int32_t *lden, const int32_t *loff,
               int iters, const uint8_t *init, uint8_t *out)
{
    if (W < 1 || H < 1 || nleaf < 0 || iters < 0) return ORC_EINVAL;
    uint8_t *cur = (uint8_t *)malloc((size_t)W * H);
    uint8_t *nxt = (uint8_t *)malloc((size_t)W * H);
    int32_t *d4 = (int32_t *)malloc(sizeof(int32_t) * 32 * 32);
    if (!cur || !nxt || !d4) { free(cur); free(nxt); free(d4); return ORC_ENOMEM; }
    memset(cur, 0, (size_t)W * H);
    if (init) {
        memcpy(cur, init, (size_t)W * H);
    } else {
        for (int l = 0; l < nleaf; ++l)
            for (int y = 0; y < lb[l]; ++y)
                for (int x = 0; x < lb[l]; ++x)
                    cur[(size_t)(ly[l] + y) * W + lx[l] + x] = (uint8_t)loff[l];
    }
    for (int it = 0; it < iters; ++it) {
        memcpy(nxt, cur, (size_t)W * H);
        for (int l = 0; l < nleaf; ++l) {
            int B = lb[l];
            int64_t n = (int64_t)B * B;
            decimate(cur, W, dx[l], dy[l], B, d4);
            int64_t s4 = 0;
            for (int j = 0; j < B * B; ++j) s4 += d4[j];
            int64_t q = 4 * n * lden[l];
            for (int y = 0; y < B; ++y)
                for (int x = 0; x < B; ++x) {
                    int sy, sx;
                    orc_iso_source(liso[l], B, y, x, &sy, &sx);
                    int64_t num = (int64_t)lnum[l] * (n * d4[sy * B + sx] - s4);
                    int64_t v = loff[l] + floor_div(2 * num + q, 2 * q);
                    if (v < 0) v = 0;
                    if (v > 255) v = 255;
                    nxt[(size_t)(ly[l] + y) * W + lx[l] + x] = (uint8_t)v;
                }
        }
        uint8_t *tmp = cur; cur = nxt; nxt = tmp;
    }
    memcpy(out, cur, (size_t)W * H);
    free(cur); free(nxt); free(d4);
    return ORC_OK;
}
