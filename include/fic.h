/*
 * fic.h -- C ABI of the MI355X (gfx950) fractal image encoder.
 *
 * The method (Salarian & Miar Naimi, "Modified Fast Fractal Image
 * Compression Algorithm in spatial domain"): an N x N gray image is cut into
 * B x B range blocks; each range is matched against a pool of 2B x 2B domain
 * blocks taken at integer step L, decimated 2 x 2 and seen under 8
 * rotations/mirrors (Sec. 2); the pool keeps only high-entropy domains
 * (Sec. 3, Eq 5-6); the contrast s is drawn from a predefined set instead of
 * Eq 2 (Sec. 2, Sec. 3.2) and the stored offset is the range mean (Sec. 3.3);
 * a range whose error misses the level threshold splits into four and the
 * search repeats one quadtree level down (Sec. 2, Fig 1).
 *
 * Conventions for every entry point:
 *  - Image, pool, range and code buffers are DEVICE pointers owned by the
 *    caller; the library never frees them.  Scalars marked "device" are
 *    single int32 values in device memory, so consecutive levels chain on the
 *    stream without a host round trip.
 *  - stream is a hipStream_t (NULL = the legacy default stream).  All work is
 *    enqueued on it; no call waits for the device unless stated.
 *  - A fic_ctx owns scratch memory and is bound to one device and one stream
 *    at a time; it is not thread safe.
 *  - Every call returns an int status (FIC_OK or a negative FIC_E_*) and
 *    validates all sizes on the host before it enqueues anything; on error
 *    nothing is written.  fic_strerror() names a status.
 *  - Coordinates are packed xy = (y << 16) | x of a block's top-left pixel.
 *  - Level order (BFS): level 0 lists every B x B range in raster order;
 *    level l+1 lists the quarters of every range level l split, in parent
 *    order, each as top-left, top-right, bottom-left, bottom-right.
 *
 * Exact arithmetic (no floating point decides any output):
 *  n = B^2; r = range pixels; D4 = 2x2 sums of the domain; s = num/den;
 *  A  = n*sum(D4^2) - (sum D4)^2,    Cr = n*sum(r^2) - (sum r)^2,
 *  Bx = n*sum(r * T_t(D4)) - sum(r)*sum(D4),
 *  val = num^2*A - 8*num*den*Bx + 16*den^2*Cr  (= 16 den^2 n E, Eq 1 with
 *  the Eq 3 offset).  The search returns the lexicographically lowest
 *  (domain, isometry, s index) of minimal val.
 */
#ifndef FIC_H
#define FIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FIC_OK = 0,
    FIC_E_INVALID = -1,   /* bad argument (see fic_validate_params) */
    FIC_E_NOMEM = -2,     /* scratch allocation failed or exceeds the ctx limit, or a
                             launch would need 2^31 or more workgroups */
    FIC_E_HIP = -3,       /* a HIP runtime call failed (no device, launch error) */
    FIC_E_CAPACITY = -4,  /* a caller buffer is smaller than the worst case */
    FIC_E_ARCH = -5,      /* the device is not gfx950 */
    FIC_E_LIMIT = -6      /* the input exceeds the fixed scratch of an
                             allocation-free entry point */
};

/* Search engines; all give identical codes.
 *   MFMA:     matrix cores, the faster form per block size: MFMA_F16 at
 *             B = 2 and 4, MFMA_F16_16X16 at B = 8, MFMA_I8 at B = 16
 *             and 32.
 *   FP32:     plain vector FP32 with the same exact epilogue (baseline).
 *   MFMA_I8:  int8 matrix cores for B = 4, 8, 16, 32 (raw pixels at B = 4,
 *             decimated hi/lo planes above); FP32 at B = 2.
 *   MFMA_F16: f16 matrix cores with exact f32 accumulation over the B^2
 *             decimated positions for B = 2 (zero-padded to 16), 4, 8, 16;
 *             FP32 at B = 32 (32 x 32 result tiles).
 *   MFMA_F16_16X16: f16 matrix cores in the 16 x 16 result tiles of the
 *             int8 engine for B = 2..16; at B = 2 and 4 the prune threshold
 *             rides in the same contraction; FP32 at B = 32. */
enum {
    FIC_ENGINE_MFMA = 0,
    FIC_ENGINE_FP32 = 1,
    FIC_ENGINE_MFMA_I8 = 2,
    FIC_ENGINE_MFMA_F16 = 3,
    FIC_ENGINE_MFMA_F16_16X16 = 4
};
enum { FIC_MAX_LEVELS = 4, FIC_MAX_S = 32 };
/* Pool keys.  Entropy (Sec. 3, Eq 5-6): G = sum over gray levels of
 * T[count], larger G = lower entropy.  Variance (the alternative the paper
 * cites in Sec. 1, low-variance domains deleted): 2^47 - (M sum p^2 -
 * (sum p)^2) over the M = 4B^2 raw pixels, larger key = lower variance.  Both
 * go through the same rule: drop the largest keys, cap to the smallest. */
enum { FIC_POOL_ENTROPY = 0, FIC_POOL_VARIANCE = 1 };

typedef struct fic_ctx fic_ctx;
typedef void *fic_stream;            /* hipStream_t */

typedef struct { int32_t num, den; } fic_ratio;

/* An 8-bit gray image in device memory, row pitch in bytes. */
typedef struct { const uint8_t *pix; int32_t width, height, pitch; } fic_image;

/* Encoder parameters (Sec. 2-3).  Level l uses B_l = block0 >> l. */
typedef struct {
    int32_t levels;                  /* 1..4 quadtree steps (2-bit step field, Sec. 3.3) */
    int32_t block0;                  /* B at level 0, power of two, B_last >= 2, block0 <= 32 */
    int32_t step[FIC_MAX_LEVELS];    /* domain step L per level, >= 1 (Sec. 2) */
    fic_ratio pool_pct;              /* drop the ceil(p*Nd) lowest-entropy candidates, 0 <= p < 1 */
    int32_t pool_max;                /* 0 = no cap; else keep at most DN highest-entropy (Sec. 3.2.1) */
    int32_t s_count[FIC_MAX_LEVELS]; /* contrast set per level: s_k = s_num[l][k] / s_den[l] */
    int32_t s_den[FIC_MAX_LEVELS];   /* 1..1024 */
    int32_t s_num[FIC_MAX_LEVELS][FIC_MAX_S]; /* strictly ascending, 0 <= num <= den */
    fic_ratio split_rms[FIC_MAX_LEVELS]; /* split iff RMS error > num/den; den 1..16; unused at the last level */
    int32_t engine;                  /* FIC_ENGINE_MFMA (default), _FP32, _MFMA_I8, _MFMA_F16, _MFMA_F16_16X16 */
    int32_t pool_key;                /* FIC_POOL_ENTROPY (default, Sec. 3) or FIC_POOL_VARIANCE */
} fic_params;

/* Domain pool of one level (Sec. 3.3: the domain address is the list index).
 * Entries are in raster order of xy.  key = integer entropy key G (larger =
 * lower entropy), sum4 = sum of the 4B^2 raw pixels, a = A above. */
typedef struct {
    int32_t capacity;                /* entries the arrays can hold */
    int32_t *count;                  /* device: entries written */
    uint32_t *xy;
    int64_t *key;
    uint32_t *sum4;
    int64_t *a;
} fic_pool;

/* Codes of one level, one entry per range of that level (BFS order).
 * err = val_q = 16 den^2 n E_q, the error with the stored 8-bit offset. */
typedef struct {
    int32_t capacity;
    int32_t *count;                  /* device: ranges of this level */
    uint32_t *xy;                    /* range top-left */
    uint8_t *split;                  /* 1 = split into four at the next level */
    uint32_t *domain;                /* index into the level's pool */
    uint8_t *iso;                    /* t = 4m + r: r clockwise quarter turns, then mirror if m */
    uint8_t *s_idx;                  /* index into the level's contrast set */
    uint8_t *offset;                 /* round-half-up of the range mean (Sec. 3.3) */
    int64_t *err;
} fic_level_codes;

/* ---- context ---------------------------------------------------------- */

/* Binds device `device`; fails with FIC_E_ARCH unless it is gfx950 and with
 * FIC_E_HIP when no device is present. */
int fic_ctx_create(fic_ctx **ctx, int device);
void fic_ctx_destroy(fic_ctx *ctx);
/* Caps the scratch the ctx may hold (bytes, 0 = unlimited); a call that
 * needs more fails with FIC_E_NOMEM before enqueuing anything. */
int fic_ctx_set_scratch_limit(fic_ctx *ctx, int64_t bytes);
const char *fic_strerror(int status);

/* Graph replay of fic_encode (launch-bound small images, repeated batches).
 * With max_graphs > 0, an encode is captured into a HIP graph the first time
 * its exact arguments (image pointers and sizes, params, every pool and code
 * buffer) are seen and replayed on later calls with the same arguments: no
 * host planning, no table upload, one graph launch on the caller's stream.
 * Image contents may change between replays.  At most max_graphs graphs are
 * kept (least recently used first out); each holds its own device copy of
 * the level tables.  All graphs are dropped when the context reallocates
 * its scratch, and encodes run eagerly while stage timing is on.  0 turns
 * replay off and frees the graphs.  Graphs contain kernel nodes only. */
int fic_ctx_set_graphs(fic_ctx *ctx, int32_t max_graphs);

/* Number of graphs currently cached by the context. */
int fic_ctx_graph_count(fic_ctx *ctx);

/* Stage timing with HIP events recorded on the caller's stream around each
 * stage a call enqueues (measurement aid; off by default).  Stages: pool build,
 * search operand preparation (range moments and operand layouts), the search
 * kernel, the per-range finalisation (argmin merge, isometry, split, child
 * list), and one decoder iteration.  Slots are indexed by log2(B). */
enum { FIC_T_POOL = 0, FIC_T_PREP = 1, FIC_T_SEARCH = 2, FIC_T_FINAL = 3, FIC_T_DECODE = 4, FIC_T_KINDS = 5 };
typedef struct {
    double ms[FIC_T_KINDS][6];       /* summed event time per stage and log2(B) */
    int32_t launches[FIC_T_KINDS][6];
} fic_timing;
/* enable != 0 starts recording (discarding earlier records); 0 stops. */
int fic_ctx_set_timing(fic_ctx *ctx, int enable);
/* Waits for the recorded events, writes their sums to *out and clears them. */
int fic_ctx_read_timing(fic_ctx *ctx, fic_timing *out);

/* Tile shapes of the matrix search kernels.  Each matrix form has, per block
 * size B, a list of compiled shapes (operand form, range quads per wave,
 * domain tiles per LDS stage, waves per SIMD the register allocation aims
 * at); candidate 0 is the measured default.  A context keeps one choice per
 * (form, log2 B) that every later plan of that context uses; all shapes give
 * identical codes.  Forms: the 16-row kernel in int8 (MFMA_I8), the 16-row
 * kernel in f16 (MFMA_F16_16X16), the 32x32 f16 kernel (MFMA_F16).  The
 * FIC_MFMA_SHAPE / FIC_F16_SHAPE environment overrides take precedence. */
enum { FIC_FORM_I8 = 0, FIC_FORM_F16_16X16 = 1, FIC_FORM_F16 = 2, FIC_FORMS = 3 };
typedef struct {
    int32_t choice[FIC_FORMS][6];    /* candidate per form and log2(B); -1 = the default */
} fic_tuning;

/* Number of compiled shapes for (form, B); 0 when the form has none. */
int fic_shape_count(int32_t form, int32_t B);
/* out[4] = (operand form, range quads per wave, tiles per stage, waves per
 * SIMD) of candidate index; FIC_E_INVALID when it does not exist.  The
 * operand form is 1 raw int8, 2 int8 hi/lo planes, 3 f16, 4 f16 with the
 * fused threshold, 0 for the 32x32 f16 kernel. */
int fic_shape_describe(int32_t form, int32_t B, int32_t index, int32_t *out);
/* The context's current choices (all -1 after fic_ctx_create). */
int fic_ctx_get_tuning(fic_ctx *ctx, fic_tuning *out);
/* Replaces the context's choices; every entry must be -1 or an existing
 * candidate (FIC_E_INVALID otherwise, nothing changed).  Drops cached graphs. */
int fic_ctx_set_tuning(fic_ctx *ctx, const fic_tuning *in);
/* Autotuner: for every level of p searched by a matrix form, times each
 * compiled shape of that (form, B) on these images and keeps the fastest in
 * the context (entries of other forms and sizes keep their values); *out,
 * if not null, receives the resulting choices.  Per candidate: one warm-up
 * encode, then reps (1..100) encodes with stage timing, scored by the summed
 * operand preparation, search and finalisation time of that level; a
 * candidate displaces the best so far (candidate 0 first) only when at
 * least 3 % faster.  The
 * buffers are those of fic_encode and end up holding an ordinary encode.
 * Blocks the host until done; stage timing must be off (FIC_E_INVALID);
 * drops cached graphs.  Errors of the encodes are returned as they are. */
int fic_autotune(fic_ctx *ctx, const fic_image *imgs, int32_t n_images, const fic_params *p, fic_pool *pools,
                 fic_level_codes *codes, int32_t reps, fic_stream stream, fic_tuning *out);

/* ---- host-only helpers (no device needed) ----------------------------- */

/* FIC_OK if params are usable for a width x height image:
 * levels in 1..4; block0 a power of two <= 32 with block0 >> (levels-1) >= 2;
 * width, height multiples of block0 and >= 2*block0, both <= 65535;
 * step >= 1; 0 <= pool_pct < 1 with den >= 1; pool_max >= 0;
 * per level 1 <= s_count <= 32, 1 <= s_den <= 1024, nums strictly ascending
 * in [0, s_den]; split_rms num >= 0, den in 1..16; engine known. */
int fic_validate_params(const fic_params *p, int32_t width, int32_t height);

/* Worst-case pool entries and ranges per level (candidates, and all ranges
 * split) for a width x height image; arrays of FIC_MAX_LEVELS entries. */
int fic_query_capacity(const fic_params *p, int32_t width, int32_t height,
                       int64_t *pool_cap, int64_t *range_cap);

/* The engine that runs the search of a level with block size B when engine
 * is requested: FIC_ENGINE_MFMA resolves to MFMA_F16, MFMA_F16_16X16,
 * MFMA_I8 or FP32 per B,
 * and the matrix engines fall back to FP32 where they have no form.
 * Returns FIC_E_INVALID for an unknown engine or B outside 2..32. */
int fic_level_engine(int32_t engine, int32_t B);

/* Copies the first n (<= 4097) entries of the entropy key table
 * T[q] = q * sum over prime powers p^e || q of e * round(ln p * 2^32), so the
 * key of a block is G = sum over gray levels of T[count]. */
int fic_entropy_table(int64_t *out, int32_t n);

/* ---- encoder and decoder ---------------------------------------------- */

/* Sec. 3, Eq 5-6 and Sec. 3.2.1: the domain pool for range size B at step L.
 * Candidates are all 2B x 2B blocks at multiples of L, raster order.  With
 * c = ceil(pct*Nd) > 0, the c-th largest key is the threshold t and the pool
 * keeps keys < t (entropy, or variance, strictly greater); if none, it keeps
 * the keys equal to the minimum.  pool_max > 0 then keeps the pool_max
 * smallest (key, index) pairs.  pool_key: FIC_POOL_ENTROPY or
 * FIC_POOL_VARIANCE.  out->capacity must be >= the pool size bound. */
int fic_build_domain_pool(fic_ctx *ctx, const fic_image *img, int32_t B, int32_t L,
                          fic_ratio pct, int32_t pool_max, int32_t pool_key, fic_pool *out, fic_stream stream);

/* One quadtree step (Sec. 2): searches the *n_ranges (device) ranges
 * ranges_xy against every pool domain, 8 isometries and s_count contrasts,
 * writes one code per range to out (out->xy copies ranges_xy), and appends the
 * four children of every split range to children_xy with their number in
 * *n_children (device).  Split iff !is_last and RMS(E_q) > split_rms.
 * range_capacity bounds *n_ranges; out->capacity >= range_capacity;
 * children_xy may be NULL when is_last, else it holds 4*range_capacity. */
int fic_encode_level(fic_ctx *ctx, const fic_image *img, const fic_pool *pool,
                     const uint32_t *ranges_xy, const int32_t *n_ranges, int32_t range_capacity,
                     int32_t B, const int32_t *s_num, int32_t s_count, int32_t s_den,
                     fic_ratio split_rms, int32_t is_last, int32_t engine,
                     fic_level_codes *out, uint32_t *children_xy, int32_t *n_children,
                     fic_stream stream);

/* Sec. 2, Fig 1 (the quadtree steps), applied to every image of a batch:
 * level 0 searches every B x B range of each image against that image's
 * level-0 pool (Sec. 3, Eq 5-6); each later level searches the quarters of
 * the ranges the previous level split, with B halved and its own pool, step
 * and contrast set; the last level accepts every range.  Images are
 * independent: a batch gives the same codes as encoding each image alone.
 * imgs: n_images device images (n_images >= 0; 0 is a no-op).  pools and
 * codes are caller arrays of n_images*levels entries, image-major
 * (entry i*levels + l is image i, level l), each with device buffers of at
 * least the fic_query_capacity sizes for that image (FIC_E_CAPACITY
 * otherwise, nothing enqueued); codes[i*levels+l].xy and .count receive
 * level l's ranges.  Every image is validated against p first
 * (FIC_E_INVALID).  Scratch comes from the context (FIC_E_NOMEM when it
 * cannot grow).  With graph replay on (fic_ctx_set_graphs) a repeat of the
 * exact arguments replays the captured encode. */
int fic_encode(fic_ctx *ctx, const fic_image *imgs, int32_t n_images, const fic_params *p,
               fic_pool *pools, fic_level_codes *codes, fic_stream stream);

/* Decoder (Sec. 1-2): X0 = every accepted range filled with its offset; each
 * iteration rebuilds every accepted range from the previous image,
 * pixel = clamp(O + floor(s*(T_t(D4)/4 - mean(D4)/4) + 1/2), 0, 255).
 * pools/codes as written by fic_encode for one image; out is width x height,
 * pitch width (device). */
int fic_decode(fic_ctx *ctx, const fic_params *p, const fic_pool *pools, const fic_level_codes *codes,
               int32_t width, int32_t height, int32_t iterations, uint8_t *out, fic_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fic_decode
 * with the same arguments, results and kernels, but its second image buffer
 * is a fixed array in the library's device memory instead of context
 * scratch, so the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine) and records no stage timing.
 * width * height must be <= FIC_DECODE_NOALLOC_MAX_PIXELS (16 MiB of pixels,
 * e.g. 4096 x 4096), else FIC_E_LIMIT and nothing is enqueued; other
 * argument errors as fic_decode.  Each GPU holds one such array for the
 * life of the process (reserved when the library's code is loaded on it,
 * its address taken by fic_ctx_create on that device), shared by every
 * context and call on that GPU: calls that overlap on one GPU (two streams,
 * two threads) race on it and must be serialised by the caller.  Every
 * scratch pixel a call reads is written by that call first, so nothing
 * carries over from an earlier call. */
#define FIC_DECODE_NOALLOC_MAX_PIXELS (1 << 24)
int fic_decode_noalloc(fic_ctx *ctx, const fic_params *p, const fic_pool *pools, const fic_level_codes *codes,
                       int32_t width, int32_t height, int32_t iterations, uint8_t *out, fic_stream stream);

/* ---- contrast diagnostic (Sec. 3.2, Fig 5; Sec. 3.2.1, Fig 6) ---------- */

/* Histograms over the ranges accepted at each level of one encoded image
 * (its image, pools and codes, device buffers as written by fic_encode):
 * the least-squares contrast of the chosen match (Eq 2 with d = D4 / 4),
 * s* = 4 Bx / A, binned exactly over [0, 1) into nbins (1..4096) bins, and
 * the chosen contrast index.  out (device, int64) receives per level
 * nbins + 3 + 32 counts: [s* < 0, nbins bins, s* >= 1, A = 0 (s* undefined),
 * then one count per contrast index 0..31].  Runs on the stream. */
int fic_s_histogram(fic_ctx *ctx, const fic_image *img, const fic_params *p, const fic_pool *pools,
                    const fic_level_codes *codes, int32_t nbins, int64_t *out, fic_stream stream);

/* ---- bitstream (Sec. 3.3, Fig 7, Eq 8) -------------------------------- */

/* Stream layout, all fields most significant bit first, zero-padded to a
 * whole byte:
 *   header   W (16), H (16), levels-1 (2), log2 block0 (3); per level:
 *            L-1 (8), |S|-1 (5), den-1 (10), each num (11)
 *   pools    per level: DN (32), mode (1); mode 0: bitmap over the Nd
 *            candidates in raster order; mode 1: the DN candidate indices in
 *            ascending order, ceil(log2 Nd) bits each (used only when
 *            strictly shorter than the bitmap).  The pool list is the
 *            decoder's address table (the domain field indexes it).
 *   records  per accepted range (Fig 7): step (2) = its level, O (8),
 *            isometry (3), domain (ceil(log2 DN), Eq 8), s index
 *            (ceil(log2 |S|): none for one value, 1 bit for two).  Order:
 *            level-0 blocks in raster order, each split block's quarters
 *            top-left, top-right, bottom-left, bottom-right, depth first;
 *            range positions are implied and not stored.
 * Requires every step L <= 256. */

/* Upper bound of the packed size in bytes (a multiple of 4). */
int fic_pack_capacity(const fic_params *p, int32_t width, int32_t height, int64_t *bytes);

/* Packs one encoded image (its per-level pools and codes, device buffers as
 * written by fic_encode) into out (device, 4-byte aligned, capacity bytes
 * from fic_pack_capacity).  sizes (device, 4 x int64) receives the bits of
 * the header, the pool side information, the records and the total; the
 * stream is ceil(total / 8) bytes.  Everything runs on the stream. */
int fic_pack(fic_ctx *ctx, const fic_params *p, int32_t width, int32_t height, const fic_pool *pools,
             const fic_level_codes *codes, uint8_t *out, int64_t capacity, int64_t *sizes, fic_stream stream);

/* Host-only.  Reads the header of a packed stream (host memory): params
 * (levels, block0, steps, contrast sets; pool_pct 0, pool_max 0, split_rms
 * 0/1, engine MFMA) and the image size.  FIC_E_INVALID on a malformed
 * header. */
int fic_unpack_header(const uint8_t *data, int64_t nbytes, fic_params *p, int32_t *width, int32_t *height);

/* Host-only.  Unpacks a stream into host buffers (capacities as
 * fic_query_capacity for the header's params): per level the pool list
 * (xy; key, sum4 and a are zeroed) and the codes in the encoder's
 * breadth-first order with split flags (err is 0: the stream does not
 * carry it).  The result decodes with fic_decode once copied to the device.
 * FIC_E_INVALID on a malformed or truncated stream. */
int fic_unpack(const uint8_t *data, int64_t nbytes, fic_pool *pools, fic_level_codes *codes);

#ifdef __cplusplus
}
#endif

#endif /* FIC_H */
