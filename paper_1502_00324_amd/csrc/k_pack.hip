// Bitstream of one encoded image (Sec. 3.3, Fig 7, Eq 8): the GPU packer and
// the host unpacker.  The format is documented with fic_pack in fic.h.
//
// The packer needs no sort: the depth-first position of an accepted range is
// the Morton code of its top-left corner inside its level-0 block (quarters
// top-left, top-right, bottom-left, bottom-right nest as consecutive Morton
// intervals), so every range marks a slot keyed by (level-0 block, Morton
// code at the finest block size); one exclusive scan of the record lengths
// over the slots gives each record's bit offset, and every record, pool entry
// and header field is OR-ed into 32-bit words (most significant bit first),
// byte-swapped at the end so the stream reads MSB first byte by byte.
#include <string.h>

#include <vector>

#include "fic_internal.h"

namespace fic {

namespace {

constexpr int kPackBlock = 1024;   // slots per scan block

__host__ __device__ inline int ceil_log2(int64_t v) {
    int b = 0;
    while (b < 63 && ((int64_t)1 << b) < v) ++b;
    return b;
}

struct PackLevel {
    const int32_t *ccount, *pcount;
    const uint32_t *cxy, *pxy, *cdom;
    const uint8_t *csplit, *ciso, *csidx, *coff;
    int B, L, nx, sbits, last, range_cap, pool_cap, xw;   // xw = ceil(log2 Nd)
    int64_t nd;
};

struct PackArgs {
    PackLevel lv[kMaxLevels];
    int levels, block0, W, H, blast, spb, nbx;   // spb: slots per level-0 block
    int64_t nslots, nwords;
    uint32_t *words, *lens, *ref, *bsum;
    uint64_t *offs, *meta;   // meta: pool start of each level, record base, sizes
    int64_t *sizes;          // caller: header, pool, record, total bits
    // header fields known on the host
    int hdr_L[kMaxLevels], hdr_ns[kMaxLevels], hdr_den[kMaxLevels], hdr_num[kMaxLevels][kMaxS];
};

// MSB-first: stream bit pos + k holds bit (width - 1 - k) of value; width <= 32.
__device__ inline void put_bits(uint32_t *w, uint64_t pos, uint32_t value, int width) {
    if (width <= 0) return;
    const uint64_t word = pos >> 5;
    const int off = (int)(pos & 31);
    const int n1 = min(width, 32 - off);
    const uint32_t hi = width - n1 >= 32 ? 0u : value >> (width - n1);
    atomicOr(&w[word], n1 == 32 ? hi : (hi & ((1u << n1) - 1)) << (32 - off - n1));
    if (n1 < width) {
        const int n2 = width - n1;
        atomicOr(&w[word + 1], (value & ((1u << n2) - 1)) << (32 - n2));
    }
}

__device__ inline uint32_t morton2(uint32_t u, uint32_t v) {
    uint32_t m = 0;
    for (int k = 0; k < 8; ++k) m |= ((u >> k) & 1u) << (2 * k) | ((v >> k) & 1u) << (2 * k + 1);
    return m;
}

__global__ void k_pack_fill(PackArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.nwords) a.words[i] = 0u;
    if (i < a.nslots) a.lens[i] = 0u;
}

// One thread per range of level l: accepted ranges mark their slot.
__global__ void k_pack_mark(PackArgs a, int l) {
    const PackLevel &v = a.lv[l];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= min(*v.ccount, v.range_cap)) return;
    if (!v.last && v.csplit[r]) return;
    const uint32_t xy = v.cxy[r];
    const int x = xy & 0xffff, y = xy >> 16;
    const int64_t blk = (int64_t)(y / a.block0) * a.nbx + x / a.block0;
    const uint32_t m = morton2((x % a.block0) / a.blast, (y % a.block0) / a.blast);
    const int64_t s = blk * a.spb + m;
    const int dn = min(*v.pcount, v.pool_cap);
    a.lens[s] = 13u + (uint32_t)ceil_log2(dn) + (uint32_t)v.sbits;
    a.ref[s] = ((uint32_t)l << 28) | (uint32_t)r;
}

// Exclusive scan of lens over the slots: block sums, one scan of the sums,
// then each block's local scan plus its offset.
__global__ __launch_bounds__(256) void k_pack_bsum(PackArgs a) {
    __shared__ uint32_t red[256];
    const int64_t base = (int64_t)blockIdx.x * kPackBlock;
    uint32_t s = 0;
    for (int i = threadIdx.x; i < kPackBlock; i += 256)
        if (base + i < a.nslots) s += a.lens[base + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.bsum[blockIdx.x] = red[0];
}

__global__ void k_pack_btop(PackArgs a, int nblocks) {
    // one thread: nblocks <= a few thousand
    uint64_t run = 0;
    for (int b = 0; b < nblocks; ++b) {
        const uint32_t s = a.bsum[b];
        a.offs[(int64_t)b * kPackBlock] = run;   // block start, expanded below
        run += s;
    }
    a.meta[kMaxLevels + 1] = run;   // record bits
}

__global__ __launch_bounds__(256) void k_pack_bscan(PackArgs a) {
    __shared__ uint64_t part[256];
    const int64_t base = (int64_t)blockIdx.x * kPackBlock;
    const uint64_t start = a.offs[base];
    // 256 threads x 4 consecutive slots
    uint32_t v[4];
    uint64_t t = 0;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + threadIdx.x * 4 + k;
        v[k] = i < a.nslots ? a.lens[i] : 0u;
        t += v[k];
    }
    part[threadIdx.x] = t;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint64_t add = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint64_t run = start + part[threadIdx.x] - t;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + threadIdx.x * 4 + k;
        if (i < a.nslots) a.offs[i] = run;
        run += v[k];
    }
}

// One thread: header, pool section layout, sizes.
__global__ void k_pack_head(PackArgs a, int header_bits) {
    uint64_t pos = 0;
    put_bits(a.words, pos, (uint32_t)a.W, 16), pos += 16;
    put_bits(a.words, pos, (uint32_t)a.H, 16), pos += 16;
    put_bits(a.words, pos, (uint32_t)(a.levels - 1), 2), pos += 2;
    put_bits(a.words, pos, (uint32_t)ceil_log2(a.block0), 3), pos += 3;
    for (int l = 0; l < a.levels; ++l) {
        put_bits(a.words, pos, (uint32_t)(a.hdr_L[l] - 1), 8), pos += 8;
        put_bits(a.words, pos, (uint32_t)(a.hdr_ns[l] - 1), 5), pos += 5;
        put_bits(a.words, pos, (uint32_t)(a.hdr_den[l] - 1), 10), pos += 10;
        for (int k = 0; k < a.hdr_ns[l]; ++k) put_bits(a.words, pos, (uint32_t)a.hdr_num[l][k], 11), pos += 11;
    }
    const uint64_t pool0 = pos;
    for (int l = 0; l < a.levels; ++l) {
        const PackLevel &v = a.lv[l];
        const int64_t dn = min(*v.pcount, v.pool_cap);
        const bool list = dn * v.xw < v.nd;
        put_bits(a.words, pos, (uint32_t)dn, 32), pos += 32;
        put_bits(a.words, pos, list ? 1u : 0u, 1), pos += 1;
        a.meta[l] = pos | (list ? (1ull << 63) : 0ull);
        pos += list ? (uint64_t)dn * v.xw : (uint64_t)v.nd;
    }
    a.meta[kMaxLevels] = pos;   // record base
    const uint64_t rec = a.meta[kMaxLevels + 1];
    a.sizes[0] = header_bits;
    a.sizes[1] = (int64_t)(pos - pool0);
    a.sizes[2] = (int64_t)rec;
    a.sizes[3] = (int64_t)(pos + rec);
}

// Pool side information of level l, one thread per pool entry.
__global__ void k_pack_pool(PackArgs a, int l) {
    const PackLevel &v = a.lv[l];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= min(*v.pcount, v.pool_cap)) return;
    const uint32_t xy = v.pxy[p];
    const int64_t idx = (int64_t)((xy >> 16) / v.L) * v.nx + (xy & 0xffff) / v.L;
    const uint64_t m = a.meta[l];
    const uint64_t start = m & ~(1ull << 63);
    if (m >> 63) put_bits(a.words, start + (uint64_t)p * v.xw, (uint32_t)idx, v.xw);
    else put_bits(a.words, start + (uint64_t)idx, 1u, 1);
}

__global__ void k_pack_records(PackArgs a) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.nslots || a.lens[s] == 0) return;
    const uint32_t rf = a.ref[s];
    const int l = rf >> 28, r = rf & 0x0fffffff;
    const PackLevel &v = a.lv[l];
    uint64_t pos = a.meta[kMaxLevels] + a.offs[s];
    const int xb = ceil_log2(min(*v.pcount, v.pool_cap));
    put_bits(a.words, pos, (uint32_t)l, 2), pos += 2;
    put_bits(a.words, pos, v.coff[r], 8), pos += 8;
    put_bits(a.words, pos, v.ciso[r], 3), pos += 3;
    put_bits(a.words, pos, v.cdom[r], xb), pos += xb;
    put_bits(a.words, pos, v.csidx[r], v.sbits);
}

__global__ void k_pack_bswap(PackArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.nwords) a.words[i] = __builtin_bswap32(a.words[i]);
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int header_bits(const fic_params *p) {
    int bits = 16 + 16 + 2 + 3;
    for (int l = 0; l < p->levels; ++l) bits += 8 + 5 + 10 + 11 * p->s_count[l];
    return bits;
}

// ---------------------------------------------------------------- host unpacker
struct Reader {
    const uint8_t *d;
    int64_t nbits, pos = 0;
    bool bad = false;
    uint64_t get(int w) {
        uint64_t v = 0;
        for (int k = 0; k < w; ++k) {
            if (pos >= nbits) {
                bad = true;
                return 0;
            }
            v = (v << 1) | ((d[pos >> 3] >> (7 - (pos & 7))) & 1u);
            ++pos;
        }
        return v;
    }
};

int read_header(Reader &rd, fic_params *p, int32_t *W, int32_t *H) {
    memset(p, 0, sizeof(*p));
    *W = (int32_t)rd.get(16);
    *H = (int32_t)rd.get(16);
    p->levels = (int32_t)rd.get(2) + 1;
    p->block0 = 1 << rd.get(3);
    for (int l = 0; l < p->levels; ++l) {
        p->step[l] = (int32_t)rd.get(8) + 1;
        p->s_count[l] = (int32_t)rd.get(5) + 1;
        p->s_den[l] = (int32_t)rd.get(10) + 1;
        for (int k = 0; k < p->s_count[l]; ++k) p->s_num[l][k] = (int32_t)rd.get(11);
        p->split_rms[l].den = 1;
    }
    p->pool_pct.den = 1;
    p->engine = FIC_ENGINE_MFMA;
    if (rd.bad) return FIC_E_INVALID;
    return fic_validate_params(p, *W, *H);
}

}  // namespace

}  // namespace fic

using namespace fic;

extern "C" {

int fic_pack_capacity(const fic_params *p, int32_t width, int32_t height, int64_t *bytes) {
    if (!bytes) return FIC_E_INVALID;
    int st = fic_validate_params(p, width, height);
    if (st != FIC_OK) return st;
    int64_t pcap[kMaxLevels], rcap[kMaxLevels];
    fic_query_capacity(p, width, height, pcap, rcap);
    int64_t bits = header_bits(p);
    for (int l = 0; l < p->levels; ++l) {
        const int B = p->block0 >> l, L = p->step[l];
        if (L > 256) return FIC_E_INVALID;
        const int64_t nd = (int64_t)((width - 2 * B) / L + 1) * ((height - 2 * B) / L + 1);
        bits += 33 + nd + rcap[l] * (13 + ceil_log2(pcap[l]) + ceil_log2(p->s_count[l]));
    }
    *bytes = ceil_div(bits, 32) * 4;
    return FIC_OK;
}

int fic_pack(fic_ctx *ctx, const fic_params *p, int32_t width, int32_t height, const fic_pool *pools,
             const fic_level_codes *codes, uint8_t *out, int64_t capacity, int64_t *sizes, fic_stream stream) {
    if (!ctx || !pools || !codes || !out || !sizes || ((uintptr_t)out & 3)) return FIC_E_INVALID;
    int64_t need = 0;
    int st = fic_pack_capacity(p, width, height, &need);
    if (st != FIC_OK) return st;
    if (capacity < need) return FIC_E_CAPACITY;
    int64_t pcap[kMaxLevels], rcap[kMaxLevels];
    fic_query_capacity(p, width, height, pcap, rcap);
    PackArgs a;
    memset(&a, 0, sizeof(a));
    a.levels = p->levels;
    a.block0 = p->block0;
    a.W = width;
    a.H = height;
    a.blast = p->block0 >> (p->levels - 1);
    a.spb = (a.block0 / a.blast) * (a.block0 / a.blast);
    a.nbx = width / a.block0;
    a.nslots = (int64_t)a.nbx * (height / a.block0) * a.spb;
    a.nwords = capacity / 4;
    for (int l = 0; l < p->levels; ++l) {
        const fic_pool &q = pools[l];
        const fic_level_codes &c = codes[l];
        if (!q.count || !q.xy || !c.count || !c.xy || !c.split || !c.domain || !c.iso || !c.s_idx || !c.offset)
            return FIC_E_INVALID;
        if (q.capacity < pcap[l] || c.capacity < rcap[l]) return FIC_E_CAPACITY;
        PackLevel &v = a.lv[l];
        v.ccount = c.count;
        v.pcount = q.count;
        v.cxy = c.xy;
        v.pxy = q.xy;
        v.cdom = c.domain;
        v.csplit = c.split;
        v.ciso = c.iso;
        v.csidx = c.s_idx;
        v.coff = c.offset;
        v.B = p->block0 >> l;
        v.L = p->step[l];
        v.nx = (width - 2 * v.B) / v.L + 1;
        v.nd = (int64_t)v.nx * ((height - 2 * v.B) / v.L + 1);
        v.xw = ceil_log2(v.nd);
        v.sbits = ceil_log2(p->s_count[l]);
        v.last = l == p->levels - 1;
        v.range_cap = (int)rcap[l];
        v.pool_cap = (int)pcap[l];
        a.hdr_L[l] = p->step[l];
        a.hdr_ns[l] = p->s_count[l];
        a.hdr_den[l] = p->s_den[l];
        for (int k = 0; k < p->s_count[l]; ++k) a.hdr_num[l][k] = p->s_num[l][k];
    }
    st = enter(ctx);
    if (st != FIC_OK) return st;
    const int nblocks = (int)ceil_div(a.nslots, kPackBlock);
    size_t bytes[S_NUM_SLOTS] = {0};
    const size_t lens_b = (size_t)a.nslots * 4, offs_b = (size_t)a.nslots * 8, bs_b = (size_t)nblocks * 4;
    bytes[S_PACK] = lens_b * 2 + offs_b + bs_b + 8 * (kMaxLevels + 2) + 1024;
    st = reserve(ctx, bytes);
    if (st != FIC_OK) return st;
    char *base = (char *)ctx->slot[S_PACK].ptr;
    a.offs = (uint64_t *)base;
    a.meta = (uint64_t *)(base + offs_b);
    a.lens = (uint32_t *)(base + offs_b + 8 * (kMaxLevels + 2));
    a.ref = a.lens + a.nslots;
    a.bsum = a.ref + a.nslots;
    a.words = (uint32_t *)out;
    a.sizes = sizes;
    hipStream_t s = (hipStream_t)stream;
    const int64_t fill = a.nwords > a.nslots ? a.nwords : a.nslots;
    k_pack_fill<<<(unsigned)ceil_div(fill, 256), 256, 0, s>>>(a);
    for (int l = 0; l < p->levels; ++l)
        if (rcap[l] > 0) k_pack_mark<<<(unsigned)ceil_div(rcap[l], 256), 256, 0, s>>>(a, l);
    k_pack_bsum<<<nblocks, 256, 0, s>>>(a);
    k_pack_btop<<<1, 1, 0, s>>>(a, nblocks);
    k_pack_bscan<<<nblocks, 256, 0, s>>>(a);
    k_pack_head<<<1, 1, 0, s>>>(a, header_bits(p));
    for (int l = 0; l < p->levels; ++l)
        if (pcap[l] > 0) k_pack_pool<<<(unsigned)ceil_div(pcap[l], 256), 256, 0, s>>>(a, l);
    k_pack_records<<<(unsigned)ceil_div(a.nslots, 256), 256, 0, s>>>(a);
    k_pack_bswap<<<(unsigned)ceil_div(a.nwords, 256), 256, 0, s>>>(a);
    return hip_status(hipGetLastError());
}

int fic_unpack_header(const uint8_t *data, int64_t nbytes, fic_params *p, int32_t *width, int32_t *height) {
    if (!data || nbytes < 0 || !p || !width || !height) return FIC_E_INVALID;
    Reader rd{data, nbytes * 8};
    return read_header(rd, p, width, height);
}

int fic_unpack(const uint8_t *data, int64_t nbytes, fic_pool *pools, fic_level_codes *codes) {
    if (!data || nbytes < 0 || !pools || !codes) return FIC_E_INVALID;
    Reader rd{data, nbytes * 8};
    fic_params p;
    int32_t W, H;
    int st = read_header(rd, &p, &W, &H);
    if (st != FIC_OK) return st;
    int64_t pcap[kMaxLevels], rcap[kMaxLevels];
    fic_query_capacity(&p, W, H, pcap, rcap);
    const int NL = p.levels;
    int xb[kMaxLevels], sb[kMaxLevels];
    for (int l = 0; l < NL; ++l) {
        const fic_pool &q = pools[l];
        const fic_level_codes &c = codes[l];
        if (!q.count || !q.xy || !c.count || !c.xy || !c.split || !c.domain || !c.iso || !c.s_idx || !c.offset ||
            !c.err)
            return FIC_E_INVALID;
        if (q.capacity < pcap[l] || c.capacity < rcap[l]) return FIC_E_CAPACITY;
        const int B = p.block0 >> l, L = p.step[l];
        const int nx = (W - 2 * B) / L + 1;
        const int64_t nd = (int64_t)nx * ((H - 2 * B) / L + 1);
        const int64_t dn = (int64_t)rd.get(32);
        const bool list = rd.get(1) != 0;
        if (rd.bad || dn > pcap[l]) return FIC_E_INVALID;
        int64_t k = 0;
        if (list) {
            const int w = ceil_log2(nd);
            int64_t prev = -1;
            for (; k < dn; ++k) {
                const int64_t i = (int64_t)rd.get(w);
                if (i >= nd || i <= prev) return FIC_E_INVALID;   // ascending candidate indices
                prev = i;
                q.xy[k] = ((uint32_t)((i / nx) * L) << 16) | (uint32_t)((i % nx) * L);
            }
        } else {
            for (int64_t i = 0; i < nd; ++i)
                if (rd.get(1)) {
                    if (k >= dn) return FIC_E_INVALID;
                    q.xy[k++] = ((uint32_t)((i / nx) * L) << 16) | (uint32_t)((i % nx) * L);
                }
            if (k != dn) return FIC_E_INVALID;
        }
        if (q.key) memset(q.key, 0, sizeof(int64_t) * dn);
        if (q.sum4) memset(q.sum4, 0, sizeof(uint32_t) * dn);
        if (q.a) memset(q.a, 0, sizeof(int64_t) * dn);
        *q.count = (int32_t)dn;
        *c.count = 0;
        xb[l] = ceil_log2(dn);
        sb[l] = ceil_log2(p.s_count[l]);
    }
    // depth first over the quadtree; nodes of a level are met in breadth-first
    // order (parents in order, quarters in order), so appending reproduces
    // the per-level lists of the encoder
    struct Node { int l, x, y; };
    std::vector<Node> stack;
    const int nbx = W / p.block0, nby = H / p.block0;
    for (int by = 0; by < nby; ++by)
        for (int bx = 0; bx < nbx; ++bx) {
            stack.push_back({0, bx * p.block0, by * p.block0});
            while (!stack.empty()) {
                const Node nd = stack.back();
                stack.pop_back();
                const int64_t save = rd.pos;
                const int step = (int)rd.get(2);
                if (rd.bad || step < nd.l || step >= NL) return FIC_E_INVALID;
                fic_level_codes &c = codes[nd.l];
                const int r = *c.count;
                if (r >= rcap[nd.l]) return FIC_E_INVALID;
                c.xy[r] = ((uint32_t)nd.y << 16) | (uint32_t)nd.x;
                c.err[r] = 0;
                *c.count = r + 1;
                if (step > nd.l) {
                    rd.pos = save;   // the record belongs to a quarter
                    c.split[r] = 1;
                    c.domain[r] = 0;
                    c.iso[r] = 0;
                    c.s_idx[r] = 0;
                    c.offset[r] = 0;
                    const int h = (p.block0 >> nd.l) / 2;
                    stack.push_back({nd.l + 1, nd.x + h, nd.y + h});   // popped last
                    stack.push_back({nd.l + 1, nd.x, nd.y + h});
                    stack.push_back({nd.l + 1, nd.x + h, nd.y});
                    stack.push_back({nd.l + 1, nd.x, nd.y});
                    continue;
                }
                c.split[r] = 0;
                c.offset[r] = (uint8_t)rd.get(8);
                c.iso[r] = (uint8_t)rd.get(3);
                c.domain[r] = (uint32_t)rd.get(xb[nd.l]);
                c.s_idx[r] = (uint8_t)rd.get(sb[nd.l]);
                if (rd.bad || (int64_t)c.domain[r] >= *pools[nd.l].count || c.s_idx[r] >= p.s_count[nd.l])
                    return FIC_E_INVALID;
            }
        }
    return FIC_OK;
}

}  // extern "C"
