// Integral images of every image of a batch (summed-area tables), computed
// once per encode and shared by all levels, so block moments cost O(1):
//   SI[y][x]  = sum of I over [0, y) x [0, x)          ((H+1) x (W+1))
//   SII[y][x] = the same for I^2
//   SQ_q      = four parity classes q = 2 py + px of Q^2, where
//               Q(x, y) = I[y][x] + I[y][x+1] + I[y+1][x] + I[y+1][x+1] is the
//               2x2 sum (D4 of Sec. 3.1 at that corner), gathered on the grid
//               x = 2i + px, y = 2j + py and prefix-summed over (j, i)
//               ((H/2+1) x (W/2+1) each; cells outside the image count 0).
// A domain at (x, y) has Sd4 = box of SI over 2B x 2B and sum D4^2 = box of
// SQ_{2(y&1)+(x&1)} over B x B at (x>>1, y>>1); a range has Sr, Srr from SI
// and SII.  All tables are uint32 and wrap mod 2^32: every box the encoder
// reads (at most 4096 pixels, sums below 1.1e9) fits, so the wrapped
// differences are exact.
//
// Row pass: one wave per table row scans along x.  Column pass: the rows are
// cut into chunks of kChunkRows; chunk sums, a scan of the chunk sums per
// column, then each chunk adds its offset while scanning down.
#include "fic_internal.h"

namespace fic {

constexpr int kChunkRows = 64;

__device__ inline uint32_t wave_incl_scan_u32(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// Row y of SI/SII (y = 0: zero rows of every table); pixel row y-1 also
// feeds Q row y-1 (zero when it has no row below it).
__global__ __launch_bounds__(256) void k_integ_rows(BatchDev b) {
    const int *pre = b.pre + K_IROW * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int y = (blockIdx.x - pre[im]) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const IntegGeom g = integ_geom(d.W, d.H);
    if (y > g.H) return;
    uint32_t *si = g.si(d.integ), *sii = g.sii(d.integ);
    if (y == 0) {
        for (int x = lane; x < g.ws; x += 64) si[x] = sii[x] = 0u;
        for (int q = 0; q < 4; ++q) {
            uint32_t *s = g.sq(d.integ, q);
            for (int i = lane; i < g.wq; i += 64) s[i] = 0u;
        }
        return;
    }
    const uint8_t *row = d.pix + (size_t)(y - 1) * d.pitch;
    uint32_t *o1 = si + (size_t)y * g.ws, *o2 = sii + (size_t)y * g.ws;
    if (lane == 0) o1[0] = o2[0] = 0u;
    uint32_t c1 = 0u, c2 = 0u;
    for (int x0 = 0; x0 < g.W; x0 += 64) {
        const int x = x0 + lane;
        const uint32_t v = x < g.W ? row[x] : 0u;
        const uint32_t p1 = wave_incl_scan_u32(v), p2 = wave_incl_scan_u32(v * v);
        if (x < g.W) {
            o1[x + 1] = c1 + p1;
            o2[x + 1] = c2 + p2;
        }
        c1 += __shfl(p1, 63, 64);
        c2 += __shfl(p2, 63, 64);
    }
    // Q row yq = y - 1: grid row j = yq / 2 of the classes with py = yq % 2
    const int yq = y - 1, py = yq & 1, j = yq >> 1;
    const bool has_q = yq <= g.H - 2;
    const uint8_t *row2 = row + d.pitch;
    for (int px = 0; px < 2; ++px) {
        uint32_t *o = g.sq(d.integ, 2 * py + px) + (size_t)(j + 1) * g.wq;
        if (lane == 0) o[0] = 0u;
        uint32_t c = 0u;
        for (int i0 = 0; i0 < g.wq - 1; i0 += 64) {
            const int i = i0 + lane, x = 2 * i + px;
            uint32_t v = 0u;
            if (has_q && i < g.wq - 1 && x <= g.W - 2) {
                const uint32_t q = (uint32_t)row[x] + row[x + 1] + row2[x] + row2[x + 1];
                v = q * q;
            }
            const uint32_t p = wave_incl_scan_u32(v);
            if (i < g.wq - 1) o[i + 1] = c + p;
            c += __shfl(p, 63, 64);
        }
    }
}

// Work item of the column pass within one image: table a, column, chunk
// (column fastest, so a wave touches consecutive addresses of one row).
__device__ inline bool col_item(const IntegGeom &g, uint32_t *base, int item, uint32_t *&p, int &rows, int &cols,
                                int &col, int &ch, int &nch) {
    for (int a = 0; a < 6; ++a) {
        g.table(base, a, p, rows, cols);
        nch = (rows + kChunkRows - 1) / kChunkRows;
        const int items = cols * nch;
        if (item < items) {
            ch = item / cols;
            col = item - ch * cols;
            return true;
        }
        item -= items;
    }
    return false;
}

// Phase 1: sum of each (table, column, chunk).
__global__ __launch_bounds__(256) void k_integ_colsum(BatchDev b) {
    const int *pre = b.pre + K_ICOL * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int item = (blockIdx.x - pre[im]) * 256 + threadIdx.x;
    const IntegGeom g = integ_geom(d.W, d.H);
    uint32_t *p;
    int rows, cols, col, ch, nch;
    if (!col_item(g, d.integ, item, p, rows, cols, col, ch, nch)) return;
    const int r1 = min(rows, (ch + 1) * kChunkRows);
    uint32_t s = 0u;
    for (int r = ch * kChunkRows; r < r1; ++r) s += p[(size_t)r * cols + col];
    d.itmp[item] = s;
}

// Phase 2: exclusive scan of the chunk sums of each (table, column).
__global__ __launch_bounds__(256) void k_integ_colscan(BatchDev b) {
    const int *pre = b.pre + K_ICSCAN * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    int item = (blockIdx.x - pre[im]) * 256 + threadIdx.x;
    const IntegGeom g = integ_geom(d.W, d.H);
    int base_item = 0;
    for (int a = 0; a < 6; ++a) {
        uint32_t *p;
        int rows, cols;
        g.table(d.integ, a, p, rows, cols);
        const int nch = (rows + kChunkRows - 1) / kChunkRows;
        if (item < cols) {
            uint32_t off = 0u;
            for (int ch = 0; ch < nch; ++ch) {
                uint32_t *t = d.itmp + base_item + ch * cols + item;
                const uint32_t s = *t;
                *t = off;
                off += s;
            }
            return;
        }
        item -= cols;
        base_item += cols * nch;
    }
}

// Phase 3: running sum down each chunk from its offset.
__global__ __launch_bounds__(256) void k_integ_coladd(BatchDev b) {
    const int *pre = b.pre + K_ICOL * (b.n + 1);
    const int im = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[im];
    const int item = (blockIdx.x - pre[im]) * 256 + threadIdx.x;
    const IntegGeom g = integ_geom(d.W, d.H);
    uint32_t *p;
    int rows, cols, col, ch, nch;
    if (!col_item(g, d.integ, item, p, rows, cols, col, ch, nch)) return;
    const int r1 = min(rows, (ch + 1) * kChunkRows);
    uint32_t s = d.itmp[item];
    for (int r = ch * kChunkRows; r < r1; ++r) {
        uint32_t *q = p + (size_t)r * cols + col;
        s += *q;
        *q = s;
    }
}

hipError_t launch_integ_b(const BatchHost &b, hipStream_t st) {
    if (b.blocks[K_IROW] == 0) return hipSuccess;
    k_integ_rows<<<b.blocks[K_IROW], 256, 0, st>>>(b.dev);
    k_integ_colsum<<<b.blocks[K_ICOL], 256, 0, st>>>(b.dev);
    k_integ_colscan<<<b.blocks[K_ICSCAN], 256, 0, st>>>(b.dev);
    k_integ_coladd<<<b.blocks[K_ICOL], 256, 0, st>>>(b.dev);
    return hipGetLastError();
}

// Host side: table and chunk-sum sizes of a W x H image.
size_t integ_words(int W, int H) {
    return 2 * (size_t)(H + 1) * (W + 1) + 4 * (size_t)(H / 2 + 1) * (W / 2 + 1);
}

int integ_col_items(int W, int H) {
    const int nc1 = (H + 1 + kChunkRows - 1) / kChunkRows, nc2 = (H / 2 + 1 + kChunkRows - 1) / kChunkRows;
    return 2 * (W + 1) * nc1 + 4 * (W / 2 + 1) * nc2;
}

int integ_scan_items(int W, int H) { return 2 * (W + 1) + 4 * (W / 2 + 1); }

}  // namespace fic
