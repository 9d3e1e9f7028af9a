// Exact epilogue shared by both search engines.
//
// Both engines produce, per (range, domain, isometry), the integer cross term
//   C' = sum over the 4B^2 raw domain pixels (view - 128) * (pixel - 128)
//      = X4 - 128*Sd4 - 512*Sr + 65536*n,      X4 = sum r * T_t(D4),
// where view is the range seen through the inverse isometry, each range
// pixel covering its 2x2 domain cell.  For a fixed (range, domain) the best
// val over the contrast set is non-increasing in X4 (all s >= 0), so only the
// isometry maximum of C' matters; the isometry itself is recovered once per
// range for the winning domain.
//
// Prune test (float, conservative): for A > 0 the least val over every real s
// is 16 den^2 (Cr - Bx^2/A), so a pair can reach val <= best only if
//   Bx > sqrt(A) * sqrt(c),  c = Cr - best/(16 den^2)  (c >= 0),
// i.e.  C'max > tn*sqrtA - bn*Sd4 - an  with tn = sqrt(c)/n rounded down,
// bn = (128n - Sr)/n, an = 512 Sr - 65536 n + margin.  When c < 0 every pair
// passes (tn = -1e30).  The margin (n/4 + 4) exceeds the float rounding of the
// test (< n/16), so no pair that could win is ever rejected.  Passing pairs
// are evaluated exactly in int64.
#pragma once

#include "fic_internal.h"

namespace fic {

__device__ inline bool lex_less_vp(int64_t va, int pa, int64_t vb, int pb) {
    return va < vb || (va == vb && pa < pb);
}

__device__ __forceinline__ int max8(int a0, int a1, int a2, int a3, int b0, int b1, int b2, int b3) {
    return max(max(max(a0, a1), max(a2, a3)), max(max(b0, b1), max(b2, b3)));
}

__device__ inline float sqrt_down(double v) {
    const double s = sqrt(v);
    float f = (float)s;
    if ((double)f > s) f = __int_as_float(__float_as_int(f) - 1);
    return f;
}

// Exact evaluation of one (range, domain) pair given C'max.  Updates the
// lane's running best with a strict comparison: along a lane the domain index
// only grows, so equal values keep the earlier domain.
__device__ __forceinline__ void confirm_pair(int cmax, int p, int r, int n, const RInfo *__restrict__ ri,
                                          const uint32_t *__restrict__ sum4, const int64_t *__restrict__ pa,
                                          const SSet &ss, int64_t &best, int &bp, int &bk, float &tn) {
    const RInfo x = ri[r];
    const int64_t sd4 = sum4[p], A = pa[p];
    const int64_t sr = x.sr;
    const int64_t x4 = (int64_t)cmax + 128 * sd4 + 512 * sr - 65536 * (int64_t)n;
    const int64_t bx = (int64_t)n * x4 - sr * sd4;
    const int64_t den = ss.den;
    const int64_t lhs = 8 * den * bx;
    // midpoint rule: s_{j+1} beats s_j iff 8 den Bx > A (num_j + num_{j+1});
    // the predicate is monotone in j, so k* is the last j+1 where it holds
    int k = 0;
    int64_t nk = ss.num[0];
    for (int j = 0; j + 1 < ss.count; ++j) {
        const int64_t a = ss.num[j], b = ss.num[j + 1];
        if (lhs > A * (a + b)) {
            k = j + 1;
            nk = b;
        }
    }
    const int64_t val = nk * nk * A - 8 * nk * den * bx + 16 * den * den * x.cr;
    if (val < best) {
        best = val;
        bp = p;
        bk = k;
        const int64_t scale = 16 * den * den;
        const int64_t num = scale * x.cr - val;
        tn = num < 0 ? -1e30f : sqrt_down((double)num / (double)scale * (1.0 - 1.0 / 1048576.0)) / (float)n;
    }
}

// Merge (val, domain, k) over 16-lane groups (xor offsets < 16) or 32-lane
// groups (width 32) in lexicographic (val, domain) order.
template <int WIDTH>
__device__ inline void group_min(int64_t &v, int &p, int &k) {
#pragma unroll
    for (int off = WIDTH / 2; off > 0; off >>= 1) {
        const int64_t ov = __shfl_xor(v, off, 64);
        const int op = __shfl_xor(p, off, 64), ok = __shfl_xor(k, off, 64);
        if (lex_less_vp(ov, op, v, p)) {
            v = ov;
            p = op;
            k = ok;
        }
    }
}

}  // namespace fic
