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
// where best is the smallest val found so far by any lane holding the range
// (a pair is rejected only when it cannot even tie that value),
// bn = (128n - Sr)/n, an = 512 Sr - 65536 n + margin.  When c < 0 every pair
// passes (tn = -1e30).  The margin (n/4 + 4) exceeds the float rounding of the
// test (< n/16), so no pair that could win is ever rejected.  Passing pairs
// are evaluated exactly in int64.
#pragma once

#include "fic_internal.h"

namespace fic {

// Class types (uint4, float2) cannot be copied out of another address
// space; they are read as the plain vectors they hold.
typedef uint32_t gv4u __attribute__((ext_vector_type(4)));
typedef float gv2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint4 ldg(gptr<uint4> p, size_t i) {
    const gv4u v = ((gptr<gv4u>)p)[i];
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ldg(gptr<float2> p, size_t i) {
    const gv2f v = ((gptr<gv2f>)p)[i];
    return make_float2(v.x, v.y);
}

// Values every lane holds alike, moved to scalar registers: a buffer
// resource built from them then lives in scalar registers, as the buffer
// instructions require (else the compiler loops over the lanes' values).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <class T>
__device__ __forceinline__ T *uniform(T *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

// Raw buffer resource over `bytes` bytes at p (p and bytes alike in every
// lane): unit stride, the gfx9 data-format word.
template <class T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const T *p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)uniform(p), 0, bytes, 0x00020000);
}

__device__ inline bool lex_less_vp(int64_t va, int pa, int64_t vb, int pb) {
    return va < vb || (va == vb && pa < pb);
}

// Written as three 3-input maxima and one 2-input one (v_max3_i32 x3, v_max_i32).
__device__ __forceinline__ int max8(int a0, int a1, int a2, int a3, int b0, int b1, int b2, int b3) {
    const int m1 = max(max(a0, a1), a2), m2 = max(max(a3, b0), b1), m3 = max(b2, b3);
    return max(max(m1, m2), m3);
}

// NaN-propagating 3-input maximum (one v_maximum3_f32).
#define FIC_MAX3(x, y, z) __builtin_elementwise_maximum(__builtin_elementwise_maximum(x, y), z)

// Maximum of 8 floats as four v_maximum3_f32.  The NaN-propagating maximum
// needs no input canonicalisation (fmaxf would add one v_max per input in IEEE
// mode); the inputs here are finite integers, where both agree.
__device__ __forceinline__ float max8f(float a0, float a1, float a2, float a3, float b0, float b1, float b2,
                                       float b3) {
#define FIC_MAX2(x, y) __builtin_elementwise_maximum(x, y)
    const float m1 = FIC_MAX2(FIC_MAX2(a0, a1), a2), m2 = FIC_MAX2(FIC_MAX2(a3, b0), b1);
    return FIC_MAX2(FIC_MAX2(m1, m2), FIC_MAX2(b2, b3));
#undef FIC_MAX2
}

// The maximum of 8 floats and a ninth (the spare input of the 2-input step
// above): still four v_maximum3_f32.
__device__ __forceinline__ float max9f(float a0, float a1, float a2, float a3, float b0, float b1, float b2,
                                       float b3, float c) {
    const float m1 = FIC_MAX3(a0, a1, a2), m2 = FIC_MAX3(a3, b0, b1);
    return FIC_MAX3(m1, m2, FIC_MAX3(b2, b3, c));
}

__device__ inline float sqrt_down(double v) {
    const double s = sqrt(v);
    float f = (float)s;
    if ((double)f > s) f = __int_as_float(__float_as_int(f) - 1);
    return f;
}

// Contrast numerators in LDS, so lanes may index them independently, and
// the line through the first and last of them (num_j ~ num_0 + j d), from
// which the exact search below takes its starting index.
struct SLds {
    int32_t num[kMaxS];
    float g_c0, g_inv;   // 2 num_0 + d and 1 / (2 d) (0 for a single value)
};

__device__ inline void load_sset(SLds &dst, const SSet &ss) {
    if (threadIdx.x < kMaxS) dst.num[threadIdx.x] = ss.num[threadIdx.x];
    if (threadIdx.x == 0) {
        const int c = ss.count;   // numerators strictly ascending: d > 0 when c > 1
        const float d = c > 1 ? (float)(ss.num[c - 1] - ss.num[0]) / (float)(c - 1) : 0.f;
        dst.g_c0 = 2.f * (float)ss.num[0] + d;
        dst.g_inv = c > 1 ? 0.5f / d : 0.f;
    }
}

// Uniform constants of the contrast set, built once per workgroup from the
// kernel argument (scalar registers), so the tile loop reloads nothing.
struct SConst {
    int count;
    int64_t den, scale;   // scale = 16 den^2 (<= 2^24, exact in float)
    float inv_scale;      // 1 / scale, correctly rounded
};

__device__ inline SConst make_sconst(const SSet &ss) {
    SConst c;
    c.count = ss.count;
    c.den = ss.den;
    c.scale = 16 * c.den * c.den;
    c.inv_scale = 1.0f / (float)c.scale;
    return c;
}

// Exact evaluation of one (range, domain) pair, all in integers: from
// Bx = n X4 - Sr Sd4, A and Cr (confirm_bx), or from C'max and the moments
// Sd4, A, Sr, Cr (confirm_pair).  Updates the lane's running best with a
// strict comparison (along a lane the domain index only grows, so equal
// values keep the earlier domain) and returns whether it improved.
__device__ __forceinline__ bool confirm_bx(int64_t bx, int p, int64_t A, int64_t cr, const SLds &ss,
                                           const SConst &sc, int64_t &best, int &bp, int &bk) {
    const int64_t den = sc.den;
    const int64_t lhs = 8 * den * bx;
    // midpoint rule: s_{j+1} beats s_j iff 8 den Bx > A (num_j + num_{j+1}); the
    // predicate is monotone (true, then false) in j, so k* = the first false j.
    // Start where the line through the end numerators puts q = 8 den Bx / A
    // (num_j + num_{j+1} ~ 2 num_0 + (2j + 1) d), then step to k* with the
    // exact predicate: the walk ends at k* from any start, and for an evenly
    // spaced set the start is k* or next to it, so the three table reads
    // below are usually all there is (no dependent chain of reads).  A = 0
    // gives an infinite or NaN q, which the clamp turns into an end index.
    const int last = sc.count - 1;
    const float lf = fmaf((float)(int32_t)(lhs >> 32), 4294967296.0f, (float)(uint32_t)lhs);
    const float af = fmaf((float)(int32_t)(A >> 32), 4294967296.0f, (float)(uint32_t)A);
    const float t = (lf * __builtin_amdgcn_rcpf(af) - ss.g_c0) * ss.g_inv;
    int k = (int)ceilf(fminf(fmaxf(t, 0.f), (float)last));   // fmaxf drops NaN
    int64_t nb = ss.num[max(k - 1, 0)], nk = ss.num[k], na = ss.num[min(k + 1, last)];
    while (k > 0 && !(lhs > A * (nb + nk))) {   // s_{k-1} is not beaten by s_k
        --k;
        na = nk;
        nk = nb;
        nb = ss.num[max(k - 1, 0)];
    }
    while (k < last && lhs > A * (nk + na)) {   // s_{k+1} beats s_k
        ++k;
        nk = na;
        na = ss.num[min(k + 1, last)];
    }
    const int64_t val = nk * nk * A - 8 * nk * den * bx + sc.scale * cr;
    if (val < best) {
        best = val;
        bp = p;
        bk = k;
        return true;
    }
    return false;
}

__device__ __forceinline__ bool confirm_pair(int cmax, int p, int64_t sd4, int64_t A, int64_t sr, int64_t cr, int n,
                                             const SLds &ss, const SConst &sc, int64_t &best, int &bp, int &bk) {
    const int64_t x4 = (int64_t)cmax + 128 * sd4 + 512 * sr - 65536 * (int64_t)n;
    return confirm_bx((int64_t)n * x4 - sr * sd4, p, A, cr, ss, sc, best, bp, bk);
}

// Rounded block mean round(s/n) (half up): the centre of the operands of the
// fused-threshold form.
__device__ inline int round_mean(int64_t s, int n) { return (int)((2 * s + n) / (2 * n)); }

__device__ inline uint32_t pack_h2(_Float16 lo, _Float16 hi) {
    return (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
}

// (1 - 2^-20) / n, the final factor of the prune threshold below.
__device__ inline float tn_factor(int n) { return (1.0f - 1.0f / 1048576.0f) / (float)n; }

// Prune threshold tn = sqrt(Cr - best/(16 den^2)) / n, rounded down.  The
// numerator 0 <= num < 2^60 goes to float from its 32-bit halves (two
// conversions and one fma, each rounding by at most 2^-24 relative, and the
// high half times 2^32 is at most num since the low half is non-negative);
// the product with 1/(16 den^2) and that reciprocal round by 2^-24 each, the
// hardware square root (v_sqrt_f32) is within 1 ulp (2^-23) and halves the
// relative error of its input, and the final product and the factor round
// by 2^-24 each: together below 7 * 2^-24, which the 1 - 2^-20 in the factor
// covers.  No best yet (or c < 0): every pair passes.  A pair is rejected
// only when it cannot even tie best, so best may come from any pair of the
// range, found by this workgroup or another.
__device__ __forceinline__ float tn_shared(int64_t best, int64_t cr, const SConst &sc, float factor) {
    if (best == INT64_MAX) return -1e30f;
    const int64_t num = sc.scale * cr - best;
    if (num < 0) return -1e30f;
    const float f = fmaf((float)(int32_t)(num >> 32), 4294967296.0f, (float)(uint32_t)num);
    return __builtin_amdgcn_sqrtf(f * sc.inv_scale) * factor;
}

// Threshold from the best of this workgroup's own walk.  A best of 0 cannot
// be beaten (val >= 0) and the walk's later domains have larger indices, so
// they lose ties: NaN makes every later comparison false.  This matters for
// flat ranges, where every pair ties at 0 and would pass a non-strict test.
__device__ __forceinline__ float tn_from(int64_t best, int64_t cr, const SConst &sc, float factor) {
    if (best == 0) return __builtin_nanf("");
    return tn_shared(best, cr, sc, factor);
}

// The best of every workgroup searching a range, kept as an atomic minimum.
// (global address space: a flat access would make every later wait drain
// both counters)
__device__ __forceinline__ int64_t gbest_load(const int64_t *p) {
    return __hip_atomic_load((gptr<int64_t>)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gbest_push(int64_t *p, int64_t v) {
    __hip_atomic_fetch_min((__attribute__((address_space(1))) int64_t *)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

template <int WIDTH>
__device__ inline int64_t group_min_val(int64_t v) {
#pragma unroll
    for (int off = WIDTH / 2; off > 0; off >>= 1) v = min(v, (int64_t)__shfl_xor(v, off, 64));
    return v;
}

// v of another lane of the same 16-lane row by a DPP row permutation (a lane
// whose source is inactive keeps its own value)
template <int CTRL>
__device__ __forceinline__ int64_t dpp64(int64_t v) {
    const int lo = (int)(uint32_t)v, hi = (int)(v >> 32);
    const uint32_t l = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    const uint32_t h = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
    return (int64_t)(((uint64_t)h << 32) | l);
}

// The minimum over aligned groups of 16 or 32 lanes, in every lane of the
// group, without the LDS crossbar: quad swaps, the mirrors within 8 and 16
// lanes, and for 32 the exchange of rows 0 and 1 (2 and 3).  For a wave whose
// lanes are all active.
template <int WIDTH>
__device__ inline int64_t group_min_val_wave(int64_t v) {
    static_assert(WIDTH == 16 || WIDTH == 32, "16- or 32-lane groups");
    v = min(v, dpp64<0xB1>(v));    // quad_perm [1, 0, 3, 2]: lane ^ 1
    v = min(v, dpp64<0x4E>(v));    // quad_perm [2, 3, 0, 1]: lane ^ 2
    v = min(v, dpp64<0x141>(v));   // row_half_mirror: 7 - i within 8
    v = min(v, dpp64<0x140>(v));   // row_mirror: 15 - i within 16
    if constexpr (WIDTH == 32) {
        // both results of the swap: row r and row r ^ 1 at the same lane
        const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        v = min((int64_t)(((uint64_t)h[0] << 32) | l[0]), (int64_t)(((uint64_t)h[1] << 32) | l[1]));
    }
    return v;
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
