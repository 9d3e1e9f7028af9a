// Block-wide reductions, scans and stable stream compaction for 256-thread blocks.
#pragma once

#include "fic_internal.h"

namespace fic {

__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

// Exclusive scan over a 256-thread block; *total receives the block sum.
__device__ inline int block_excl_scan_256(int v, int *total) {
    __shared__ int wsum[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = wave_incl_scan(v);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        before += (i < w) ? wsum[i] : 0;
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

__device__ inline int block_sum_256(int v) {
    int total;
    (void)block_excl_scan_256(v, &total);
    return total;
}

// ---- batched stable compaction: image i owns flattened blocks
// [pre[i], pre[i+1]) of kScanBlock items each, 4 consecutive per thread.
// Op supplies items(d), pred(d, idx), emit(d, idx, pos), sums(d), offs(d),
// total(d) and mult.
template <class Op>
__global__ __launch_bounds__(256) void k_bcount(BatchDev b, int kind, Op op) {
    const int *pre = b.pre + kind * (b.n + 1);
    const int i = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[i];
    const int lb = blockIdx.x - pre[i];
    const int n = op.items(d);
    const int base = lb * kScanBlock + threadIdx.x * 4;
    int c = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (base + j < n && op.pred(d, base + j)) ++c;
    c = block_sum_256(c);
    if (threadIdx.x == 0) op.sums(d)[lb] = c;
}

// One 1024-thread workgroup per image: exclusive block offsets, total * mult.
template <class Op>
__global__ __launch_bounds__(1024) void k_bscan(BatchDev b, int kind, Op op) {
    __shared__ int wsum[16];
    __shared__ int carry_s;
    const int *pre = b.pre + kind * (b.n + 1);
    const ImgLvl &d = b.d[blockIdx.x];
    const int nb = pre[blockIdx.x + 1] - pre[blockIdx.x];
    const int *sums = op.sums(d);
    int *offs = op.offs(d);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int v = base + t < nb ? sums[base + t] : 0;
        const int incl = wave_incl_scan(v);
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int before = 0, all = 0;
        for (int k = 0; k < 16; ++k) {
            before += k < w ? wsum[k] : 0;
            all += wsum[k];
        }
        const int carry = carry_s;
        if (base + t < nb) offs[base + t] = carry + before + incl - v;
        __syncthreads();
        if (t == 0) carry_s = carry + all;
        __syncthreads();
    }
    if (t == 0) *op.total(d) = carry_s * op.mult;
}

template <class Op>
__global__ __launch_bounds__(256) void k_bscatter(BatchDev b, int kind, Op op) {
    const int *pre = b.pre + kind * (b.n + 1);
    const int i = find_img(pre, b.n, blockIdx.x);
    const ImgLvl &d = b.d[i];
    const int lb = blockIdx.x - pre[i];
    const int n = op.items(d);
    const int base = lb * kScanBlock + threadIdx.x * 4;
    bool f[4];
    int c = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f[j] = base + j < n && op.pred(d, base + j);
        c += f[j] ? 1 : 0;
    }
    int total;
    int pos = op.offs(d)[lb] + block_excl_scan_256(c, &total);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (f[j]) op.emit(d, base + j, pos++);
}

template <class Op>
hipError_t compact_b(const BatchDev &b, int kind, int blocks, Op op, hipStream_t st) {
    if (blocks > 0) k_bcount<Op><<<blocks, 256, 0, st>>>(b, kind, op);
    k_bscan<Op><<<b.n, 1024, 0, st>>>(b, kind, op);
    if (blocks > 0) k_bscatter<Op><<<blocks, 256, 0, st>>>(b, kind, op);
    return hipGetLastError();
}

// wave-wide sums (64 lanes)
__device__ inline int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline int wave_sum_i32(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace fic
