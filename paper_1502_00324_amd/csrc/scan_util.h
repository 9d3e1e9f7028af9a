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

// ---- stable compaction: items [0, n) in kScanBlock chunks, 4 consecutive per thread
template <class Pred>
__global__ __launch_bounds__(256) void k_flag_count(int n_cap, const int32_t *n_dev, Pred pred, int *blocksum) {
    const int n = n_dev ? min(*n_dev, n_cap) : n_cap;
    const int base = blockIdx.x * kScanBlock + threadIdx.x * 4;
    int c = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (base + j < n && pred(base + j)) ++c;
    c = block_sum_256(c);
    if (threadIdx.x == 0) blocksum[blockIdx.x] = c;
}

// One 1024-thread block: exclusive offsets of nb block counts, total * mult to
// *total_out (written also when nb == 0).
hipError_t launch_scan_blocks(int nb, const int *blocksum, int *blockoff, int32_t *total_out, int mult,
                              hipStream_t st);

template <class Pred, class Emit>
__global__ __launch_bounds__(256) void k_flag_scatter(int n_cap, const int32_t *n_dev, Pred pred, const int *blockoff,
                                                      Emit emit) {
    const int n = n_dev ? min(*n_dev, n_cap) : n_cap;
    const int base = blockIdx.x * kScanBlock + threadIdx.x * 4;
    bool f[4];
    int c = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f[j] = base + j < n && pred(base + j);
        c += f[j] ? 1 : 0;
    }
    int total;
    int pos = blockoff[blockIdx.x] + block_excl_scan_256(c, &total);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (f[j]) emit(base + j, pos++);
}

template <class Pred, class Emit>
hipError_t compact(int n_cap, const int32_t *n_dev, Pred pred, Emit emit, int *blocksum, int *blockoff,
                   int32_t *total_out, int mult, hipStream_t st) {
    const int nb = (n_cap + kScanBlock - 1) / kScanBlock;
    if (nb > 0) k_flag_count<Pred><<<nb, 256, 0, st>>>(n_cap, n_dev, pred, blocksum);
    hipError_t e = launch_scan_blocks(nb, blocksum, blockoff, total_out, mult, st);
    if (e != hipSuccess) return e;
    if (nb > 0) k_flag_scatter<Pred, Emit><<<nb, 256, 0, st>>>(n_cap, n_dev, pred, blockoff, emit);
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
