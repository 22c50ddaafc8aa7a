// Deterministic two-stage reductions for 64-wide wavefronts.
//
// Stage 1 (inside the producing kernel): each block folds its per-thread
// values with a wave shuffle tree and an LDS pass in a fixed order and writes
// one partial per value with a plain store.  Stage 2 is a separate one-block
// kernel (k_finalize, blas.hip) that sums the partials in block order and runs
// the scalar logic of the solver.  The kernel boundary makes the partials
// visible; no block ever waits on, or fences against, another block, so the
// per-XCD L2 caches keep the stencil's working set.  Accumulation is FP64 and
// the summation order is fixed, so results are bit-reproducible.
#pragma once

#include "common.hpp"
#include "internal.hpp"

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

template <int N> __device__ __forceinline__ void wave_fold(double (&v)[N]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < N; k++) v[k] += __shfl_down(v[k], off, 64);
    }
}

// Block-wide fold; the total is valid in thread 0.
template <int N> __device__ __forceinline__ void block_fold(double (&v)[N], double (*sh)[kWaves]) {
    wave_fold<N>(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; k++) sh[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;  // 1, 2 or 4 waves
#pragma unroll
        for (int k = 0; k < N; k++) {
            double s = 0.0;
            for (int w = 0; w < nw; w++) s += sh[k][w];
            v[k] = s;
        }
    }
}

// Stage 1: per-block partials of one system, laid out [k][G] with G the
// system's number of blocks and blk this block's index among them.  Every
// thread of the block must call this.
template <int N>
__device__ __forceinline__ void block_partials(double (&v)[N], double *partials, int G, int blk) {
    __shared__ double sh[N][kWaves];
    block_fold<N>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; k++) partials[(size_t)k * G + blk] = v[k];
    }
}

// A batched launch covers several systems.  Concatenated: system s owns the
// logical blocks [off[s], off[s+1]).  Interleaved (all systems on one lattice,
// equal block counts): logical block L belongs to system L mod S, block L / S.
struct BatchHdr {
    int S;
    int interleave;
    int chunk;  // blocks per XCD chunk of the stencil's block remap (xcd_block)
    int off[kMaxSys + 1];
};

__device__ __forceinline__ void batch_locate(const BatchHdr &h, int L, int &s, int &lb) {
    if (h.interleave) {
        s = L % h.S;
        lb = L / h.S;
    } else {
        s = 0;
        while (s + 1 < h.S && L >= h.off[s + 1]) s++;
        lb = L - h.off[s];
    }
}

// complex helpers on the device scalar block
__device__ __forceinline__ cx<double> ld_c(const double *s, int slot) { return {s[slot], s[slot + 1]}; }
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
    double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
