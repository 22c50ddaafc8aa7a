// Deterministic single-pass grid reduction for 64-wide wavefronts.
//
// Each block folds its per-thread values with a wave shuffle tree and an LDS
// pass in a fixed order, publishes one partial per value, and takes a ticket.
// The block that draws the last ticket sums all partials in block order (a
// fixed strided split over its threads, then the same fixed tree), so the
// result does not depend on block scheduling.  Accumulation is in FP64.
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
#pragma unroll
        for (int k = 0; k < N; k++) {
            double s = 0.0;
            for (int w = 0; w < kWaves; w++) s += sh[k][w];
            v[k] = s;
        }
    }
}

// Returns true in thread 0 of the last block, after the grid totals have been
// written to t.result[0..N).  `tot` then holds the totals in that thread.
// Every thread of every block must call this (no early returns before it).
template <int N>
__device__ __forceinline__ bool grid_reduce(double (&v)[N], const RedTarget &t, double (&tot)[N]) {
    __shared__ double sh[N][kWaves];
    __shared__ int last;
    block_fold<N>(v, sh);
    const int G = gridDim.x;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; k++)
            __hip_atomic_store(t.partials + (size_t)k * G + blockIdx.x, v[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        unsigned prev = __hip_atomic_fetch_add(t.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == (unsigned)G - 1u);
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double a[N];
#pragma unroll
    for (int k = 0; k < N; k++) a[k] = 0.0;
    for (int j = threadIdx.x; j < G; j += blockDim.x) {
#pragma unroll
        for (int k = 0; k < N; k++)
            a[k] += __hip_atomic_load(t.partials + (size_t)k * G + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();  // sh is reused
    block_fold<N>(a, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; k++) {
            tot[k] = a[k];
            t.result[k] = a[k];
        }
        __hip_atomic_store(t.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    return false;
}

// complex helpers on the device scalar block
__device__ __forceinline__ cx<double> ld_c(const double *s, int slot) { return {s[slot], s[slot + 1]}; }
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
    double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
