// kt_sort.h -- counting sort of the ids 0 .. n-1 by a small integer key, on
// the device.  Three kernels: per-tile LDS histograms added into a global
// one (the key of every id is stored on the way), the exclusive scan of the
// global histogram, and a scatter in which each tile reserves its range of
// every bin it touches.  The scatter reads the stored keys, so every bin
// receives exactly the ids it counted and the positions stay below the list
// length.  The order within a bin is whatever the atomics give.
//
// It orders the trace kernel's dispatch (key: distance from the photon ring)
// and the adjoint's work list (key: forward step count; ids outside the list
// get SORT_SKIP).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kt_internal.h"

namespace kt {

constexpr int SORT_BLOCK = 256;
constexpr int SORT_PER_THREAD = 16;
constexpr int SORT_TILE = SORT_BLOCK * SORT_PER_THREAD;

struct SortBufs {
    int64_t n;       // ids 0 .. n-1
    uint32_t* hist;  // [SORT_BINS + 1]: zero before the count pass; after the
                     // scan, bin offsets and [SORT_BINS] = list length
    uint16_t* keys;  // [n] key of each id, SORT_SKIP if not listed
    uint32_t* out;   // [n] the listed ids in key order
};

// KeyFn: a small struct with `__device__ int operator()(int64_t id) const`
// returning a key in [0, SORT_BINS) or SORT_SKIP.
template <class KeyFn>
__global__ void __launch_bounds__(SORT_BLOCK) sort_count_kernel(const SortBufs b, const KeyFn key) {
    __shared__ uint32_t cnt[SORT_BINS];
    const int t = threadIdx.x;
    for (int k = t; k < SORT_BINS; k += SORT_BLOCK) cnt[k] = 0u;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SORT_TILE;
    for (int k = 0; k < SORT_PER_THREAD; ++k) {
        const int64_t id = base + k * SORT_BLOCK + t;
        if (id < b.n) {
            const int v = key(id);
            b.keys[id] = static_cast<uint16_t>(v);
            if (v != SORT_SKIP) atomicAdd(&cnt[v], 1u);
        }
    }
    __syncthreads();
    for (int k = t; k < SORT_BINS; k += SORT_BLOCK)
        if (cnt[k]) atomicAdd(&b.hist[k], cnt[k]);
}

// Exclusive scan of the bin counts in place (one block); the total goes to
// hist[SORT_BINS].
template <int BINS>
__global__ void __launch_bounds__(SORT_BLOCK) sort_scan_kernel(uint32_t* h) {
    constexpr int PER = BINS / SORT_BLOCK;
    static_assert(BINS % SORT_BLOCK == 0, "bins must split evenly over the block");
    __shared__ uint32_t part[SORT_BLOCK];
    const int t = threadIdx.x;
    uint32_t v[PER], sum = 0;
    for (int k = 0; k < PER; ++k) {
        v[k] = h[t * PER + k];
        sum += v[k];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < SORT_BLOCK; off <<= 1) {
        const uint32_t add = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int k = 0; k < PER; ++k) {
        h[t * PER + k] = run;
        run += v[k];
    }
    if (t == SORT_BLOCK - 1) h[BINS] = run;
}

template <int BINS>
__global__ void __launch_bounds__(SORT_BLOCK) sort_scatter_kernel(const SortBufs b) {
    __shared__ uint32_t cnt[BINS];
    const int t = threadIdx.x;
    for (int k = t; k < BINS; k += SORT_BLOCK) cnt[k] = 0u;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SORT_TILE;
    int bin[SORT_PER_THREAD];
    uint32_t rank[SORT_PER_THREAD];
    for (int k = 0; k < SORT_PER_THREAD; ++k) {
        const int64_t id = base + k * SORT_BLOCK + t;
        bin[k] = -1;
        rank[k] = 0u;
        if (id < b.n && b.keys[id] != SORT_SKIP) {
            bin[k] = b.keys[id];
            rank[k] = atomicAdd(&cnt[bin[k]], 1u);
        }
    }
    __syncthreads();
    for (int k = t; k < BINS; k += SORT_BLOCK)
        if (cnt[k]) cnt[k] = atomicAdd(&b.hist[k], cnt[k]);
    __syncthreads();
    const uint32_t n_list = b.hist[BINS];
    for (int k = 0; k < SORT_PER_THREAD; ++k)
        if (bin[k] >= 0) {
            const uint32_t pos = cnt[bin[k]] + rank[k];
            if (pos < n_list) b.out[pos] = static_cast<uint32_t>(base + k * SORT_BLOCK + t);
        }
}

// The three passes on `stream`; b.hist must be zero.  Returns 0 or -1 (a
// launch failed).
template <class KeyFn>
inline int launch_sort(const SortBufs& b, const KeyFn& key, hipStream_t stream) {
    const int tiles = static_cast<int>((b.n + SORT_TILE - 1) / SORT_TILE);
    hipLaunchKernelGGL(sort_count_kernel<KeyFn>, dim3(tiles), dim3(SORT_BLOCK), 0, stream, b, key);
    if (hipGetLastError() != hipSuccess) return -1;
    hipLaunchKernelGGL(sort_scan_kernel<SORT_BINS>, dim3(1), dim3(SORT_BLOCK), 0, stream, b.hist);
    if (hipGetLastError() != hipSuccess) return -1;
    hipLaunchKernelGGL(sort_scatter_kernel<SORT_BINS>, dim3(tiles), dim3(SORT_BLOCK), 0, stream, b);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace kt
