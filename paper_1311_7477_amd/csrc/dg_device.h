// Device helpers shared by the HIP kernels of libdgark: XCD-aware tile
// order, vector loads/stores and the deterministic grid reduction.
#pragma once

#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dgk {

constexpr int kPwThreads = 256;

// Fused multiply-add written out: the library is compiled with
// -ffp-contract=off, so every rounding is the one the source states and a
// body computes bit-identical results in every kernel that inlines it.
__device__ __forceinline__ double fmx(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}
__device__ __forceinline__ float fmx(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

// Block index -> tile index such that the blocks the dispatcher sends to one
// XCD (block b goes to XCD b mod 8) get a contiguous run of tiles: halo
// reads of neighbouring tiles then hit the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
    const int xcd = b & 7, idx = b >> 3;
    const int q = nblocks >> 3, r = nblocks & 7;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <int M, class T>
__device__ __forceinline__ void load_vec(const T* __restrict__ f, long off,
                                         T (&u)[M]) {
#pragma unroll
    for (int i = 0; i < M; ++i) u[i] = f[off + i];
}

template <int M, class T>
__device__ __forceinline__ void store_vec(T* __restrict__ f, long off,
                                          const T (&u)[M]) {
#pragma unroll
    for (int i = 0; i < M; ++i) f[off + i] = u[i];
}

// ---------------------------------------------------------------------------
// Deterministic block reduction + last-block-done final sum.
//
// Partials are published with agent-scope atomic stores (coherent across
// the XCDs' L2 caches), the publishing wave waits for their completion, then
// takes a ticket with an agent-scope atomic add.  Tickets are two-level:
// block b counts in group b mod G (G = min(kTicketGroups, nblocks)), the
// block completing its group counts in the global counter, and the block
// completing that is the last one; it reads all partials with agent-scope
// atomic loads and sums them in block order, so the result does not depend
// on the order of arrival.  (One counter for all blocks made the tickets of
// blocks finishing together wait on each other: about 4 us at 256 blocks and
// 12 us at 1024 per launch; two levels take about 1.5 and 2.5 us.)  No L2
// write-back or invalidate is needed because only atomics carry data
// between blocks; results for the next kernel are ordinary stores made
// visible by the kernel boundary.
//
// The guarantee relied on: s_waitcnt with every counter at zero returns only
// after the wave's agent-scope atomic stores have been performed at the
// device's point of coherence, so they precede the ticket's atomic add there;
// a group's last block adds to the global counter only after its group add
// has returned (after every member's add), and the last block's agent-scope
// atomic loads, issued after its global add has returned, read that point.  This is the
// instruction sequence the memory model's agent-scope release / acquire
// lowering emits for atomic data on this target; the L2 write-back /
// invalidate such a release / acquire would add concerns non-atomic data,
// which this reduction never passes between blocks.
// b is the block's index among the nblocks blocks of this reduction (its
// partial slot).  Returns true in the last block, where tot[] holds the sums.
// ---------------------------------------------------------------------------
template <int NV, int NT>
__device__ bool reduce_last(double (&v)[NV], double* partials,
                            unsigned* counter, int nblocks, int b,
                            double (&tot)[NV]) {
    __shared__ double red[(NT / 64) * NV];
    __shared__ int is_last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w * NV + k];
            __hip_atomic_store(&partials[(long)b * NV + k], s,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_s_waitcnt(0);   // partials performed before the ticket
        const int G = nblocks < kTicketGroups ? nblocks : kTicketGroups;
        const int g = b % G;
        const unsigned gsize = (unsigned)((nblocks - g + G - 1) / G);
        unsigned* gc = counter + kCntLine * (1 + g);
        const unsigned t = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        int last = 0;
        if (t == gsize - 1) {
            // every member of the group has counted: reset it for the next
            // launch, then count the group
            __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned t2 = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            last = (t2 == (unsigned)(G - 1));
        }
        is_last = last;
    }
    __syncthreads();
    if (!is_last) return false;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int q = threadIdx.x; q < nblocks; q += NT)
#pragma unroll
        for (int k = 0; k < NV; ++k)
            acc[k] += __hip_atomic_load(&partials[(long)q * NV + k],
                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave * NV + k] = acc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w * NV + k];
        tot[k] = s;
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

#define DG_DISPATCH_N(n, ...) \
    switch (n) {              \
        case 1: { constexpr int NN = 1; __VA_ARGS__; } break; \
        case 2: { constexpr int NN = 2; __VA_ARGS__; } break; \
        case 3: { constexpr int NN = 3; __VA_ARGS__; } break; \
        case 4: { constexpr int NN = 4; __VA_ARGS__; } break; \
        case 5: { constexpr int NN = 5; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue; \
    }

// Dispatch on the polynomial order n (NN) and the tile height w in waves
// (WW, one of 4, 8, 16) of a cell-per-lane or row-per-lane kernel.
#define DG_DISPATCH_NW(n, w, ...)                                          \
    switch (w) {                                                           \
        case 4: { constexpr int WW = 4; DG_DISPATCH_N(n, __VA_ARGS__); } break;   \
        case 8: { constexpr int WW = 8; DG_DISPATCH_N(n, __VA_ARGS__); } break;   \
        case 16: { constexpr int WW = 16; DG_DISPATCH_N(n, __VA_ARGS__); } break; \
        default: return hipErrorInvalidValue;                              \
    }

// Dispatch on n (NN) and the bracket kernel's tile height (WW, 8 or 16).
#define DG_DISPATCH_NR(n, w, ...)                                          \
    switch (w) {                                                           \
        case 8: { constexpr int WW = 8; DG_DISPATCH_N(n, __VA_ARGS__); } break;   \
        case 16: { constexpr int WW = 16; DG_DISPATCH_N(n, __VA_ARGS__); } break; \
        default: return hipErrorInvalidValue;                              \
    }

inline int pw_blocks(long rows, int cap) {
    long b = (rows + kPwThreads - 1) / kPwThreads;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}


// Node e of the cell whose lane-interleaved offset is l64 (group base + lane,
// the group base a multiple of 64 n^2): nodes are stored in pairs, so a
// lane's nodes 2m and 2m + 1 are adjacent ([m][lane][2]) and one 16-byte
// access (8 bytes in FP32) moves both; an odd last node follows alone.
template <int N>
__device__ __forceinline__ long l64_at(long l64, int e) {
    constexpr int P = (N * N) & ~1;
    const long lane = l64 & 63, base = l64 - lane;
    return e < P ? base + (long)(e >> 1) * 128 + 2 * lane + (e & 1)
                 : base + (long)(P >> 1) * 128 + lane;
}

}  // namespace dgk
