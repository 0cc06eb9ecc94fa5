// kin_order.hip -- cost order of an instance's cells for its next advance.
//
// The advance kernels hand cells to lanes (or wavefronts) from a work counter, so a launch
// ends when its last cells finish; cells that need many Newton iterations and are taken late
// leave the rest of the device idle.  The iterations a cell needed in the previous advance of
// the same instance predict its cost well, so the next advance takes the cells in kOrderClasses
// geometric classes, most expensive first: >= 320, 160-319, ..., 10-19, 5-9 and < 5
// iterations.  A first advance (no counts yet) may pass classes computed otherwise (direct).  Within a class cells keep their index order, which keeps the state accesses of
// neighbouring lanes coalesced.  Which cell a lane takes does not change that cell's
// arithmetic: results are bitwise the same in any order.
//
// A stable counting sort in three kernels over tiles of kOrderTile cells: per-tile class
// counts, one block that turns them into each tile's first position per class, and a scatter
// that ranks a tile's cells within their class by wavefront ballots.
#include <hip/hip_runtime.h>

#include "kin_internal.h"

namespace kin {
namespace {

constexpr int kC = kOrderClasses;
constexpr int kOrderThreads = 256;
constexpr int kOrderRounds = kOrderTile / kOrderThreads;
constexpr int kScanThreads = 1024;

// class of a cell that needed `it` iterations: 0 below 5, then one class per doubling; with
// direct, the key is the class
__device__ __forceinline__ int cost_class(int it, int direct)
{
    if (direct) return it < 0 ? 0 : (it >= kC ? kC - 1 : it);
    int k = 0;
#pragma unroll
    for (int b = 5; b <= (5 << (kC - 2)); b <<= 1) k += it >= b;
    return k;
}

// ocount[kC t + c] = cells of class c in tile t
__global__ void __launch_bounds__(kOrderThreads) order_count_kernel(const int *iters, long long n, int direct,
                                                                    int *ocount)
{
    __shared__ int cnt[kC];
    if (threadIdx.x < kC) cnt[threadIdx.x] = 0;
    __syncthreads();
    const long long t0 = (long long)blockIdx.x * kOrderTile;
    for (int r = 0; r < kOrderRounds; ++r) {
        const long long i = t0 + (long long)r * kOrderThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[cost_class(iters[i], direct)], 1);
    }
    __syncthreads();
    if (threadIdx.x < kC) ocount[(size_t)blockIdx.x * kC + threadIdx.x] = cnt[threadIdx.x];
}

// In place: ocount[kC t + c] becomes the first position of tile t's class-c cells.  Classes
// are laid out from kC - 1 down to 0; within a class, tiles in order.  One block; thread u
// owns a contiguous run of tiles.
__global__ void __launch_bounds__(kScanThreads) order_scan_kernel(int *ocount, long long tiles,
                                                                  unsigned long long *clear)
{
    if (clear && threadIdx.x == 0) *clear = 0ull;  // the advance's work counter
    __shared__ int sc[kC][kScanThreads];
    __shared__ int tot[kC];
    const int u = threadIdx.x;
    const long long per = (tiles + kScanThreads - 1) / kScanThreads;
    const long long b0 = (long long)u * per, b1 = b0 + per < tiles ? b0 + per : tiles;
    int s[kC];
#pragma unroll
    for (int c = 0; c < kC; ++c) s[c] = 0;
    for (long long b = b0; b < b1; ++b)
#pragma unroll
        for (int c = 0; c < kC; ++c) s[c] += ocount[b * kC + c];
#pragma unroll
    for (int c = 0; c < kC; ++c) sc[c][u] = s[c];
    __syncthreads();
    // inclusive scans over the threads (Hillis-Steele)
    for (int d = 1; d < kScanThreads; d <<= 1) {
        int v[kC];
#pragma unroll
        for (int c = 0; c < kC; ++c) v[c] = u >= d ? sc[c][u - d] : 0;
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kC; ++c) sc[c][u] += v[c];
        __syncthreads();
    }
    if (u < kC) tot[u] = sc[u][kScanThreads - 1];
    __syncthreads();
    int run[kC];
    int acc = 0;
#pragma unroll
    for (int c = kC - 1; c >= 0; --c) {
        run[c] = acc + sc[c][u] - s[c];
        acc += tot[c];
    }
    for (long long b = b0; b < b1; ++b)
#pragma unroll
        for (int c = 0; c < kC; ++c) {
            const int k = ocount[b * kC + c];
            ocount[b * kC + c] = run[c];
            run[c] += k;
        }
}

// order[position] = cell, stable within each class
__global__ void __launch_bounds__(kOrderThreads) order_scatter_kernel(const int *iters, long long n, int direct,
                                                                      const int *ocount, int *order)
{
    constexpr int kWaves = kOrderThreads / 64;
    __shared__ int run[kC];
    __shared__ int wcnt[kWaves][kC];
    if (threadIdx.x < kC) run[threadIdx.x] = ocount[(size_t)blockIdx.x * kC + threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long t0 = (long long)blockIdx.x * kOrderTile;
    for (int r = 0; r < kOrderRounds; ++r) {
        const long long i = t0 + (long long)r * kOrderThreads + threadIdx.x;
        const bool valid = i < n;
        const int k = valid ? cost_class(iters[i], direct) : -1;
        unsigned long long mine = 0;
#pragma unroll
        for (int c = 0; c < kC; ++c) {
            const unsigned long long b = __ballot(k == c);
            if (k == c) mine = b;
            if (lane == 0) wcnt[w][c] = __popcll(b);
        }
        __syncthreads();
        if (valid) {
            const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mine >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((unsigned)mine, 0u));
            int p = run[k] + rank;
            for (int w2 = 0; w2 < w; ++w2) p += wcnt[w2][k];
            if (p >= 0 && p < n) order[p] = (int)i;
        }
        __syncthreads();
        if (threadIdx.x < kC) {
            int add = 0;
            for (int w2 = 0; w2 < kWaves; ++w2) add += wcnt[w2][threadIdx.x];
            run[threadIdx.x] += add;
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_cost_order(const int *key, long long n, bool direct, int *order, int *ocount,
                              unsigned long long *clear, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (n > 0x7fffffffLL) return hipErrorInvalidValue;
    const long long tiles = order_tiles(n);
    const int d = direct ? 1 : 0;
    hipLaunchKernelGGL(order_count_kernel, dim3((unsigned)tiles), dim3(kOrderThreads), 0, s, key, n, d, ocount);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, ocount, tiles, clear);
    hipLaunchKernelGGL(order_scatter_kernel, dim3((unsigned)tiles), dim3(kOrderThreads), 0, s, key, n, d, ocount,
                       order);
    return hipGetLastError();
}

}  // namespace kin
