// Device-wide exclusive scan of uint32 and fill kernels.
//
// 2048 elements per 256-thread block.  Up to kSmallTiles tiles: two passes (block
// sums, then each block adds up the sums before it and scans its tile); more:
// three (block sums -> scan of block sums -> block scan + offset).  The element count may live in device
// memory (counts produced by an earlier kernel), so the whole chain can be
// enqueued (and captured in a graph) without a host round trip.
#include "tpc_internal.h"

namespace tpc {

namespace {

constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// exclusive scan of one value per thread across a 256-thread block; returns the block total in *tot
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* tot) {
    __shared__ uint32_t wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        if (i < w) off += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *tot = all;
    return off + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_reduce(const uint32_t* __restrict__ in, int64_t n_max,
                                                   const uint32_t* __restrict__ n_dev, uint32_t* __restrict__ part) {
    const int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t s = 0;
    if (base < n) {
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            int64_t k = base + (int64_t)i * kBlock + threadIdx.x;
            if (k < n) s += in[k];
        }
    }
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_parts(uint32_t* __restrict__ part, int64_t nb,
                                                       uint32_t* __restrict__ total) {
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kBlock) {
        int64_t k = base + threadIdx.x;
        uint32_t v = k < nb ? part[k] : 0;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, &tot);
        if (k < nb) part[k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kBlock) void k_apply(const uint32_t* in, uint32_t* out, int64_t n_max,
                                                  const uint32_t* __restrict__ n_dev,
                                                  const uint32_t* __restrict__ part) {
    const int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (base >= n) return;
    // each thread owns kItems consecutive elements
    const int64_t my = base + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = (my + i < n) ? in[my + i] : 0;
        s += v[i];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(s, &tot) + part[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        if (my + i < n) out[my + i] = off;
        off += v[i];
    }
}

// Second pass of the two-pass scan: the tile's offset is the sum of the block sums
// before it (at most kSmallTiles, read by the whole block), then as k_apply.
constexpr int64_t kSmallTiles = 2048;

__global__ __launch_bounds__(kBlock) void k_apply_pre(const uint32_t* in, uint32_t* out, int64_t n_max,
                                                      const uint32_t* __restrict__ n_dev,
                                                      const uint32_t* __restrict__ part, uint32_t* __restrict__ total) {
    const int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (base >= n) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && total) *total = 0;  // n == 0
        return;
    }
    uint32_t pre = 0;
    for (int64_t k = threadIdx.x; k < (int64_t)blockIdx.x; k += kBlock) pre += part[k];
    uint32_t prefix;
    block_excl_scan(pre, &prefix);
    const int64_t my = base + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = (my + i < n) ? in[my + i] : 0;
        s += v[i];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(s, &tot) + prefix;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        if (my + i < n) out[my + i] = off;
        off += v[i];
    }
    // the last tile's last thread holds the grand total
    if (total && base + kTile >= n && threadIdx.x == kBlock - 1) *total = off;
}

__global__ void k_fill32(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill64(uint64_t* p, uint64_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

inline int grid_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (int)b;
}

}  // namespace

size_t scan_scratch_bytes(int64_t n_max) { return sizeof(uint32_t) * (size_t)((n_max + kTile - 1) / kTile + 1); }

void scan_u32(const uint32_t* in, uint32_t* out, int64_t n_max, const uint32_t* n_dev, uint32_t* total_dev,
              void* scratch, hipStream_t s) {
    int64_t nb = (n_max + kTile - 1) / kTile;
    if (nb < 1) nb = 1;
    uint32_t* part = (uint32_t*)scratch;
    k_reduce<<<(unsigned)nb, kBlock, 0, s>>>(in, n_max, n_dev, part);
    if (nb <= kSmallTiles) {
        k_apply_pre<<<(unsigned)nb, kBlock, 0, s>>>(in, out, n_max, n_dev, part, total_dev);
        return;
    }
    k_scan_parts<<<1, kBlock, 0, s>>>(part, nb, total_dev);
    k_apply<<<(unsigned)nb, kBlock, 0, s>>>(in, out, n_max, n_dev, part);
}

void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill32<<<grid_for(n), kBlock, 0, s>>>(p, v, n);
}
void fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill64<<<grid_for(n), kBlock, 0, s>>>(p, v, n);
}

}  // namespace tpc
