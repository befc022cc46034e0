// Row-binned hit grid: per (sector,row) a uniform ny x nz (y,z) bin grid, bins
// z-major, hits ordered by (sector, row, bin, cluster id).
//
// Counting sort in three passes.  The count pass computes each cluster's bin
// (FP32: floor((y - ymin) * inv_bin), clamped) and counts with atomics; after the
// scan the scatter pass places cluster ids with atomics (arbitrary order inside
// a bin); the finalize pass sorts each bin's ids (bins hold a handful of hits)
// which makes the order deterministic and stable, then gathers the 16-byte hit
// records so that every later candidate test is one coalescable load.
#include "tpc_internal.h"

namespace tpc {

namespace {

__device__ inline int32_t bin_coord(float v, int32_t nmax) {
    if (!(v > 0.0f)) return 0;
    if (v >= (float)nmax) return nmax - 1;
    return (int32_t)v;
}

__global__ __launch_bounds__(kBlock) void k_count(tpc_clusters_t cl, GridDesc g, uint32_t* __restrict__ bin_of,
                                                  uint32_t* __restrict__ bin_cnt, uint32_t* __restrict__ pos_of) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= cl.n) return;
    const int r = cl.row[i], s = cl.sector[i];
    if (r >= g.R || s >= g.S) {
        bin_of[i] = 0xFFFFFFFFu;
        pos_of[i] = 0xFFFFFFFFu;
        return;
    }
    const int32_t ny = g.row_ny[r];
    // two fp32 operations, no contraction possible: identical on every IEEE implementation
    const float vy = (cl.y[i] - g.row_ymin[r]) * g.inv_by;
    const float vz = (cl.z[i] - g.z_min) * g.inv_bz;
    const uint32_t b = g.bin_base[s * g.R + r] + (uint32_t)(bin_coord(vz, g.nz) * ny + bin_coord(vy, ny));
    bin_of[i] = b;
    atomicAdd(&bin_cnt[b], 1u);
}

__global__ __launch_bounds__(kBlock) void k_scatter(int64_t n, const uint32_t* __restrict__ bin_of,
                                                    const uint32_t* __restrict__ bin_off,
                                                    uint32_t* __restrict__ bin_fill, uint32_t* __restrict__ sorted_id) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t b = bin_of[i];
    if (b == 0xFFFFFFFFu) return;
    sorted_id[bin_off[b] + atomicAdd(&bin_fill[b], 1u)] = (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_finalize(tpc_clusters_t cl, GridDesc g, const uint32_t* __restrict__ bin_off,
                                                     uint32_t* __restrict__ sorted_id, Hit* __restrict__ hits,
                                                     uint32_t* __restrict__ pos_of) {
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= g.n_bins) return;
    const uint32_t k0 = bin_off[b], k1 = bin_off[b + 1];
    if (k1 == k0) return;
    // insertion sort of the bin's ids (small), in place
    for (uint32_t a = k0 + 1; a < k1; ++a) {
        const uint32_t v = sorted_id[a];
        uint32_t j = a;
        while (j > k0 && sorted_id[j - 1] > v) {
            sorted_id[j] = sorted_id[j - 1];
            --j;
        }
        sorted_id[j] = v;
    }
    const uint32_t id0 = sorted_id[k0];
    const uint32_t rs = (uint32_t)cl.sector[id0] * (uint32_t)g.R + cl.row[id0];
    for (uint32_t k = k0; k < k1; ++k) {
        const uint32_t id = sorted_id[k];
        Hit h;
        h.y = cl.y[id];
        h.z = cl.z[id];
        h.id = id;
        h.rs = rs;
        hits[k] = h;
        pos_of[id] = k;
    }
}

__global__ void k_row_off(GridDesc g, const uint32_t* __restrict__ bin_off, uint32_t* __restrict__ row_off,
                          uint32_t* __restrict__ counters) {
    const int rs = blockIdx.x * blockDim.x + threadIdx.x;
    if (rs > g.S * g.R) return;
    row_off[rs] = bin_off[g.bin_base[rs]];
    if (rs == g.S * g.R) counters[C_N_VALID_CLU] = bin_off[g.n_bins];
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock > 0 ? (n + kBlock - 1) / kBlock : 1); }

}  // namespace

void grid_count(const tpc_clusters_t& cl, const GridDesc& g, uint32_t* bin_of, uint32_t* bin_cnt,
                    uint32_t* pos_of, hipStream_t s) {
    if (cl.n > 0) k_count<<<blocks(cl.n), kBlock, 0, s>>>(cl, g, bin_of, bin_cnt, pos_of);
}

void grid_scatter(const tpc_clusters_t& cl, const uint32_t* bin_of, const uint32_t* bin_off, uint32_t* bin_fill,
                  uint32_t* sorted_id, hipStream_t s) {
    if (cl.n > 0) k_scatter<<<blocks(cl.n), kBlock, 0, s>>>(cl.n, bin_of, bin_off, bin_fill, sorted_id);
}

void grid_finalize(const tpc_clusters_t& cl, const GridDesc& g, const uint32_t* bin_off, uint32_t* sorted_id,
                   Hit* hits, uint32_t* pos_of, uint32_t* row_off, uint32_t* counters, hipStream_t s) {
    k_finalize<<<blocks(g.n_bins), kBlock, 0, s>>>(cl, g, bin_off, sorted_id, hits, pos_of);
    k_row_off<<<blocks(g.S * g.R + 1), kBlock, 0, s>>>(g, bin_off, row_off, counters);
}

}  // namespace tpc
