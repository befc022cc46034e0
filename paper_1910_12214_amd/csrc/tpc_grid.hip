// Row-binned hit grid: per (sector,row) a uniform ny x nz (y,z) bin grid, bins
// z-major, hits ordered by (sector, row, bin, cluster id).
//
// Counting sort in three passes over the clusters.  The count pass computes each
// cluster's bin (FP32: floor((y - ymin) * inv_bin), clamped) and takes a slot in
// it with the value an atomic increment returns (arbitrary order inside a bin);
// after the scan of the bin counts the scatter pass writes cluster ids to those
// slots; the finalize pass, one thread per sorted position, moves each cluster to
// its rank by id inside its bin (bins hold a handful of hits), which makes the
// order deterministic, and writes the 16-byte hit record so that every later
// candidate test is one coalescable load.  No pass walks the bins themselves,
// so the cost follows the cluster count even where most bins are empty.
#include "tpc_internal.h"

namespace tpc {

namespace {

__device__ inline int32_t bin_coord(float v, int32_t nmax) {
    if (!(v > 0.0f)) return 0;
    if (v >= (float)nmax) return nmax - 1;
    return (int32_t)v;
}

__global__ __launch_bounds__(kBlock) void k_count(tpc_clusters_t cl, GridDesc g, uint32_t* __restrict__ bin_of,
                                                  uint32_t* __restrict__ bin_cnt, uint32_t* __restrict__ slot_of,
                                                  uint32_t* __restrict__ pos_of) {
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
    slot_of[i] = atomicAdd(&bin_cnt[b], 1u);
}

__global__ __launch_bounds__(kBlock) void k_scatter(int64_t n, const uint32_t* __restrict__ bin_of,
                                                    const uint32_t* __restrict__ slot_of,
                                                    const uint32_t* __restrict__ bin_off,
                                                    uint32_t* __restrict__ sorted_id) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t b = bin_of[i];
    if (b == 0xFFFFFFFFu) return;
    sorted_id[bin_off[b] + slot_of[i]] = (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_finalize(tpc_clusters_t cl, GridDesc g, const uint32_t* __restrict__ bin_of,
                                                     const uint32_t* __restrict__ bin_off,
                                                     const uint32_t* __restrict__ sorted_id, Hit* __restrict__ hits,
                                                     uint32_t* __restrict__ pos_of) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= bin_off[g.n_bins]) return;
    const uint32_t id = sorted_id[k];
    const uint32_t b = bin_of[id];
    const uint32_t k0 = bin_off[b], k1 = bin_off[b + 1];
    uint32_t f = k0;
    for (uint32_t j = k0; j < k1; ++j) f += sorted_id[j] < id;
    Hit h;
    h.y = cl.y[id];
    h.z = cl.z[id];
    h.id = id;
    h.rs = (uint32_t)cl.sector[id] * (uint32_t)g.R + cl.row[id];
    hits[f] = h;
    pos_of[id] = f;
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

void grid_count(const tpc_clusters_t& cl, const GridDesc& g, uint32_t* bin_of, uint32_t* bin_cnt, uint32_t* slot_of,
                uint32_t* pos_of, hipStream_t s) {
    if (cl.n > 0) k_count<<<blocks(cl.n), kBlock, 0, s>>>(cl, g, bin_of, bin_cnt, slot_of, pos_of);
}

void grid_scatter(const tpc_clusters_t& cl, const uint32_t* bin_of, const uint32_t* slot_of, const uint32_t* bin_off,
                  uint32_t* sorted_id, hipStream_t s) {
    if (cl.n > 0) k_scatter<<<blocks(cl.n), kBlock, 0, s>>>(cl.n, bin_of, slot_of, bin_off, sorted_id);
}

void grid_finalize(const tpc_clusters_t& cl, const GridDesc& g, const uint32_t* bin_of, const uint32_t* bin_off,
                   const uint32_t* sorted_id, Hit* hits, uint32_t* pos_of, uint32_t* row_off, uint32_t* counters,
                   hipStream_t s) {
    if (cl.n > 0) k_finalize<<<blocks(cl.n), kBlock, 0, s>>>(cl, g, bin_of, bin_off, sorted_id, hits, pos_of);
    k_row_off<<<blocks(g.S * g.R + 1), kBlock, 0, s>>>(g, bin_off, row_off, counters);
}

}  // namespace tpc
