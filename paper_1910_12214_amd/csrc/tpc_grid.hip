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
//
// Row-sector path (used for inputs of at least kRsMinPerKey clusters per row-sector on
// average, when the row-sectors fit a workgroup's LDS histogram; smaller inputs keep the
// bin-counting path, whose fixed costs are lower): the same
// order by three counting sorts whose counters all live in LDS.  First by row-sector:
// each of kRsBlocks workgroups histograms its stretch of clusters over the row-sectors,
// a scan of the (row-sector, workgroup) counts gives every workgroup its place in every
// row-sector, and the clusters are copied there as hit records.  Then one workgroup per
// row-sector orders its hits by piece, a piece being a run of z-bins with at most
// kRsPieceBins bins (bins are z-major, so a piece's bins are contiguous).  Then one
// workgroup per piece counts its hits per bin, scans the counts (its bins' offsets),
// places each hit in its bin and finally moves it to its rank by id inside the bin.  Each
// pass reads records that lie together in memory; only the first scatters.
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

// ---------------------------------------------------------------- row-sector path
__device__ inline bool cl_rs(const tpc_clusters_t& cl, const GridDesc& g, int64_t i, uint32_t& rs) {
    const int r = cl.row[i], s = cl.sector[i];
    rs = (uint32_t)s * (uint32_t)g.R + (uint32_t)r;
    return r < g.R && s < g.S;
}

// The stretch of clusters of workgroup b of kRsBlocks.
__device__ inline void rs_stretch(int64_t n, int64_t& lo, int64_t& hi) {
    lo = n * (int64_t)blockIdx.x / kRsBlocks;
    hi = n * (int64_t)(blockIdx.x + 1) / kRsBlocks;
}

// hist[rs * kRsBlocks + b] = clusters of row-sector rs in workgroup b's stretch; clusters
// with row or sector out of range get no grid position.
__global__ __launch_bounds__(kBlock) void k_rs_count(tpc_clusters_t cl, GridDesc g, uint32_t* __restrict__ hist,
                                                     uint32_t* __restrict__ pos_of) {
    extern __shared__ uint32_t h[];
    const uint32_t RS = (uint32_t)(g.S * g.R);
    for (uint32_t k = threadIdx.x; k < RS; k += kBlock) h[k] = 0;
    __syncthreads();
    int64_t lo, hi;
    rs_stretch(cl.n, lo, hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
        uint32_t rs;
        if (cl_rs(cl, g, i, rs))
            atomicAdd(&h[rs], 1u);
        else
            pos_of[i] = 0xFFFFFFFFu;
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < RS; k += kBlock) hist[(size_t)k * kRsBlocks + blockIdx.x] = h[k];
}

// Copies each cluster as a hit record to its row-sector's segment (arbitrary order
// inside the segment).
__global__ __launch_bounds__(kBlock) void k_rs_scatter(tpc_clusters_t cl, GridDesc g,
                                                       const uint32_t* __restrict__ hoff, Hit* __restrict__ rec) {
    extern __shared__ uint32_t cur[];
    const uint32_t RS = (uint32_t)(g.S * g.R);
    for (uint32_t k = threadIdx.x; k < RS; k += kBlock) cur[k] = hoff[(size_t)k * kRsBlocks + blockIdx.x];
    __syncthreads();
    int64_t lo, hi;
    rs_stretch(cl.n, lo, hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
        uint32_t rs;
        if (!cl_rs(cl, g, i, rs)) continue;
        Hit hr;
        hr.y = cl.y[i];
        hr.z = cl.z[i];
        hr.id = (uint32_t)i;
        hr.rs = rs;
        rec[atomicAdd(&cur[rs], 1u)] = hr;
    }
}

// z-bin and y-bin of a hit (the count pass's expressions).
__device__ inline void hit_bins(const GridDesc& g, const Hit& hr, int r, int32_t ny, int32_t& bz, int32_t& by) {
    const float vy = (hr.y - g.row_ymin[r]) * g.inv_by;
    const float vz = (hr.z - g.z_min) * g.inv_bz;
    bz = bin_coord(vz, g.nz);
    by = bin_coord(vy, ny);
}

// Exclusive scan of one value per thread across a kBlock-thread workgroup.
__device__ inline uint32_t rs_block_scan(uint32_t v, uint32_t* wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int i = 0; i < w; ++i) off += wsum[i];
    __syncthreads();
    return off + inc - v;
}

// Records k0, k0 + kBlock, ... (up to kRsUnroll of them, below end) loaded together, so
// a thread has several loads in flight.
constexpr int kRsUnroll = 4;
__device__ inline void load_run(const Hit* __restrict__ rec, uint32_t k0, uint32_t end, Hit hr[kRsUnroll]) {
#pragma unroll
    for (int u = 0; u < kRsUnroll; ++u)
        if (k0 + u * kBlock < end) hr[u] = rec[k0 + u * kBlock];
}

// One workgroup per row-sector: its hits in z order of pieces (piece p holds z-bins
// [p zs, (p + 1) zs)), arbitrary order inside a piece; piece_off[rs * P + p] is each
// piece's first position.
__global__ __launch_bounds__(kBlock) void k_rs_pieces(GridDesc g, int P, int zs, const uint32_t* __restrict__ hoff,
                                                      const Hit* __restrict__ recA, Hit* __restrict__ recB,
                                                      uint32_t* __restrict__ piece_off) {
    __shared__ uint32_t cnt[kRsMaxPieces];
    __shared__ uint32_t wsum[kBlock / 64];
    const uint32_t rs = blockIdx.x;
    const uint32_t seg0 = hoff[(size_t)rs * kRsBlocks], seg1 = hoff[(size_t)(rs + 1) * kRsBlocks];
    const int r = (int)(rs % (uint32_t)g.R);
    const int32_t ny = g.row_ny[r];
    for (int p = threadIdx.x; p < P; p += kBlock) cnt[p] = 0;
    __syncthreads();
    for (uint32_t k0 = seg0 + threadIdx.x; k0 < seg1; k0 += kRsUnroll * kBlock) {
        Hit hr[kRsUnroll];
        load_run(recA, k0, seg1, hr);
#pragma unroll
        for (int u = 0; u < kRsUnroll; ++u) {
            if (k0 + u * kBlock >= seg1) break;
            int32_t bz, by;
            hit_bins(g, hr[u], r, ny, bz, by);
            atomicAdd(&cnt[bz / zs], 1u);
        }
    }
    __syncthreads();
    const uint32_t c = threadIdx.x < (uint32_t)P ? cnt[threadIdx.x] : 0u;  // P <= kBlock
    const uint32_t off = rs_block_scan(c, wsum);
    if (threadIdx.x < (uint32_t)P) {
        cnt[threadIdx.x] = off;
        piece_off[(size_t)rs * P + threadIdx.x] = seg0 + off;
    }
    if (rs + 1 == (uint32_t)(g.S * g.R) && threadIdx.x == 0) piece_off[(size_t)(rs + 1) * P] = seg1;  // the total
    __syncthreads();
    for (uint32_t k0 = seg0 + threadIdx.x; k0 < seg1; k0 += kRsUnroll * kBlock) {
        Hit hr[kRsUnroll];
        load_run(recA, k0, seg1, hr);
#pragma unroll
        for (int u = 0; u < kRsUnroll; ++u) {
            if (k0 + u * kBlock >= seg1) break;
            int32_t bz, by;
            hit_bins(g, hr[u], r, ny, bz, by);
            recB[seg0 + atomicAdd(&cnt[bz / zs], 1u)] = hr[u];
        }
    }
}

// One workgroup per piece: counts its hits per bin in LDS, scans the counts (its bins'
// offsets), places each hit in its bin (arbitrary order), then moves it to its rank by
// id inside the bin and writes the hit record and the cluster's grid position.
__global__ __launch_bounds__(kBlock) void k_rs_bins(GridDesc g, int P, int zs, const uint32_t* __restrict__ piece_off,
                                                    const Hit* __restrict__ recB, Hit* __restrict__ recA,
                                                    uint32_t* __restrict__ bin_off, Hit* __restrict__ hits,
                                                    uint32_t* __restrict__ pos_of) {
    __shared__ uint32_t cnt[kRsPieceBins];
    __shared__ uint32_t wsum[kBlock / 64];
    const uint32_t q = blockIdx.x, rs = q / (uint32_t)P, p = q % (uint32_t)P;
    const uint32_t h0 = piece_off[q], h1 = piece_off[q + 1];
    const int r = (int)(rs % (uint32_t)g.R);
    const int32_t ny = g.row_ny[r];
    const int32_t bz0 = (int32_t)p * zs, bz1 = bz0 + zs < g.nz ? bz0 + zs : g.nz;
    if (bz0 >= bz1) return;  // a piece past the last z-bin (no bins, no hits)
    const uint32_t nb = (uint32_t)(bz1 - bz0) * (uint32_t)ny;
    const uint32_t b0 = g.bin_base[rs] + (uint32_t)bz0 * (uint32_t)ny;
    for (uint32_t j = threadIdx.x; j < nb; j += kBlock) cnt[j] = 0;
    __syncthreads();
    for (uint32_t k0 = h0 + threadIdx.x; k0 < h1; k0 += kRsUnroll * kBlock) {
        Hit hr[kRsUnroll];
        load_run(recB, k0, h1, hr);
#pragma unroll
        for (int u = 0; u < kRsUnroll; ++u) {
            if (k0 + u * kBlock >= h1) break;
            int32_t bz, by;
            hit_bins(g, hr[u], r, ny, bz, by);
            atomicAdd(&cnt[(uint32_t)(bz - bz0) * (uint32_t)ny + (uint32_t)by], 1u);
        }
    }
    __syncthreads();
    // scan: thread t takes a contiguous run of per counters
    const uint32_t per = (nb + kBlock - 1) / kBlock, j0 = threadIdx.x * per;
    const uint32_t j1 = j0 + per < nb ? j0 + per : nb;
    uint32_t sum = 0;
    for (uint32_t j = j0; j < j1; ++j) sum += cnt[j];
    uint32_t off = rs_block_scan(sum, wsum);
    for (uint32_t j = j0; j < j1; ++j) {
        const uint32_t c = cnt[j];
        cnt[j] = off;
        off += c;
    }
    if (q + 1 == (uint32_t)(g.S * g.R) * (uint32_t)P && threadIdx.x == 0) bin_off[g.n_bins] = h1;  // the total
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < nb; j += kBlock) bin_off[b0 + j] = h0 + cnt[j];  // coalesced
    __syncthreads();  // the counters become the placement cursors only after every offset is read
    for (uint32_t k0 = h0 + threadIdx.x; k0 < h1; k0 += kRsUnroll * kBlock) {
        Hit hr[kRsUnroll];
        load_run(recB, k0, h1, hr);
#pragma unroll
        for (int u = 0; u < kRsUnroll; ++u) {
            if (k0 + u * kBlock >= h1) break;
            int32_t bz, by;
            hit_bins(g, hr[u], r, ny, bz, by);
            recA[h0 + atomicAdd(&cnt[(uint32_t)(bz - bz0) * (uint32_t)ny + (uint32_t)by], 1u)] = hr[u];
        }
    }
    __syncthreads();
    // each bin's counter now holds its end, which is the next bin's start
    for (uint32_t k = h0 + threadIdx.x; k < h1; k += kBlock) {
        const Hit hr = recA[k];
        int32_t bz, by;
        hit_bins(g, hr, r, ny, bz, by);
        const uint32_t lb = (uint32_t)(bz - bz0) * (uint32_t)ny + (uint32_t)by;
        const uint32_t e = cnt[lb], b = lb == 0 ? 0u : cnt[lb - 1];
        uint32_t f = h0 + b;
        for (uint32_t j = h0 + b; j < h0 + e; ++j) f += recA[j].id < hr.id;
        hits[f] = hr;
        pos_of[hr.id] = f;
    }
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

// Pieces of a row-sector: z-bins per piece such that a piece has at most kRsPieceBins bins.
static void rs_piece_shape(const GridDesc& g, int& P, int& zs) {
    zs = g.ny_max > 0 ? kRsPieceBins / g.ny_max : 1;
    if (zs < 1) zs = 1;
    P = (g.nz + zs - 1) / zs;
}

bool grid_rs_fits(const GridDesc& g, int64_t n) {
    int P, zs;
    rs_piece_shape(g, P, zs);
    const int64_t RS = (int64_t)g.S * g.R;
    return RS <= kRsMaxKeys && g.ny_max <= kRsPieceBins && P <= kRsMaxPieces && n >= kRsMinPerKey * RS;
}

size_t grid_rs_hist_entries(const GridDesc& g) { return (size_t)g.S * g.R * kRsBlocks + 1; }

size_t grid_rs_piece_entries(const GridDesc& g) {
    int P, zs;
    rs_piece_shape(g, P, zs);
    return (size_t)g.S * g.R * P + 1;
}

void grid_build_rs(const tpc_clusters_t& cl, const GridDesc& g, uint32_t* hist, uint32_t* hoff, uint32_t* piece_off,
                   void* scan_scratch, Hit* recA, Hit* recB, uint32_t* bin_off, Hit* hits, uint32_t* pos_of,
                   uint32_t* row_off, uint32_t* counters, hipStream_t s) {
    const int64_t RS = (int64_t)g.S * g.R;
    int P, zs;
    rs_piece_shape(g, P, zs);
    const size_t lds = sizeof(uint32_t) * (size_t)RS;
    k_rs_count<<<kRsBlocks, kBlock, lds, s>>>(cl, g, hist, pos_of);
    scan_u32(hist, hoff, RS * kRsBlocks, nullptr, hoff + RS * kRsBlocks, scan_scratch, s);
    k_rs_scatter<<<kRsBlocks, kBlock, lds, s>>>(cl, g, hoff, recA);
    k_rs_pieces<<<(unsigned)RS, kBlock, 0, s>>>(g, P, zs, hoff, recA, recB, piece_off);
    k_rs_bins<<<(unsigned)(RS * P), kBlock, 0, s>>>(g, P, zs, piece_off, recB, recA, bin_off, hits, pos_of);
    k_row_off<<<blocks(RS + 1), kBlock, 0, s>>>(g, bin_off, row_off, counters);
}

}  // namespace tpc
