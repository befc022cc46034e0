// Neighbour finding, cleaning and start-hit selection.
//
// Neighbour finding: one lane per grid hit m (row r); the candidates u (row r+1)
// and d (row r-1) inside the window are enumerated from the row grids (the
// bins that can hold a window hit, then exact FP64 window tests); the pair with the
// smallest straight-line deviation D below the cut wins, equal D broken by the
// smaller (id_u, id_d).  Because lanes of a wave hold consecutive grid hits
// (same row, neighbouring bins) their candidate loads hit the same cache lines.
//
// Cleaning keeps reciprocal links; start hits are chain heads with at least
// l_min linked hits.  Both run in one pass: the cleaned successor of any hit is
// recomputed on the fly from the raw links while walking a chain.  Start flags
// are written in cluster-id order and compacted with wave ballots, so the
// tracklet order is the ascending start id whatever the thread timing.
#include "tpc_internal.h"
#include "tpc_device.h"

namespace tpc {

namespace {

constexpr int kListD = 6;  // down-window candidates held in registers per hit

__global__ __launch_bounds__(kBlock) void k_neighbours(GridDesc g, KParams kp, const Hit* __restrict__ hits,
                                                       const uint32_t* __restrict__ bin_off,
                                                       const uint32_t* __restrict__ counters,
                                                       int32_t* __restrict__ up, int32_t* __restrict__ dn,
                                                       uint32_t* __restrict__ cnt) {
    const uint32_t n = counters[C_N_VALID_CLU];
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    uint32_t pairs = 0, linked = 0;
    if (p < n) {
        const Hit m = hits[p];
        const int r = (int)(m.rs % (uint32_t)g.R), s = (int)(m.rs / (uint32_t)g.R);
        int32_t bu = -1, bd = -1;
        if (r > 0 && r < g.R - 1) {
            const double xm = g.row_x[r], xu = g.row_x[r + 1], xd = g.row_x[r - 1];
            const double ym = m.y, zm = m.z;
            const double wyu = kp.win_y * (xu - xm), wzu = kp.win_z * (xu - xm);
            const double wyd = kp.win_y * (xm - xd), wzd = kp.win_z * (xm - xd);
            const BinRange U = bin_range(g, s, r + 1, ym - wyu, ym + wyu, zm - wzu, zm + wzu);
            const BinRange D = bin_range(g, s, r - 1, ym - wyd, ym + wyd, zm - wzd, zm + wzd);
            if (!U.empty && !D.empty) {
                const double w = (xm - xd) / (xu - xd);
                double best = 1e300;
                uint32_t bu_id = 0xFFFFFFFFu, bd_id = 0xFFFFFFFFu;
                // the down-window candidates, once, into a register list (selects with
                // constant indices); more than kListD of them: the nested walk below
                float ly[kListD], lz[kListD];
                uint32_t lid[kListD];
                int32_t lpos[kListD];
                int nd = 0;
#pragma unroll
                for (int q = 0; q < kListD; ++q) {
                    ly[q] = lz[q] = 0.f;
                    lid[q] = 0;
                    lpos[q] = -1;
                }
                for (int jz = D.iz0; jz <= D.iz1; ++jz) {
                    const uint32_t j1 = bin_off[D.base + jz * D.ny + D.iy1 + 1];
                    for (uint32_t j = bin_off[D.base + jz * D.ny + D.iy0]; j < j1; ++j) {
                        const Hit d = hits[j];
                        if (!(fabs((double)d.y - ym) <= wyd) || !(fabs((double)d.z - zm) <= wzd)) continue;
#pragma unroll
                        for (int q = 0; q < kListD; ++q) {
                            const bool here = q == nd;
                            ly[q] = here ? d.y : ly[q];
                            lz[q] = here ? d.z : lz[q];
                            lid[q] = here ? d.id : lid[q];
                            lpos[q] = here ? (int32_t)j : lpos[q];
                        }
                        ++nd;
                    }
                }
                for (int iz = U.iz0; iz <= U.iz1; ++iz) {
                    const uint32_t k1 = bin_off[U.base + iz * U.ny + U.iy1 + 1];
                    for (uint32_t k = bin_off[U.base + iz * U.ny + U.iy0]; k < k1; ++k) {
                        const Hit u = hits[k];
                        const double yu = u.y, zu = u.z;
                        if (!(fabs(yu - ym) <= wyu) || !(fabs(zu - zm) <= wzu)) continue;
                        pairs += (uint32_t)nd;
                        if (nd <= kListD) {
#pragma unroll
                            for (int q = 0; q < kListD; ++q) {
                                const double yd = ly[q], zd = lz[q];
                                const double py = yd + (yu - yd) * w, pz = zd + (zu - zd) * w;
                                const double Dv = (ym - py) * (ym - py) * kp.ivy15 + (zm - pz) * (zm - pz) * kp.ivz15;
                                const bool take = (q < nd) & (Dv <= kp.nb_cut) &
                                                  ((Dv < best) | ((Dv == best) & ((u.id < bu_id) |
                                                                                   ((u.id == bu_id) & (lid[q] < bd_id)))));
                                best = take ? Dv : best;
                                bu = take ? (int32_t)k : bu;
                                bd = take ? lpos[q] : bd;
                                bu_id = take ? u.id : bu_id;
                                bd_id = take ? lid[q] : bd_id;
                            }
                        } else {
                            for (int jz = D.iz0; jz <= D.iz1; ++jz) {
                                const uint32_t j1 = bin_off[D.base + jz * D.ny + D.iy1 + 1];
                                for (uint32_t j = bin_off[D.base + jz * D.ny + D.iy0]; j < j1; ++j) {
                                    const Hit d = hits[j];
                                    const double yd = d.y, zd = d.z;
                                    if (!(fabs(yd - ym) <= wyd) || !(fabs(zd - zm) <= wzd)) continue;
                                    const double py = yd + (yu - yd) * w, pz = zd + (zu - zd) * w;
                                    const double Dv =
                                        (ym - py) * (ym - py) * kp.ivy15 + (zm - pz) * (zm - pz) * kp.ivz15;
                                    if (!(Dv <= kp.nb_cut)) continue;
                                    if (Dv < best || (Dv == best && (u.id < bu_id || (u.id == bu_id && d.id < bd_id)))) {
                                        best = Dv;
                                        bu = (int32_t)k;
                                        bd = (int32_t)j;
                                        bu_id = u.id;
                                        bd_id = d.id;
                                    }
                                }
                            }
                        }
                    }
                }
            }
        }
        up[p] = bu;
        dn[p] = bd;
        linked = bu >= 0;
    }
    block_tally2(pairs, linked, C_N_PAIRS, C_N_LINKS_RAW, cnt);
}

__device__ inline int32_t clean_up(const int32_t* __restrict__ up, const int32_t* __restrict__ dn, int32_t p) {
    const int32_t u = up[p];
    return (u >= 0 && dn[u] == p) ? u : -1;
}

__global__ __launch_bounds__(kBlock) void k_clean_flag(KParams kp, const Hit* __restrict__ hits,
                                                       const uint32_t* __restrict__ counters,
                                                       const int32_t* __restrict__ up, const int32_t* __restrict__ dn,
                                                       int32_t* __restrict__ upc, int32_t* __restrict__ dnc,
                                                       TlHit* __restrict__ tl_hits, uint8_t* __restrict__ start_flag,
                                                       uint32_t* __restrict__ cnt) {
    const uint32_t n = counters[C_N_VALID_CLU];
    const int32_t p = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    uint32_t clean = 0;
    if ((uint32_t)p < n) {
        const int32_t u = clean_up(up, dn, p);
        const int32_t d0 = dn[p];
        const int32_t d = (d0 >= 0 && up[d0] == p) ? d0 : -1;
        const Hit h = hits[p];
        upc[p] = u;
        dnc[p] = d;
        tl_hits[p] = TlHit{h.y, h.z, h.id, u};
        clean = u >= 0;
        uint8_t flag = 0;
        if (d < 0) {
            int len = 1;
            int32_t c = p;
            while (len < kp.l_min) {
                const int32_t nx = clean_up(up, dn, c);
                if (nx < 0) break;
                c = nx;
                ++len;
            }
            flag = len >= kp.l_min;
        }
        // the flags start zeroed (cleared with the grid): only starts are written, a
        // scattered byte write for 7% of the hits instead of all of them
        if (flag) start_flag[h.id] = 1;
    }
    block_tally2(clean, 0, C_N_LINKS_CLEAN, -1, cnt);
}

// per-block number of set flags over cluster ids
__global__ __launch_bounds__(kBlock) void k_flag_count(const uint8_t* __restrict__ flag, int64_t n,
                                                       uint32_t* __restrict__ block_cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool f = i < n && flag[i];
    const uint64_t mask = __ballot(f);
    __shared__ uint32_t wc[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kBlock / 64; ++k) t += wc[k];
        block_cnt[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_flag_write(const uint8_t* __restrict__ flag, int64_t n,
                                                       const uint32_t* __restrict__ block_off,
                                                       const uint32_t* __restrict__ pos_of,
                                                       uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool f = i < n && flag[i];
    const uint64_t mask = __ballot(f);
    __shared__ uint32_t wc[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wc[w] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint32_t off = block_off[blockIdx.x];
    for (int k = 0; k < w; ++k) off += wc[k];
    if (f) {
        const uint64_t below = lane ? (mask & (~0ull >> (64 - lane))) : 0ull;  // mbcnt
        const uint32_t k = off + (uint32_t)__popcll(below);
        out[k] = pos_of[i];
    }
}

// Processing order of the tracklets: start indices grouped by (sector, z slab, row)
// of the start hit.  Tracklets taken from the queue together read the hits of one
// sector and a narrow z range (inside a time frame, one group of collisions), and
// the lanes of a wave start on the same row, so they tend to be in the same pass
// at the same time.  The order inside a group is the arbitrary order of the slot
// atomics: tracklet results do not depend on which lane builds which tracklet.
__device__ inline uint32_t slab_of(const GridDesc& g, const Hit& h, int slab_bins, int n_slab) {
    const float vz = (h.z - g.z_min) * g.inv_bz;
    const int iz = !(vz > 0.0f) ? 0 : (vz >= (float)g.nz ? g.nz - 1 : (int)vz);
    const uint32_t s = h.rs / (uint32_t)g.R, r = h.rs % (uint32_t)g.R;
    return (s * (uint32_t)n_slab + (uint32_t)(iz / slab_bins)) * (uint32_t)g.R + r;
}

__global__ __launch_bounds__(kBlock) void k_slab_count(GridDesc g, const Hit* __restrict__ hits,
                                                       const uint32_t* __restrict__ starts,
                                                       const uint32_t* __restrict__ counters, int slab_bins,
                                                       int n_slab, uint32_t* __restrict__ slab_cnt,
                                                       uint32_t* __restrict__ slot) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= counters[C_N_STARTS]) return;
    slot[k] = atomicAdd(&slab_cnt[slab_of(g, hits[starts[k]], slab_bins, n_slab)], 1u);
}

__global__ __launch_bounds__(kBlock) void k_slab_write(GridDesc g, const Hit* __restrict__ hits,
                                                       const uint32_t* __restrict__ starts,
                                                       const uint32_t* __restrict__ counters, int slab_bins,
                                                       int n_slab, const uint32_t* __restrict__ slab_off,
                                                       const uint32_t* __restrict__ slot, uint32_t* __restrict__ proc) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= counters[C_N_STARTS]) return;
    proc[slab_off[slab_of(g, hits[starts[k]], slab_bins, n_slab)] + slot[k]] = k;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock > 0 ? (n + kBlock - 1) / kBlock : 1); }

}  // namespace

void find_neighbours(const GridDesc& g, const KParams& kp, const Hit* hits, const uint32_t* bin_off,
                     const uint32_t* row_off, int64_t n_max, const uint32_t* counters, int32_t* up, int32_t* dn,
                     const float* mlp_q, uint32_t* cnt, hipStream_t s) {
    (void)row_off;
    (void)mlp_q;
    k_neighbours<<<blocks(n_max), kBlock, 0, s>>>(g, kp, hits, bin_off, counters, up, dn, cnt);
}

void clean_and_flag(const KParams& kp, const Hit* hits, int64_t n_max, const uint32_t* counters, const int32_t* up,
                    const int32_t* dn, int32_t* upc, int32_t* dnc, TlHit* tl_hits, uint8_t* start_flag, uint32_t* cnt,
                    hipStream_t s) {
    k_clean_flag<<<blocks(n_max), kBlock, 0, s>>>(kp, hits, counters, up, dn, upc, dnc, tl_hits, start_flag,
                                                  cnt);
}

void compact_starts(const uint8_t* start_flag, const uint32_t* pos_of, int64_t n, uint32_t* starts,
                    uint32_t* block_cnt, void* scan_scratch, uint32_t* n_starts_dev, hipStream_t s) {
    const unsigned nb = blocks(n);
    k_flag_count<<<nb, kBlock, 0, s>>>(start_flag, n, block_cnt);
    scan_u32(block_cnt, block_cnt, nb, nullptr, n_starts_dev, scan_scratch, s);
    k_flag_write<<<nb, kBlock, 0, s>>>(start_flag, n, block_cnt, pos_of, starts);
}

int slab_count(const GridDesc& g, int slab_bins) { return (g.nz + slab_bins - 1) / slab_bins; }

void order_starts(const GridDesc& g, const Hit* hits, const uint32_t* starts, int64_t t_max, const uint32_t* counters,
                  int slab_bins, uint32_t* slab_cnt, uint32_t* slot, uint32_t* proc, void* scan_scratch,
                  hipStream_t s) {
    const int n_slab = slab_count(g, slab_bins);
    const int64_t nb = (int64_t)g.S * n_slab * g.R;
    fill_u32(slab_cnt, 0u, nb, s);
    k_slab_count<<<blocks(t_max), kBlock, 0, s>>>(g, hits, starts, counters, slab_bins, n_slab, slab_cnt, slot);
    scan_u32(slab_cnt, slab_cnt, nb, nullptr, nullptr, scan_scratch, s);
    k_slab_write<<<blocks(t_max), kBlock, 0, s>>>(g, hits, starts, counters, slab_bins, n_slab, slab_cnt, slot, proc);
}

}  // namespace tpc
