// Tracklet selection and track output.
//
// key(t) = (n_hits << 32) | (0xFFFFFFFF - start cluster id): longer tracklets win,
// equal lengths go to the lower start id.  hitKey[c] = max over valid tracklets
// containing c, by 64-bit atomicMax; the maximum does not depend on the order
// in which lanes apply their atomics, so hit ownership is independent of
// processing order.  A tracklet owns the hits whose key equals its own and
// becomes a track with at least n_min_track owned hits.  Track and hit offsets
// come from exclusive scans in start order, so the output is in ascending
// start id.
#include "tpc_device.h"
#include "tpc_internal.h"

namespace tpc {

namespace {

__device__ inline uint64_t tl_key(uint32_t nh, uint32_t start_id) {
    return ((uint64_t)nh << 32) | (uint64_t)(0xFFFFFFFFu - start_id);
}

// One wave per tracklet.  Waves walk the processing order restricted to their
// workgroup's XCD slice (the same slices the tracklet kernel drained, so the hits
// are still in that XCD's L2); the lanes of a wave share the tracklet's hit list,
// so slot reads are contiguous and the output hit ids are written coalesced.
struct WaveWalk {
    uint32_t j, hi, step;
    __device__ WaveWalk(uint32_t n) {
        const uint32_t x = blockIdx.x % kXcd, per = gridDim.x / kXcd, b = blockIdx.x / kXcd;
        const uint32_t wpb = blockDim.x >> 6;
        const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const uint32_t lo = (uint32_t)((uint64_t)n * x / kXcd);
        hi = (uint32_t)((uint64_t)n * (x + 1) / kXcd);
        j = lo + b * wpb + wave;
        step = per * wpb;
    }
    __device__ bool ok() const { return j < hi; }
    __device__ void next() { j += step; }
};

// Key pass order: valid tracklets by decreasing hit count (counting sort, one
// bucket per count, arbitrary order inside a bucket).  Processed in this order,
// the longest tracklet of a track tends to set its hits' keys first and its
// shorter duplicates read a larger key and skip the atomic.  The keys themselves
// do not depend on the order.
constexpr int kSortBlocks = 1024;

__global__ __launch_bounds__(kBlock) void k_len_count(TrackletOut o, const uint32_t* __restrict__ counters,
                                                      uint32_t* __restrict__ cnt) {
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = counters[C_N_STARTS];
    for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < n; k += kSortBlocks * kBlock)
        if (o.flags[k] & 1u) atomicAdd(&hist[255 - min(o.nhits[k], 255)], 1u);
    __syncthreads();
    cnt[threadIdx.x * kSortBlocks + blockIdx.x] = hist[threadIdx.x];  // bucket-major: the scan gives the order
}

__global__ __launch_bounds__(kBlock) void k_len_scatter(TrackletOut o, const uint32_t* __restrict__ counters,
                                                        const uint32_t* __restrict__ off, uint32_t* __restrict__ order) {
    __shared__ uint32_t base[256];
    base[threadIdx.x] = off[threadIdx.x * kSortBlocks + blockIdx.x];
    __syncthreads();
    const uint32_t n = counters[C_N_STARTS];
    for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < n; k += kSortBlocks * kBlock)
        if (o.flags[k] & 1u) order[atomicAdd(&base[255 - min(o.nhits[k], 255)], 1u)] = k;
}

// One tracklet per wave (the launch covers every valid tracklet once when it can):
// all slot entries are loaded, then all keys read, then the atomics issued, and
// the wave ends.  A wave never issues a load after an atomic, so no load waits for
// an atomic to complete (vector memory operations retire in order).
__global__ __launch_bounds__(kBlock) void k_keys(const Hit* __restrict__ hits, const uint32_t* __restrict__ starts,
                                                 const uint32_t* __restrict__ order, TrackletOut o, int R,
                                                 const uint32_t* __restrict__ counters, uint64_t* __restrict__ hit_key) {
    const uint32_t n = counters[C_N_VALID_TL];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t wave = blockIdx.x * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint32_t j = wave; j < n; j += gridDim.x * wpb) {  // in order of decreasing length
        const uint32_t k = order[j];
        const uint32_t nh = (uint32_t)o.nhits[k];
        const uint64_t key = tl_key(nh, hits[starts[k]].id);
        const int32_t* slot = o.hits + (size_t)k * R + (R - (int)nh);
        int32_t pos[4];
        uint64_t cur[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {  // R <= 255 < 4 * 64
            const uint32_t i = lane + 64u * q;
            pos[q] = i < nh ? slot[i] : -1;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) cur[q] = pos[q] >= 0 ? hit_key[pos[q]] : ~0ull;
        // keys only grow: a plain read at or above ours makes the atomic unnecessary
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (cur[q] < key) atomicMax((unsigned long long*)&hit_key[pos[q]], (unsigned long long)key);
    }
}

__global__ __launch_bounds__(kBlock) void k_own(const Hit* __restrict__ hits, const uint32_t* __restrict__ starts,
                                                const uint32_t* __restrict__ proc, TrackletOut o, int R,
                                                const uint32_t* __restrict__ counters,
                                                const uint64_t* __restrict__ hit_key, int n_min_trk,
                                                uint32_t* __restrict__ own_cnt, uint32_t* __restrict__ trk_flag,
                                                uint64_t* __restrict__ own_mask) {
    const uint32_t n = counters[C_N_STARTS];
    const uint32_t lane = threadIdx.x & 63;
    for (WaveWalk w(n); w.ok(); w.next()) {
        const uint32_t k = proc[w.j];
        uint32_t owned = 0;
        if (o.flags[k] & 1u) {
            const uint32_t nh = (uint32_t)o.nhits[k];
            const uint64_t key = tl_key(nh, hits[starts[k]].id);
            const int32_t* slot = o.hits + (size_t)k * R + (R - (int)nh);
            uint64_t mq = 0;  // lane q < 4 keeps the ownership bits of slot entries 64 q .. 64 q + 63
            for (uint32_t base = 0; base < nh; base += 64) {
                const uint32_t j = base + lane;
                const uint64_t m = __ballot(j < nh && hit_key[slot[j]] == key);
                if (lane == base / 64) mq = m;
                owned += (uint32_t)__popcll(m);
            }
            if ((int)owned < n_min_trk) owned = 0;
            if (owned && lane < 4) own_mask[(size_t)k * 4 + lane] = mq;
        }
        if (lane == 0) {
            own_cnt[k] = owned;
            trk_flag[k] = owned ? 1u : 0u;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_write(const Hit* __restrict__ hits, const uint32_t* __restrict__ starts,
                                                  const uint32_t* __restrict__ proc, TrackletOut o, GridDesc g,
                                                  const uint32_t* __restrict__ counters,
                                                  const uint64_t* __restrict__ hit_key,
                                                  const uint32_t* __restrict__ own_cnt,
                                                  const uint32_t* __restrict__ hit_off,
                                                  const uint32_t* __restrict__ trk_idx, tpc_tracks_t out,
                                                  const uint64_t* __restrict__ own_mask) {
    const uint32_t n = counters[C_N_STARTS];
    const int R = g.R;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (WaveWalk w(n); w.ok(); w.next()) {
        const uint32_t k = proc[w.j];
        const uint32_t cnt = own_cnt[k];
        if (!cnt) continue;
        const uint32_t t = trk_idx[k], off = hit_off[k];
        if (t >= (uint32_t)out.cap_tracks || (uint64_t)off + cnt > (uint64_t)out.cap_hits) continue;
        const uint32_t nh = (uint32_t)o.nhits[k];
        const Hit hs = hits[starts[k]];
        const uint64_t key = tl_key(nh, hs.id);
        const int32_t* slot = o.hits + (size_t)k * R + (R - (int)nh);
        uint32_t wr = off;
        for (uint32_t base = 0; base < nh; base += 64) {
            const uint64_t m = own_mask[(size_t)k * 4 + base / 64];  // the entries k owns
            if ((m >> lane) & 1ull)
                out.hit_ids[wr + (uint32_t)__popcll(m & below)] = (int32_t)hits[slot[base + lane]].id;
            wr += (uint32_t)__popcll(m);
        }
        if (lane < 5) out.state[(size_t)t * 5 + lane] = o.state[(size_t)k * 5 + lane];
        else if (lane < 20) out.cov[(size_t)t * 15 + (lane - 5)] = o.cov[(size_t)k * 15 + (lane - 5)];
        else if (lane == 20) out.hit_offset[t] = (int32_t)off;
        else if (lane == 21) out.n_hits[t] = (int32_t)cnt;
        else if (lane == 22) out.start_id[t] = (int32_t)hs.id;
        else if (lane == 23) out.sector[t] = (int32_t)(hs.rs / (uint32_t)R);
        else if (lane == 24) {
            const int rr = o.row_ref[k];
            out.row_ref[t] = rr;
            out.x_ref[t] = g.row_x[rr];
        } else if (lane == 25) out.chi2[t] = o.chi2[k];
        else if (lane == 26) out.ndf[t] = o.ndf[k];
    }
}

// 256 threads: thread l adds up tally line l.
__global__ __launch_bounds__(kTallyLines) void k_finish(const uint32_t* __restrict__ c, int32_t* __restrict__ out) {
    __shared__ uint32_t part[kTallyLines / 64][4];
    const int l = threadIdx.x, w = l >> 6;
    const uint32_t* line = c + C_N_COUNTERS + l * kTallyStride;
    const uint32_t v0 = wave_sum(line[C_N_PAIRS]), v1 = wave_sum(line[C_N_PAIRS_KEPT]);
    const uint32_t v2 = wave_sum(line[C_N_LINKS_RAW]), v3 = wave_sum(line[C_N_LINKS_CLEAN]);
    if ((l & 63) == 0) {
        part[w][0] = v0;
        part[w][1] = v1;
        part[w][2] = v2;
        part[w][3] = v3;
    }
    __syncthreads();
    if (l != 0) return;
    uint32_t t[4] = {0, 0, 0, 0};
    for (int k = 0; k < kTallyLines / 64; ++k)
        for (int j = 0; j < 4; ++j) t[j] += part[k][j];
    out[TPC_CNT_TRACKS] = (int32_t)c[C_N_TRACKS];
    out[TPC_CNT_TRACK_HITS] = (int32_t)c[C_N_TRACK_HITS];
    out[TPC_CNT_TRACKLETS] = (int32_t)c[C_N_STARTS];
    out[TPC_CNT_VALID_TRACKLETS] = (int32_t)c[C_N_VALID_TL];
    out[TPC_CNT_FIT_FAILURES] = (int32_t)c[C_N_FAIL];
    out[TPC_CNT_LINKS_RAW] = (int32_t)(c[C_N_LINKS_RAW] + t[2]);
    out[TPC_CNT_LINKS_CLEAN] = (int32_t)(c[C_N_LINKS_CLEAN] + t[3]);
    out[TPC_CNT_VALID_CLUSTERS] = (int32_t)c[C_N_VALID_CLU];
    out[TPC_CNT_PAIRS] = (int32_t)(c[C_N_PAIRS] + t[0]);
    out[TPC_CNT_PAIRS_KEPT] = (int32_t)(c[C_N_PAIRS_KEPT] + t[1]);
    out[TPC_CNT_NB_OVERFLOW] = (int32_t)c[C_NB_OVF];
}

inline unsigned sel_blocks(int64_t t_max) {
    int64_t b = (t_max + kBlock / 64 - 1) / (kBlock / 64);  // one wave per tracklet
    if (b > 8192) b = 8192;
    b = (b + kXcd - 1) / kXcd * kXcd;  // whole rounds over the XCDs
    return (unsigned)(b < kXcd ? kXcd : b);
}

}  // namespace

size_t select_sort_entries() { return (size_t)256 * kSortBlocks + 1; }

void select_keys(const Hit* hits, const uint32_t* starts, const TrackletOut& o, int R, uint32_t* counters,
                 uint64_t* hit_key, uint32_t* sort_cnt, uint32_t* order, void* scan_scratch, int64_t t_max,
                 hipStream_t s) {
    k_len_count<<<kSortBlocks, kBlock, 0, s>>>(o, counters, sort_cnt);
    scan_u32(sort_cnt, sort_cnt, (int64_t)256 * kSortBlocks, nullptr, nullptr, scan_scratch, s);
    k_len_scatter<<<kSortBlocks, kBlock, 0, s>>>(o, counters, sort_cnt, order);
    // About one wave per 96 tracklet slots: with roughly a fifth of the slots holding a
    // valid tracklet, each wave walks some 18 neighbours in the length order (fewer waves
    // with more work each, or more with less, were both slower on the pp and Pb-Pb frames);
    // at least 8 workgroups per CU so that small inputs still fill the chip.
    int64_t kb = t_max / 384;
    if (kb > 65536) kb = 65536;
    if (kb < 2048) kb = 2048;
    k_keys<<<(unsigned)(kb > 0 ? kb : 1), kBlock, 0, s>>>(hits, starts, order, o, R, counters, hit_key);
}

void select_own(const Hit* hits, const uint32_t* starts, const uint32_t* proc, const TrackletOut& o, int R,
                const uint32_t* counters, const uint64_t* hit_key, int n_min_trk, uint32_t* own_cnt,
                uint32_t* trk_flag, uint64_t* own_mask, int64_t t_max, hipStream_t s) {
    k_own<<<sel_blocks(t_max), kBlock, 0, s>>>(hits, starts, proc, o, R, counters, hit_key, n_min_trk, own_cnt,
                                               trk_flag, own_mask);
}

void select_write(const Hit* hits, const uint32_t* starts, const uint32_t* proc, const TrackletOut& o,
                  const GridDesc& g, const uint32_t* counters, const uint64_t* hit_key, const uint32_t* own_cnt,
                  const uint32_t* trk_flag, const uint32_t* hit_off, const uint32_t* trk_idx,
                  const tpc_tracks_t& out, const uint64_t* own_mask, int64_t t_max, hipStream_t s) {
    (void)trk_flag;
    k_write<<<sel_blocks(t_max), kBlock, 0, s>>>(hits, starts, proc, o, g, counters, hit_key, own_cnt, hit_off,
                                                 trk_idx, out, own_mask);
}

void finish_counts(const uint32_t* counters, int32_t* out_counts, hipStream_t s) {
    k_finish<<<1, kTallyLines, 0, s>>>(counters, out_counts);
}

}  // namespace tpc
