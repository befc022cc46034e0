// Cluster attachment, adjacency, protection and the two removal strategies
// (Sec. 4, cluster removal), for the tracks of one event or time frame.
//
// A cluster is attached to its track, and adjacent to a track when it lies on a
// pad row the track spans (innermost to outermost hit row) within a tube of
// radius `tube` around it, measured on the row plane from the track's helix
// propagated to that row.  Ambiguities go to the higher-momentum track (smaller
// |q/pT|, then the smaller track index): the 64-bit key (~bits(|q/pT|), ~k) is
// maximised per cluster.  The assigned track protects the cluster when its pT
// exceeds pt_min and its local inclination on the cluster's row is below
// phi_max; strategy A removes unprotected clusters that are attached or
// adjacent to a track, strategy B every unprotected cluster.  Tracks are not
// merged into legs, so every track counts as a primary leg.
//
// One wave per track, one lane per spanned row (rows of a track are
// independent: each lane propagates the track's reference state to its row in
// closed form).  One walk marks adjacency and attachment and raises the cluster
// keys, which carry the candidate track's protection decision in their lowest
// bit; a per-cluster pass assembles the flags.
#include "tpc_device.h"
#include "tpc_internal.h"

namespace tpc {

namespace {

struct FlagArgs {
    const uint8_t* row;  // cluster rows (the grid's hit records give y, z, id)
    int64_t n;              // clusters
    const int32_t* counts;  // tracks: counts[TPC_CNT_TRACKS] (device)
    int32_t cap_tracks, cap_hits;
    const int32_t *off, *nh, *ids, *sector;
    const float *x_ref, *state;
    double kq, s_max, t2;
    float qpt_max;
    double sin_phi_max;
};

// The track's helix at x (sector-local helix model): y, z, sin phi; false when
// |sin phi| would reach s_max on the way.
__device__ inline bool helix_at(const FlagArgs& a, int32_t k, double x, double& yt, double& zt, double& st) {
    return helix_at_state(a.state + 5 * k, (double)a.x_ref[k], x, a.kq, a.s_max, yt, zt, st);
}

// Key of track k for a cluster on a row where the track's protection decision is
// `prot`: (~bits(|q/pT|), ~k) orders the tracks (higher momentum, then smaller
// index); the decision rides in the lowest bit, which never decides between two
// tracks (their upper 63 bits differ), so the maximum over a cluster's
// candidates carries its assigned track's decision with it.
__device__ inline uint64_t track_key(const FlagArgs& a, int32_t k, bool prot) {
    const float q = fabsf(a.state[5 * k + 4]);
    return ((uint64_t)(0xFFFFFFFFu - __float_as_uint(q)) << 32) |
           ((uint64_t)(0x7FFFFFFFu - (uint32_t)k) << 1) | (prot ? 1ull : 0ull);
}

__global__ __launch_bounds__(kBlock) void k_fl_tube(GridDesc g, FlagArgs a, const Hit* __restrict__ hits,
                                                    const uint32_t* __restrict__ bin_off, uint64_t* __restrict__ key,
                                                    uint8_t* __restrict__ att, uint8_t* __restrict__ adj) {
    const int lane = threadIdx.x & 63;
    const int32_t cnt = a.counts[TPC_CNT_TRACKS];
    const int32_t n_trk = cnt < a.cap_tracks ? cnt : a.cap_tracks;
    const int32_t wpb = (int32_t)(blockDim.x >> 6);
    for (int32_t k = (int32_t)blockIdx.x * wpb + (int32_t)(threadIdx.x >> 6); k < n_trk;
         k += (int32_t)gridDim.x * wpb) {  // wave-uniform
        // entries a tracking call could not write (hits beyond cap_hits) may hold anything:
        // every index is checked before it is used
        const int32_t nh = a.nh[k], s = a.sector[k], off = a.off[k];
        if (nh <= 0 || off < 0 || (int64_t)off + nh > (int64_t)a.cap_hits || s < 0 || s >= g.S) continue;
        const int32_t* ids = a.ids + off;
        const int32_t c0 = ids[0], c1 = ids[nh - 1];
        if ((uint64_t)(uint32_t)c0 >= (uint64_t)a.n || (uint64_t)(uint32_t)c1 >= (uint64_t)a.n) continue;
        const int r0 = a.row[c0], r1 = a.row[c1];
        if (r1 >= g.R || r0 > r1) continue;
        const bool fast = fabsf(a.state[5 * k + 4]) < a.qpt_max;  // pT > pt_min
        const uint64_t k_no = track_key(a, k, false), k_yes = track_key(a, k, true);
        // the rows the track spans
        for (int r = r0 + lane; r <= r1; r += 64) {
            double yt, zt, st;
            if (!helix_at(a, k, (double)g.row_x[r], yt, zt, st)) continue;
            const double rad = sqrt(a.t2);
            const BinRange br = bin_range(g, s, r, yt - rad, yt + rad, zt - rad, zt + rad);
            if (br.empty) continue;
            const uint64_t tk = (fast && fabs(st) < a.sin_phi_max) ? k_yes : k_no;
            for (int iz = br.iz0; iz <= br.iz1; ++iz) {
                const uint32_t e = bin_off[br.base + iz * br.ny + br.iy1 + 1];
                for (uint32_t j = bin_off[br.base + iz * br.ny + br.iy0]; j < e; ++j) {
                    const Hit h = hits[j];
                    const double dy = (double)h.y - yt, dz = (double)h.z - zt;
                    if (!(dy * dy + dz * dz <= a.t2)) continue;
                    adj[h.id] = 1;
                    atomicMax((unsigned long long*)&key[h.id], (unsigned long long)tk);
                }
            }
        }
        // the track's own clusters, inside the tube or not (decision on the cluster's row)
        for (int i = lane; i < nh; i += 64) {
            const int32_t c = ids[i];
            if ((uint64_t)(uint32_t)c >= (uint64_t)a.n) continue;
            double yt, zt, st;
            const bool ok = a.row[c] < g.R && helix_at(a, k, (double)g.row_x[a.row[c]], yt, zt, st);
            att[c] = 1;
            atomicMax((unsigned long long*)&key[c],
                      (unsigned long long)((ok && fast && fabs(st) < a.sin_phi_max) ? k_yes : k_no));
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_fl_final(int64_t n, const uint64_t* __restrict__ key,
                                                     const uint8_t* __restrict__ att, const uint8_t* __restrict__ adj,
                                                     uint8_t* __restrict__ flags) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    const uint64_t kk = key[c];
    uint8_t f = (att[c] ? TPC_FLAG_ATTACHED : 0) | (adj[c] ? TPC_FLAG_ADJACENT : 0);
    if (kk & 1ull) f |= TPC_FLAG_PROTECTED;
    else f |= TPC_FLAG_REMOVE_B | (kk ? TPC_FLAG_REMOVE_A : 0);
    flags[c] = f;
}

}  // namespace

void cluster_flags(const GridDesc& g, const KParams& kp, const tpc_clusters_t& cl, const Hit* hits,
                   const uint32_t* bin_off, const tpc_tracks_t& trk, const tpc_flag_params_t& fp, uint64_t* key,
                   uint8_t* att, uint8_t* adj, uint8_t* flags, hipStream_t s) {
    const int64_t n = cl.n;
    if (n <= 0) return;
    fill_u64(key, 0ull, n, s);
    fill_u32((uint32_t*)att, 0u, (n + 3) / 4, s);
    fill_u32((uint32_t*)adj, 0u, (n + 3) / 4, s);
    FlagArgs a;
    a.row = cl.row;
    a.n = n;
    a.counts = trk.counts;
    a.cap_tracks = trk.cap_tracks;
    a.cap_hits = trk.cap_hits;
    a.off = trk.hit_offset;
    a.nh = trk.n_hits;
    a.ids = trk.hit_ids;
    a.sector = trk.sector;
    a.x_ref = trk.x_ref;
    a.state = trk.state;
    a.kq = kp.kq;
    a.s_max = kp.s_max;
    a.t2 = fp.tube_cm * fp.tube_cm;
    a.qpt_max = (float)(1.0 / fp.pt_min);
    a.sin_phi_max = sin(fp.phi_max_deg * (3.14159265358979323846 / 180.0));
    if (trk.cap_tracks > 0) {
        // one wave per track index: a wave walking several tracks would wait on its atomics
        // before each next track's loads (vector memory operations retire in order)
        const int64_t nb = ((int64_t)trk.cap_tracks + kBlock / 64 - 1) / (kBlock / 64);
        k_fl_tube<<<(unsigned)nb, kBlock, 0, s>>>(g, a, hits, bin_off, key, att, adj);
    }
    k_fl_final<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(n, key, att, adj, flags);
}

}  // namespace tpc
