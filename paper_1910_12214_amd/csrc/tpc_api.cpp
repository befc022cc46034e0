// C-ABI entry points: validation, scratch management, geometry tables and the
// enqueue order of the track-finding chain.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <queue>
#include <string>
#include <vector>

#include "tpc_internal.h"

namespace tpc {

int fail(tpc_ctx_t* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

void* buf(tpc_ctx_t* c, const char* name, size_t bytes) {
    if (bytes == 0) bytes = 16;
    DevBuf& b = c->bufs[name];
    if (b.bytes >= bytes) return b.p;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    c->geo_key.clear();
    ++c->buf_gen;
    // grow with headroom so that slightly larger inputs do not reallocate
    size_t want = bytes + bytes / 8;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        b.p = nullptr;
        c->err = std::string("hipMalloc failed for scratch buffer ") + name + " (" + std::to_string(want) + " bytes)";
        return nullptr;
    }
    b.bytes = want;
    return b.p;
}

// Length in bits of the optimal prefix (Huffman) code of symbols with these counts: the
// sum of the weights of the merged nodes when the two lightest subtrees are merged until
// one is left (one present symbol: one bit each).
uint64_t huffman_bits(const uint32_t* count, int n_sym) {
    std::priority_queue<uint64_t, std::vector<uint64_t>, std::greater<uint64_t>> q;
    for (int i = 0; i < n_sym; ++i)
        if (count[i]) q.push(count[i]);
    if (q.empty()) return 0;
    if (q.size() == 1) return q.top();
    uint64_t bits = 0;
    while (q.size() > 1) {
        const uint64_t a = q.top();
        q.pop();
        const uint64_t b = q.top();
        q.pop();
        bits += a + b;
        q.push(a + b);
    }
    return bits;
}

void* buf_peek(tpc_ctx_t* c, const char* name, size_t* bytes) {
    auto it = c->bufs.find(name);
    if (it == c->bufs.end()) {
        if (bytes) *bytes = 0;
        return nullptr;
    }
    if (bytes) *bytes = it->second.bytes;
    return it->second.p;
}

}  // namespace tpc

using namespace tpc;

namespace {

struct Prepared {
    GridDesc g{};
    KParams kp{};
    int64_t n = 0;
    int64_t t_max = 0;
    uint32_t n_bins = 0;
    int slab_bins = 1;  // z bins per slab of the tracklet processing order
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int check_params(tpc_ctx_t* c, const tpc_params_t* p) {
    if (!p) return fail(c, TPC_ERR_ARG, "params is NULL");
    if (!finite_pos(p->win_y) || !finite_pos(p->win_z)) return fail(c, TPC_ERR_ARG, "window slopes must be > 0");
    if (!finite_pos(p->nb_chi2_max) || !finite_pos(p->fol_chi2_max)) return fail(c, TPC_ERR_ARG, "cuts must be > 0");
    if (!finite_pos(p->sigma_y) || !finite_pos(p->sigma_z)) return fail(c, TPC_ERR_ARG, "cluster errors must be > 0");
    if (!(p->s_max > 0.0 && p->s_max < 1.0)) return fail(c, TPC_ERR_ARG, "s_max must be in (0, 1)");
    if (!std::isfinite(p->edge_margin)) return fail(c, TPC_ERR_ARG, "edge_margin must be finite");
    if (p->l_min_chain < 2 || p->l_min_chain > 255) return fail(c, TPC_ERR_ARG, "l_min_chain must be in [2, 255]");
    if (p->n_miss_max < 0 || p->n_min_tracklet < 1 || p->n_min_track < 1)
        return fail(c, TPC_ERR_ARG, "n_miss_max >= 0, n_min_tracklet >= 1, n_min_track >= 1 required");
    if (!finite_pos(p->c0_sinphi) || !finite_pos(p->c0_dzds) || !finite_pos(p->c0_qpt))
        return fail(c, TPC_ERR_ARG, "initial variances must be > 0");
    if (!(p->bin_y > 0.f) || !(p->bin_z > 0.f) || !std::isfinite(p->bin_y) || !std::isfinite(p->bin_z))
        return fail(c, TPC_ERR_ARG, "bin sizes must be > 0");
    if (p->mlp && !std::isfinite(p->mlp_tau_logit)) return fail(c, TPC_ERR_ARG, "mlp_tau_logit must be finite");
    return TPC_OK;
}

int check_geometry(tpc_ctx_t* c, const tpc_geometry_t* g) {
    if (!g || !g->row_x) return fail(c, TPC_ERR_ARG, "geometry or row_x is NULL");
    if (g->n_rows < 3 || g->n_rows > kMaxRows) return fail(c, TPC_ERR_ARG, "n_rows must be in [3, 255]");
    if (g->n_sectors < 1 || g->n_sectors > 256) return fail(c, TPC_ERR_ARG, "n_sectors must be in [1, 256]");
    for (int r = 0; r < g->n_rows; ++r) {
        if (!std::isfinite(g->row_x[r]) || !(g->row_x[r] > 0.f)) return fail(c, TPC_ERR_ARG, "row_x must be finite and > 0");
        if (r && !(g->row_x[r] > g->row_x[r - 1])) return fail(c, TPC_ERR_ARG, "row_x must increase strictly");
    }
    if (!std::isfinite(g->tan_half) || !(g->tan_half > 0.f)) return fail(c, TPC_ERR_ARG, "tan_half must be > 0");
    if (!std::isfinite(g->z_min) || !std::isfinite(g->z_max) || !(g->z_max > g->z_min))
        return fail(c, TPC_ERR_ARG, "z range must be finite with z_max > z_min");
    return TPC_OK;
}

int check_clusters(tpc_ctx_t* c, const tpc_clusters_t* cl) {
    if (!cl) return fail(c, TPC_ERR_ARG, "clusters is NULL");
    if (cl->n < 0 || cl->n >= (int64_t(1) << 31)) return fail(c, TPC_ERR_ARG, "cluster count must be in [0, 2^31)");
    if (cl->n > 0 && (!cl->y || !cl->z || !cl->row || !cl->sector)) return fail(c, TPC_ERR_ARG, "cluster arrays are NULL");
    return TPC_OK;
}

int check_out(tpc_ctx_t* c, const tpc_tracks_t* o) {
    if (!o || !o->counts) return fail(c, TPC_ERR_ARG, "output or counts is NULL");
    if (o->cap_tracks < 0 || o->cap_hits < 0) return fail(c, TPC_ERR_ARG, "capacities must be >= 0");
    if (o->cap_tracks > 0 && (!o->hit_offset || !o->n_hits || !o->start_id || !o->sector || !o->row_ref || !o->x_ref ||
                              !o->state || !o->cov || !o->chi2 || !o->ndf))
        return fail(c, TPC_ERR_ARG, "track output arrays are NULL");
    if (o->cap_hits > 0 && !o->hit_ids) return fail(c, TPC_ERR_ARG, "hit_ids is NULL");
    return TPC_OK;
}

// Geometry tables on the device (cached while geometry and bin sizes do not change).
int prepare(tpc_ctx_t* c, const tpc_clusters_t* cl, const tpc_geometry_t* geo, double bz, const tpc_params_t* p,
            float bin_y, float bin_z, Prepared* pr) {
    const int R = geo->n_rows, S = geo->n_sectors;
    std::vector<float> ymin(R);
    std::vector<int32_t> ny(R);
    for (int r = 0; r < R; ++r) {
        const float hw = geo->row_x[r] * geo->tan_half;  // fp32 product
        ymin[r] = -hw;
        double v = std::ceil((2.0 * (double)hw) / (double)bin_y);
        ny[r] = v < 1 ? 1 : (v > 65535 ? 65535 : (int32_t)v);
    }
    double vz = std::ceil(((double)geo->z_max - (double)geo->z_min) / (double)bin_z);
    const int32_t nz = vz < 1 ? 1 : (vz > 1048576 ? 1048576 : (int32_t)vz);
    std::vector<uint32_t> base(S * R + 1);
    uint64_t nb = 0;
    for (int s = 0; s < S; ++s)
        for (int r = 0; r < R; ++r) {
            base[s * R + r] = (uint32_t)nb;
            nb += (uint64_t)ny[r] * (uint64_t)nz;
        }
    if (nb >= (uint64_t(1) << 31)) return fail(c, TPC_ERR_ARG, "grid too fine: more than 2^31 bins (raise bin_y/bin_z)");
    base[S * R] = (uint32_t)nb;
    // upload (small, synchronous) only when the tables change
    float* d_rowx = (float*)buf(c, "row_x", sizeof(float) * R);
    float* d_ymin = (float*)buf(c, "row_ymin", sizeof(float) * R);
    int32_t* d_ny = (int32_t*)buf(c, "row_ny", sizeof(int32_t) * R);
    uint32_t* d_base = (uint32_t*)buf(c, "bin_base", sizeof(uint32_t) * (S * R + 1));
    if (!d_rowx || !d_ymin || !d_ny || !d_base) return TPC_ERR_HIP;
    std::string key((const char*)geo->row_x, sizeof(float) * R);
    key.append((const char*)ymin.data(), sizeof(float) * R);
    key.append((const char*)ny.data(), sizeof(int32_t) * R);
    key.append((const char*)base.data(), sizeof(uint32_t) * (S * R + 1));
    if (key != c->geo_key) {
        // earlier calls on any stream may still read the old tables
        TPC_HIP(c, hipDeviceSynchronize());
        TPC_HIP(c, hipMemcpy(d_rowx, geo->row_x, sizeof(float) * R, hipMemcpyHostToDevice));
        TPC_HIP(c, hipMemcpy(d_ymin, ymin.data(), sizeof(float) * R, hipMemcpyHostToDevice));
        TPC_HIP(c, hipMemcpy(d_ny, ny.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice));
        TPC_HIP(c, hipMemcpy(d_base, base.data(), sizeof(uint32_t) * (S * R + 1), hipMemcpyHostToDevice));
        c->geo_key.swap(key);
    }
    GridDesc& g = pr->g;
    g.R = R;
    g.S = S;
    g.nz = nz;
    g.ny_max = *std::max_element(ny.begin(), ny.end());
    g.z_min = geo->z_min;
    g.inv_by = 1.0f / bin_y;
    g.inv_bz = 1.0f / bin_z;
    g.n_bins = (uint32_t)nb;
    g.row_x = d_rowx;
    g.row_ymin = d_ymin;
    g.row_ny = d_ny;
    g.bin_base = d_base;
    KParams& k = pr->kp;
    k.win_y = p->win_y;
    k.win_z = p->win_z;
    k.nb_cut = p->nb_chi2_max;
    k.fol_cut = p->fol_chi2_max;
    k.vy = p->sigma_y * p->sigma_y;
    k.vz = p->sigma_z * p->sigma_z;
    k.vy15 = 1.5 * p->sigma_y * p->sigma_y;
    k.vz15 = 1.5 * p->sigma_z * p->sigma_z;
    k.ivy15 = 1.0 / k.vy15;
    k.ivz15 = 1.0 / k.vz15;
    k.s_max = p->s_max;
    k.edge = p->edge_margin;
    k.tan_half = (double)geo->tan_half;
    k.kq = -0.00299792458 * bz;
    k.c0s = p->c0_sinphi;
    k.c0t = p->c0_dzds;
    k.c0q = p->c0_qpt;
    k.l_min = p->l_min_chain;
    k.n_miss = p->n_miss_max;
    k.n_min_tl = p->n_min_tracklet;
    k.n_min_trk = p->n_min_track;
    k.tau = p->mlp_tau_logit;
    pr->n = cl->n;
    pr->n_bins = (uint32_t)nb;
    pr->t_max = cl->n / p->l_min_chain + 1;
    pr->slab_bins = std::max(1, (int)std::lround(kSlabCm / bin_z));
    return TPC_OK;
}

struct Scratch {
    uint32_t *counters, *bin_of, *pos_of, *sorted_id, *bin_cnt, *slot_of, *bin_off, *row_off, *block_cnt, *starts;
    uint32_t *rs_hist = nullptr, *rs_hoff = nullptr, *rs_piece = nullptr;  // row-sector grid path
    Hit *rs_recA = nullptr, *rs_recB = nullptr;
    uint32_t *tl_slot, *proc, *slab_cnt, *nb_ovf;
    void* seeds;
    void* nb_cand = nullptr;  // fused neighbour finding with a scorer only
    uint32_t *nb_nund = nullptr, *nb_wrec = nullptr;
    uint32_t *sort_cnt, *sel_order;
    uint32_t *own_cnt, *trk_flag, *hit_off, *trk_idx;
    uint64_t* own_mask;
    Hit* hits;
    TlHit* tl_hits;
    int32_t *up, *dn, *upc, *dnc;
    uint8_t* start_flag;
    uint64_t* hit_key;
    void* scan;
    TrackletOut tl;
};

int alloc_scratch(tpc_ctx_t* c, const Prepared& pr, Scratch* s, bool mlp) {
    const int64_t n = pr.n > 0 ? pr.n : 1, T = pr.t_max, NB = pr.n_bins, R = pr.g.R, S = pr.g.S;
    const int64_t nblk = (n + kBlock - 1) / kBlock + 1;
    int64_t scan_n = n;
    if (NB > scan_n) scan_n = NB;
    if (T > scan_n) scan_n = T;
    if (nblk > scan_n) scan_n = nblk;
    if ((int64_t)select_sort_entries() > scan_n) scan_n = (int64_t)select_sort_entries();
    const bool rs_path = grid_rs_fits(pr.g, pr.n);
    const int64_t rs_entries = rs_path ? (int64_t)grid_rs_hist_entries(pr.g) : 0;
    if (rs_entries > scan_n) scan_n = rs_entries;
#define B(field, name, bytes)                                   \
    s->field = (decltype(s->field))buf(c, name, (size_t)(bytes)); \
    if (!s->field) return TPC_ERR_HIP;
    B(counters, "counters", sizeof(uint32_t) * kCounterWords);
    B(pos_of, "pos_of", 4 * n);
    if (!rs_path) {  // the bin-counting grid path only
        B(bin_of, "bin_of", 4 * n);
        B(sorted_id, "sorted_id", 4 * n);
        B(slot_of, "slot_of", 4 * n);
    } else {
        s->bin_of = s->sorted_id = s->slot_of = nullptr;
    }
    B(hits, "hits", sizeof(Hit) * n);
    B(tl_hits, "tl_hits_rec", sizeof(TlHit) * n);
    B(up, "up", 4 * n);
    B(dn, "dn", 4 * n);
    B(upc, "upc", 4 * n);
    B(dnc, "dnc", 4 * n);
    B(start_flag, "start_flag", 4 * ((n + 3) / 4));
    B(hit_key, "hit_key", 8 * n);
    if (!rs_path) {
        B(bin_cnt, "bin_cnt", 4 * (NB + 1));
    } else {
        s->bin_cnt = nullptr;
    }
    if (rs_path) {
        B(rs_hist, "rs_hist", 4 * rs_entries);
        B(rs_hoff, "rs_hoff", 4 * rs_entries);
        B(rs_piece, "rs_piece_off", 4 * (int64_t)grid_rs_piece_entries(pr.g));
        B(rs_recA, "rs_rec_a", sizeof(Hit) * n);
        B(rs_recB, "rs_rec_b", sizeof(Hit) * n);
    }
    B(bin_off, "bin_off", 4 * (NB + 1));
    B(row_off, "row_off", 4 * (S * R + 1));
    B(block_cnt, "block_cnt", 4 * nblk);
    B(starts, "starts", 4 * T);
    B(tl_slot, "tl_slot", 4 * T);
    B(slab_cnt, "slab_cnt", 4 * ((int64_t)S * slab_count(pr.g, pr.slab_bins) * R + 1));
    B(proc, "proc", 4 * T);
    B(seeds, "tl_seeds", seed_bytes() * T);
    B(sort_cnt, "sort_cnt", 4 * select_sort_entries());
    B(sel_order, "sel_order", 4 * T);
    B(nb_ovf, "nb_ovf", 4 * nb_overflow_entries(n));
    if (mlp) {
        B(nb_cand, "nb_cand", 16 * nb_cand_entries(n));
        B(nb_nund, "nb_nund", 4 * n);
        B(nb_wrec, "nb_wrec", 4 * nb_overflow_entries(n));
    }
    B(own_cnt, "own_cnt", 4 * T);
    B(own_mask, "own_mask", 32 * T);
    B(trk_flag, "trk_flag", 4 * T);
    B(hit_off, "hit_off", 4 * T);
    B(trk_idx, "trk_idx", 4 * T);
    B(scan, "scan", scan_scratch_bytes(scan_n));
    B(tl.nhits, "tl_nhits", 4 * T);
    B(tl.hits, "tl_hits", 4 * T * R);
    B(tl.state, "tl_state", 4 * 5 * T);
    B(tl.cov, "tl_cov", 4 * 15 * T);
    B(tl.chi2, "tl_chi2", 4 * T);
    B(tl.ndf, "tl_ndf", 4 * T);
    B(tl.row_ref, "tl_row_ref", 4 * T);
    B(tl.flags, "tl_flags", 4 * T);
#undef B
    return TPC_OK;
}

// The whole chain on one stream.  No host synchronisation inside: every count
// that sizes later work stays in device memory.
// Stage timing events (only while profiling is enabled).
struct Marks {
    tpc_ctx_t* c;
    hipStream_t st;
    std::vector<hipEvent_t> ev;
    void mark() {
        if (!c->prof_on) return;
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        (void)hipEventRecord(e, st);
        ev.push_back(e);
    }
    void done() {
        if (c->prof_on && ev.size() == TPC_N_PROF + 1) c->prof_events.push_back(ev);
        else
            for (auto e : ev) (void)hipEventDestroy(e);
    }
};

// a1: counting sort into the row grids (counters reset first).
void enqueue_grid(const tpc_clusters_t& cl, const Prepared& pr, const Scratch& s, hipStream_t st) {
    const int64_t n = pr.n, NB = pr.n_bins;
    const GridDesc& g = pr.g;
    fill_u32(s.counters, 0u, kCounterWords, st);
    fill_u32((uint32_t*)s.start_flag, 0u, (n + 3) / 4, st);
    if (grid_rs_fits(g, n)) {
        grid_build_rs(cl, g, s.rs_hist, s.rs_hoff, s.rs_piece, s.scan, s.rs_recA, s.rs_recB, s.bin_off, s.hits, s.pos_of,
                      s.row_off, s.counters, st);
        return;
    }
    fill_u32(s.bin_cnt, 0u, NB, st);
    grid_count(cl, g, s.bin_of, s.bin_cnt, s.slot_of, s.pos_of, st);
    scan_u32(s.bin_cnt, s.bin_off, NB, nullptr, s.bin_off + NB, s.scan, st);
    grid_scatter(cl, s.bin_of, s.slot_of, s.bin_off, s.sorted_id, st);
    grid_finalize(cl, g, s.bin_of, s.bin_off, s.sorted_id, s.hits, s.pos_of, s.row_off, s.counters, st);
}

void enqueue_chain(tpc_ctx_t* c, const tpc_clusters_t& cl, const Prepared& pr, const Scratch& s,
                   const tpc_tracks_t& out, const float* mlp_q, int tl_blocks, int chunk, int waves, hipStream_t st) {
    const int64_t n = pr.n, T = pr.t_max;
    const GridDesc& g = pr.g;
    Marks mk{c, st, {}};
    mk.mark();
    enqueue_grid(cl, pr, s, st);
    mk.mark();
    // a2 neighbours (a3: with the learned scorer fused), a4/a5 cleaning and starts
    if (mlp_q)
        neighbours_mlp(g, pr.kp, s.hits, s.bin_off, n, s.counters, mlp_q, s.up, s.dn, s.nb_ovf, s.nb_cand, s.nb_nund,
                       s.nb_wrec, st, c->aux_stream, c->ev_fork, c->ev_join);
    else
        find_neighbours(g, pr.kp, s.hits, s.bin_off, s.row_off, n, s.counters, s.up, s.dn, nullptr, s.counters, st);
    mk.mark();
    clean_and_flag(pr.kp, s.hits, n, s.counters, s.up, s.dn, s.upc, s.dnc, s.tl_hits, s.start_flag, s.counters,
                   st);
    compact_starts(s.start_flag, s.pos_of, n, s.starts, s.block_cnt, s.scan, s.counters + C_N_STARTS, st);
    order_starts(g, s.hits, s.starts, T, s.counters, pr.slab_bins, s.slab_cnt, s.tl_slot, s.proc, s.scan, st);
    mk.mark();
    // a6 tracklets
    build_tracklets(g, pr.kp, s.hits, s.tl_hits, s.bin_off, s.row_off, s.upc, s.starts, s.proc, s.seeds, s.counters,
                    s.tl, T, tl_blocks, chunk, waves, st);
    mk.mark();
    // a7 selection
    fill_u64(s.hit_key, 0ull, n, st);
    select_keys(s.hits, s.starts, s.tl, g.R, s.counters, s.hit_key, s.sort_cnt, s.sel_order, s.scan, T, st);
    select_own(s.hits, s.starts, s.proc, s.tl, g.R, s.counters, s.hit_key, pr.kp.n_min_trk, s.own_cnt, s.trk_flag,
               s.own_mask, T, st);
    scan_u32(s.own_cnt, s.hit_off, T, s.counters + C_N_STARTS, s.counters + C_N_TRACK_HITS, s.scan, st);
    scan_u32(s.trk_flag, s.trk_idx, T, s.counters + C_N_STARTS, s.counters + C_N_TRACKS, s.scan, st);
    select_write(s.hits, s.starts, s.proc, s.tl, g, s.counters, s.hit_key, s.own_cnt, s.trk_flag, s.hit_off,
                 s.trk_idx, out, s.own_mask, T, st);
    finish_counts(s.counters, out.counts, st);
    mk.mark();
    mk.done();
}

int capacity_check(tpc_ctx_t* c, const tpc_tracks_t* out, hipStream_t st) {
    TPC_HIP(c, hipStreamSynchronize(st));
    int32_t cnt[TPC_N_COUNTS];
    TPC_HIP(c, hipMemcpy(cnt, out->counts, sizeof cnt, hipMemcpyDeviceToHost));
    if (cnt[TPC_CNT_TRACKS] > out->cap_tracks || cnt[TPC_CNT_TRACK_HITS] > out->cap_hits)
        return fail(c, TPC_ERR_CAPACITY,
                    "outputs too small: need " + std::to_string(cnt[TPC_CNT_TRACKS]) + " tracks and " +
                        std::to_string(cnt[TPC_CNT_TRACK_HITS]) + " hits");
    return TPC_OK;
}

}  // namespace

extern "C" {

void tpc_params_default(tpc_params_t* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->win_y = 2.0;
    p->win_z = 2.0;
    p->nb_chi2_max = 13.8;
    p->fol_chi2_max = 13.8;
    p->sigma_y = 0.06;
    p->sigma_z = 0.1;
    p->s_max = 0.999;
    p->edge_margin = 2.0;
    p->l_min_chain = 3;
    p->n_miss_max = 10;
    p->n_min_tracklet = 10;
    p->n_min_track = 10;
    p->c0_sinphi = 1.0;
    p->c0_dzds = 1.0;
    p->c0_qpt = 100.0;
    p->bin_y = 8.0f;
    p->bin_z = 8.0f;
    p->mlp = nullptr;
    p->mlp_tau_logit = 0.0;
}

int tpc_ctx_create(tpc_ctx_t** out, int device) {
    if (!out) return TPC_ERR_ARG;
    *out = nullptr;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev) return TPC_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return TPC_ERR_HIP;
    tpc_ctx_t* c = new tpc_ctx_t();
    c->device = device;
    noalloc_init(device);  // device address of the allocation-free entry point's fixed scratch
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0) {
        c->n_cu = prop.multiProcessorCount;
        c->arch = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
    }
    // the auxiliary stream (default priority) and its fork/join events; without them the
    // chain simply runs on one stream
    if (hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking) != hipSuccess) c->aux_stream = nullptr;
    if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess) c->ev_fork = nullptr;
    if (hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) c->ev_join = nullptr;
    *out = c;
    return TPC_OK;
}

void tpc_ctx_destroy(tpc_ctx_t* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : c->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    for (auto& kv : c->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    delete c;
}

const char* tpc_last_error(tpc_ctx_t* c) { return c ? c->err.c_str() : "null context"; }

int tpc_track_sectors(tpc_ctx_t* c, const tpc_clusters_t* cl, const tpc_geometry_t* geo, double bz,
                      const tpc_params_t* p, tpc_tracks_t* out, void* stream, int sync_check) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_clusters(c, cl)) || (rc = check_geometry(c, geo)) || (rc = check_params(c, p)) ||
        (rc = check_out(c, out)))
        return rc;
    if (!std::isfinite(bz)) return fail(c, TPC_ERR_ARG, "bz must be finite");
    TPC_HIP(c, hipSetDevice(c->device));
    Prepared pr;
    if ((rc = prepare(c, cl, geo, bz, p, p->bin_y, p->bin_z, &pr))) return rc;
    Scratch s;
    if ((rc = alloc_scratch(c, pr, &s, p->mlp != nullptr))) return rc;
    hipStream_t st = (hipStream_t)stream;
    float* q = nullptr;
    if (p->mlp) {
        q = (float*)buf(c, "mlp_q", sizeof(float) * mlp_q_floats());
        if (!q) return TPC_ERR_HIP;
        mlp_quantize(p->mlp, q, st);
    }
    enqueue_chain(c, *cl, pr, s, *out, q, c->n_cu * 4, 1, 2, st);
    TPC_HIP(c, hipGetLastError());
    c->last_n = pr.n;
    c->last_R = pr.g.R;
    c->last_S = pr.g.S;
    c->last_n_bins = pr.n_bins;
    c->last_n_starts_cap = pr.t_max;
    if (sync_check) return capacity_check(c, out, st);
    return TPC_OK;
}

void tpc_flag_params_default(tpc_flag_params_t* p) {
    if (!p) return;
    p->tube_cm = 1.5;
    p->pt_min = 0.05;
    p->phi_max_deg = 70.0;
}

int tpc_cluster_flags(tpc_ctx_t* c, const tpc_clusters_t* cl, const tpc_geometry_t* geo, double bz,
                      const tpc_params_t* p, const tpc_flag_params_t* fp, const tpc_tracks_t* trk, uint8_t* flags,
                      void* stream) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_clusters(c, cl)) || (rc = check_geometry(c, geo)) || (rc = check_params(c, p))) return rc;
    if (!std::isfinite(bz)) return fail(c, TPC_ERR_ARG, "bz must be finite");
    if (!fp || !(fp->tube_cm > 0.0) || !std::isfinite(fp->tube_cm) || !(fp->pt_min > 0.0) ||
        !std::isfinite(fp->pt_min) || !(fp->phi_max_deg > 0.0) || !(fp->phi_max_deg < 90.0))
        return fail(c, TPC_ERR_ARG, "flag parameters: need tube_cm > 0, pt_min > 0, 0 < phi_max_deg < 90");
    if (!trk || trk->cap_tracks < 0 || trk->cap_hits < 0 || !trk->counts ||
        (trk->cap_tracks > 0 && (!trk->hit_offset || !trk->n_hits || !trk->hit_ids || !trk->sector ||
                                 !trk->x_ref || !trk->state)))
        return fail(c, TPC_ERR_ARG, "tracks: counts and, for cap_tracks > 0, hit_offset, n_hits, hit_ids, "
                                    "sector, x_ref and state are required");
    if (cl->n > 0 && !flags) return fail(c, TPC_ERR_ARG, "flags output is NULL");
    TPC_HIP(c, hipSetDevice(c->device));
    Prepared pr;
    if ((rc = prepare(c, cl, geo, bz, p, p->bin_y, p->bin_z, &pr))) return rc;
    Scratch s;
    if ((rc = alloc_scratch(c, pr, &s, false))) return rc;
    const int64_t n = pr.n > 0 ? pr.n : 1;
    uint64_t* key = (uint64_t*)buf(c, "fl_key", 8 * n);
    uint8_t* att = (uint8_t*)buf(c, "fl_att", 4 * ((n + 3) / 4));
    uint8_t* adj = (uint8_t*)buf(c, "fl_adj", 4 * ((n + 3) / 4));
    if (!key || !att || !adj) return TPC_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    enqueue_grid(*cl, pr, s, st);
    cluster_flags(pr.g, pr.kp, *cl, s.hits, s.bin_off, *trk, *fp, key, att, adj, flags, st);
    TPC_HIP(c, hipGetLastError());
    return TPC_OK;
}

void tpc_compress_params_default(tpc_compress_params_t* p) {
    if (!p) return;
    p->q_y = 0.0075;
    p->q_z = 0.0125;
    p->n_charge = 4;
    p->n_width = 3;
}

void tpc_merge_params_default(tpc_merge_params_t* p) {
    if (!p) return;
    p->rho_max = 600.0;
    p->centre_window = 16.0;
    p->chi2_max = 60.0;
    p->phase_sigmas = 5.0;
    p->phase_floor = 0.1;
    p->max_turns = 5;
    p->sectors_per_side = 18;
    p->max_iter = 50;
    p->pair_queue = 4;
}


}  // extern "C"

namespace {

int check_compress_params(tpc_ctx_t* c, const tpc_compress_params_t* cp) {
    if (!cp || !finite_pos(cp->q_y) || !finite_pos(cp->q_z) || cp->n_charge < 0 || cp->n_charge > 15 ||
        cp->n_width < 0 || cp->n_width > 15)
        return fail(c, TPC_ERR_ARG, "compress params: need q_y, q_z > 0 and n_charge, n_width in [0, 15]");
    return TPC_OK;
}

int check_track_input(tpc_ctx_t* c, const tpc_tracks_t* t) {
    if (!t || t->cap_tracks < 0 || t->cap_hits < 0 || !t->counts ||
        (t->cap_tracks > 0 && (!t->hit_offset || !t->n_hits || !t->sector || !t->row_ref || !t->x_ref || !t->state)) ||
        (t->cap_hits > 0 && !t->hit_ids))
        return fail(c, TPC_ERR_ARG, "tracks: counts and, for cap_tracks > 0, hit_offset, n_hits, sector, row_ref, "
                                    "x_ref, state (hit_ids for cap_hits > 0) are required");
    return TPC_OK;
}

int check_compressed(tpc_ctx_t* c, const tpc_compressed_t* o, int64_t n, int64_t SR, int32_t cap_tracks) {
    if (!o || !o->counts || !o->sym || !o->freq || !o->block_bytes || o->cap_sym < n + SR || o->cap_esc < 0 ||
        o->cap_bytes < 0 || (o->cap_esc > 0 && !o->esc) || (o->cap_bytes > 0 && !o->bytes) || (n > 0 && !o->order) ||
        (cap_tracks > 0 && !o->track_len))
        return fail(c, TPC_ERR_ARG, "compressed output: counts, sym, freq, block_bytes, order (n > 0), track_len "
                                    "(tracks), esc and bytes for nonzero capacities; cap_sym >= n + n_sectors * "
                                    "n_rows");
    return TPC_OK;
}

}  // namespace

extern "C" {

int tpc_compress(tpc_ctx_t* c, const tpc_clusters_t* cl, const tpc_cluster_props_t* props,
                 const tpc_geometry_t* geo, double bz, const tpc_params_t* p, const tpc_compress_params_t* cp,
                 const tpc_tracks_t* trk, tpc_compressed_t* out, void* stream, int sync_check) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_clusters(c, cl)) || (rc = check_geometry(c, geo)) || (rc = check_params(c, p)) ||
        (rc = check_compress_params(c, cp)) || (rc = check_track_input(c, trk)))
        return rc;
    if (!std::isfinite(bz)) return fail(c, TPC_ERR_ARG, "bz must be finite");
    if (cl->n > 0 && (!props || !props->qtot || !props->sigma_y || !props->sigma_z))
        return fail(c, TPC_ERR_ARG, "cluster properties (qtot, sigma_y, sigma_z) are required");
    if ((rc = check_compressed(c, out, cl->n, (int64_t)geo->n_sectors * geo->n_rows, trk->cap_tracks))) return rc;
    TPC_HIP(c, hipSetDevice(c->device));
    Prepared pr;
    if ((rc = prepare(c, cl, geo, bz, p, p->bin_y, p->bin_z, &pr))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = compress_run(c, *cl, *props, pr.g, pr.kp.kq, pr.kp.s_max, *cp, *trk, *out, st))) return rc;
    TPC_HIP(c, hipGetLastError());
    if (!sync_check) return TPC_OK;
    TPC_HIP(c, hipStreamSynchronize(st));
    int64_t cnt[TPC_N_CSTREAMS * TPC_CSC_N + TPC_CST_N];
    TPC_HIP(c, hipMemcpy(cnt, out->counts, sizeof cnt, hipMemcpyDeviceToHost));
    if (cnt[TPC_N_CSTREAMS * TPC_CSC_N + TPC_CST_ATTACHED] + cnt[TPC_N_CSTREAMS * TPC_CSC_N + TPC_CST_UNATTACHED] >
        cl->n)
        return fail(c, TPC_ERR_ARG, "a cluster appears on more than one track: the streams are not valid");
    int64_t bytes = 0;
    for (int s = 0; s < TPC_N_CSTREAMS; ++s) {
        bytes += cnt[s * TPC_CSC_N + TPC_CSC_BYTES];
        if (cnt[s * TPC_CSC_N + TPC_CSC_ESCAPES] > out->cap_esc)
            return fail(c, TPC_ERR_CAPACITY, "escape list too small: stream " + std::to_string(s) + " needs " +
                                                 std::to_string(cnt[s * TPC_CSC_N + TPC_CSC_ESCAPES]));
    }
    if (bytes > out->cap_bytes)
        return fail(c, TPC_ERR_CAPACITY, "coded output too small: needs " + std::to_string(bytes) + " bytes");
    return TPC_OK;
}

int tpc_decompress(tpc_ctx_t* c, const tpc_compressed_t* in, const tpc_geometry_t* geo, double bz,
                   const tpc_params_t* p, const tpc_compress_params_t* cp, const tpc_tracks_t* trk, uint16_t* syms,
                   uint8_t* sector, uint8_t* row, int32_t* yq, int32_t* zq, uint16_t* qtot, uint8_t* sigma_y,
                   uint8_t* sigma_z, void* stream) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_geometry(c, geo)) || (rc = check_params(c, p)) || (rc = check_compress_params(c, cp)) ||
        (rc = check_track_input(c, trk)))
        return rc;
    if (!std::isfinite(bz)) return fail(c, TPC_ERR_ARG, "bz must be finite");
    if (!in || !in->counts || !in->sym || !in->freq || !in->block_bytes ||
        in->cap_sym < (int64_t)geo->n_sectors * geo->n_rows || in->cap_sym < 1 || in->cap_esc < 0 ||
        (in->cap_esc > 0 && !in->esc) || (in->cap_bytes > 0 && !in->bytes) || (trk->cap_tracks > 0 && !in->track_len))
        return fail(c, TPC_ERR_ARG, "compressed input: counts, sym, freq, block_bytes, esc, bytes, track_len");
    if (!syms || !sector || !row || !yq || !zq || !qtot || !sigma_y || !sigma_z)
        return fail(c, TPC_ERR_ARG, "decoded outputs are NULL");
    TPC_HIP(c, hipSetDevice(c->device));
    tpc_clusters_t none{};
    Prepared pr;
    if ((rc = prepare(c, &none, geo, bz, p, p->bin_y, p->bin_z, &pr))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = decompress_run(c, *in, pr.g, pr.kp.kq, pr.kp.s_max, *cp, *trk, syms, sector, row, yq, zq, qtot, sigma_y,
                             sigma_z, st)))
        return rc;
    TPC_HIP(c, hipGetLastError());
    return TPC_OK;
}

int tpc_compress_sizes(tpc_ctx_t* c, const tpc_compressed_t* o, double* bits) {
    if (!c || !o || !o->counts || !bits) return TPC_ERR_ARG;
    c->err.clear();
    TPC_HIP(c, hipSetDevice(c->device));
    size_t hb = 0;
    const uint32_t* dh = (const uint32_t*)buf_peek(c, "cq_hist", &hb);
    if (!dh || hb < sizeof(uint32_t) * TPC_N_CSTREAMS * TPC_CS_ALPHABET)
        return fail(c, TPC_ERR_STATE, "no tpc_compress call on this context yet");
    TPC_HIP(c, hipDeviceSynchronize());
    std::vector<uint32_t> h((size_t)TPC_N_CSTREAMS * TPC_CS_ALPHABET);
    int64_t cnt[TPC_N_CSTREAMS * TPC_CSC_N];
    TPC_HIP(c, hipMemcpy(h.data(), dh, sizeof(uint32_t) * h.size(), hipMemcpyDeviceToHost));
    TPC_HIP(c, hipMemcpy(cnt, o->counts, sizeof cnt, hipMemcpyDeviceToHost));
    for (int s = 0; s < TPC_N_CSTREAMS; ++s) {
        const uint32_t* hs = h.data() + (size_t)s * TPC_CS_ALPHABET;
        double total = 0.0, ent = 0.0;
        for (int i = 0; i < TPC_CS_ALPHABET; ++i) total += hs[i];
        for (int i = 0; i < TPC_CS_ALPHABET; ++i)
            if (hs[i]) ent -= hs[i] * std::log2(hs[i] / total);
        bits[3 * s + 0] = ent;
        bits[3 * s + 1] = (double)huffman_bits(hs, TPC_CS_ALPHABET);
        bits[3 * s + 2] = 8.0 * (double)cnt[s * TPC_CSC_N + TPC_CSC_BYTES];
    }
    return TPC_OK;
}

int tpc_merge(tpc_ctx_t* c, const tpc_clusters_t* cl, const tpc_geometry_t* geo, double bz, const tpc_params_t* p,
              const tpc_merge_params_t* mp, const tpc_tracks_t* trk, tpc_merged_t* out, void* stream) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_clusters(c, cl)) || (rc = check_geometry(c, geo)) || (rc = check_params(c, p)) ||
        (rc = check_track_input(c, trk)))
        return rc;
    if (!std::isfinite(bz) || bz == 0.0) return fail(c, TPC_ERR_ARG, "bz must be finite and nonzero");
    if (trk->cap_tracks > 0 && !trk->cov) return fail(c, TPC_ERR_ARG, "tracks: cov is required");
    if (!mp || !finite_pos(mp->rho_max) || !finite_pos(mp->centre_window) || !finite_pos(mp->chi2_max) ||
        !finite_pos(mp->phase_sigmas) || !std::isfinite(mp->phase_floor) || mp->phase_floor < 0.0 ||
        mp->max_turns < 0 || mp->max_turns > 1000 || mp->sectors_per_side < 1 || mp->sectors_per_side > 128 ||
        geo->n_sectors > 2 * mp->sectors_per_side || mp->max_iter < 1 || mp->max_iter > 1000 || mp->pair_queue < 0 ||
        mp->pair_queue > 64)
        return fail(c, TPC_ERR_ARG, "merge params: need rho_max, centre_window, chi2_max, phase_sigmas > 0, "
                                    "phase_floor >= 0, max_turns in [0, 1000], sectors_per_side in [1, 128] with "
                                    "n_sectors <= 2 * sectors_per_side, max_iter in [1, 1000], pair_queue in [0, 64]");
    if (!out || out->cap_tracks < trk->cap_tracks || !out->counts ||
        (trk->cap_tracks > 0 && (!out->label || !out->n_members || !out->helix || !out->helix_cov || !out->theta ||
                                 !out->theta_cov || !out->chi2 || !out->ndf)))
        return fail(c, TPC_ERR_ARG, "merge output: every array for cap_tracks >= tracks->cap_tracks, and counts");
    TPC_HIP(c, hipSetDevice(c->device));
    Prepared pr;
    if ((rc = prepare(c, cl, geo, bz, p, p->bin_y, p->bin_z, &pr))) return rc;
    double xmax = 0.0;
    for (int r = 0; r < geo->n_rows; ++r) xmax = std::max(xmax, (double)geo->row_x[r]);
    hipStream_t st = (hipStream_t)stream;
    if ((rc = merge_run(c, *cl, pr.g, pr.kp.kq, p->sigma_y, p->sigma_z, xmax, *mp, *trk, *out, st))) return rc;
    TPC_HIP(c, hipGetLastError());
    return TPC_OK;
}

// ------------------------------------------------------------ time frames
}  // extern "C"

namespace {

std::string bytes_of(const void* p, size_t n) { return std::string((const char*)p, n); }

// One eager run of the chain with the given tiles; returns its time in ms (synchronises).
int timed_run(tpc_ctx_t* c, const tpc_clusters_t* cl, const tpc_geometry_t* geo, double bz, const tpc_params_t* p,
              tpc_tracks_t* out, hipStream_t st, const Tuning& t, float* ms) {
    tpc_params_t p2 = *p;
    p2.bin_y = t.bin_y;
    p2.bin_z = t.bin_z;
    Prepared pr;
    int rc;
    if ((rc = prepare(c, cl, geo, bz, &p2, t.bin_y, t.bin_z, &pr))) return rc;
    Scratch s;
    if ((rc = alloc_scratch(c, pr, &s, p->mlp != nullptr))) return rc;
    float* q = nullptr;
    if (p->mlp) {
        q = (float*)buf(c, "mlp_q", sizeof(float) * mlp_q_floats());
        if (!q) return TPC_ERR_HIP;
        mlp_quantize(p->mlp, q, st);
    }
    const bool prof = c->prof_on;
    c->prof_on = false;
    enqueue_chain(c, *cl, pr, s, *out, q, c->n_cu * t.blocks_per_cu, t.chunk, t.waves, st);  // warm (sizes, caches)
    hipEvent_t e0, e1;
    TPC_HIP(c, hipEventCreate(&e0));
    TPC_HIP(c, hipEventCreate(&e1));
    TPC_HIP(c, hipEventRecord(e0, st));
    enqueue_chain(c, *cl, pr, s, *out, q, c->n_cu * t.blocks_per_cu, t.chunk, t.waves, st);
    TPC_HIP(c, hipEventRecord(e1, st));
    TPC_HIP(c, hipEventSynchronize(e1));
    TPC_HIP(c, hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->prof_on = prof;
    TPC_HIP(c, hipGetLastError());
    return TPC_OK;
}

// Two-stage search: grid bin size first (default tracklet tiles), then the tracklet
// kernel's occupancy variant x queue chunk; persistent blocks per CU follow the
// occupancy (two waves per block: 2 x waves per SIMD).
int autotune(tpc_ctx_t* c, const tpc_clusters_t* cl, const tpc_geometry_t* geo, double bz, const tpc_params_t* p,
             tpc_tracks_t* out, hipStream_t st) {
    static const float bins[][2] = {{6.f, 6.f}, {8.f, 6.f}, {6.f, 8.f}, {8.f, 8.f}, {8.f, 16.f}, {12.f, 24.f}, {16.f, 32.f}};
    static const int chunks[] = {1, 2, 4};
    static const int wavess[] = {2, 3};
    Tuning best;
    best.best_ms = 1e30f;
    int n = 0, rc;
    for (auto& b : bins) {
        Tuning t;
        t.bin_y = b[0];
        t.bin_z = b[1];
        t.chunk = 1;
        t.waves = 2;
        t.blocks_per_cu = 4;
        float ms = 0.f;
        if ((rc = timed_run(c, cl, geo, bz, p, out, st, t, &ms))) return rc;
        ++n;
        if (ms < best.best_ms) {
            best = t;
            best.best_ms = ms;
        }
    }
    const Tuning base = best;
    for (int w : wavess)
        for (int ch : chunks) {
            if (ch == base.chunk && w == base.waves) continue;
            Tuning t = base;
            t.chunk = ch;
            t.waves = w;
            t.blocks_per_cu = 2 * w;
            float ms = 0.f;
            if ((rc = timed_run(c, cl, geo, bz, p, out, st, t, &ms))) return rc;
            ++n;
            if (ms < best.best_ms) {
                best = t;
                best.best_ms = ms;
            }
        }
    best.n_candidates = n;
    c->tuning = best;
    return TPC_OK;
}

// Tile cache file: one line per tuned shape, "<key> bin_y bin_z chunk blocks_per_cu waves best_ms
// n_candidates", the key a 64-bit FNV-1a hash (hex) of the shape, the device and the library
// build.  The last valid line of a key wins; unreadable files and malformed lines are ignored.
#ifndef TPC_BUILD_ID
#define TPC_BUILD_ID "unversioned"
#endif

std::string cache_key(const tpc_ctx_t* c, const std::string& shape) {
    std::string s = shape + "|" + c->arch + "|" + TPC_BUILD_ID;
    uint64_t h = 1469598103934665603ull;
    for (unsigned char ch : s) h = (h ^ ch) * 1099511628211ull;
    char buf[17];
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    return buf;
}

bool cache_lookup(const std::string& path, const std::string& key, Tuning* t) {
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[64];
        Tuning x;
        if (line[0] == '#' || std::sscanf(line, "%63s %f %f %d %d %d %f %d", k, &x.bin_y, &x.bin_z, &x.chunk,
                                          &x.blocks_per_cu, &x.waves, &x.best_ms, &x.n_candidates) != 8)
            continue;
        const bool ok = key == k && std::isfinite(x.bin_y) && x.bin_y > 0.f && std::isfinite(x.bin_z) &&
                        x.bin_z > 0.f && x.chunk >= 1 && x.chunk <= 64 && x.blocks_per_cu >= 1 &&
                        x.blocks_per_cu <= 64 && x.waves >= 2 && x.waves <= 3;
        if (ok) {
            *t = x;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const std::string& path, const std::string& key, const Tuning& t) {
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;  // the cache is an optimisation: a read-only location only costs the next tuning
    if (std::ftell(f) == 0) std::fputs("# tpcca time-frame tile cache v1\n", f);
    std::fprintf(f, "%s %.9g %.9g %d %d %d %.6g %d\n", key.c_str(), t.bin_y, t.bin_z, t.chunk, t.blocks_per_cu,
                 t.waves, t.best_ms, t.n_candidates);
    std::fclose(f);
}

}  // namespace
extern "C" {

int tpc_track_timeframe(tpc_ctx_t* c, const tpc_clusters_t* cl, const tpc_geometry_t* geo, double bz,
                        const tpc_params_t* p, tpc_tracks_t* out, void* stream, int sync_check) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_clusters(c, cl)) || (rc = check_geometry(c, geo)) || (rc = check_params(c, p)) ||
        (rc = check_out(c, out)))
        return rc;
    if (!std::isfinite(bz)) return fail(c, TPC_ERR_ARG, "bz must be finite");
    TPC_HIP(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    // tiles: forced, or tuned once per shape (cluster count bucket, geometry)
    int lg = 0;
    while ((int64_t(1) << lg) < cl->n) ++lg;
    std::string shape = std::to_string(lg) + "|" + bytes_of(geo->row_x, sizeof(float) * geo->n_rows) +
                        bytes_of(&geo->z_min, sizeof(float)) + bytes_of(&geo->z_max, sizeof(float)) +
                        std::to_string(geo->n_sectors) + (p->mlp ? "|mlp" : "");
    if (!c->tune_forced && (!c->tuned || c->tuned_key != shape)) {
        auto known = c->tuned_shapes.find(shape);
        Tuning cached;
        if (known != c->tuned_shapes.end()) {
            c->tuning = known->second;
        } else if (!c->tune_cache.empty() && cache_lookup(c->tune_cache, cache_key(c, shape), &cached)) {
            c->tuning = cached;
        } else {
            if ((rc = autotune(c, cl, geo, bz, p, out, st))) return rc;
            if (!c->tune_cache.empty()) cache_store(c->tune_cache, cache_key(c, shape), c->tuning);
        }
        c->tuned_shapes[shape] = c->tuning;
        c->tuned = true;
        c->tuned_key = shape;
    }
    const Tuning t = c->tuning;
    tpc_params_t p2 = *p;
    p2.bin_y = t.bin_y;
    p2.bin_z = t.bin_z;
    Prepared pr;
    if ((rc = prepare(c, cl, geo, bz, &p2, t.bin_y, t.bin_z, &pr))) return rc;
    Scratch s;
    if ((rc = alloc_scratch(c, pr, &s, p->mlp != nullptr))) return rc;
    float* q = nullptr;
    if (p->mlp) {
        q = (float*)buf(c, "mlp_q", sizeof(float) * mlp_q_floats());
        if (!q) return TPC_ERR_HIP;
    }
    const int blocks = c->n_cu * t.blocks_per_cu;
    c->last_n = pr.n;
    c->last_R = pr.g.R;
    c->last_S = pr.g.S;
    c->last_n_bins = pr.n_bins;
    c->last_n_starts_cap = pr.t_max;
    if (c->prof_on) {  // stage timing needs eager launches
        if (q) mlp_quantize(p->mlp, q, st);
        enqueue_chain(c, *cl, pr, s, *out, q, blocks, t.chunk, t.waves, st);
        TPC_HIP(c, hipGetLastError());
    } else {
        // every kernel argument is part of the key (the prepared grid description and kernel
        // parameters as the kernels receive them, z range included): a replay runs exactly the
        // captured chain
        std::string key = bytes_of(cl, sizeof *cl) + bytes_of(&p2, sizeof p2) + bytes_of(out, sizeof *out) +
                          bytes_of(&bz, sizeof bz) + bytes_of(&t, sizeof t) + bytes_of(&c->buf_gen, sizeof c->buf_gen) +
                          bytes_of(&pr.g, sizeof pr.g) + bytes_of(&pr.kp, sizeof pr.kp) + bytes_of(&pr.n, sizeof pr.n) +
                          bytes_of(&pr.t_max, sizeof pr.t_max) + bytes_of(&pr.slab_bins, sizeof pr.slab_bins) +
                          c->geo_key;
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            if (c->graphs.size() >= 8) {  // bounded cache
                for (auto& kv : c->graphs) {
                    (void)hipGraphExecDestroy(kv.second.exec);
                    (void)hipGraphDestroy(kv.second.graph);
                }
                c->graphs.clear();
            }
            if (!c->own_stream) TPC_HIP(c, hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
            TPC_HIP(c, hipStreamSynchronize(st));
            GraphEntry ge;
            TPC_HIP(c, hipStreamBeginCapture(c->own_stream, hipStreamCaptureModeThreadLocal));
            if (q) mlp_quantize(p->mlp, q, c->own_stream);
            enqueue_chain(c, *cl, pr, s, *out, q, blocks, t.chunk, t.waves, c->own_stream);
            TPC_HIP(c, hipStreamEndCapture(c->own_stream, &ge.graph));
            TPC_HIP(c, hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0));
            it = c->graphs.emplace(key, ge).first;
        }
        TPC_HIP(c, hipGraphLaunch(it->second.exec, st));
    }
    if (sync_check) return capacity_check(c, out, st);
    return TPC_OK;
}

int tpc_timeframe_tuning(tpc_ctx_t* c, tpc_tuning_t* o) {
    if (!c || !o) return TPC_ERR_ARG;
    if (!c->tuned && !c->tune_forced) return fail(c, TPC_ERR_STATE, "no time frame tuned yet");
    o->bin_y = c->tuning.bin_y;
    o->bin_z = c->tuning.bin_z;
    o->tracklet_chunk = c->tuning.chunk;
    o->blocks_per_cu = c->tuning.blocks_per_cu;
    o->waves_per_simd = c->tuning.waves;
    o->best_ms = c->tuning.best_ms;
    o->n_candidates = c->tuning.n_candidates;
    return TPC_OK;
}

int tpc_timeframe_tune_cache(tpc_ctx_t* c, const char* path) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    c->tune_cache = path ? path : "";
    return TPC_OK;
}

int tpc_timeframe_set_tuning(tpc_ctx_t* c, const tpc_tuning_t* t) {
    if (!c) return TPC_ERR_ARG;
    if (!t) {
        c->tune_forced = false;
        c->tuned = false;
        return TPC_OK;
    }
    if (!(t->bin_y > 0.f) || !(t->bin_z > 0.f) || t->tracklet_chunk < 1 || t->tracklet_chunk > 64 ||
        t->blocks_per_cu < 1 || t->blocks_per_cu > 64 || t->waves_per_simd < 2 || t->waves_per_simd > 3)
        return fail(c, TPC_ERR_ARG, "bad tiles");
    c->tuning.bin_y = t->bin_y;
    c->tuning.bin_z = t->bin_z;
    c->tuning.chunk = t->tracklet_chunk;
    c->tuning.blocks_per_cu = t->blocks_per_cu;
    c->tuning.waves = t->waves_per_simd;
    c->tuning.best_ms = 0.f;
    c->tuning.n_candidates = 0;
    c->tune_forced = true;
    return TPC_OK;
}

int tpc_profile_enable(tpc_ctx_t* c, int on) {
    if (!c) return TPC_ERR_ARG;
    c->prof_on = on != 0;
    return TPC_OK;
}

int tpc_profile_read(tpc_ctx_t* c, double* ms, int* n_calls) {
    if (!c || !ms) return TPC_ERR_ARG;
    TPC_HIP(c, hipSetDevice(c->device));
    for (int i = 0; i < TPC_N_PROF; ++i) ms[i] = 0.0;
    int n = 0;
    for (auto& ev : c->prof_events) {
        TPC_HIP(c, hipEventSynchronize(ev.back()));
        for (int i = 0; i < TPC_N_PROF; ++i) {
            float t = 0.f;
            TPC_HIP(c, hipEventElapsedTime(&t, ev[i], ev[i + 1]));
            ms[i] += t;
        }
        for (auto e : ev) (void)hipEventDestroy(e);
        ++n;
    }
    c->prof_events.clear();
    if (n_calls) *n_calls = n;
    return TPC_OK;
}

int tpc_mlp_infer(tpc_ctx_t* c, const float* feats, int64_t n, const float* mlp, float* logits, void* stream) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    if (n < 0 || (n > 0 && (!feats || !logits)) || !mlp) return fail(c, TPC_ERR_ARG, "bad scorer arguments");
    TPC_HIP(c, hipSetDevice(c->device));
    float* q = (float*)buf(c, "mlp_q", sizeof(float) * mlp_q_floats());
    if (!q) return TPC_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    mlp_quantize(mlp, q, st);
    mlp_infer(q, feats, n, logits, st);
    TPC_HIP(c, hipGetLastError());
    return TPC_OK;
}

int tpc_triplets(tpc_ctx_t* c, const tpc_clusters_t* cl, const tpc_geometry_t* geo, const tpc_params_t* p,
                 int32_t* trip, float* feats, int64_t cap, int64_t* n_out, void* stream) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    int rc;
    if ((rc = check_clusters(c, cl)) || (rc = check_geometry(c, geo)) || (rc = check_params(c, p))) return rc;
    if (!n_out || cap < 0 || (cap > 0 && (!trip || !feats))) return fail(c, TPC_ERR_ARG, "bad triplet outputs");
    TPC_HIP(c, hipSetDevice(c->device));
    Prepared pr;
    if ((rc = prepare(c, cl, geo, 0.0, p, p->bin_y, p->bin_z, &pr))) return rc;
    Scratch s;
    if ((rc = alloc_scratch(c, pr, &s, false))) return rc;
    hipStream_t st = (hipStream_t)stream;
    enqueue_grid(*cl, pr, s, st);
    const int64_t n = pr.n;
    // per-hit pair counts (reuse the link arrays as scratch), then offsets
    uint32_t* cnt = (uint32_t*)s.up;
    uint32_t* off = (uint32_t*)s.dn;
    triplet_count(pr.g, pr.kp, s.hits, s.bin_off, n, s.counters, cnt, st);
    uint32_t* total = s.counters + C_N_PAIRS;
    scan_u32(cnt, off, n, s.counters + C_N_VALID_CLU, total, s.scan, st);
    uint32_t tot = 0;
    TPC_HIP(c, hipMemcpyAsync(&tot, total, sizeof tot, hipMemcpyDeviceToHost, st));
    TPC_HIP(c, hipStreamSynchronize(st));
    *n_out = tot;
    if (tot > 0 && cap > 0) triplet_write(pr.g, pr.kp, s.hits, s.bin_off, n, s.counters, off, trip, feats, cap, st);
    TPC_HIP(c, hipGetLastError());
    TPC_HIP(c, hipStreamSynchronize(st));
    return TPC_OK;
}

int tpc_mlp_grad(tpc_ctx_t* c, const float* feats, const uint8_t* labels, const int32_t* idx, int32_t n_batch,
                 const float* mlp, float* grad, float* loss, void* stream) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    if (n_batch < 1 || n_batch > 65536 || !feats || !labels || !idx || !mlp || !grad || !loss)
        return fail(c, TPC_ERR_ARG, "bad gradient arguments");
    TPC_HIP(c, hipSetDevice(c->device));
    float* q = (float*)buf(c, "mlp_q", sizeof(float) * mlp_q_floats());
    float* part = (float*)buf(c, "mlp_part", sizeof(float) * (size_t)mlp_grad_blocks(n_batch) * (TPC_MLP_N_PARAMS + 1));
    if (!q || !part) return TPC_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    mlp_quantize(mlp, q, st);
    mlp_grad_step(q, feats, labels, idx, n_batch, part, st);
    mlp_reduce(part, n_batch, grad, loss, nullptr, nullptr, nullptr, 1, 0.f, 0.f, 0.f, 0.f, st);
    TPC_HIP(c, hipGetLastError());
    return TPC_OK;
}

int tpc_mlp_train(tpc_ctx_t* c, const float* feats, const uint8_t* labels, const int32_t* order,
                  const tpc_train_cfg_t* cfg, float* mlp, float* m, float* v, float* loss, void* stream) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    if (!cfg || cfg->batch < 1 || cfg->batch > 65536 || cfg->n_steps < 0 || cfg->step0 < 0 || !feats || !labels ||
        !order || !mlp || !m || !v || !loss || !(cfg->lr > 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) ||
        !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) || !(cfg->eps > 0.f))
        return fail(c, TPC_ERR_ARG, "bad training arguments");
    TPC_HIP(c, hipSetDevice(c->device));
    float* q = (float*)buf(c, "mlp_q", sizeof(float) * mlp_q_floats());
    float* part = (float*)buf(c, "mlp_part", sizeof(float) * (size_t)mlp_grad_blocks(cfg->batch) * (TPC_MLP_N_PARAMS + 1));
    if (!q || !part) return TPC_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    mlp_quantize(mlp, q, st);
    for (int k = 0; k < cfg->n_steps; ++k) {
        mlp_grad_step(q, feats, labels, order + (size_t)k * cfg->batch, cfg->batch, part, st);
        mlp_reduce(part, cfg->batch, nullptr, loss + k, mlp, m, v, cfg->step0 + k + 1, cfg->lr, cfg->beta1, cfg->beta2,
                   cfg->eps, st);
        mlp_quantize(mlp, q, st);
    }
    TPC_HIP(c, hipGetLastError());
    return TPC_OK;
}

int tpc_stage_size(tpc_ctx_t* c, int stage, size_t* bytes) {
    if (!c || !bytes || stage < 0 || stage >= TPC_N_STAGES) return TPC_ERR_ARG;
    TPC_HIP(c, hipSetDevice(c->device));
    size_t cb = 0;
    uint32_t* counters = (uint32_t*)buf_peek(c, "counters", &cb);
    if (!counters) return fail(c, TPC_ERR_STATE, "no tracking call yet");
    uint32_t cnt[C_N_COUNTERS];
    TPC_HIP(c, hipDeviceSynchronize());
    TPC_HIP(c, hipMemcpy(cnt, counters, sizeof cnt, hipMemcpyDeviceToHost));
    const size_t nv = cnt[C_N_VALID_CLU], ns = cnt[C_N_STARTS], R = c->last_R, S = c->last_S;
    switch (stage) {
        case TPC_STAGE_HITS: *bytes = nv * sizeof(Hit); break;
        case TPC_STAGE_ROW_OFF:
        case TPC_STAGE_BIN_BASE: *bytes = 4 * (S * R + 1); break;
        case TPC_STAGE_BIN_OFF: *bytes = 4 * ((size_t)c->last_n_bins + 1); break;
        case TPC_STAGE_UP:
        case TPC_STAGE_DN:
        case TPC_STAGE_UP_CLEAN:
        case TPC_STAGE_DN_CLEAN: *bytes = 4 * nv; break;
        case TPC_STAGE_STARTS:
        case TPC_STAGE_TL_NHITS:
        case TPC_STAGE_TL_FLAGS: *bytes = 4 * ns; break;
        case TPC_STAGE_TL_HITS: *bytes = 4 * ns * R; break;
        case TPC_STAGE_TL_STATE: *bytes = 4 * 5 * ns; break;
        case TPC_STAGE_TL_COV: *bytes = 4 * 15 * ns; break;
        case TPC_STAGE_HIT_KEY: *bytes = 8 * nv; break;
        case TPC_STAGE_PAIR_LOGIT: *bytes = 4 * (size_t)c->last_n_pairs; break;
        default: return TPC_ERR_ARG;
    }
    return TPC_OK;
}

int tpc_stage_copy(tpc_ctx_t* c, int stage, void* dst, size_t cap_bytes) {
    size_t bytes = 0;
    int rc = tpc_stage_size(c, stage, &bytes);
    if (rc) return rc;
    if (!dst && bytes) return fail(c, TPC_ERR_ARG, "dst is NULL");
    if (bytes > cap_bytes) return fail(c, TPC_ERR_CAPACITY, "destination too small for stage " + std::to_string(stage));
    static const char* names[TPC_N_STAGES] = {"hits",     "row_off",  "bin_base", "bin_off",   "up",
                                              "dn",       "upc",      "dnc",      "starts",    "tl_nhits",
                                              "tl_hits",  "tl_state", "tl_cov",   "tl_flags",  "hit_key",
                                              "pair_logit"};
    if (bytes == 0) return TPC_OK;
    void* src = buf_peek(c, names[stage], nullptr);
    if (!src) return fail(c, TPC_ERR_STATE, "stage not computed");
    TPC_HIP(c, hipMemcpy(dst, src, bytes, hipMemcpyDefault));
    return TPC_OK;
}

}  // extern "C"
