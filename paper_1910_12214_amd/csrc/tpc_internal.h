// Internal declarations of the HIP track finder (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/tpc_ca.h"

namespace tpc {

constexpr int kMaxRows = 255;
constexpr int kBlock = 256;

// One grid hit, 16 bytes: a single coalescable load per candidate.
struct alignas(16) Hit {
    float y, z;
    uint32_t id;  // cluster id
    uint32_t rs;  // sector * n_rows + row
};

// Hit record of the tracklet kernel: position, cluster id and cleaned upward link in
// one 16-byte line segment, so following a link chain reads one line per row.
struct alignas(16) TlHit {
    float y, z;
    uint32_t id;
    int32_t upc;
};

// Grid description handed to kernels by value.
struct GridDesc {
    int R, S, nz, ny_max;
    float z_min, inv_by, inv_bz;
    uint32_t n_bins;
    const float* row_x;      // [R]
    const float* row_ymin;   // [R] fp32 -(x * tan_half)
    const int32_t* row_ny;   // [R]
    const uint32_t* bin_base;  // [S*R+1]
};

// Method parameters in the form kernels use them (FP64 decisions).
struct KParams {
    double win_y, win_z, nb_cut, fol_cut;
    double vy, vz, vy15, vz15;
    double ivy15, ivz15;  // 1 / vy15, 1 / vz15 (the pair criterion multiplies)
    double s_max, edge, tan_half, kq;
    double c0s, c0t, c0q;
    int32_t l_min, n_miss, n_min_tl, n_min_trk;
    double tau;  // scorer logit threshold
};

// Growable device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

enum Counter {  // device scratch counters (uint32)
    C_N_STARTS = 0,
    C_QUEUE_TL,
    C_QUEUE_SEL,
    C_N_PAIRS,
    C_N_FAIL,
    C_N_VALID_TL,
    C_N_LINKS_RAW,
    C_N_LINKS_CLEAN,
    C_N_TRACKS,
    C_N_TRACK_HITS,
    C_N_PAIRS_KEPT,
    C_N_VALID_CLU,
    C_QUEUE_XCD0,  // 8 per-XCD tracklet queues follow
    C_NB_OVF = C_QUEUE_XCD0 + 8,  // 64-hit groups on the scorer's overflow list (per-lane kernel)
    C_N_COUNTERS = 32
};

// Spread tallies, stored after the counters.  Sums from many blocks go to one of
// kTallyLines 64-byte lines (slot = counter index) rather than to one address: a
// device-scope atomic on a single shared address is serialised chip-wide.  The
// final count kernel adds the lines to the counters.  Slot kSlotCandSeg of line
// l is the fill level of segment l of the scorer's candidate list.
constexpr int kTallyLines = 256, kTallyStride = 16, kSlotCandSeg = 15;
constexpr int kCounterWords = C_N_COUNTERS + kTallyLines * kTallyStride;
static_assert(C_N_PAIRS < kSlotCandSeg && C_N_LINKS_RAW < kSlotCandSeg && C_N_LINKS_CLEAN < kSlotCandSeg &&
                  C_N_PAIRS_KEPT < kSlotCandSeg,
              "tallied counters must fit a tally line");

struct Tuning {
    float bin_y = 8.f, bin_z = 8.f;
    int chunk = 1;         // tracklets an idle lane reserves per queue pop
    int blocks_per_cu = 8;
    int waves = 2;         // tracklet kernel occupancy variant (waves per SIMD)
    float best_ms = 0.f;
    int n_candidates = 0;
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace tpc

struct tpc_ctx {
    int device = 0;
    int n_cu = 256;
    std::string err;
    // scratch
    std::map<std::string, tpc::DevBuf> bufs;
    // shapes of the last tracking call (for stage export)
    int64_t last_n = 0, last_nvalid_cap = 0, last_n_starts_cap = 0;
    int last_R = 0, last_S = 0;
    uint32_t last_n_bins = 0;
    int64_t last_n_pairs = 0;
    uint32_t* counters_host = nullptr;  // pinned mirror used for synchronous reads
    // time-frame path
    bool tune_forced = false;
    bool tuned = false;
    std::string tuned_key;
    tpc::Tuning tuning;
    std::map<std::string, tpc::Tuning> tuned_shapes;  // every shape tuned or read from the cache
    std::string tune_cache;                            // tile cache file ("" = none)
    std::string arch;                                  // device architecture and CU count (cache key)
    std::map<std::string, tpc::GraphEntry> graphs;
    hipStream_t own_stream = nullptr;
    // second stream for work that can run beside the main chain (the scorer's fallback
    // waves), joined back through the two events; created on first use
    hipStream_t aux_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // geometry tables already on the device (key of the last upload)
    std::string geo_key;
    uint64_t buf_gen = 0;  // bumped whenever a scratch buffer moves (invalidates captured graphs)
    // stage timing
    bool prof_on = false;
    std::vector<std::vector<hipEvent_t>> prof_events;  // per call: TPC_N_PROF + 1 events
};

namespace tpc {

int fail(tpc_ctx_t* c, int code, const std::string& msg);
#define TPC_HIP(c, call)                                                                          \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return ::tpc::fail((c), TPC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// returns nullptr on allocation failure (error recorded)
void* buf(tpc_ctx_t* c, const char* name, size_t bytes);
void* buf_peek(tpc_ctx_t* c, const char* name, size_t* bytes);
uint64_t huffman_bits(const uint32_t* count, int n_sym);

// ---------------------------------------------------------------- launchers
// scan.hip
size_t scan_scratch_bytes(int64_t n_max);
// exclusive scan of n (device count if n_dev != nullptr, else n_max) uint32 values,
// out may alias in; total written to *total_dev if non-null.
void scan_u32(const uint32_t* in, uint32_t* out, int64_t n_max, const uint32_t* n_dev, uint32_t* total_dev,
              void* scratch, hipStream_t s);
void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s);

// grid.hip
// Row-sector path (when grid_rs_fits): hist, hoff: [grid_rs_hist_entries]; piece_off:
// [grid_rs_piece_entries]; recA, recB, hits, pos_of: [n]; bin_off: [n_bins + 1].
constexpr int kRsBlocks = 1024, kRsMaxKeys = 16384, kRsPieceBins = 4096, kRsMaxPieces = 256, kRsMinPerKey = 1024;
bool grid_rs_fits(const GridDesc& g, int64_t n);
size_t grid_rs_hist_entries(const GridDesc& g);
size_t grid_rs_piece_entries(const GridDesc& g);
void grid_build_rs(const tpc_clusters_t& cl, const GridDesc& g, uint32_t* hist, uint32_t* hoff, uint32_t* piece_off,
                   void* scan_scratch, Hit* recA, Hit* recB, uint32_t* bin_off, Hit* hits, uint32_t* pos_of,
                   uint32_t* row_off, uint32_t* counters, hipStream_t s);
// bin_of, slot_of, pos_of, sorted_id: [n]; bin_cnt: [n_bins] zeroed; hits: [n]
void grid_count(const tpc_clusters_t& cl, const GridDesc& g, uint32_t* bin_of, uint32_t* bin_cnt, uint32_t* slot_of,
                uint32_t* pos_of, hipStream_t s);
void grid_scatter(const tpc_clusters_t& cl, const uint32_t* bin_of, const uint32_t* slot_of, const uint32_t* bin_off,
                  uint32_t* sorted_id, hipStream_t s);
void grid_finalize(const tpc_clusters_t& cl, const GridDesc& g, const uint32_t* bin_of, const uint32_t* bin_off,
                   const uint32_t* sorted_id, Hit* hits, uint32_t* pos_of, uint32_t* row_off, uint32_t* counters,
                   hipStream_t s);

// links.hip
void find_neighbours(const GridDesc& g, const KParams& kp, const Hit* hits, const uint32_t* bin_off,
                     const uint32_t* row_off, int64_t n_max, const uint32_t* counters, int32_t* up, int32_t* dn,
                     const float* mlp_q, uint32_t* cnt, hipStream_t s);
void clean_and_flag(const KParams& kp, const Hit* hits, int64_t n_max, const uint32_t* counters, const int32_t* up,
                    const int32_t* dn, int32_t* upc, int32_t* dnc, TlHit* tl_hits, uint8_t* start_flag, uint32_t* cnt,
                    hipStream_t s);
void compact_starts(const uint8_t* start_flag, const uint32_t* pos_of, int64_t n, uint32_t* starts,
                    uint32_t* block_cnt, void* scan_scratch, uint32_t* n_starts_dev, hipStream_t s);
// processing order: start indices k grouped by (sector, z slab of slab_bins z bins, row)
// of their start hits; slab_cnt: [S * slab_count * R + 1], slot: [t_max]
constexpr float kSlabCm = 64.f;
int slab_count(const GridDesc& g, int slab_bins);
void order_starts(const GridDesc& g, const Hit* hits, const uint32_t* starts, int64_t t_max, const uint32_t* counters,
                  int slab_bins, uint32_t* slab_cnt, uint32_t* slot, uint32_t* proc, void* scan_scratch,
                  hipStream_t s);
constexpr int kXcd = 8;  // MI355X: 8 accelerator complex dies, workgroups dispatched round-robin

// tracklets.hip
struct TrackletOut {
    int32_t* nhits;
    int32_t* hits;       // [T * R]
    float* state;        // [T * 5]
    float* cov;          // [T * 15]
    float* chi2;
    int32_t* ndf;
    int32_t* row_ref;
    uint32_t* flags;     // bit0 valid, bit1 fail
};
size_t seed_bytes();  // bytes of one precomputed tracklet start record
// seeds: [t_max] start records in processing order (written here, then consumed)
void build_tracklets(const GridDesc& g, const KParams& kp, const Hit* hits, const TlHit* tl_hits,
                     const uint32_t* bin_off, const uint32_t* row_off, const int32_t* upc, const uint32_t* starts,
                     const uint32_t* proc, void* seeds,
                     uint32_t* counters, const TrackletOut& o, int64_t t_max, int grid_blocks, int chunk, int waves,
                     hipStream_t s);

// select.hip
// sort_cnt: [select_sort_entries()], order: [t_max] (valid tracklets by decreasing length)
size_t select_sort_entries();
void select_keys(const Hit* hits, const uint32_t* starts, const TrackletOut& o, int R, uint32_t* counters,
                 uint64_t* hit_key, uint32_t* sort_cnt, uint32_t* order, void* scan_scratch, int64_t t_max,
                 hipStream_t s);
void select_own(const Hit* hits, const uint32_t* starts, const uint32_t* proc, const TrackletOut& o, int R,
                const uint32_t* counters, const uint64_t* hit_key, int n_min_trk, uint32_t* own_cnt,
                uint32_t* trk_flag, uint64_t* own_mask, int64_t t_max, hipStream_t s);
// own_mask: [t_max * 4] ownership bits of each track's slot entries (written for tracks only)
void select_write(const Hit* hits, const uint32_t* starts, const uint32_t* proc, const TrackletOut& o,
                  const GridDesc& g, const uint32_t* counters, const uint64_t* hit_key, const uint32_t* own_cnt,
                  const uint32_t* trk_flag, const uint32_t* hit_off, const uint32_t* trk_idx,
                  const tpc_tracks_t& out, const uint64_t* own_mask, int64_t t_max, hipStream_t s);
void finish_counts(const uint32_t* counters, int32_t* out_counts, hipStream_t s);

// flags.hip: key [n] u64, att/adj [n] u8 scratch (cleared here); flags [n] u8 output
void cluster_flags(const GridDesc& g, const KParams& kp, const tpc_clusters_t& cl, const Hit* hits,
                   const uint32_t* bin_off, const tpc_tracks_t& trk, const tpc_flag_params_t& fp, uint64_t* key,
                   uint8_t* att, uint8_t* adj, uint8_t* flags, hipStream_t s);

// compress.hip: cluster compression (Sec. 4, steps 2-4) and its decoder; the scratch
// lives in the context (the last histogram stays in buffer "cq_hist").
int compress_run(tpc_ctx_t* c, const tpc_clusters_t& cl, const tpc_cluster_props_t& pr, const GridDesc& g, double kq,
                 double s_max, const tpc_compress_params_t& cp, const tpc_tracks_t& trk, tpc_compressed_t& out,
                 hipStream_t st);
// merge.hip: track merging and the merged refit (Sec. 4); scratch in the context.
// max_row_x: the largest pad-row radius (sizes the grid of helix centres).
int merge_run(tpc_ctx_t* c, const tpc_clusters_t& cl, const GridDesc& g, double kq, double sigma_y, double sigma_z,
              double max_row_x, const tpc_merge_params_t& mp, const tpc_tracks_t& trk, tpc_merged_t& out,
              hipStream_t st);
int decompress_run(tpc_ctx_t* c, const tpc_compressed_t& in, const GridDesc& g, double kq, double s_max,
                   const tpc_compress_params_t& cp, const tpc_tracks_t& trk, uint16_t* syms, uint8_t* sector,
                   uint8_t* row, int32_t* yq, int32_t* zq, uint16_t* qtot, uint8_t* sig_y, uint8_t* sig_z,
                   hipStream_t st);

// mlp.hip
// Sizes of the training scratch: the packed BF16 weights (bytes) and one partial gradient of
// TPC_MLP_N_PARAMS + 1 floats (the last one the loss sum) per block of kMlpTrainChunk rows.
// tpc_mlp.hip checks them against its layout.
constexpr size_t kMlpQBytes = 25360;
constexpr int kMlpTrainChunk = 256;
constexpr int kMlpMaxBatch = 65536;  // rows per training step accepted by the training entry points
size_t mlp_q_floats();
void mlp_quantize(const float* master, float* q, hipStream_t s);  // q: packed kernel layout
void mlp_infer(const float* q, const float* feats, int64_t n, float* logits, hipStream_t s);
// ovf: [nb_overflow_entries(n_max)] wave indices (counted in counters[C_NB_OVF]);
// cand: [nb_cand_entries(n_max)] 16-byte candidate records; nund: [n_max];
// wrec: [nb_overflow_entries(n_max)]
// aux, ev_fork, ev_join: a second stream on which the fallback waves run beside the
// scoring kernel (forked after the candidate kernel, joined before returning), or null
// for one stream.
void neighbours_mlp(const GridDesc& g, const KParams& kp, const Hit* hits, const uint32_t* bin_off, int64_t n_max,
                    uint32_t* counters, const float* q, int32_t* up, int32_t* dn, uint32_t* ovf, void* cand,
                    uint32_t* nund, uint32_t* wrec, hipStream_t s, hipStream_t aux, hipEvent_t ev_fork,
                    hipEvent_t ev_join);
size_t nb_overflow_entries(int64_t n_max);
size_t nb_cand_entries(int64_t n_max);
void triplet_count(const GridDesc& g, const KParams& kp, const Hit* hits, const uint32_t* bin_off, int64_t n_max,
                   const uint32_t* counters, uint32_t* cnt, hipStream_t s);
void triplet_write(const GridDesc& g, const KParams& kp, const Hit* hits, const uint32_t* bin_off, int64_t n_max,
                   const uint32_t* counters, const uint32_t* off, int32_t* trip, float* feats, int64_t cap,
                   hipStream_t s);
int mlp_grad_blocks(int batch);
void mlp_grad_step(const float* q, const float* feats, const uint8_t* labels, const int32_t* idx, int batch,
                   float* part, hipStream_t s);
void mlp_reduce(const float* part, int batch, float* grad, float* loss, float* master, float* m, float* v, int step,
                float lr, float b1, float b2, float eps, hipStream_t s);

// noalloc.hip: the fixed per-device scratch of tpc_mlp_train_noalloc.  noalloc_init looks up
// the array's device address once per device (the device must be current); noalloc_scratch
// returns it, or nullptr with the HIP error of the lookup in *err.
void noalloc_init(int device);
void* noalloc_scratch(int device, hipError_t* err);
size_t noalloc_scratch_bytes();

}  // namespace tpc
