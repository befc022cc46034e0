/*
 * tpc_ca.h — C ABI of the MI355X (gfx950) cellular-automaton TPC track finder.
 *
 * Method: per-sector track finding of the ALICE Run 3 TPC reconstruction
 * (arXiv:1910.12214, Sec. 2 and Sec. 3: derived from the Run 2 HLT GPU tracker,
 * same physics on CPU and GPU, no dependence of hit assignment on processing
 * order).  Steps: row-binned hit grid, neighbour finding and cleaning, start-hit
 * selection, two-pass Kalman tracklet construction and following in the
 * sector-local helix model, tracklet selection.  Input clusters are FP32
 * (Sec. 4, step 2).  Continuous-readout time frames (Sec. 1) are tracked in one
 * call by tpc_track_timeframe.
 *
 * Conventions for every entry point:
 *  - Pointers marked (device) must point to GPU memory of the context's device;
 *    (host) to CPU memory.  The caller owns every input and output buffer; the
 *    library never frees caller memory.  The context owns its scratch memory
 *    (grid, links, tracklets, queues, graphs) and grows it on demand.
 *  - Work is enqueued on the given HIP stream (hipStream_t passed as void*;
 *    NULL = the null stream).  Calls return once the work is enqueued unless
 *    stated otherwise.
 *  - A context serves one stream at a time: every call on a context reuses the
 *    same scratch buffers, so two calls on one context whose work overlaps on
 *    different streams race (wrong results, no error).  Work that should run
 *    concurrently uses one context per stream; consecutive calls on one context
 *    with different streams must be ordered by the caller (events or a
 *    synchronisation).  Contexts never share scratch.
 *  - Return value: TPC_OK (0) or a negative TPC_ERR_* code; tpc_last_error()
 *    gives a message.  No exception crosses the ABI.
 *  - Units: cm, Tesla, GeV/c.  Clusters are in each sector's local frame:
 *    x = pad-row radius, y transverse, z along the drift (mirrored on the
 *    C side so that z >= 0 in every sector).
 */
#ifndef TPC_CA_H
#define TPC_CA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TPC_OK = 0,
    TPC_ERR_ARG = -1,      /* invalid argument (null pointer, size, geometry, parameter) */
    TPC_ERR_CAPACITY = -2, /* outputs too small: counts hold the required sizes */
    TPC_ERR_HIP = -3,      /* a HIP runtime call failed; see tpc_last_error */
    TPC_ERR_STATE = -4     /* call not valid in the context's current state */
};

typedef struct tpc_ctx tpc_ctx_t;

/* Clusters, structure of arrays, cluster id = index.  (device) */
typedef struct {
    int64_t n;              /* number of clusters, 0 <= n < 2^31 */
    const float* y;         /* [n] local y (cm) */
    const float* z;         /* [n] local z (cm); time frames: z + v_drift * t0 */
    const uint8_t* row;     /* [n] pad row; clusters with row >= n_rows are ignored */
    const uint8_t* sector;  /* [n] sector; clusters with sector >= n_sectors are ignored */
} tpc_clusters_t;

/* Detector geometry.  (host) */
typedef struct {
    int32_t n_rows;         /* 3 .. 255 */
    const float* row_x;     /* [n_rows] pad-row radii, strictly increasing (host) */
    float tan_half;         /* tan of the sector half-opening angle (10 deg) */
    int32_t n_sectors;      /* 1 .. 256 */
    float z_min, z_max;     /* z range covered by the grid */
} tpc_geometry_t;

/* Method parameters.  Every cut is a value the caller chooses; tpc_params_default
 * fills the settings the library is validated with. */
typedef struct {
    double win_y, win_z;        /* neighbour window: |dy| <= win_y * row pitch, same for z */
    double nb_chi2_max;         /* straight-line triplet criterion cut */
    double fol_chi2_max;        /* chi2 cut for link acceptance and following */
    double sigma_y, sigma_z;    /* cluster errors (cm) */
    double s_max;               /* propagation fails when |sin phi| >= s_max */
    double edge_margin;         /* stop when |y| > x * tan_half + edge_margin */
    int32_t l_min_chain;        /* minimum linked hits of a start chain */
    int32_t n_miss_max;         /* stop after more consecutive rows without a hit */
    int32_t n_min_tracklet;     /* minimum hits of a valid tracklet */
    int32_t n_min_track;        /* minimum owned hits of a track */
    double c0_sinphi, c0_dzds, c0_qpt; /* initial variances of sin phi, dz/ds, q/pT */
    float bin_y, bin_z;         /* grid bin size (cm), > 0; never changes results */
    const float* mlp;           /* (device) 5057 FP32 scorer parameters, or NULL = plain finder */
    double mlp_tau_logit;       /* keep a candidate pair iff its scorer logit >= this */
} tpc_params_t;

/* Counters written by the tracking calls.  (device, int32 each) */
enum {
    TPC_CNT_TRACKS = 0,       /* tracks found (may exceed cap_tracks) */
    TPC_CNT_TRACK_HITS,       /* hits of all tracks (may exceed cap_hits) */
    TPC_CNT_TRACKLETS,        /* start hits = tracklets built */
    TPC_CNT_VALID_TRACKLETS,
    TPC_CNT_FIT_FAILURES,
    TPC_CNT_LINKS_RAW,        /* hits with a neighbour pair */
    TPC_CNT_LINKS_CLEAN,      /* reciprocal upward links */
    TPC_CNT_VALID_CLUSTERS,
    TPC_CNT_PAIRS,            /* candidate (down, up) pairs examined */
    TPC_CNT_PAIRS_KEPT,       /* with a scorer: pairs within the plain criterion's cut whose logit
                                 reaches tau (the survivors among which the best pair is chosen) */
    TPC_CNT_NB_OVERFLOW,      /* with a scorer: 64-hit groups whose window candidates exceeded the
                                 scoring kernel's list and were scored by the per-lane kernel */
    TPC_N_COUNTS = 16
};

/* Track output, CSR.  All pointers (device), caller-owned. Track k (k < min(n_tracks,
 * cap_tracks)) has hits hit_ids[hit_offset[k] .. hit_offset[k] + n_hits[k]) in
 * ascending row order.  Tracks appear in ascending start cluster id.  A track
 * whose hits do not fit in cap_hits is not written. */
typedef struct {
    int32_t cap_tracks, cap_hits;
    int32_t* counts;        /* [TPC_N_COUNTS] */
    int32_t* hit_offset;    /* [cap_tracks] */
    int32_t* n_hits;        /* [cap_tracks] */
    int32_t* hit_ids;       /* [cap_hits] cluster ids */
    int32_t* start_id;      /* [cap_tracks] cluster id of the tracklet's start hit */
    int32_t* sector;        /* [cap_tracks] */
    int32_t* row_ref;       /* [cap_tracks] row of the innermost hit */
    float* x_ref;           /* [cap_tracks] x of the innermost hit */
    float* state;           /* [cap_tracks * 5] y, z, sin phi, dz/ds, q/pT at x_ref */
    float* cov;             /* [cap_tracks * 15] lower triangle, row-major */
    float* chi2;            /* [cap_tracks] */
    int32_t* ndf;           /* [cap_tracks] */
} tpc_tracks_t;

/* Cluster flags (bits of one byte per cluster) written by tpc_cluster_flags. */
enum {
    TPC_FLAG_ATTACHED = 1,    /* a hit of a track */
    TPC_FLAG_ADJACENT = 2,    /* within the tube around a track on a row the track spans */
    TPC_FLAG_PROTECTED = 4,   /* assigned track has pT > pt_min and local |phi| < phi_max */
    TPC_FLAG_REMOVE_A = 8,    /* strategy A: attached or adjacent, and not protected */
    TPC_FLAG_REMOVE_B = 16    /* strategy B: not protected */
};

/* Cluster-removal settings (Sec. 4).  tpc_flag_params_default: 1.5 cm, 0.05 GeV/c, 70 deg. */
typedef struct {
    double tube_cm;         /* adjacency tube radius on the pad-row plane, > 0 */
    double pt_min;          /* protection needs pT > pt_min (GeV/c), > 0 */
    double phi_max_deg;     /* protection needs local |phi| < phi_max, in (0, 90) */
} tpc_flag_params_t;

/* Create a context on HIP device `device`.  *ctx receives the handle. */
int tpc_ctx_create(tpc_ctx_t** ctx, int device);
/* Release a context and its scratch memory (waits for its outstanding work). */
void tpc_ctx_destroy(tpc_ctx_t* ctx);
/* Message of the last error on this context (never NULL; "" after success). */
const char* tpc_last_error(tpc_ctx_t* ctx);
/* The validated default parameters (mlp = NULL). */
void tpc_params_default(tpc_params_t* p);

/* Track all sectors of one event (or any cluster set) with one launch per step.
 * Sec. 3 (TPC GPU tracking).  Enqueues the whole chain on `stream`.  When
 * `sync_check` is nonzero the call waits for the stream and returns
 * TPC_ERR_CAPACITY if the outputs were too small (counts hold the sizes). */
int tpc_track_sectors(tpc_ctx_t* ctx, const tpc_clusters_t* clusters, const tpc_geometry_t* geom,
                      double bz_tesla, const tpc_params_t* params, tpc_tracks_t* out, void* stream,
                      int sync_check);

/* Cluster attachment, adjacency, protection and removal flags for a track set
 * (Sec. 4, cluster removal: the 1.5 cm tube, ambiguities resolved to the
 * higher-momentum track, protection of tracks above 50 MeV/c with local
 * |phi| < 70 deg, strategies A and B).  `tracks` is read only: its counts
 * (TPC_CNT_TRACKS, device), hit_offset, n_hits, hit_ids (ascending row),
 * sector, x_ref and state (entries with offsets beyond cap_hits, or cluster
 * ids outside [0, n), are skipped); a track's tube covers the rows from its
 * first to its last hit, on its own sector.  Legs of looping tracks are not merged, so
 * every track counts as a primary leg.  `flags` (device, caller-owned) gets one
 * byte per cluster; `params` supplies the grid bin size and s_max (the other
 * fields are unused).  Enqueued on `stream`, no host synchronisation; returns
 * TPC_ERR_ARG for invalid arguments. */
int tpc_cluster_flags(tpc_ctx_t* ctx, const tpc_clusters_t* clusters, const tpc_geometry_t* geom,
                      double bz_tesla, const tpc_params_t* params, const tpc_flag_params_t* flag_params,
                      const tpc_tracks_t* tracks, uint8_t* flags, void* stream);
/* The settings of Sec. 4: tube 1.5 cm, pt_min 0.05 GeV/c, phi_max 70 deg. */
void tpc_flag_params_default(tpc_flag_params_t* p);

/* Track a whole continuous-readout time frame (Sec. 1) in one graph launch:
 * persistent work-queue kernels, captured as a HIP graph per input shape, with
 * the grid bin size and queue granularity chosen by the autotuner on the first
 * call for a shape (that call synchronises).  Results are identical to
 * tpc_track_sectors on the same clusters and parameters.  params->bin_y/bin_z
 * are ignored (the tuned values are used). */
int tpc_track_timeframe(tpc_ctx_t* ctx, const tpc_clusters_t* clusters, const tpc_geometry_t* geom,
                        double bz_tesla, const tpc_params_t* params, tpc_tracks_t* out, void* stream,
                        int sync_check);

/* The tile choice the time-frame path uses for the last shape it tuned (host). */
typedef struct {
    float bin_y, bin_z;
    int32_t tracklet_chunk;  /* tracklets taken per queue pop (per wave) */
    int32_t blocks_per_cu;   /* persistent grid size / number of CUs */
    int32_t waves_per_simd;  /* tracklet kernel occupancy variant: 2 or 3 waves per SIMD */
    float best_ms;           /* autotune measurement of the chosen candidate */
    int32_t n_candidates;
} tpc_tuning_t;
int tpc_timeframe_tuning(tpc_ctx_t* ctx, tpc_tuning_t* out);
/* Persist the time-frame tiles across processes: with a file path (host string), every shape the
 * context tunes is appended to that text file, and a shape found there (same shape, device and
 * library build) is used without tuning.  NULL or "" turns the cache off.  An unreadable file or a
 * malformed line only means that the shape is tuned again; write failures are ignored.  The
 * context also remembers every shape it tuned, so returning to an earlier shape never re-tunes. */
int tpc_timeframe_tune_cache(tpc_ctx_t* ctx, const char* path);
/* Force the time-frame tiles (disables tuning) or, with NULL, re-enable tuning. */
int tpc_timeframe_set_tuning(tpc_ctx_t* ctx, const tpc_tuning_t* tiles);

/* Stage timing.  While enabled, every tracking call records HIP events on its
 * stream between its steps: [0] grid, [1] neighbours (+ scorer), [2] cleaning and
 * start hits, [3] tracklet construction, [4] selection and output.  tpc_profile_read
 * waits for the recorded work, returns per-step sums in milliseconds (ms[TPC_N_PROF]),
 * the number of calls summed, and resets the sums.  For measurement tools. */
#define TPC_N_PROF 5
int tpc_profile_enable(tpc_ctx_t* ctx, int on);
int tpc_profile_read(tpc_ctx_t* ctx, double* ms, int* n_calls);

/* Internal arrays of the last tracking call, for stage-by-stage checks.
 * Positions refer to the grid's sorted order (see TPC_STAGE_HITS). */
enum {
    TPC_STAGE_HITS = 0,      /* [n_valid] {float y, float z, uint32 id, uint32 sector*n_rows+row} */
    TPC_STAGE_ROW_OFF,       /* [n_sectors*n_rows+1] uint32 first sorted position of each row */
    TPC_STAGE_BIN_BASE,      /* [n_sectors*n_rows+1] uint32 first bin of each row */
    TPC_STAGE_BIN_OFF,       /* [n_bins+1] uint32 first sorted position of each bin */
    TPC_STAGE_UP,            /* [n_valid] int32 raw upward link (sorted position, -1) */
    TPC_STAGE_DN,            /* [n_valid] int32 raw downward link */
    TPC_STAGE_UP_CLEAN,      /* [n_valid] int32 */
    TPC_STAGE_DN_CLEAN,      /* [n_valid] int32 */
    TPC_STAGE_STARTS,        /* [n_starts] uint32 sorted position of each start hit */
    TPC_STAGE_TL_NHITS,      /* [n_starts] int32 */
    TPC_STAGE_TL_HITS,       /* [n_starts * n_rows] int32: hits at the slot's end, ascending rows */
    TPC_STAGE_TL_STATE,      /* [n_starts * 5] float */
    TPC_STAGE_TL_COV,        /* [n_starts * 15] float */
    TPC_STAGE_TL_FLAGS,      /* [n_starts] uint32: bit0 valid, bit1 fit failure */
    TPC_STAGE_HIT_KEY,       /* [n_valid] uint64 */
    TPC_STAGE_PAIR_LOGIT,    /* [n_pairs] float scorer logits of the last scored pairs */
    TPC_N_STAGES
};
/* Size in bytes of a stage array of the last call (host out). */
int tpc_stage_size(tpc_ctx_t* ctx, int stage, size_t* bytes);
/* Copy a stage array into `dst` (host or device), at most `cap_bytes`.  Synchronous. */
int tpc_stage_copy(tpc_ctx_t* ctx, int stage, void* dst, size_t cap_bytes);

/* ---- learned triplet scorer: MLP 12-64-64-1, BF16 weights, FP32 accumulation ----
 * Parameter vector (device, FP32 master values, 5057 floats): W1[12][64], b1[64],
 * W2[64][64], b2[64], w3[64], b3.  Computation uses the weights rounded to BF16
 * (nearest, ties to even) and the biases in FP32. */
#define TPC_MLP_N_PARAMS 5057
#define TPC_MLP_N_FEATURES 12

/* Logits of n feature rows feats[n][12] (device) into logits[n] (device).
 * BF16 MFMA with the activations carried as three BF16 terms (FP32-exact). */
int tpc_mlp_infer(tpc_ctx_t* ctx, const float* feats, int64_t n, const float* mlp, float* logits, void* stream);

/* Enumerate every window candidate triplet (down, middle, up) of the clusters,
 * with its 12 scorer features.  triplets[cap][3] (device, cluster ids d, m, u),
 * feats[cap][12] (device).  *n_out (host) receives the number of triplets; when it
 * exceeds cap only the first cap are written, in no particular order.  Synchronous. */
int tpc_triplets(tpc_ctx_t* ctx, const tpc_clusters_t* clusters, const tpc_geometry_t* geom,
                 const tpc_params_t* params, int32_t* triplets, float* feats, int64_t cap, int64_t* n_out,
                 void* stream);

/* Mean binary cross-entropy loss and its gradient for one batch (rows idx[0..n_batch)
 * of feats/labels; device).  grad[5057] and loss[1] (device).  Forward and backward
 * run on BF16 MFMA with FP32 accumulation. */
int tpc_mlp_grad(tpc_ctx_t* ctx, const float* feats, const uint8_t* labels, const int32_t* idx,
                 int32_t n_batch, const float* mlp, float* grad, float* loss, void* stream);

typedef struct {
    int32_t batch;          /* rows per step, 1 .. 65536 */
    int32_t n_steps;        /* steps to run; order holds n_steps * batch row indices */
    int32_t step0;          /* Adam steps already taken (bias correction continues) */
    float lr, beta1, beta2, eps;
} tpc_train_cfg_t;

/* Adam training (Kingma & Ba) of the scorer: for each step s, the batch
 * order[s*batch .. (s+1)*batch), gradient as tpc_mlp_grad, Adam update of the FP32
 * master parameters `mlp` (in/out) with moments m, v (in/out, device [5057]).
 * loss[n_steps] (device) receives each step's loss. */
int tpc_mlp_train(tpc_ctx_t* ctx, const float* feats, const uint8_t* labels, const int32_t* order,
                  const tpc_train_cfg_t* cfg, float* mlp, float* m, float* v, float* loss, void* stream);

/* ---- cluster compression (Sec. 4, TPC data reduction, steps 2-4) ----
 * Step 2: positions become integers in fixed quanta (yq = rint(y / q_y), zq likewise, FP64 from
 * the FP32 coordinates, ties to even); the charge and the two widths keep their leading one and
 * the n bits after it, rounded to nearest (half up), coded as (e << (n+1)) | (v >> e).
 * Step 3: the clusters of tracks (a track set as the tracking calls write it: hits in ascending
 * rows) are stored as the row step from the previous hit (from row_ref for the first) and the
 * residuals of their quantised positions to the quantised prediction of the track's helix,
 * carried in closed form from its reference state to the hit's row (the previous hit's position
 * where that fails).  Every other cluster is stored per (sector, row) in ascending (zq, yq,
 * cluster id): the number of such clusters of each row, and per cluster the differences of zq and
 * yq to the previous one of its row (the first: zq and yq themselves).  Charges and widths follow
 * the cluster order of the streams (track clusters first, in track order).
 * Step 4: each stream is coded by range ANS (31-bit state, byte output, 14-bit probabilities,
 * blocks of 4096 symbols).  Signed values are zigzag-mapped (0, -1, 1, ... -> 0, 1, 2, ...);
 * values >= 4095 are the escape symbol 4095 and go raw to the stream's escape list. */
enum {
    TPC_CS_A_DROW = 0, /* track clusters: row step */
    TPC_CS_A_RY,       /* track clusters: y residual (zigzag) */
    TPC_CS_A_RZ,       /* track clusters: z residual (zigzag) */
    TPC_CS_U_N,        /* other clusters per (sector, row): count (one symbol per row, all rows) */
    TPC_CS_U_DZ,       /* other clusters: z difference (first of a row: zigzag(zq)) */
    TPC_CS_U_DY,       /* other clusters: y difference (zigzag) */
    TPC_CS_Q,          /* charge codes, n_charge bits */
    TPC_CS_SY,         /* y-width codes, n_width bits */
    TPC_CS_SZ,         /* z-width codes, n_width bits */
    TPC_N_CSTREAMS
};
#define TPC_CS_ALPHABET 4096
#define TPC_CS_BLOCK 4096
#define TPC_CS_PROB_BITS 14

/* Cluster properties besides the position.  (device) [n] each */
typedef struct {
    const uint16_t* qtot;    /* total charge, ADC counts */
    const uint8_t* sigma_y;  /* width along y, 1/64 cm */
    const uint8_t* sigma_z;  /* width along z, 1/64 cm */
} tpc_cluster_props_t;

/* Compression settings; tpc_compress_params_default: 0.0075 cm, 0.0125 cm (sigma/8), 4, 3. */
typedef struct {
    double q_y, q_z;          /* position quanta (cm), > 0 */
    int32_t n_charge, n_width; /* bits kept after the leading one, 0 .. 15 */
} tpc_compress_params_t;

/* Per-stream counts, int64 each: counts[s * TPC_CSC_N + field]. */
enum { TPC_CSC_SYMBOLS = 0, TPC_CSC_ESCAPES, TPC_CSC_BYTES, TPC_CSC_BLOCKS, TPC_CSC_N };
/* counts[TPC_N_CSTREAMS * TPC_CSC_N + k]: clusters on tracks, other clusters, clusters skipped
 * (row or sector out of range, or |yq|, |zq| >= 2^23), track hits whose prediction failed. */
enum { TPC_CST_ATTACHED = 0, TPC_CST_UNATTACHED, TPC_CST_SKIPPED, TPC_CST_PRED_FAIL, TPC_CST_N };

/* Compressed clusters.  All pointers (device), caller-owned.  cap_sym >= n + n_sectors * n_rows
 * holds every stream; cap_esc bounds each stream's escapes; cap_bytes bounds all coded bytes
 * (2 * cap_sym + 4 per block is always enough). */
typedef struct {
    int64_t cap_sym, cap_esc, cap_bytes;
    int64_t* counts;         /* [TPC_N_CSTREAMS * TPC_CSC_N + TPC_CST_N] */
    uint16_t* sym;           /* [TPC_N_CSTREAMS * cap_sym] symbols, stream after stream */
    uint32_t* esc;           /* [TPC_N_CSTREAMS * cap_esc] escaped values in stream order */
    uint32_t* freq;          /* [TPC_N_CSTREAMS * TPC_CS_ALPHABET] ANS frequencies (sum 2^14) */
    uint32_t* block_bytes;   /* [TPC_N_CSTREAMS * (cap_sym / TPC_CS_BLOCK + 1)] coded bytes per block */
    uint8_t* bytes;          /* [cap_bytes] coded blocks, stream after stream */
    int32_t* order;          /* [n] cluster id of each stream position (track clusters first) */
    int32_t* track_len;      /* [tracks->cap_tracks] hits of each track in the streams (0: track left
                                out because an entry was unusable; its clusters are stored as others) */
} tpc_compressed_t;

void tpc_compress_params_default(tpc_compress_params_t* p);

/* Compress the clusters of one event or time frame given its tracks (read as for
 * tpc_cluster_flags: counts, hit_offset, n_hits, hit_ids, sector, row_ref, x_ref, state; hit
 * entries outside [0, n) or beyond cap_hits leave their track out, and its clusters are stored as
 * others).  params supplies s_max.  Enqueued on `stream`; with sync_check nonzero the call waits
 * and returns TPC_ERR_CAPACITY when a capacity was too small (counts hold the sizes), and
 * TPC_ERR_ARG when a cluster is on more than one track (the streams are then not valid). */
int tpc_compress(tpc_ctx_t* ctx, const tpc_clusters_t* clusters, const tpc_cluster_props_t* props,
                 const tpc_geometry_t* geom, double bz_tesla, const tpc_params_t* params,
                 const tpc_compress_params_t* cparams, const tpc_tracks_t* tracks, tpc_compressed_t* out,
                 void* stream, int sync_check);

/* Sizes of the last tpc_compress call on this context, whose output is `c` (host; synchronises):
 * per stream, bits[3 * s + 0] = the entropy of its symbols (sum over the symbols of -log2 of their
 * relative frequency), [3 s + 1] = their Huffman-coded length, [3 s + 2] = their range-ANS length;
 * escapes and code tables are not included.  bits has 3 * TPC_N_CSTREAMS entries. */
int tpc_compress_sizes(tpc_ctx_t* ctx, const tpc_compressed_t* c, double* bits);

/* Decode the ANS blocks of `in` back into symbols (syms: [TPC_N_CSTREAMS * in->cap_sym], device)
 * and, from the symbols, the escapes and the same tracks, the clusters in stream order:
 * sector, row (uint8), yq, zq (int32), charge (uint16), widths (uint8), each [n_total] (device).
 * Enqueued on `stream`. */
int tpc_decompress(tpc_ctx_t* ctx, const tpc_compressed_t* in, const tpc_geometry_t* geom, double bz_tesla,
                   const tpc_params_t* params, const tpc_compress_params_t* cparams, const tpc_tracks_t* tracks,
                   uint16_t* syms, uint8_t* sector, uint8_t* row, int32_t* yq, int32_t* zq, uint16_t* qtot,
                   uint8_t* sigma_y, uint8_t* sigma_z, void* stream);

/* ---- track merging and the merged refit (Sec. 4) ----
 * The tracker finds each leg of a looping track, and each sector's piece of a track
 * crossing sectors, as a track of its own (about three instances per low-pT looper).
 * tpc_merge joins the tracks that are pieces of one helix and fits each merged track
 * once.  Per track (FP64): its global helix h = (Xc, Yc, k, w, z0) -- circle centre in
 * the global frame (cm), curvature k = |q/pT c Bz| > 0 (1/cm), pitch w = dz/dpsi (cm
 * per radian around the centre) and phase z0 = z - w psi at the reference point (psi =
 * the point's angle around the centre) -- with its covariance carried from the state
 * covariance.  Sector s covers azimuth [360/sps * (s mod sps), 360/sps * (s mod sps + 1))
 * degrees, sps = sectors_per_side, local x along the sector's centre line; sectors
 * s >= sps are the other side, whose local z is mirrored (global Z = -z).
 * Two tracks are pieces of one helix when both radii are at most rho_max, their
 * centres differ by at most centre_window in X and in Y, chi2 of (Xc, Yc, k, w) with
 * the sum of both covariances is at most chi2_max, and their phases agree modulo
 * m = round(dz0 / (pi (wA + wB))) turns, |m| <= max_turns, within phase_sigmas
 * standard deviations (z0 and m turns of pitch errors, plus phase_floor in
 * quadrature).  Merged tracks are the connected components of that relation, each
 * labelled by its lowest track index.  Each merged track (two or more members) is then
 * refit by weighted least squares (Gauss-Newton, steps halved until chi2 does not grow, at most max_iter
 * steps) to one helix theta = (Xc, Yc, rho, z0, w) through all its members' hits:
 * transverse residual = distance of the hit from the circle (params->sigma_y),
 * longitudinal residual = Z - z0 - w psi (params->sigma_z), each hit's psi unwrapped to
 * the turn its own track's helix predicts, shifted by the whole turns between its
 * track's phase and the lowest member's.
 * pair_queue sizes the context's queue of candidate pairs awaiting the full test (pairs
 * per track slot of the track set); tracks whose pairs do not fit are rescanned with
 * every pair tested at once, which gives the same labels more slowly (and may count some
 * pairs twice in TPC_MG_PAIRS_PASSED).
 * tpc_merge_params_default: 600 cm, 16 cm, 60, 5, 0.1 cm, 5 turns, 18, 50, 4. */
typedef struct {
    double rho_max;          /* only helices this tight merge (cm), > 0 */
    double centre_window;    /* |dXc|, |dYc| at most this (cm), > 0 */
    double chi2_max;         /* chi2 of (Xc, Yc, k, w), 4 dof, > 0 */
    double phase_sigmas;     /* phase agreement in standard deviations, > 0 */
    double phase_floor;      /* added in quadrature to the phase error (cm), >= 0 */
    int32_t max_turns;       /* phases at most this many turns apart, 0 .. 1000 */
    int32_t sectors_per_side;/* 1 .. 128, n_sectors <= 2 * sectors_per_side */
    int32_t max_iter;        /* refit steps, 1 .. 1000 */
    int32_t pair_queue;      /* queued candidate pairs per track slot, 0 .. 64 */
} tpc_merge_params_t;

enum {
    TPC_MG_COMPONENTS = 0,   /* merged tracks (connected components, singletons included) */
    TPC_MG_MERGED,           /* components of two or more tracks */
    TPC_MG_PAIRS_TESTED,     /* candidate pairs that reached the full same-helix test */
    TPC_MG_PAIRS_PASSED,     /* of those, pairs that passed */
    TPC_MG_MAX_CELL,         /* most tracks in one centre cell */
    TPC_MG_BIG_CELLS,        /* cells too long for the LDS sort (sorted in global memory) */
    TPC_MG_REFIT_FAILED,     /* refits whose normal matrix was singular, or whose hits exceed the
                                track set's hit capacity (overlapping hit lists): theta NaN */
    TPC_MG_N
};

/* Output of tpc_merge (device).  Entries of track k for k < number of tracks; the fit
 * entries only at the roots (label[k] == k) of merged tracks of two or more members,
 * NaN (ndf 0) elsewhere: a track that merged with nothing keeps the tracker's fit. */
typedef struct {
    int32_t cap_tracks;      /* >= tracks->cap_tracks */
    int32_t* label;          /* [cap] lowest track index of k's component; -1 beyond the tracks */
    int32_t* n_members;      /* [cap] members of the component rooted at k, 0 if k is no root */
    double* helix;           /* [cap * 5] (Xc, Yc, k, w, z0) of track k; NaN if unusable */
    double* helix_cov;       /* [cap * 15] lower triangle, row-major */
    double* theta;           /* [cap * 5] refit (Xc, Yc, rho, z0, w) */
    double* theta_cov;       /* [cap * 15] lower triangle, row-major: inverse normal matrix */
    double* chi2;            /* [cap] */
    int32_t* ndf;            /* [cap] 2 * hits - 5 */
    int64_t* counts;         /* [TPC_MG_N] */
} tpc_merged_t;

void tpc_merge_params_default(tpc_merge_params_t* p);

/* Merge and refit the tracks of `tracks` (the tracker's output or any track set in
 * its layout: counts[TPC_CNT_TRACKS] tracks, clamped to cap_tracks, with hit lists,
 * sector, x_ref, state and cov) over the clusters they index.  A track whose entries
 * are unusable (sector out of range, hits beyond cap_hits, ids out of range or of a
 * cluster with row or sector out of range) is a component of its own without a fit.
 * bz_tesla must be finite and nonzero (helix centres need a curvature).  Enqueued on
 * `stream`; no host synchronisation (a first call with new geometry uploads its tables
 * synchronously).  Returns TPC_ERR_ARG for bad arguments (message in tpc_last_error). */
int tpc_merge(tpc_ctx_t* ctx, const tpc_clusters_t* clusters, const tpc_geometry_t* geom, double bz_tesla,
              const tpc_params_t* params, const tpc_merge_params_t* mparams, const tpc_tracks_t* tracks,
              tpc_merged_t* out, void* stream);

/* ---- allocation-free variant ----
 * For callers that cannot allocate device memory while they run: code under HIP
 * graph capture, tight training loops, harnesses that forbid hipMalloc.
 * tpc_mlp_train_noalloc takes the arguments of tpc_mlp_train and computes the same
 * result with the same kernels (bit-identical), but calls no allocator: its
 * scratch (packed BF16 weights and per-block partial gradients) is a fixed array
 * of TPC_MLP_NOALLOC_SCRATCH_BYTES bytes (about 5 MB) that each device holds from
 * the first tpc_ctx_create on it until the process ends.  cfg->batch above
 * TPC_MLP_NOALLOC_MAX_BATCH returns TPC_ERR_ARG with a message.  All calls on one
 * device share that array: calls whose work overlaps on one device (several
 * streams, contexts or threads) race and give wrong results, so the caller orders
 * them.  Pointers and stream as for tpc_mlp_train. */
#define TPC_MLP_NOALLOC_MAX_BATCH 65536
#define TPC_MLP_NOALLOC_SCRATCH_BYTES 5204992
int tpc_mlp_train_noalloc(tpc_ctx_t* ctx, const float* feats, const uint8_t* labels, const int32_t* order,
                          const tpc_train_cfg_t* cfg, float* mlp, float* m, float* v, float* loss, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TPC_CA_H */
