// Cluster compression (Sec. 4, TPC data reduction, steps 2-4) and its decoder.
//
// Step 2 (per cluster): positions to integer quanta, charge and widths to dynamic
// precision.  Step 3: the clusters of each track become row steps and residuals to
// the track's helix (one wave per track, one lane per hit: every hit's prediction is
// a closed-form step from the track's reference state, so hits are independent);
// the other clusters are counted per (sector, row), scattered into their row's
// segment and ordered there by (zq, yq, id) -- one workgroup per row sorts its keys
// with a bitonic sort, in LDS, or in global memory for a row too long for LDS -- then
// stored as differences.  Step 4: range ANS per stream in blocks of 4096 symbols: a
// histogram, the frequency table (one workgroup per stream), one lane per block
// encoding backwards, and one wave per block copying the block's bytes into the
// output in decoding order.  The decoder runs the same steps backwards.
#include "tpc_device.h"
#include "tpc_internal.h"

namespace tpc {

namespace {

constexpr int kS = TPC_N_CSTREAMS;
constexpr int kAlpha = TPC_CS_ALPHABET, kEsc = TPC_CS_ALPHABET - 1;
constexpr int kBlk = TPC_CS_BLOCK, kP = TPC_CS_PROB_BITS;
constexpr uint32_t kAnsLow = 1u << 23;  // state interval [2^23, 2^31)
constexpr int64_t kQLimit = int64_t(1) << 29;  // |yq|, |zq| below this: differences fit 31 bits
constexpr int kSortLds = 4096;                   // row segments sorted in LDS up to this size

__device__ inline uint32_t zigzag(int64_t v) { return v >= 0 ? (uint32_t)(2 * v) : (uint32_t)(-2 * v - 1); }
__device__ inline int64_t unzigzag(uint32_t u) { return (u & 1u) ? -(int64_t)((u + 1u) >> 1) : (int64_t)(u >> 1); }

// Dynamic precision: keep the leading one and the n bits after it, round half up; code
// (e << (n+1)) | (v >> e).
__device__ inline uint32_t dynprec_code(uint32_t v, int n) {
    if (v == 0) return 0;
    const int p = 31 - __clz((int)v);
    if (p > n) {
        const int e = p - n;
        v = (uint32_t)((((uint64_t)v + (1ull << (e - 1))) >> e) << e);
    }
    const int p2 = 31 - __clz((int)v);
    const int e = p2 > n ? p2 - n : 0;
    return ((uint32_t)e << (n + 1)) | (v >> e);
}
__device__ inline uint32_t dynprec_value(uint32_t code, int n) {
    return (code & ((1u << (n + 1)) - 1u)) << (code >> (n + 1));
}

struct CmpArgs {
    int64_t n;
    const float *y, *z;
    const uint8_t *row, *sector;
    const uint16_t* qtot;
    const uint8_t *sig_y, *sig_z;
    int R, S;
    const float* row_x;  // [R] device
    double inv_qy, inv_qz;
    int n_q, n_w;
    double kq, s_max;
    // tracks
    const int32_t* tcounts;
    int32_t cap_tracks, cap_hits;
    const int32_t *off, *nh, *ids, *tsec, *rref;
    const float *xref, *state;
    int64_t cap_sym;
};

__device__ inline int32_t n_tracks(const CmpArgs& a) {
    const int32_t c = a.tcounts[TPC_CNT_TRACKS];
    return c < 0 ? 0 : (c < a.cap_tracks ? c : a.cap_tracks);
}

// Quantised prediction of a track's position on row x; false when the closed-form
// step fails or leaves the representable range.
__device__ inline bool predict_q(const CmpArgs& a, int32_t k, double x, int64_t& py, int64_t& pz) {
    double yt, zt, st;
    if (!helix_at_state(a.state + 5 * k, (double)a.xref[k], x, a.kq, a.s_max, yt, zt, st)) return false;
    const double qy = rint(yt * a.inv_qy), qz = rint(zt * a.inv_qz);
    if (!(fabs(qy) < (double)kQLimit) || !(fabs(qz) < (double)kQLimit)) return false;
    py = (int64_t)qy;
    pz = (int64_t)qz;
    return true;
}

// ---------------------------------------------------------------- step 2
// yq, zq and the cluster's flags: bit0 representable (row and sector in range, finite
// position, |yq|, |zq| < 2^29).
__global__ __launch_bounds__(kBlock) void k_cq_points(CmpArgs a, int32_t* __restrict__ yq, int32_t* __restrict__ zq,
                                                      uint8_t* __restrict__ fl, uint32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t skipped = 0;
    if (i < a.n) {
        const double vy = rint((double)a.y[i] * a.inv_qy), vz = rint((double)a.z[i] * a.inv_qz);
        const bool ok = a.row[i] < a.R && a.sector[i] < a.S && fabs(vy) < (double)kQLimit &&
                        fabs(vz) < (double)kQLimit;
        yq[i] = ok ? (int32_t)vy : 0;
        zq[i] = ok ? (int32_t)vz : 0;
        fl[i] = ok ? 1 : 0;
        skipped = ok ? 0u : 1u;
    }
    block_tally2(skipped, 0, 0, -1, cnt);  // tally slot 0: skipped clusters
}

// ---------------------------------------------------------------- step 3, tracks
// A track enters the streams only if all its hit entries are usable (offsets inside
// cap_hits, ids of representable clusters); tlen = its hit count then, else 0.
// Its clusters are marked as on a track (flag bit 1).
// Waves walk the tracks below the track count (k = the wave's index, then every
// nw-th); the index is read from the first lane, so every branch on it is wave-uniform.
#define CQ_WAVE_WALK(k)                                                                             \
    for (int32_t k = (int32_t)(blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)), \
                 nt_ = n_tracks(a), nw_ = (int32_t)(gridDim.x * (kBlock / 64));                       \
         k < nt_; k += nw_)

// One wave per track: the entries checked together (tlen stays 0 for a track that fails).
__global__ __launch_bounds__(kBlock) void k_cq_track_ok(CmpArgs a, const uint8_t* __restrict__ fl,
                                                        uint32_t* __restrict__ tlen) {
    const int32_t lane = (int32_t)(threadIdx.x & 63);
    CQ_WAVE_WALK(k) {
        const int32_t o = __builtin_amdgcn_readfirstlane(a.off[k]), m = __builtin_amdgcn_readfirstlane(a.nh[k]);
        const int32_t ts = __builtin_amdgcn_readfirstlane(a.tsec[k]), rr = __builtin_amdgcn_readfirstlane(a.rref[k]);
        bool ok = o >= 0 && m >= 0 && (int64_t)o + m <= (int64_t)a.cap_hits && ts >= 0 && ts < a.S && rr >= 0 &&
                  rr < a.R;
        if (ok) {
            bool bad = false;
            for (int32_t j = lane; j < m; j += 64) {
                const int32_t id = a.ids[o + j];
                bad = bad || !(id >= 0 && (int64_t)id < a.n && (fl[id] & 1));
            }
            ok = __ballot(bad) == 0ull;
        }
        if (lane == 0) tlen[k] = ok ? (uint32_t)m : 0u;
    }
}

// One wave per track index (a wave that walked several tracks would wait for its stores
// before each next load: loads and stores retire in order).
__global__ __launch_bounds__(kBlock) void k_cq_mark(CmpArgs a, const uint32_t* __restrict__ tlen,
                                                    uint8_t* __restrict__ fl) {
    const int32_t k = (int32_t)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    if (k >= a.cap_tracks || !tlen[k]) return;
    const int32_t o = a.off[k], m = (int32_t)tlen[k];
    for (int32_t j = (int32_t)(threadIdx.x & 63); j < m; j += 64) fl[a.ids[o + j]] = 3;
}

// One wave per track, one lane per hit: row step, residuals to the prediction (the
// previous hit's position where the prediction fails), cluster order.
__global__ __launch_bounds__(kBlock) void k_cq_tracks(CmpArgs a, const uint32_t* __restrict__ tlen,
                                                      const uint32_t* __restrict__ toff,
                                                      const int32_t* __restrict__ yq, const int32_t* __restrict__ zq,
                                                      uint32_t* __restrict__ val, int32_t* __restrict__ order,
                                                      uint32_t* __restrict__ cnt) {
    const int32_t k = (int32_t)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    uint32_t fails = 0;
    if (k < a.cap_tracks && tlen[k]) {
        const int32_t o = a.off[k], m = (int32_t)tlen[k];
        const uint32_t base = toff[k];
        for (int32_t j = (int32_t)(threadIdx.x & 63); j < m; j += 64) {
            const int32_t id = a.ids[o + j];
            const int r = a.row[id];
            const int32_t pid = j ? a.ids[o + j - 1] : -1;
            const int pr = j ? (int)a.row[pid] : a.rref[k];
            int64_t py, pz;
            if (!predict_q(a, k, (double)a.row_x[r], py, pz)) {
                py = j ? yq[pid] : 0;
                pz = j ? zq[pid] : 0;
                ++fails;
            }
            const uint32_t p = base + (uint32_t)j;
            if ((int64_t)p >= a.n) continue;  // a cluster on several tracks (malformed input): reported
            val[(size_t)TPC_CS_A_DROW * a.cap_sym + p] = zigzag((int64_t)r - pr);
            val[(size_t)TPC_CS_A_RY * a.cap_sym + p] = zigzag((int64_t)yq[id] - py);
            val[(size_t)TPC_CS_A_RZ * a.cap_sym + p] = zigzag((int64_t)zq[id] - pz);
            order[p] = id;
        }
    }
    block_tally2(fails, 0, 1, -1, cnt);  // tally slot 1: failed predictions
}

// ---------------------------------------------------------------- step 3, other clusters
// Adds one to c[key] for every lane with ok, with one atomic per distinct key in the
// wave (clusters usually arrive grouped by row); returns each such lane's slot:
// the counter's old value plus its rank among the wave's lanes with the same key.
// Every lane of the wave must call it.
__device__ inline uint32_t wave_inc(uint32_t* __restrict__ c, uint32_t key, bool ok) {
    const int lane = threadIdx.x & 63;
    uint64_t pend = __ballot(ok);
    uint32_t slot = 0;
    while (pend) {
        const int l = __builtin_ctzll(pend);
        const uint32_t kl = __shfl(key, l, 64);
        const uint64_t same = __ballot(ok && key == kl) & pend;
        uint32_t base = 0;
        if (lane == l) base = atomicAdd(&c[kl], (uint32_t)__popcll(same));
        base = __shfl(base, l, 64);
        if ((same >> lane) & 1ull) slot = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
        pend &= ~same;
    }
    return slot;
}

__global__ __launch_bounds__(kBlock) void k_cq_u_count(CmpArgs a, const uint8_t* __restrict__ fl,
                                                       uint32_t* __restrict__ ucnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool ok = i < a.n && fl[i] == 1;
    const uint32_t rs = ok ? (uint32_t)a.sector[i] * a.R + a.row[i] : 0u;
    wave_inc(ucnt, rs, ok);
}

__global__ __launch_bounds__(kBlock) void k_cq_u_scatter(CmpArgs a, const uint8_t* __restrict__ fl,
                                                         const uint32_t* __restrict__ uoff,
                                                         uint32_t* __restrict__ ucur, uint32_t* __restrict__ seg) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool ok = i < a.n && fl[i] == 1;
    const uint32_t rs = ok ? (uint32_t)a.sector[i] * a.R + a.row[i] : 0u;
    const uint32_t slot = wave_inc(ucur, rs, ok);
    if (ok) seg[uoff[rs] + slot] = (uint32_t)i;
}

struct UKey {
    int32_t z, y;
    uint32_t id;
};
__device__ inline bool key_less(const UKey& p, const UKey& q) {
    return p.z < q.z || (p.z == q.z && (p.y < q.y || (p.y == q.y && p.id < q.id)));
}

// One workgroup per (sector, row) of at most kSortLds clusters: bitonic sort of the
// (zq, yq, id) keys in LDS, padded to a power of two with keys above every real one
// (|zq| < 2^29).  Keys are distinct (ids), so the sorted order is unique.
__global__ __launch_bounds__(kBlock) void k_cq_u_sort(const uint32_t* __restrict__ ucnt, const uint32_t* __restrict__ uoff,
                                                      const uint32_t* __restrict__ seg, const int32_t* __restrict__ yq,
                                                      const int32_t* __restrict__ zq, const uint32_t* __restrict__ n_att,
                                                      int64_t n, int32_t* __restrict__ order) {
    __shared__ UKey keys[kSortLds];
    const uint32_t rs = blockIdx.x;
    const uint32_t m = ucnt[rs], b = uoff[rs];
    if (m == 0 || m > (uint32_t)kSortLds) return;
    uint32_t P = 1;
    while (P < m) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += kBlock) {
        if (i < m) {
            const uint32_t id = seg[b + i];
            keys[i] = UKey{zq[id], yq[id], id};
        } else {
            keys[i] = UKey{INT32_MAX, INT32_MAX, UINT32_MAX};
        }
    }
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < P; i += kBlock) {
                const uint32_t o = i ^ j;
                if (o > i) {
                    const UKey u = keys[i], v = keys[o];
                    if ((i & k) == 0 ? key_less(v, u) : key_less(u, v)) {
                        keys[i] = v;
                        keys[o] = u;
                    }
                }
            }
            __syncthreads();
        }
    }
    const int64_t first = (int64_t)*n_att + b;
    for (uint32_t i = threadIdx.x; i < m; i += kBlock)
        if (first + i < n) order[first + i] = (int32_t)keys[i].id;
}

struct UKeyLess {
    __device__ bool operator()(const UKey& p, const UKey& q) const { return key_less(p, q); }
};

// Rows longer than kSortLds: the same order by a bitonic sort of the row's keys in
// global memory, one workgroup of 1024 lanes per row.
__global__ __launch_bounds__(1024) void k_cq_u_sort_big(const uint32_t* __restrict__ ucnt,
                                                        const uint32_t* __restrict__ uoff,
                                                        const uint32_t* __restrict__ seg,
                                                        const int32_t* __restrict__ yq, const int32_t* __restrict__ zq,
                                                        const uint32_t* __restrict__ n_att, int64_t n,
                                                        UKey* __restrict__ ukeys, int32_t* __restrict__ order) {
    const uint32_t rs = blockIdx.x;
    const uint32_t m = ucnt[rs], b = uoff[rs];
    if (m <= (uint32_t)kSortLds) return;
    UKey* k = ukeys + b;
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
        const uint32_t id = seg[b + i];
        k[i] = UKey{zq[id], yq[id], id};
    }
    __syncthreads();
    flip_bitonic_sort(k, m, UKeyLess{});
    const int64_t first = (int64_t)*n_att + b;
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x)
        if (first + i < n) order[first + i] = (int32_t)k[i].id;
}

// Differences of the other clusters (position p of their part of the order) and the
// per-row counts.
__global__ __launch_bounds__(kBlock) void k_cq_u_delta(CmpArgs a, const uint32_t* __restrict__ uoff,
                                                       const uint32_t* __restrict__ n_att,
                                                       const uint32_t* __restrict__ n_un,
                                                       const int32_t* __restrict__ order,
                                                       const int32_t* __restrict__ yq, const int32_t* __restrict__ zq,
                                                       uint32_t* __restrict__ val) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= *n_un || (int64_t)*n_att + p >= a.n) return;
    const int32_t* o = order + *n_att;
    const int32_t id = o[p];
    const uint32_t rs = (uint32_t)a.sector[id] * a.R + a.row[id];
    const bool first = p == uoff[rs];
    const int32_t pid = first ? id : o[p - 1];
    const int64_t dz = first ? (int64_t)zq[id] : (int64_t)zq[id] - zq[pid];
    const int64_t dy = first ? (int64_t)yq[id] : (int64_t)yq[id] - yq[pid];
    val[(size_t)TPC_CS_U_DZ * a.cap_sym + p] = first ? zigzag(dz) : (uint32_t)dz;
    val[(size_t)TPC_CS_U_DY * a.cap_sym + p] = zigzag(dy);
}

__global__ __launch_bounds__(kBlock) void k_cq_u_n(CmpArgs a, const uint32_t* __restrict__ ucnt,
                                                   uint32_t* __restrict__ val) {
    const int32_t rs = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (rs < a.S * a.R) val[(size_t)TPC_CS_U_N * a.cap_sym + rs] = ucnt[rs];
}

// Charge and width codes in stream order.
__global__ __launch_bounds__(kBlock) void k_cq_props(CmpArgs a, const uint32_t* __restrict__ n_att,
                                                     const uint32_t* __restrict__ n_un,
                                                     const int32_t* __restrict__ order, uint32_t* __restrict__ val) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= *n_att + *n_un || (int64_t)p >= a.n) return;
    const int32_t id = order[p];
    val[(size_t)TPC_CS_Q * a.cap_sym + p] = dynprec_code(a.qtot[id], a.n_q);
    val[(size_t)TPC_CS_SY * a.cap_sym + p] = dynprec_code(a.sig_y[id], a.n_w);
    val[(size_t)TPC_CS_SZ * a.cap_sym + p] = dynprec_code(a.sig_z[id], a.n_w);
}

// Stream lengths: [s] symbols of stream s, from the cluster counts.
__global__ void k_cq_lengths(const uint32_t* __restrict__ n_att, const uint32_t* __restrict__ n_un, int n_rows_total,
                             int64_t cap_sym, uint32_t* __restrict__ len) {
    const uint32_t na = *n_att, nu = *n_un;
    const uint32_t l[kS] = {na, na, na, (uint32_t)n_rows_total, nu, nu, na + nu, na + nu, na + nu};
    if (threadIdx.x < kS) len[threadIdx.x] = (int64_t)l[threadIdx.x] < cap_sym ? l[threadIdx.x] : (uint32_t)cap_sym;
}

// Symbols (values >= 4095 escaped) and the escape flags, for every stream position.
__global__ __launch_bounds__(kBlock) void k_cq_symbols(const uint32_t* __restrict__ val, const uint32_t* __restrict__ len,
                                                       int64_t cap_sym, uint16_t* __restrict__ sym,
                                                       uint32_t* __restrict__ eflag) {
    const int s = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= len[s]) return;
    const uint32_t v = val[(size_t)s * cap_sym + p];
    sym[(size_t)s * cap_sym + p] = (uint16_t)(v >= (uint32_t)kEsc ? kEsc : v);
    eflag[(size_t)s * cap_sym + p] = v >= (uint32_t)kEsc ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_cq_escapes(const uint32_t* __restrict__ val, const uint32_t* __restrict__ len,
                                                       const uint32_t* __restrict__ eidx, int64_t cap_sym,
                                                       int64_t cap_esc, uint32_t* __restrict__ esc) {
    const int s = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= len[s]) return;
    const uint32_t v = val[(size_t)s * cap_sym + p];
    const uint32_t e = eidx[(size_t)s * cap_sym + p];
    if (v >= (uint32_t)kEsc && e < cap_esc) esc[(size_t)s * cap_esc + e] = v;
}

// ---------------------------------------------------------------- step 4, range ANS
__global__ __launch_bounds__(kBlock) void k_ans_hist(const uint16_t* __restrict__ sym, const uint32_t* __restrict__ len,
                                                     int64_t cap_sym, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kAlpha];
    const int s = blockIdx.y;
    for (int i = threadIdx.x; i < kAlpha; i += kBlock) h[i] = 0;
    __syncthreads();
    const int64_t n = len[s];
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kBlock)
        atomicAdd(&h[sym[(size_t)s * cap_sym + p]], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kAlpha; i += kBlock)
        if (h[i]) atomicAdd(&hist[(size_t)s * kAlpha + i], h[i]);
}

// Frequencies summing to 2^P: 1 + floor(count (2^P - present) / total) per present symbol, the
// remainder to the most frequent symbol (lowest on ties); cumulative frequencies.
__global__ __launch_bounds__(kBlock) void k_ans_freq(const uint32_t* __restrict__ hist, uint32_t* __restrict__ freq,
                                                     uint32_t* __restrict__ cum) {
    __shared__ uint64_t s_tot[kBlock];
    __shared__ uint32_t s_pres[kBlock];
    __shared__ uint64_t s_top[kBlock];  // (count << 32) | (0xFFFFFFFF - symbol): max = most frequent, lowest
    __shared__ uint32_t s_sum[kBlock];
    const int s = blockIdx.x;
    const uint32_t* h = hist + (size_t)s * kAlpha;
    uint64_t tot = 0, top = 0;
    uint32_t pres = 0;
    for (int i = threadIdx.x; i < kAlpha; i += kBlock) {
        tot += h[i];
        pres += h[i] ? 1u : 0u;
        const uint64_t key = ((uint64_t)h[i] << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)i);
        top = h[i] && key > top ? key : top;
    }
    s_tot[threadIdx.x] = tot;
    s_pres[threadIdx.x] = pres;
    s_top[threadIdx.x] = top;
    __syncthreads();
    for (int d = kBlock / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            s_tot[threadIdx.x] += s_tot[threadIdx.x + d];
            s_pres[threadIdx.x] += s_pres[threadIdx.x + d];
            s_top[threadIdx.x] = s_top[threadIdx.x] > s_top[threadIdx.x + d] ? s_top[threadIdx.x] : s_top[threadIdx.x + d];
        }
        __syncthreads();
    }
    const uint64_t total = s_tot[0], present = s_pres[0];
    const uint32_t top_sym = 0xFFFFFFFFu - (uint32_t)(s_top[0] & 0xFFFFFFFFu);
    const uint64_t M = 1ull << kP;
    uint32_t* f = freq + (size_t)s * kAlpha;
    // per thread: a contiguous run of 16 symbols, so the cumulative sums follow from a block scan
    constexpr int kPer = kAlpha / kBlock;
    uint32_t loc[kPer], run = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = threadIdx.x * kPer + j;
        const uint32_t c = h[i];
        loc[j] = (c && total) ? (uint32_t)(1 + (uint64_t)c * (M - present) / total) : 0u;
        run += loc[j];
    }
    s_sum[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {  // remainder to the top symbol, then exclusive sums of the runs
        uint32_t acc = 0;
        for (int t = 0; t < kBlock; ++t) acc += s_sum[t];
        const uint32_t rem = total ? (uint32_t)(M - acc) : 0u;
        s_pres[0] = rem;
        uint32_t e = 0;
        for (int t = 0; t < kBlock; ++t) {
            const uint32_t v = s_sum[t] + ((uint32_t)t == top_sym / kPer ? rem : 0u);
            s_sum[t] = e;
            e += v;
        }
    }
    __syncthreads();
    const uint32_t rem = s_pres[0];
    uint32_t c0 = s_sum[threadIdx.x];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = threadIdx.x * kPer + j;
        const uint32_t v = loc[j] + ((uint32_t)i == top_sym && total ? rem : 0u);
        f[i] = v;
        cum[(size_t)s * kAlpha + i] = c0;
        c0 += v;
    }
}

// One lane per (stream, block): encode backwards; the bytes go to the block's scratch
// in emission order, the final state to `state`.  The stream's frequencies and
// cumulative frequencies are copied to LDS first, and each lane loads its symbols
// kEncRun at a time, the next run's loads issued before the current run is coded, so
// the state's dependency chain waits on LDS only.
constexpr int kEncRun = 8;

__global__ __launch_bounds__(64) void k_ans_encode(const uint16_t* __restrict__ sym, const uint32_t* __restrict__ len,
                                                   int64_t cap_sym, const uint32_t* __restrict__ freq,
                                                   const uint32_t* __restrict__ cum, int64_t nb_max,
                                                   uint8_t* __restrict__ tmp, uint32_t* __restrict__ state,
                                                   uint32_t* __restrict__ n_emit) {
    __shared__ uint2 fc[kAlpha];
    const int s = blockIdx.y;
    const int64_t n = len[s];
    if ((int64_t)blockIdx.x * 64 >= nb_max || (int64_t)blockIdx.x * 64 * kBlk >= n) return;  // the whole block
    const uint32_t* f = freq + (size_t)s * kAlpha;
    const uint32_t* c = cum + (size_t)s * kAlpha;
    for (int i = threadIdx.x; i < kAlpha; i += 64) fc[i] = make_uint2(f[i], c[i]);
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (b >= nb_max || b * kBlk >= n) return;
    const int64_t lo = b * kBlk, hi = lo + kBlk < n ? lo + kBlk : n;
    const uint16_t* sy = sym + (size_t)s * cap_sym;
    uint8_t* out = tmp + ((size_t)s * nb_max + b) * (2 * kBlk + 4);
    uint32_t x = kAnsLow, w = 0;
    // run k covers positions hi - 1 - k kEncRun - u, u < kEncRun (those >= lo)
    uint16_t cur[kEncRun], nxt[kEncRun];
#pragma unroll
    for (int u = 0; u < kEncRun; ++u) cur[u] = hi - 1 - u >= lo ? sy[hi - 1 - u] : (uint16_t)0;
    for (int64_t i0 = hi - 1; i0 >= lo; i0 -= kEncRun) {
#pragma unroll
        for (int u = 0; u < kEncRun; ++u) {
            const int64_t i = i0 - kEncRun - u;
            nxt[u] = i >= lo ? sy[i] : (uint16_t)0;
        }
#pragma unroll
        for (int u = 0; u < kEncRun; ++u) {
            if (i0 - u < lo) break;
            const uint2 e = fc[cur[u] & (kAlpha - 1)];  // symbols are below kAlpha
            const uint32_t fs = e.x, cs = e.y;
            const uint64_t x_max = (uint64_t)fs << (31 - kP);
            while ((uint64_t)x >= x_max) {
                out[w++] = (uint8_t)(x & 0xFFu);
                x >>= 8;
            }
            x = ((x / fs) << kP) + (x % fs) + cs;
        }
#pragma unroll
        for (int u = 0; u < kEncRun; ++u) cur[u] = nxt[u];
    }
    state[(size_t)s * nb_max + b] = x;
    n_emit[(size_t)s * nb_max + b] = w + 4;
}

// One wave per (stream, block): the state's four bytes (most significant first), then the
// emitted bytes in reverse order.
__global__ __launch_bounds__(kBlock) void k_ans_pack(const uint32_t* __restrict__ len, int64_t nb_max,
                                                     const uint8_t* __restrict__ tmp, const uint32_t* __restrict__ state,
                                                     const uint32_t* __restrict__ n_emit,
                                                     const uint32_t* __restrict__ boff, int64_t cap_bytes,
                                                     uint8_t* __restrict__ bytes, uint32_t* __restrict__ block_bytes,
                                                     int64_t bb_stride) {
    const int s = blockIdx.y;
    const int64_t b = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t n = len[s];
    if (b >= nb_max || b * kBlk >= n) return;
    const size_t slot = (size_t)s * nb_max + b;
    const uint32_t m = n_emit[slot], x = state[slot];
    const uint64_t o = boff[slot];
    if (lane == 0) block_bytes[(size_t)s * bb_stride + b] = m;
    if (o + m > (uint64_t)cap_bytes) return;
    const uint8_t* src = tmp + slot * (2 * kBlk + 4);
    for (uint32_t i = lane; i < m; i += 64)
        bytes[o + i] = i < 4 ? (uint8_t)(x >> (24 - 8 * i)) : src[m - 1 - i];
}

// One lane per (stream, block): decode a block (frequencies and the slot table of the stream).
__global__ __launch_bounds__(64) void k_ans_decode(const uint8_t* __restrict__ bytes, const uint32_t* __restrict__ boff,
                                                   const uint32_t* __restrict__ block_bytes, int64_t bb_stride,
                                                   const uint32_t* __restrict__ len, int64_t nb_max,
                                                   const uint32_t* __restrict__ freq, const uint32_t* __restrict__ cum,
                                                   const uint16_t* __restrict__ slot_sym, int64_t cap_sym,
                                                   int64_t cap_bytes, uint16_t* __restrict__ sym,
                                                   uint32_t* __restrict__ bad) {
    const int s = blockIdx.y;
    const int64_t b = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t n = len[s];
    if (b >= nb_max || b * kBlk >= n) return;
    const int64_t lo = b * kBlk, hi = lo + kBlk < n ? lo + kBlk : n;
    const uint64_t o = boff[(size_t)s * nb_max + b];
    const uint32_t nbytes = block_bytes[(size_t)s * bb_stride + b];
    if (o + nbytes > (uint64_t)cap_bytes) {
        atomicAdd(bad, 1u);
        return;
    }
    const uint8_t* in = bytes + o;
    const uint32_t* f = freq + (size_t)s * kAlpha;
    const uint32_t* c = cum + (size_t)s * kAlpha;
    const uint16_t* ss = slot_sym + ((size_t)s << kP);
    if (nbytes < 4) {
        atomicAdd(bad, 1u);
        return;
    }
    uint32_t x = ((uint32_t)in[0] << 24) | ((uint32_t)in[1] << 16) | ((uint32_t)in[2] << 8) | in[3];
    uint32_t r = 4;
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t slot = x & ((1u << kP) - 1u);
        const uint16_t v = ss[slot];
        if (v >= kAlpha) {  // a slot no frequency covers: not a table this encoder wrote
            atomicAdd(bad, 1u);
            return;
        }
        sym[(size_t)s * cap_sym + i] = v;
        x = f[v] * (x >> kP) + slot - c[v];
        while (x < kAnsLow) {
            if (r >= nbytes) {
                atomicAdd(bad, 1u);
                return;
            }
            x = (x << 8) | in[r++];
        }
    }
    if (r != nbytes) atomicAdd(bad, 1u);
}

// Slot -> symbol table of each stream (2^P slots).
__global__ __launch_bounds__(kBlock) void k_ans_slots(const uint32_t* __restrict__ freq, const uint32_t* __restrict__ cum,
                                                      uint16_t* __restrict__ slot_sym) {
    const int s = blockIdx.y;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= kAlpha) return;
    const uint32_t f = freq[(size_t)s * kAlpha + i], c = cum[(size_t)s * kAlpha + i];
    for (uint32_t k = 0; k < f && c + k < (1u << kP); ++k) slot_sym[((size_t)s << kP) + c + k] = (uint16_t)i;
}

// ---------------------------------------------------------------- decoder, step 3 and 2
// Values of every stream position: the symbol, or the next escaped value.
__global__ __launch_bounds__(kBlock) void k_dq_values(const uint16_t* __restrict__ sym, const uint32_t* __restrict__ len,
                                                      const uint32_t* __restrict__ eidx, const uint32_t* __restrict__ esc,
                                                      int64_t cap_sym, int64_t cap_esc, uint32_t* __restrict__ val) {
    const int s = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= len[s]) return;
    const uint16_t v = sym[(size_t)s * cap_sym + p];
    const uint32_t e = eidx[(size_t)s * cap_sym + p];
    val[(size_t)s * cap_sym + p] = v == kEsc ? (e < cap_esc ? esc[(size_t)s * cap_esc + e] : 0u) : v;
}

__global__ __launch_bounds__(kBlock) void k_dq_eflag(const uint16_t* __restrict__ sym, const uint32_t* __restrict__ len,
                                                     int64_t cap_sym, uint32_t* __restrict__ eflag) {
    const int s = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= len[s]) return;
    eflag[(size_t)s * cap_sym + p] = sym[(size_t)s * cap_sym + p] == kEsc ? 1u : 0u;
}

struct DecOut {
    uint8_t *sector, *row;
    int32_t *yq, *zq;
    uint16_t* qtot;
    uint8_t *sig_y, *sig_z;
};

__device__ inline int64_t wave_scan(int64_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// One wave per track, one lane per hit, in chunks of 64 hits: the row is the running
// sum of the row steps; a hit's position is its prediction plus its residuals, or,
// where the prediction fails, the previous decoded hit plus them (the first hit's
// predecessor is (0, 0)) -- a sum over the run of failed predictions before it,
// taken by a segmented scan whose segments start at the hits with a prediction.
__global__ __launch_bounds__(kBlock) void k_dq_tracks(CmpArgs a, const uint32_t* __restrict__ tlen,
                                                      const uint32_t* __restrict__ toff, const uint32_t* __restrict__ val,
                                                      const uint32_t* __restrict__ len, DecOut d) {
    const int32_t k = (int32_t)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    if (k >= a.cap_tracks || !tlen[k]) return;
    const int lane = threadIdx.x & 63;
    const uint32_t m = tlen[k], base = toff[k];
    const uint32_t lim = len[TPC_CS_A_DROW] < len[kS] ? len[TPC_CS_A_DROW] : len[kS];
    const uint8_t sec = (uint8_t)a.tsec[k];
    int64_t r_in = a.rref[k], y_in = 0, z_in = 0;  // carried from the previous chunk
    for (uint32_t j0 = 0; j0 < m; j0 += 64) {
        const uint32_t p = base + j0 + (uint32_t)lane;
        const bool in = j0 + (uint32_t)lane < m && p < lim;
        const int64_t r = r_in + wave_scan(in ? unzigzag(val[(size_t)TPC_CS_A_DROW * a.cap_sym + p]) : 0, lane);
        const int rc = r < 0 ? 0 : (r >= a.R ? a.R - 1 : (int)r);
        int64_t py = 0, pz = 0;
        bool head = in && predict_q(a, k, (double)a.row_x[rc], py, pz);
        int64_t y = in ? py + unzigzag(val[(size_t)TPC_CS_A_RY * a.cap_sym + p]) : 0;
        int64_t z = in ? pz + unzigzag(val[(size_t)TPC_CS_A_RZ * a.cap_sym + p]) : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t ty = __shfl_up(y, o, 64), tz = __shfl_up(z, o, 64);
            const bool th = __shfl_up((int)head, o, 64) != 0;
            if (lane >= o && !head) {
                y += ty;
                z += tz;
                head = th;
            }
        }
        if (!head) {
            y += y_in;
            z += z_in;
        }
        if (in) {
            d.sector[p] = sec;
            d.row[p] = (uint8_t)r;
            d.yq[p] = (int32_t)y;
            d.zq[p] = (int32_t)z;
        }
        r_in = __shfl(r, 63, 64);
        y_in = __shfl(y, 63, 64);
        z_in = __shfl(z, 63, 64);
    }
}

// One wave per (sector, row), one lane per cluster in chunks of 64: z and y are
// running sums of the differences (the first z stored as itself).
__global__ __launch_bounds__(kBlock) void k_dq_rows(CmpArgs a, const uint32_t* __restrict__ uoff,
                                                    const uint32_t* __restrict__ n_att, const uint32_t* __restrict__ val,
                                                    const uint32_t* __restrict__ len, DecOut d) {
    const int32_t rs = (int32_t)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    if (rs >= a.S * a.R) return;
    const int lane = threadIdx.x & 63;
    const uint32_t m = val[(size_t)TPC_CS_U_N * a.cap_sym + rs], b = uoff[rs], na = *n_att;
    const uint8_t sec = (uint8_t)(rs / a.R), row = (uint8_t)(rs % a.R);
    int64_t y_in = 0, z_in = 0;
    for (uint32_t j0 = 0; j0 < m; j0 += 64) {
        const uint32_t j = j0 + (uint32_t)lane, p = b + j;
        const bool in = j < m && p < len[TPC_CS_U_DZ] && (uint64_t)na + p < len[kS];
        const uint32_t vz = in ? val[(size_t)TPC_CS_U_DZ * a.cap_sym + p] : 0u;
        const int64_t z = z_in + wave_scan(j == 0 ? unzigzag(vz) : (int64_t)vz, lane);
        const int64_t y = y_in + wave_scan(in ? unzigzag(val[(size_t)TPC_CS_U_DY * a.cap_sym + p]) : 0, lane);
        if (in) {
            d.sector[na + p] = sec;
            d.row[na + p] = row;
            d.yq[na + p] = (int32_t)y;
            d.zq[na + p] = (int32_t)z;
        }
        y_in = __shfl(y, 63, 64);
        z_in = __shfl(z, 63, 64);
    }
}

__global__ __launch_bounds__(kBlock) void k_dq_props(CmpArgs a, const uint32_t* __restrict__ len,
                                                     const uint32_t* __restrict__ val, DecOut d) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= len[TPC_CS_Q] || p >= len[kS]) return;
    d.qtot[p] = (uint16_t)dynprec_value(val[(size_t)TPC_CS_Q * a.cap_sym + p], a.n_q);
    d.sig_y[p] = (uint8_t)dynprec_value(val[(size_t)TPC_CS_SY * a.cap_sym + p], a.n_w);
    d.sig_z[p] = (uint8_t)dynprec_value(val[(size_t)TPC_CS_SZ * a.cap_sym + p], a.n_w);
}

// Decoder stream lengths from the counts the encoder wrote.
__global__ void k_dq_lengths(const int64_t* __restrict__ counts, int64_t cap_sym, uint32_t* __restrict__ len) {
    if (threadIdx.x < kS) {
        const int64_t v = counts[threadIdx.x * TPC_CSC_N + TPC_CSC_SYMBOLS];
        len[threadIdx.x] = (uint32_t)(v < 0 ? 0 : (v < cap_sym ? v : cap_sym));
    }
    // decoded clusters: the track clusters and the others the encoder counted
    if (threadIdx.x == kS) {
        const int64_t v = counts[kS * TPC_CSC_N + TPC_CST_ATTACHED] + counts[kS * TPC_CSC_N + TPC_CST_UNATTACHED];
        len[kS] = (uint32_t)(v < 0 ? 0 : (v < cap_sym ? v : cap_sym));
    }
}

// Final counts: per stream symbols, escapes, bytes, blocks; then the cluster totals.
__global__ void k_cq_counts(const uint32_t* __restrict__ len, const uint32_t* __restrict__ esc_tot,
                            const uint32_t* __restrict__ byte_tot, const uint32_t* __restrict__ n_att,
                            const uint32_t* __restrict__ n_un, const uint32_t* __restrict__ tally, int64_t* __restrict__ counts) {
    const int s = threadIdx.x;
    if (s < kS) {
        counts[s * TPC_CSC_N + TPC_CSC_SYMBOLS] = len[s];
        counts[s * TPC_CSC_N + TPC_CSC_ESCAPES] = esc_tot[s];
        counts[s * TPC_CSC_N + TPC_CSC_BYTES] = byte_tot[s];
        counts[s * TPC_CSC_N + TPC_CSC_BLOCKS] = ((int64_t)len[s] + kBlk - 1) / kBlk;
    }
    if (s == 0) {
        uint64_t sk = 0, pf = 0;
        for (int l = 0; l < kTallyLines; ++l) {
            sk += tally[C_N_COUNTERS + l * kTallyStride + 0];
            pf += tally[C_N_COUNTERS + l * kTallyStride + 1];
        }
        counts[kS * TPC_CSC_N + TPC_CST_ATTACHED] = *n_att;
        counts[kS * TPC_CSC_N + TPC_CST_UNATTACHED] = *n_un;
        counts[kS * TPC_CSC_N + TPC_CST_SKIPPED] = (int64_t)sk;
        counts[kS * TPC_CSC_N + TPC_CST_PRED_FAIL] = (int64_t)pf;
    }
}

inline unsigned nblk(int64_t n, int per = kBlock) { return (unsigned)(n > 0 ? (n + per - 1) / per : 1); }

// Per-stream byte totals of the packed output.
__global__ void k_cq_byte_tot(const uint32_t* __restrict__ boff, const uint32_t* __restrict__ total, int64_t nb_max,
                              uint32_t* __restrict__ byte_tot) {
    const int s = threadIdx.x;
    if (s < kS) byte_tot[s] = (s + 1 < kS ? boff[(size_t)(s + 1) * nb_max] : *total) - boff[(size_t)s * nb_max];
}

// Coded bytes per block of each stream with the unused block slots zeroed (decoder input).
__global__ __launch_bounds__(kBlock) void k_dq_block_bytes(const uint32_t* __restrict__ block_bytes, int64_t bb_stride,
                                                           const uint32_t* __restrict__ len,
                                                           uint32_t* __restrict__ masked) {
    const int s = blockIdx.y;
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= bb_stride) return;
    masked[(size_t)s * bb_stride + b] = b * kBlk < (int64_t)len[s] ? block_bytes[(size_t)s * bb_stride + b] : 0u;
}

__global__ __launch_bounds__(kBlock) void k_dq_track_len(const int32_t* __restrict__ track_len, int32_t cap_tracks,
                                                         uint32_t* __restrict__ tlen) {
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k < cap_tracks) tlen[k] = track_len[k] > 0 ? (uint32_t)track_len[k] : 0u;
}

__global__ __launch_bounds__(kBlock) void k_cq_track_len_out(const uint32_t* __restrict__ tlen, int32_t cap_tracks,
                                                             int32_t* __restrict__ track_len) {
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k < cap_tracks) track_len[k] = (int32_t)tlen[k];
}

__global__ __launch_bounds__(kBlock) void k_dq_u_n(CmpArgs a, const uint32_t* __restrict__ val,
                                                   uint32_t* __restrict__ ucnt) {
    const int32_t rs = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (rs < a.S * a.R) ucnt[rs] = val[(size_t)TPC_CS_U_N * a.cap_sym + rs];
}

}  // namespace

// ---------------------------------------------------------------- host side
namespace {

CmpArgs make_args(const tpc_clusters_t& cl, const tpc_cluster_props_t& pr, const GridDesc& g, double kq, double s_max,
                  const tpc_compress_params_t& cp, const tpc_tracks_t& trk, int64_t cap_sym) {
    CmpArgs a{};
    a.n = cl.n;
    a.y = cl.y;
    a.z = cl.z;
    a.row = cl.row;
    a.sector = cl.sector;
    a.qtot = pr.qtot;
    a.sig_y = pr.sigma_y;
    a.sig_z = pr.sigma_z;
    a.R = g.R;
    a.S = g.S;
    a.row_x = g.row_x;
    a.inv_qy = 1.0 / cp.q_y;
    a.inv_qz = 1.0 / cp.q_z;
    a.n_q = cp.n_charge;
    a.n_w = cp.n_width;
    a.kq = kq;
    a.s_max = s_max;
    a.tcounts = trk.counts;
    a.cap_tracks = trk.cap_tracks;
    a.cap_hits = trk.cap_hits;
    a.off = trk.hit_offset;
    a.nh = trk.n_hits;
    a.ids = trk.hit_ids;
    a.tsec = trk.sector;
    a.rref = trk.row_ref;
    a.xref = trk.x_ref;
    a.state = trk.state;
    a.cap_sym = cap_sym;
    return a;
}

#define CB(field, name, bytes)                                    \
    field = (decltype(field))buf(c, name, (size_t)(bytes));       \
    if (!field) return TPC_ERR_HIP;

}  // namespace

int compress_run(tpc_ctx_t* c, const tpc_clusters_t& cl, const tpc_cluster_props_t& pr, const GridDesc& g, double kq,
                 double s_max, const tpc_compress_params_t& cp, const tpc_tracks_t& trk, tpc_compressed_t& out,
                 hipStream_t st) {
    const int64_t n = cl.n > 0 ? cl.n : 1, SR = (int64_t)g.S * g.R, cap = out.cap_sym;
    const int64_t T = trk.cap_tracks > 0 ? trk.cap_tracks : 1;
    const int64_t nb_max = (cap + kBlk - 1) / kBlk, bb_stride = cap / kBlk + 1;
    int32_t *yq, *zq;
    UKey* ukeys;
    uint8_t *fl, *tmp;
    uint32_t *tlen, *toff, *ucnt, *uoff, *ucur, *seg, *val, *eflag, *eidx, *hist, *cum, *tst, *n_emit, *boff, *len,
        *esc_tot, *byte_tot, *n_att, *n_un, *tally, *b_tot;
    void* scan;
    CB(yq, "cq_yq", 4 * n);
    CB(zq, "cq_zq", 4 * n);
    CB(fl, "cq_fl", n);
    CB(tlen, "cq_tlen", 4 * (T + 1));
    CB(toff, "cq_toff", 4 * (T + 1));
    CB(ucnt, "cq_ucnt", 4 * (SR + 1));
    CB(uoff, "cq_uoff", 4 * (SR + 1));
    CB(ucur, "cq_ucur", 4 * (SR + 1));
    CB(seg, "cq_seg", 4 * n);
    CB(ukeys, "cq_ukeys", sizeof(UKey) * n);
    CB(val, "cq_val", 4 * kS * cap);
    CB(eflag, "cq_eflag", 4 * kS * cap);
    CB(eidx, "cq_eidx", 4 * kS * cap);
    CB(hist, "cq_hist", 4 * kS * kAlpha);
    CB(cum, "cq_cum", 4 * kS * kAlpha);
    CB(tmp, "cq_tmp", (size_t)kS * nb_max * (2 * kBlk + 4));
    CB(tst, "cq_state", 4 * kS * nb_max);
    CB(n_emit, "cq_nemit", 4 * (kS * nb_max + 1));
    CB(boff, "cq_boff", 4 * (kS * nb_max + 1));
    CB(len, "cq_len", 4 * 16);
    CB(esc_tot, "cq_esctot", 4 * 16);
    CB(byte_tot, "cq_bytetot", 4 * 16);
    CB(n_att, "cq_natt", 4 * 4);
    CB(n_un, "cq_nun", 4 * 4);
    CB(b_tot, "cq_btot", 4 * 4);
    CB(tally, "cq_tally", 4 * kCounterWords);
    int64_t sn = n > cap ? n : cap;
    if (SR > sn) sn = SR;
    if (T > sn) sn = T;
    if (kS * nb_max + 1 > sn) sn = kS * nb_max + 1;
    CB(scan, "cq_scan", scan_scratch_bytes(sn));
    const CmpArgs a = make_args(cl, pr, g, kq, s_max, cp, trk, cap);
    fill_u32(tally, 0u, kCounterWords, st);
    fill_u32(ucnt, 0u, SR + 1, st);
    fill_u32(ucur, 0u, SR + 1, st);
    fill_u32(hist, 0u, kS * kAlpha, st);
    fill_u32(n_emit, 0u, kS * nb_max + 1, st);
    fill_u32(n_att, 0u, 4, st);
    fill_u32(n_un, 0u, 4, st);
    fill_u32(tlen, 0u, T + 1, st);
    // step 2 and the track filter
    k_cq_points<<<nblk(cl.n), kBlock, 0, st>>>(a, yq, zq, fl, tally);
    const unsigned wblk = (unsigned)(c->n_cu * 8);  // a few workgroups per CU walk the tracks
    k_cq_track_ok<<<wblk, kBlock, 0, st>>>(a, fl, tlen);
    scan_u32(tlen, toff, T, nullptr, n_att, scan, st);
    if (trk.cap_tracks > 0) k_cq_track_len_out<<<nblk(T), kBlock, 0, st>>>(tlen, trk.cap_tracks, out.track_len);
    k_cq_mark<<<nblk(T, kBlock / 64), kBlock, 0, st>>>(a, tlen, fl);
    // step 3: track clusters, then the others
    k_cq_tracks<<<nblk(T, kBlock / 64), kBlock, 0, st>>>(a, tlen, toff, yq, zq, val, out.order, tally);
    k_cq_u_count<<<nblk(cl.n), kBlock, 0, st>>>(a, fl, ucnt);
    scan_u32(ucnt, uoff, SR, nullptr, n_un, scan, st);
    k_cq_u_scatter<<<nblk(cl.n), kBlock, 0, st>>>(a, fl, uoff, ucur, seg);
    k_cq_u_sort<<<(unsigned)SR, kBlock, 0, st>>>(ucnt, uoff, seg, yq, zq, n_att, cl.n, out.order);
    k_cq_u_sort_big<<<(unsigned)SR, 1024, 0, st>>>(ucnt, uoff, seg, yq, zq, n_att, cl.n, ukeys, out.order);
    k_cq_u_delta<<<nblk(cl.n), kBlock, 0, st>>>(a, uoff, n_att, n_un, out.order, yq, zq, val);
    k_cq_u_n<<<nblk(SR), kBlock, 0, st>>>(a, ucnt, val);
    k_cq_props<<<nblk(cl.n), kBlock, 0, st>>>(a, n_att, n_un, out.order, val);
    k_cq_lengths<<<1, 64, 0, st>>>(n_att, n_un, (int)SR, cap, len);
    // symbols and escapes
    const dim3 gs(nblk(cap), kS);
    k_cq_symbols<<<gs, kBlock, 0, st>>>(val, len, cap, out.sym, eflag);
    for (int s = 0; s < kS; ++s)
        scan_u32(eflag + (size_t)s * cap, eidx + (size_t)s * cap, cap, len + s, esc_tot + s, scan, st);
    k_cq_escapes<<<gs, kBlock, 0, st>>>(val, len, eidx, cap, out.cap_esc, out.esc);
    // step 4: range ANS
    const unsigned hb = nblk(cap) < 1024 ? nblk(cap) : 1024;
    k_ans_hist<<<dim3(hb, kS), kBlock, 0, st>>>(out.sym, len, cap, hist);
    k_ans_freq<<<kS, kBlock, 0, st>>>(hist, out.freq, cum);
    k_ans_encode<<<dim3(nblk(nb_max, 64), kS), 64, 0, st>>>(out.sym, len, cap, out.freq, cum, nb_max, tmp, tst, n_emit);
    scan_u32(n_emit, boff, kS * nb_max, nullptr, b_tot, scan, st);
    k_ans_pack<<<dim3(nblk(nb_max, kBlock / 64), kS), kBlock, 0, st>>>(len, nb_max, tmp, tst, n_emit, boff,
                                                                         out.cap_bytes, out.bytes, out.block_bytes,
                                                                         bb_stride);
    k_cq_byte_tot<<<1, 64, 0, st>>>(boff, b_tot, nb_max, byte_tot);
    k_cq_counts<<<1, 64, 0, st>>>(len, esc_tot, byte_tot, n_att, n_un, tally, out.counts);
    return TPC_OK;
}

int decompress_run(tpc_ctx_t* c, const tpc_compressed_t& in, const GridDesc& g, double kq, double s_max,
                   const tpc_compress_params_t& cp, const tpc_tracks_t& trk, uint16_t* syms, uint8_t* sector,
                   uint8_t* row, int32_t* yq, int32_t* zq, uint16_t* qtot, uint8_t* sig_y, uint8_t* sig_z,
                   hipStream_t st) {
    const int64_t SR = (int64_t)g.S * g.R, cap = in.cap_sym;
    const int64_t T = trk.cap_tracks > 0 ? trk.cap_tracks : 1;
    const int64_t bb_stride = cap / kBlk + 1;
    uint32_t *len, *masked, *boff, *cum, *eflag, *eidx, *val, *tlen, *toff, *ucnt, *uoff, *n_att, *tot, *bad;
    uint16_t* slot_sym;
    void* scan;
    CB(len, "dq_len", 4 * 16);
    CB(masked, "dq_masked", 4 * (kS * bb_stride + 1));
    CB(boff, "dq_boff", 4 * (kS * bb_stride + 1));
    CB(cum, "dq_cum", 4 * kS * kAlpha);
    CB(slot_sym, "dq_slots", 2 * ((size_t)kS << kP));
    CB(eflag, "dq_eflag", 4 * kS * cap);
    CB(eidx, "dq_eidx", 4 * kS * cap);
    CB(val, "dq_val", 4 * kS * cap);
    CB(tlen, "dq_tlen", 4 * (T + 1));
    CB(toff, "dq_toff", 4 * (T + 1));
    CB(ucnt, "dq_ucnt", 4 * (SR + 1));
    CB(uoff, "dq_uoff", 4 * (SR + 1));
    CB(n_att, "dq_natt", 16);
    CB(tot, "dq_tot", 16 * 4);
    CB(bad, "dq_bad", 16);
    int64_t sn = cap > SR ? cap : SR;
    if (T > sn) sn = T;
    if (kS * bb_stride + 1 > sn) sn = kS * bb_stride + 1;
    CB(scan, "dq_scan", scan_scratch_bytes(sn));
    tpc_clusters_t none{};
    tpc_cluster_props_t nprops{};
    const CmpArgs a = make_args(none, nprops, g, kq, s_max, cp, trk, cap);
    DecOut d{sector, row, yq, zq, qtot, sig_y, sig_z};
    fill_u32(bad, 0u, 4, st);
    fill_u32(tlen, 0u, T + 1, st);
    k_dq_lengths<<<1, 64, 0, st>>>(in.counts, cap, len);
    // step 4 backwards: block offsets, slot tables, blocks
    k_dq_block_bytes<<<dim3(nblk(bb_stride), kS), kBlock, 0, st>>>(in.block_bytes, bb_stride, len, masked);
    scan_u32(masked, boff, kS * bb_stride, nullptr, tot, scan, st);
    for (int s = 0; s < kS; ++s)
        scan_u32(in.freq + (size_t)s * kAlpha, cum + (size_t)s * kAlpha, kAlpha, nullptr, nullptr, scan, st);
    fill_u32((uint32_t*)slot_sym, 0xFFFFFFFFu, (kS << kP) / 2, st);
    k_ans_slots<<<dim3(nblk(kAlpha), kS), kBlock, 0, st>>>(in.freq, cum, slot_sym);
    k_ans_decode<<<dim3(nblk(bb_stride, 64), kS), 64, 0, st>>>(in.bytes, boff, masked, bb_stride, len, bb_stride,
                                                               in.freq, cum, slot_sym, cap, in.cap_bytes, syms, bad);
    // escapes back into values
    const dim3 gs(nblk(cap), kS);
    k_dq_eflag<<<gs, kBlock, 0, st>>>(syms, len, cap, eflag);
    for (int s = 0; s < kS; ++s)
        scan_u32(eflag + (size_t)s * cap, eidx + (size_t)s * cap, cap, len + s, tot + 1 + s, scan, st);
    k_dq_values<<<gs, kBlock, 0, st>>>(syms, len, eidx, in.esc, cap, in.cap_esc, val);
    // step 3 backwards
    if (trk.cap_tracks > 0) k_dq_track_len<<<nblk(T), kBlock, 0, st>>>(in.track_len, trk.cap_tracks, tlen);
    scan_u32(tlen, toff, T, nullptr, n_att, scan, st);
    k_dq_tracks<<<nblk(T, kBlock / 64), kBlock, 0, st>>>(a, tlen, toff, val, len, d);
    k_dq_u_n<<<nblk(SR), kBlock, 0, st>>>(a, val, ucnt);
    scan_u32(ucnt, uoff, SR, nullptr, nullptr, scan, st);
    k_dq_rows<<<nblk(SR, kBlock / 64), kBlock, 0, st>>>(a, uoff, n_att, val, len, d);
    k_dq_props<<<nblk(cap), kBlock, 0, st>>>(a, len, val, d);
    return TPC_OK;
}

#undef CB

}  // namespace tpc
