// Track merging and the merged refit (Sec. 4: the legs of a looping track, and the
// pieces of one track in neighbouring sectors, are found as separate tracks; they are
// merged into one track, which is then fitted once).  FP64 throughout.
//
//  1. helix: each track's entries checked by one wave, then one lane per track.  Its
//     global helix h = (Xc, Yc, k, w, z0) -- circle centre, curvature k > 0, pitch
//     w = dz/dpsi (z advance per radian around the centre) and phase z0 = z - w psi at
//     the reference point -- and the covariance of h carried from the track's state
//     covariance by the Jacobian.  A track takes part when its hit entries are usable,
//     h is finite and its radius 1/k is at most rho_max.
//  2. cells: centres closer than the window in X and Y lie in neighbouring cells of a
//     grid of window-sized cells.  Each track also gets a phase interval
//     [z0 - reach, z0 + reach] such that two tracks can pass the phase test only when
//     their intervals overlap (bound below).  Tracks are counted per cell, scattered,
//     and each cell is sorted by interval start (bitonic in LDS; in global memory for a
//     cell too long for LDS), then laid out as candidate arrays.
//  3. pairs: a group of eight lanes per track A walks the nine cells around its own and
//     reads, in turn, the candidates B whose interval starts inside A's (the pairs left
//     after the prefilter are queued and tested by the next kernel), so every overlapping
//     pair is reached from the track that starts first (from both on equal starts).  A
//     prefilter drops pairs that cannot pass: the centre window, and |d_i| <=
//     sqrt(chi2_max) (sigma_A,i + sigma_B,i) for each of Xc, Yc, k, w (implied by the chi2
//     cut when both tracks' covariance blocks are positive definite).  The same-helix
//     test decides, always evaluated with the lower track index first.
//  4. labels: passing pairs join a union-find forest whose links always point to a
//     smaller index (a root is linked under the smaller root by compare-and-swap), so
//     each root is the lowest index of its component whatever the order in which the
//     pairs are found.
//  5. refit: members are grouped by label in ascending index; the roots of merged tracks
//     (two or more members) are listed, those with many hits first, each with a range of
//     its own for its hits packed together.  Persistent waves take the listed components
//     one at a time: Gauss-Newton on (Xc, Yc, rho, z0, w), lanes over hits, normal
//     equations summed across the wave in a fixed order, each step halved until chi2 does
//     not grow.
//
// Phase bound.  The test takes m = round(dz0 / p) turns, p = pi (wA + wB), rejects
// |m| > M, and passes when (dz0 - m p)^2 <= n^2 var with var = CA_z0 + CB_z0 +
// (pi m)^2 (CA_w + CB_w) + f^2.  Then |dz0| <= M pi (|wA| + |wB|) + n sqrt(var), and
// sqrt(var) <= sA + sB with s = sqrt(max(C_z0, 0) + (pi M)^2 max(C_w, 0) + f^2 / 2), so
// |dz0| <= reach_A + reach_B with reach = M pi |w| + n s (the same for p = 0, where
// the test is |dz0| <= n sqrt(CA_z0 + CB_z0 + f^2)).  A reach that is not a number
// becomes infinite: such a track is tested against every track of its cells.
#include "tpc_device.h"
#include "tpc_internal.h"

namespace tpc {

namespace {

constexpr int kCellSortLds = 4096;  // cells sorted in LDS up to this many tracks

struct MgArgs {
    // tracks
    const int32_t* tcounts;
    int32_t cap_tracks, cap_hits;
    const int32_t *off, *nh, *ids, *tsec;
    const float *xref, *state, *cov;
    // clusters
    int64_t n;
    const float *y, *z;
    const uint8_t *row, *sector;
    const float* row_x;
    int R, S;
    int sps;      // sectors per side
    double dphi;  // azimuth width of a sector
    double kq;    // -c Bz
    // merging
    double rho_max, win, chi2_max, n_sig, floor2;
    int max_turns;
    double cell_w, cell_lo;
    int nc;
    // refit
    double wy, wz;  // hit weights 1 / sigma^2
    int max_iter;
};

enum MgTally { T_PAIRS = 0, T_PASSED, T_BIG_CELLS, T_FAILED, T_MERGED, T_COMPONENTS, T_MAX_CELL, T_FIT_HITS, T_N };

__device__ inline int32_t n_tracks(const MgArgs& a) {
    const int32_t c = a.tcounts[TPC_CNT_TRACKS];
    return c < 0 ? 0 : (c < a.cap_tracks ? c : a.cap_tracks);
}

__device__ inline int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Adds one to c[key] for every lane with ok, one atomic per distinct key of the wave;
// returns each such lane's slot (the old count plus its rank among equal keys).  Every
// lane of the wave must call it.
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

// Wave total of v added to tally[t] by lane 0.  Every lane of the wave must call it.
__device__ inline void wave_tally(unsigned long long* tally, int t, uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(&tally[t], (unsigned long long)v);
}

// Exclusive prefix sum of v over the wave's lanes (lane order); total gets the wave's sum.
// Every lane of the wave must call it.
__device__ inline uint32_t wave_excl_scan(uint32_t v, uint32_t& total) {
    const int lane = threadIdx.x & 63;
    uint32_t s = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(s, d, 64);
        if (lane >= d) s += t;
    }
    total = __shfl(s, 63, 64);
    return s - v;
}

// Solves A x = b (n x n, row-major, overwritten) by elimination with partial pivoting
// (the first row of largest magnitude); false when a pivot is exactly zero.
template <int N>
__device__ inline bool solve(double A[N][N], double b[N], double x[N]) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
        int p = c;
        double best = fabs(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < N; ++r)
            if (fabs(A[r][c]) > best) {
                best = fabs(A[r][c]);
                p = r;
            }
        // row swap by selects (constant indices keep the matrix in registers)
#pragma unroll
        for (int r = c + 1; r < N; ++r) {
            const bool sw = r == p;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const double t = A[c][k];
                A[c][k] = sw ? A[r][k] : t;
                A[r][k] = sw ? t : A[r][k];
            }
            const double t = b[c];
            b[c] = sw ? b[r] : t;
            b[r] = sw ? t : b[r];
        }
        if (A[c][c] == 0.0) return false;
#pragma unroll
        for (int r = c + 1; r < N; ++r) {
            const double f = A[r][c] / A[c][c];
#pragma unroll
            for (int k = c; k < N; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
#pragma unroll
    for (int r = N - 1; r >= 0; --r) {
        double s = b[r];
#pragma unroll
        for (int k = r + 1; k < N; ++k) s -= A[r][k] * x[k];
        x[r] = s / A[r][r];
    }
    return true;
}

// ---------------------------------------------------------------- 1. helix per track
// use[k]: bit0 the track is refit (its entries are usable -- sector in range, hits inside
// cap_hits, ids of clusters with row and sector in range -- and its helix is finite),
// bit1 it also takes part in merging.
//
// Entry check first, one wave per track index (its hit ids read together): ok[k] = 1
// when the sector is in range, the hits lie inside cap_hits and every id is of a
// cluster with row and sector in range.  (A wave walking several tracks waited on its
// store before each next track's loads: vector memory operations retire in order.)
__global__ __launch_bounds__(kBlock) void k_mg_valid(MgArgs a, uint8_t* __restrict__ ok) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t k = blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (k >= (uint32_t)n_tracks(a)) return;
    const int32_t o = __builtin_amdgcn_readfirstlane(a.off[k]), m = __builtin_amdgcn_readfirstlane(a.nh[k]);
    const int32_t s = __builtin_amdgcn_readfirstlane(a.tsec[k]);
    bool v = s >= 0 && s < a.S && o >= 0 && m > 0 && (int64_t)o + m <= (int64_t)a.cap_hits;
    if (v) {
        bool bad = false;
        for (int32_t j = (int32_t)lane; j < m; j += 64) {
            const int32_t id = a.ids[o + j];
            bad = bad || !(id >= 0 && (int64_t)id < a.n && a.row[id] < a.R && a.sector[id] < a.S);
        }
        v = __ballot(bad) == 0ull;
    }
    if (lane == 0) ok[k] = v ? 1 : 0;
}

// Helix per track (one lane each); the no-helix values (NaN) are written for unusable
// tracks below the track count.
__global__ __launch_bounds__(kBlock) void k_mg_helix(MgArgs a, const uint8_t* __restrict__ ok,
                                                     double* __restrict__ H, double* __restrict__ CH,
                                                     uint8_t* __restrict__ use, uint32_t* __restrict__ cell,
                                                     double* __restrict__ lo, double* __restrict__ hi,
                                                     float* __restrict__ rad, uint32_t* __restrict__ ccnt) {
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    const bool in = k < a.cap_tracks;
    uint8_t u = 0;
    uint32_t ck = 0;
    if (in) {
        double h[5], ch[15];
        for (int i = 0; i < 5; ++i) h[i] = NAN;
        for (int i = 0; i < 15; ++i) ch[i] = NAN;
        const bool listed = k < n_tracks(a);
        const bool valid = listed && ok[k];
        if (valid) {
            const int s = a.tsec[k];
            const double side = s >= a.sps ? -1.0 : 1.0;
            const double al = a.dphi * (double)(s % a.sps) + 0.5 * a.dphi;
            const float* st = a.state + 5 * (size_t)k;
            const double x = a.xref[k], y = st[0], z = st[1], sn = st[2], t = st[3], q = st[4];
            const double kq = a.kq, kap = kq * q;
            const double c = sqrt(fmax(1.0 - sn * sn, 0.0));
            const double phi = asin(sn) + al;
            const double ca = cos(al), sa = sin(al), sp = sin(phi), cp = cos(phi);
            const double X = x * ca - y * sa, Y = x * sa + y * ca;
            const double Xc = X - sp / kap, Yc = Y + cp / kap;
            const double tg = side * t, w = tg / kap;
            const double psi = atan2(Y - Yc, X - Xc);
            h[0] = Xc;
            h[1] = Yc;
            h[2] = fabs(kap);
            h[3] = w;
            h[4] = side * z - w * psi;
            // Jacobian d(Xc, Yc, k, w, z0) / d(y, z, sin phi, dz/ds, q/pT); psi moves with
            // phi, so d psi / d sin phi = 1 / cos phi
            double J[5][5] = {};
            const double k2 = kap * kap;
            J[0][0] = -sa;
            J[0][2] = -cp / (kap * c);
            J[0][4] = sp * kq / k2;
            J[1][0] = ca;
            J[1][2] = -sp / (kap * c);
            J[1][4] = -cp * kq / k2;
            J[2][4] = (double)((kap > 0.0) - (kap < 0.0)) * kq;
            J[3][3] = side / kap;
            J[3][4] = -tg * kq / k2;
            J[4][1] = side;
            J[4][2] = -w / c;
            J[4][3] = -psi * J[3][3];
            J[4][4] = -psi * J[3][4];
            const float* cv = a.cov + 15 * (size_t)k;
            double JC[5][5];
            for (int i = 0; i < 5; ++i)
                for (int j = 0; j < 5; ++j) {
                    double v = 0.0;
                    for (int l = 0; l < 5; ++l) v += J[i][l] * (double)cv[tri(l, j)];
                    JC[i][j] = v;
                }
            for (int i = 0; i < 5; ++i)
                for (int j = 0; j <= i; ++j) {
                    double v = 0.0;
                    for (int l = 0; l < 5; ++l) v += JC[i][l] * J[j][l];
                    ch[tri(i, j)] = v;
                }
            bool fin = true;
            for (int i = 0; i < 5; ++i) fin = fin && isfinite(h[i]);
            u = fin ? 1 : 0;
            if (fin && 1.0 / h[2] <= a.rho_max) {
                u = 3;
                const double M = (double)a.max_turns, pm = M_PI * M;
                const double v = fmax(ch[14], 0.0) + pm * pm * fmax(ch[9], 0.0) + 0.5 * a.floor2;
                double reach = pm * fabs(w) + a.n_sig * sqrt(v);
                reach = reach >= 0.0 ? reach * (1.0 + 1e-9) + 1e-9 * (fabs(h[4]) + 1.0) : INFINITY;
                lo[k] = h[4] - reach;
                hi[k] = h[4] + reach;
                // Prefilter radii: for a positive definite S = CA + CB, chi2 = d' S^-1 d >=
                // d_i^2 / S_ii, so a passing pair has |d_i| <= sqrt(chi2_max) (sA_i + sB_i).  Only
                // a track whose (Xc, Yc, k, w) block is positive definite (Cholesky) gets finite
                // radii: the sum of two such blocks is positive definite.
                bool pd = true;
                double L[4][4] = {};
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j <= i; ++j) {
                        double v = ch[tri(i, j)];
#pragma unroll
                        for (int l = 0; l < j; ++l) v -= L[i][l] * L[j][l];
                        if (i == j) {
                            pd = pd && v > 0.0;
                            L[i][i] = v > 0.0 ? sqrt(v) : 1.0;
                        } else {
                            L[i][j] = v / L[j][j];
                        }
                    }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double r = sqrt(a.chi2_max * ch[tri(i, i)]) * (1.0 + 1e-9);
                    float f = (float)r;
                    if ((double)f < r) f = nextafterf(f, INFINITY);
                    rad[4 * (size_t)k + i] = pd && r >= 0.0 ? f : INFINITY;
                }
                const double top = (double)(a.nc - 1);
                double fx = floor((Xc - a.cell_lo) / a.cell_w), fy = floor((Yc - a.cell_lo) / a.cell_w);
                fx = fx < 0.0 ? 0.0 : (fx > top ? top : fx);
                fy = fy < 0.0 ? 0.0 : (fy > top ? top : fy);
                ck = (uint32_t)fy * (uint32_t)a.nc + (uint32_t)fx;
                cell[k] = ck;
            }
        }
        if (listed) {
            for (int i = 0; i < 5; ++i) H[5 * (size_t)k + i] = h[i];
            for (int i = 0; i < 15; ++i) CH[15 * (size_t)k + i] = ch[i];
        }
        use[k] = u;
    }
    wave_inc(ccnt, ck, u == 3);
}

struct CKey {
    double lo;
    uint32_t k;
};
__device__ inline bool ckey_less(const CKey& p, const CKey& q) { return p.lo < q.lo || (p.lo == q.lo && p.k < q.k); }
struct CKeyLess {
    __device__ bool operator()(const CKey& p, const CKey& q) const { return ckey_less(p, q); }
};

__global__ __launch_bounds__(kBlock) void k_mg_scatter(MgArgs a, const uint8_t* __restrict__ use,
                                                       const uint32_t* __restrict__ cell,
                                                       const uint32_t* __restrict__ coff, uint32_t* __restrict__ ccur,
                                                       const double* __restrict__ lo, CKey* __restrict__ keys) {
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    const bool ok = k < a.cap_tracks && use[k] == 3;
    const uint32_t ck = ok ? cell[k] : 0u;
    const uint32_t slot = wave_inc(ccur, ck, ok);
    if (ok) keys[coff[ck] + slot] = CKey{lo[k], (uint32_t)k};
}

// ---------------------------------------------------------------- 2. cells sorted by interval start
// One workgroup per cell of at most kCellSortLds tracks: bitonic sort of (start, index)
// in LDS, padded with keys above every real one.
__global__ __launch_bounds__(kBlock) void k_mg_cell_sort(const uint32_t* __restrict__ ccnt,
                                                         const uint32_t* __restrict__ coff, CKey* __restrict__ gkeys,
                                                         unsigned long long* __restrict__ tally) {
    __shared__ CKey keys[kCellSortLds];
    const uint32_t cc = blockIdx.x;
    const uint32_t m = ccnt[cc], b = coff[cc];
    if (m == 0) return;
    if (threadIdx.x == 0) atomicMax(&tally[T_MAX_CELL], (unsigned long long)m);
    if (m > (uint32_t)kCellSortLds) {
        if (threadIdx.x == 0) atomicAdd(&tally[T_BIG_CELLS], 1ull);
        return;
    }
    uint32_t P = 1;
    while (P < m) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += kBlock) keys[i] = i < m ? gkeys[b + i] : CKey{INFINITY, UINT32_MAX};
    __syncthreads();
    for (uint32_t s = 2; s <= P; s <<= 1) {
        for (uint32_t j = s >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < P; i += kBlock) {
                const uint32_t o = i ^ j;
                if (o > i) {
                    const CKey u = keys[i], v = keys[o];
                    if ((i & s) == 0 ? ckey_less(v, u) : ckey_less(u, v)) {
                        keys[i] = v;
                        keys[o] = u;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < m; i += kBlock) gkeys[b + i] = keys[i];
}

// Cells longer than kCellSortLds (dense cells of low-momentum loopers in a time frame):
// the same network in global memory, one workgroup of 1024 lanes per cell.
__global__ __launch_bounds__(1024) void k_mg_cell_sort_big(const uint32_t* __restrict__ ccnt,
                                                           const uint32_t* __restrict__ coff, CKey* __restrict__ gkeys) {
    const uint32_t cc = blockIdx.x;
    const uint32_t m = ccnt[cc];
    if (m <= (uint32_t)kCellSortLds) return;
    flip_bitonic_sort(gkeys + coff[cc], m, CKeyLess{});
}

// Candidates of the cell positions, as arrays (read in sequence by the groups of the pair
// search, so consecutive lanes read consecutive entries): the interval start, the centre,
// (k, w), the prefilter radii of (Xc, Yc, k, w) (rounded up to FP32) and the track index.
struct Cands {
    double* lo;
    double2* xy;
    double2* kw;
    float4* r;
    uint32_t* idx;
};

__global__ __launch_bounds__(kBlock) void k_mg_records(const uint32_t* __restrict__ n_elig,
                                                       const CKey* __restrict__ keys, const double* __restrict__ H,
                                                       const float* __restrict__ rad, Cands cd) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= *n_elig) return;
    const CKey key = keys[i];
    const double* h = H + 5 * (size_t)key.k;
    const float* r = rad + 4 * (size_t)key.k;
    cd.lo[i] = key.lo;
    cd.xy[i] = make_double2(h[0], h[1]);
    cd.kw[i] = make_double2(h[2], h[3]);
    cd.r[i] = make_float4(r[0], r[1], r[2], r[3]);
    cd.idx[i] = key.k;
}

// ---------------------------------------------------------------- 3. same-helix test
__device__ bool same_helix(const MgArgs& a, const double* hA, const double* cA, const double* hB, const double* cB) {
    if (fabs(hA[0] - hB[0]) > a.win || fabs(hA[1] - hB[1]) > a.win) return false;
    double S[4][4], d[4], x[4], dd[4];
    for (int i = 0; i < 4; ++i) {
        d[i] = hA[i] - hB[i];
        dd[i] = d[i];
        for (int j = 0; j < 4; ++j) S[i][j] = cA[tri(i, j)] + cB[tri(i, j)];
    }
    if (!solve<4>(S, dd, x)) return false;
    const double chi2 = d[0] * x[0] + d[1] * x[1] + d[2] * x[2] + d[3] * x[3];
    if (!(chi2 <= a.chi2_max)) return false;
    const double pitch = 2.0 * M_PI * 0.5 * (hA[3] + hB[3]);
    const double dz0 = hA[4] - hB[4];
    if (!(fabs(pitch) > 0.0)) return fabs(dz0) <= a.n_sig * sqrt(cA[14] + cB[14] + a.floor2);
    const double m = rint(dz0 / pitch);
    if (fabs(m) > (double)a.max_turns) return false;
    const double dz = dz0 - m * pitch;
    const double pm = M_PI * m;
    const double var = cA[14] + cB[14] + pm * pm * (cA[9] + cB[9]) + a.floor2;
    return dz * dz <= a.n_sig * a.n_sig * var;
}

// ---------------------------------------------------------------- 4. union-find
__device__ inline int32_t uf_ld(const int32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void uf_st(int32_t* p, int32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Root of x, halving the path on the way (every link keeps pointing to a smaller index
// of the same tree, whatever other lanes do meanwhile).
__device__ inline int32_t uf_find(int32_t* par, int32_t x) {
    int32_t cur = uf_ld(par + x);
    if (cur != x) {
        int32_t prev = x, next;
        while (cur > (next = uf_ld(par + cur))) {
            uf_st(par + prev, next);
            prev = cur;
            cur = next;
        }
    }
    return cur;
}

__device__ inline void uf_unite(int32_t* par, int32_t a, int32_t b) {
    int32_t ra = uf_find(par, a), rb = uf_find(par, b);
    while (ra != rb) {
        if (ra < rb) {
            const int32_t t = ra;
            ra = rb;
            rb = t;
        }
        const int32_t old = atomicCAS(par + ra, ra, rb);  // the larger root under the smaller
        if (old == ra) return;
        ra = uf_find(par, old);
        rb = uf_find(par, rb);
    }
}

// A group of kPairGrp lanes per track A (tracks in cell order, a grid-stride walk).  The
// candidates of a neighbouring cell are the entries whose interval starts inside A's
// interval; lane g of the group takes the g-th, (g + kPairGrp)-th, ... of them.  A
// candidate passing the prefilter (centre window, and the marginal chi2 bounds on Xc, Yc,
// k and w) is queued for the full test: each lane appends to a chunk of kPairChunk
// entries that it reserves in one of kPairSegs queue segments (one atomic per chunk).
// The queued pairs are tested by the next kernel, one per lane, so the few lanes with a
// full test do not hold up the scan (and the scan keeps few registers).  A lane whose
// segment has no chunk left lists the tracks it could not queue for a rescan that tests
// every pair of theirs at once.  Chunk entries a lane leaves unused are marked empty.
constexpr uint32_t kPairGrp = 8, kPairChunk = 8, kPairSegs = 256, kSegStride = 32;
constexpr uint32_t kNoPair = 0xFFFFFFFFu;

// Scan of the candidates of track position i for lane g of its group: calls f(A, B) for
// every pair that passes the prefilter.
template <class F>
__device__ inline void scan_pairs(const MgArgs& a, const Cands& cd, const uint32_t* __restrict__ coff,
                                  const uint32_t* __restrict__ cell, const double* __restrict__ hi, uint32_t i,
                                  uint32_t g, F&& f) {
    const double win = a.win;
    const uint32_t A = cd.idx[i], ca = cell[A];
    const double loA = cd.lo[i], hiA = hi[A];
    const double2 xyA = cd.xy[i], kwA = cd.kw[i];
    const float4 rA = cd.r[i];
    const int cx = (int)(ca % (uint32_t)a.nc), cy = (int)(ca / (uint32_t)a.nc);
    for (int dy = -1; dy <= 1; ++dy) {
        const int y = cy + dy;
        if (y < 0 || y >= a.nc) continue;
        for (int dx = -1; dx <= 1; ++dx) {
            const int x = cx + dx;
            if (x < 0 || x >= a.nc) continue;
            const uint32_t cc = (uint32_t)y * (uint32_t)a.nc + (uint32_t)x;
            uint32_t b = coff[cc], e = coff[cc + 1];
            // first start >= loA (every lane of the group searches alike)
            while (b < e) {
                const uint32_t mid = b + (e - b) / 2;
                if (cd.lo[mid] < loA)
                    b = mid + 1;
                else
                    e = mid;
            }
            e = coff[cc + 1];
            for (uint32_t j = b + g; j < e; j += kPairGrp) {
                if (!(cd.lo[j] <= hiA)) break;
                const double2 xyB = cd.xy[j];
                const double ex = fabs(xyA.x - xyB.x), ey = fabs(xyA.y - xyB.y);
                if (!(ex <= win && ey <= win)) continue;
                const float4 rB = cd.r[j];
                const double2 kwB = cd.kw[j];
                const uint32_t B = cd.idx[j];
                const bool pre = B != A && ex <= (double)rA.x + (double)rB.x && ey <= (double)rA.y + (double)rB.y &&
                                 fabs(kwA.x - kwB.x) <= (double)rA.z + (double)rB.z &&
                                 fabs(kwA.y - kwB.y) <= (double)rA.w + (double)rB.w;
                if (pre) f(A, B);
            }
        }
    }
}

__device__ inline void test_pair(const MgArgs& a, uint32_t A, uint32_t B, const double* __restrict__ H,
                                 const double* __restrict__ CH, int32_t* __restrict__ par, uint64_t& passed) {
    const uint32_t p = A < B ? A : B, q = A < B ? B : A;
    if (same_helix(a, H + 5 * (size_t)p, CH + 15 * (size_t)p, H + 5 * (size_t)q, CH + 15 * (size_t)q)) {
        ++passed;
        uf_unite(par, (int32_t)A, (int32_t)B);
    }
}

__global__ __launch_bounds__(kBlock) void k_mg_pairs(MgArgs a, const uint32_t* __restrict__ n_elig, Cands cd,
                                                     const uint32_t* __restrict__ coff,
                                                     const uint32_t* __restrict__ cell, const double* __restrict__ hi,
                                                     uint2* __restrict__ pq, uint32_t seg_cap,
                                                     uint32_t* __restrict__ seg_fill, uint32_t* __restrict__ ovf_flag,
                                                     uint32_t* __restrict__ ovf, uint32_t* __restrict__ n_ovf,
                                                     unsigned long long* __restrict__ tally) {
    const uint32_t ne = *n_elig;
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t g = threadIdx.x % kPairGrp;
    const uint32_t n_grp = gridDim.x * (kBlock / kPairGrp);
    const uint32_t seg = gid % kPairSegs;
    uint2* const segq = pq + (size_t)seg * seg_cap;
    uint32_t qpos = 0, qend = 0;  // the lane's current chunk in its segment
    bool room = true;             // false once the segment had no chunk left for this lane
    uint64_t tested = 0;
    for (uint32_t i = gid / kPairGrp; i < ne; i += n_grp) {
        scan_pairs(a, cd, coff, cell, hi, i, g, [&](uint32_t A, uint32_t B) {
            ++tested;
            if (qpos == qend && room) {
                // chunks start at multiples of kPairChunk, and seg_cap is one: a chunk
                // either fits whole or starts at or past seg_cap
                const uint32_t c = atomicAdd(&seg_fill[seg * kSegStride], kPairChunk);
                room = c < seg_cap;
                qpos = c;
                qend = room ? c + kPairChunk : c;
            }
            if (qpos < qend)
                segq[qpos++] = make_uint2(A, B);
            else if (atomicOr(&ovf_flag[i], 1u) == 0u)
                ovf[atomicAdd(n_ovf, 1u)] = i;
        });
    }
    for (; qpos < qend; ++qpos) segq[qpos] = make_uint2(kNoPair, kNoPair);
    wave_tally(tally, T_PAIRS, tested);
}

// The queued pairs, one per lane (a grid-stride walk over the segments' filled chunks).
__global__ __launch_bounds__(kBlock) void k_mg_pair_tests(MgArgs a, const double* __restrict__ H,
                                                          const double* __restrict__ CH, const uint2* __restrict__ pq,
                                                          uint32_t seg_cap, const uint32_t* __restrict__ seg_fill,
                                                          int32_t* __restrict__ par,
                                                          unsigned long long* __restrict__ tally) {
    const uint64_t n = (uint64_t)seg_cap * kPairSegs;
    uint64_t passed = 0;
    for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (uint64_t)gridDim.x * kBlock) {
        const uint32_t seg = (uint32_t)(t / seg_cap), off = (uint32_t)(t % seg_cap);
        const uint32_t f = seg_fill[seg * kSegStride];
        if (off >= (f < seg_cap ? f : seg_cap)) continue;
        const uint2 pr = pq[t];
        if (pr.x != kNoPair) test_pair(a, pr.x, pr.y, H, CH, par, passed);
    }
    wave_tally(tally, T_PASSED, passed);
}

// Rescan of the listed tracks (a group per track), every prefilter pair tested at once.
// Pairs that were queued before the queue filled are tested a second time (the union
// is unchanged by that).
__global__ __launch_bounds__(kBlock) void k_mg_pairs_rescan(MgArgs a, Cands cd, const uint32_t* __restrict__ coff,
                                                            const uint32_t* __restrict__ cell,
                                                            const double* __restrict__ hi, const double* __restrict__ H,
                                                            const double* __restrict__ CH,
                                                            const uint32_t* __restrict__ ovf,
                                                            const uint32_t* __restrict__ n_ovf, int32_t* __restrict__ par,
                                                            unsigned long long* __restrict__ tally) {
    const uint32_t n = *n_ovf;
    const uint32_t g = threadIdx.x % kPairGrp;
    const uint32_t n_grp = gridDim.x * (kBlock / kPairGrp);
    uint64_t passed = 0;
    for (uint32_t k = (blockIdx.x * kBlock + threadIdx.x) / kPairGrp; k < n; k += n_grp)
        scan_pairs(a, cd, coff, cell, hi, ovf[k], g,
                   [&](uint32_t A, uint32_t B) { test_pair(a, A, B, H, CH, par, passed); });
    wave_tally(tally, T_PASSED, passed);
}

__global__ __launch_bounds__(kBlock) void k_mg_init(int32_t cap, int32_t* __restrict__ par) {
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k < cap) par[k] = k;
}

// Labels (the root of every track) and member counts per root.
__global__ __launch_bounds__(kBlock) void k_mg_label(MgArgs a, const uint8_t* __restrict__ use,
                                                     const int32_t* __restrict__ par, int32_t* __restrict__ label,
                                                     uint32_t* __restrict__ gcnt) {
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k >= a.cap_tracks) return;
    if (k >= n_tracks(a)) {
        label[k] = -1;
        return;
    }
    int32_t r = k;
    while (par[r] != r) r = par[r];
    label[k] = r;
    atomicAdd(&gcnt[r], 1u);
}

__global__ __launch_bounds__(kBlock) void k_mg_group(MgArgs a, const int32_t* __restrict__ label,
                                                     const uint32_t* __restrict__ goff, uint32_t* __restrict__ gcur,
                                                     int32_t* __restrict__ mem) {
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k >= n_tracks(a)) return;
    const int32_t r = label[k];
    mem[goff[r] + atomicAdd(&gcur[r], 1u)] = k;
}

// ---------------------------------------------------------------- 5. refit: the list
// Per hit of a component being fitted: its global position and the angle unwrapped at
// the start.  A component's hits are packed together (members in ascending index, each
// member's hits in its list order) from its item's hb on.
struct alignas(32) FitHit {
    double X, Y, Z, ps0;
};

// One component to fit: its root, its hit count and where its packed hits start.
struct FitItem {
    int32_t k;
    uint32_t nhit;
    uint64_t hb;
};

// Components of at least this many hits are fitted first (listed from the front of the
// fit list, the others from its back).
constexpr uint32_t kLargeFit = 1024;

// Members of each component in ascending index: insertion sort by one lane for components
// of at most kSmallComp members (nearly all); larger ones are listed for a workgroup sort.
// Roots of components of two or more usable members are listed for the refit with their
// packed hit range; every other track below the track count gets the no-fit outputs.
constexpr uint32_t kSmallComp = 64;

__global__ __launch_bounds__(kBlock) void k_mg_sort_members(
    MgArgs a, const uint8_t* __restrict__ use, const int32_t* __restrict__ label, const uint32_t* __restrict__ gcnt,
    const uint32_t* __restrict__ goff, int32_t* __restrict__ mem, int32_t* __restrict__ n_members,
    uint32_t* __restrict__ big, uint32_t* __restrict__ n_big, FitItem* __restrict__ fit, uint32_t* __restrict__ n_fit,
    double* __restrict__ theta, double* __restrict__ theta_cov, double* __restrict__ chi2_out,
    int32_t* __restrict__ ndf_out, unsigned long long* __restrict__ tally) {
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    const int lane = threadIdx.x & 63;
    const bool in = k < n_tracks(a);
    const bool root = in && label[k] == k;
    uint32_t m = 0;
    uint64_t hits = 0;
    if (root) {
        m = gcnt[k];
        int32_t* p = mem + goff[k];
        if (m > kSmallComp) {
            big[atomicAdd(n_big, 1u)] = (uint32_t)k;
        } else {
            for (uint32_t i = 1; i < m; ++i) {
                const int32_t v = p[i];
                uint32_t j = i;
                while (j > 0 && p[j - 1] > v) {
                    p[j] = p[j - 1];
                    --j;
                }
                p[j] = v;
            }
        }
        if (m >= 2 && (use[k] & 1))
            for (uint32_t i = 0; i < m; ++i) hits += (uint64_t)a.nh[p[i]];
    }
    // more hits than 2^31 in one component only with overlapping hit lists: no fit
    const bool fitted = root && m >= 2 && (use[k] & 1) && hits < (1ull << 31);
    uint32_t tot;
    const uint32_t pre = wave_excl_scan(fitted ? (uint32_t)hits : 0u, tot);
    const bool large = fitted && hits >= kLargeFit;
    const uint64_t bl = __ballot(large), bs = __ballot(fitted && !large);
    unsigned long long hb0 = 0;
    uint32_t l0 = 0, s0 = 0;
    if (lane == 0) {
        if (tot) hb0 = atomicAdd(&tally[T_FIT_HITS], (unsigned long long)tot);
        if (bl) l0 = atomicAdd(&n_fit[0], (uint32_t)__popcll(bl));
        if (bs) s0 = atomicAdd(&n_fit[1], (uint32_t)__popcll(bs));
    }
    hb0 = __shfl(hb0, 0, 64);
    l0 = __shfl(l0, 0, 64);
    s0 = __shfl(s0, 0, 64);
    const uint64_t below = (1ull << lane) - 1ull;
    if (fitted) {
        const uint32_t slot = large ? l0 + (uint32_t)__popcll(bl & below)
                                    : (uint32_t)a.cap_tracks - 1u - (s0 + (uint32_t)__popcll(bs & below));
        fit[slot] = FitItem{k, (uint32_t)hits, (uint64_t)hb0 + pre};
    } else if (in) {  // no fit at this index
        for (int p = 0; p < 5; ++p) theta[5 * (size_t)k + p] = NAN;
        for (int i = 0; i < 15; ++i) theta_cov[15 * (size_t)k + i] = NAN;
        chi2_out[k] = NAN;
        ndf_out[k] = 0;
    }
    if (k < a.cap_tracks) n_members[k] = root ? (int32_t)m : 0;
    wave_tally(tally, T_COMPONENTS, root ? 1u : 0u);
    wave_tally(tally, T_MERGED, m >= 2 ? 1u : 0u);
}

struct IntLess {
    __device__ bool operator()(int32_t p, int32_t q) const { return p < q; }
};

// The listed large components, one workgroup each (bitonic sort in global memory).
__global__ __launch_bounds__(1024) void k_mg_sort_big(const uint32_t* __restrict__ big,
                                                      const uint32_t* __restrict__ n_big,
                                                      const uint32_t* __restrict__ gcnt,
                                                      const uint32_t* __restrict__ goff, int32_t* __restrict__ mem) {
    const uint32_t nb = *n_big;
    for (uint32_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const uint32_t k = big[i];
        flip_bitonic_sort(mem + goff[k], gcnt[k], IntLess{});
        __syncthreads();
    }
}

// ---------------------------------------------------------------- 5. refit: the fit
// Sums over a component's n packed hits at th (every lane ends with the same totals):
// chi2, and with `normal` also the normal matrix (lower triangle) and gradient.  Hit f
// belongs to lane f mod 64, which also wrote it.
// The residual derivatives are jt = (-dx/r, -dy/r, -1, 0, 0) (transverse) and
// jz = (-w dy/r^2, w dx/r^2, 0, -1, -psi) (longitudinal), so N22 = wy n, N33 = wz n and
// N32 = N42 = 0 need no sums; the other eleven entries, the gradient and chi2 are summed.
__device__ inline void fit_sums(const FitHit* __restrict__ fh, uint32_t n, const double th[5], double wy,
                                double wz, bool normal, double& chi2, double N[15], double g[5]) {
    const uint32_t lane = threadIdx.x & 63;
    double s[17];
#pragma unroll
    for (int i = 0; i < 17; ++i) s[i] = 0.0;
    const double tau = 2.0 * M_PI, itau = 1.0 / tau;
#pragma unroll 1
    for (uint32_t f = lane; f < n; f += 64) {
        const FitHit h = fh[f];
        const double dx = h.X - th[0], dy = h.Y - th[1];
        const double r = hypot(dx, dy);
        const double d = atan2(dy, dx) - h.ps0;
        const double ps = h.ps0 + (d - tau * rint(d * itau));
        const double rt = r - th[2], rz = h.Z - th[3] - th[4] * ps;
        s[0] += wy * rt * rt + wz * rz * rz;
        if (normal) {
            const double ir = 1.0 / r;
            const double ja = -dx * ir, jb = -dy * ir;
            const double jc = -th[4] * dy * ir * ir, jd = th[4] * dx * ir * ir;
            const double wzps = wz * ps;
            s[1] += wy * ja * ja + wz * jc * jc;  // N00
            s[2] += wy * ja * jb + wz * jc * jd;  // N10
            s[3] += wy * jb * jb + wz * jd * jd;  // N11
            s[4] -= wy * ja;                      // N20
            s[5] -= wy * jb;                      // N21
            s[6] -= wz * jc;                      // N30
            s[7] -= wz * jd;                      // N31
            s[8] -= wzps * jc;                    // N40
            s[9] -= wzps * jd;                    // N41
            s[10] += wzps;                        // N43
            s[11] += wzps * ps;                   // N44
            s[12] += wy * ja * rt + wz * jc * rz; // g0
            s[13] += wy * jb * rt + wz * jd * rz; // g1
            s[14] -= wy * rt;                     // g2
            s[15] -= wz * rz;                     // g3
            s[16] -= wzps * rz;                   // g4
        }
    }
    chi2 = wave_sum_d(s[0]);
    if (normal) {
#pragma unroll
        for (int i = 1; i < 17; ++i) s[i] = wave_sum_d(s[i]);
        const double nd = (double)n;
        N[tri(0, 0)] = s[1];
        N[tri(1, 0)] = s[2];
        N[tri(1, 1)] = s[3];
        N[tri(2, 0)] = s[4];
        N[tri(2, 1)] = s[5];
        N[tri(2, 2)] = wy * nd;
        N[tri(3, 0)] = s[6];
        N[tri(3, 1)] = s[7];
        N[tri(3, 2)] = 0.0;
        N[tri(3, 3)] = wz * nd;
        N[tri(4, 0)] = s[8];
        N[tri(4, 1)] = s[9];
        N[tri(4, 2)] = 0.0;
        N[tri(4, 3)] = s[10];
        N[tri(4, 4)] = s[11];
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = s[12 + i];
    }
}

// Fits one component (the calling wave): places its hits with their starting turn, then
// Gauss-Newton from the root's helix.
__device__ void fit_component(const MgArgs& a, const FitItem& it, const double* __restrict__ sec_cs,
                              const uint32_t* __restrict__ gcnt, const uint32_t* __restrict__ goff,
                              const int32_t* __restrict__ mem, const double* __restrict__ H, FitHit* __restrict__ fhc,
                              double* __restrict__ theta, double* __restrict__ theta_cov,
                              double* __restrict__ chi2_out, int32_t* __restrict__ ndf_out,
                              unsigned long long* __restrict__ tally) {
    const int lane = threadIdx.x & 63;
    const int32_t k = it.k;
    const double tau = 2.0 * M_PI;
    const double* h0 = H + 5 * (size_t)k;
    double th[5] = {h0[0], h0[1], 1.0 / h0[2], h0[4], h0[3]};
    const int32_t* mk = mem + goff[k];
    const uint32_t m = gcnt[k];
    uint32_t base = 0;
    for (uint32_t mi = 0; mi < m; ++mi) {
        const int32_t t = mk[mi];
        const int32_t o = a.off[t], nt = a.nh[t];
        const double* hh = H + 5 * (size_t)t;
        // this lane writes the component's hits f = base + j with f = lane mod 64
        const int32_t j0 = (int32_t)(((uint32_t)lane + 64u - (base & 63u)) & 63u);
        for (int32_t j = j0; j < nt; j += 64) {
            const int32_t id = a.ids[o + j];
            const int s = a.sector[id];
            const double x = (double)a.row_x[a.row[id]], y = (double)a.y[id];
            const double ca = sec_cs[2 * s], sa = sec_cs[2 * s + 1];
            FitHit f;
            f.X = x * ca - y * sa;
            f.Y = x * sa + y * ca;
            f.Z = (s >= a.sps ? -1.0 : 1.0) * (double)a.z[id];
            const double psi = atan2(f.Y - th[1], f.X - th[0]);
            double turns = 0.0;
            if (th[4] != 0.0) {
                const double own =
                    rint((f.Z - hh[4] - hh[3] * atan2(f.Y - hh[1], f.X - hh[0])) / (tau * hh[3]));
                const double shift = rint((hh[4] - th[3]) / (tau * th[4]));
                const double b = own + shift;
                const double z_of = th[3] + th[4] * (psi + tau * b);
                turns = b + rint((f.Z - z_of) / (tau * th[4]));
            }
            f.ps0 = psi + tau * turns;
            fhc[base + (uint32_t)j] = f;
        }
        base += (uint32_t)nt;
    }
    const uint32_t n = it.nhit;
    double chi2, N[15], g[5];
    fit_sums(fhc, n, th, a.wy, a.wz, false, chi2, N, g);
    bool failed = false;
    for (int iter = 0; iter < a.max_iter; ++iter) {
        double c2;
        fit_sums(fhc, n, th, a.wy, a.wz, true, c2, N, g);
        double A[5][5], b[5], step[5];
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            b[p] = -g[p];
#pragma unroll
            for (int q = 0; q < 5; ++q) A[p][q] = N[tri(p, q)];
        }
        if (!solve<5>(A, b, step)) {
            failed = true;
            break;
        }
        bool accepted = false;
        double cand[5];
        for (int h = 0; h < 30; ++h) {
            for (int p = 0; p < 5; ++p) cand[p] = th[p] + step[p];
            fit_sums(fhc, n, cand, a.wy, a.wz, false, c2, N, g);
            if (c2 <= chi2) {
                accepted = true;
                break;
            }
            for (int p = 0; p < 5; ++p) step[p] = 0.5 * step[p];
        }
        if (!accepted) break;
        const bool done = chi2 - c2 <= 1e-12 * chi2;
        for (int p = 0; p < 5; ++p) th[p] = cand[p];
        chi2 = c2;
        if (done) break;
    }
    // covariance: the inverse of the normal matrix at the result, column c solved by lane c
    // (the elimination depends on the matrix only, so every lane fails or succeeds alike)
    double c2;
    fit_sums(fhc, n, th, a.wy, a.wz, true, c2, N, g);
    {
        double A[5][5], b[5], x[5];
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            b[p] = p == lane ? 1.0 : 0.0;
#pragma unroll
            for (int q = 0; q < 5; ++q) A[p][q] = N[tri(p, q)];
        }
        failed = failed || !solve<5>(A, b, x);
        if (lane < 5)
#pragma unroll
            for (int p = 0; p < 5; ++p)
                if (p >= lane) theta_cov[15 * (size_t)k + tri(p, lane)] = failed ? NAN : x[p];
    }
    if (lane == 0) {
        for (int p = 0; p < 5; ++p) theta[5 * (size_t)k + p] = failed ? NAN : th[p];
        chi2_out[k] = failed ? NAN : chi2;
        ndf_out[k] = (int32_t)(2 * (int64_t)n - 5 < INT32_MAX ? 2 * (int64_t)n - 5 : INT32_MAX);
        if (failed) atomicAdd(&tally[T_FAILED], 1ull);
    }
}

// Work counters of the refit, one per group of workgroups (blockIdx mod 8, the XCD a
// workgroup is dispatched to), each on a line of its own.
constexpr int kFitCtrs = 8, kFitCtrStride = 32;

// Persistent refit: each wave takes the next item of its counter's share of the fit
// list (item i belongs to counter i mod 8), large components first.  The sector angles'
// cos and sin are the helix kernel's expressions, kept in LDS.  A component whose packed
// hits would pass the end of the fit-hit buffer (possible only with overlapping hit
// lists) gets no fit and counts as failed.
__global__ __launch_bounds__(kBlock) void k_mg_refit(MgArgs a, const FitItem* __restrict__ fit,
                                                     const uint32_t* __restrict__ n_fit, uint32_t* __restrict__ ctr,
                                                     const uint32_t* __restrict__ gcnt,
                                                     const uint32_t* __restrict__ goff, const int32_t* __restrict__ mem,
                                                     const double* __restrict__ H, FitHit* __restrict__ fh,
                                                     uint64_t fh_cap, double* __restrict__ theta,
                                                     double* __restrict__ theta_cov, double* __restrict__ chi2_out,
                                                     int32_t* __restrict__ ndf_out,
                                                     unsigned long long* __restrict__ tally) {
    __shared__ double sec_cs[2 * 256];
    for (int s = threadIdx.x; s < a.S; s += kBlock) {
        const double al = a.dphi * (double)(s % a.sps) + 0.5 * a.dphi;
        sec_cs[2 * s] = cos(al);
        sec_cs[2 * s + 1] = sin(al);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint32_t grp = blockIdx.x % kFitCtrs;
    const uint32_t nl = n_fit[0], nf = nl + n_fit[1];
    // The loop's control is wave-uniform by construction (read from the first lane): every
    // lane takes part in the ticket atomic (lane 0 adds one, the others zero) and no branch
    // depends on the lane, so the compiler cannot split the wave's lanes over different
    // iterations around the cross-lane sums of the fit.
    for (;;) {
        const uint32_t t = atomicAdd(&ctr[grp * kFitCtrStride], lane == 0 ? 1u : 0u);
        const uint32_t j = __builtin_amdgcn_readfirstlane(t);
        const uint64_t i = (uint64_t)grp + (uint64_t)kFitCtrs * j;
        if (i >= nf) break;
        const FitItem raw = fit[i < nl ? i : (uint64_t)a.cap_tracks - 1u - (i - nl)];
        FitItem it;
        it.k = __builtin_amdgcn_readfirstlane(raw.k);
        it.nhit = __builtin_amdgcn_readfirstlane(raw.nhit);
        it.hb = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(raw.hb >> 32)) << 32) |
                (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)raw.hb);
        if (it.hb + it.nhit <= fh_cap) {
            fit_component(a, it, sec_cs, gcnt, goff, mem, H, fh + it.hb, theta, theta_cov, chi2_out, ndf_out, tally);
        } else {
            if (lane < 5) theta[5 * (size_t)it.k + lane] = NAN;
            if (lane < 15) theta_cov[15 * (size_t)it.k + lane] = NAN;
            if (lane == 0) {
                chi2_out[it.k] = NAN;
                ndf_out[it.k] = 0;
                atomicAdd(&tally[T_FAILED], 1ull);
            }
        }
    }
}

__global__ void k_mg_counts(const unsigned long long* __restrict__ tally, int64_t* __restrict__ counts) {
    if (threadIdx.x != 0) return;
    counts[TPC_MG_COMPONENTS] = (int64_t)tally[T_COMPONENTS];
    counts[TPC_MG_MERGED] = (int64_t)tally[T_MERGED];
    counts[TPC_MG_PAIRS_TESTED] = (int64_t)tally[T_PAIRS];
    counts[TPC_MG_PAIRS_PASSED] = (int64_t)tally[T_PASSED];
    counts[TPC_MG_MAX_CELL] = (int64_t)tally[T_MAX_CELL];
    counts[TPC_MG_BIG_CELLS] = (int64_t)tally[T_BIG_CELLS];
    counts[TPC_MG_REFIT_FAILED] = (int64_t)tally[T_FAILED];
}

inline unsigned nblk(int64_t n, int per = kBlock) { return (unsigned)(n > 0 ? (n + per - 1) / per : 1); }

#define MB(field, name, bytes)                              \
    field = (decltype(field))buf(c, name, (size_t)(bytes)); \
    if (!field) return TPC_ERR_HIP;

}  // namespace

int merge_run(tpc_ctx_t* c, const tpc_clusters_t& cl, const GridDesc& g, double kq, double sigma_y, double sigma_z,
              double max_row_x, const tpc_merge_params_t& mp, const tpc_tracks_t& trk, tpc_merged_t& out,
              hipStream_t st) {
    const int64_t T = trk.cap_tracks > 0 ? trk.cap_tracks : 1;
    const int64_t NH = trk.cap_hits > 0 ? trk.cap_hits : 1;
    MgArgs a{};
    a.tcounts = trk.counts;
    a.cap_tracks = trk.cap_tracks;
    a.cap_hits = trk.cap_hits;
    a.off = trk.hit_offset;
    a.nh = trk.n_hits;
    a.ids = trk.hit_ids;
    a.tsec = trk.sector;
    a.xref = trk.x_ref;
    a.state = trk.state;
    a.cov = trk.cov;
    a.n = cl.n;
    a.y = cl.y;
    a.z = cl.z;
    a.row = cl.row;
    a.sector = cl.sector;
    a.row_x = g.row_x;
    a.R = g.R;
    a.S = g.S;
    a.sps = mp.sectors_per_side;
    a.dphi = 2.0 * M_PI / (double)mp.sectors_per_side;
    a.kq = kq;
    a.rho_max = mp.rho_max;
    a.win = mp.centre_window;
    a.chi2_max = mp.chi2_max;
    a.n_sig = mp.phase_sigmas;
    a.floor2 = mp.phase_floor * mp.phase_floor;
    a.max_turns = mp.max_turns;
    // cells a little wider than the window, so centres within the window always fall in
    // neighbouring cells despite rounding; centres beyond the grid go to its edge cells
    a.cell_w = mp.centre_window * (1.0 + 1e-9);
    const double reach = max_row_x * std::sqrt(2.0) + mp.rho_max + mp.centre_window;
    int64_t nc = (int64_t)std::ceil(2.0 * reach / a.cell_w);
    nc = nc < 1 ? 1 : (nc > 4096 ? 4096 : nc);
    a.nc = (int)nc;
    a.cell_lo = -0.5 * (double)nc * a.cell_w;
    a.wy = 1.0 / (sigma_y * sigma_y);
    a.wz = 1.0 / (sigma_z * sigma_z);
    a.max_iter = mp.max_iter;
    const int64_t NC = nc * nc;
    uint8_t* use;
    uint32_t *cell, *ccnt, *coff, *ccur, *gcnt, *goff, *gcur, *n_elig, *big;
    int32_t *par, *mem;
    double *lo, *hi;
    float* rad;
    CKey* keys;
    Cands cd;
    uint2* pq;
    uint32_t *seg_fill, *ovf_flag, *ovf;
    FitHit* fh;
    FitItem* fit;
    uint32_t* fctr;
    unsigned long long* tally;
    void* scan;
    MB(use, "mg_use", T);
    uint8_t* ok;
    MB(ok, "mg_ok", T);
    MB(cell, "mg_cell", 4 * T);
    MB(ccnt, "mg_ccnt", 4 * (NC + 1));
    MB(coff, "mg_coff", 4 * (NC + 1));
    MB(ccur, "mg_ccur", 4 * (NC + 1));
    MB(keys, "mg_keys", sizeof(CKey) * T);
    MB(cd.lo, "mg_c_lo", 8 * T);
    MB(cd.xy, "mg_c_xy", 16 * T);
    MB(cd.kw, "mg_c_kw", 16 * T);
    MB(cd.r, "mg_c_r", 16 * T);
    MB(cd.idx, "mg_c_idx", 4 * T);
    // pair queue: pair_queue pairs per track slot, in kPairSegs segments of whole chunks
    const int64_t qcap = (int64_t)mp.pair_queue * T;
    const uint32_t seg_cap =
        qcap > 0 ? (uint32_t)((qcap / kPairSegs + kPairChunk - 1) / kPairChunk * kPairChunk) : 0u;
    MB(pq, "mg_pair_queue", sizeof(uint2) * ((size_t)seg_cap * kPairSegs + 1));
    MB(seg_fill, "mg_pair_fill", 4 * kPairSegs * kSegStride);
    MB(ovf_flag, "mg_pair_ovf_flag", 4 * T);
    MB(ovf, "mg_pair_ovf", 4 * T);
    MB(rad, "mg_rad", 16 * T);
    MB(lo, "mg_lo", 8 * T);
    MB(hi, "mg_hi", 8 * T);
    MB(par, "mg_par", 4 * T);
    MB(gcnt, "mg_gcnt", 4 * (T + 1));
    MB(goff, "mg_goff", 4 * (T + 1));
    MB(gcur, "mg_gcur", 4 * (T + 1));
    MB(mem, "mg_mem", 4 * T);
    MB(big, "mg_big", 4 * T);
    MB(n_elig, "mg_nelig", 32);
    MB(fh, "mg_fithits", sizeof(FitHit) * NH);
    MB(fit, "mg_fitlist", sizeof(FitItem) * T);
    MB(fctr, "mg_fitctr", 4 * kFitCtrs * kFitCtrStride);
    MB(tally, "mg_tally", 8 * T_N);
    int64_t sn = NC + 1 > T + 1 ? NC + 1 : T + 1;
    MB(scan, "mg_scan", scan_scratch_bytes(sn));
    // [0] eligible tracks (scan total), [1] large components, [2] [3] fit items, [4] tracks
    // to rescan for pairs
    fill_u32(n_elig, 0u, 8, st);
    fill_u32(fctr, 0u, kFitCtrs * kFitCtrStride, st);
    fill_u32(seg_fill, 0u, kPairSegs * kSegStride, st);
    fill_u32(ovf_flag, 0u, T, st);
    fill_u32(ccnt, 0u, NC + 1, st);
    fill_u32(ccur, 0u, NC + 1, st);
    fill_u32(gcnt, 0u, T + 1, st);
    fill_u32(gcur, 0u, T + 1, st);
    fill_u64((uint64_t*)tally, 0ull, T_N, st);
    const unsigned nb = nblk(T);
    k_mg_valid<<<nblk(T, kBlock / 64), kBlock, 0, st>>>(a, ok);
    k_mg_helix<<<nb, kBlock, 0, st>>>(a, ok, out.helix, out.helix_cov, use, cell, lo, hi, rad, ccnt);
    scan_u32(ccnt, coff, NC + 1, nullptr, n_elig, scan, st);
    k_mg_scatter<<<nb, kBlock, 0, st>>>(a, use, cell, coff, ccur, lo, keys);
    k_mg_cell_sort<<<(unsigned)NC, kBlock, 0, st>>>(ccnt, coff, keys, tally);
    k_mg_cell_sort_big<<<(unsigned)NC, 1024, 0, st>>>(ccnt, coff, keys);
    k_mg_records<<<nb, kBlock, 0, st>>>(n_elig, keys, out.helix, rad, cd);
    k_mg_init<<<nb, kBlock, 0, st>>>(trk.cap_tracks, par);
    k_mg_pairs<<<(unsigned)(c->n_cu * 16), kBlock, 0, st>>>(a, n_elig, cd, coff, cell, hi, pq, seg_cap, seg_fill,
                                                          ovf_flag, ovf, n_elig + 4, tally);
    k_mg_pair_tests<<<(unsigned)(c->n_cu * 16), kBlock, 0, st>>>(a, out.helix, out.helix_cov, pq, seg_cap, seg_fill, par,
                                                               tally);
    k_mg_pairs_rescan<<<(unsigned)(c->n_cu * 4), kBlock, 0, st>>>(a, cd, coff, cell, hi, out.helix, out.helix_cov, ovf,
                                                                n_elig + 4, par, tally);
    k_mg_label<<<nb, kBlock, 0, st>>>(a, use, par, out.label, gcnt);
    scan_u32(gcnt, goff, T, nullptr, nullptr, scan, st);
    k_mg_group<<<nb, kBlock, 0, st>>>(a, out.label, goff, gcur, mem);
    k_mg_sort_members<<<nb, kBlock, 0, st>>>(a, use, out.label, gcnt, goff, mem, out.n_members, big, n_elig + 1,
                                              fit, n_elig + 2, out.theta, out.theta_cov, out.chi2, out.ndf, tally);
    k_mg_sort_big<<<256, 1024, 0, st>>>(big, n_elig + 1, gcnt, goff, mem);
    // a whole number of counter groups, a few workgroups per CU
    const unsigned fit_blocks = (unsigned)((c->n_cu * 8 + kFitCtrs - 1) / kFitCtrs * kFitCtrs);
    k_mg_refit<<<fit_blocks, kBlock, 0, st>>>(a, fit, n_elig + 2, fctr, gcnt, goff, mem, out.helix, fh, (uint64_t)NH,
                                              out.theta, out.theta_cov, out.chi2, out.ndf, tally);
    k_mg_counts<<<1, 64, 0, st>>>(tally, out.counts);
    return TPC_OK;
}

#undef MB

}  // namespace tpc
