// Tracklet construction and following (sector-local helix model, Kalman filter).
//
// One lane per start hit.  Pass A starts at the start hit with the slope of its
// first link, follows the cleaned chain upward while the chain hit passes the
// chi2 cut, then searches each further row for the nearest hit (smallest chi2
// inside the chi2 ellipse's bounding box, ties by cluster id).  Pass B restarts
// at the outermost pass-A hit with pass A's direction and curvature and runs
// inward, re-using the pass-A hits and following below the start row; its state
// at the innermost hit is the tracklet's.
//
// The filter runs in FP64: MI355X executes FP64 vector FMA at half the FP32
// rate, and this kernel is bound by dependent gather latency, not arithmetic.
// FP64 makes every arg-min and cut decision agree with an FP64 reference except
// at genuine near-ties.
//
// Work distribution: a persistent grid; each wave pops `chunk` x 64 tracklets
// from an atomic queue, so long tracklets do not stall a statically assigned
// block.  Results do not depend on which lane builds which tracklet.
//
// Per-tracklet hit slot of n_rows entries: pass A appends ascending from the
// front, pass B writes its hits from the back (descending rows), so the final
// list is slot[R - n_hits .. R) in ascending rows; pass B only overwrites
// pass-A entries it has already consumed.
#include "tpc_device.h"
#include "tpc_internal.h"

namespace tpc {

namespace {

__device__ inline void asin_over(double u, double& g, double& gp) {
    if (fabs(u) < 1e-2) {
        const double u2 = u * u;
        g = 1.0 + u2 * (1.0 / 6.0 + u2 * (3.0 / 40.0 + u2 * (5.0 / 112.0 + u2 * (35.0 / 1152.0))));
        gp = u * (1.0 / 3.0 + u2 * (3.0 / 10.0 + u2 * (15.0 / 56.0 + u2 * (35.0 / 144.0))));
    } else {
        const double a = asin(u);
        g = a / u;
        gp = (u / sqrt(1.0 - u * u) - a) / (u * u);
    }
}

// symmetric element (i, j) of the packed lower triangle
#define CS(i, j) C[((i) >= (j)) ? ((i) * ((i) + 1) / 2 + (j)) : ((j) * ((j) + 1) / 2 + (i))]

// Propagate state and covariance from x0 to x1.  false = |sin phi| reached s_max.
__device__ inline bool propagate(double p[5], double C[15], double x0, double x1, const KParams& kp) {
    const double dx = x1 - x0;
    const double k = kp.kq * p[4];
    const double s0 = p[2], s1 = s0 + k * dx;
    if (!(fabs(s1) < kp.s_max) || !(fabs(s0) < kp.s_max)) return false;
    if (dx == 0.0) return true;
    const double c0 = sqrt(1.0 - s0 * s0), c1 = sqrt(1.0 - s1 * s1);
    const double A = s0 + s1, B = c0 + c1;
    const double dy = dx * A / B;
    const double L = copysign(sqrt(dx * dx + dy * dy), dx);
    const double u = 0.5 * k * L;
    double g, gp;
    asin_over(u, g, gp);
    const double arc = L * g;
    const double t = p[3];
    // Jacobian: F = I + {(0,2)=a, (0,4)=b, (1,2)=c, (1,3)=d, (1,4)=e, (2,4)=f}
    const double iB2 = 1.0 / (B * B);
    const double dB_s = -s0 / c0 - s1 / c1, dA_q = kp.kq * dx, dB_q = -(s1 / c1) * kp.kq * dx;
    const double a = dx * (2.0 * B - A * dB_s) * iB2;
    const double b = dx * (dA_q * B - A * dB_q) * iB2;
    const double dL_s = dy / L * a, dL_q = dy / L * b;
    const double du_s = 0.5 * k * dL_s, du_q = 0.5 * kp.kq * L + 0.5 * k * dL_q;
    const double c = t * (dL_s * g + L * gp * du_s);
    const double d = arc;
    const double e = t * (dL_q * g + L * gp * du_q);
    const double f = kp.kq * dx;
    p[0] += dy;
    p[1] += t * arc;
    p[2] = s1;
    // G = F C
    double G[5][5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        G[0][j] = CS(0, j) + a * CS(2, j) + b * CS(4, j);
        G[1][j] = CS(1, j) + c * CS(2, j) + d * CS(3, j) + e * CS(4, j);
        G[2][j] = CS(2, j) + f * CS(4, j);
        G[3][j] = CS(3, j);
        G[4][j] = CS(4, j);
    }
    // C' = G F^T (lower triangle)
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const double r0 = G[i][0] + a * G[i][2] + b * G[i][4];
        const double r1 = G[i][1] + c * G[i][2] + d * G[i][3] + e * G[i][4];
        const double r2 = G[i][2] + f * G[i][4];
        const double rr[5] = {r0, r1, r2, G[i][3], G[i][4]};
#pragma unroll
        for (int j = 0; j <= i; ++j) C[i * (i + 1) / 2 + j] = rr[j];
    }
    return true;
}

__device__ inline double chi2_of(const double p[5], const double C[15], double my, double mz, const KParams& kp) {
    const double syy = C[0] + kp.vy, syz = C[1], szz = C[2] + kp.vz;
    const double det = syy * szz - syz * syz;
    const double ry = my - p[0], rz = mz - p[1];
    return (ry * ry * szz - 2.0 * ry * rz * syz + rz * rz * syy) / det;
}

// Kalman update; false = fit failure.
__device__ inline bool kf_update(double p[5], double C[15], double my, double mz, const KParams& kp, double& chi2) {
    const double syy = C[0] + kp.vy, syz = C[1], szz = C[2] + kp.vz;
    const double det = syy * szz - syz * syz;
    const double i00 = szz / det, i01 = -syz / det, i11 = syy / det;
    const double ry = my - p[0], rz = mz - p[1];
    chi2 = ry * (i00 * ry + i01 * rz) + rz * (i01 * ry + i11 * rz);
    const double c0[5] = {C[0], C[1], C[3], C[6], C[10]};
    const double c1[5] = {C[1], C[2], C[4], C[7], C[11]};
    double K0[5], K1[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        K0[i] = c0[i] * i00 + c1[i] * i01;
        K1[i] = c0[i] * i01 + c1[i] * i11;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) p[i] += K0[i] * ry + K1[i] * rz;
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) C[i * (i + 1) / 2 + j] -= K0[i] * c0[j] + K1[i] * c1[j];
    bool ok = det > 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) ok = ok && isfinite(p[i]);
#pragma unroll
    for (int i = 0; i < 15; ++i) ok = ok && isfinite(C[i]);
    ok = ok && C[0] > 0.0 && C[2] > 0.0 && C[5] > 0.0 && C[9] > 0.0 && C[14] > 0.0;
    return ok;
}

// Nearest hit in row r of sector s: smallest chi2 <= cut inside the ellipse's box.
__device__ inline int32_t search_row(const GridDesc& g, const KParams& kp, const Hit* __restrict__ hits,
                                     const uint32_t* __restrict__ bin_off, int s, int r, const double p[5],
                                     const double C[15]) {
    const double syy = C[0] + kp.vy, syz = C[1], szz = C[2] + kp.vz;
    const double det = syy * szz - syz * syz;
    const double i00 = szz / det, i01 = -syz / det, i11 = syy / det;
    const double bx = sqrt(kp.fol_cut * syy), bz = sqrt(kp.fol_cut * szz);
    if (!(det > 0.0) || !isfinite(bx) || !isfinite(bz)) return -1;
    const BinRange br = bin_range(g, s, r, p[0] - bx, p[0] + bx, p[1] - bz, p[1] + bz);
    if (br.empty) return -1;
    double best = 1e300;
    uint32_t best_id = 0xFFFFFFFFu;
    int32_t best_pos = -1;
    for (int iz = br.iz0; iz <= br.iz1; ++iz) {
        const uint32_t k1 = bin_off[br.base + iz * br.ny + br.iy1 + 1];
        for (uint32_t k = bin_off[br.base + iz * br.ny + br.iy0]; k < k1; ++k) {
            const Hit h = hits[k];
            const double ry = (double)h.y - p[0], rz = (double)h.z - p[1];
            if (fabs(ry) > bx || fabs(rz) > bz) continue;
            const double c2 = ry * (i00 * ry + i01 * rz) + rz * (i01 * ry + i11 * rz);
            if (!(c2 <= kp.fol_cut)) continue;
            if (c2 < best || (c2 == best && h.id < best_id)) {
                best = c2;
                best_id = h.id;
                best_pos = (int32_t)k;
            }
        }
    }
    return best_pos;
}

__device__ inline void c0_init(double C[15], const KParams& kp) {
#pragma unroll
    for (int i = 0; i < 15; ++i) C[i] = 0.0;
    C[0] = kp.vy;
    C[2] = kp.vz;
    C[5] = kp.c0s;
    C[9] = kp.c0t;
    C[14] = kp.c0q;
}

// Builds tracklet k; returns bit0 = valid, bit1 = fit failure.
__device__ uint32_t build_one(uint32_t k, const GridDesc& g, const KParams& kp, const Hit* __restrict__ hits,
                              const uint32_t* __restrict__ bin_off, const int32_t* __restrict__ upc,
                              const uint32_t* __restrict__ starts, const TrackletOut& o) {
    const int R = g.R;
    const uint32_t p0 = starts[k];
    const Hit h0 = hits[p0];
    const int s = (int)(h0.rs / (uint32_t)R), r0 = (int)(h0.rs % (uint32_t)R);
    int32_t* slot = o.hits + (size_t)k * R;
    const double tanh_ = kp.tan_half;
    // ---- pass A
    const int32_t p1 = upc[p0];
    const Hit h1 = hits[p1];
    const double x0 = g.row_x[r0], x1 = g.row_x[h1.rs % (uint32_t)R];
    const double ty = ((double)h1.y - (double)h0.y) / (x1 - x0);
    const double tz = ((double)h1.z - (double)h0.z) / (x1 - x0);
    double p[5], C[15];
    p[0] = h0.y;
    p[1] = h0.z;
    p[2] = ty / sqrt(1.0 + ty * ty);
    p[3] = tz * sqrt(1.0 - p[2] * p[2]);
    p[4] = 0.0;
    c0_init(C, kp);
    slot[0] = (int32_t)p0;
    int nA = 1, last = r0;
    double pl2 = p[2], pl3 = p[3], pl4 = p[4];
    int32_t next = p1;
    bool on = true, fail = false;
    int miss = 0;
    double x = x0;
    for (int r = r0 + 1; r < R; ++r) {
        const double xr = g.row_x[r];
        if (!propagate(p, C, x, xr, kp)) break;
        x = xr;
        if (fabs(p[0]) > x * tanh_ + kp.edge) break;
        int32_t acc = -1;
        Hit ha;
        if (on) {
            if (next >= 0) {
                const Hit hn = hits[next];
                if ((int)(hn.rs % (uint32_t)R) == r && chi2_of(p, C, hn.y, hn.z, kp) <= kp.fol_cut) {
                    acc = next;
                    ha = hn;
                    next = upc[next];
                } else {
                    on = false;
                }
            } else {
                on = false;
            }
        }
        if (acc < 0) {
            acc = search_row(g, kp, hits, bin_off, s, r, p, C);
            if (acc >= 0) ha = hits[acc];
        }
        if (acc >= 0) {
            double c2;
            if (!kf_update(p, C, ha.y, ha.z, kp, c2)) {
                fail = true;
                break;
            }
            slot[nA++] = acc;
            last = r;
            pl2 = p[2];
            pl3 = p[3];
            pl4 = p[4];
            miss = 0;
        } else if (++miss > kp.n_miss) {
            break;
        }
    }
    // ---- pass B
    int nB = 0, inner = last, ndf = 0;
    double chi2 = 0.0;
    double pin[5], cin[15];
    if (!fail) {
        const int32_t pb = slot[nA - 1];
        const Hit hb = hits[pb];
        p[0] = hb.y;
        p[1] = hb.z;
        p[2] = pl2;
        p[3] = pl3;
        p[4] = pl4;
        c0_init(C, kp);
        slot[R - 1] = pb;
        nB = 1;
#pragma unroll
        for (int i = 0; i < 5; ++i) pin[i] = p[i];
#pragma unroll
        for (int i = 0; i < 15; ++i) cin[i] = C[i];
        x = g.row_x[last];
        miss = 0;
        int ia = nA - 2;
        for (int r = last - 1; r >= 0; --r) {
            const double xr = g.row_x[r];
            if (!propagate(p, C, x, xr, kp)) break;
            x = xr;
            if (fabs(p[0]) > x * tanh_ + kp.edge) break;
            int32_t acc = -1;
            Hit ha;
            if (r >= r0) {
                if (ia >= 0) {
                    const int32_t pa = slot[ia];
                    const Hit hp = hits[pa];
                    if ((int)(hp.rs % (uint32_t)R) == r) {
                        acc = pa;
                        ha = hp;
                        --ia;
                    }
                }
            } else {
                acc = search_row(g, kp, hits, bin_off, s, r, p, C);
                if (acc >= 0) ha = hits[acc];
            }
            if (acc >= 0) {
                double c2;
                if (!kf_update(p, C, ha.y, ha.z, kp, c2)) {
                    fail = true;
                    break;
                }
                chi2 += c2;
                ndf += 2;
                slot[R - 1 - nB] = acc;
                ++nB;
                inner = r;
#pragma unroll
                for (int i = 0; i < 5; ++i) pin[i] = p[i];
#pragma unroll
                for (int i = 0; i < 15; ++i) cin[i] = C[i];
                miss = 0;
            } else if (++miss > kp.n_miss) {
                break;
            }
        }
    }
    const bool valid = !fail && nB >= kp.n_min_tl;
    o.nhits[k] = fail ? 0 : nB;
    o.chi2[k] = (float)chi2;
    o.ndf[k] = ndf;
    o.row_ref[k] = inner;
    o.flags[k] = (valid ? 1u : 0u) | (fail ? 2u : 0u);
#pragma unroll
    for (int i = 0; i < 5; ++i) o.state[(size_t)k * 5 + i] = fail ? 0.f : (float)pin[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) o.cov[(size_t)k * 15 + i] = fail ? 0.f : (float)cin[i];
    return (valid ? 1u : 0u) | (fail ? 2u : 0u);
}

constexpr int kTlBlock = 128;

__global__ __launch_bounds__(kTlBlock) void k_tracklets(GridDesc g, KParams kp, const Hit* __restrict__ hits,
                                                        const uint32_t* __restrict__ bin_off,
                                                        const int32_t* __restrict__ upc,
                                                        const uint32_t* __restrict__ starts,
                                                        uint32_t* __restrict__ counters, TrackletOut o, int chunk) {
    const uint32_t n = counters[C_N_STARTS];
    const int lane = threadIdx.x & 63;
    uint32_t n_valid = 0, n_fail = 0;
    while (true) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&counters[C_QUEUE_TL], 64u * (uint32_t)chunk);
        base = __shfl(base, 0, 64);
        if (base >= n) break;
        for (int c = 0; c < chunk; ++c) {
            const uint32_t k = base + (uint32_t)c * 64u + (uint32_t)lane;
            if (k < n) {
                const uint32_t f = build_one(k, g, kp, hits, bin_off, upc, starts, o);
                n_valid += f & 1u;
                n_fail += (f >> 1) & 1u;
            }
        }
    }
    __shared__ uint32_t sv[kTlBlock / 64], sf[kTlBlock / 64];
    const uint32_t wv = wave_sum(n_valid), wf = wave_sum(n_fail);
    if (lane == 0) {
        sv[threadIdx.x >> 6] = wv;
        sf[threadIdx.x >> 6] = wf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tv = 0, tf = 0;
        for (int i = 0; i < kTlBlock / 64; ++i) {
            tv += sv[i];
            tf += sf[i];
        }
        if (tv) atomicAdd(&counters[C_N_VALID_TL], tv);
        if (tf) atomicAdd(&counters[C_N_FAIL], tf);
    }
}

}  // namespace

void build_tracklets(const GridDesc& g, const KParams& kp, const Hit* hits, const uint32_t* bin_off,
                     const int32_t* upc, const uint32_t* starts, uint32_t* counters, const TrackletOut& o,
                     int grid_blocks, int chunk, hipStream_t s) {
    k_tracklets<<<grid_blocks, kTlBlock, 0, s>>>(g, kp, hits, bin_off, upc, starts, counters, o, chunk);
}

}  // namespace tpc
