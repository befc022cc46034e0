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
// Work distribution: a persistent grid of waves; each lane runs its tracklet as a
// small state machine (pass A row, pass B row, finished) and takes a new
// tracklet from an atomic queue as soon as its current one ends, so the wave
// stays busy until the queue is empty.  Results do not depend on which lane
// builds which tracklet.
//
// Per-tracklet hit slot of n_rows entries: pass A appends ascending from the
// front, pass B writes its hits from the back (descending rows), so the final
// list is slot[R - n_hits .. R) in ascending rows; pass B only overwrites
// pass-A entries it has already consumed.
#include "tpc_device.h"
#include "tpc_internal.h"

namespace tpc {

namespace {

// 1/x from the hardware estimate refined by two Newton-Raphson steps
// (r <- r + r(1 - x r)); each step squares the relative error, so the result is
// within an ulp or two of the rounded quotient.  x = 0 gives NaN; every caller's
// divisor is positive (c = cos phi > 0, B > 0, L != 0, det > 0 or rejected by the
// caller's own det > 0 test).
__device__ inline double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// sqrt(x) for x >= 0 by Goldschmidt's iteration on the hardware 1/sqrt estimate
// (s ~ sqrt(x), h ~ 1/(2 sqrt(x)) refined together), then two Newton corrections
// of s from the residual x - s^2.
__device__ inline double sqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y, h = 0.5 * y;
    const double e = fma(-s, h, 0.5);
    s = fma(s, e, s);
    h = fma(h, e, h);
    double d = fma(-s, s, x);
    s = fma(d, h, s);
    d = fma(-s, s, x);
    s = fma(d, h, s);
    return x == 0.0 ? 0.0 : s;
}

// 1/sqrt(x) for x > 0: the hardware estimate and two Newton-Raphson steps
// (r <- r (3 - x r^2) / 2); x < 0 gives NaN.
__device__ inline double rsq_pos(double x) {
    double r = __builtin_amdgcn_rsq(x);
    r = r * fma(-0.5 * x, r * r, 1.5);
    return r * fma(-0.5 * x, r * r, 1.5);
}

// g(u) = asin(u)/u and g'(u).  Row steps keep |u| = |k L / 2| well below 0.05
// (0.02 for the lowest momenta), where the Maclaurin series of asin(u)/u to u^12
// is exact to rounding (the first omitted term is below 1e-18 relative).  Larger
// |u| (fit states far from any real track) are first brought below 0.05 by the
// half-angle identity asin(u) = 2 asin(u / sqrt(2 (1 + sqrt(1 - u^2)))), at most
// five times for |u| <= 1; |u| > 1 gives NaN, as asin does.
__device__ inline double asin_series(double u2) {  // asin(u)/u as a series in u^2
    return 1.0 + u2 * (1.0 / 6.0 + u2 * (3.0 / 40.0 + u2 * (5.0 / 112.0 + u2 * (35.0 / 1152.0 +
           u2 * (63.0 / 2816.0 + u2 * (231.0 / 13312.0))))));
}

__device__ inline void asin_over(double u, double& g, double& gp) {
    const double u2 = u * u;
    if (fabs(u) < 0.05) {
        g = asin_series(u2);
        gp = u * (1.0 / 3.0 + u2 * (3.0 / 10.0 + u2 * (15.0 / 56.0 + u2 * (35.0 / 144.0 +
             u2 * (315.0 / 1408.0 + u2 * (693.0 / 3328.0 + u2 * (1001.0 / 5120.0)))))));
    } else {
        double v = u, m = 1.0;
        for (int i = 0; i < 8 && fabs(v) >= 0.05; ++i) {
            v *= rsq_pos(2.0 * (1.0 + sqrt_pos(1.0 - v * v)));
            m *= 2.0;
        }
        const double a = m * v * asin_series(v * v);  // asin(u); NaN for |u| > 1
        const double iu = rcp(u);
        g = a * iu;
        gp = (u * rsq_pos(1.0 - u2) - a) * iu * iu;
    }
}

// Propagate state and covariance from x0 to x1.  false = |sin phi| reached s_max;
// then p and C hold meaningless values (the caller ends the pass and discards
// them), which keeps this free of branches.
__device__ inline bool propagate(double p[5], double C[15], double x0, double x1, const KParams& kp) {
    const double dx = x1 - x0;
    const double k = kp.kq * p[4];
    const double s0 = p[2], s1 = s0 + k * dx;
    const bool ok = fabs(s1) < kp.s_max && fabs(s0) < kp.s_max;
    if (dx == 0.0) return ok;
    const double c0 = sqrt_pos(1.0 - s0 * s0), c1 = sqrt_pos(1.0 - s1 * s1);
    const double A = s0 + s1, B = c0 + c1;
    const double iB = rcp(B);
    const double dy = dx * A * iB;
    const double L = copysign(sqrt_pos(dx * dx + dy * dy), dx);
    const double u = 0.5 * k * L;
    double g, gp;
    asin_over(u, g, gp);
    const double arc = L * g;
    const double t = p[3];
    // Jacobian: F = I + {(0,2)=a, (0,4)=b, (1,2)=c, (1,3)=d, (1,4)=e, (2,4)=f}
    const double iB2 = iB * iB;
    const double t1 = s1 * rcp(c1);
    const double dB_s = -s0 * rcp(c0) - t1, dA_q = kp.kq * dx, dB_q = -t1 * kp.kq * dx;
    const double a = dx * (2.0 * B - A * dB_s) * iB2;
    const double b = dx * (dA_q * B - A * dB_q) * iB2;
    const double dyL = dy * rcp(L);
    const double dL_s = dyL * a, dL_q = dyL * b;
    const double du_s = 0.5 * k * dL_s, du_q = 0.5 * kp.kq * L + 0.5 * k * dL_q;
    const double c = t * (dL_s * g + L * gp * du_s);
    const double d = arc;
    const double e = t * (dL_q * g + L * gp * du_q);
    const double f = kp.kq * dx;
    p[0] += dy;
    p[1] += t * arc;
    p[2] = s1;
    // C' = F C F^T with F = I + {(0,2)=a, (0,4)=b, (1,2)=c, (1,3)=d, (1,4)=e, (2,4)=f}, written
    // element by element on the packed lower triangle (index i(i+1)/2 + j): rows 3 and 4 of F C
    // equal those of C, and each new element is formed while the old ones it needs are still there.
    const double C00 = C[0], C10 = C[1], C11 = C[2], C20 = C[3], C21 = C[4], C22 = C[5];
    const double C30 = C[6], C31 = C[7], C32 = C[8], C33 = C[9];
    const double C40 = C[10], C41 = C[11], C42 = C[12], C43 = C[13], C44 = C[14];
    // rows of N = F C that differ from C (only the columns the products below need)
    const double n00 = C00 + a * C20 + b * C40, n02 = C20 + a * C22 + b * C42, n04 = C40 + a * C42 + b * C44;
    const double n10 = C10 + c * C20 + d * C30 + e * C40, n11 = C11 + c * C21 + d * C31 + e * C41;
    const double n12 = C21 + c * C22 + d * C32 + e * C42, n13 = C31 + c * C32 + d * C33 + e * C43;
    const double n14 = C41 + c * C42 + d * C43 + e * C44;
    const double n20 = C20 + f * C40, n21 = C21 + f * C41, n22 = C22 + f * C42, n23 = C32 + f * C43;
    const double n24 = C42 + f * C44;
    C[0] = n00 + a * n02 + b * n04;
    C[1] = n10 + a * n12 + b * n14;
    C[2] = n11 + c * n12 + d * n13 + e * n14;
    C[3] = n20 + a * n22 + b * n24;
    C[4] = n21 + c * n22 + d * n23 + e * n24;
    C[5] = n22 + f * n24;
    C[6] = C30 + a * C32 + b * C43;
    C[7] = C31 + c * C32 + d * C33 + e * C43;
    C[8] = C32 + f * C43;
    C[10] = C40 + a * C42 + b * C44;
    C[11] = C41 + c * C42 + d * C43 + e * C44;
    C[12] = C42 + f * C44;
    return ok;
}

__device__ inline double chi2_of(const double p[5], const double C[15], double my, double mz, const KParams& kp) {
    const double syy = C[0] + kp.vy, syz = C[1], szz = C[2] + kp.vz;
    const double det = syy * szz - syz * syz;
    const double ry = my - p[0], rz = mz - p[1];
    return (ry * ry * szz - 2.0 * ry * rz * syz + rz * rz * syy) * rcp(det);
}

// Kalman update; false = fit failure.
__device__ inline bool kf_update(double p[5], double C[15], double my, double mz, const KParams& kp, double& chi2) {
    const double syy = C[0] + kp.vy, syz = C[1], szz = C[2] + kp.vz;
    const double det = syy * szz - syz * syz;
    const double idet = rcp(det);
    const double i00 = szz * idet, i01 = -syz * idet, i11 = syy * idet;
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
    for (int i = 0; i < 5; ++i) ok &= (bool)isfinite(p[i]);
#pragma unroll
    for (int i = 0; i < 15; ++i) ok &= (bool)isfinite(C[i]);
    ok &= (C[0] > 0.0) & (C[2] > 0.0) & (C[5] > 0.0) & (C[9] > 0.0) & (C[14] > 0.0);
    return ok;
}

// Nearest hit in one row: smallest chi2 <= cut inside the ellipse's box, ties by
// cluster id; -1 if none.  The winner's coordinates come back in (hy, hz).  Loads
// run ahead of their use: the next z row's bin bounds while this row's hits are
// tested, and the first four candidates of a bin range in one go (a range rarely
// holds more), so a row search waits for two loads in sequence, not one per hit.
struct Best {
    double c2;
    uint32_t id;
    int32_t pos;
    float y, z;
};

__device__ inline void consider(Best& b, const TlHit& h, uint32_t k, bool valid, const double p[5], double bx,
                                double bz, double i00, double i01, double i11, double cut) {
    const double ry = (double)h.y - p[0], rz = (double)h.z - p[1];
    const double c2 = ry * (i00 * ry + i01 * rz) + rz * (i01 * ry + i11 * rz);
    // bitwise, not short-circuit: no branches inside the candidate loop
    const bool take = valid & (fabs(ry) <= bx) & (fabs(rz) <= bz) & (c2 <= cut) &
                      ((c2 < b.c2) | ((c2 == b.c2) & (h.id < b.id)));
    b.c2 = take ? c2 : b.c2;
    b.id = take ? h.id : b.id;
    b.pos = take ? (int32_t)k : b.pos;
    b.y = take ? h.y : b.y;
    b.z = take ? h.z : b.z;
}

__device__ inline int32_t search_row(const GridDesc& g, const KParams& kp, const TlHit* __restrict__ hits,
                                     const uint32_t* __restrict__ bin_off, const RowBins& rb, const double p[5],
                                     const double C[15], float& hy, float& hz) {
    const double syy = C[0] + kp.vy, syz = C[1], szz = C[2] + kp.vz;
    const double det = syy * szz - syz * syz;
    const double idet = rcp(det);
    const double i00 = szz * idet, i01 = -syz * idet, i11 = syy * idet;
    const double bx = sqrt_pos(kp.fol_cut * syy), bz = sqrt_pos(kp.fol_cut * szz);
    if (!(det > 0.0) || !isfinite(bx) || !isfinite(bz)) return -1;
    const BinRange br = bin_range(g, rb, p[0] - bx, p[0] + bx, p[1] - bz, p[1] + bz);
    if (br.empty) return -1;
    Best b{1e300, 0xFFFFFFFFu, -1, hy, hz};
    const double cut = kp.fol_cut;
    uint32_t zrow = br.base + br.iz0 * br.ny;
    uint32_t kb = bin_off[zrow + br.iy0], ke = bin_off[zrow + br.iy1 + 1];
    for (int iz = br.iz0; iz <= br.iz1; ++iz) {
        uint32_t nb = 0, ne = 0;
        if (iz < br.iz1) {
            zrow += br.ny;
            nb = bin_off[zrow + br.iy0];
            ne = bin_off[zrow + br.iy1 + 1];
        }
        if (kb < ke) {
            const uint32_t last = ke - 1;
            const TlHit h0 = hits[kb];
            const TlHit h1 = hits[kb + 1 < last ? kb + 1 : last];
            const TlHit h2 = hits[kb + 2 < last ? kb + 2 : last];
            const TlHit h3 = hits[kb + 3 < last ? kb + 3 : last];
            consider(b, h0, kb, true, p, bx, bz, i00, i01, i11, cut);
            consider(b, h1, kb + 1, kb + 1 < ke, p, bx, bz, i00, i01, i11, cut);
            consider(b, h2, kb + 2, kb + 2 < ke, p, bx, bz, i00, i01, i11, cut);
            consider(b, h3, kb + 3, kb + 3 < ke, p, bx, bz, i00, i01, i11, cut);
            for (uint32_t k = kb + 4; k < ke; ++k) consider(b, hits[k], k, true, p, bx, bz, i00, i01, i11, cut);
        }
        kb = nb;
        ke = ne;
    }
    hy = b.y;
    hz = b.z;
    return b.pos;
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

// Per-row tables in LDS (the same for every sector: bins of sector s, row r start
// at s * bins_per_sector + base[r]).
struct RowTab {
    const float* x;
    const float* ymin;
    const int32_t* ny;
    const uint32_t* base;
    uint32_t per_sector;
};

__device__ inline RowBins row_bins_lds(const RowTab& rt, int s, int r) {
    return RowBins{(double)rt.ymin[r], rt.ny[r], (uint32_t)s * rt.per_sector + rt.base[r]};
}

// Per-lane tracklet state between row steps.
// Rarely touched per-lane values live in LDS, not registers: pass A's direction
// and curvature at its outermost hit, pass B's state at its innermost hit and its
// chi2 sum, and the slot chunk being filled.  The register state is kept to what
// every row step reads, and the x of the state's row is taken from the row table
// rather than kept, so the kernel fits three waves per SIMD without spills.
struct Spare {
    double pl[3];      // pass A at its outermost hit: sin phi, dz/ds, q/pT
    float ly, lz;      // that hit's coordinates
    int32_t lpos;      // and grid position
    float pin[5], cin[15];
    double chi2;       // pass B's chi2 sum
    int32_t w[8];      // the slot's current aligned 8-entry chunk, stored once complete
};

// Start of one tracklet, precomputed in processing order (three 16-byte loads).
struct alignas(16) Seed {
    uint32_t k;        // start index
    int32_t p0, p1;    // grid positions of the start hit and its cleaned upward link
    uint32_t rs;       // sector * n_rows + row of the start hit
    float y0, z0;
    uint32_t pad0, pad1;
    double s0, t0;     // initial sin phi and dz/ds from the first link
};

struct Lane {
    int phase;  // 0 needs work, 1 pass A, 2 pass B, 3 retired
    uint32_t k;
    int s, r0, r, edge, nh, ia, miss;  // edge: last row of pass A, then innermost row of pass B;
                                       // nh: hits of the current pass (pass B's ndf is 2 (nh - 1))
    int32_t link;  // pass A: the chain's next hit; pass B: position of pass A's hit number ia
                   // (loaded one step ahead)
    bool on, fail;
    double p[5], C[15];
    Spare* sp;
};

__device__ inline void save_inner(Lane& L) {
#pragma unroll
    for (int i = 0; i < 5; ++i) L.sp->pin[i] = (float)L.p[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) L.sp->cin[i] = (float)L.C[i];
}

__device__ inline void save_dir(Lane& L, float hy, float hz, int32_t pos) {
    L.sp->pl[0] = L.p[2];
    L.sp->pl[1] = L.p[3];
    L.sp->pl[2] = L.p[4];
    L.sp->ly = hy;
    L.sp->lz = hz;
    L.sp->lpos = pos;
}

// Slot entries are collected per aligned chunk of kSlotChunk and stored as two
// 16-byte writes when the chunk is complete (or the pass ends), so a slot line is
// touched once per eight hits instead of once per hit (fewer partial lines leaving
// L2).  Needs 32-byte aligned slots (n_rows a multiple of kSlotChunk); otherwise
// entries are stored one by one.  Entries outside [0, nA) in pass A and
// [R - nB, R) in pass B are never read, so a partly filled chunk may be stored with
// stale values.
constexpr int kSlotChunk = 8;

__device__ inline void slot_flush(const Lane& L, int32_t* slot, int idx, bool wide) {
    if (!wide) return;
    int4* c = (int4*)(slot + (idx & ~(kSlotChunk - 1)));
    c[0] = make_int4(L.sp->w[0], L.sp->w[1], L.sp->w[2], L.sp->w[3]);
    c[1] = make_int4(L.sp->w[4], L.sp->w[5], L.sp->w[6], L.sp->w[7]);
}

__device__ inline void slot_put(Lane& L, int32_t* slot, int idx, int32_t v, bool wide, bool last_in_chunk) {
    if (!wide) {
        slot[idx] = v;
        return;
    }
    L.sp->w[idx & (kSlotChunk - 1)] = v;
    if (last_in_chunk) slot_flush(L, slot, idx, true);
}

__device__ inline void start_pass_a(Lane& L, const Seed& sd, const GridDesc& g, const RowTab& rt, const KParams& kp,
                                    const TrackletOut& o) {
    const int R = g.R;
    L.k = sd.k;
    L.s = (int)(sd.rs / (uint32_t)R);
    L.r0 = (int)(sd.rs % (uint32_t)R);
    L.p[0] = sd.y0;
    L.p[1] = sd.z0;
    L.p[2] = sd.s0;
    L.p[3] = sd.t0;
    L.p[4] = 0.0;
    c0_init(L.C, kp);
    slot_put(L, o.hits + (size_t)sd.k * R, 0, sd.p0, (R & (kSlotChunk - 1)) == 0, false);
    L.nh = 1;
    L.edge = L.r0;
    save_dir(L, sd.y0, sd.z0, sd.p0);
    L.link = sd.p1;
    L.on = true;
    L.fail = false;
    L.miss = 0;
    L.r = L.r0 + 1;
    L.phase = 1;
}

__device__ inline void start_pass_b(Lane& L, const GridDesc& g, const RowTab& rt, const KParams& kp,
                                    const TrackletOut& o) {
    const int R = g.R;
    int32_t* slot = o.hits + (size_t)L.k * R;
    const int32_t pb = L.sp->lpos;
    L.p[0] = L.sp->ly;
    L.p[1] = L.sp->lz;
    L.p[2] = L.sp->pl[0];
    L.p[3] = L.sp->pl[1];
    L.p[4] = L.sp->pl[2];
    c0_init(L.C, kp);
    const bool wide = (R & (kSlotChunk - 1)) == 0;
    if ((L.nh & (kSlotChunk - 1)) != 0) slot_flush(L, slot, L.nh - 1, wide);  // pass A's last, partial chunk
    slot_put(L, slot, R - 1, pb, wide, ((R - 1) & (kSlotChunk - 1)) == 0);
    L.ia = L.nh - 2;
    L.nh = 1;
    L.sp->chi2 = 0.0;
    save_inner(L);
    L.miss = 0;
    L.link = L.ia >= 0 ? slot[L.ia] : -1;
    L.r = L.edge - 1;
    L.phase = 2;
}

// Writes the tracklet's outputs; returns bit0 = valid, bit1 = fit failure.
__device__ inline uint32_t finish(Lane& L, int R, const KParams& kp, const TrackletOut& o) {
    const bool fail = L.fail;
    if (L.phase == 2 && !fail && ((R - L.nh) & (kSlotChunk - 1)) != 0)
        slot_flush(L, o.hits + (size_t)L.k * R, R - L.nh, (R & (kSlotChunk - 1)) == 0);
    const int nB = fail ? 0 : L.nh;
    const bool valid = !fail && nB >= kp.n_min_tl;
    const uint32_t k = L.k;
    o.nhits[k] = nB;
    o.chi2[k] = fail ? 0.f : (float)L.sp->chi2;
    o.ndf[k] = fail ? 0 : 2 * (nB - 1);
    o.row_ref[k] = L.edge;
    o.flags[k] = (valid ? 1u : 0u) | (fail ? 2u : 0u);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float v = L.sp->pin[i];
        o.state[(size_t)k * 5 + i] = fail ? 0.f : v;
    }
#pragma unroll
    for (int i = 0; i < 15; ++i) {
        const float v = L.sp->cin[i];
        o.cov[(size_t)k * 15 + i] = fail ? 0.f : v;
    }
    L.phase = 0;
    return (valid ? 1u : 0u) | (fail ? 2u : 0u);
}

// One row of the lane's current pass (A upward, B inward); true when the pass has
// ended.  Both passes share one propagation, one row search and one filter update,
// so a wave whose lanes are in different passes issues each of them once per row.
//   pass A: take the next chain hit if it lies on this row and passes the chi2 cut,
//           else (and for the rest of the pass) search the row;
//   pass B: rows at or above the start row re-use pass A's hit on that row (if any),
//           rows below it are searched.
__device__ inline bool step(Lane& L, const GridDesc& g, const RowTab& rt, const KParams& kp,
                            const TlHit* __restrict__ hits, const uint32_t* __restrict__ bin_off,
                            const uint32_t* __restrict__ row_off, const TrackletOut& o) {
    // Straight-line: every lane runs the same instructions and results are blended
    // with selects; only the row search and the filter update are branches.  Values
    // a lane computes after its pass has ended are discarded by the caller.
    const int R = g.R;
    const bool A = L.phase == 1;
    const int r = L.r;
    bool end = A ? r >= R : r < 0;
    const int rc = r < 0 ? 0 : (r >= R ? R - 1 : r);
    int32_t* slot = o.hits + (size_t)L.k * R;
    // Loads that do not depend on the propagated state go out before it is computed:
    // the hit this row may take without a search (the next chain hit in pass A, pass
    // A's hit on this row in pass B) with its upward link, and in pass B the slot
    // entry of the pass-A hit after it.
    const double xr = rt.x[rc];
    const RowBins rb = row_bins_lds(rt, L.s, rc);
    const int32_t cand = A ? (L.on ? L.link : -1) : ((r >= L.r0 && L.ia >= 0) ? L.link : -1);
    const int32_t cc = cand < 0 ? 0 : cand;
    const TlHit hc = hits[cc];
    const int32_t cand_up = hc.upc;
    // pass B: is pass A's hit on this row (its position inside the row's range)?  In
    // pass A the candidate is the upward link of the previous row's hit, always on this
    // row (links join adjacent rows), while the chain lasts.
    const uint32_t* ro = row_off + (size_t)L.s * R + rc;
    const uint32_t rlo = A ? 0u : ro[0], rhi = A ? 0u : ro[1];
    const int ia1 = L.ia < 1 ? 0 : (L.ia > R ? R - 1 : L.ia - 1);
    const int32_t pf_next = A ? -1 : slot[ia1];  // pass A lanes load nothing (no slot lines into L2)
    // x of the row the state is at: the row before this one in the pass's direction
    const double x0 = rt.x[A ? r - 1 : r + 1];
    end = end || !propagate(L.p, L.C, x0, xr, kp);
    end = end || fabs(L.p[0]) > xr * kp.tan_half + kp.edge;
    const bool on_row = (cand >= 0) & (A | (((uint32_t)cand >= rlo) & ((uint32_t)cand < rhi)));
    const bool link = A & L.on & on_row & (chi2_of(L.p, L.C, hc.y, hc.z, kp) <= kp.fol_cut);
    const bool reused = !A & on_row;
    L.on = A ? link : L.on;
    L.link = link ? cand_up : L.link;
    L.ia = reused ? L.ia - 1 : L.ia;
    L.link = reused ? pf_next : L.link;
    int32_t acc = (link || reused) ? cand : -1;
    float hy = hc.y, hz = hc.z;
    if (!end && (A ? !link : r < L.r0)) acc = search_row(g, kp, hits, bin_off, rb, L.p, L.C, hy, hz);
    const bool has = !end && acc >= 0;
    bool ok = true;
    double c2 = 0.0;
    if (has) ok = kf_update(L.p, L.C, hy, hz, kp, c2);
    const bool good = has && ok;
    L.r = A ? r + 1 : r - 1;
    L.miss = good ? 0 : L.miss + 1;
    L.fail = L.fail || (has && !ok);
    end = end || (has && !ok) || (!has && L.miss > kp.n_miss);
    if (good) {
        // pass A appends from the front of the slot, pass B from the back; the saved
        // direction only matters in pass A and the saved inner state only in pass B
        const int idx = A ? L.nh : R - 1 - L.nh;
        slot_put(L, slot, idx, acc, (R & (kSlotChunk - 1)) == 0,
                 A ? (idx & (kSlotChunk - 1)) == kSlotChunk - 1 : (idx & (kSlotChunk - 1)) == 0);
        L.nh += 1;
        L.edge = r;
        if (!A) L.sp->chi2 += c2;
        save_dir(L, hy, hz, acc);
        save_inner(L);
    }
    return end;
}

constexpr int kTlBlock = 128;

__global__ __launch_bounds__(kBlock) void k_seeds(GridDesc g, const Hit* __restrict__ hits,
                                                  const int32_t* __restrict__ upc, const uint32_t* __restrict__ starts,
                                                  const uint32_t* __restrict__ proc,
                                                  const uint32_t* __restrict__ counters, Seed* __restrict__ seeds) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= counters[C_N_STARTS]) return;
    const int R = g.R;
    Seed sd;
    sd.k = proc[j];
    sd.p0 = (int32_t)starts[sd.k];
    const Hit h0 = hits[sd.p0];
    sd.p1 = upc[sd.p0];
    const Hit h1 = hits[sd.p1];
    sd.rs = h0.rs;
    sd.y0 = h0.y;
    sd.z0 = h0.z;
    sd.pad0 = sd.pad1 = 0;
    const double x0 = g.row_x[h0.rs % (uint32_t)R], x1 = g.row_x[h1.rs % (uint32_t)R];
    const double ty = ((double)h1.y - (double)h0.y) / (x1 - x0);
    const double tz = ((double)h1.z - (double)h0.z) / (x1 - x0);
    sd.s0 = ty / sqrt(1.0 + ty * ty);
    sd.t0 = tz * sqrt(1.0 - sd.s0 * sd.s0);
    seeds[j] = sd;
}

// Persistent kernel.  Every lane advances its own tracklet by one row per
// iteration; a lane whose tracklet is finished takes the next one at once, so
// long and short tracklets share a wave without idling it.
//
// Work comes from the processing order (tracklets grouped by sector and z slab
// of their start hit), split into one contiguous slice per XCD.  Workgroup b is
// dispatched to XCD b mod 8 and drains that XCD's slice first, then steals from
// the others, so the tracklets an XCD builds at any moment read the hits of one
// sector and a narrow z range, which its L2 holds.  A wave reserves 64 * chunk
// entries per atomic and hands them to its idle lanes by rank; a lane that
// receives an entry starts pass A after the row step of the busy lanes.  With two
// waves per SIMD its seed record is loaded before that step, so the load latency
// hides behind it; with three it is loaded after the step: held across the step,
// the record's twelve registers were what kept the kernel from three waves per
// SIMD without spills, and three waves hide the load behind each other's work.
template <int WAVES>
__global__ __launch_bounds__(kTlBlock) __attribute__((amdgpu_waves_per_eu(WAVES, WAVES))) void k_tracklets(
    GridDesc g, KParams kp, const TlHit* __restrict__ hits, const uint32_t* __restrict__ bin_off,
    const uint32_t* __restrict__ row_off, const Seed* __restrict__ seeds, uint32_t* __restrict__ counters,
    TrackletOut o, int chunk) {
    const uint32_t n = counters[C_N_STARTS];
    const int lane = threadIdx.x & 63;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int xcd = blockIdx.x % kXcd;
    const uint32_t grab = 64u * (uint32_t)chunk;
    uint32_t n_valid = 0, n_fail = 0;
    __shared__ Spare spare[kTlBlock];
    __shared__ float t_x[kMaxRows + 1], t_ymin[kMaxRows + 1];
    __shared__ int32_t t_ny[kMaxRows + 1];
    __shared__ uint32_t t_base[kMaxRows + 1];
    for (int r = threadIdx.x; r <= g.R; r += kTlBlock) {
        t_x[r] = r < g.R ? g.row_x[r] : 0.f;
        t_ymin[r] = r < g.R ? g.row_ymin[r] : 0.f;
        t_ny[r] = r < g.R ? g.row_ny[r] : 0;
        t_base[r] = g.bin_base[r];
    }
    __syncthreads();
    const RowTab rt{t_x, t_ymin, t_ny, t_base, t_base[g.R]};
    Lane L;
    L.phase = 0;  // 0 idle, 1 pass A, 2 pass B, 3 retired, 4 seed loading
    L.k = 0;
    L.s = L.r0 = L.r = L.edge = L.nh = L.ia = L.miss = 0;
    L.link = -1;
    L.on = L.fail = false;
    L.sp = &spare[threadIdx.x];
    for (int i = 0; i < kSlotChunk; ++i) L.sp->w[i] = -1;
    uint32_t plo = 0, phi = 0;  // wave-uniform: reserved, not yet handed out
    uint32_t my_j = 0;
    int cur = 0;                // slices this wave has found empty (wave-uniform)
    while (true) {
        uint64_t need = __ballot(L.phase == 0);
        while (need && cur < kXcd) {
            if (plo == phi) {
                const int x = (xcd + cur) % kXcd;
                const uint32_t lo = (uint32_t)((uint64_t)n * x / kXcd);
                const uint32_t hi = (uint32_t)((uint64_t)n * (x + 1) / kXcd);
                uint32_t b = 0;
                if (lane == 0) b = atomicAdd(&counters[C_QUEUE_XCD0 + x], grab);
                b = __shfl(b, 0, 64);
                if (lo + b >= hi || b >= hi - lo) {
                    ++cur;
                    continue;
                }
                plo = lo + b;
                phi = hi - plo < grab ? hi : plo + grab;
            }
            const uint32_t avail = phi - plo;
            const uint32_t rank = (uint32_t)__popcll(need & below);
            if (((need >> lane) & 1ull) && rank < avail) {
                my_j = plo + rank;
                L.phase = 4;
            }
            const uint32_t take = (uint32_t)__popcll(need) < avail ? (uint32_t)__popcll(need) : avail;
            plo += take;
            need = __ballot(L.phase == 0);
        }
        if (L.phase == 0) L.phase = 3;  // every slice is drained
        if (!__ballot(L.phase == 1 || L.phase == 2 || L.phase == 4)) break;
        Seed sd;
        if (WAVES == 2 && L.phase == 4) sd = seeds[my_j];  // two waves: the load hides behind the step
        if ((L.phase == 1 || L.phase == 2) && step(L, g, rt, kp, hits, bin_off, row_off, o)) {
            if (L.phase == 1 && !L.fail) {
                start_pass_b(L, g, rt, kp, o);
            } else {
                const uint32_t f = finish(L, g.R, kp, o);
                n_valid += f & 1u;
                n_fail += (f >> 1) & 1u;
            }
        }
        if (L.phase == 4) {
            if (WAVES != 2) sd = seeds[my_j];
            start_pass_a(L, sd, g, rt, kp, o);
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

size_t seed_bytes() { return sizeof(Seed); }

void build_tracklets(const GridDesc& g, const KParams& kp, const Hit* hits, const TlHit* tl_hits,
                     const uint32_t* bin_off, const uint32_t* row_off, const int32_t* upc, const uint32_t* starts,
                     const uint32_t* proc, void* seeds,
                     uint32_t* counters, const TrackletOut& o, int64_t t_max, int grid_blocks, int chunk, int waves,
                     hipStream_t s) {
    Seed* sd = (Seed*)seeds;
    const unsigned nb = (unsigned)((t_max + kBlock - 1) / kBlock > 0 ? (t_max + kBlock - 1) / kBlock : 1);
    k_seeds<<<nb, kBlock, 0, s>>>(g, hits, upc, starts, proc, counters, sd);
    grid_blocks = (grid_blocks + kXcd - 1) / kXcd * kXcd;
    // occupancy variants: 3 waves per SIMD (168 registers, no spills) or 2 (more registers for the
    // compiler's schedule)
    if (waves >= 3)
        k_tracklets<3><<<grid_blocks, kTlBlock, 0, s>>>(g, kp, tl_hits, bin_off, row_off, sd, counters, o, chunk);
    else
        k_tracklets<2><<<grid_blocks, kTlBlock, 0, s>>>(g, kp, tl_hits, bin_off, row_off, sd, counters, o, chunk);
}

}  // namespace tpc
