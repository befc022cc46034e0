// Device helpers shared by the HIP kernels.
#pragma once

#include "tpc_internal.h"

namespace tpc {

// Bins of row-sector (s, r) overlapping [y0,y1] x [z0,z1].  A hit's bin index is
// floor(fl32(fl32(y - ymin) * inv_bin)), within a relative 2^-23 of the exact
// coordinate V(y) = (y - ymin) * inv_bin that this range is computed from, so a
// margin of 1e-6 |V| + 1e-6 (bin units) keeps every hit inside [y0, y1] in the
// range; the caller's window tests are exact, so the margin only adds candidates.
// Hits outside the grid's y or z range are stored in its edge bins, so the range
// is clamped to the grid, never dropped: a box lying beyond the grid visits the
// edge bins.  Only NaN bounds give an empty range.
struct BinRange {
    int iy0, iy1, iz0, iz1, ny;
    uint32_t base;
    bool empty;
};

// Row tables bin_range needs, loaded ahead of the arithmetic that sets the box.
struct RowBins {
    double ymin;
    int ny;
    uint32_t base;
};

__device__ inline RowBins row_bins(const GridDesc& g, int s, int r) {
    return RowBins{(double)g.row_ymin[r], g.row_ny[r], g.bin_base[s * g.R + r]};
}

__device__ inline BinRange bin_range(const GridDesc& g, const RowBins& rb, double y0, double y1, double z0, double z1) {
    BinRange b;
    b.ny = rb.ny;
    const double ymin = rb.ymin, iby = g.inv_by, ibz = g.inv_bz, zmin = g.z_min;
    const double vy0 = (y0 - ymin) * iby, vy1 = (y1 - ymin) * iby;
    const double vz0 = (z0 - zmin) * ibz, vz1 = (z1 - zmin) * ibz;
    const double fy0 = floor(vy0 - (1e-6 * fabs(vy0) + 1e-6)), fy1 = floor(vy1 + (1e-6 * fabs(vy1) + 1e-6));
    const double fz0 = floor(vz0 - (1e-6 * fabs(vz0) + 1e-6)), fz1 = floor(vz1 + (1e-6 * fabs(vz1) + 1e-6));
    b.empty = !(fy0 <= fy1) || !(fz0 <= fz1);
    const double ym = (double)(b.ny - 1), zm = (double)(g.nz - 1);
    b.iy0 = fy0 < 0.0 ? 0 : (fy0 > ym ? b.ny - 1 : (int)fy0);
    b.iy1 = fy1 < 0.0 ? 0 : (fy1 > ym ? b.ny - 1 : (int)fy1);
    b.iz0 = fz0 < 0.0 ? 0 : (fz0 > zm ? g.nz - 1 : (int)fz0);
    b.iz1 = fz1 < 0.0 ? 0 : (fz1 > zm ? g.nz - 1 : (int)fz1);
    b.base = rb.base;
    return b;
}

__device__ inline BinRange bin_range(const GridDesc& g, int s, int r, double y0, double y1, double z0, double z1) {
    return bin_range(g, row_bins(g, s, r), y0, y1, z0, z1);
}

// A track's helix at x in the sector-local model, carried in one closed-form step from
// its FP32 reference state st5 = (y, z, sin phi, dz/ds, q/pT) at x_ref: y, z and sin phi
// there; false when |sin phi| reaches s_max on the way.  kq = -c Bz.
__device__ inline bool helix_at_state(const float* st5, double x_ref, double x, double kq, double s_max, double& yt,
                                      double& zt, double& st) {
    const double y0 = st5[0], z0 = st5[1], s0 = st5[2];
    const double t = st5[3], q = st5[4];
    const double dx = x - x_ref;
    const double kc = kq * q, s1 = s0 + kc * dx;
    if (!(fabs(s1) < s_max) || !(fabs(s0) < s_max)) return false;
    st = s1;
    if (dx == 0.0) {
        yt = y0;
        zt = z0;
        return true;
    }
    const double c0 = sqrt(1.0 - s0 * s0), c1 = sqrt(1.0 - s1 * s1);
    const double dy = dx * (s0 + s1) / (c0 + c1);
    const double L = copysign(sqrt(dx * dx + dy * dy), dx);
    const double u = 0.5 * kc * L;
    const double g = fabs(u) < 1e-4 ? 1.0 + u * u * (1.0 / 6.0) : asin(u) / u;  // asin(u)/u, exact to rounding
    yt = y0 + dy;
    zt = z0 + t * (L * g);
    return true;
}

// Ascending sort of a[0, m) in global memory by one workgroup: the bitonic network in
// its flip form, where every compare-exchange puts the smaller key at the lower index,
// over the next power of two P >= m.  Positions [m, P) hold virtual keys above every
// real key; such a key never has to move below a real one, so nothing is stored beyond
// m.  Every thread of the workgroup must call it; the workgroup's barriers order the
// global accesses (all its waves share one CU's caches).
template <class K, class Less>
__device__ void flip_bitonic_sort(K* a, uint32_t m, Less less) {
    uint32_t P = 1;
    while (P < m) P <<= 1;
    for (uint32_t k = 2; k <= P; k <<= 1) {
        const uint32_t h = k >> 1;
        for (uint32_t t = threadIdx.x; t < (P >> 1); t += blockDim.x) {
            const uint32_t i = (t / h) * k + (t % h), o = (t / h) * k + (k - 1 - (t % h));
            if (o < m) {
                const K x = a[i], y = a[o];
                if (less(y, x)) {
                    a[i] = y;
                    a[o] = x;
                }
            }
        }
        __syncthreads();
        for (uint32_t j = k >> 2; j > 0; j >>= 1) {
            for (uint32_t t = threadIdx.x; t < (P >> 1); t += blockDim.x) {
                const uint32_t i = (t / j) * 2 * j + (t % j), o = i + j;
                if (o < m) {
                    const K x = a[i], y = a[o];
                    if (less(y, x)) {
                        a[i] = y;
                        a[o] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__device__ inline uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Adds v to counter c (< kSlotCandSeg) through tally line `line` (any value).
__device__ inline void tally_add(uint32_t* counters, uint32_t line, int c, uint32_t v) {
    if (v) atomicAdd(&counters[C_N_COUNTERS + (line & (uint32_t)(kTallyLines - 1)) * kTallyStride + c], v);
}

// Block-wide sums of two per-thread values into counters ca and cb (cb < 0: none),
// one tally atomic per block each.  Every thread of the block must call it.
__device__ inline void block_tally2(uint32_t a, uint32_t b, int ca, int cb, uint32_t* counters) {
    __shared__ uint32_t sa[kBlock / 64], sb[kBlock / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t ta = 0, tb = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            ta += sa[k];
            tb += sb[k];
        }
        tally_add(counters, blockIdx.x, ca, ta);
        if (cb >= 0) tally_add(counters, blockIdx.x, cb, tb);
    }
}

}  // namespace tpc
