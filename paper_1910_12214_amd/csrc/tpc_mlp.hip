// Learned triplet scorer: MLP 12-64-64-1 on BF16 MFMA (v_mfma_f32_16x16x32_bf16).
//
// Layout.  Every layer is computed transposed, Out[unit][triplet] = W^T In, so a
// wave's 16 x 16 accumulator tile holds units 4g..4g+3 (g = lane / 16) of triplet
// lane % 16.  Those are exactly the eight k-values the next layer's B operand
// needs from that lane when the k order of the weight fragments is permuted to
// match (a dot product does not care about k order), so activations never leave
// the registers between layers.
//
// Precision.  Weights are BF16 (round to nearest even of the FP32 master values),
// biases FP32, products accumulate in FP32.  Activations are carried into the
// next MFMA as three BF16 terms (hi + mid + lo represents the FP32 value to
// ~2^-24), so the logits are FP32-faithful and a pruning decision logit >= tau
// agrees with an FP64 evaluation of the same BF16-weight network except within
// ~1e-5 of tau.  Training's backward pass uses single BF16 operands (its result
// is a gradient, compared at BF16 tolerance).
//
// Neighbour finding with a scorer: a candidate kernel lists the window
// candidates of each 64-hit group, a scoring kernel numbers the group's
// (down, up) pairs by a wave prefix sum, applies the plain criterion, scores the
// pairs within its cut 16 per MFMA tile from LDS-staged features, and each hit
// then chooses its best surviving pair.
#include "tpc_device.h"
#include "tpc_internal.h"

namespace tpc {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f4;

// packed weight layout (bytes offsets in the q buffer)
constexpr int kW1A = 0;                  // [T=4][j=2][lane=64][8] bf16
constexpr int kW2A = kW1A + 4096 * 2;    // [T2=4][pair=2][lane=64][8] bf16 (forward)
constexpr int kW2B = kW2A + 4096 * 2;    // [T1=4][pair=2][lane=64][8] bf16 (backward dh1 = W2 dz2)
constexpr int kB1 = kW2B + 4096 * 2;     // [64] f32
constexpr int kB2 = kB1 + 64 * 4;        // [64] f32
constexpr int kW3 = kB2 + 64 * 4;        // [64] f32 (BF16-valued)
constexpr int kB3 = kW3 + 64 * 4;        // [1] f32
constexpr int kQBytes = kB3 + 16;
static_assert(kQBytes == (int)kMlpQBytes, "packed weight size known to the scratch layout");

// master layout (floats)
constexpr int mW1 = 0, mB1 = 768, mW2 = 832, mB2 = 4928, mW3 = 4992, mB3 = 5056;
constexpr int kNP = 5057;

__device__ inline uint16_t bf16_bits(float f) {  // round to nearest, ties to even (v_cvt_pk_bf16_f32)
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ inline float bf16_val(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
__device__ inline __bf16 as_bf16(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

// three-term split of an FP32 value into BF16 terms
__device__ inline void split3(float x, uint16_t& h, uint16_t& m, uint16_t& l) {
    h = bf16_bits(x);
    const float r1 = x - bf16_val(h);
    m = bf16_bits(r1);
    const float r2 = r1 - bf16_val(m);
    l = bf16_bits(r2);
}

__device__ inline f4 mfma(const bf16x8& a, const bf16x8& b, const f4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Per-lane copy of the forward weights.
struct Frag {
    bf16x8 w1[4][2];
    bf16x8 w2[4][2];
    float b1[4][4], b2[4][4], w3[4][4];
    float b3;
};

__device__ inline void load_frag(const uint8_t* __restrict__ q, Frag& F) {
    const int lane = threadIdx.x & 63, g = lane >> 4;
    const bf16x8* w1 = (const bf16x8*)(q + kW1A);
    const bf16x8* w2 = (const bf16x8*)(q + kW2A);
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            F.w1[T][j] = w1[(T * 2 + j) * 64 + lane];
            F.w2[T][j] = w2[(T * 2 + j) * 64 + lane];
        }
    const float* b1 = (const float*)(q + kB1);
    const float* b2 = (const float*)(q + kB2);
    const float* w3 = (const float*)(q + kW3);
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            F.b1[T][i] = b1[16 * T + 4 * g + i];
            F.b2[T][i] = b2[16 * T + 4 * g + i];
            F.w3[T][i] = w3[16 * T + 4 * g + i];
        }
    F.b3 = *(const float*)(q + kB3);
}

// Activations of one 16-triplet tile in accumulator layout.
struct Act {
    f4 z1[4], z2[4];
    float z3;  // logit of triplet lane % 16 (same in all four lane groups)
};

// Layer-1 B operand for K-step j from an LDS row of 40 BF16 (36 split features + zero pad).
__device__ inline bf16x8 x_frag(const uint16_t* __restrict__ row, int j, int g) {
    const int k0 = 32 * j + 8 * g;
    bf16x8 b;
    if (k0 >= 40) {
#pragma unroll
        for (int i = 0; i < 8; ++i) b[i] = as_bf16(0);
    } else {
        const uint4 v = *(const uint4*)(row + k0);
        b = __builtin_bit_cast(bf16x8, v);
    }
    return b;
}

// Forward pass of one tile; xs points to the tile's 16 LDS rows (stride 40 BF16).
__device__ inline void forward_tile(const Frag& F, const uint16_t* __restrict__ xs, Act& A) {
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
    const uint16_t* row = xs + n * 40;
    const bf16x8 x0 = x_frag(row, 0, g), x1 = x_frag(row, 1, g);
#pragma unroll
    for (int T = 0; T < 4; ++T) {
        f4 c = {F.b1[T][0], F.b1[T][1], F.b1[T][2], F.b1[T][3]};
        c = mfma(F.w1[T][0], x0, c);
        c = mfma(F.w1[T][1], x1, c);
        A.z1[T] = c;
    }
    // layer 2: the lane's 16 hidden values, three BF16 terms each
    uint16_t hs[3][4][4];
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float h = A.z1[T][i] > 0.f ? A.z1[T][i] : 0.f;
            split3(h, hs[0][T][i], hs[1][T][i], hs[2][T][i]);
        }
    f4 c2[4];
#pragma unroll
    for (int T2 = 0; T2 < 4; ++T2) c2[T2] = f4{F.b2[T2][0], F.b2[T2][1], F.b2[T2][2], F.b2[T2][3]};
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
            bf16x8 b;
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) b[4 * t + i] = as_bf16(hs[s][2 * pr + t][i]);
#pragma unroll
            for (int T2 = 0; T2 < 4; ++T2) c2[T2] = mfma(F.w2[T2][pr], b, c2[T2]);
        }
    float part = 0.f;
#pragma unroll
    for (int T2 = 0; T2 < 4; ++T2) {
        A.z2[T2] = c2[T2];
#pragma unroll
        for (int i = 0; i < 4; ++i) part += F.w3[T2][i] * (c2[T2][i] > 0.f ? c2[T2][i] : 0.f);
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    A.z3 = part + F.b3;
}

// Weight fragments only; biases and output weights stay in LDS (kSbFloats floats:
// b1[64], b2[64], w3[64], b3), 48 registers fewer than Frag.
struct FragW {
    bf16x8 w1[4][2];
    bf16x8 w2[4][2];
};
constexpr int kSbFloats = 3 * 64 + 4;

__device__ inline void load_fragw(const uint8_t* __restrict__ q, FragW& F) {
    const int lane = threadIdx.x & 63;
    const bf16x8* w1 = (const bf16x8*)(q + kW1A);
    const bf16x8* w2 = (const bf16x8*)(q + kW2A);
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            F.w1[T][j] = w1[(T * 2 + j) * 64 + lane];
            F.w2[T][j] = w2[(T * 2 + j) * 64 + lane];
        }
}

// Logits of one 16-pair tile (rows xs, stride 40 BF16), the same arithmetic as
// forward_tile with the biases and output weights read from LDS (sb: b1, b2, w3, b3).
__device__ inline float tile_logit(const FragW& F, const float* __restrict__ sb, const uint16_t* __restrict__ xs) {
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
    const float* b1 = sb + 4 * g;
    const float* b2 = sb + 64 + 4 * g;
    const float* w3 = sb + 128 + 4 * g;
    const uint16_t* row = xs + n * 40;
    const bf16x8 x0 = x_frag(row, 0, g), x1 = x_frag(row, 1, g);
    f4 c1[4];
#pragma unroll
    for (int T = 0; T < 4; ++T) {
        f4 c = *(const f4*)(b1 + 16 * T);
        c = mfma(F.w1[T][0], x0, c);
        c1[T] = mfma(F.w1[T][1], x1, c);
    }
    uint16_t hs[3][4][4];
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float h = c1[T][i] > 0.f ? c1[T][i] : 0.f;
            split3(h, hs[0][T][i], hs[1][T][i], hs[2][T][i]);
        }
    f4 c2[4];
#pragma unroll
    for (int T2 = 0; T2 < 4; ++T2) c2[T2] = *(const f4*)(b2 + 16 * T2);
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
            bf16x8 b;
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int i = 0; i < 4; ++i) b[4 * u + i] = as_bf16(hs[s][2 * pr + u][i]);
#pragma unroll
            for (int T2 = 0; T2 < 4; ++T2) c2[T2] = mfma(F.w2[T2][pr], b, c2[T2]);
        }
    float part = 0.f;
#pragma unroll
    for (int T2 = 0; T2 < 4; ++T2) {
        const f4 w = *(const f4*)(w3 + 16 * T2);
#pragma unroll
        for (int i = 0; i < 4; ++i) part += w[i] * (c2[T2][i] > 0.f ? c2[T2][i] : 0.f);
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    return part + sb[192];
}

// Features of a triplet (down d, middle m, up u), FP32.
__device__ inline void features(float xd, float yd, float zd, float xm, float ym, float zm, float xu, float yu, float zu,
                                float wy, float wz, int nu, int nd, float f[12]) {
    const float dxd = xm - xd, dxu = xu - xm, dxt = xu - xd;
    f[0] = (xd - 166.0f) / 81.0f;
    f[1] = (xm - 166.0f) / 81.0f;
    f[2] = (xu - 166.0f) / 81.0f;
    f[3] = (yd - ym) / (wy * dxd);
    f[4] = (yu - ym) / (wy * dxu);
    f[5] = (zd - zm) / (wz * dxd);
    f[6] = (zu - zm) / (wz * dxu);
    f[7] = (yu - yd) / dxt;
    f[8] = (zu - zd) / dxt;
    const float ax = dxd, ay = ym - yd, bx = dxu, by = yu - ym, cx = dxt, cy = yu - yd;
    const float cross = ax * cy - ay * cx;
    const float la = sqrtf(ax * ax + ay * ay), lb = sqrtf(bx * bx + by * by), lc = sqrtf(cx * cx + cy * cy);
    f[9] = 20.0f * cross / (la * lb * lc);
    f[10] = 0.25f * (float)nu;
    f[11] = 0.25f * (float)nd;
}

// write the 36 split terms (+4 zeros) of 12 features into an LDS row of 40 BF16
__device__ inline void stage_row(uint16_t* __restrict__ row, const float f[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        uint16_t h, m, l;
        split3(f[k], h, m, l);
        row[k] = h;
        row[12 + k] = m;
        row[24 + k] = l;
    }
#pragma unroll
    for (int k = 36; k < 40; ++k) row[k] = 0;
}

// ------------------------------------------------------------ weight packing
__global__ void k_quantize(const float* __restrict__ m, uint8_t* __restrict__ q) {
    uint16_t* w1a = (uint16_t*)(q + kW1A);
    uint16_t* w2a = (uint16_t*)(q + kW2A);
    uint16_t* w2b = (uint16_t*)(q + kW2B);
    for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
        const int i = e & 7, lane = (e >> 3) & 63, j = (e >> 9) & 1, T = e >> 10;
        const int row = lane & 15, g = lane >> 4;
        // W1: A[unit][k], k = 32 j + 8 g + i -> feature k % 12 of split k / 12 (zero for k >= 36)
        const int k = 32 * j + 8 * g + i;
        const int unit = 16 * T + row;
        w1a[e] = k < 36 ? bf16_bits(m[mW1 + (k % 12) * 64 + unit]) : 0;
        // W2 forward: A[unit2][k1], k1 = 16 (2 pair + t) + 4 g + i' with i = 4 t + i'
        const int t = i >> 2, ii = i & 3;
        const int k1 = 16 * (2 * j + t) + 4 * g + ii;
        w2a[e] = bf16_bits(m[mW2 + k1 * 64 + unit]);
        // W2 backward: A[hidden1 unit][hidden2 u], u = 16 (2 pair + t) + 4 g + i'
        w2b[e] = bf16_bits(m[mW2 + unit * 64 + k1]);
    }
    float* b1 = (float*)(q + kB1);
    float* b2 = (float*)(q + kB2);
    float* w3 = (float*)(q + kW3);
    for (int e = threadIdx.x; e < 64; e += blockDim.x) {
        b1[e] = m[mB1 + e];
        b2[e] = m[mB2 + e];
        w3[e] = bf16_val(bf16_bits(m[mW3 + e]));
    }
    if (threadIdx.x == 0) *(float*)(q + kB3) = m[mB3];
}

// ------------------------------------------------------------ inference
constexpr int kInferWaves = 4;

__global__ __launch_bounds__(64 * kInferWaves) void k_infer(const uint8_t* __restrict__ q, const float* __restrict__ feats,
                                                            int64_t n, float* __restrict__ logits) {
    __shared__ __attribute__((aligned(16))) uint16_t xs_all[kInferWaves][16 * 40];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, nn = lane & 15;
    uint16_t* xs = xs_all[w];
    Frag F;
    load_frag(q, F);
    const int64_t n_tiles = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * kInferWaves + w; tile < n_tiles; tile += (int64_t)gridDim.x * kInferWaves) {
        const int64_t t = tile * 16 + nn;
        if (g == 0) {
            float f[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) f[k] = t < n ? feats[t * 12 + k] : 0.f;
            stage_row(xs + nn * 40, f);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        Act A;
        forward_tile(F, xs, A);
        if (g == 0 && t < n) logits[t] = A.z3;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ------------------------------------------------- triplet enumeration (training data)
__device__ inline int count_window(const GridDesc& g, const Hit* __restrict__ hits, const uint32_t* __restrict__ bin_off,
                                   const BinRange& B, double ym, double zm, double wy, double wz) {
    int c = 0;
    if (B.empty) return 0;
    for (int iz = B.iz0; iz <= B.iz1; ++iz) {
        const uint32_t k1 = bin_off[B.base + iz * B.ny + B.iy1 + 1];
        for (uint32_t k = bin_off[B.base + iz * B.ny + B.iy0]; k < k1; ++k) {
            const Hit h = hits[k];
            c += (fabs((double)h.y - ym) <= wy) && (fabs((double)h.z - zm) <= wz);
        }
    }
    return c;
}

// Calls fn(pos, hit) for each window candidate of range B (exact FP64 window test).
template <typename Fn>
__device__ inline void for_window(const Hit* __restrict__ hits, const uint32_t* __restrict__ bin_off, const BinRange& B,
                                  double ym, double zm, double wy, double wz, Fn fn) {
    if (B.empty) return;
    for (int iz = B.iz0; iz <= B.iz1; ++iz) {
        const uint32_t k1 = bin_off[B.base + iz * B.ny + B.iy1 + 1];
        for (uint32_t k = bin_off[B.base + iz * B.ny + B.iy0]; k < k1; ++k) {
            const Hit h = hits[k];
            if (fabs((double)h.y - ym) <= wy && fabs((double)h.z - zm) <= wz) fn(k, h);
        }
    }
}

struct Win {
    bool ok;
    int r, s;
    double xm, xu, xd, wyu, wzu, wyd, wzd;
    BinRange U, D;
};

__device__ inline Win window_of(const GridDesc& g, const KParams& kp, const Hit& m) {
    Win w;
    w.r = (int)(m.rs % (uint32_t)g.R);
    w.s = (int)(m.rs / (uint32_t)g.R);
    w.ok = w.r > 0 && w.r < g.R - 1;
    if (!w.ok) return w;
    w.xm = g.row_x[w.r];
    w.xu = g.row_x[w.r + 1];
    w.xd = g.row_x[w.r - 1];
    const double ym = m.y, zm = m.z;
    w.wyu = kp.win_y * (w.xu - w.xm);
    w.wzu = kp.win_z * (w.xu - w.xm);
    w.wyd = kp.win_y * (w.xm - w.xd);
    w.wzd = kp.win_z * (w.xm - w.xd);
    w.U = bin_range(g, w.s, w.r + 1, ym - w.wyu, ym + w.wyu, zm - w.wzu, zm + w.wzu);
    w.D = bin_range(g, w.s, w.r - 1, ym - w.wyd, ym + w.wyd, zm - w.wzd, zm + w.wzd);
    w.ok = !w.U.empty && !w.D.empty;
    return w;
}

__global__ __launch_bounds__(kBlock) void k_trip_count(GridDesc g, KParams kp, const Hit* __restrict__ hits,
                                                       const uint32_t* __restrict__ bin_off,
                                                       const uint32_t* __restrict__ counters, uint32_t* __restrict__ cnt) {
    const uint32_t n = counters[C_N_VALID_CLU];
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const Hit m = hits[p];
    const Win w = window_of(g, kp, m);
    uint32_t c = 0;
    if (w.ok) {
        const int nu = count_window(g, hits, bin_off, w.U, m.y, m.z, w.wyu, w.wzu);
        const int nd = count_window(g, hits, bin_off, w.D, m.y, m.z, w.wyd, w.wzd);
        c = (uint32_t)(nu * nd);
    }
    cnt[p] = c;
}

__global__ __launch_bounds__(kBlock) void k_trip_write(GridDesc g, KParams kp, const Hit* __restrict__ hits,
                                                       const uint32_t* __restrict__ bin_off,
                                                       const uint32_t* __restrict__ counters,
                                                       const uint32_t* __restrict__ off, int32_t* __restrict__ trip,
                                                       float* __restrict__ feats, int64_t cap) {
    const uint32_t n = counters[C_N_VALID_CLU];
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const Hit m = hits[p];
    const Win w = window_of(g, kp, m);
    if (!w.ok) return;
    const int nu = count_window(g, hits, bin_off, w.U, m.y, m.z, w.wyu, w.wzu);
    const int nd = count_window(g, hits, bin_off, w.D, m.y, m.z, w.wyd, w.wzd);
    int64_t slot = off[p];
    const float wy = (float)kp.win_y, wz = (float)kp.win_z;
    for_window(hits, bin_off, w.U, m.y, m.z, w.wyu, w.wzu, [&](uint32_t, const Hit& u) {
        for_window(hits, bin_off, w.D, m.y, m.z, w.wyd, w.wzd, [&](uint32_t, const Hit& d) {
            if (slot < cap) {
                trip[slot * 3 + 0] = (int32_t)d.id;
                trip[slot * 3 + 1] = (int32_t)m.id;
                trip[slot * 3 + 2] = (int32_t)u.id;
                float f[12];
                features((float)w.xd, d.y, d.z, (float)w.xm, m.y, m.z, (float)w.xu, u.y, u.z, wy, wz, nu, nd, f);
#pragma unroll
                for (int k = 0; k < 12; ++k) feats[slot * 12 + k] = f[k];
            }
            ++slot;
        });
    });
}

// ------------------------------------------------- fused neighbour finding with pruning
// Two kernels over the same 64-hit waves.
//
// Candidates (lane = hit, full occupancy: the window walks are chains of
// dependent loads): count the up and down window candidates of each hit, keeping
// the first kListC of each window in registers; a wave prefix sum numbers the
// wave's candidates (only hits that have pairs) and its pairs (nu * nd per hit);
// lane 0 reserves the wave's candidate records with one atomic in segment
// (wave mod kTallyLines) of a global list (one fill counter per segment, each on
// its own line: a single shared counter would serialise every wave of the chip),
// and the hits write their records there.  A wave without pairs writes its empty
// links at once; a wave whose candidates exceed kCapC, or do not fit its segment,
// goes to an overflow list served by the per-lane kernel below.
//
// Scoring (lane = pair, MFMA): the wave copies its candidate records into LDS
// (coalesced), recomputes the same prefix sums from the per-hit counts, then in
// rounds of 64 pairs: the plain criterion D in FP64 from the LDS list; the pairs
// with D <= cut (only they can survive) stage their features into consecutive
// rows, scored by as many 16-pair MFMA tiles as they fill; a pair survives if
// also its logit >= tau.  Lane = hit again: the best surviving pair over this
// round's slots of the hit (smallest D, ties by (id_up, id_down)).
constexpr int kPW = 4;        // waves per block (scoring)
constexpr int kCapC = 512;    // candidate records per wave (10-bit offsets and counts)
constexpr int kListC = 4;     // window candidates held in registers per window
constexpr uint32_t kNoWave = 0xFFFFFFFFu;

struct alignas(16) Cand {
    float y, z;
    uint32_t id;
    int32_t pos;
};

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave prefix sums of the candidate counts (hits with pairs only) and pair counts.
struct WaveOffs {
    uint32_t coff, pofs, ctot, ptot;
};
__device__ inline WaveOffs wave_offsets(int nu, int nd, int lane) {
    const uint32_t np = (uint32_t)(nu * nd), nc = np ? (uint32_t)(nu + nd) : 0u;
    uint32_t ic = nc, ip = np;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t a = __shfl_up(ic, d, 64), b = __shfl_up(ip, d, 64);
        if (lane >= d) {
            ic += a;
            ip += b;
        }
    }
    WaveOffs o;
    o.ctot = __shfl(ic, 63, 64);
    o.ptot = __shfl(ip, 63, 64);
    o.coff = ic - nc;
    o.pofs = ip - np;
    return o;
}

// Window candidates of range B (the same exact FP64 test as for_window): their
// number, the positions of the first kListC in l (selects with constant indices).
__device__ inline int list_window(const Hit* __restrict__ hits, const uint32_t* __restrict__ bin_off,
                                  const BinRange& B, double ym, double zm, double wy, double wz,
                                  uint32_t (&l)[kListC]) {
    int c = 0;
    if (B.empty) return 0;
    for (int iz = B.iz0; iz <= B.iz1; ++iz) {
        const uint32_t k1 = bin_off[B.base + iz * B.ny + B.iy1 + 1];
        for (uint32_t k = bin_off[B.base + iz * B.ny + B.iy0]; k < k1; ++k) {
            const Hit h = hits[k];
            if (fabs((double)h.y - ym) <= wy && fabs((double)h.z - zm) <= wz) {
#pragma unroll
                for (int q = 0; q < kListC; ++q) l[q] = q == c ? k : l[q];
                ++c;
            }
        }
    }
    return c;
}

__device__ inline void write_window(const Hit* __restrict__ hits, const uint32_t* __restrict__ bin_off,
                                    const BinRange& B, double ym, double zm, double wy, double wz, int cnt,
                                    const uint32_t (&l)[kListC], Cand* __restrict__ out) {
    if (cnt <= kListC) {
#pragma unroll
        for (int q = 0; q < kListC; ++q)
            if (q < cnt) {
                const Hit h = hits[l[q]];
                out[q] = Cand{h.y, h.z, h.id, (int32_t)l[q]};
            }
    } else {
        int j = 0;
        for_window(hits, bin_off, B, ym, zm, wy, wz,
                   [&](uint32_t k, const Hit& h) { out[j++] = Cand{h.y, h.z, h.id, (int32_t)k}; });
    }
}

__global__ __launch_bounds__(kBlock) void k_nb_cand(GridDesc g, KParams kp, const Hit* __restrict__ hits,
                                                    const uint32_t* __restrict__ bin_off,
                                                    uint32_t* __restrict__ counters, Cand* __restrict__ cand,
                                                    uint32_t seg_cap, uint32_t* __restrict__ nund,
                                                    uint32_t* __restrict__ wrec, int32_t* __restrict__ up,
                                                    int32_t* __restrict__ dn, uint32_t* __restrict__ ovf) {
    const int lane = threadIdx.x & 63;
    const uint32_t n = counters[C_N_VALID_CLU];
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    if (wave * 64u >= n) return;  // wave-uniform
    const uint32_t p = wave * 64 + lane;
    const bool act = p < n;
    Hit m;
    m.y = m.z = 0.f;
    Win win;
    win.ok = false;
    int nu = 0, nd = 0;
    uint32_t lu[kListC], ld[kListC];
#pragma unroll
    for (int q = 0; q < kListC; ++q) lu[q] = ld[q] = 0;
    if (act) {
        m = hits[p];
        win = window_of(g, kp, m);
        if (win.ok) {
            nu = list_window(hits, bin_off, win.U, m.y, m.z, win.wyu, win.wzu, lu);
            if (nu) nd = list_window(hits, bin_off, win.D, m.y, m.z, win.wyd, win.wzd, ld);
        }
    }
    const WaveOffs o = wave_offsets(nu, nd, lane);
    uint32_t cb = kNoWave;
    if (o.ptot && o.ctot <= (uint32_t)kCapC) {  // wave-uniform
        const uint32_t seg = wave & (uint32_t)(kTallyLines - 1);
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(&counters[C_N_COUNTERS + seg * kTallyStride + kSlotCandSeg], o.ctot);
        b = __shfl(b, 0, 64);
        if ((uint64_t)b + o.ctot <= (uint64_t)seg_cap) cb = seg * seg_cap + b;
    }
    if (lane == 0) {
        wrec[wave] = cb;
        if (o.ptot && cb == kNoWave) ovf[atomicAdd(&counters[C_NB_OVF], 1u)] = wave;
    }
    if (cb == kNoWave) {
        if (!o.ptot && act) {
            up[p] = -1;
            dn[p] = -1;
        }
        return;
    }
    if (act) nund[p] = (uint32_t)nu | ((uint32_t)nd << 16);
    if (nu * nd) {
        Cand* c = cand + cb + o.coff;
        write_window(hits, bin_off, win.U, m.y, m.z, win.wyu, win.wzu, nu, lu, c);
        write_window(hits, bin_off, win.D, m.y, m.z, win.wyd, win.wzd, nd, ld, c + nu);
    }
}

__global__ __launch_bounds__(64 * kPW) __attribute__((amdgpu_waves_per_eu(2))) void k_nb_score(GridDesc g, KParams kp, const Hit* __restrict__ hits,
                                                       uint32_t* __restrict__ counters, const uint8_t* __restrict__ q,
                                                       const Cand* __restrict__ cand_g,
                                                       const uint32_t* __restrict__ nund,
                                                       const uint32_t* __restrict__ wrec, int32_t* __restrict__ up,
                                                       int32_t* __restrict__ dn) {
    __shared__ Cand cand_all[kPW][kCapC];
    __shared__ __attribute__((aligned(16))) uint16_t xs_all[kPW][64 * 40];
    __shared__ float lg_all[kPW][64];
    __shared__ double dv_all[kPW][64];
    __shared__ uint32_t ps0_all[kPW][64], meta_all[kPW][64];
    __shared__ float ym_all[kPW][64], zm_all[kPW][64];
    __shared__ float xd_all[kPW][64], xm_all[kPW][64], xu_all[kPW][64];
    __shared__ uint8_t own_all[kPW][64];
    __shared__ __attribute__((aligned(16))) float sb[kSbFloats];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < kSbFloats; i += blockDim.x)  // b1, b2, w3 (64 each), b3
        sb[i] = i < 192 ? ((const float*)(q + kB1))[i] : (i == 192 ? *(const float*)(q + kB3) : 0.f);
    __syncthreads();
    Cand* cand = cand_all[w];
    uint16_t* xs = xs_all[w];
    float* lg = lg_all[w];
    double* dv = dv_all[w];
    uint32_t* ps0s = ps0_all[w];
    uint32_t* meta = meta_all[w];
    const uint32_t n = counters[C_N_VALID_CLU];
    const uint32_t wave = blockIdx.x * kPW + w;
    if (wave * 64u >= n) return;  // wave-uniform
    const uint32_t cb = wrec[wave];
    if (cb == kNoWave) return;  // no pairs (links written) or on the overflow list
    const uint32_t p = wave * 64 + lane;
    const bool act = p < n;
    int nu = 0, nd = 0;
    float ymv = 0.f, zmv = 0.f, xdv = 0.f, xmv = 0.f, xuv = 0.f;
    if (act) {
        const uint32_t v = nund[p];
        nu = (int)(v & 0xFFFFu);
        nd = (int)(v >> 16);
        if (nu * nd) {  // such a hit passed window_of: 0 < r < R - 1
            const Hit m = hits[p];
            const int r = (int)(m.rs % (uint32_t)g.R);
            ymv = m.y;
            zmv = m.z;
            xdv = g.row_x[r - 1];
            xmv = g.row_x[r];
            xuv = g.row_x[r + 1];
        }
    }
    const WaveOffs o = wave_offsets(nu, nd, lane);
    const uint32_t np = (uint32_t)(nu * nd), coff = o.coff, pofs = o.pofs, ptot = o.ptot;
    for (uint32_t i = (uint32_t)lane; i < o.ctot; i += 64) cand[i] = cand_g[cb + i];
    ps0s[lane] = pofs;
    meta[lane] = coff | ((uint32_t)nu << 10) | ((uint32_t)nd << 20);
    ym_all[w][lane] = ymv;
    zm_all[w][lane] = zmv;
    xd_all[w][lane] = xdv;
    xm_all[w][lane] = xmv;
    xu_all[w][lane] = xuv;
    wave_sync();
    double best = 1e300;
    uint32_t bu_id = 0xFFFFFFFFu, bd_id = 0xFFFFFFFFu;
    int32_t bu = -1, bd = -1;
    uint32_t kept = 0;
    FragW F;
    load_fragw(q, F);
    const float wy = (float)kp.win_y, wz = (float)kp.win_z;
    uint8_t* own = own_all[w];
    for (uint32_t base = 0; base < ptot; base += 64) {
        const uint32_t t = base + (uint32_t)lane;
        const bool has = t < ptot;
        // this hit's slots in the round: [s0, s1)
        const bool mine = np && pofs < base + 64 && pofs + np > base;
        const uint32_t s0 = mine ? (pofs > base ? pofs - base : 0u) : 0u;
        const uint32_t s1 = mine ? (pofs + np < base + 64 ? pofs + np - base : 64u) : 0u;
        for (uint32_t sl = s0; sl < s1; ++sl) own[sl] = (uint8_t)lane;  // owner of each slot
        wave_sync();
        // the plain criterion first: only pairs within its cut need a logit (a pair
        // survives if D <= cut and logit >= tau, in either order)
        double Dv = -1.0;
        Cand cu, cd;
        float xd = 0.f, xm = 0.f, xu = 0.f, ymh = 0.f, zmh = 0.f;
        uint32_t nuh = 0, ndh = 0;
        if (has) {
            const int lo = own[lane];
            const uint32_t mt = meta[lo];
            const uint32_t co = mt & 1023u;
            nuh = (mt >> 10) & 1023u;
            ndh = mt >> 20;
            const uint32_t idx = t - ps0s[lo];
            const uint32_t iu = idx / ndh, id = idx - iu * ndh;
            cu = cand[co + iu];
            cd = cand[co + nuh + id];
            xd = xd_all[w][lo];
            xm = xm_all[w][lo];
            xu = xu_all[w][lo];
            ymh = ym_all[w][lo];
            zmh = zm_all[w][lo];
            const double wgt = ((double)xm - (double)xd) / ((double)xu - (double)xd);
            const double yu = cu.y, zu = cu.z, yd = cd.y, zd = cd.z;
            const double py = yd + (yu - yd) * wgt, pz = zd + (zu - zd) * wgt;
            const double ym = ymh, zm = zmh;
            Dv = (ym - py) * (ym - py) * kp.ivy15 + (zm - pz) * (zm - pz) * kp.ivz15;
        }
        const bool pass = has && Dv <= kp.nb_cut;
        const uint64_t pm = __ballot(pass);
        const uint32_t n_pass = (uint32_t)__builtin_popcountll(pm);
        // rank among the passing lanes: their features fill tile rows 0 .. n_pass - 1
        const uint32_t ci = __builtin_amdgcn_mbcnt_hi((uint32_t)(pm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)pm, 0u));
        if (pass) {
            float f[12];
            features(xd, cd.y, cd.z, xm, ymh, zmh, xu, cu.y, cu.z, wy, wz, (int)nuh, (int)ndh, f);
            stage_row(xs + ci * 40, f);
        }
        wave_sync();
        for (uint32_t T = 0; 16 * T < n_pass; ++T) {  // rows past n_pass: stale, their logits unused
            const float z = tile_logit(F, sb, xs + T * 16 * 40);
            if (lane < 16) lg[16 * T + lane] = z;
        }
        wave_sync();
        const bool keep = pass && (double)lg[ci] >= kp.tau;
        kept += keep;
        // surviving pairs of the round: a ballot, so that a hit visits only its survivors
        const uint64_t surv = __ballot(keep);
        dv[lane] = Dv;
        wave_sync();
        if (mine) {
            const uint64_t hi_mask = s1 == 64u ? ~0ull : ((1ull << s1) - 1ull);
            uint64_t bits = surv & hi_mask & ~((1ull << s0) - 1ull);
            while (bits) {
                const uint32_t j = (uint32_t)__builtin_ctzll(bits);
                bits &= bits - 1ull;
                const double d = dv[j];
                const uint32_t idx = base + j - pofs;
                const uint32_t iu = idx / (uint32_t)nd, id = idx - iu * (uint32_t)nd;
                const Cand cu = cand[coff + iu], cd = cand[coff + (uint32_t)nu + id];
                if (d < best || (d == best && (cu.id < bu_id || (cu.id == bu_id && cd.id < bd_id)))) {
                    best = d;
                    bu = cu.pos;
                    bd = cd.pos;
                    bu_id = cu.id;
                    bd_id = cd.id;
                }
            }
        }
        wave_sync();
    }
    if (act) {
        up[p] = bu;
        dn[p] = bd;
    }
    const uint32_t linked = bu >= 0;
    uint32_t a = wave_sum(np), b = wave_sum(kept), c = wave_sum(linked);
    if (lane == 0) {
        tally_add(counters, wave, C_N_PAIRS, a);
        tally_add(counters, wave, C_N_PAIRS_KEPT, b);
        tally_add(counters, wave, C_N_LINKS_RAW, c);
    }
}

// ------------------------------------------------- fused neighbour finding with pruning
constexpr int kNbWaves = 4;
constexpr int kCap = 128;  // staged pairs per wave and round

// One wave's 64 hits by per-lane enumeration (staged pairs in rounds of kCap);
// used for the waves whose window candidates do not fit the pair-parallel
// kernel's LDS list.
__device__ void nb_mlp_wave(uint32_t wave, const GridDesc& g, const KParams& kp, const Hit* __restrict__ hits,
                            const uint32_t* __restrict__ bin_off, uint32_t n, const uint8_t* __restrict__ q,
                            int32_t* __restrict__ up, int32_t* __restrict__ dn, uint32_t* __restrict__ cnt,
                            uint16_t* xs, float* lg) {
    const int lane = threadIdx.x & 63;
    const uint32_t p = wave * 64 + lane;
    const bool act = p < n;
    Hit m;
    Win win;
    win.ok = false;
    int nu = 0, nd = 0;
    if (act) {
        m = hits[p];
        win = window_of(g, kp, m);
        if (win.ok) {
            nu = count_window(g, hits, bin_off, win.U, m.y, m.z, win.wyu, win.wzu);
            nd = count_window(g, hits, bin_off, win.D, m.y, m.z, win.wyd, win.wzd);
        }
    }
    const uint32_t np = (uint32_t)(nu * nd);
    // wave prefix sum of the pair counts
    uint32_t incl = np;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    const uint32_t slot0 = incl - np;
    const uint32_t total = __shfl(incl, 63, 64);
    Frag F;
    if (total) load_frag(q, F);
    double best = 1e300;
    uint32_t bu_id = 0xFFFFFFFFu, bd_id = 0xFFFFFFFFu;
    int32_t bu = -1, bd = -1;
    uint32_t kept = 0;
    const float wy = (float)kp.win_y, wz = (float)kp.win_z;
    for (uint32_t base = 0; base < total; base += kCap) {
        const uint32_t lim = total - base < (uint32_t)kCap ? total - base : (uint32_t)kCap;
        // stage features of the pairs whose slots fall in this round
        if (np && slot0 < base + lim && slot0 + np > base) {
            uint32_t j = 0;
            for_window(hits, bin_off, win.U, m.y, m.z, win.wyu, win.wzu, [&](uint32_t, const Hit& u) {
                for_window(hits, bin_off, win.D, m.y, m.z, win.wyd, win.wzd, [&](uint32_t, const Hit& d) {
                    const uint32_t sl = slot0 + j++;
                    if (sl >= base && sl < base + lim) {
                        float f[12];
                        features((float)win.xd, d.y, d.z, (float)win.xm, m.y, m.z, (float)win.xu, u.y, u.z, wy, wz, nu,
                                 nd, f);
                        stage_row(xs + (sl - base) * 40, f);
                    }
                });
            });
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t t0 = 0; t0 < lim; t0 += 16) {
            Act A;
            forward_tile(F, xs + t0 * 40, A);
            const int nn = lane & 15;
            if (lane < 16 && t0 + nn < lim) lg[t0 + nn] = A.z3;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // choose among the kept pairs of this round
        if (np && slot0 < base + lim && slot0 + np > base) {
            const double xm = win.xm, xd = win.xd, xu = win.xu;
            const double ym = m.y, zm = m.z;
            const double wgt = (xm - xd) / (xu - xd);
            uint32_t j = 0;
            for_window(hits, bin_off, win.U, m.y, m.z, win.wyu, win.wzu, [&](uint32_t ku, const Hit& u) {
                for_window(hits, bin_off, win.D, m.y, m.z, win.wyd, win.wzd, [&](uint32_t kd, const Hit& d) {
                    const uint32_t sl = slot0 + j++;
                    if (sl < base || sl >= base + lim) return;
                    if (!((double)lg[sl - base] >= kp.tau)) return;
                    const double yu = u.y, zu = u.z, yd = d.y, zd = d.z;
                    const double py = yd + (yu - yd) * wgt, pz = zd + (zu - zd) * wgt;
                    const double Dv = (ym - py) * (ym - py) * kp.ivy15 + (zm - pz) * (zm - pz) * kp.ivz15;
                    if (!(Dv <= kp.nb_cut)) return;
                    ++kept;
                    if (Dv < best || (Dv == best && (u.id < bu_id || (u.id == bu_id && d.id < bd_id)))) {
                        best = Dv;
                        bu = (int32_t)ku;
                        bd = (int32_t)kd;
                        bu_id = u.id;
                        bd_id = d.id;
                    }
                });
            });
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (act) {
        up[p] = bu;
        dn[p] = bd;
    }
    const uint32_t linked = bu >= 0;
    // per-wave sums (no block barrier needed: one atomic per wave)
    uint32_t a = wave_sum(np), b = wave_sum(kept), c = wave_sum(linked);
    if (lane == 0) {
        tally_add(cnt, wave, C_N_PAIRS, a);
        tally_add(cnt, wave, C_N_PAIRS_KEPT, b);
        tally_add(cnt, wave, C_N_LINKS_RAW, c);
    }
}

__global__ __launch_bounds__(64 * kNbWaves) void k_nb_mlp_fallback(GridDesc g, KParams kp, const Hit* __restrict__ hits,
                                                                   const uint32_t* __restrict__ bin_off,
                                                                   uint32_t* __restrict__ counters,
                                                                   const uint8_t* __restrict__ q,
                                                                   const uint32_t* __restrict__ ovf,
                                                                   int32_t* __restrict__ up, int32_t* __restrict__ dn) {
    __shared__ __attribute__((aligned(16))) uint16_t xs_all[kNbWaves][kCap * 40];
    __shared__ float lg_all[kNbWaves][kCap];
    const int w = threadIdx.x >> 6;
    const uint32_t n = counters[C_N_VALID_CLU], n_ovf = counters[C_NB_OVF];
    for (uint32_t i = blockIdx.x * kNbWaves + w; i < n_ovf; i += gridDim.x * kNbWaves)
        nb_mlp_wave(ovf[i], g, kp, hits, bin_off, n, q, up, dn, counters, xs_all[w], lg_all[w]);
}

// ------------------------------------------------------------ training
constexpr int kTrainChunk = kMlpTrainChunk;  // triplets per block (one wave) and step

__device__ inline float sigmoidf_(float z) { return 1.0f / (1.0f + expf(-z)); }

// One wave per block; block b handles rows [b*chunk, (b+1)*chunk) of the batch.
// Writes the block's gradient contribution (master layout) and loss sum to part[b].
__global__ __launch_bounds__(64) void k_train_grad(const uint8_t* __restrict__ q, const float* __restrict__ feats,
                                                   const uint8_t* __restrict__ labels, const int32_t* __restrict__ idx,
                                                   int batch, float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[16 * 40];
    // transposed BF16 stages for the weight gradients: [unit][32 triplets]
    __shared__ __attribute__((aligned(16))) uint16_t h1s[64 * 32], dz2s[64 * 32], dz1s[64 * 32], xts[16 * 32];
    const int lane = threadIdx.x, g = lane >> 4, nn = lane & 15;
    Frag F;
    load_frag(q, F);
    const bf16x8* w2b = (const bf16x8*)(q + kW2B);
    bf16x8 wb[4][2];
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
        for (int j = 0; j < 2; ++j) wb[T][j] = w2b[(T * 2 + j) * 64 + lane];
    f4 gW2[4][4], gW1[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f4{0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = f4{0, 0, 0, 0};
    }
    float gb1[4][4], gb2[4][4], gw3[4][4];
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
        for (int i = 0; i < 4; ++i) gb1[T][i] = gb2[T][i] = gw3[T][i] = 0.f;
    float gb3 = 0.f, loss = 0.f;
    const float inv_b = 1.0f / (float)batch;
    const int r0 = blockIdx.x * kTrainChunk;
    const int r1 = min(batch, r0 + kTrainChunk);
    for (int base = r0; base < r1; base += 32) {
        // two 16-triplet tiles fill 32 columns of the transposed stages
        for (int half = 0; half < 2; ++half) {
            const int row = base + 16 * half + nn;
            const bool valid = row < r1;
            const int id = valid ? idx[row] : 0;
            float f[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) f[k] = valid ? feats[(int64_t)id * 12 + k] : 0.f;
            if (g == 0) stage_row(xs + nn * 40, f);
            __syncthreads();
            Act A;
            forward_tile(F, xs, A);
            const float y = valid ? (float)labels[id] : 0.f;
            const float dz3 = valid ? (sigmoidf_(A.z3) - y) * inv_b : 0.f;
            if (g == 0 && valid) {
                // BCE = softplus(z) - y z, stable form
                const float z = A.z3;
                loss += fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - y * z;
                gb3 += dz3;
            }
            // dz2 = w3 * dz3 * (z2 > 0); bias and w3 gradients
            float dz2[4][4];
            uint16_t dz2b[4][4];
#pragma unroll
            for (int T = 0; T < 4; ++T)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float z2 = A.z2[T][i];
                    const float h2 = z2 > 0.f ? z2 : 0.f;
                    gw3[T][i] += h2 * dz3;
                    dz2[T][i] = z2 > 0.f ? F.w3[T][i] * dz3 : 0.f;
                    gb2[T][i] += dz2[T][i];
                    dz2b[T][i] = bf16_bits(dz2[T][i]);
                }
            // dh1 = W2 dz2 (MFMA, K = hidden-2 units in the lane-held order)
            f4 dh1[4];
#pragma unroll
            for (int T = 0; T < 4; ++T) dh1[T] = f4{0, 0, 0, 0};
#pragma unroll
            for (int pr = 0; pr < 2; ++pr) {
                bf16x8 b;
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int i = 0; i < 4; ++i) b[4 * t + i] = as_bf16(dz2b[2 * pr + t][i]);
#pragma unroll
                for (int T = 0; T < 4; ++T) dh1[T] = mfma(wb[T][pr], b, dh1[T]);
            }
            // stage h1, dz2, dz1 (unit-major) and x (feature-major) for the batch contractions
            const int col = 16 * half + nn;
#pragma unroll
            for (int T = 0; T < 4; ++T)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int u = 16 * T + 4 * g + i;
                    const float z1 = A.z1[T][i];
                    const float dz1 = z1 > 0.f ? dh1[T][i] : 0.f;
                    gb1[T][i] += dz1;
                    h1s[u * 32 + col] = bf16_bits(z1 > 0.f ? z1 : 0.f);
                    dz2s[u * 32 + col] = dz2b[T][i];
                    dz1s[u * 32 + col] = bf16_bits(dz1);
                }
            if (g == 0) {
#pragma unroll
                for (int k = 0; k < 12; ++k) xts[k * 32 + col] = bf16_bits(f[k]);
#pragma unroll
                for (int k = 12; k < 16; ++k) xts[k * 32 + col] = 0;
            }
            __syncthreads();
        }
        // dW2[k1][u] += sum_n h1[k1][n] dz2[u][n];  dW1[f][k1] += sum_n x[f][n] dz1[k1][n]
        bf16x8 ah[4], bz[4], bz1[4];
#pragma unroll
        for (int T = 0; T < 4; ++T) {
            ah[T] = __builtin_bit_cast(bf16x8, *(const uint4*)(h1s + (16 * T + nn) * 32 + 8 * g));
            bz[T] = __builtin_bit_cast(bf16x8, *(const uint4*)(dz2s + (16 * T + nn) * 32 + 8 * g));
            bz1[T] = __builtin_bit_cast(bf16x8, *(const uint4*)(dz1s + (16 * T + nn) * 32 + 8 * g));
        }
        const bf16x8 ax = __builtin_bit_cast(bf16x8, *(const uint4*)(xts + nn * 32 + 8 * g));
#pragma unroll
        for (int Tk = 0; Tk < 4; ++Tk)
#pragma unroll
            for (int Tu = 0; Tu < 4; ++Tu) gW2[Tk][Tu] = mfma(ah[Tk], bz[Tu], gW2[Tk][Tu]);
#pragma unroll
        for (int T = 0; T < 4; ++T) gW1[T] = mfma(ax, bz1[T], gW1[T]);
        __syncthreads();
    }
    // reduce the per-lane vectors over the 16 triplet lanes of each group
    float* out = part + (size_t)blockIdx.x * (kNP + 1);
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float a = gb1[T][i], b = gb2[T][i], c = gw3[T][i];
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                a += __shfl_xor(a, d, 64);
                b += __shfl_xor(b, d, 64);
                c += __shfl_xor(c, d, 64);
            }
            if (nn == 0) {
                const int u = 16 * T + 4 * g + i;
                out[mB1 + u] = a;
                out[mB2 + u] = b;
                out[mW3 + u] = c;
            }
        }
    // accumulator tiles: lane (g, col) holds rows 4g+i of column col
#pragma unroll
    for (int Tk = 0; Tk < 4; ++Tk)
#pragma unroll
        for (int Tu = 0; Tu < 4; ++Tu)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[mW2 + (16 * Tk + 4 * g + i) * 64 + 16 * Tu + nn] = gW2[Tk][Tu][i];
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = 4 * g + i;
            if (f < 12) out[mW1 + f * 64 + 16 * T + nn] = gW1[T][i];
        }
    float s3 = gb3, sl = loss;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        s3 += __shfl_xor(s3, d, 64);
        sl += __shfl_xor(sl, d, 64);
    }
    if (lane == 0) {
        out[mB3] = s3;
        out[kNP] = sl;
    }
}

// Sum the block partials in a fixed order; optionally apply Adam and repack the weights.
__global__ __launch_bounds__(256) void k_reduce_adam(const float* __restrict__ part, int n_part, int batch,
                                                     float* __restrict__ grad, float* __restrict__ loss, float* master,
                                                     float* m, float* v, int step, float lr, float b1, float b2,
                                                     float eps) {
    for (int i = threadIdx.x; i <= kNP; i += blockDim.x) {
        float s = 0.f;
        for (int b = 0; b < n_part; ++b) s += part[(size_t)b * (kNP + 1) + i];
        if (i == kNP) {
            if (loss) *loss = s / (float)batch;
            continue;
        }
        if (grad) grad[i] = s;
        if (master) {
            const float mi = b1 * m[i] + (1.f - b1) * s;
            const float vi = b2 * v[i] + (1.f - b2) * s * s;
            m[i] = mi;
            v[i] = vi;
            const float mh = mi / (1.f - powf(b1, (float)step));
            const float vh = vi / (1.f - powf(b2, (float)step));
            master[i] -= lr * mh / (sqrtf(vh) + eps);
        }
    }
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock > 0 ? (n + kBlock - 1) / kBlock : 1); }

}  // namespace

size_t mlp_q_floats() { return (kQBytes + 3) / 4; }

void mlp_quantize(const float* master, float* q, hipStream_t s) {
    k_quantize<<<1, 256, 0, s>>>(master, (uint8_t*)q);
}

void mlp_infer(const float* q, const float* feats, int64_t n, float* logits, hipStream_t s) {
    if (n <= 0) return;
    int64_t tiles = (n + 15) / 16;
    int64_t nb = (tiles + kInferWaves - 1) / kInferWaves;
    if (nb > 8192) nb = 8192;
    k_infer<<<(unsigned)nb, 64 * kInferWaves, 0, s>>>((const uint8_t*)q, feats, n, logits);
}

void neighbours_mlp(const GridDesc& g, const KParams& kp, const Hit* hits, const uint32_t* bin_off, int64_t n_max,
                    uint32_t* counters, const float* q, int32_t* up, int32_t* dn, uint32_t* ovf, void* cand,
                    uint32_t* nund, uint32_t* wrec, hipStream_t s, hipStream_t aux, hipEvent_t ev_fork,
                    hipEvent_t ev_join) {
    const int64_t waves = (n_max + 63) / 64;
    const unsigned nb = (unsigned)((waves + kPW - 1) / kPW > 0 ? (waves + kPW - 1) / kPW : 1);
    const uint32_t seg_cap = (uint32_t)(nb_cand_entries(n_max) / kTallyLines);
    k_nb_cand<<<blocks(n_max), kBlock, 0, s>>>(g, kp, hits, bin_off, counters, (Cand*)cand, seg_cap, nund, wrec, up,
                                                dn, ovf);
    // Waves whose candidates overflowed the list (dense noise near the inner rows of a time
    // frame) are enumerated per lane by the fallback, grid-stride over the overflow list; it
    // writes other hits' links than the scoring kernel, so the two run side by side when a
    // second stream is given (a few heavy waves make the fallback a long tail).
    const bool fork = aux && ev_fork && ev_join;
    hipStream_t sf = s;
    if (fork && hipEventRecord(ev_fork, s) == hipSuccess && hipStreamWaitEvent(aux, ev_fork, 0) == hipSuccess) sf = aux;
    k_nb_mlp_fallback<<<1024, 64 * kNbWaves, 0, sf>>>(g, kp, hits, bin_off, counters, (const uint8_t*)q, ovf, up, dn);
    k_nb_score<<<nb, 64 * kPW, 0, s>>>(g, kp, hits, counters, (const uint8_t*)q, (const Cand*)cand, nund, wrec, up,
                                       dn);
    if (sf != s) {
        (void)hipEventRecord(ev_join, aux);
        (void)hipStreamWaitEvent(s, ev_join, 0);
    }
}

size_t nb_overflow_entries(int64_t n_max) { return (size_t)((n_max + 63) / 64 + 1); }

// room for three candidate records per hit (typical events use about two), and
// at least one full wave list per segment; a wave that does not fit its segment
// goes to the overflow list
size_t nb_cand_entries(int64_t n_max) {
    int64_t e = 3 * n_max;
    if (e < (int64_t)kTallyLines * kCapC) e = (int64_t)kTallyLines * kCapC;
    if (e > 0xF0000000ll) e = 0xF0000000ll;
    return (size_t)(e / kTallyLines * kTallyLines);
}

void triplet_count(const GridDesc& g, const KParams& kp, const Hit* hits, const uint32_t* bin_off, int64_t n_max,
                   const uint32_t* counters, uint32_t* cnt, hipStream_t s) {
    k_trip_count<<<blocks(n_max), kBlock, 0, s>>>(g, kp, hits, bin_off, counters, cnt);
}

void triplet_write(const GridDesc& g, const KParams& kp, const Hit* hits, const uint32_t* bin_off, int64_t n_max,
                   const uint32_t* counters, const uint32_t* off, int32_t* trip, float* feats, int64_t cap,
                   hipStream_t s) {
    k_trip_write<<<blocks(n_max), kBlock, 0, s>>>(g, kp, hits, bin_off, counters, off, trip, feats, cap);
}

int mlp_grad_blocks(int batch) { return (batch + kTrainChunk - 1) / kTrainChunk; }

void mlp_grad_step(const float* q, const float* feats, const uint8_t* labels, const int32_t* idx, int batch,
                   float* part, hipStream_t s) {
    k_train_grad<<<mlp_grad_blocks(batch), 64, 0, s>>>((const uint8_t*)q, feats, labels, idx, batch, part);
}

void mlp_reduce(const float* part, int batch, float* grad, float* loss, float* master, float* m, float* v, int step,
                float lr, float b1, float b2, float eps, hipStream_t s) {
    k_reduce_adam<<<1, 256, 0, s>>>(part, mlp_grad_blocks(batch), batch, grad, loss, master, m, v, step, lr, b1, b2,
                                    eps);
}

}  // namespace tpc
