/*
 * FP64 / integer CPU oracle of the TPC cluster compression (TEST INFRASTRUCTURE ONLY).
 *
 * Sec. 4 of arXiv:1910.12214 (TPC data reduction), steps 2-4:
 *   step 2: cluster properties converted to integers; charge and size with a dynamic
 *           precision -- the leading one and the n bits after it are kept, the rest is
 *           rounded away (n = 4 for the charge, n = 3 for the sizes);
 *   step 3: clusters on tracks stored as residuals to the extrapolated track, the others
 *           ordered in z and y and stored as differences to the previous cluster;
 *   step 4: entropy coding -- ANS (here: range ANS) against Huffman coding.
 * Plain, sequential C.  Shares no code with the HIP library; compiled into the oracle's
 * library next to tpc_oracle.c (whose helix propagation or_propagate gives the predictions).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int or_propagate(const double p0[5], double x0, double x1, double kq, double s_max, double tie_rel,
                 double p1[5], double F[25], int* flag);

/* ---- step 2: dynamic precision ------------------------------------------------------ */

/* Keep the leading one of v and the n bits after it; the bits below are rounded to the
 * nearest multiple (half up; a carry may lengthen the number by one bit). */
uint32_t or_dynprec(uint32_t v, int n) {
    if (v == 0) return 0;
    int p = 31;
    while (!((v >> p) & 1u)) --p; /* leading one */
    if (p <= n) return v;
    const int e = p - n;
    const uint64_t r = ((uint64_t)v + (1ull << (e - 1))) >> e;
    return (uint32_t)(r << e);
}

/* Symbol of a dynamic-precision value: (e << (n + 1)) | (v >> e), e = max(0, leading bit - n). */
uint32_t or_dynprec_code(uint32_t v, int n) {
    int p = 0;
    for (int b = 31; b >= 0; --b)
        if ((v >> b) & 1u) {
            p = b;
            break;
        }
    const int e = p > n ? p - n : 0;
    return ((uint32_t)e << (n + 1)) | (v >> e);
}

uint32_t or_dynprec_decode(uint32_t code, int n) {
    const uint32_t e = code >> (n + 1), m = code & ((1u << (n + 1)) - 1u);
    return m << e;
}

/* ---- step 3: track-model prediction -------------------------------------------------- */

/* Predicted position of hit i of a track: its reference state p (y, z, sin phi, dz/ds, q/pT
 * at x_ref) carried along the helix to x_row[i] in one closed-form step.  fail[i] = 1 when the
 * step fails (|sin phi| reaches s_max) or is not finite. */
void or_predict(int64_t n, const double* p5, const double* x_ref, const double* x_row, double kq, double s_max,
                double* y_out, double* z_out, int32_t* fail) {
    for (int64_t i = 0; i < n; ++i) {
        double p1[5];
        const int bad = or_propagate(p5 + 5 * i, x_ref[i], x_row[i], kq, s_max, 0.0, p1, NULL, NULL);
        const int f = bad || !isfinite(p1[0]) || !isfinite(p1[1]);
        y_out[i] = f ? 0.0 : p1[0];
        z_out[i] = f ? 0.0 : p1[1];
        fail[i] = f;
    }
}

/* ---- step 4: range ANS ----------------------------------------------------------------
 * State x in [2^23, 2^31); symbols of probability f/2^P (P <= 16); output in bytes.
 * Encoding symbol s (frequency f, cumulative c): while x >= f * 2^(31-P) emit the low byte
 * and shift x right by 8; then x <- floor(x / f) * 2^P + (x mod f) + c.  The encoder runs
 * backwards over a block starting from x = 2^23 and finally emits x as four bytes; the
 * decoder reads the block forwards: slot = x mod 2^P gives s (c <= slot < c + f),
 * x <- f * (x >> P) + slot - c, and bytes are read while x < 2^23. */

/* Frequencies of the present symbols summing to 2^P: 1 + floor(count (2^P - n_present) / total)
 * each, the remainder to the most frequent symbol (lowest symbol on ties).  Returns n_present,
 * or -1 when 2^P < n_present. */
int or_ans_freqs(const uint32_t* count, int n_sym, int P, uint32_t* freq) {
    uint64_t total = 0;
    int present = 0, top = -1;
    for (int s = 0; s < n_sym; ++s) {
        total += count[s];
        if (count[s]) {
            ++present;
            if (top < 0 || count[s] > count[top]) top = s;
        }
    }
    memset(freq, 0, sizeof(uint32_t) * (size_t)n_sym);
    if (present == 0) return 0;
    const uint64_t M = 1ull << P;
    if ((uint64_t)present > M) return -1;
    uint64_t sum = 0;
    for (int s = 0; s < n_sym; ++s)
        if (count[s]) {
            freq[s] = (uint32_t)(1 + (uint64_t)count[s] * (M - (uint64_t)present) / total);
            sum += freq[s];
        }
    freq[top] += (uint32_t)(M - sum);
    return present;
}

/* Encode syms[0..n) as one block.  out[] receives the block's bytes in decoding order (the
 * final state first, most significant byte first); returns their number (<= 2 n + 4). */
int64_t or_ans_encode_block(const uint16_t* syms, int64_t n, const uint32_t* freq, const uint32_t* cum, int P,
                            uint8_t* out) {
    uint8_t* tmp = (uint8_t*)malloc((size_t)(2 * n + 4));
    int64_t w = 0;
    uint32_t x = 1u << 23;
    for (int64_t i = n - 1; i >= 0; --i) {
        const uint32_t f = freq[syms[i]], c = cum[syms[i]];
        const uint64_t x_max = (uint64_t)f << (31 - P);
        while ((uint64_t)x >= x_max) {
            tmp[w++] = (uint8_t)(x & 0xFFu);
            x >>= 8;
        }
        x = ((x / f) << P) + (x % f) + c;
    }
    for (int b = 0; b < 4; ++b) out[b] = (uint8_t)(x >> (24 - 8 * b));
    for (int64_t k = 0; k < w; ++k) out[4 + k] = tmp[w - 1 - k];
    free(tmp);
    return w + 4;
}

/* Decode n symbols of one block; returns the number of bytes read, or -1 on malformed input. */
int64_t or_ans_decode_block(const uint8_t* in, int64_t n_bytes, int64_t n, const uint32_t* freq,
                            const uint32_t* cum, const uint16_t* slot_sym, int P, uint16_t* syms) {
    if (n_bytes < 4) return -1;
    uint32_t x = ((uint32_t)in[0] << 24) | ((uint32_t)in[1] << 16) | ((uint32_t)in[2] << 8) | in[3];
    int64_t r = 4;
    const uint32_t mask = (1u << P) - 1u;
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t slot = x & mask;
        const uint16_t s = slot_sym[slot];
        syms[i] = s;
        x = freq[s] * (x >> P) + slot - cum[s];
        while (x < (1u << 23)) {
            if (r >= n_bytes) return -1;
            x = (x << 8) | in[r++];
        }
    }
    return r;
}

/* ---- Huffman code lengths (the comparison coder) -------------------------------------
 * Optimal prefix code lengths for the present symbols by repeatedly merging the two least
 * frequent subtrees (ties: the subtree created first, leaves before merged nodes); a single
 * present symbol gets length 1.  Returns the total coded length in bits. */
uint64_t or_huffman_lengths(const uint32_t* count, int n_sym, uint8_t* len) {
    int n = 0;
    for (int s = 0; s < n_sym; ++s) n += count[s] != 0;
    memset(len, 0, (size_t)n_sym);
    if (n == 0) return 0;
    if (n == 1) {
        uint64_t bits = 0;
        for (int s = 0; s < n_sym; ++s)
            if (count[s]) {
                len[s] = 1;
                bits = count[s];
            }
        return bits;
    }
    /* node arrays: leaves 0..n-1 (sorted by count, then symbol), internal n..2n-2 */
    const int nn = 2 * n - 1;
    uint64_t* w = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nn);
    int* parent = (int*)malloc(sizeof(int) * (size_t)nn);
    int* sym = (int*)malloc(sizeof(int) * (size_t)n);
    int k = 0;
    for (int s = 0; s < n_sym; ++s)
        if (count[s]) sym[k++] = s;
    /* insertion sort of the leaves by (count, symbol) -- alphabets here are small */
    for (int i = 1; i < n; ++i) {
        int v = sym[i], j = i - 1;
        while (j >= 0 && (count[sym[j]] > count[v] || (count[sym[j]] == count[v] && sym[j] > v))) {
            sym[j + 1] = sym[j];
            --j;
        }
        sym[j + 1] = v;
    }
    for (int i = 0; i < n; ++i) w[i] = count[sym[i]];
    int leaf = 0, node = n, made = n; /* two queues: leaves in order, internal nodes in creation order */
    for (int m = 0; m < n - 1; ++m) {
        int pick[2];
        for (int t = 0; t < 2; ++t) {
            if (leaf < n && (node >= made || w[leaf] <= w[node])) pick[t] = leaf++;
            else pick[t] = node++;
        }
        w[made] = w[pick[0]] + w[pick[1]];
        parent[pick[0]] = parent[pick[1]] = made;
        ++made;
    }
    parent[nn - 1] = -1;
    uint64_t bits = 0;
    for (int i = 0; i < n; ++i) {
        int d = 0;
        for (int v = i; parent[v] >= 0; v = parent[v]) ++d;
        len[sym[i]] = (uint8_t)(d > 255 ? 255 : d);
        bits += (uint64_t)count[sym[i]] * (uint64_t)d;
    }
    free(w);
    free(parent);
    free(sym);
    return bits;
}
