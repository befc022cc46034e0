/*
 * FP64 CPU ORACLE for per-sector cellular-automaton TPC track finding.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP library.
 *
 * The paper (Sec. 2 and Sec. 3) states that the Run 3 TPC tracking derives
 * from the Run 2 HLT GPU tracker and must give the same physics on CPU and
 * GPU (Sec. 3: a hit near two tracks must not be assigned by processing
 * order).  It does not spell out the steps; this file follows the written
 * reading of each step (grid, neighbour finding, cleaning, start hits,
 * two-pass Kalman tracklets, selection) step by step, in double precision,
 * with plain loops, no fusion and no reordering beyond what each step states.
 *
 * Every arg-min and every cut decision also records a near-tie flag: a
 * relative gap below tie_rel between the best and second-best value, or a
 * value within tie_rel of its cut.  Parity checks exclude flagged decisions.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- types */
typedef struct {
    double win_y, win_z;        /* neighbour window slopes (|dy| <= win_y * dx) */
    double nb_chi2_max;         /* neighbour criterion cut D_max */
    double fol_chi2_max;        /* following / link-acceptance chi2 cut */
    double sigma_y, sigma_z;    /* cluster errors (cm) */
    double s_max;               /* propagation fails if |sin phi| >= s_max */
    double edge_margin;         /* stop if |y| > x tan(half) + margin */
    int32_t l_min_chain, n_miss_max, n_min_tracklet, n_min_track;
    double c0_sinphi, c0_dzds, c0_qpt; /* initial variances of s, t, q/pT */
    float bin_y, bin_z;         /* grid bin size (cm): enumeration only */
    double tie_rel;             /* near-tie threshold */
    const double* mlp;          /* 5057 parameters (BF16-valued) or NULL */
    double mlp_tau_logit;       /* keep a pair iff logit >= tau */
    double mlp_flag_abs;        /* flag a pair if |logit - tau| <= this */
} or_params_t;

typedef struct {
    int64_t n;
    const float *y, *z;
    const uint8_t *row, *sector;
    int32_t n_rows;
    const float* row_x;
    float tan_half;
    int32_t n_sectors;
    float z_min, z_max;
    double bz;
    int32_t n_threads;
} or_input_t;

/* near-tie flag bits */
enum {
    F_ARGMIN = 1, F_CUT = 2, F_WINDOW = 4, F_SMAX = 8, F_EDGE = 16, F_MLP = 32
};

typedef struct {
    /* grid */
    int64_t n_valid, n_bins;
    uint32_t* sorted_id;   /* [n_valid] cluster id at sorted position */
    uint32_t* row_off;     /* [S*R+1] */
    uint32_t* bin_base;    /* [S*R+1] first bin of each row-sector */
    uint32_t* bin_off;     /* [n_bins+1] */
    /* links in cluster-id space, -1 = none */
    int32_t *up, *dn, *up_c, *dn_c;
    uint8_t* nb_flag;      /* [n] near-tie flags of the neighbour decision */
    int32_t* n_pairs;      /* [n] window pairs considered (before cut / pruning) */
    /* starts, ascending cluster id */
    int64_t n_starts;
    uint32_t* start_id;
    /* tracklets, one per start */
    int32_t* tl_nhits;
    int32_t* tl_hits;      /* [n_starts * R], -1 = no hit in that row */
    double* tl_state;      /* [n_starts * 5] at x_ref */
    double* tl_cov;        /* [n_starts * 15] lower triangle, row-major */
    double* tl_chi2;
    int32_t* tl_ndf;
    int32_t* tl_row_ref;   /* row of the innermost hit */
    uint8_t* tl_valid;
    uint8_t* tl_fail;
    uint8_t* tl_flag;
    /* selection */
    uint64_t* hit_key;     /* [n] */
    int64_t n_tracks, n_track_hits;
    int32_t* trk_tl;       /* tracklet index of each track */
    int32_t* trk_off;      /* [n_tracks+1] */
    int32_t* trk_hits;     /* cluster ids, row-ascending */
    int64_t n_fit_fail, n_links_raw, n_links_clean;
} or_output_t;

/* ------------------------------------------------------------ small math */
static void sym_unpack(const double c[15], double M[5][5]) {
    int k = 0;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) { M[i][j] = c[k]; M[j][i] = c[k]; ++k; }
}
static void sym_pack(double M[5][5], double c[15]) {
    int k = 0;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) c[k++] = 0.5 * (M[i][j] + M[j][i]);
}

/* g(u) = asin(u)/u and its derivative (series near 0) */
static void asin_over(double u, double* g, double* gp) {
    if (fabs(u) < 1e-2) {
        double u2 = u * u;
        *g = 1.0 + u2 * (1.0 / 6.0 + u2 * (3.0 / 40.0 + u2 * (5.0 / 112.0 + u2 * (35.0 / 1152.0))));
        *gp = u * (1.0 / 3.0 + u2 * (3.0 / 10.0 + u2 * (15.0 / 56.0 + u2 * (35.0 / 144.0))));
    } else {
        double a = asin(u);
        *g = a / u;
        *gp = (u / sqrt(1.0 - u * u) - a) / (u * u);
    }
}

/*
 * Sector-local helix propagation of p = (y, z, s = sin phi, t = dz/ds, q = q/pT)
 * from x0 to x1 (either direction).  kq = -c Bz, curvature k = kq q.
 *   s1 = s0 + k dx,  dy = dx (s0+s1)/(c0+c1),
 *   chord L = sign(dx) sqrt(dx^2+dy^2),  arc = L asin(kL/2)/(kL/2),  dz = t arc.
 * F (row-major 5x5) is the exact derivative dp1/dp0.  Returns 1 on failure.
 */
int or_propagate(const double p0[5], double x0, double x1, double kq, double s_max, double tie_rel,
                 double p1[5], double F[25], int* flag) {
    double dx = x1 - x0;
    double k = kq * p0[4];
    double s0 = p0[2], s1 = s0 + k * dx;
    if (flag && fabs(fabs(s1) - s_max) <= tie_rel * s_max) *flag |= F_SMAX;
    if (!(fabs(s1) < s_max) || !(fabs(s0) < s_max)) return 1;
    for (int i = 0; i < 25; ++i) if (F) F[i] = (i % 6 == 0) ? 1.0 : 0.0;
    if (dx == 0.0) { memcpy(p1, p0, 5 * sizeof(double)); return 0; }
    double c0 = sqrt(1.0 - s0 * s0), c1 = sqrt(1.0 - s1 * s1);
    double A = s0 + s1, B = c0 + c1;
    double dy = dx * A / B;
    double L = copysign(sqrt(dx * dx + dy * dy), dx);
    double u = 0.5 * k * L;
    double g, gp;
    asin_over(u, &g, &gp);
    double arc = L * g;
    double t = p0[3];
    p1[0] = p0[0] + dy;
    p1[1] = p0[1] + t * arc;
    p1[2] = s1;
    p1[3] = t;
    p1[4] = p0[4];
    if (F) {
        double dA_s = 2.0, dA_q = kq * dx;
        double dB_s = -s0 / c0 - s1 / c1, dB_q = -(s1 / c1) * kq * dx;
        double dy_s = dx * (dA_s * B - A * dB_s) / (B * B);
        double dy_q = dx * (dA_q * B - A * dB_q) / (B * B);
        double dL_s = dy / L * dy_s, dL_q = dy / L * dy_q;
        double du_s = 0.5 * k * dL_s, du_q = 0.5 * kq * L + 0.5 * k * dL_q;
        double darc_s = dL_s * g + L * gp * du_s;
        double darc_q = dL_q * g + L * gp * du_q;
        F[0 * 5 + 2] = dy_s;
        F[0 * 5 + 4] = dy_q;
        F[1 * 5 + 2] = t * darc_s;
        F[1 * 5 + 3] = arc;
        F[1 * 5 + 4] = t * darc_q;
        F[2 * 5 + 4] = kq * dx;
    }
    return 0;
}

/* C <- F C F^T (no process noise) */
void or_cov_propagate(double c[15], const double F[25]) {
    double C[5][5], T[5][5], R[5][5];
    sym_unpack(c, C);
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            double s = 0;
            for (int k = 0; k < 5; ++k) s += F[i * 5 + k] * C[k][j];
            T[i][j] = s;
        }
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            double s = 0;
            for (int k = 0; k < 5; ++k) s += T[i][k] * F[j * 5 + k];
            R[i][j] = s;
        }
    sym_pack(R, c);
}

/* residual chi2 of measurement (my, mz) against the predicted state, with S = HCH^T + V */
static double chi2_of(const double p[5], const double c[15], double my, double mz, double vy, double vz) {
    double syy = c[0] + vy, syz = c[1], szz = c[2] + vz;
    double det = syy * szz - syz * syz;
    double ry = my - p[0], rz = mz - p[1];
    return (ry * ry * szz - 2.0 * ry * rz * syz + rz * rz * syy) / det;
}

/* Kalman update with m = (my, mz), H = [I2 0], V = diag(vy, vz).
 * Returns 1 on a fit failure (non-finite values or a non-positive diagonal). */
int or_kf_update(double p[5], double c[15], double my, double mz, double vy, double vz, double* chi2) {
    double C[5][5];
    sym_unpack(c, C);
    double syy = C[0][0] + vy, syz = C[0][1], szz = C[1][1] + vz;
    double det = syy * szz - syz * syz;
    double i00 = szz / det, i01 = -syz / det, i11 = syy / det;
    double ry = my - p[0], rz = mz - p[1];
    if (chi2) *chi2 = ry * (i00 * ry + i01 * rz) + rz * (i01 * ry + i11 * rz);
    double K[5][2];
    for (int i = 0; i < 5; ++i) {
        K[i][0] = C[i][0] * i00 + C[i][1] * i01;
        K[i][1] = C[i][0] * i01 + C[i][1] * i11;
    }
    for (int i = 0; i < 5; ++i) p[i] += K[i][0] * ry + K[i][1] * rz;
    double N[5][5];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) N[i][j] = C[i][j] - (K[i][0] * C[0][j] + K[i][1] * C[1][j]);
    sym_pack(N, c);
    int bad = !(det > 0.0);
    for (int i = 0; i < 5; ++i) bad |= !isfinite(p[i]);
    for (int i = 0; i < 15; ++i) bad |= !isfinite(c[i]);
    bad |= !(c[0] > 0 && c[2] > 0 && c[5] > 0 && c[9] > 0 && c[14] > 0);
    return bad;
}

/* ------------------------------------------------------------- the MLP */
/* Parameter layout: W1[12][64], b1[64], W2[64][64], b2[64], w3[64], b3. */
double or_mlp_logit(const double* w, const double f[12]) {
    const double *W1 = w, *b1 = w + 768, *W2 = w + 832, *b2 = w + 4928, *w3 = w + 4992, *b3 = w + 5056;
    double h1[64], h2[64];
    for (int j = 0; j < 64; ++j) {
        double s = b1[j];
        for (int i = 0; i < 12; ++i) s += W1[i * 64 + j] * f[i];
        h1[j] = s > 0 ? s : 0;
    }
    for (int j = 0; j < 64; ++j) {
        double s = b2[j];
        for (int i = 0; i < 64; ++i) s += W2[i * 64 + j] * h1[i];
        h2[j] = s > 0 ? s : 0;
    }
    double s = b3[0];
    for (int j = 0; j < 64; ++j) s += w3[j] * h2[j];
    return s;
}

/* ------------------------------------------------------------ the grid */
typedef struct {
    const or_input_t* in;
    const or_params_t* prm;
    int R, S;
    double* x;          /* row radii as double */
    float* ymin;        /* per row, fp32: -(row_x * tan_half) */
    int32_t* ny;        /* per row */
    int32_t nz;
    float inv_by, inv_bz;
    or_output_t* out;
    double kq;
} ctx_t;

static int32_t bin_iy(const ctx_t* g, int r, float y) {
    float v = (y - g->ymin[r]) * g->inv_by;
    if (!(v > 0.0f)) return 0;
    if (v >= (float)g->ny[r]) return g->ny[r] - 1;
    return (int32_t)v;
}
static int32_t bin_iz(const ctx_t* g, float z) {
    float v = (z - g->in->z_min) * g->inv_bz;
    if (!(v > 0.0f)) return 0;
    if (v >= (float)g->nz) return g->nz - 1;
    return (int32_t)v;
}

typedef struct { uint64_t key; uint32_t id; } sortrec_t;
static int cmp_rec(const void* a, const void* b) {
    const sortrec_t *x = (const sortrec_t*)a, *y = (const sortrec_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

/* Row-binned grid: per (sector,row) a uniform ny x nz bin grid, bins z-major,
 * hits ordered by (sector, row, bin, cluster id). */
static void build_grid(ctx_t* g) {
    const or_input_t* in = g->in;
    int R = g->R, S = g->S;
    or_output_t* o = g->out;
    o->bin_base = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(S * R + 1));
    uint64_t nb = 0;
    for (int s = 0; s < S; ++s)
        for (int r = 0; r < R; ++r) {
            o->bin_base[s * R + r] = (uint32_t)nb;
            nb += (uint64_t)g->ny[r] * (uint64_t)g->nz;
        }
    o->bin_base[S * R] = (uint32_t)nb;
    o->n_bins = (int64_t)nb;
    sortrec_t* rec = (sortrec_t*)malloc(sizeof(sortrec_t) * (size_t)(in->n > 0 ? in->n : 1));
    int64_t nv = 0;
    for (int64_t i = 0; i < in->n; ++i) {
        int r = in->row[i], s = in->sector[i];
        if (r >= R || s >= S) continue;
        int32_t b = bin_iz(g, in->z[i]) * g->ny[r] + bin_iy(g, r, in->y[i]);
        rec[nv].key = (uint64_t)o->bin_base[s * R + r] + (uint64_t)b;
        rec[nv].id = (uint32_t)i;
        ++nv;
    }
    qsort(rec, (size_t)nv, sizeof(sortrec_t), cmp_rec);
    o->n_valid = nv;
    o->sorted_id = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nv > 0 ? nv : 1));
    o->bin_off = (uint32_t*)calloc((size_t)nb + 1, sizeof(uint32_t));
    o->row_off = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(S * R + 1));
    for (int64_t k = 0; k < nv; ++k) { o->sorted_id[k] = rec[k].id; o->bin_off[rec[k].key + 1]++; }
    for (uint64_t b = 0; b < nb; ++b) o->bin_off[b + 1] += o->bin_off[b];
    for (int rs = 0; rs <= S * R; ++rs) o->row_off[rs] = o->bin_off[o->bin_base[rs]];
    free(rec);
}

/* Calls fn(id) for every hit of row-sector (s,r) in the bins overlapping
 * [y0,y1] x [z0,z1] (one extra bin on every side: the window tests are exact).
 * Hits beyond the grid's range sit in its edge bins, so the bin range is clamped
 * to the grid: a box beyond the grid visits the edge bins (bins only enumerate
 * candidates, whatever the coordinates).  NaN bounds visit nothing. */
typedef void (*visit_fn)(void* st, uint32_t id);
static void visit_box(const ctx_t* g, int s, int r, double y0, double y1, double z0, double z1, visit_fn fn, void* st) {
    const or_output_t* o = g->out;
    int ny = g->ny[r], nz = g->nz;
    double fy0 = floor((y0 - (double)g->ymin[r]) * (double)g->inv_by) - 1;
    double fy1 = floor((y1 - (double)g->ymin[r]) * (double)g->inv_by) + 1;
    double fz0 = floor((z0 - (double)g->in->z_min) * (double)g->inv_bz) - 1;
    double fz1 = floor((z1 - (double)g->in->z_min) * (double)g->inv_bz) + 1;
    if (!(fy0 <= fy1) || !(fz0 <= fz1)) return;
    int iy0 = fy0 < 0 ? 0 : (fy0 > ny - 1 ? ny - 1 : (int)fy0);
    int iy1 = fy1 < 0 ? 0 : (fy1 > ny - 1 ? ny - 1 : (int)fy1);
    int iz0 = fz0 < 0 ? 0 : (fz0 > nz - 1 ? nz - 1 : (int)fz0);
    int iz1 = fz1 < 0 ? 0 : (fz1 > nz - 1 ? nz - 1 : (int)fz1);
    uint32_t base = o->bin_base[s * g->R + r];
    for (int iz = iz0; iz <= iz1; ++iz) {
        uint32_t b0 = base + (uint32_t)(iz * ny + iy0), b1 = base + (uint32_t)(iz * ny + iy1);
        for (uint32_t k = o->bin_off[b0]; k < o->bin_off[b1 + 1]; ++k) fn(st, o->sorted_id[k]);
    }
}

/* --------------------------------------------------------- neighbours */
typedef struct { uint32_t* v; int n, cap; } idlist_t;
static void idl_push(void* st, uint32_t id) {
    idlist_t* l = (idlist_t*)st;
    if (l->n == l->cap) { l->cap = l->cap ? 2 * l->cap : 16; l->v = (uint32_t*)realloc(l->v, sizeof(uint32_t) * (size_t)l->cap); }
    l->v[l->n++] = id;
}

/* window test |a - b| <= w with a near-boundary flag */
static int in_win(double d, double w, double tie, int* flag) {
    double a = fabs(d);
    if (fabs(a - w) <= tie * w) *flag |= F_WINDOW;
    return a <= w;
}

/* Triplet descriptor for the learned scorer (12 features). */
void or_features(double xd, double yd, double zd, double xm, double ym, double zm, double xu, double yu, double zu,
                 double win_y, double win_z, int n_up, int n_dn, double f[12]) {
    double dxd = xm - xd, dxu = xu - xm, dxt = xu - xd;
    f[0] = (xd - 166.0) / 81.0;
    f[1] = (xm - 166.0) / 81.0;
    f[2] = (xu - 166.0) / 81.0;
    f[3] = (yd - ym) / (win_y * dxd);
    f[4] = (yu - ym) / (win_y * dxu);
    f[5] = (zd - zm) / (win_z * dxd);
    f[6] = (zu - zm) / (win_z * dxu);
    f[7] = (yu - yd) / dxt;
    f[8] = (zu - zd) / dxt;
    double ax = xm - xd, ay = ym - yd, bx = xu - xm, by = yu - ym, cx = xu - xd, cy = yu - yd;
    double cross = ax * cy - ay * cx;
    double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by), lc = sqrt(cx * cx + cy * cy);
    f[9] = 10.0 * 2.0 * cross / (la * lb * lc);
    f[10] = 0.25 * n_up;
    f[11] = 0.25 * n_dn;
}

typedef struct { int64_t lo, hi; ctx_t* g; } range_t;

static void* neighbours_range(void* arg) {
    range_t* rg = (range_t*)arg;
    ctx_t* g = rg->g;
    const or_input_t* in = g->in;
    const or_params_t* P = g->prm;
    or_output_t* o = g->out;
    idlist_t U = {0}, D = {0};
    const double vy15 = 1.5 * P->sigma_y * P->sigma_y, vz15 = 1.5 * P->sigma_z * P->sigma_z;
    for (int64_t k = rg->lo; k < rg->hi; ++k) {
        uint32_t m = o->sorted_id[k];
        int r = in->row[m], s = in->sector[m];
        o->up[m] = -1; o->dn[m] = -1; o->nb_flag[m] = 0; o->n_pairs[m] = 0;
        if (r == 0 || r == g->R - 1) continue;
        double xm = g->x[r], xu = g->x[r + 1], xd = g->x[r - 1];
        double ym = in->y[m], zm = in->z[m];
        double wyu = P->win_y * (xu - xm), wzu = P->win_z * (xu - xm);
        double wyd = P->win_y * (xm - xd), wzd = P->win_z * (xm - xd);
        int flag = 0;
        /* window candidates, exact tests */
        U.n = 0; D.n = 0;
        visit_box(g, s, r + 1, ym - wyu, ym + wyu, zm - wzu, zm + wzu, idl_push, &U);
        visit_box(g, s, r - 1, ym - wyd, ym + wyd, zm - wzd, zm + wzd, idl_push, &D);
        int nu = 0, nd = 0;
        for (int i = 0; i < U.n; ++i) {
            uint32_t c = U.v[i];
            int a = in_win((double)in->y[c] - ym, wyu, P->tie_rel, &flag);
            int b = in_win((double)in->z[c] - zm, wzu, P->tie_rel, &flag);
            if (a && b) U.v[nu++] = c;
        }
        for (int i = 0; i < D.n; ++i) {
            uint32_t c = D.v[i];
            int a = in_win((double)in->y[c] - ym, wyd, P->tie_rel, &flag);
            int b = in_win((double)in->z[c] - zm, wzd, P->tie_rel, &flag);
            if (a && b) D.v[nd++] = c;
        }
        o->n_pairs[m] = nu * nd;
        double best = INFINITY, second = INFINITY;
        int64_t bu = -1, bd = -1;
        for (int i = 0; i < nu; ++i)
            for (int j = 0; j < nd; ++j) {
                uint32_t u = U.v[i], d = D.v[j];
                double yu = in->y[u], zu = in->z[u], yd = in->y[d], zd = in->z[d];
                if (P->mlp) {
                    double f[12];
                    or_features(xd, yd, zd, xm, ym, zm, xu, yu, zu, P->win_y, P->win_z, nu, nd, f);
                    double lg = or_mlp_logit(P->mlp, f);
                    if (fabs(lg - P->mlp_tau_logit) <= P->mlp_flag_abs) flag |= F_MLP;
                    if (!(lg >= P->mlp_tau_logit)) continue;
                }
                double w = (xm - xd) / (xu - xd);
                double py = yd + (yu - yd) * w, pz = zd + (zu - zd) * w;
                double Dv = (ym - py) * (ym - py) / vy15 + (zm - pz) * (zm - pz) / vz15;
                if (fabs(Dv - P->nb_chi2_max) <= P->tie_rel * P->nb_chi2_max) flag |= F_CUT;
                if (!(Dv <= P->nb_chi2_max)) continue;
                int better = Dv < best || (Dv == best && (u < (uint32_t)bu || (u == (uint32_t)bu && d < (uint32_t)bd)));
                if (better) { second = best; best = Dv; bu = u; bd = d; }
                else if (Dv < second) second = Dv;
            }
        if (bu >= 0) {
            if (isfinite(second)) {
                double den = fabs(second) > 1e-12 ? fabs(second) : 1e-12;
                if ((second - best) / den < P->tie_rel) flag |= F_ARGMIN;
            }
            o->up[m] = (int32_t)bu;
            o->dn[m] = (int32_t)bd;
        }
        o->nb_flag[m] = (uint8_t)flag;
    }
    free(U.v); free(D.v);
    return NULL;
}

/* ----------------------------------------------------------- tracklets */
typedef struct {
    ctx_t* g;
    int s, r;
    double py, pz, bx, bz;   /* prediction and box half-sizes */
    double i00, i01, i11;    /* S^-1 */
    double cut, tie;
    double best, second;
    int64_t bid;
    int flag;
} search_t;

static void search_visit(void* st, uint32_t id) {
    search_t* q = (search_t*)st;
    const or_input_t* in = q->g->in;
    double ry = (double)in->y[id] - q->py, rz = (double)in->z[id] - q->pz;
    if (fabs(ry) > q->bx || fabs(rz) > q->bz) return;
    double c2 = ry * (q->i00 * ry + q->i01 * rz) + rz * (q->i01 * ry + q->i11 * rz);
    if (fabs(c2 - q->cut) <= q->tie * q->cut) q->flag |= F_CUT;
    if (!(c2 <= q->cut)) return;
    if (c2 < q->best || (c2 == q->best && id < (uint32_t)q->bid)) { q->second = q->best; q->best = c2; q->bid = id; }
    else if (c2 < q->second) q->second = c2;
}

/* Following search in row r: smallest chi2 inside the chi2 ellipse's bounding box. */
static int64_t follow_search(ctx_t* g, int s, int r, const double p[5], const double c[15], int* flag) {
    const or_params_t* P = g->prm;
    double vy = P->sigma_y * P->sigma_y, vz = P->sigma_z * P->sigma_z;
    search_t q;
    q.g = g; q.s = s; q.r = r; q.py = p[0]; q.pz = p[1];
    double syy = c[0] + vy, syz = c[1], szz = c[2] + vz;
    double det = syy * szz - syz * syz;
    q.i00 = szz / det; q.i01 = -syz / det; q.i11 = syy / det;
    q.cut = P->fol_chi2_max; q.tie = P->tie_rel;
    q.bx = sqrt(q.cut * syy); q.bz = sqrt(q.cut * szz);
    q.best = INFINITY; q.second = INFINITY; q.bid = -1; q.flag = 0;
    if (!(det > 0) || !isfinite(q.bx) || !isfinite(q.bz)) return -1;
    visit_box(g, s, r, p[0] - q.bx, p[0] + q.bx, p[1] - q.bz, p[1] + q.bz, search_visit, &q);
    if (q.bid >= 0 && isfinite(q.second)) {
        double den = fabs(q.second) > 1e-12 ? fabs(q.second) : 1e-12;
        if ((q.second - q.best) / den < q.tie) q.flag |= F_ARGMIN;
    }
    *flag |= q.flag;
    return q.bid;
}

static void c0_init(const or_params_t* P, double c[15]) {
    memset(c, 0, 15 * sizeof(double));
    c[0] = P->sigma_y * P->sigma_y;
    c[2] = P->sigma_z * P->sigma_z;
    c[5] = P->c0_sinphi;
    c[9] = P->c0_dzds;
    c[14] = P->c0_qpt;
}

/* propagate state and covariance; 1 = failure */
static int step_to(ctx_t* g, double p[5], double c[15], double x0, double x1, int* flag) {
    double F[25], p1[5];
    if (or_propagate(p, x0, x1, g->kq, g->prm->s_max, g->prm->tie_rel, p1, F, flag)) return 1;
    memcpy(p, p1, sizeof p1);
    or_cov_propagate(c, F);
    return 0;
}

static int edge_stop(ctx_t* g, int r, double y, int* flag) {
    double lim = g->x[r] * (double)g->in->tan_half + g->prm->edge_margin;
    if (fabs(fabs(y) - lim) <= g->prm->tie_rel * lim) *flag |= F_EDGE;
    return fabs(y) > lim;
}

static void build_tracklet(ctx_t* g, int64_t t) {
    const or_input_t* in = g->in;
    const or_params_t* P = g->prm;
    or_output_t* o = g->out;
    const int R = g->R;
    const double vy = P->sigma_y * P->sigma_y, vz = P->sigma_z * P->sigma_z;
    uint32_t h0 = o->start_id[t];
    int s = in->sector[h0], r0 = in->row[h0];
    int32_t* hits = o->tl_hits + (size_t)t * R;
    for (int r = 0; r < R; ++r) hits[r] = -1;
    int32_t hitsA[256];
    for (int r = 0; r < R; ++r) hitsA[r] = -1;
    int flag = 0, fail = 0;
    /* pass A: initialise from the start hit and its first link */
    uint32_t h1 = (uint32_t)o->up_c[h0];
    double x0 = g->x[r0], x1 = g->x[in->row[h1]];
    double ty = ((double)in->y[h1] - in->y[h0]) / (x1 - x0);
    double tz = ((double)in->z[h1] - in->z[h0]) / (x1 - x0);
    double p[5], c[15];
    p[0] = in->y[h0]; p[1] = in->z[h0];
    p[2] = ty / sqrt(1.0 + ty * ty);
    p[3] = tz * sqrt(1.0 - p[2] * p[2]);
    p[4] = 0.0;
    c0_init(P, c);
    hitsA[r0] = (int32_t)h0;
    int last = r0;
    double pl[5];
    memcpy(pl, p, sizeof p);
    int64_t next = h1;
    int on = 1, miss = 0;
    double x = x0;
    for (int r = r0 + 1; r < R && !fail; ++r) {
        if (step_to(g, p, c, x, g->x[r], &flag)) break;
        x = g->x[r];
        if (edge_stop(g, r, p[0], &flag)) break;
        int64_t acc = -1;
        if (on) {
            if (next >= 0 && in->row[next] == r) {
                double c2 = chi2_of(p, c, in->y[next], in->z[next], vy, vz);
                if (fabs(c2 - P->fol_chi2_max) <= P->tie_rel * P->fol_chi2_max) flag |= F_CUT;
                if (c2 <= P->fol_chi2_max) { acc = next; next = o->up_c[next]; }
                else on = 0;
            } else on = 0;
        }
        if (acc < 0) acc = follow_search(g, s, r, p, c, &flag);
        if (acc >= 0) {
            double c2;
            if (or_kf_update(p, c, in->y[acc], in->z[acc], vy, vz, &c2)) { fail = 1; break; }
            hitsA[r] = (int32_t)acc;
            last = r;
            memcpy(pl, p, sizeof p);
            miss = 0;
        } else if (++miss > P->n_miss_max) break;
    }
    /* pass B: re-initialise at the outermost pass-A hit, run inward */
    int nh = 0, inner = last;
    double chi2 = 0.0;
    int ndf = 0;
    double pin[5], cin[15];
    if (!fail) {
        uint32_t hb = (uint32_t)hitsA[last];
        p[0] = in->y[hb]; p[1] = in->z[hb]; p[2] = pl[2]; p[3] = pl[3]; p[4] = pl[4];
        c0_init(P, c);
        hits[last] = (int32_t)hb;
        nh = 1;
        memcpy(pin, p, sizeof p); memcpy(cin, c, sizeof c);
        x = g->x[last];
        miss = 0;
        for (int r = last - 1; r >= 0; --r) {
            if (step_to(g, p, c, x, g->x[r], &flag)) break;
            x = g->x[r];
            if (edge_stop(g, r, p[0], &flag)) break;
            int64_t acc = (r >= r0) ? hitsA[r] : follow_search(g, s, r, p, c, &flag);
            if (acc >= 0) {
                double c2;
                if (or_kf_update(p, c, in->y[acc], in->z[acc], vy, vz, &c2)) { fail = 1; break; }
                chi2 += c2;
                ndf += 2;
                hits[r] = (int32_t)acc;
                ++nh;
                inner = r;
                memcpy(pin, p, sizeof p); memcpy(cin, c, sizeof c);
                miss = 0;
            } else if (++miss > P->n_miss_max) break;
        }
    }
    if (fail) { nh = 0; for (int r = 0; r < R; ++r) hits[r] = -1; }
    o->tl_nhits[t] = nh;
    o->tl_fail[t] = (uint8_t)fail;
    o->tl_valid[t] = (uint8_t)(!fail && nh >= P->n_min_tracklet);
    o->tl_flag[t] = (uint8_t)flag;
    o->tl_chi2[t] = chi2;
    o->tl_ndf[t] = ndf;
    o->tl_row_ref[t] = inner;
    if (!fail) {
        memcpy(o->tl_state + t * 5, pin, sizeof pin);
        memcpy(o->tl_cov + t * 15, cin, sizeof cin);
    } else {
        memset(o->tl_state + t * 5, 0, 5 * sizeof(double));
        memset(o->tl_cov + t * 15, 0, 15 * sizeof(double));
    }
}

static void* tracklets_range(void* arg) {
    range_t* rg = (range_t*)arg;
    for (int64_t t = rg->lo; t < rg->hi; ++t) build_tracklet(rg->g, t);
    return NULL;
}

static void parallel(ctx_t* g, int64_t n, void* (*fn)(void*)) {
    int nt = g->in->n_threads > 0 ? g->in->n_threads : 1;
    if (nt > 256) nt = 256;
    if (n < 1024 || nt == 1) { range_t r = {0, n, g}; fn(&r); return; }
    pthread_t th[256];
    range_t rg[256];
    for (int i = 0; i < nt; ++i) {
        rg[i].lo = n * i / nt; rg[i].hi = n * (i + 1) / nt; rg[i].g = g;
        pthread_create(&th[i], NULL, fn, &rg[i]);
    }
    for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------- driver */
void or_free(or_output_t* o) {
    free(o->sorted_id); free(o->row_off); free(o->bin_base); free(o->bin_off);
    free(o->up); free(o->dn); free(o->up_c); free(o->dn_c); free(o->nb_flag); free(o->n_pairs);
    free(o->start_id);
    free(o->tl_nhits); free(o->tl_hits); free(o->tl_state); free(o->tl_cov); free(o->tl_chi2);
    free(o->tl_ndf); free(o->tl_row_ref); free(o->tl_valid); free(o->tl_fail); free(o->tl_flag);
    free(o->hit_key); free(o->trk_tl); free(o->trk_off); free(o->trk_hits);
    memset(o, 0, sizeof *o);
}

/* Row tables of the grid (x, fp32 y origin, bins per row) in caller storage; 1 = invalid input. */
typedef struct { double x[256]; float ymin[256]; int32_t ny[256]; } rowtab_t;
static int setup_ctx(ctx_t* g, const or_input_t* in, const or_params_t* P, or_output_t* o, rowtab_t* t) {
    memset(o, 0, sizeof *o);
    if (in->n_rows < 3 || in->n_rows > 255 || in->n_sectors < 1 || in->n_sectors > 256 || in->n < 0) return 1;
    if (!(P->bin_y > 0) || !(P->bin_z > 0) || !(in->z_max > in->z_min)) return 1;
    memset(g, 0, sizeof *g);
    g->in = in; g->prm = P; g->out = o;
    g->R = in->n_rows; g->S = in->n_sectors;
    g->kq = -0.00299792458 * in->bz;
    g->x = t->x; g->ymin = t->ymin; g->ny = t->ny;
    for (int r = 0; r < g->R; ++r) {
        t->x[r] = (double)in->row_x[r];
        float hw = in->row_x[r] * in->tan_half;
        t->ymin[r] = -hw;
        double v = ceil((2.0 * (double)hw) / (double)P->bin_y);
        t->ny[r] = v < 1 ? 1 : (v > 65535 ? 65535 : (int32_t)v);
    }
    {
        double v = ceil(((double)in->z_max - (double)in->z_min) / (double)P->bin_z);
        g->nz = v < 1 ? 1 : (v > 1048576 ? 1048576 : (int32_t)v);
    }
    g->inv_by = 1.0f / P->bin_y;
    g->inv_bz = 1.0f / P->bin_z;
    build_grid(g);
    return 0;
}

/* The following search of one row on its own (for tests): the cluster id chosen in row-sector
 * (s, r) for the predicted state p with covariance c, or -1; *flag gets the near-tie bits. */
int64_t or_follow_search(const or_input_t* in, const or_params_t* P, int s, int r, const double p[5],
                         const double c[15], int* flag) {
    ctx_t g;
    rowtab_t t;
    or_output_t o;
    *flag = 0;
    if (setup_ctx(&g, in, P, &o, &t) || s < 0 || s >= g.S || r < 0 || r >= g.R) { or_free(&o); return -2; }
    int64_t id = follow_search(&g, s, r, p, c, flag);
    or_free(&o);
    return id;
}

/* stage mask: 1 grid, 2 neighbours, 4 cleaning+starts, 8 tracklets, 16 selection */
int or_track(const or_input_t* in, const or_params_t* P, int stages, or_output_t* o) {
    if (P->l_min_chain < 2) { memset(o, 0, sizeof *o); return -1; } /* a start needs a first link */
    ctx_t g;
    rowtab_t tabs;
    if (setup_ctx(&g, in, P, o, &tabs)) return -1;
    int64_t n = in->n;
    size_t n1 = (size_t)(n > 0 ? n : 1);
    if (!(stages & 2)) return 0;
    o->up = (int32_t*)malloc(4 * n1); o->dn = (int32_t*)malloc(4 * n1);
    o->up_c = (int32_t*)malloc(4 * n1); o->dn_c = (int32_t*)malloc(4 * n1);
    o->nb_flag = (uint8_t*)calloc(n1, 1);
    o->n_pairs = (int32_t*)calloc(n1, 4);
    for (int64_t i = 0; i < n; ++i) { o->up[i] = o->dn[i] = o->up_c[i] = o->dn_c[i] = -1; }
    parallel(&g, o->n_valid, neighbours_range);
    for (int64_t i = 0; i < n; ++i) o->n_links_raw += (o->up[i] >= 0);
    if (!(stages & 4)) return 0;
    /* cleaning: keep reciprocal links only */
    for (int64_t h = 0; h < n; ++h) {
        int32_t u = o->up[h], d = o->dn[h];
        o->up_c[h] = (u >= 0 && o->dn[u] == (int32_t)h) ? u : -1;
        o->dn_c[h] = (d >= 0 && o->up[d] == (int32_t)h) ? d : -1;
        o->n_links_clean += (o->up_c[h] >= 0);
    }
    /* start hits: chain heads with at least l_min_chain hits, ascending id */
    o->start_id = (uint32_t*)malloc(4 * n1);
    for (int64_t h = 0; h < n; ++h) {
        if (in->row[h] >= g.R || in->sector[h] >= g.S) continue;
        if (o->dn_c[h] >= 0) continue;
        int len = 1;
        int64_t c = h;
        while (o->up_c[c] >= 0 && len < P->l_min_chain) { c = o->up_c[c]; ++len; }
        if (len >= P->l_min_chain) o->start_id[o->n_starts++] = (uint32_t)h;
    }
    if (!(stages & 8)) return 0;
    int64_t T = o->n_starts;
    size_t t1 = (size_t)(T > 0 ? T : 1);
    o->tl_nhits = (int32_t*)calloc(t1, 4);
    o->tl_hits = (int32_t*)malloc(4 * t1 * (size_t)g.R);
    o->tl_state = (double*)calloc(t1 * 5, 8);
    o->tl_cov = (double*)calloc(t1 * 15, 8);
    o->tl_chi2 = (double*)calloc(t1, 8);
    o->tl_ndf = (int32_t*)calloc(t1, 4);
    o->tl_row_ref = (int32_t*)calloc(t1, 4);
    o->tl_valid = (uint8_t*)calloc(t1, 1);
    o->tl_fail = (uint8_t*)calloc(t1, 1);
    o->tl_flag = (uint8_t*)calloc(t1, 1);
    parallel(&g, T, tracklets_range);
    for (int64_t t = 0; t < T; ++t) o->n_fit_fail += o->tl_fail[t];
    if (!(stages & 16)) return 0;
    /* selection: hitKey[c] = max key of the valid tracklets containing c */
    o->hit_key = (uint64_t*)calloc(n1, 8);
    for (int64_t t = 0; t < T; ++t) {
        if (!o->tl_valid[t]) continue;
        uint64_t key = ((uint64_t)(uint32_t)o->tl_nhits[t] << 32) | (uint64_t)(0xFFFFFFFFu - o->start_id[t]);
        const int32_t* hs = o->tl_hits + (size_t)t * g.R;
        for (int r = 0; r < g.R; ++r)
            if (hs[r] >= 0 && o->hit_key[hs[r]] < key) o->hit_key[hs[r]] = key;
    }
    o->trk_tl = (int32_t*)malloc(4 * t1);
    o->trk_off = (int32_t*)malloc(4 * (t1 + 1));
    o->trk_hits = (int32_t*)malloc(4 * n1);
    o->trk_off[0] = 0;
    for (int64_t t = 0; t < T; ++t) {
        if (!o->tl_valid[t]) continue;
        uint64_t key = ((uint64_t)(uint32_t)o->tl_nhits[t] << 32) | (uint64_t)(0xFFFFFFFFu - o->start_id[t]);
        const int32_t* hs = o->tl_hits + (size_t)t * g.R;
        int owned = 0;
        for (int r = 0; r < g.R; ++r) owned += (hs[r] >= 0 && o->hit_key[hs[r]] == key);
        if (owned < P->n_min_track) continue;
        int64_t k = o->n_tracks++;
        o->trk_tl[k] = (int32_t)t;
        int32_t off = o->trk_off[k];
        for (int r = 0; r < g.R; ++r)
            if (hs[r] >= 0 && o->hit_key[hs[r]] == key) o->trk_hits[off++] = hs[r];
        o->trk_off[k + 1] = off;
    }
    o->n_track_hits = o->trk_off[o->n_tracks];
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Cluster attachment, adjacency and the removal strategies (Sec. 4, cluster removal).
 *
 * A cluster is attached to the track it belongs to.  It is adjacent to a track when it lies on
 * a pad row the track spans (innermost to outermost hit row) within a tube of radius `tube`
 * around it: (y - y_t)^2 + (z - z_t)^2 <= tube^2 on the row plane, with (y_t, z_t) the track's
 * helix propagated from its reference state to that row.  Ambiguities go to the higher-momentum
 * track (smaller |q/pT|, then the smaller track index).  The cluster is protected when that track
 * has pT > pt_min and a local inclination |phi| < phi_max on the cluster's row; strategy A removes
 * the unprotected clusters that are attached or adjacent to a track, strategy B every unprotected
 * cluster.  Tracks are not merged into legs here, so every track counts as a primary leg.
 * Brute force: every cluster of the track's sector and row is tested.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    const float *y, *z;
    const uint8_t *row, *sector;
    int n_rows, n_sectors;
    const float* row_x;
    double kq, s_max;
    int32_t n_tracks;
    const int32_t *off, *nh, *hits, *trk_sector;
    const float *x_ref, *state;   /* state: 5 per track (y, z, sin phi, dz/ds, q/pT) */
    double tube, pt_min, sin_phi_max;
} or_flags_in_t;

enum { OF_ATTACHED = 1, OF_ADJACENT = 2, OF_PROTECTED = 4, OF_REMOVE_A = 8, OF_REMOVE_B = 16 };

/* track k's helix at x: y, z and sin phi; 0 when the helix does not reach x */
static int or_helix_at(const or_flags_in_t* in, int32_t k, double x, double* yt, double* zt, double* st) {
    double p0[5], p1[5];
    for (int i = 0; i < 5; ++i) p0[i] = (double)in->state[5 * k + i];
    if (or_propagate(p0, (double)in->x_ref[k], x, in->kq, in->s_max, 0.0, p1, NULL, NULL)) return 0;
    *yt = p1[0];
    *zt = p1[1];
    *st = p1[2];
    return 1;
}

/* key of track k: larger for higher momentum, then for the smaller index */
static uint64_t or_track_key(const or_flags_in_t* in, int32_t k) {
    float a = fabsf(in->state[5 * k + 4]);
    uint32_t bits;
    memcpy(&bits, &a, 4);
    return ((uint64_t)(0xFFFFFFFFu - bits) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)k);
}

/* flags[n]; tie[n] (may be NULL): 1 where a decision lies within 1e-9 (relative) of its cut */
int or_cluster_flags(const or_flags_in_t* in, uint8_t* flags, uint8_t* tie) {
    const int64_t n = in->n;
    const int R = in->n_rows, S = in->n_sectors;
    uint64_t* best = (uint64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    double* best_s = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    uint8_t* att = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    uint8_t* adj = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t* first = (int64_t*)malloc(sizeof(int64_t) * ((size_t)S * R + 1));
    int64_t* list = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!best || !best_s || !att || !adj || !first || !list) return 1;
    if (tie) memset(tie, 0, (size_t)n);
    /* clusters listed per (sector, row) */
    for (int64_t i = 0; i <= (int64_t)S * R; ++i) first[i] = 0;
    for (int64_t c = 0; c < n; ++c)
        if (in->row[c] < R && in->sector[c] < S) ++first[in->sector[c] * R + in->row[c] + 1];
    for (int64_t i = 0; i < (int64_t)S * R; ++i) first[i + 1] += first[i];
    {
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)S * R));
        for (int64_t i = 0; i < (int64_t)S * R; ++i) fill[i] = first[i];
        for (int64_t c = 0; c < n; ++c)
            if (in->row[c] < R && in->sector[c] < S) list[fill[in->sector[c] * R + in->row[c]]++] = c;
        free(fill);
    }
    const double t2 = in->tube * in->tube;
    for (int32_t k = 0; k < in->n_tracks; ++k) {
        const uint64_t key = or_track_key(in, k);
        const int s = in->trk_sector[k];
        const int32_t* h = in->hits + in->off[k];
        const int nh = in->nh[k];
        if (nh <= 0) continue;
        const int r0 = in->row[h[0]], r1 = in->row[h[nh - 1]];
        /* adjacency: every cluster of the spanned rows within the tube */
        for (int r = r0; r <= r1; ++r) {
            double yt, zt, st;
            if (!or_helix_at(in, k, (double)in->row_x[r], &yt, &zt, &st)) continue;
            for (int64_t j = first[s * R + r]; j < first[s * R + r + 1]; ++j) {
                const int64_t c = list[j];
                const double dy = (double)in->y[c] - yt, dz = (double)in->z[c] - zt;
                const double d2 = dy * dy + dz * dz;
                if (tie && fabs(d2 - t2) <= 1e-9 * t2) tie[c] = 1;
                if (!(d2 <= t2)) continue;
                adj[c] = 1;
                if (key > best[c]) {
                    best[c] = key;
                    best_s[c] = st;
                }
            }
        }
        /* attachment: the track's own clusters, inside the tube or not */
        for (int i = 0; i < nh; ++i) {
            const int64_t c = h[i];
            att[c] = 1;
            double yt, zt, st;
            if (!or_helix_at(in, k, (double)in->row_x[in->row[c]], &yt, &zt, &st)) st = 2.0; /* never protected */
            if (key > best[c]) {
                best[c] = key;
                best_s[c] = st;
            }
        }
    }
    const float qpt_max = (float)(1.0 / in->pt_min);
    for (int64_t c = 0; c < n; ++c) {
        uint8_t f = (att[c] ? OF_ATTACHED : 0) | (adj[c] ? OF_ADJACENT : 0);
        int prot = 0;
        if (best[c]) {
            /* the assigned track: its |q/pT| and its sin phi on this row */
            const int32_t k = (int32_t)(0xFFFFFFFFu - (uint32_t)(best[c] & 0xFFFFFFFFu));
            const float a = fabsf(in->state[5 * k + 4]);
            prot = a < qpt_max && fabs(best_s[c]) < in->sin_phi_max;
            if (tie && fabs(fabs(best_s[c]) - in->sin_phi_max) <= 1e-9) tie[c] = 1;
            f |= prot ? OF_PROTECTED : OF_REMOVE_A;
        }
        if (!prot) f |= OF_REMOVE_B;
        flags[c] = f;
    }
    free(best); free(best_s); free(att); free(adj); free(first); free(list);
    return 0;
}
