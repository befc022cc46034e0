/*
 * Seeded synthetic TPC cluster generator (input side only).
 *
 * Stands in for the ALICE simulation the paper uses for its TPC studies
 * (Sec. 4, Figs. 4-7): charged helices in a uniform solenoidal field Bz,
 * intersected with the 152 pad-row planes of 36 azimuthal sectors
 * (18 per z side), one cluster per plane crossing, Gaussian smearing,
 * per-crossing efficiency and uniform noise.  Continuous-readout time
 * frames (Sec. 1: 50 kHz Pb-Pb, 0.2-1 MHz pp) shift each collision's
 * clusters in z by v_drift * t0.
 *
 * This file holds none of the tracking method's arithmetic: the crossings
 * are found analytically in the global frame (circle/plane intersection),
 * not by the track-model propagation the tracker uses.
 *
 * Random numbers: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), counter = (item, stream tag,
 * draw index), key = the 64-bit seed.  Every collision, particle and noise
 * sector owns its own counter space, so the output does not depend on the
 * number of worker threads.
 *
 * Units: cm, T, GeV/c, microseconds.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define N_WEDGES 18
#define MAX_ROWS 255

/* ------------------------------------------------------------------ Philox */
typedef struct { uint32_t c[4]; } ph4;

static ph4 philox4x32_10(ph4 x, uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x.c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x.c[2];
        ph4 y;
        y.c[0] = (uint32_t)(p1 >> 32) ^ x.c[1] ^ k0;
        y.c[1] = (uint32_t)p1;
        y.c[2] = (uint32_t)(p0 >> 32) ^ x.c[3] ^ k1;
        y.c[3] = (uint32_t)p0;
        x = y;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x;
}

typedef struct {
    uint32_t k0, k1, item, tag, n;
    uint32_t buf[4];
    int pos;
} rng_t;

static void rng_init(rng_t* g, uint64_t seed, uint32_t item, uint32_t tag) {
    g->k0 = (uint32_t)seed; g->k1 = (uint32_t)(seed >> 32);
    g->item = item; g->tag = tag; g->n = 0; g->pos = 4;
}
static uint32_t rng_u32(rng_t* g) {
    if (g->pos == 4) {
        ph4 x = {{g->item, g->tag, g->n++, 0x7C5A11u}};
        ph4 y = philox4x32_10(x, g->k0, g->k1);
        memcpy(g->buf, y.c, sizeof g->buf);
        g->pos = 0;
    }
    return g->buf[g->pos++];
}
/* uniform in the open interval (0,1), 53 random bits */
static double rng_uni(rng_t* g) {
    uint32_t a = rng_u32(g) >> 5, b = rng_u32(g) >> 6;
    return ((double)a * 67108864.0 + (double)b + 0.5) * (1.0 / 9007199254740992.0);
}
static double rng_normal(rng_t* g) { /* Box-Muller, one value per call */
    double u1 = rng_uni(g), u2 = rng_uni(g);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}
static double rng_exp(rng_t* g, double mean) { return -mean * log(rng_uni(g)); }
static int rng_poisson(rng_t* g, double mean) { /* Knuth's product method */
    double L = exp(-mean), p = 1.0;
    int k = 0;
    do { ++k; p *= rng_uni(g); } while (p > L);
    return k - 1;
}

/* ------------------------------------------------------------------ config */
typedef struct {
    uint64_t seed;
    int32_t n_collisions;
    int32_t mult_mode;        /* 0 fixed, 1 exponential(mean) capped, 2 Poisson(mean) */
    int32_t mult_fixed, mult_cap;
    double mult_mean;
    int32_t pt_mode;          /* 0 log-uniform [pt_lo,pt_hi], 1 exponential(pt_mean), redrawn below pt_floor */
    double pt_lo, pt_hi, pt_mean, pt_floor;
    double eta_max;
    int32_t eta_one_side;     /* 1: eta in [0, eta_max] (a one-sector workload covers z >= 0 only) */
    int32_t phi_mode;         /* 0 uniform inside sector 0 (inset from the edges), 1 uniform in 2 pi */
    double phi_inset_deg;
    double sec_frac, sec_rmax; /* secondaries per primary, vertex disk radius at z = 0 */
    int32_t only_sector;      /* -1: all 36 sectors; else clusters of that sector only */
    double sigma_y, sigma_z, eff, noise_frac;
    double bz, max_turns, z_len;
    double t_frame_us, v_drift; /* t0 ~ U[0, t_frame_us) per collision when t_frame_us > 0 */
    int32_t order;            /* 0 grouped by (sector,row), generation order inside; 1 seeded permutation */
    int32_t want_exact;       /* also fill the exact (unsmeared) truth arrays */
    int32_t n_threads;
    int32_t n_rows;
    const float* row_x;       /* [n_rows] pad-row radii (float, as the tracker sees them) */
    float tan_half;           /* tan(sector half angle) */
} synth_cfg_t;

typedef struct {
    int64_t n;
    float *y, *z;
    uint8_t *row, *sector;
    int32_t *particle, *leg, *crossing, *collision;
    double *y_true, *z_true, *phi_loc, *dzds, *qpt; /* only when want_exact */
    int64_t n_signal, n_noise, n_particles, n_legs;
} synth_out_t;

/* one accepted plane crossing */
typedef struct {
    double s, y, z, philoc, dzds, qpt;
    int32_t wedge, row, side; /* side 0: z >= 0 (sectors 0..17), 1: z < 0 */
} xing_t;

typedef struct {
    float y, z;
    uint8_t row, sector;
    int32_t particle, leg, crossing, collision;
    double yt, zt, ph, tz, qp;
} clu_t;

typedef struct {
    clu_t* v;
    int64_t n, cap;
    int64_t n_particles, n_legs;
} cbuf_t;

static void cbuf_push(cbuf_t* b, const clu_t* c) {
    if (b->n == b->cap) {
        b->cap = b->cap ? b->cap * 2 : 4096;
        b->v = (clu_t*)realloc(b->v, (size_t)b->cap * sizeof(clu_t));
    }
    b->v[b->n++] = *c;
}

static int cmp_xing(const void* a, const void* b) {
    double sa = ((const xing_t*)a)->s, sb = ((const xing_t*)b)->s;
    return sa < sb ? -1 : sa > sb ? 1 : 0;
}

static double wrap_2pi(double a) {
    a = fmod(a, 2.0 * M_PI);
    return a < 0 ? a + 2.0 * M_PI : a;
}

/* All crossings of one helix with the pad-row planes, sorted by path length.
 * Helix: P(s) = V + (sin(phi0 + k s) - sin phi0, -(cos(phi0 + k s) - cos phi0)) / k,
 * z(s) = tl * s, k = -0.00299792458 * bz * q / pT  (cm^-1), s = transverse arc length. */
static int helix_crossings(const synth_cfg_t* cfg, double vx, double vy, double phi0, double tl,
                           double qpt, xing_t** out, int* cap) {
    const double kc = 0.00299792458;
    double k = -kc * cfg->bz * qpt;
    if (fabs(k) < 1e-12) k = (k < 0 ? -1e-12 : 1e-12);
    const double r_out = (double)cfg->row_x[cfg->n_rows - 1] / cos(atan((double)cfg->tan_half)) + 0.5;
    const double r_in = (double)cfg->row_x[0] - 0.5;
    /* path limits: max turns, |z| beyond the drift length, leaving the outer radius */
    double s_end = cfg->max_turns * 2.0 * M_PI / fabs(k);
    if (fabs(tl) > 1e-15) { double sz = cfg->z_len / fabs(tl); if (sz < s_end) s_end = sz; }
    const double ds = 5.0;
    int cand[N_WEDGES];
    memset(cand, 0, sizeof cand);
    const double wedge = 2.0 * M_PI / N_WEDGES, margin = 4.0 * M_PI / 180.0;
    double s_prev = 0.0;
    int out_seen = 0;
    for (double s = 0.0;; s += ds) {
        if (s > s_end) s = s_end;
        double ph = phi0 + k * s;
        double X = vx + (sin(ph) - sin(phi0)) / k, Y = vy - (cos(ph) - cos(phi0)) / k;
        double r = sqrt(X * X + Y * Y);
        if (r > r_out && !out_seen) {
            /* first exit through the outer radius: refine by bisection, stop there */
            double a = s_prev, b = s;
            for (int it = 0; it < 80; ++it) {
                double m = 0.5 * (a + b), pm = phi0 + k * m;
                double Xm = vx + (sin(pm) - sin(phi0)) / k, Ym = vy - (cos(pm) - cos(phi0)) / k;
                if (Xm * Xm + Ym * Ym > r_out * r_out) b = m; else a = m;
            }
            s_end = b;
            out_seen = 1;
        }
        if (r >= r_in - ds && r <= r_out + ds) {
            double th = wrap_2pi(atan2(Y, X));
            for (int w = 0; w < N_WEDGES; ++w) {
                double c = (w + 0.5) * wedge;
                double d = fabs(remainder(th - c, 2.0 * M_PI));
                if (d <= 0.5 * wedge + margin) cand[w] = 1;
            }
        }
        s_prev = s;
        if (s >= s_end) break;
    }
    int n = 0;
    for (int w = 0; w < N_WEDGES; ++w) {
        if (!cand[w]) continue;
        double al = (w + 0.5) * wedge, ca = cos(al), sa = sin(al);
        double psi0 = phi0 - al;
        double A = vx * ca + vy * sa - sin(psi0) / k;
        double B = -vx * sa + vy * ca + cos(psi0) / k;
        double psi_a = psi0, psi_b = psi0 + k * s_end;
        double plo = psi_a < psi_b ? psi_a : psi_b, phi_ = psi_a < psi_b ? psi_b : psi_a;
        for (int i = 0; i < cfg->n_rows; ++i) {
            double xi = (double)cfg->row_x[i];
            double S = k * (xi - A);
            if (S < -1.0 || S > 1.0) continue;
            double as = asin(S);
            double base[2] = {as, M_PI - as};
            for (int b = 0; b < 2; ++b) {
                /* all psi = base + 2 pi n inside [plo, phi_] */
                double n0 = ceil((plo - base[b]) / (2.0 * M_PI));
                for (double nn = n0;; nn += 1.0) {
                    double psi = base[b] + 2.0 * M_PI * nn;
                    if (psi > phi_) break;
                    double s = (psi - psi0) / k;
                    if (s <= 0.0 || s > s_end) continue;
                    double yl = B - cos(psi) / k;
                    if (fabs(yl) > xi * (double)cfg->tan_half) continue;
                    double zz = tl * s;
                    if (fabs(zz) > cfg->z_len) continue;
                    if (n == *cap) {
                        *cap = *cap ? *cap * 2 : 256;
                        *out = (xing_t*)realloc(*out, (size_t)*cap * sizeof(xing_t));
                    }
                    xing_t* x = &(*out)[n++];
                    x->s = s;
                    x->y = yl;
                    x->side = zz >= 0.0 ? 0 : 1;
                    x->z = x->side ? -zz : zz;
                    /* direction in the sector frame; z mirrored on the C side */
                    x->philoc = psi;
                    x->dzds = x->side ? -tl : tl;
                    x->qpt = qpt;
                    x->wedge = w;
                    x->row = i;
                }
            }
        }
    }
    qsort(*out, (size_t)n, sizeof(xing_t), cmp_xing);
    return n;
}

/* sector index of a crossing: 0..17 A side (z >= 0), 18..35 C side */
static int xing_sector(const xing_t* x) { return x->wedge + (x->side ? N_WEDGES : 0); }

/* The C side keeps the same transverse (x, y) rotation as the A side and
 * mirrors z only, so a helix keeps its transverse curvature there and its
 * dz/ds changes sign. */

typedef struct {
    const synth_cfg_t* cfg;
    int32_t c0, c1;
    cbuf_t buf;
} work_t;

static void gen_collision(const synth_cfg_t* cfg, int32_t coll, cbuf_t* buf) {
    rng_t gc;
    rng_init(&gc, cfg->seed, (uint32_t)coll, 0xC011u);
    int n_prim;
    if (cfg->mult_mode == 0) n_prim = cfg->mult_fixed;
    else if (cfg->mult_mode == 1) {
        double m = floor(rng_exp(&gc, cfg->mult_mean) + 0.5);
        n_prim = m > cfg->mult_cap ? cfg->mult_cap : (int)m;
    } else n_prim = rng_poisson(&gc, cfg->mult_mean);
    double t0 = cfg->t_frame_us > 0 ? rng_uni(&gc) * cfg->t_frame_us : 0.0;
    double zshift = cfg->v_drift * t0;
    int n_sec = (int)floor(cfg->sec_frac * n_prim + 0.5);
    int n_tot = n_prim + n_sec;
    xing_t* xs = NULL;
    int xcap = 0;
    for (int p = 0; p < n_tot; ++p) {
        rng_t g;
        rng_init(&g, cfg->seed, (uint32_t)coll, 0x10000u + (uint32_t)p);
        double pt;
        if (cfg->pt_mode == 0) pt = cfg->pt_lo * exp(rng_uni(&g) * log(cfg->pt_hi / cfg->pt_lo));
        else { do { pt = rng_exp(&g, cfg->pt_mean); } while (pt < cfg->pt_floor); }
        double eta = cfg->eta_one_side ? rng_uni(&g) * cfg->eta_max : (2.0 * rng_uni(&g) - 1.0) * cfg->eta_max;
        double tl = sinh(eta);
        double phi0;
        if (cfg->phi_mode == 0) {
            double half = (10.0 - cfg->phi_inset_deg) * M_PI / 180.0;
            phi0 = (2.0 * rng_uni(&g) - 1.0) * half + 10.0 * M_PI / 180.0; /* sector 0 is centred at 10 deg */
        } else phi0 = 2.0 * M_PI * rng_uni(&g);
        double q = rng_uni(&g) < 0.5 ? -1.0 : 1.0;
        double vx = 0.0, vy = 0.0;
        if (p >= n_prim) {
            double r = cfg->sec_rmax * sqrt(rng_uni(&g)), a = 2.0 * M_PI * rng_uni(&g);
            vx = r * cos(a); vy = r * sin(a);
        }
        int nx = helix_crossings(cfg, vx, vy, phi0, tl, q / pt, &xs, &xcap);
        int64_t pid = buf->n_particles++;
        int leg = -1, dir = 0;
        for (int i = 0; i < nx; ++i) {
            const xing_t* x = &xs[i];
            int sec = xing_sector(x);
            int newleg = (i == 0);
            if (!newleg) {
                const xing_t* pv = &xs[i - 1];
                int d = x->row - pv->row;
                int sd = d > 0 ? 1 : (d < 0 ? -1 : 0);
                if (xing_sector(pv) != sec || sd == 0 || (dir != 0 && sd != dir)) newleg = 1;
                else dir = sd;
            }
            if (newleg) { leg = (int)buf->n_legs++; dir = 0; }
            int keep = rng_uni(&g) < cfg->eff;
            double ny = rng_normal(&g), nz = rng_normal(&g);
            if (!keep) continue;
            if (cfg->only_sector >= 0 && sec != cfg->only_sector) continue;
            clu_t c;
            c.y = (float)(x->y + cfg->sigma_y * ny);
            c.z = (float)(x->z + cfg->sigma_z * nz + zshift);
            c.row = (uint8_t)x->row;
            c.sector = (uint8_t)sec;
            c.particle = (int32_t)pid;
            c.leg = leg;
            c.crossing = i;
            c.collision = coll;
            c.yt = x->y; c.zt = x->z + zshift; c.ph = x->philoc; c.tz = x->dzds; c.qp = x->qpt;
            cbuf_push(buf, &c);
        }
    }
    free(xs);
}

static void* worker(void* arg) {
    work_t* w = (work_t*)arg;
    for (int32_t c = w->c0; c < w->c1; ++c) gen_collision(w->cfg, c, &w->buf);
    return NULL;
}

void synth_free(synth_out_t* o) {
    free(o->y); free(o->z); free(o->row); free(o->sector);
    free(o->particle); free(o->leg); free(o->crossing); free(o->collision);
    free(o->y_true); free(o->z_true); free(o->phi_loc); free(o->dzds); free(o->qpt);
    memset(o, 0, sizeof *o);
}

int synth_generate(const synth_cfg_t* cfg, synth_out_t* out) {
    memset(out, 0, sizeof *out);
    if (cfg->n_rows <= 0 || cfg->n_rows > MAX_ROWS || cfg->n_collisions < 0) return -1;
    int nt = cfg->n_threads > 0 ? cfg->n_threads : 1;
    if (nt > cfg->n_collisions) nt = cfg->n_collisions > 0 ? cfg->n_collisions : 1;
    work_t* ws = (work_t*)calloc((size_t)nt, sizeof(work_t));
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    /* contiguous collision ranges per thread keep the concatenation order fixed */
    for (int t = 0; t < nt; ++t) {
        ws[t].cfg = cfg;
        ws[t].c0 = (int32_t)((int64_t)cfg->n_collisions * t / nt);
        ws[t].c1 = (int32_t)((int64_t)cfg->n_collisions * (t + 1) / nt);
        pthread_create(&th[t], NULL, worker, &ws[t]);
    }
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    /* concatenate; particle and leg ids become global by offsetting */
    cbuf_t all = {0};
    for (int t = 0; t < nt; ++t) {
        for (int64_t i = 0; i < ws[t].buf.n; ++i) {
            clu_t c = ws[t].buf.v[i];
            c.particle += (int32_t)all.n_particles;
            c.leg += (int32_t)all.n_legs;
            cbuf_push(&all, &c);
        }
        all.n_particles += ws[t].buf.n_particles;
        all.n_legs += ws[t].buf.n_legs;
        free(ws[t].buf.v);
    }
    free(ws); free(th);
    int64_t n_signal = all.n;
    /* noise: per sector, round(noise_frac * signal clusters of that sector) */
    int64_t per_sec[36] = {0};
    for (int64_t i = 0; i < n_signal; ++i) per_sec[all.v[i].sector]++;
    double zmax_tf = cfg->z_len + (cfg->t_frame_us > 0 ? cfg->v_drift * cfg->t_frame_us : 0.0);
    for (int s = 0; s < 36; ++s) {
        if (cfg->only_sector >= 0 && s != cfg->only_sector) continue;
        int64_t nn = (int64_t)floor(cfg->noise_frac * (double)per_sec[s] + 0.5);
        rng_t g;
        rng_init(&g, cfg->seed, (uint32_t)s, 0x0015Eu);
        for (int64_t j = 0; j < nn; ++j) {
            clu_t c;
            int r = (int)(rng_uni(&g) * cfg->n_rows);
            if (r >= cfg->n_rows) r = cfg->n_rows - 1;
            double hw = (double)cfg->row_x[r] * (double)cfg->tan_half;
            double yy = (2.0 * rng_uni(&g) - 1.0) * hw, zz = rng_uni(&g) * zmax_tf;
            c.y = (float)yy; c.z = (float)zz; c.row = (uint8_t)r; c.sector = (uint8_t)s;
            c.particle = -1; c.leg = -1; c.crossing = -1; c.collision = -1;
            c.yt = yy; c.zt = zz; c.ph = 0; c.tz = 0; c.qp = 0;
            cbuf_push(&all, &c);
        }
    }
    int64_t N = all.n;
    /* output order */
    int64_t* perm = (int64_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int64_t));
    if (cfg->order == 1) {
        for (int64_t i = 0; i < N; ++i) perm[i] = i;
        rng_t g;
        rng_init(&g, cfg->seed, 0xFFFFFFFFu, 0x5EEDu);
        for (int64_t i = N - 1; i > 0; --i) { /* Fisher-Yates */
            int64_t j = (int64_t)(rng_uni(&g) * (double)(i + 1));
            if (j > i) j = i;
            int64_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
    } else {
        int nkeys = 36 * cfg->n_rows;
        int64_t* cnt = (int64_t*)calloc((size_t)nkeys + 1, sizeof(int64_t));
        for (int64_t i = 0; i < N; ++i) cnt[all.v[i].sector * cfg->n_rows + all.v[i].row + 1]++;
        for (int k = 0; k < nkeys; ++k) cnt[k + 1] += cnt[k];
        for (int64_t i = 0; i < N; ++i) perm[cnt[all.v[i].sector * cfg->n_rows + all.v[i].row]++] = i;
        free(cnt);
    }
    size_t n1 = (size_t)(N > 0 ? N : 1);
    out->n = N;
    out->y = (float*)malloc(n1 * 4); out->z = (float*)malloc(n1 * 4);
    out->row = (uint8_t*)malloc(n1); out->sector = (uint8_t*)malloc(n1);
    out->particle = (int32_t*)malloc(n1 * 4); out->leg = (int32_t*)malloc(n1 * 4);
    out->crossing = (int32_t*)malloc(n1 * 4); out->collision = (int32_t*)malloc(n1 * 4);
    if (cfg->want_exact) {
        out->y_true = (double*)malloc(n1 * 8); out->z_true = (double*)malloc(n1 * 8);
        out->phi_loc = (double*)malloc(n1 * 8); out->dzds = (double*)malloc(n1 * 8);
        out->qpt = (double*)malloc(n1 * 8);
    }
    for (int64_t i = 0; i < N; ++i) {
        const clu_t* c = &all.v[perm[i]];
        out->y[i] = c->y; out->z[i] = c->z; out->row[i] = c->row; out->sector[i] = c->sector;
        out->particle[i] = c->particle; out->leg[i] = c->leg;
        out->crossing[i] = c->crossing; out->collision[i] = c->collision;
        if (cfg->want_exact) {
            out->y_true[i] = c->yt; out->z_true[i] = c->zt; out->phi_loc[i] = c->ph;
            out->dzds[i] = c->tz; out->qpt[i] = c->qp;
        }
    }
    out->n_signal = n_signal;
    out->n_noise = N - n_signal;
    out->n_particles = all.n_particles;
    out->n_legs = all.n_legs;
    free(perm);
    free(all.v);
    return 0;
}
