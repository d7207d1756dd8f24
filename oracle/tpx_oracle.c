/*
 * FP64 CPU oracle for the probed adjoint-state FWI gradient
 * (Louboutin & Herrmann, "Ultra-low memory seismic inversion with randomized
 * trace estimation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header, table
 * or helper with the HIP library; the two are written independently from the
 * paper's equations.
 *
 * Everything is double precision and written as plain loops.  OpenMP only
 * splits the outermost spatial loop of independent per-point work; no sum is
 * split across threads, so results do not depend on the thread count.
 *
 * Notation (paper, Methodology):
 *   m      squared slowness (ms^2/m^2), the unknown of the misfit, Eq. (2);
 *   u^k    forward wavefield at t_k = k dt;  lambda^k the adjoint wavefield
 *          (the paper's v);
 *   Z      the n_t x r probing matrix of Eq. (1) / Eq. (4);
 *   ubar_j = sum_s Z[s,j] u^s,  vbar_j = sum_s Z[s,j] w^s  (Algorithm 1,
 *          accumulations in the forward and in the back-propagation loop).
 *
 * Readings where the paper is silent (its discretisation, boundary, damping,
 * time ranges of Algorithm 1, which pass carries the second time derivative,
 * probe generator) are listed in the design notes; each function below names
 * the one it uses.
 *
 * Parity status: every exported function is pinned by the CPU test suite
 * (stencil exactness, manufactured-solution convergence, adjoint dot test,
 * Taylor test, brute-force finite differences, identity-probe recovery,
 * Philox known-answer vectors, probe moments, Monte Carlo unbiasedness).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Problem description                                                        */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t ndim;      /* 2 or 3 */
    int64_t n[3];      /* physical nodes along x, y, z (2D: x and z, n[1] = 1) */
    double  h;         /* grid spacing, m */
    int32_t nbl;       /* absorbing-layer width in nodes, on every face */
    int32_t order;     /* spatial order of the Laplacian: 4 or 8 */
    double  dt;        /* time step, ms */
    int32_t nt;        /* number of time samples t_k = k dt, k = 0..nt-1 */
    double  damp_vmax; /* velocity used by the damping profile, km/s */
    double  damp_R;    /* target reflection coefficient of the layer */
} orc_grid;

typedef struct {
    int32_t nshots;
    int32_t nrec;
    const double *src_pos; /* [S][3] (x, y, z) in m */
    const double *rec_pos; /* [S][nrec][3] */
    const double *wavelet; /* [S][nt] source time function q^k */
} orc_geom;

enum { ORC_OK = 0, ORC_E_INVAL = 1, ORC_E_GEOM = 2, ORC_E_NOMEM = 3 };
enum { ORC_PROBE_RADEMACHER = 0, ORC_PROBE_GAUSS_B64 = 1, ORC_PROBE_IDENTITY = 2,
       ORC_PROBE_EXPLICIT = 3 };

/* padded sizes: nbl nodes are added on both sides of every active axis */
static int64_t padded(const orc_grid *g, int a) {
    if (g->ndim == 2 && a == 1) return 1;
    return g->n[a] + 2 * (int64_t)g->nbl;
}
static int64_t npad_total(const orc_grid *g) { return padded(g, 0) * padded(g, 1) * padded(g, 2); }
static int64_t nphys_total(const orc_grid *g) { return g->n[0] * g->n[1] * g->n[2]; }
static int64_t pidx(const orc_grid *g, int64_t ix, int64_t iy, int64_t iz) {
    return (iz * padded(g, 1) + iy) * padded(g, 0) + ix;
}
static int offset_y(const orc_grid *g) { return g->ndim == 3 ? g->nbl : 0; }

static int valid_grid(const orc_grid *g) {
    if (!g || (g->ndim != 2 && g->ndim != 3)) return 0;
    if (g->order != 4 && g->order != 8) return 0;
    if (g->n[0] < 2 || g->n[2] < 2) return 0;
    if (g->ndim == 2 && g->n[1] != 1) return 0;
    if (g->ndim == 3 && g->n[1] < 2) return 0;
    if (!(g->h > 0) || !(g->dt > 0) || g->nt < 2 || g->nbl < 0) return 0;
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Model padding (edge replication) and the damping profile                  */
/* ------------------------------------------------------------------------- */

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* m_pad[I] = m[clamp(I - nbl, 0, n - 1)] along every active axis. */
void orc_pad_model(const orc_grid *g, const double *m, double *mpad) {
    const int64_t P0 = padded(g, 0), P1 = padded(g, 1), P2 = padded(g, 2);
    const int oy = offset_y(g);
    for (int64_t iz = 0; iz < P2; ++iz)
        for (int64_t iy = 0; iy < P1; ++iy)
            for (int64_t ix = 0; ix < P0; ++ix) {
                int64_t x = clampi(ix - g->nbl, 0, g->n[0] - 1);
                int64_t y = clampi(iy - oy, 0, g->n[1] - 1);
                int64_t z = clampi(iz - g->nbl, 0, g->n[2] - 1);
                mpad[pidx(g, ix, iy, iz)] = m[(z * g->n[1] + y) * g->n[0] + x];
            }
}

/* Quadratic absorbing profile: d = sum over active axes of dmax * delta^2,
 * delta = distance into the layer / nbl, dmax = 3 vmax / (2 nbl h) ln(1/R). */
void orc_damping(const orc_grid *g, double *damp) {
    const int64_t P0 = padded(g, 0), P1 = padded(g, 1), P2 = padded(g, 2);
    const double nb = (double)g->nbl;
    const double dmax = g->nbl > 0 ? 3.0 * g->damp_vmax / (2.0 * nb * g->h) * log(1.0 / g->damp_R) : 0.0;
    for (int64_t iz = 0; iz < P2; ++iz)
        for (int64_t iy = 0; iy < P1; ++iy)
            for (int64_t ix = 0; ix < P0; ++ix) {
                int64_t I[3] = {ix, iy, iz};
                double d = 0.0;
                for (int a = 0; a < 3; ++a) {
                    if (g->ndim == 2 && a == 1) continue;
                    if (g->nbl == 0) continue;
                    int64_t into = 0;
                    if (I[a] < g->nbl) into = g->nbl - I[a];
                    if (I[a] > g->nbl + g->n[a] - 1) into = I[a] - (g->nbl + g->n[a] - 1);
                    double delta = (double)into / nb;
                    d += dmax * delta * delta;
                }
                damp[pidx(g, ix, iy, iz)] = d;
            }
}

/* ------------------------------------------------------------------------- */
/* Spatial operator: the centred Laplacian of the acoustic wave equation      */
/* ------------------------------------------------------------------------- */

/* Central second-derivative weights from Taylor expansion: c[0] is the centre,
 * c[k] the weight of the two nodes at distance k. */
static int stencil_weights(int order, double c[5]) {
    memset(c, 0, 5 * sizeof(double));
    if (order == 4) {
        c[0] = -5.0 / 2.0; c[1] = 4.0 / 3.0; c[2] = -1.0 / 12.0;
        return 2;
    }
    c[0] = -205.0 / 72.0; c[1] = 8.0 / 5.0; c[2] = -1.0 / 5.0; c[3] = 8.0 / 315.0; c[4] = -1.0 / 560.0;
    return 4;
}

/* out = L u over the padded box; values outside the box are zero (Dirichlet).
 * Per node: for each active axis, sum_{k=-R..R} c_|k| u[I + k e_axis] / h^2. */
void orc_laplacian(const orc_grid *g, const double *u, double *out) {
    double c[5];
    const int R = stencil_weights(g->order, c);
    const int64_t P[3] = {padded(g, 0), padded(g, 1), padded(g, 2)};
    const int64_t stride[3] = {1, P[0], P[0] * P[1]};
    const double ih2 = 1.0 / (g->h * g->h);
#pragma omp parallel for schedule(static)
    for (int64_t iz = 0; iz < P[2]; ++iz)
        for (int64_t iy = 0; iy < P[1]; ++iy)
            for (int64_t ix = 0; ix < P[0]; ++ix) {
                const int64_t I[3] = {ix, iy, iz};
                const int64_t idx = pidx(g, ix, iy, iz);
                double acc = 0.0;
                for (int a = 0; a < 3; ++a) {
                    if (g->ndim == 2 && a == 1) continue;
                    double s = 0.0;
                    for (int k = -R; k <= R; ++k) {
                        const int64_t J = I[a] + k;
                        if (J < 0 || J >= P[a]) continue;
                        s += c[k < 0 ? -k : k] * u[idx + k * stride[a]];
                    }
                    acc += s * ih2;
                }
                out[idx] = acc;
            }
}

/* ------------------------------------------------------------------------- */
/* Point sources and receivers: bilinear / trilinear interpolation            */
/* ------------------------------------------------------------------------- */

typedef struct {
    int cnt;
    int64_t idx[8]; /* padded linear index */
    double w[8];
} orc_interp;

/* Weights of the 2^D nodes around a position.  Base node i0 = min(floor(x/h),
 * n-2), fraction f = x/h - i0; nodes outside [0,(n-1)h] are rejected. */
static int interp_weights(const orc_grid *g, const double pos[3], orc_interp *out) {
    int64_t i0[3] = {0, 0, 0};
    double f[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        if (g->ndim == 2 && a == 1) continue;
        double x = pos[a] / g->h;
        if (!(x >= 0.0) || x > (double)(g->n[a] - 1) * (1.0 + 1e-12)) return 0;
        int64_t b = (int64_t)floor(x);
        if (b > g->n[a] - 2) b = g->n[a] - 2;
        i0[a] = b;
        f[a] = x - (double)b;
    }
    out->cnt = 0;
    const int ny = g->ndim == 3 ? 2 : 1;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < ny; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? f[0] : 1.0 - f[0]) * (dz ? f[2] : 1.0 - f[2]);
                if (g->ndim == 3) w *= (dy ? f[1] : 1.0 - f[1]);
                int64_t ix = i0[0] + dx + g->nbl;
                int64_t iy = i0[1] + dy + offset_y(g);
                int64_t iz = i0[2] + dz + g->nbl;
                out->idx[out->cnt] = pidx(g, ix, iy, iz);
                out->w[out->cnt] = w;
                out->cnt++;
            }
    return 1;
}

static double sample(const orc_interp *p, const double *u) {
    double s = 0.0;
    for (int i = 0; i < p->cnt; ++i) s += p->w[i] * u[p->idx[i]];
    return s;
}
static void spread(const orc_interp *p, double value, double *field) {
    for (int i = 0; i < p->cnt; ++i) field[p->idx[i]] += p->w[i] * value;
}

/* ------------------------------------------------------------------------- */
/* One leapfrog step of  m u_tt + m d u_t - Lap u = q  (second order in time,
 * centred damping term):
 *   (1 + d dt/2) next = 2 cur - (1 - d dt/2) prev + (dt^2/m) (L cur + src).
 * The same step, run backwards with the receivers as sources, is the discrete
 * adjoint (L is symmetric).                                                  */
/* ------------------------------------------------------------------------- */

typedef struct {
    const orc_grid *g;
    int64_t np;
    double *mpad, *damp, *lap;
} orc_prop;

static int prop_init(orc_prop *p, const orc_grid *g, const double *m) {
    p->g = g;
    p->np = npad_total(g);
    p->mpad = (double *)malloc(sizeof(double) * p->np);
    p->damp = (double *)malloc(sizeof(double) * p->np);
    p->lap = (double *)malloc(sizeof(double) * p->np);
    if (!p->mpad || !p->damp || !p->lap) return 0;
    orc_pad_model(g, m, p->mpad);
    orc_damping(g, p->damp);
    return 1;
}
static void prop_free(orc_prop *p) {
    free(p->mpad); free(p->damp); free(p->lap);
}

static void leapfrog(orc_prop *p, const double *cur, const double *prev, const double *src, double *next) {
    const double dt = p->g->dt;
    orc_laplacian(p->g, cur, p->lap);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < p->np; ++i) {
        double beta = dt * dt / p->mpad[i];
        double ap = 1.0 + 0.5 * p->damp[i] * dt;
        double am = 1.0 - 0.5 * p->damp[i] * dt;
        double rhs = p->lap[i] + (src ? src[i] : 0.0);
        next[i] = (2.0 * cur[i] - am * prev[i] + beta * rhs) / ap;
    }
}

/* physical node -> padded index */
static int64_t phys_to_pad(const orc_grid *g, int64_t q) {
    int64_t x = q % g->n[0];
    int64_t y = (q / g->n[0]) % g->n[1];
    int64_t z = q / (g->n[0] * g->n[1]);
    return pidx(g, x + g->nbl, y + offset_y(g), z + g->nbl);
}

/* ------------------------------------------------------------------------- */
/* Probing matrix: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)          */
/* ------------------------------------------------------------------------- */

static void philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c[0];
        unsigned __int128 p1 = (unsigned __int128)M1 * c[2];
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    philox4x64_10(ctr, key, out);
}

static int popcount64(uint64_t v) {
    int c = 0;
    while (v) { c += (int)(v & 1u); v >>= 1; }
    return c;
}

/* Z[t][j] for one shot.  Counter (t+1, j, shot, 0), key (seed, 0); the first
 * output word w0 decides the entry:
 *   Rademacher:  1 - 2 * (top bit of w0)                 (random +-1)
 *   Gauss-B64:   (popcount(w0) - 32) / 4                 (centred binomial,
 *                unit variance, exact in binary floating point)
 *   Identity:    [t == j]  (needs r == nt; the complete orthonormal basis) */
int orc_probe_matrix(int32_t kind, int32_t r, uint64_t seed, int32_t nt, int32_t shot, double *Z) {
    if (r < 1 || nt < 1 || shot < 0) return ORC_E_INVAL;
    if (kind == ORC_PROBE_IDENTITY && r != nt) return ORC_E_INVAL;
    if (kind != ORC_PROBE_RADEMACHER && kind != ORC_PROBE_GAUSS_B64 && kind != ORC_PROBE_IDENTITY)
        return ORC_E_INVAL;
    const uint64_t key[2] = {seed, 0};
    for (int32_t t = 0; t < nt; ++t)
        for (int32_t j = 0; j < r; ++j) {
            double z;
            if (kind == ORC_PROBE_IDENTITY) {
                z = (t == j) ? 1.0 : 0.0;
            } else {
                uint64_t ctr[4] = {(uint64_t)t + 1, (uint64_t)j, (uint64_t)shot, 0};
                uint64_t w[4];
                philox4x64_10(ctr, key, w);
                if (kind == ORC_PROBE_RADEMACHER) z = 1.0 - 2.0 * (double)(w[0] >> 63);
                else z = ((double)popcount64(w[0]) - 32.0) / 4.0;
            }
            Z[(int64_t)t * r + j] = z;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Forward modelling F(m; q) and its adjoint                                  */
/* ------------------------------------------------------------------------- */

/* Forward modelling for one shot.  u^{-1} = u^0 = 0; for k = 0..nt-2 the step
 * injects q^k and produces u^{k+1}; the trace is d^k = R u^k for k = 0..nt-1.
 * Optional outputs: u_hist[k][phys] = u^k on the physical region (k = 0..nt-1),
 * ubar[j][pt] += Z[s][j] u^s (s = 1..nt-1) at the listed physical points
 * (Algorithm 1, forward loop; the default side: the wavefield itself is probed),
 * ubar2[j][pt] += Z[k][j] (u^{k+1} - 2u^k + u^{k-1}) (k = 0..nt-2; the paper's
 * Algorithm 1 side, second time difference probed in the forward loop). */
typedef struct {
    double *u_hist;
    const double *Z; int32_t r;
    const int64_t *pts; int64_t npts;
    double *ubar;
    double *ubar2;
} orc_fwd_extra;

static int forward_one(orc_prop *p, const orc_geom *geo, int32_t shot, double *d, orc_fwd_extra *ex) {
    const orc_grid *g = p->g;
    const int64_t np = p->np, nphys = nphys_total(g);
    orc_interp srcw;
    if (!interp_weights(g, &geo->src_pos[3 * shot], &srcw)) return ORC_E_GEOM;
    orc_interp *recw = (orc_interp *)malloc(sizeof(orc_interp) * (geo->nrec > 0 ? geo->nrec : 1));
    double *prev = (double *)calloc(np, sizeof(double));
    double *cur = (double *)calloc(np, sizeof(double));
    double *next = (double *)calloc(np, sizeof(double));
    double *src = (double *)calloc(np, sizeof(double));
    if (!recw || !prev || !cur || !next || !src) {
        free(recw); free(prev); free(cur); free(next); free(src);
        return ORC_E_NOMEM;
    }
    int st = ORC_OK;
    for (int32_t i = 0; i < geo->nrec; ++i)
        if (!interp_weights(g, &geo->rec_pos[3 * ((int64_t)shot * geo->nrec + i)], &recw[i])) st = ORC_E_GEOM;
    if (st != ORC_OK) goto done;

    for (int32_t k = 0; k <= g->nt - 1; ++k) {
        /* cur = u^k, prev = u^{k-1} */
        for (int32_t i = 0; i < geo->nrec; ++i) d[(int64_t)k * geo->nrec + i] = sample(&recw[i], cur);
        if (ex && ex->u_hist) {
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < nphys; ++q) ex->u_hist[(int64_t)k * nphys + q] = cur[phys_to_pad(g, q)];
        }
        if (k == g->nt - 1) break;
        memset(src, 0, sizeof(double) * np);
        spread(&srcw, geo->wavelet[(int64_t)shot * g->nt + k], src);
        leapfrog(p, cur, prev, src, next);
        /* next = u^{k+1} */
        if (ex && ex->ubar) {
            const double *zrow = &ex->Z[(int64_t)(k + 1) * ex->r];
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < ex->npts; ++q) {
                double uq = next[phys_to_pad(g, ex->pts[q])];
                for (int32_t j = 0; j < ex->r; ++j) ex->ubar[(int64_t)j * ex->npts + q] += zrow[j] * uq;
            }
        }
        if (ex && ex->ubar2) {
            const double *zrow = &ex->Z[(int64_t)k * ex->r];
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < ex->npts; ++q) {
                int64_t I = phys_to_pad(g, ex->pts[q]);
                double udd = next[I] - 2.0 * cur[I] + prev[I];
                for (int32_t j = 0; j < ex->r; ++j) ex->ubar2[(int64_t)j * ex->npts + q] += zrow[j] * udd;
            }
        }
        double *tmp = prev; prev = cur; cur = next; next = tmp;
    }
done:
    free(recw); free(prev); free(cur); free(next); free(src);
    return st;
}

/* Adjoint propagation for one shot, derived from the Lagrangian of the forward
 * recurrence.  lambda^{nt} = lambda^{nt-1} = 0; for k = nt-1..1 the step
 * injects R^T dd^k / dt^2 and produces lambda^{k-1}.  Outputs:
 *   q_adj[k] = dt^2 S lambda^k  (k = 0..nt-1; zero at k = nt-1),
 *   lam_hist[k][phys] = lambda^k (optional),
 *   vbar[j][pt] += Z[s][j] w^s, w^s = lambda^{s-1} - 2 lambda^s + lambda^{s+1},
 *                  s = 1..nt-1  (the default side),
 *   vbar2[j][pt] += Z[k][j] lambda^k, k = 0..nt-2  (the paper's side). */
typedef struct {
    double *lam_hist;
    const double *Z; int32_t r;
    const int64_t *pts; int64_t npts;
    double *vbar;
    double *vbar2;
} orc_adj_extra;

static int adjoint_one(orc_prop *p, const orc_geom *geo, int32_t shot, const double *dres, double *q_adj,
                       orc_adj_extra *ex) {
    const orc_grid *g = p->g;
    const int64_t np = p->np, nphys = nphys_total(g);
    const double dt = g->dt;
    orc_interp srcw;
    if (!interp_weights(g, &geo->src_pos[3 * shot], &srcw)) return ORC_E_GEOM;
    orc_interp *recw = (orc_interp *)malloc(sizeof(orc_interp) * (geo->nrec > 0 ? geo->nrec : 1));
    double *nxt = (double *)calloc(np, sizeof(double)); /* lambda^{k+1} */
    double *cur = (double *)calloc(np, sizeof(double)); /* lambda^k */
    double *prv = (double *)calloc(np, sizeof(double)); /* lambda^{k-1} */
    double *src = (double *)calloc(np, sizeof(double));
    if (!recw || !nxt || !cur || !prv || !src) {
        free(recw); free(nxt); free(cur); free(prv); free(src);
        return ORC_E_NOMEM;
    }
    int st = ORC_OK;
    for (int32_t i = 0; i < geo->nrec; ++i)
        if (!interp_weights(g, &geo->rec_pos[3 * ((int64_t)shot * geo->nrec + i)], &recw[i])) st = ORC_E_GEOM;
    if (st != ORC_OK) goto done;

    if (q_adj) q_adj[g->nt - 1] = 0.0;
    if (ex && ex->lam_hist) memset(&ex->lam_hist[(int64_t)(g->nt - 1) * nphys], 0, sizeof(double) * nphys);
    for (int32_t k = g->nt - 1; k >= 1; --k) {
        if (q_adj && k <= g->nt - 2) q_adj[k] = dt * dt * sample(&srcw, cur);
        memset(src, 0, sizeof(double) * np);
        for (int32_t i = 0; i < geo->nrec; ++i)
            spread(&recw[i], dres[(int64_t)k * geo->nrec + i] / (dt * dt), src);
        leapfrog(p, cur, nxt, src, prv);
        /* prv = lambda^{k-1}: w^k = lambda^{k-1} - 2 lambda^k + lambda^{k+1} */
        if (ex && ex->vbar) {
            const double *zrow = &ex->Z[(int64_t)k * ex->r];
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < ex->npts; ++q) {
                int64_t I = phys_to_pad(g, ex->pts[q]);
                double w = prv[I] - 2.0 * cur[I] + nxt[I];
                for (int32_t j = 0; j < ex->r; ++j) ex->vbar[(int64_t)j * ex->npts + q] += zrow[j] * w;
            }
        }
        if (ex && ex->vbar2) {
            /* lambda^{k-1} is now known; k-1 runs over nt-2..0 */
            const double *zrow = &ex->Z[(int64_t)(k - 1) * ex->r];
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < ex->npts; ++q) {
                double l = prv[phys_to_pad(g, ex->pts[q])];
                for (int32_t j = 0; j < ex->r; ++j) ex->vbar2[(int64_t)j * ex->npts + q] += zrow[j] * l;
            }
        }
        if (ex && ex->lam_hist) {
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < nphys; ++q) ex->lam_hist[(int64_t)(k - 1) * nphys + q] = prv[phys_to_pad(g, q)];
        }
        double *tmp = nxt; nxt = cur; cur = prv; prv = tmp;
    }
    /* cur = lambda^0 */
    if (q_adj) q_adj[0] = dt * dt * sample(&srcw, cur);
done:
    free(recw); free(nxt); free(cur); free(prv); free(src);
    return st;
}

static int valid_geom(const orc_grid *g, const orc_geom *geo) {
    if (!geo || geo->nshots < 1 || geo->nrec < 0 || !geo->src_pos || !geo->wavelet) return 0;
    if (geo->nrec > 0 && !geo->rec_pos) return 0;
    (void)g;
    return 1;
}

/* d[S][nt][nrec] = F(m; q) */
int orc_forward(const orc_grid *g, const orc_geom *geo, const double *m, double *d, double *u_hist) {
    if (!valid_grid(g) || !valid_geom(g, geo)) return ORC_E_INVAL;
    orc_prop p;
    if (!prop_init(&p, g, m)) { prop_free(&p); return ORC_E_NOMEM; }
    int st = ORC_OK;
    for (int32_t s = 0; s < geo->nshots && st == ORC_OK; ++s) {
        orc_fwd_extra ex;
        memset(&ex, 0, sizeof(ex));
        ex.u_hist = u_hist ? &u_hist[(int64_t)s * g->nt * nphys_total(g)] : NULL;
        st = forward_one(&p, geo, s, &d[(int64_t)s * g->nt * geo->nrec], &ex);
    }
    prop_free(&p);
    return st;
}

/* q_adj[S][nt] = F^T d_in (the adjoint of the source-to-trace map) */
int orc_adjoint(const orc_grid *g, const orc_geom *geo, const double *m, const double *d_in, double *q_adj,
                double *lam_hist) {
    if (!valid_grid(g) || !valid_geom(g, geo)) return ORC_E_INVAL;
    orc_prop p;
    if (!prop_init(&p, g, m)) { prop_free(&p); return ORC_E_NOMEM; }
    int st = ORC_OK;
    for (int32_t s = 0; s < geo->nshots && st == ORC_OK; ++s) {
        orc_adj_extra ex;
        memset(&ex, 0, sizeof(ex));
        ex.lam_hist = lam_hist ? &lam_hist[(int64_t)s * g->nt * nphys_total(g)] : NULL;
        st = adjoint_one(&p, geo, s, &d_in[(int64_t)s * g->nt * geo->nrec], &q_adj[(int64_t)s * g->nt], &ex);
    }
    prop_free(&p);
    return st;
}

/* J = 1/2 sum (d - d_obs)^2 (Eq. 2, no dt weighting); dres = d - d_obs */
static double residual(int64_t n, const double *d, const double *dobs, double *dres) {
    double J = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        dres[i] = d[i] - dobs[i];
        J += 0.5 * dres[i] * dres[i];
    }
    return J;
}

/* Exact adjoint-state gradient (Eq. 3), cropped to the physical region.
 *   form 0:  g = - sum_{s=1}^{nt-1} u^s (lambda^{s-1} - 2 lambda^s + lambda^{s+1})
 *   form 1:  g = - sum_{k=0}^{nt-2} lambda^k (u^{k+1} - 2 u^k + u^{k-1})
 * The two are equal by summation by parts (u^{-1} = u^0 = 0,
 * lambda^{nt-1} = lambda^{nt} = 0).  Uses the full forward history. */
int orc_gradient_full(const orc_grid *g, const orc_geom *geo, const double *m, const double *d_obs, int32_t form,
                      double *grad, double *J, double *d_out) {
    if (!valid_grid(g) || !valid_geom(g, geo) || (form != 0 && form != 1)) return ORC_E_INVAL;
    const int64_t nphys = nphys_total(g), nt = g->nt;
    const int64_t ntr = (int64_t)nt * geo->nrec;
    orc_prop p;
    if (!prop_init(&p, g, m)) { prop_free(&p); return ORC_E_NOMEM; }
    double *uh = (double *)malloc(sizeof(double) * nt * nphys);
    double *lh = (double *)malloc(sizeof(double) * nt * nphys);
    double *d = (double *)malloc(sizeof(double) * (ntr > 0 ? ntr : 1));
    double *dres = (double *)malloc(sizeof(double) * (ntr > 0 ? ntr : 1));
    int st = (uh && lh && d && dres) ? ORC_OK : ORC_E_NOMEM;
    double Jtot = 0.0;
    for (int64_t q = 0; q < nphys; ++q) grad[q] = 0.0;
    for (int32_t s = 0; s < geo->nshots && st == ORC_OK; ++s) {
        orc_fwd_extra fx;
        memset(&fx, 0, sizeof(fx));
        fx.u_hist = uh;
        st = forward_one(&p, geo, s, d, &fx);
        if (st != ORC_OK) break;
        if (d_out) memcpy(&d_out[(int64_t)s * ntr], d, sizeof(double) * ntr);
        Jtot += residual(ntr, d, &d_obs[(int64_t)s * ntr], dres);
        orc_adj_extra ax;
        memset(&ax, 0, sizeof(ax));
        ax.lam_hist = lh;
        st = adjoint_one(&p, geo, s, dres, NULL, &ax);
        if (st != ORC_OK) break;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < nphys; ++q) {
            double acc = 0.0;
            if (form == 0) {
                for (int64_t t = 1; t <= nt - 1; ++t) {
                    double lm = lh[(t - 1) * nphys + q];
                    double l0 = lh[t * nphys + q];
                    double lp = (t + 1 <= nt - 1) ? lh[(t + 1) * nphys + q] : 0.0;
                    acc += uh[t * nphys + q] * (lm - 2.0 * l0 + lp);
                }
            } else {
                for (int64_t k = 0; k <= nt - 2; ++k) {
                    double up = uh[(k + 1) * nphys + q];
                    double u0 = uh[k * nphys + q];
                    double um = (k >= 1) ? uh[(k - 1) * nphys + q] : 0.0;
                    acc += lh[k * nphys + q] * (up - 2.0 * u0 + um);
                }
            }
            grad[q] -= acc;
        }
    }
    if (J) *J = Jtot;
    free(uh); free(lh); free(d); free(dres);
    prop_free(&p);
    return st;
}

/* Probed gradient (Eq. 4, Algorithm 1): per shot, ubar and vbar are
 * accumulated on the fly during the forward and the back-propagation loop, and
 * g~ = -c sum_shots sum_j ubar_j * vbar_j (the trace of the outer product,
 * computed as the sum over probes of pointwise products).
 *   c = 1/r for Rademacher and Gauss-B64 probes, 1 for the identity, `scale`
 *   for an explicit Z.
 *   side 0: probes u and the second time difference of lambda (default);
 *   side 1: probes the second time difference of u and lambda (as printed).
 * pts/npts: physical points at which g~ is computed (NULL = every point). */
/* Inner product of the centred spatial gradients of two fields on the
 * physical grid at node q = (x, y, z): sum over axes of
 * (a[q+e] - a[q-e]) / (2h) * (b[q+e] - b[q-e]) / (2h); 0 on the outermost
 * physical nodes. */
static double grad_dot(const orc_grid *g, const double *a, const double *b, int64_t q) {
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const int64_t x = q % nx, y = (q / nx) % ny, z = q / (nx * ny);
    if (x == 0 || x == nx - 1 || z == 0 || z == nz - 1) return 0.0;
    if (g->ndim == 3 && (y == 0 || y == ny - 1)) return 0.0;
    const int64_t strides[3] = {1, nx, nx * ny};
    const double ih2 = 1.0 / (2.0 * g->h);
    double s = 0.0;
    for (int a3 = 0; a3 < 3; ++a3) {
        if (a3 == 1 && g->ndim == 2) continue;
        const int64_t e = strides[a3];
        s += ((a[q + e] - a[q - e]) * ih2) * ((b[q + e] - b[q - e]) * ih2);
    }
    return s;
}

/* imaging = 0: pointwise product of the probed fields (Eq. 4); imaging = 1:
 * inner product of their spatial gradients (Eq. 5 with the space-only operator
 * D_x = grad), which needs the whole physical grid (no point subset). */
int orc_gradient_probed(const orc_grid *g, const orc_geom *geo, const double *m, const double *d_obs,
                        int32_t kind, int32_t r, uint64_t seed, const double *Zexp, double scale, int32_t side,
                        int32_t imaging, const int64_t *pts_in, int64_t npts_in, double *grad, double *J,
                        double *d_out) {
    if (!valid_grid(g) || !valid_geom(g, geo) || r < 1 || (side != 0 && side != 1)) return ORC_E_INVAL;
    if ((imaging != 0 && imaging != 1) || (imaging == 1 && pts_in)) return ORC_E_INVAL;
    if (kind == ORC_PROBE_EXPLICIT && !Zexp) return ORC_E_INVAL;
    if (kind == ORC_PROBE_IDENTITY && r != g->nt) return ORC_E_INVAL;
    const int64_t nphys = nphys_total(g), nt = g->nt;
    const int64_t ntr = nt * geo->nrec;
    int64_t npts = pts_in ? npts_in : nphys;
    double c;
    if (kind == ORC_PROBE_RADEMACHER || kind == ORC_PROBE_GAUSS_B64) c = 1.0 / (double)r;
    else if (kind == ORC_PROBE_IDENTITY) c = 1.0;
    else if (kind == ORC_PROBE_EXPLICIT) c = scale;
    else return ORC_E_INVAL;

    orc_prop p;
    if (!prop_init(&p, g, m)) { prop_free(&p); return ORC_E_NOMEM; }
    int64_t *pts = (int64_t *)malloc(sizeof(int64_t) * (npts > 0 ? npts : 1));
    double *Z = (double *)malloc(sizeof(double) * nt * r);
    double *ub = (double *)malloc(sizeof(double) * r * (npts > 0 ? npts : 1));
    double *vb = (double *)malloc(sizeof(double) * r * (npts > 0 ? npts : 1));
    double *d = (double *)malloc(sizeof(double) * (ntr > 0 ? ntr : 1));
    double *dres = (double *)malloc(sizeof(double) * (ntr > 0 ? ntr : 1));
    int st = (pts && Z && ub && vb && d && dres) ? ORC_OK : ORC_E_NOMEM;
    if (st == ORC_OK)
        for (int64_t q = 0; q < npts; ++q) pts[q] = pts_in ? pts_in[q] : q;
    for (int64_t q = 0; q < npts; ++q) grad[q] = 0.0;
    double Jtot = 0.0;
    for (int32_t s = 0; s < geo->nshots && st == ORC_OK; ++s) {
        if (kind == ORC_PROBE_EXPLICIT) memcpy(Z, &Zexp[(int64_t)s * nt * r], sizeof(double) * nt * r);
        else st = orc_probe_matrix(kind, r, seed, g->nt, s, Z);
        if (st != ORC_OK) break;
        memset(ub, 0, sizeof(double) * r * npts);
        memset(vb, 0, sizeof(double) * r * npts);
        orc_fwd_extra fx;
        memset(&fx, 0, sizeof(fx));
        fx.Z = Z; fx.r = r; fx.pts = pts; fx.npts = npts;
        if (side == 0) fx.ubar = ub; else fx.ubar2 = ub;
        st = forward_one(&p, geo, s, d, &fx);
        if (st != ORC_OK) break;
        if (d_out) memcpy(&d_out[(int64_t)s * ntr], d, sizeof(double) * ntr);
        Jtot += residual(ntr, d, &d_obs[(int64_t)s * ntr], dres);
        orc_adj_extra ax;
        memset(&ax, 0, sizeof(ax));
        ax.Z = Z; ax.r = r; ax.pts = pts; ax.npts = npts;
        if (side == 0) ax.vbar = vb; else ax.vbar2 = vb;
        st = adjoint_one(&p, geo, s, dres, NULL, &ax);
        if (st != ORC_OK) break;
        for (int64_t q = 0; q < npts; ++q) {
            double tr = 0.0;
            for (int32_t j = 0; j < r; ++j) {
                if (imaging == 0) tr += ub[(int64_t)j * npts + q] * vb[(int64_t)j * npts + q];
                else tr += grad_dot(g, &ub[(int64_t)j * npts], &vb[(int64_t)j * npts], q);
            }
            grad[q] -= c * tr;
        }
    }
    if (J) *J = Jtot;
    free(pts); free(Z); free(ub); free(vb); free(d); free(dres);
    prop_free(&p);
    return st;
}

/* Manufactured-solution hook: propagate with a distributed source field
 * f[k][padded] (k = 0..nt-2) from zero initial state and return u^{nt-1} on the
 * padded box. */
int orc_propagate_field(const orc_grid *g, const double *m, const double *f, double *u_last) {
    if (!valid_grid(g)) return ORC_E_INVAL;
    orc_prop p;
    if (!prop_init(&p, g, m)) { prop_free(&p); return ORC_E_NOMEM; }
    const int64_t np = p.np;
    double *prev = (double *)calloc(np, sizeof(double));
    double *cur = (double *)calloc(np, sizeof(double));
    double *next = (double *)calloc(np, sizeof(double));
    if (!prev || !cur || !next) {
        free(prev); free(cur); free(next); prop_free(&p);
        return ORC_E_NOMEM;
    }
    for (int32_t k = 0; k <= g->nt - 2; ++k) {
        leapfrog(&p, cur, prev, &f[(int64_t)k * np], next);
        double *tmp = prev; prev = cur; cur = next; next = tmp;
    }
    memcpy(u_last, cur, sizeof(double) * np);
    free(prev); free(cur); free(next);
    prop_free(&p);
    return ORC_OK;
}
