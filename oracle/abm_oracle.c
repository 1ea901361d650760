/*
 * abm_oracle.c -- plain, slow, FP64 CPU oracle for one iteration of
 * spherical-agent mechanics (uniform-grid neighbour search, sphere-sphere
 * force, adherence-thresholded and capped displacement, static-agent skip,
 * growth and division), the spheroid statistics, and the helper
 * definitions they need (Morton order, Philox4x32-10, cube root).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * execute this file: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Source of every rule (thesis arXiv 2503.10796):
 *   - grid: box length = largest agent or user value, agent box from its
 *     centre, 27 surrounding boxes searched                       (Sec 4.4.3)
 *   - open boundary: the space grows to enclose all agents        (Sec 4.4.11)
 *   - force magnitude F_N = k*delta - gamma*sqrt(r*delta),
 *     r = r1*r2/(r1+r2), k = 2, gamma = 1                    (Sec 4.5.1, Eq 4.1-4.2)
 *   - copy execution context: every agent reads the start-of-iteration
 *     state; additions become visible next iteration              (Sec 5.2.1)
 *   - force threshold that must be exceeded to move the agent and the
 *     four static-agent conditions                                 (Sec 5.5)
 *   - maximum displacement parameter and the cell mass        (Tutorial E.15)
 *   - cell behaviour: Brownian step, apoptosis after a minimum age
 *     with a death probability, grow or divide with a division
 *     probability                                  (Algorithm 2, Table 4.2)
 *   - removals take effect at the start of the next iteration     (Sec 5.2.1)
 *   - removals do not end the static state of neighbours, which
 *     condition (iv) makes safe                                    (Sec 5.5)
 *   - Morton order with x in the lowest bit                  (Sec 5.4.2, Fig 5.4)
 *   - counter-based generator for per-agent randomness            (Sec 7.1.4)
 * Readings where the thesis is silent (force direction, radii, threshold
 * comparison, displacement = F*dt/m, cap on the Euclidean norm, division
 * trigger on volume, daughter placement, Archimedes direction sampling,
 * summation order) are stated next to the code that takes them.
 *
 * Parity pins: every function here is pinned by a "not gpu" test against
 * closed forms, worked examples of the thesis, brute force or invariants.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Parameters and state (plain arrays owned by the caller).                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double dt, k, gamma, adherence, mass, max_disp;
    double box_len;     /* > 0: fixed box length; 0: largest diameter (Sec 4.4.3) */
    double div_vol;     /* > 0: grow below, divide at or above this volume; 0: off */
    double shift_frac;  /* each cell of a division moves shift_frac * r_mother */
    int32_t detect_static;
    int32_t brute_force; /* 1: neighbour sets by an O(N^2) scan instead of the grid */
    uint64_t seed;
    uint32_t sim_id;
    uint32_t pad;
    /* Algorithm 2 cell behaviour (Table 4.2): Brownian step length per
       iteration (0: off), death probability per iteration for cells of at
       least min_age iterations (0: off), division probability per iteration
       once the division volume is reached (1: always) */
    double brownian_rate, death_prob, division_prob;
    int32_t min_age;
    int32_t pad2;
} orc_params;

typedef struct {
    int64_t n, cap, next_uid, iter;
    double *x, *y, *z, *diam, *vol, *growth;
    uint64_t *uid;
    uint8_t *is_static; /* flag used by the coming iteration */
    int32_t *nz;        /* last computed number of non-zero neighbour forces */
    /* per-agent outputs of the last step (index = agent before appends) */
    int32_t *nbr, *contacts;          /* -1 for skipped (static) agents */
    double *fx, *fy, *fz;             /* force; 0 for skipped agents */
    double *dx, *dy, *dz;             /* displacement */
    int64_t *box;                     /* linear box id, x fastest */
    double *sum_abs_fn;               /* sum over contacts of |F_N| */
    double *sum_dfn;                  /* sum over contacts of |dF_N/d delta| */
    double *sum_fn_d;                 /* sum over contacts of |F_N| / distance (the conditioning of the
                                         force direction: centre-line error over distance) */
    uint8_t *moved, *grew, *divided, *is_new;
    double grid_lo[3], grid_hi[3], grid_L;
    int64_t grid_dims[3];
    int32_t *age;      /* iterations since the cell was created (Algorithm 2) */
    int64_t n_removed; /* agents the last step removed */
} orc_state;

/* ------------------------------------------------------------------------ */
/* Morton order: bit b of x goes to bit 3b, of y to 3b+1, of z to 3b+2       */
/* (x in the lowest bit, as in the 2-D example of Fig 5.4).                   */
/* ------------------------------------------------------------------------ */
uint64_t orc_morton3(uint32_t bx, uint32_t by, uint32_t bz)
{
    uint64_t code = 0;
    for (int b = 0; b < 21; ++b) {
        code |= (uint64_t)((bx >> b) & 1u) << (3 * b);
        code |= (uint64_t)((by >> b) & 1u) << (3 * b + 1);
        code |= (uint64_t)((bz >> b) & 1u) << (3 * b + 2);
    }
    return code;
}

uint64_t orc_morton2(uint32_t bx, uint32_t by)
{
    uint64_t code = 0;
    for (int b = 0; b < 32; ++b) {
        code |= (uint64_t)((bx >> b) & 1u) << (2 * b);
        code |= (uint64_t)((by >> b) & 1u) << (2 * b + 1);
    }
    return code;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two      */
/* 32x32->64 multiplications with the key bumped by the Weyl constants.       */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Division direction of the cell with this uid at this iteration, uniform on
 * the unit sphere by Archimedes' construction (z uniform in [-1,1), azimuth
 * uniform).  Counter = (uid low, uid high, iteration, simulation), key = seed.
 * Two 53-bit uniforms are taken from the four output words. */
void orc_direction(uint64_t seed, uint32_t sim_id, uint64_t uid, uint64_t iter, double u[3])
{
    uint32_t ctr[4] = {(uint32_t)uid, (uint32_t)(uid >> 32), (uint32_t)iter, sim_id};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    double u1 = (double)((((uint64_t)o[0] << 32) | o[1]) >> 11) * 0x1.0p-53;
    double u2 = (double)((((uint64_t)o[2] << 32) | o[3]) >> 11) * 0x1.0p-53;
    double zc = 2.0 * u1 - 1.0;
    double phi = 2.0 * ORC_PI * u2;
    double rho = sqrt((1.0 - zc) * (1.0 + zc));
    u[0] = rho * cos(phi);
    u[1] = rho * sin(phi);
    u[2] = zc;
}

/* Per-agent random words of Algorithm 2: Philox4x32-10 with counter (uid
 * low, uid high, iteration, simulation) and key (seed low XOR tag, seed
 * high), one tag per purpose, so that every draw is a pure function of the
 * agent and the iteration.  A word w gives the uniform (w + 1/2) 2^-32 in
 * the open interval (0, 1) (exact in double). */
#define ORC_TAG_BROWNIAN 0x42524f57u
#define ORC_TAG_DEATH 0x44454154u
#define ORC_TAG_DIVISION 0x44495650u

void orc_draw(uint64_t seed, uint32_t tag, uint32_t sim_id, uint64_t uid, uint64_t iter, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)uid, (uint32_t)(uid >> 32), (uint32_t)iter, sim_id};
    uint32_t key[2] = {(uint32_t)seed ^ tag, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

static double uniform_open(uint32_t w) { return ((double)w + 0.5) * 0x1.0p-32; }

/* The Brownian step of Algorithm 2: a vector of three uniforms in (-1, 1), divided by
 * its Euclidean norm, times the displacement rate.  (The normalised cube
 * vector is what the algorithm computes; it is not uniform on the sphere.) */
void orc_brownian(uint64_t seed, uint32_t sim_id, uint64_t uid, uint64_t iter, double rate, double d[3])
{
    uint32_t o[4];
    orc_draw(seed, ORC_TAG_BROWNIAN, sim_id, uid, iter, o);
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = 2.0 * uniform_open(o[a]) - 1.0;
    double norm = sqrt(fma(v[2], v[2], fma(v[1], v[1], v[0] * v[0])));
    for (int a = 0; a < 3; ++a) d[a] = (v[a] / norm) * rate;
}

/* Algorithm 2's removal of a cell of at least min_age iterations. */
int orc_dies(const orc_params *p, uint64_t uid, uint64_t iter, int32_t age)
{
    if (!(p->death_prob > 0.0) || age < p->min_age) return 0;
    uint32_t o[4];
    orc_draw(p->seed, ORC_TAG_DEATH, p->sim_id, uid, iter, o);
    return uniform_open(o[0]) < p->death_prob;
}

/* Algorithm 2's division draw of a cell at the division size. */
int orc_divides(const orc_params *p, uint64_t uid, uint64_t iter)
{
    uint32_t o[4];
    orc_draw(p->seed, ORC_TAG_DIVISION, p->sim_id, uid, iter, o);
    return uniform_open(o[0]) < p->division_prob;
}

/* Diameter of a sphere of volume V: the double nearest to cbrt(6V/pi), with
 * 6V/pi evaluated as (6*V)/pi in double.  The cube root is taken in 113-bit
 * precision and rounded once, so the result is the correctly rounded root. */
double orc_diameter_from_volume(double vol)
{
    double t = (6.0 * vol) / ORC_PI;
    return (double)cbrtq((__float128)t);
}

/* Eq 4.1-4.2: magnitude of the pair force for overlap delta > 0. */
double orc_pair_force(double r1, double r2, double delta, double k, double gamma)
{
    double rbar = r1 * r2 / (r1 + r2);
    return k * delta - gamma * sqrt(rbar * delta);
}

static double sq_dist(double xi, double yi, double zi, double xj, double yj, double zj)
{
    double ddx = xi - xj, ddy = yi - yj, ddz = zi - zj;
    return fma(ddz, ddz, fma(ddy, ddy, ddx * ddx));
}

/* ------------------------------------------------------------------------ */
/* Uniform grid over the bounding box of the agents (Sec 4.4.3, 4.4.11).     */
/* ------------------------------------------------------------------------ */
typedef struct {
    double lo[3], hi[3], L;
    int64_t dims[3];
    int64_t nboxes;
    int64_t *start;   /* nboxes + 1 */
    int64_t *order;   /* member indices sorted by (box, index) */
} orc_grid;

static int64_t box_coord(double v, double lo, double L, int64_t dim)
{
    double q = floor((v - lo) / L);
    int64_t b = (int64_t)q;
    if (q < 0.0) b = 0;
    if (b > dim - 1) b = dim - 1;
    return b;
}

static int64_t box_linear(const orc_grid *g, double x, double y, double z)
{
    int64_t bx = box_coord(x, g->lo[0], g->L, g->dims[0]);
    int64_t by = box_coord(y, g->lo[1], g->L, g->dims[1]);
    int64_t bz = box_coord(z, g->lo[2], g->L, g->dims[2]);
    return bx + g->dims[0] * (by + g->dims[1] * bz);
}

/* Set the geometry of the grid from agent positions and the box length. */
static void grid_geometry(orc_grid *g, int64_t n, const double *x, const double *y,
                          const double *z, double L)
{
    const double *c[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        double lo = c[a][0], hi = c[a][0];
        for (int64_t i = 1; i < n; ++i) {
            if (c[a][i] < lo) lo = c[a][i];
            if (c[a][i] > hi) hi = c[a][i];
        }
        g->lo[a] = lo;
        g->hi[a] = hi;
    }
    g->L = L;
    for (int a = 0; a < 3; ++a) g->dims[a] = (int64_t)floor((g->hi[a] - g->lo[a]) / L) + 1;
    g->nboxes = g->dims[0] * g->dims[1] * g->dims[2];
}

/* Bin m points into the grid's boxes (clamped to the grid). */
static int grid_bin(orc_grid *g, int64_t m, const double *x, const double *y, const double *z)
{
    g->start = (int64_t *)calloc((size_t)g->nboxes + 1, sizeof(int64_t));
    g->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!g->start || !g->order || !key) { free(key); return -1; }
    for (int64_t i = 0; i < m; ++i) {
        key[i] = box_linear(g, x[i], y[i], z[i]);
        g->start[key[i] + 1] += 1;
    }
    for (int64_t b = 0; b < g->nboxes; ++b) g->start[b + 1] += g->start[b];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)g->nboxes);
    if (!fill) { free(key); return -1; }
    memcpy(fill, g->start, sizeof(int64_t) * (size_t)g->nboxes);
    for (int64_t i = 0; i < m; ++i) g->order[fill[key[i]]++] = i;
    free(fill);
    free(key);
    return 0;
}

static void grid_free(orc_grid *g)
{
    free(g->start);
    free(g->order);
    g->start = g->order = NULL;
}

/* ------------------------------------------------------------------------ */
/* Neighbour collection.                                                     */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t *idx; int64_t n, cap; } orc_list;

static int list_push(orc_list *l, int64_t v)
{
    if (l->n == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 64;
        int64_t *p = (int64_t *)realloc(l->idx, sizeof(int64_t) * (size_t)nc);
        if (!p) return -1;
        l->idx = p;
        l->cap = nc;
    }
    l->idx[l->n++] = v;
    return 0;
}

/* All j != i with squared distance < L^2 (strict), from the 27 boxes around
 * the box of agent i, or from every agent when brute is set. */
static int collect_neighbours(const orc_state *s, const orc_grid *g, int64_t i, int brute,
                              orc_list *out)
{
    const double L2 = g->L * g->L;
    out->n = 0;
    if (brute) {
        for (int64_t j = 0; j < s->n; ++j) {
            if (j == i) continue;
            if (sq_dist(s->x[i], s->y[i], s->z[i], s->x[j], s->y[j], s->z[j]) < L2)
                if (list_push(out, j)) return -1;
        }
        return 0;
    }
    int64_t bx = box_coord(s->x[i], g->lo[0], g->L, g->dims[0]);
    int64_t by = box_coord(s->y[i], g->lo[1], g->L, g->dims[1]);
    int64_t bz = box_coord(s->z[i], g->lo[2], g->L, g->dims[2]);
    for (int64_t oz = -1; oz <= 1; ++oz)
        for (int64_t oy = -1; oy <= 1; ++oy)
            for (int64_t ox = -1; ox <= 1; ++ox) {
                int64_t cx = bx + ox, cy = by + oy, cz = bz + oz;
                if (cx < 0 || cy < 0 || cz < 0) continue;
                if (cx >= g->dims[0] || cy >= g->dims[1] || cz >= g->dims[2]) continue;
                int64_t b = cx + g->dims[0] * (cy + g->dims[1] * cz);
                for (int64_t p = g->start[b]; p < g->start[b + 1]; ++p) {
                    int64_t j = g->order[p];
                    if (j == i) continue;
                    if (sq_dist(s->x[i], s->y[i], s->z[i], s->x[j], s->y[j], s->z[j]) < L2)
                        if (list_push(out, j)) return -1;
                }
            }
    return 0;
}

static const uint64_t *g_sort_uid; /* uid table for the comparator below */
static int cmp_by_uid(const void *a, const void *b)
{
    uint64_t ua = g_sort_uid[*(const int64_t *)a], ub = g_sort_uid[*(const int64_t *)b];
    return (ua > ub) - (ua < ub);
}

static void sort_by_uid(int64_t *idx, int64_t n, const uint64_t *uid)
{
    /* insertion sort: neighbour lists are short and this keeps the
       comparator free of global state under threads */
    for (int64_t a = 1; a < n; ++a) {
        int64_t v = idx[a];
        int64_t b = a - 1;
        while (b >= 0 && uid[idx[b]] > uid[v]) { idx[b + 1] = idx[b]; --b; }
        idx[b + 1] = v;
    }
}

/* ------------------------------------------------------------------------ */
/* Force on one agent from the start-of-iteration state.                     */
/* Readings: the force acts along the centre line and a positive F_N pushes   */
/* the pair apart; the attractive part is kept; r is the radius (d/2); only   */
/* overlapping pairs (delta > 0, strict) interact; coincident centres give    */
/* no force; the sum runs over neighbours in ascending uid order.            */
/* ------------------------------------------------------------------------ */
typedef struct {
    double f[3];
    int32_t nbr, contacts, nz;
    double sum_abs_fn, sum_dfn, sum_fn_d;
} orc_force;

static void agent_force(const orc_state *s, const orc_params *p, int64_t i,
                        const orc_list *nbrs, orc_force *out)
{
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    int32_t contacts = 0, nz = 0;
    double sabs = 0.0, sd = 0.0, sfd = 0.0;
    double ri = 0.5 * s->diam[i];
    for (int64_t q = 0; q < nbrs->n; ++q) {
        int64_t j = nbrs->idx[q];
        double rj = 0.5 * s->diam[j];
        double ddx = s->x[i] - s->x[j], ddy = s->y[i] - s->y[j], ddz = s->z[i] - s->z[j];
        double dist = sqrt(fma(ddz, ddz, fma(ddy, ddy, ddx * ddx)));
        double delta = ri + rj - dist;
        if (!(delta > 0.0)) continue;
        contacts += 1;
        double fn = orc_pair_force(ri, rj, delta, p->k, p->gamma);
        if (fn != 0.0) nz += 1;
        double rbar = ri * rj / (ri + rj);
        sabs += fabs(fn);
        sd += fabs(p->k - p->gamma * sqrt(rbar) / (2.0 * sqrt(delta)));
        if (dist > 0.0) {
            sfd += fabs(fn) / dist;
            f0 += fn * ddx / dist;
            f1 += fn * ddy / dist;
            f2 += fn * ddz / dist;
        }
    }
    out->f[0] = f0; out->f[1] = f1; out->f[2] = f2;
    out->nbr = (int32_t)nbrs->n;
    out->contacts = contacts;
    out->nz = nz;
    out->sum_abs_fn = sabs;
    out->sum_dfn = sd;
    out->sum_fn_d = sfd;
}

/* Displacement from the force: no motion unless |F| exceeds the adherence
 * threshold (Sec 5.5); otherwise F*dt/m, capped in Euclidean norm at the
 * maximum displacement (Tutorial E.15). */
void orc_displacement(const double f[3], double adherence, double dt, double mass,
                      double max_disp, double d[3])
{
    double fnorm = sqrt(fma(f[2], f[2], fma(f[1], f[1], f[0] * f[0])));
    if (!(fnorm > adherence)) { d[0] = d[1] = d[2] = 0.0; return; }
    double scale = dt / mass;
    d[0] = f[0] * scale; d[1] = f[1] * scale; d[2] = f[2] * scale;
    double dn = sqrt(fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0])));
    if (dn > max_disp) {
        double c = max_disp / dn;
        d[0] *= c; d[1] *= c; d[2] *= c;
    }
}

/* Box length of the coming iteration: fixed, or the largest diameter. */
static double box_length(const orc_state *s, const orc_params *p)
{
    if (p->box_len > 0.0) return p->box_len;
    double L = 0.0;
    for (int64_t i = 0; i < s->n; ++i) if (s->diam[i] > L) L = s->diam[i];
    return L;
}

/* ------------------------------------------------------------------------ */
/* One iteration (copy semantics).  Returns 0, or -1 on allocation failure,  */
/* -2 when the divisions would exceed the capacity (state untouched).        */
/* ------------------------------------------------------------------------ */
int orc_step(orc_state *s, const orc_params *p)
{
    const int64_t n = s->n;
    s->n_removed = 0;
    if (n <= 0) { s->iter += 1; return 0; }
    /* with Brownian motion every cell moves every iteration: no cell can be
       static, and the combination is refused */
    if (p->detect_static && p->brownian_rate > 0.0) return -3;

    /* the decisions of Algorithm 2 from the start-of-iteration state, first,
       so that a capacity overflow leaves the state untouched: removal,
       then, for the cells that stay, division (grow below the division
       volume, else divide with the division probability) */
    uint8_t *dies = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *divs = (uint8_t *)calloc((size_t)n, 1);
    if (!dies || !divs) { free(dies); free(divs); return -1; }
    int64_t ndiv = 0, ndead = 0;
    for (int64_t i = 0; i < n; ++i) {
        dies[i] = (uint8_t)orc_dies(p, s->uid[i], (uint64_t)s->iter, s->age[i]);
        ndead += dies[i];
        if (!dies[i] && p->div_vol > 0.0 && s->vol[i] >= p->div_vol && orc_divides(p, s->uid[i], (uint64_t)s->iter)) {
            divs[i] = 1;
            ndiv += 1;
        }
    }
    if (n + ndiv > s->cap) { free(dies); free(divs); return -2; }

    orc_grid g;
    memset(&g, 0, sizeof g);
    grid_geometry(&g, n, s->x, s->y, s->z, box_length(s, p));
    if (grid_bin(&g, n, s->x, s->y, s->z)) { grid_free(&g); return -1; }
    for (int a = 0; a < 3; ++a) { s->grid_lo[a] = g.lo[a]; s->grid_hi[a] = g.hi[a]; s->grid_dims[a] = g.dims[a]; }
    s->grid_L = g.L;

    double *nx = (double *)malloc(sizeof(double) * (size_t)n);
    double *ny = (double *)malloc(sizeof(double) * (size_t)n);
    double *nzp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!nx || !ny || !nzp) { free(nx); free(ny); free(nzp); grid_free(&g); free(dies); free(divs); return -1; }

    int failed = 0;
    /* mechanics: every agent reads only the start-of-iteration state */
#pragma omp parallel
    {
        orc_list nb = {NULL, 0, 0};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            s->box[i] = box_linear(&g, s->x[i], s->y[i], s->z[i]);
            double d[3] = {0.0, 0.0, 0.0};
            if (p->detect_static && s->is_static[i]) {
                /* static agent: force not computed, no motion, nz kept */
                s->fx[i] = s->fy[i] = s->fz[i] = 0.0;
                s->nbr[i] = -1;
                s->contacts[i] = -1;
                s->sum_abs_fn[i] = 0.0;
                s->sum_dfn[i] = 0.0;
                s->sum_fn_d[i] = 0.0;
            } else {
                if (collect_neighbours(s, &g, i, p->brute_force, &nb)) { failed = 1; continue; }
                sort_by_uid(nb.idx, nb.n, s->uid);
                orc_force fo;
                agent_force(s, p, i, &nb, &fo);
                s->fx[i] = fo.f[0]; s->fy[i] = fo.f[1]; s->fz[i] = fo.f[2];
                s->nbr[i] = fo.nbr;
                s->contacts[i] = fo.contacts;
                s->nz[i] = fo.nz;
                s->sum_abs_fn[i] = fo.sum_abs_fn;
                s->sum_dfn[i] = fo.sum_dfn;
                s->sum_fn_d[i] = fo.sum_fn_d;
                orc_displacement(fo.f, p->adherence, p->dt, p->mass, p->max_disp, d);
            }
            s->dx[i] = d[0]; s->dy[i] = d[1]; s->dz[i] = d[2];
            /* Algorithm 2: the Brownian step first, then the mechanical
               displacement: x' = (x + b) + d */
            double b[3] = {0.0, 0.0, 0.0};
            if (p->brownian_rate > 0.0) orc_brownian(p->seed, p->sim_id, s->uid[i], (uint64_t)s->iter, p->brownian_rate, b);
            nx[i] = (s->x[i] + b[0]) + d[0];
            ny[i] = (s->y[i] + b[1]) + d[1];
            nzp[i] = (s->z[i] + b[2]) + d[2];
            s->moved[i] = (nx[i] != s->x[i] || ny[i] != s->y[i] || nzp[i] != s->z[i]);
            s->grew[i] = 0;
            s->divided[i] = 0;
            s->is_new[i] = 0;
        }
        free(nb.idx);
    }
    if (failed) { free(nx); free(ny); free(nzp); grid_free(&g); free(dies); free(divs); return -1; }

    /* start-of-iteration positions are kept for the static rule */
    double *sx = (double *)malloc(sizeof(double) * (size_t)n);
    double *sy = (double *)malloc(sizeof(double) * (size_t)n);
    double *sz = (double *)malloc(sizeof(double) * (size_t)n);
    if (!sx || !sy || !sz) { free(sx); free(sy); free(sz); free(nx); free(ny); free(nzp); grid_free(&g); free(dies); free(divs); return -1; }
    memcpy(sx, s->x, sizeof(double) * (size_t)n);
    memcpy(sy, s->y, sizeof(double) * (size_t)n);
    memcpy(sz, s->z, sizeof(double) * (size_t)n);
    /* commit positions */
    memcpy(s->x, nx, sizeof(double) * (size_t)n);
    memcpy(s->y, ny, sizeof(double) * (size_t)n);
    memcpy(s->z, nzp, sizeof(double) * (size_t)n);
    free(nx); free(ny); free(nzp);

    /* Algorithm 2: the cells that stay age by one iteration */
    for (int64_t i = 0; i < n; ++i)
        if (!dies[i]) s->age[i] += 1;

    /* growth or division (Algorithm 2, grow branch and divide branch), from
       the start-of-iteration volume, applied to the committed position.
       Daughter uids: next_uid + rank of the mother's uid among this
       iteration's dividers; a daughter starts at age 0 and the mother keeps
       her age.  A cell at the division volume whose division draw fails
       neither grows nor divides. */
    int64_t m = n;
    if (p->div_vol > 0.0) {
        int64_t *dividers = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ndiv > 0 ? ndiv : 1));
        if (!dividers) { free(sx); free(sy); free(sz); grid_free(&g); free(dies); free(divs); return -1; }
        int64_t q = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (dies[i]) continue;
            if (s->vol[i] < p->div_vol) {
                s->vol[i] = s->vol[i] + s->growth[i];
                s->diam[i] = orc_diameter_from_volume(s->vol[i]);
                s->grew[i] = 1;
            } else if (divs[i]) {
                dividers[q++] = i;
            }
        }
        g_sort_uid = s->uid;
        qsort(dividers, (size_t)ndiv, sizeof(int64_t), cmp_by_uid);
        for (int64_t rank = 0; rank < ndiv; ++rank) {
            int64_t i = dividers[rank];
            double u[3];
            orc_direction(p->seed, p->sim_id, s->uid[i], (uint64_t)s->iter, u);
            double shift = p->shift_frac * (0.5 * s->diam[i]);
            double half = 0.5 * s->vol[i];
            double dnew = orc_diameter_from_volume(half);
            double cx = s->x[i], cy = s->y[i], cz = s->z[i];
            int64_t j = n + rank;
            s->x[j] = cx + shift * u[0];
            s->y[j] = cy + shift * u[1];
            s->z[j] = cz + shift * u[2];
            s->x[i] = cx - shift * u[0];
            s->y[i] = cy - shift * u[1];
            s->z[i] = cz - shift * u[2];
            s->vol[i] = half;
            s->vol[j] = half;
            s->diam[i] = dnew;
            s->diam[j] = dnew;
            s->growth[j] = s->growth[i];
            s->uid[j] = (uint64_t)s->next_uid + (uint64_t)rank;
            s->nz[j] = 0;
            s->is_static[j] = 0;
            s->moved[i] = 1;
            s->divided[i] = 1;
            s->moved[j] = 1;
            s->grew[j] = 0;
            s->divided[j] = 0;
            s->is_new[j] = 1;
            s->age[j] = 0;
        }
        free(dividers);
        m = n + ndiv;
        s->next_uid += ndiv;
    }

    /* static flags for the coming iteration (Sec 5.5): not changed itself,
       at most one non-zero neighbour force, and no changed agent within the
       interaction radius L at its start or its committed position.  A
       changed agent moved, grew, divided or is new. */
    /* a removed cell is no change for its neighbours (Sec 5.5: condition
       (iv) lets cells be removed without ending the static state around
       them) */
    for (int64_t i = 0; i < n; ++i)
        if (dies[i]) s->moved[i] = s->grew[i] = s->divided[i] = 0;
    if (p->detect_static) {
        int64_t nchg = 0;
        for (int64_t j = 0; j < m; ++j)
            if (s->moved[j] || s->grew[j] || s->divided[j] || s->is_new[j]) nchg += 1;
        int64_t cap2 = 2 * (nchg > 0 ? nchg : 1);
        double *px = (double *)malloc(sizeof(double) * (size_t)cap2);
        double *py = (double *)malloc(sizeof(double) * (size_t)cap2);
        double *pz = (double *)malloc(sizeof(double) * (size_t)cap2);
        int64_t *owner = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap2);
        if (!px || !py || !pz || !owner) { free(px); free(py); free(pz); free(owner); free(sx); free(sy); free(sz); grid_free(&g); free(dies); free(divs); return -1; }
        int64_t np = 0;
        for (int64_t j = 0; j < m; ++j) {
            if (!(s->moved[j] || s->grew[j] || s->divided[j] || s->is_new[j])) continue;
            if (j < n) { px[np] = sx[j]; py[np] = sy[j]; pz[np] = sz[j]; owner[np] = j; ++np; }
            px[np] = s->x[j]; py[np] = s->y[j]; pz[np] = s->z[j]; owner[np] = j; ++np;
        }
        orc_grid cg;
        memset(&cg, 0, sizeof cg);
        memcpy(cg.lo, g.lo, sizeof g.lo);
        memcpy(cg.hi, g.hi, sizeof g.hi);
        cg.L = g.L;
        memcpy(cg.dims, g.dims, sizeof g.dims);
        cg.nboxes = g.nboxes;
        if (grid_bin(&cg, np, px, py, pz)) { grid_free(&cg); free(px); free(py); free(pz); free(owner); free(sx); free(sy); free(sz); grid_free(&g); free(dies); free(divs); return -1; }
        const double L2 = g.L * g.L;
        for (int64_t i = 0; i < m; ++i) {
            int st = !(s->moved[i] || s->grew[i] || s->divided[i] || s->is_new[i]) && s->nz[i] <= 1;
            if (st && p->brute_force) {
                for (int64_t q = 0; q < np && st; ++q)
                    if (owner[q] != i && sq_dist(s->x[i], s->y[i], s->z[i], px[q], py[q], pz[q]) < L2) st = 0;
            } else if (st) {
                int64_t bx = box_coord(s->x[i], g.lo[0], g.L, g.dims[0]);
                int64_t by = box_coord(s->y[i], g.lo[1], g.L, g.dims[1]);
                int64_t bz = box_coord(s->z[i], g.lo[2], g.L, g.dims[2]);
                for (int64_t oz = -1; oz <= 1 && st; ++oz)
                    for (int64_t oy = -1; oy <= 1 && st; ++oy)
                        for (int64_t ox = -1; ox <= 1 && st; ++ox) {
                            int64_t cx = bx + ox, cy = by + oy, cz = bz + oz;
                            if (cx < 0 || cy < 0 || cz < 0) continue;
                            if (cx >= g.dims[0] || cy >= g.dims[1] || cz >= g.dims[2]) continue;
                            int64_t b = cx + g.dims[0] * (cy + g.dims[1] * cz);
                            for (int64_t t = cg.start[b]; t < cg.start[b + 1]; ++t) {
                                int64_t q = cg.order[t];
                                if (owner[q] != i && sq_dist(s->x[i], s->y[i], s->z[i], px[q], py[q], pz[q]) < L2) { st = 0; break; }
                            }
                        }
            }
            s->is_static[i] = (uint8_t)st;
        }
        grid_free(&cg);
        free(px); free(py); free(pz); free(owner);
    } else {
        for (int64_t i = 0; i < m; ++i) s->is_static[i] = 0;
    }

    /* removals (Algorithm 2) take effect for the next iteration: the
       cells that stay keep their order (daughters, never removed in the
       iteration that creates them, follow) */
    if (ndead > 0) {
        int64_t w = 0;
        for (int64_t i = 0; i < m; ++i) {
            if (i < n && dies[i]) continue;
            if (w != i) {
                s->x[w] = s->x[i]; s->y[w] = s->y[i]; s->z[w] = s->z[i];
                s->diam[w] = s->diam[i]; s->vol[w] = s->vol[i]; s->growth[w] = s->growth[i];
                s->uid[w] = s->uid[i]; s->is_static[w] = s->is_static[i]; s->nz[w] = s->nz[i];
                s->age[w] = s->age[i];
                s->nbr[w] = s->nbr[i]; s->contacts[w] = s->contacts[i];
                s->fx[w] = s->fx[i]; s->fy[w] = s->fy[i]; s->fz[w] = s->fz[i];
                s->dx[w] = s->dx[i]; s->dy[w] = s->dy[i]; s->dz[w] = s->dz[i];
                s->box[w] = s->box[i];
                s->sum_abs_fn[w] = s->sum_abs_fn[i]; s->sum_dfn[w] = s->sum_dfn[i]; s->sum_fn_d[w] = s->sum_fn_d[i];
                s->moved[w] = s->moved[i]; s->grew[w] = s->grew[i]; s->divided[w] = s->divided[i];
                s->is_new[w] = s->is_new[i];
            }
            ++w;
        }
        m = w;
    }
    free(dies); free(divs);
    free(sx); free(sy); free(sz);
    grid_free(&g);
    s->n = m;
    s->n_removed = ndead;
    s->iter += 1;
    return 0;
}

/* Forces, counts and displacements of selected agents in the given state,
 * without changing it (used for sampled checks of large populations). */
int orc_forces_subset(const orc_state *s, const orc_params *p, int64_t nsel, const int64_t *sel,
                      double *f_out /* nsel x 3 */, int32_t *cnt_out /* nsel x 3: nbr, contacts, nz */,
                      double *d_out /* nsel x 3 */, double *tol_out /* nsel x 3: sum|F_N|, sum|dF_N/d delta|, sum|F_N|/distance */)
{
    orc_grid g;
    memset(&g, 0, sizeof g);
    grid_geometry(&g, s->n, s->x, s->y, s->z, box_length(s, p));
    if (grid_bin(&g, s->n, s->x, s->y, s->z)) { grid_free(&g); return -1; }
    int failed = 0;
#pragma omp parallel
    {
        orc_list nb = {NULL, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < nsel; ++q) {
            int64_t i = sel[q];
            if (collect_neighbours(s, &g, i, p->brute_force, &nb)) { failed = 1; continue; }
            sort_by_uid(nb.idx, nb.n, s->uid);
            orc_force fo;
            agent_force(s, p, i, &nb, &fo);
            double d[3];
            orc_displacement(fo.f, p->adherence, p->dt, p->mass, p->max_disp, d);
            for (int a = 0; a < 3; ++a) { f_out[3 * q + a] = fo.f[a]; d_out[3 * q + a] = d[a]; }
            cnt_out[3 * q] = fo.nbr;
            cnt_out[3 * q + 1] = fo.contacts;
            cnt_out[3 * q + 2] = fo.nz;
            tol_out[3 * q] = fo.sum_abs_fn;
            tol_out[3 * q + 1] = fo.sum_dfn;
            tol_out[3 * q + 2] = fo.sum_fn_d;
        }
        free(nb.idx);
    }
    grid_free(&g);
    return failed ? -1 : 0;
}

/* Neighbour uids of agent i (ascending), by the grid or by brute force.
 * Returns the number of neighbours or -1; writes at most cap uids. */
int64_t orc_neighbour_uids(const orc_state *s, const orc_params *p, int64_t i, int brute,
                           uint64_t *out, int64_t cap)
{
    orc_grid g;
    memset(&g, 0, sizeof g);
    grid_geometry(&g, s->n, s->x, s->y, s->z, box_length(s, p));
    if (grid_bin(&g, s->n, s->x, s->y, s->z)) { grid_free(&g); return -1; }
    orc_list nb = {NULL, 0, 0};
    if (collect_neighbours(s, &g, i, brute, &nb)) { free(nb.idx); grid_free(&g); return -1; }
    sort_by_uid(nb.idx, nb.n, s->uid);
    for (int64_t q = 0; q < nb.n && q < cap; ++q) out[q] = s->uid[nb.idx[q]];
    int64_t cnt = nb.n;
    free(nb.idx);
    grid_free(&g);
    return cnt;
}

/* Grid of the given state: lo[3], L, dims[3], and the box of every agent. */
int orc_grid_info(const orc_state *s, const orc_params *p, double lo[3], double *L,
                  int64_t dims[3], int64_t *box)
{
    orc_grid g;
    memset(&g, 0, sizeof g);
    grid_geometry(&g, s->n, s->x, s->y, s->z, box_length(s, p));
    for (int a = 0; a < 3; ++a) { lo[a] = g.lo[a]; dims[a] = g.dims[a]; }
    *L = g.L;
    for (int64_t i = 0; i < s->n; ++i) box[i] = box_linear(&g, s->x[i], s->y[i], s->z[i]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Spheroid statistics: centroid, radius of gyration, largest distance from   */
/* the centroid, and a 32-bin radial density histogram on [0, hist_rmax)     */
/* (agents per 1000 um^3 of shell; agents beyond hist_rmax go to the last     */
/* bin).                                                                      */
/* ------------------------------------------------------------------------ */
void orc_stats(int64_t n, const double *x, const double *y, const double *z, double hist_rmax,
               double centroid[3], double *r_gyr, double *r_max, float hist[32], int64_t counts[32])
{
    double cx = 0.0, cy = 0.0, cz = 0.0;
    for (int64_t i = 0; i < n; ++i) { cx += x[i]; cy += y[i]; cz += z[i]; }
    if (n > 0) { cx /= (double)n; cy /= (double)n; cz /= (double)n; }
    centroid[0] = cx; centroid[1] = cy; centroid[2] = cz;
    double s2 = 0.0, rmax = 0.0;
    for (int b = 0; b < 32; ++b) counts[b] = 0;
    const double w = hist_rmax / 32.0;
    for (int64_t i = 0; i < n; ++i) {
        double d2 = sq_dist(x[i], y[i], z[i], cx, cy, cz);
        double r = sqrt(d2);
        s2 += d2;
        if (r > rmax) rmax = r;
        int64_t b = (int64_t)floor(r / w);
        if (b > 31) b = 31;
        counts[b] += 1;
    }
    *r_gyr = n > 0 ? sqrt(s2 / (double)n) : 0.0;
    *r_max = rmax;
    for (int b = 0; b < 32; ++b) {
        double r0 = w * b, r1 = w * (b + 1);
        double shell = 4.0 / 3.0 * ORC_PI * (r1 * r1 * r1 - r0 * r0 * r0);
        hist[b] = (float)((double)counts[b] / shell * 1000.0);
    }
}
