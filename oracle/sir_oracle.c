/*
 * sir_oracle.c -- plain, slow, FP64 CPU oracle for the agent-based SIR
 * epidemiology model: infection, recovery and random movement of persons in
 * a cubic space with a toroidal or closed boundary.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * execute this file: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Source of every rule (thesis arXiv 2503.10796):
 *   - a susceptible person becomes infected, with the infection probability,
 *     if an infected person is within the infection radius      (Algorithm 3)
 *   - an infected person recovers with the recovery probability
 *     at every time step                                        (Algorithm 4)
 *   - random movement: three uniforms in (-1, 1) normalised to unit length,
 *     times the maximum movement per step, then every coordinate is wrapped
 *     into [0, S) with fmod (toroidal space)                    (Algorithm 5)
 *   - toroidal and closed space boundaries                     (Sec 4.4.11)
 *   - the model parameters (space length, radius, probabilities,
 *     movement per step, initial counts)                         (Table 4.3)
 *   - copy execution context: neighbours are read in their
 *     start-of-iteration state                                    (Sec 5.2.1)
 *   - counter-based generator for per-agent randomness            (Sec 7.1.4)
 * Readings where the thesis is silent:
 *   - behaviours of one person run in the order infection, recovery,
 *     movement, each on the person's own current state (a person infected
 *     in this iteration may recover in it);
 *   - "within the radius" is strict (d^2 < r^2, FP64, the squared distance
 *     summed as fma(dz, dz, fma(dy, dy, dx * dx)));
 *   - toroidal distances are minimum-image: per axis, an offset beyond half
 *     the space length is shifted by the space length (the neighbourhood of
 *     a person near a face continues on the opposite face);
 *   - a closed boundary clamps every coordinate to [0, S];
 *   - the draws: Philox4x32-10 with counter (uid, iteration, simulation)
 *     and key (seed low XOR tag, seed high), tags 'INFE', 'RECO', 'MOVE';
 *     a word w gives (w + 1/2) 2^-32 in (0, 1).
 *
 * The neighbour search is brute force over all persons: obviously correct
 * and O(N^2) per iteration, which the tests keep small.
 *
 * Parity pins: every function here is pinned by a "not gpu" test against
 * the SIR differential equations, binomial closed forms, an independent
 * image enumeration of the torus metric, and invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Philox4x32-10 draw of abm_oracle.c (the same oracle library). */
void orc_draw(uint64_t seed, uint32_t tag, uint32_t sim_id, uint64_t uid, uint64_t iter, uint32_t out[4]);

#define ORC_SIR_TAG_INFECTION 0x494e4645u /* 'INFE' */
#define ORC_SIR_TAG_RECOVERY 0x5245434fu  /* 'RECO' */
#define ORC_SIR_TAG_MOVE 0x4d4f5645u      /* 'MOVE' */

enum { ORC_SUSCEPTIBLE = 0, ORC_INFECTED = 1, ORC_RECOVERED = 2 };
enum { ORC_TOROIDAL = 0, ORC_CLOSED = 1 };

typedef struct {
    double space;           /* side S of the cubic space [0, S]^3 */
    double radius;          /* infection radius */
    double infection_prob;  /* per iteration, with an infected person in range */
    double recovery_prob;   /* per iteration */
    double speed;           /* length of the random step per iteration */
    int32_t boundary;       /* ORC_TOROIDAL or ORC_CLOSED */
    uint32_t sim_id;
    uint64_t seed;
} orc_sir_params;

static double sir_uniform(uint32_t w) { return ((double)w + 0.5) * 0x1.0p-32; }

/* Algorithm 5: the random step of a person (before the boundary). */
void orc_sir_step_vector(uint64_t seed, uint32_t sim_id, uint64_t uid, uint64_t iter, double speed, double d[3])
{
    uint32_t o[4];
    orc_draw(seed, ORC_SIR_TAG_MOVE, sim_id, uid, iter, o);
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = 2.0 * sir_uniform(o[a]) - 1.0;
    double norm = sqrt(fma(v[2], v[2], fma(v[1], v[1], v[0] * v[0])));
    for (int a = 0; a < 3; ++a) d[a] = (v[a] / norm) * speed;
}

/* Sec 4.4.11: a coordinate after the step, toroidal (Algorithm 5's wrap) or
 * closed (clamped to the walls). */
double orc_sir_bound(double v, double space, int boundary)
{
    if (boundary == ORC_CLOSED) return v < 0.0 ? 0.0 : (v > space ? space : v);
    double w = fmod(v, space);
    if (w < 0.0) w = space + w;
    return w;
}

/* Offset along one axis, minimum image on the torus. */
static double axis_offset(double a, double b, double space, int boundary)
{
    double d = b - a;
    if (boundary == ORC_TOROIDAL) {
        if (d > 0.5 * space) d -= space;
        else if (d < -0.5 * space) d += space;
    }
    return d;
}

double orc_sir_dist2(double xi, double yi, double zi, double xj, double yj, double zj, double space, int boundary)
{
    double dx = axis_offset(xi, xj, space, boundary);
    double dy = axis_offset(yi, yj, space, boundary);
    double dz = axis_offset(zi, zj, space, boundary);
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

/* Algorithm 3's draw: does the person try to catch the infection? */
int orc_sir_tries_infection(const orc_sir_params *p, uint64_t uid, uint64_t iter)
{
    uint32_t o[4];
    orc_draw(p->seed, ORC_SIR_TAG_INFECTION, p->sim_id, uid, iter, o);
    return sir_uniform(o[0]) < p->infection_prob;
}

/* Algorithm 4's draw. */
int orc_sir_recovers(const orc_sir_params *p, uint64_t uid, uint64_t iter)
{
    uint32_t o[4];
    orc_draw(p->seed, ORC_SIR_TAG_RECOVERY, p->sim_id, uid, iter, o);
    return sir_uniform(o[0]) < p->recovery_prob;
}

/* One iteration for n persons: positions and states are updated in place
 * (from copies of the start-of-iteration values); counts[0..2] receive the
 * numbers of susceptible, infected and recovered persons after it.
 * Returns 0, or -1 when memory runs out (the state is then unchanged). */
int orc_sir_step(int64_t n, double *x, double *y, double *z, uint8_t *state, const uint64_t *uid, int64_t iter,
                 const orc_sir_params *p, int64_t counts[3])
{
    counts[0] = counts[1] = counts[2] = 0;
    if (n <= 0) return 0;
    double *x0 = (double *)malloc(sizeof(double) * (size_t)n);
    double *y0 = (double *)malloc(sizeof(double) * (size_t)n);
    double *z0 = (double *)malloc(sizeof(double) * (size_t)n);
    uint8_t *s0 = (uint8_t *)malloc((size_t)n);
    if (!x0 || !y0 || !z0 || !s0) { free(x0); free(y0); free(z0); free(s0); return -1; }
    memcpy(x0, x, sizeof(double) * (size_t)n);
    memcpy(y0, y, sizeof(double) * (size_t)n);
    memcpy(z0, z, sizeof(double) * (size_t)n);
    memcpy(s0, state, (size_t)n);
    const double r2 = p->radius * p->radius;

#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        uint8_t s = s0[i];
        /* Algorithm 3: infection from an infected neighbour (start-of-iteration states) */
        if (s == ORC_SUSCEPTIBLE && orc_sir_tries_infection(p, uid[i], (uint64_t)iter)) {
            for (int64_t j = 0; j < n; ++j) {
                if (s0[j] != ORC_INFECTED) continue;
                if (orc_sir_dist2(x0[i], y0[i], z0[i], x0[j], y0[j], z0[j], p->space, p->boundary) < r2) {
                    s = ORC_INFECTED;
                    break;
                }
            }
        }
        /* Algorithm 4: recovery, on the person's state after its infection behaviour */
        if (s == ORC_INFECTED && orc_sir_recovers(p, uid[i], (uint64_t)iter)) s = ORC_RECOVERED;
        /* Algorithm 5: random step, then the boundary */
        double d[3];
        orc_sir_step_vector(p->seed, p->sim_id, uid[i], (uint64_t)iter, p->speed, d);
        x[i] = orc_sir_bound(x0[i] + d[0], p->space, p->boundary);
        y[i] = orc_sir_bound(y0[i] + d[1], p->space, p->boundary);
        z[i] = orc_sir_bound(z0[i] + d[2], p->space, p->boundary);
        state[i] = s;
    }
    for (int64_t i = 0; i < n; ++i) counts[state[i]] += 1;
    free(x0); free(y0); free(z0); free(s0);
    return 0;
}
