/*
 * soma_oracle.c -- plain, slow, FP64 CPU oracle for extracellular diffusion
 * (the central-difference scheme of Eq 4.3) and the soma clustering cell
 * behaviours (substance secretion, chemotaxis).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * execute this file: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Source of every rule (thesis arXiv 2503.10796):
 *   - concentration update per grid point: decay by (1 - mu dt), plus
 *     nu dt / dx^2 times the second difference along each axis   (Eq 4.3)
 *   - substances diffuse out of the simulation space               (Sec 4.5.2)
 *   - secretion: a cell increases the concentration of its substance
 *     at its position by the secretion quantity                  (Algorithm 6)
 *   - chemotaxis: a cell moves by the normalised gradient of its
 *     substance at its position times the gradient weight         (Algorithm 7)
 *   - two cell types, each secreting and following its own
 *     substance; secretion quantity 1, gradient weight 0.75       (Sec 4.7.1)
 *   - copy execution context                                       (Sec 5.2.1)
 * Readings where the thesis is silent:
 *   - the grid has R points per axis at the centres of R^3 equal voxels of
 *     the cubic space [lo, lo + S]^3 (dx = S / R); a position belongs to the
 *     voxel floor((x - lo) / dx), clamped to [0, R - 1];
 *   - "diffuse out" is a zero concentration beyond the grid (Dirichlet);
 *   - Eq 4.3 is evaluated as written, left to right:
 *       u (1 - mu dt) + cx ((u[x+1] - 2u) + u[x-1]) + cy (...) + cz (...)
 *     with (1 - mu dt) and c = (nu dt) / (dx dx) computed once;
 *   - the gradient is the central difference (u[+1] - u[-1]) / (2 dx) per
 *     axis at the cell's voxel (zero beyond the grid), normalised to unit
 *     length (no move where it vanishes); the new coordinate is clamped to
 *     the space;
 *   - per iteration, from the state at its start: every cell takes its
 *     chemotaxis step on the start-of-iteration concentrations and secretes
 *     at its start-of-iteration position; the secretions of the cells of one
 *     voxel are added in one sum (k cells: k times the quantity); then the
 *     concentrations take one step of Eq 4.3.
 *
 * Parity pins: every function here is pinned by a "not gpu" test against
 * the exact discrete eigenmodes of Eq 4.3, the analytic point-source
 * solution of the diffusion equation (Fig 4.9), closed forms of decay and
 * secretion, exact gradients of linear fields, and mass balance.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double lo, space;     /* cubic space [lo, lo + space]^3 */
    int32_t resolution;   /* grid points per axis */
    int32_t n_substances;
    double diffusion;     /* nu */
    double decay;         /* mu */
    double dt;
    double secretion;     /* quantity per cell and iteration */
    double gradient_weight;
} orc_soma_params;

static double at(const double *u, int64_t R, int64_t x, int64_t y, int64_t z)
{
    if (x < 0 || y < 0 || z < 0 || x >= R || y >= R || z >= R) return 0.0;
    return u[x + R * (y + R * z)];
}

/* One step of Eq 4.3 on one substance: u_out from u_in (R^3 points). */
void orc_diffusion_step(const double *u_in, double *u_out, const orc_soma_params *p)
{
    const int64_t R = p->resolution;
    const double dx = p->space / (double)R;
    const double keep = 1.0 - p->decay * p->dt;
    const double c = p->diffusion * p->dt / (dx * dx);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < R; ++z)
        for (int64_t y = 0; y < R; ++y)
            for (int64_t x = 0; x < R; ++x) {
                const double u = u_in[x + R * (y + R * z)];
                double v = u * keep;
                v = v + c * ((at(u_in, R, x + 1, y, z) - 2.0 * u) + at(u_in, R, x - 1, y, z));
                v = v + c * ((at(u_in, R, x, y + 1, z) - 2.0 * u) + at(u_in, R, x, y - 1, z));
                v = v + c * ((at(u_in, R, x, y, z + 1) - 2.0 * u) + at(u_in, R, x, y, z - 1));
                u_out[x + R * (y + R * z)] = v;
            }
}

static int64_t voxel_axis(double v, const orc_soma_params *p)
{
    const double dx = p->space / (double)p->resolution;
    double q = floor((v - p->lo) / dx);
    if (q < 0.0) return 0;
    if (q > (double)(p->resolution - 1)) return p->resolution - 1;
    return (int64_t)q;
}

/* Voxel index of a position. */
int64_t orc_soma_voxel(double x, double y, double z, const orc_soma_params *p)
{
    const int64_t R = p->resolution;
    return voxel_axis(x, p) + R * (voxel_axis(y, p) + R * voxel_axis(z, p));
}

/* Algorithm 7's gradient at the voxel of a position (not normalised). */
void orc_soma_gradient(const double *u, double x, double y, double z, const orc_soma_params *p, double g[3])
{
    const int64_t R = p->resolution;
    const double dx = p->space / (double)R;
    const int64_t i = voxel_axis(x, p), j = voxel_axis(y, p), k = voxel_axis(z, p);
    g[0] = (at(u, R, i + 1, j, k) - at(u, R, i - 1, j, k)) / (2.0 * dx);
    g[1] = (at(u, R, i, j + 1, k) - at(u, R, i, j - 1, k)) / (2.0 * dx);
    g[2] = (at(u, R, i, j, k + 1) - at(u, R, i, j, k - 1)) / (2.0 * dx);
}

static double clamp_space(double v, const orc_soma_params *p)
{
    const double hi = p->lo + p->space;
    return v < p->lo ? p->lo : (v > hi ? hi : v);
}

/* One iteration: n cells (positions x, y, z, substance index type[i]) and
 * the n_substances grids u (each R^3, contiguous, substance after
 * substance), updated in place.  Returns 0, or -1 when memory runs out. */
int orc_soma_step(int64_t n, double *x, double *y, double *z, const int32_t *type, double *u,
                  const orc_soma_params *p)
{
    const int64_t R = p->resolution, V = R * R * R;
    const int64_t total = V * (int64_t)p->n_substances;
    double *un = (double *)malloc(sizeof(double) * (size_t)(total > 0 ? total : 1));
    int64_t *cnt = (int64_t *)calloc((size_t)(total > 0 ? total : 1), sizeof(int64_t));
    int64_t *vox = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!un || !cnt || !vox) { free(un); free(cnt); free(vox); return -1; }

    /* Algorithm 6 (where) and Algorithm 7 (chemotaxis), from the start-of-iteration state */
    for (int64_t i = 0; i < n; ++i) {
        const double *us = u + V * (int64_t)type[i];
        vox[i] = V * (int64_t)type[i] + orc_soma_voxel(x[i], y[i], z[i], p);
        double g[3];
        orc_soma_gradient(us, x[i], y[i], z[i], p, g);
        const double norm = sqrt(fma(g[2], g[2], fma(g[1], g[1], g[0] * g[0])));
        if (norm > 0.0) {
            x[i] = clamp_space(x[i] + (g[0] / norm) * p->gradient_weight, p);
            y[i] = clamp_space(y[i] + (g[1] / norm) * p->gradient_weight, p);
            z[i] = clamp_space(z[i] + (g[2] / norm) * p->gradient_weight, p);
        }
    }
    /* Algorithm 6: the secretions of one voxel in one sum */
    for (int64_t i = 0; i < n; ++i) cnt[vox[i]] += 1;
    for (int64_t v = 0; v < total; ++v)
        if (cnt[v] > 0) u[v] = u[v] + (double)cnt[v] * p->secretion;
    /* Eq 4.3 on every substance */
    for (int32_t s = 0; s < p->n_substances; ++s) orc_diffusion_step(u + V * s, un + V * s, p);
    memcpy(u, un, sizeof(double) * (size_t)total);
    free(un); free(cnt); free(vox);
    return 0;
}
