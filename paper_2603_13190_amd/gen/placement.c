/* Acceptance loop of the input generator's random sequential addition of
 * particles (specimen.place_particles), as plain host C.
 *
 * Accepted particles live in a uniform hash grid of cubic cells of edge
 * `cell` (keys floor(x / cell) per axis).  A candidate centre x with radius
 * r is accepted when, for every accepted particle p in the 27 cells around
 * x's cell, |x - x_p|^2 >= ((r + r_p)(1 + gap))^2.  The candidates of one
 * particle are tried in order and the first accepted one is kept.  The
 * arithmetic is the generator's own, operation for operation and in the
 * same order (built without floating-point contraction), so the accepted
 * set is the one the generator's Python loop produces.
 *
 * Input-generator code: it computes none of the LDPM step and is linked
 * into neither the solver library nor the oracle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    double cell;
    int64_t nx, ny, nz;  /* cells per axis; keys outside [0, n) hold nothing */
    int64_t *head;       /* [nx*ny*nz] first particle of each cell, or -1 */
    int64_t *next;       /* [cap] next particle of the same cell, or -1 */
    double *x;           /* [cap][3] accepted centres */
    double *r;           /* [cap] accepted radii */
    int64_t n, cap;
} place_grid;

static int64_t key1(double v, double cell) { return (int64_t)floor(v / cell); }

void place_free(place_grid *g)
{
    if (!g) return;
    free(g->head);
    free(g->next);
    free(g->x);
    free(g->r);
    free(g);
}

/* grid covering [0, lx] x [0, ly] x [0, lz] for at most cap particles;
 * NULL on bad arguments or allocation failure */
place_grid *place_create(double cell, double lx, double ly, double lz, int64_t cap)
{
    if (!(cell > 0.0) || !(lx > 0.0) || !(ly > 0.0) || !(lz > 0.0) || cap < 0) return NULL;
    place_grid *g = (place_grid *)calloc(1, sizeof(place_grid));
    if (!g) return NULL;
    g->cell = cell;
    g->nx = key1(lx, cell) + 1;
    g->ny = key1(ly, cell) + 1;
    g->nz = key1(lz, cell) + 1;
    g->cap = cap;
    const int64_t nc = g->nx * g->ny * g->nz;
    g->head = (int64_t *)malloc((size_t)nc * sizeof(int64_t));
    g->next = (int64_t *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(int64_t));
    g->x = (double *)malloc((size_t)(cap > 0 ? cap : 1) * 3 * sizeof(double));
    g->r = (double *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(double));
    if (!g->head || !g->next || !g->x || !g->r) {
        place_free(g);
        return NULL;
    }
    for (int64_t c = 0; c < nc; c++) g->head[c] = -1;
    return g;
}

static int fits(const place_grid *g, const double *x, double r, double gap)
{
    const int64_t kx = key1(x[0], g->cell), ky = key1(x[1], g->cell), kz = key1(x[2], g->cell);
    for (int64_t i = kx - 1; i <= kx + 1; i++) {
        if (i < 0 || i >= g->nx) continue;
        for (int64_t j = ky - 1; j <= ky + 1; j++) {
            if (j < 0 || j >= g->ny) continue;
            for (int64_t k = kz - 1; k <= kz + 1; k++) {
                if (k < 0 || k >= g->nz) continue;
                for (int64_t p = g->head[(i * g->ny + j) * g->nz + k]; p >= 0; p = g->next[p]) {
                    const double *y = g->x + 3 * p;
                    const double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
                    const double dd = d0 * d0 + d1 * d1 + d2 * d2;
                    const double lim = (r + g->r[p]) * (1.0 + gap);
                    if (dd < lim * lim) return 0;
                }
            }
        }
    }
    return 1;
}

/* Try the n candidates cand[n][3] in order; the first that fits is added
 * and its index returned.  -1: none fits; -2: the grid is full or the
 * candidate lies outside the grid's box. */
int64_t place_try(place_grid *g, const double *cand, int64_t n, double r, double gap)
{
    for (int64_t c = 0; c < n; c++) {
        const double *x = cand + 3 * c;
        if (!fits(g, x, r, gap)) continue;
        const int64_t kx = key1(x[0], g->cell), ky = key1(x[1], g->cell), kz = key1(x[2], g->cell);
        if (g->n >= g->cap || kx < 0 || kx >= g->nx || ky < 0 || ky >= g->ny || kz < 0 || kz >= g->nz)
            return -2;
        const int64_t p = g->n++;
        g->x[3 * p] = x[0];
        g->x[3 * p + 1] = x[1];
        g->x[3 * p + 2] = x[2];
        g->r[p] = r;
        /* prepended to the cell's list: the order of the checks does not change the result */
        const int64_t cidx = (kx * g->ny + ky) * g->nz + kz;
        g->next[p] = g->head[cidx];
        g->head[cidx] = p;
        return c;
    }
    return -1;
}
