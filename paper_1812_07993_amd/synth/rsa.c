/*
 * rsa.c -- random sequential addition of points in a periodic box with a
 * minimum pair distance, for building synthetic vapour configurations.
 *
 * Input tooling only: no force, energy or integration arithmetic here.  The
 * caller supplies the candidate points (drawn from a seeded generator), the
 * fixed obstacle points (wall sites) and the exclusion distance; this file
 * accepts a candidate iff its minimum-image distance to every obstacle and
 * to every point accepted so far is at least dmin.  Candidates are taken in
 * the order given, so the result is a pure function of the inputs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    double box[3];
    double dmin2;
    int32_t nc[3];
    double inv[3];
    int32_t *head; /* per grid cell: first point, -1 if empty */
    int32_t *next; /* per point: next point in the same cell */
    double *pts;   /* [cap][3] obstacles first, then accepted points */
    int64_t n, cap;
} rsa_grid;

static int32_t cell_of(const rsa_grid *g, const double *p, int32_t *ck)
{
    for (int k = 0; k < 3; ++k) {
        int32_t c = (int32_t)floor(p[k] * g->inv[k]);
        if (c < 0) c = 0;
        if (c >= g->nc[k]) c = g->nc[k] - 1;
        ck[k] = c;
    }
    return ck[0] + g->nc[0] * (ck[1] + g->nc[1] * ck[2]);
}

static void insert(rsa_grid *g, const double *p)
{
    int32_t ck[3];
    int64_t i = g->n++;
    g->pts[3 * i] = p[0];
    g->pts[3 * i + 1] = p[1];
    g->pts[3 * i + 2] = p[2];
    int32_t c = cell_of(g, p, ck);
    g->next[i] = g->head[c];
    g->head[c] = (int32_t)i;
}

static int clear_of_all(const rsa_grid *g, const double *p)
{
    int32_t ck[3];
    cell_of(g, p, ck);
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int32_t cx = (ck[0] + dx + g->nc[0]) % g->nc[0];
                int32_t cy = (ck[1] + dy + g->nc[1]) % g->nc[1];
                int32_t cz = (ck[2] + dz + g->nc[2]) % g->nc[2];
                int32_t c = cx + g->nc[0] * (cy + g->nc[1] * cz);
                for (int32_t q = g->head[c]; q >= 0; q = g->next[q]) {
                    double r2 = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        double d = p[k] - g->pts[3 * q + k];
                        d -= g->box[k] * nearbyint(d / g->box[k]);
                        r2 += d * d;
                    }
                    if (r2 < g->dmin2) return 0;
                }
            }
    return 1;
}

/* Create a grid for up to cap points (obstacles plus accepted). */
void *rsa_create(const double *box, double dmin, int64_t cap)
{
    rsa_grid *g = (rsa_grid *)calloc(1, sizeof(rsa_grid));
    if (!g) return NULL;
    int64_t ncell = 1;
    for (int k = 0; k < 3; ++k) {
        g->box[k] = box[k];
        int32_t n = (int32_t)floor(box[k] / dmin);
        if (n < 3) n = 3;
        g->nc[k] = n;
        g->inv[k] = n / box[k];
        ncell *= n;
    }
    g->dmin2 = dmin * dmin;
    g->cap = cap;
    g->head = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncell);
    g->next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    g->pts = (double *)malloc(sizeof(double) * 3 * (size_t)(cap > 0 ? cap : 1));
    if (!g->head || !g->next || !g->pts) {
        free(g->head);
        free(g->next);
        free(g->pts);
        free(g);
        return NULL;
    }
    for (int64_t c = 0; c < ncell; ++c) g->head[c] = -1;
    return g;
}

void rsa_destroy(void *h)
{
    rsa_grid *g = (rsa_grid *)h;
    if (!g) return;
    free(g->head);
    free(g->next);
    free(g->pts);
    free(g);
}

/* Insert fixed obstacle points without any distance test. */
int64_t rsa_add_obstacles(void *h, const double *p, int64_t m)
{
    rsa_grid *g = (rsa_grid *)h;
    for (int64_t i = 0; i < m && g->n < g->cap; ++i) insert(g, p + 3 * i);
    return g->n;
}

/* Try candidates in order; accepted ones are appended to out (at most
 * want).  Returns the number accepted; *used receives how many candidates
 * were consumed (all of them unless want was reached). */
int64_t rsa_try(void *h, const double *cand, int64_t m, double *out,
                int64_t want, int64_t *used)
{
    rsa_grid *g = (rsa_grid *)h;
    int64_t got = 0, i = 0;
    for (; i < m && got < want && g->n < g->cap; ++i) {
        const double *p = cand + 3 * i;
        if (!clear_of_all(g, p)) continue;
        insert(g, p);
        out[3 * got] = p[0];
        out[3 * got + 1] = p[1];
        out[3 * got + 2] = p[2];
        ++got;
    }
    *used = i;
    return got;
}
