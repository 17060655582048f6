/*
 * oracle.c -- plain, slow, FP64 reference for the pore molecular-dynamics
 * hot path (Korenkov, Nikonov, Popovicova, "Molecular dynamic simulation of
 * water vapor interaction with various types of pores using hybrid computing
 * structures", arXiv:1812.07993).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * measured against.  It is loaded by the tests, by the smoke check and by
 * the benchmark's CPU-baseline leg, and by nothing else.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes, in the paper's terms:
 *   - Newton's equations m_i d^2 r_i / dt^2 = f_i            (Sec. 2, eq. 1)
 *   - f_i = -dU/dr_i + f_i^ex, with U a sum of Lennard-Jones pair terms and
 *     f^ex the field of fixed pore-wall atoms                (Sec. 2, eq. 2)
 *   - velocity Verlet in the order of the paper's GPU functions F2, F1, F3
 *     (Sec. 3, the F2 update of r and the first half of v; F1 the
 *     acceleration from r(t+dt); F3 the second half of v).
 *   Every pair is visited (O(N^2)), as in the paper's F1 ("interactions
 *   between all particles", Sec. 3).  A pair contributes only below the
 *   cutoff, which is part of the model here, not an approximation.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - 12-6 form u(r) = 4 eps [(sig/r)^12 - (sig/r)^6] (Sec. 2 names the LJ
 *     potential and its sigma, epsilon but does not write the form);
 *   - truncated at r_c (strict r < r_c) and shifted so that u(r_c) = 0; the
 *     force is not shifted;
 *   - vapour-wall pairs use (sig_w, eps_w) with the same r_c; wall-wall pairs
 *     are never evaluated; walls never move;
 *   - minimum-image periodic boundaries on all three axes; positions are
 *     wrapped into [0, L) after each drift;
 *   - Berendsen factor lambda = sqrt(1 + (dt/tau)(t0/T - 1)) with
 *     T = 2K / (3N - 3), applied after F3 (the paper gives the rise time and
 *     the per-step scaling, not the formula).
 *
 * Determinism: every per-particle sum runs over partners in ascending index
 * order (vapour first, then walls), and every total is summed serially in
 * ascending particle order, so results do not depend on the OpenMP thread
 * count.
 *
 * Parity status: the pair term, the force sum, the integrator, the
 * Berendsen step, the virial sums, the wall lattice, the cell sort and the
 * pair sets are each pinned by tests against closed forms, invariants or
 * brute force.  Long-run physical observables
 * (adsorption, density profiles) are parity unpinned: the paper prints none.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Model parameters in reduced Lennard-Jones units. */
typedef struct {
    double box[3];
    double sigma, epsilon, mass, cutoff, dt;
    double sigma_wall, epsilon_wall;
} orc_params;

/* Pore description.  kind: 0 none (no walls), 1 plain slab, 2 cylinder,
 * 3 slit (two slabs), 4 cone, 5 ink-bottle. */
typedef struct {
    int32_t kind;
    int32_t pad_;
    double lattice_a;
    double slab_center_z;
    double slab_thickness;
    double r0, r1;
    double slit_gap;
} orc_pore;

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------------- */
/* Pair term                                                               */
/* ---------------------------------------------------------------------- */

/* Lennard-Jones pair at squared distance r2, truncated and shifted.
 * *u receives the pair energy, *w the scalar with force_on_i = w * (r_i - r_j),
 * i.e. w = -(1/r) du/dr = 24 eps (2 (s/r)^12 - (s/r)^6) / r^2. */
static void lj_pair(double r2, double sig, double eps, double rc,
                    double *u, double *w)
{
    if (r2 >= rc * rc) {
        *u = 0.0;
        *w = 0.0;
        return;
    }
    double s2 = (sig * sig) / r2;
    double s6 = s2 * s2 * s2;
    double s12 = s6 * s6;
    double c2 = (sig * sig) / (rc * rc);
    double c6 = c2 * c2 * c2;
    double c12 = c6 * c6;
    *u = 4.0 * eps * (s12 - s6) - 4.0 * eps * (c12 - c6);
    *w = 24.0 * eps * (2.0 * s12 - s6) / r2;
}

/* Exported for the pair-term pins: energy and w at one distance r. */
void orc_pair(double r, double sig, double eps, double rc, double *u, double *w)
{
    lj_pair(r * r, sig, eps, rc, u, w);
}

/* Minimum-image displacement a - b on a periodic box. */
static void min_image(const double *a, const double *b, const double *box,
                      double *d)
{
    for (int k = 0; k < 3; ++k) {
        double dk = a[k] - b[k];
        dk -= box[k] * nearbyint(dk / box[k]);
        d[k] = dk;
    }
}

/* ---------------------------------------------------------------------- */
/* Forces (eq. 2), all pairs                                               */
/* ---------------------------------------------------------------------- */

/* Force on one vapour atom i from every other vapour atom and every wall
 * atom; also its vapour-vapour energy over partners j > i and its
 * vapour-wall energy. */
static void force_on(int64_t i, int64_t nv, const double *xv, int64_t nw,
                     const double *xw, const orc_params *p, double *f,
                     double *pe_vv_upper, double *pe_vw)
{
    double fx = 0.0, fy = 0.0, fz = 0.0, evv = 0.0, evw = 0.0;
    const double *xi = xv + 3 * i;
    for (int64_t j = 0; j < nv; ++j) {
        if (j == i) continue;
        double d[3], u, w;
        min_image(xi, xv + 3 * j, p->box, d);
        lj_pair(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], p->sigma,
                p->epsilon, p->cutoff, &u, &w);
        fx += w * d[0];
        fy += w * d[1];
        fz += w * d[2];
        if (j > i) evv += u;
    }
    for (int64_t k = 0; k < nw; ++k) {
        double d[3], u, w;
        min_image(xi, xw + 3 * k, p->box, d);
        lj_pair(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], p->sigma_wall,
                p->epsilon_wall, p->cutoff, &u, &w);
        fx += w * d[0];
        fy += w * d[1];
        fz += w * d[2];
        evw += u;
    }
    f[0] = fx;
    f[1] = fy;
    f[2] = fz;
    *pe_vv_upper = evv;
    *pe_vw = evw;
}

/* Forces on all vapour atoms, F[nv][3]; total vapour-vapour energy
 * (each pair once) and vapour-wall energy.  If Fwall is not NULL it receives
 * the reaction force on each wall atom, Fwall[nw][3] (used only to check
 * Newton's third law). */
void orc_forces(int64_t nv, const double *xv, int64_t nw, const double *xw,
                const orc_params *p, double *F, double *pe_vv, double *pe_vw,
                double *Fwall)
{
    double *evv = (double *)malloc(sizeof(double) * (size_t)(nv > 0 ? nv : 1));
    double *evw = (double *)malloc(sizeof(double) * (size_t)(nv > 0 ? nv : 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nv; ++i)
        force_on(i, nv, xv, nw, xw, p, F + 3 * i, &evv[i], &evw[i]);
    double svv = 0.0, svw = 0.0;
    for (int64_t i = 0; i < nv; ++i) {
        svv += evv[i];
        svw += evw[i];
    }
    *pe_vv = svv;
    *pe_vw = svw;
    free(evv);
    free(evw);
    if (Fwall) {
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nw; ++k) {
            double gx = 0.0, gy = 0.0, gz = 0.0;
            for (int64_t i = 0; i < nv; ++i) {
                double d[3], u, w;
                min_image(xw + 3 * k, xv + 3 * i, p->box, d);
                lj_pair(d[0] * d[0] + d[1] * d[1] + d[2] * d[2],
                        p->sigma_wall, p->epsilon_wall, p->cutoff, &u, &w);
                gx += w * d[0];
                gy += w * d[1];
                gz += w * d[2];
            }
            Fwall[3 * k + 0] = gx;
            Fwall[3 * k + 1] = gy;
            Fwall[3 * k + 2] = gz;
        }
    }
}

/* Forces on a chosen subset of vapour atoms: F_sel[m][3] for atoms sel[0..m).
 * pe_sel[m] (if not NULL) receives each atom's share of the potential energy,
 * half of every vapour-vapour pair plus all of its vapour-wall pairs. */
void orc_forces_subset(int64_t nv, const double *xv, int64_t nw,
                       const double *xw, const orc_params *p, int64_t m,
                       const int64_t *sel, double *F_sel, double *pe_sel)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < m; ++s) {
        int64_t i = sel[s];
        double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
        const double *xi = xv + 3 * i;
        for (int64_t j = 0; j < nv; ++j) {
            if (j == i) continue;
            double d[3], u, w;
            min_image(xi, xv + 3 * j, p->box, d);
            lj_pair(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], p->sigma,
                    p->epsilon, p->cutoff, &u, &w);
            fx += w * d[0];
            fy += w * d[1];
            fz += w * d[2];
            e += 0.5 * u;
        }
        for (int64_t k = 0; k < nw; ++k) {
            double d[3], u, w;
            min_image(xi, xw + 3 * k, p->box, d);
            lj_pair(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], p->sigma_wall,
                    p->epsilon_wall, p->cutoff, &u, &w);
            fx += w * d[0];
            fy += w * d[1];
            fz += w * d[2];
            e += u;
        }
        F_sel[3 * s + 0] = fx;
        F_sel[3 * s + 1] = fy;
        F_sel[3 * s + 2] = fz;
        if (pe_sel) pe_sel[s] = e;
    }
}

/* ---------------------------------------------------------------------- */
/* Velocity Verlet (F2, F1, F3 of Sec. 3)                                  */
/* ---------------------------------------------------------------------- */

static double kinetic(int64_t nv, const double *v, double m)
{
    double s = 0.0;
    for (int64_t i = 0; i < nv; ++i)
        s += v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] +
             v[3 * i + 2] * v[3 * i + 2];
    return 0.5 * m * s;
}

/* Wrap one coordinate into [0, L). */
static double wrap(double x, double L)
{
    x -= L * floor(x / L);
    if (x >= L) x = 0.0;
    return x;
}

/* Advance the state by nsteps velocity-Verlet steps.
 *   x, v   [nv][3], updated in place;
 *   a      [nv][3], acceleration at the current x; if have_a == 0 it is
 *          computed first (a(0) before step 1), and on return it holds the
 *          acceleration at the final x;
 *   energies, if not NULL, receives rows (ke, pe_vv, pe_vw) for step 0 and
 *          for every step that is a multiple of every_k, then the last step
 *          if not already recorded; the number of rows is returned.
 * One step is:
 *   F2: r(t+dt) = r(t) + v(t) dt + a(t) dt^2 / 2,  v(t+dt/2) = v(t) + a(t) dt/2,
 *       then r is wrapped into the periodic box;
 *   F1: a(t+dt) = f(r(t+dt)) / m;
 *   F3: v(t+dt) = v(t+dt/2) + a(t+dt) dt/2;
 *   F4 (only if tau > 0; Berendsen thermostat, Sec. 2 and the F4 listing of
 *       Sec. 3): T = 2 K / (3 nv - 3) from the F3 velocities, then
 *       v <- lambda v with lambda = sqrt(1 + (dt / tau) (t0 / T - 1)).  The
 *       paper names the thermostat, its rise time tau and the scaling of
 *       every velocity by lambda(t) each step, but not the formula for
 *       lambda: this is Berendsen's weak-coupling factor.  The recorded
 *       kinetic energy of a step is the one the thermostat measured (before
 *       the scaling). */
int64_t orc_run(int64_t nv, double *x, double *v, double *a, int have_a,
                int64_t nw, const double *xw, const orc_params *p,
                int64_t nsteps, int64_t every_k, double *energies,
                double tau, double t0)
{
    double dt = p->dt, m = p->mass, evv = 0.0, evw = 0.0;
    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)(nv > 0 ? nv : 1));
    int64_t rows = 0;
    if (!have_a || energies) {
        orc_forces(nv, x, nw, xw, p, F, &evv, &evw, NULL);
        if (!have_a)
            for (int64_t q = 0; q < 3 * nv; ++q) a[q] = F[q] / m;
    }
    if (energies) {
        energies[0] = kinetic(nv, v, m);
        energies[1] = evv;
        energies[2] = evw;
        rows = 1;
    }
    for (int64_t n = 1; n <= nsteps; ++n) {
        for (int64_t i = 0; i < nv; ++i)
            for (int k = 0; k < 3; ++k) {
                int64_t q = 3 * i + k;
                x[q] = x[q] + v[q] * dt + 0.5 * a[q] * dt * dt;
                v[q] = v[q] + 0.5 * a[q] * dt;
                x[q] = wrap(x[q], p->box[k]);
            }
        orc_forces(nv, x, nw, xw, p, F, &evv, &evw, NULL);
        for (int64_t q = 0; q < 3 * nv; ++q) {
            a[q] = F[q] / m;
            v[q] = v[q] + 0.5 * a[q] * dt;
        }
        double ke = kinetic(nv, v, m);
        int record = energies && ((every_k > 0 && n % every_k == 0) || n == nsteps);
        if (record) {
            energies[3 * rows + 0] = ke;
            energies[3 * rows + 1] = evv;
            energies[3 * rows + 2] = evw;
            ++rows;
        }
        if (tau > 0.0) {
            double dof = nv > 1 ? 3.0 * (double)nv - 3.0 : 3.0;
            double T = 2.0 * ke / dof;
            double lam = sqrt(1.0 + (dt / tau) * (t0 / T - 1.0));
            for (int64_t q = 0; q < 3 * nv; ++q) v[q] = lam * v[q];
        }
    }
    free(F);
    return rows;
}

/* Virial sums of the pressure formula (Sec. 2): w_vv = sum over vapour
 * pairs i < j of r_ij . f_ij, with r_ij = r_i - r_j (minimum image) and f_ij
 * the force on i from j (positive for repulsion); w_vw = the same sum over
 * vapour-wall pairs, f the force on the vapour atom.  Pairs contribute only
 * inside the cutoff, like the forces.  The pressure reads
 * P = (2K + w_vv) / (3V): the paper writes the pair term with a minus sign,
 * which matches a force f(r) = du/dr; here f is the force itself.  Summed
 * serially in ascending index order. */
void orc_virial(int64_t nv, const double *xv, int64_t nw, const double *xw,
                const orc_params *p, double *wvv, double *wvw)
{
    double svv = 0.0, svw = 0.0;
    for (int64_t i = 0; i < nv; ++i) {
        for (int64_t j = i + 1; j < nv; ++j) {
            double d[3], u, w;
            min_image(xv + 3 * i, xv + 3 * j, p->box, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            lj_pair(r2, p->sigma, p->epsilon, p->cutoff, &u, &w);
            svv += w * r2;
        }
        for (int64_t k = 0; k < nw; ++k) {
            double d[3], u, w;
            min_image(xv + 3 * i, xw + 3 * k, p->box, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            lj_pair(r2, p->sigma_wall, p->epsilon_wall, p->cutoff, &u, &w);
            svw += w * r2;
        }
    }
    *wvv = svv;
    *wvw = svw;
}

/* ---------------------------------------------------------------------- */
/* Pore-wall lattice                                                       */
/* ---------------------------------------------------------------------- */

/* Pore radius at a layer whose centre is a height h above the slab's lower
 * face, for a slab of thickness t. */
static double pore_radius(const orc_pore *pp, double h, double t)
{
    switch (pp->kind) {
    case 2: /* cylinder */
        return pp->r0;
    case 4: /* cone: linear from r0 at the lower face to r1 at the upper */
        return pp->r0 + (pp->r1 - pp->r0) * (h / t);
    case 5: /* ink-bottle: neck r0 in the outer quarters, cavity r1 between */
        return (h < 0.25 * t || h >= 0.75 * t) ? pp->r0 : pp->r1;
    default: /* plain slab, slit: no hole */
        return 0.0;
    }
}

/* Enumerate one slab's sites on a simple cubic lattice of spacing a:
 * x = (i + 1/2) a, y = (j + 1/2) a over the whole periodic box, and
 * z = z_lo + (k + 1/2) a for the layers inside [z_lo, z_lo + t).  A site is
 * left out when its distance from the pore axis (x = Lx/2, y = Ly/2) is
 * strictly below the pore radius of its layer.  Order: layer, then y, then
 * x.  Writes at most cap sites; returns how many there are in total. */
static int64_t slab_sites(const orc_pore *pp, const double *box, double z_lo,
                          double t, double *out, int64_t n0, int64_t cap)
{
    double a = pp->lattice_a;
    int64_t nx = (int64_t)floor(box[0] / a + 0.5);
    int64_t ny = (int64_t)floor(box[1] / a + 0.5);
    int64_t nz = (int64_t)floor(t / a + 0.5);
    double cx = 0.5 * box[0], cy = 0.5 * box[1];
    int64_t n = n0;
    for (int64_t k = 0; k < nz; ++k) {
        double h = (k + 0.5) * a;
        double r = pore_radius(pp, h, t);
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double x = (i + 0.5) * a, y = (j + 0.5) * a;
                double dx = x - cx, dy = y - cy;
                if (dx * dx + dy * dy < r * r) continue;
                if (n < cap) {
                    out[3 * n + 0] = x;
                    out[3 * n + 1] = y;
                    out[3 * n + 2] = z_lo + h;
                }
                ++n;
            }
    }
    return n;
}

/* All wall sites of a pore, in canonical order.  Slab placement:
 *   plain slab, cylinder, cone, ink-bottle: one slab of thickness t centred
 *     at slab_center_z;
 *   slit: two slabs of thickness t whose facing surfaces are slit_gap apart,
 *     centred at slab_center_z (lower slab first);
 *   none: no sites. */
int64_t orc_wall_lattice(const orc_pore *pp, const double *box, double *out,
                         int64_t cap)
{
    double t = pp->slab_thickness, c = pp->slab_center_z;
    switch (pp->kind) {
    case 0:
        return 0;
    case 3: {
        int64_t n = slab_sites(pp, box, c - 0.5 * pp->slit_gap - t, t, out, 0, cap);
        return slab_sites(pp, box, c + 0.5 * pp->slit_gap, t, out, n, cap);
    }
    default:
        return slab_sites(pp, box, c - 0.5 * t, t, out, 0, cap);
    }
}

/* ---------------------------------------------------------------------- */
/* Cell binning and pair sets (integer work, compared bit for bit)         */
/* ---------------------------------------------------------------------- */

/* Stable counting sort of atoms into a grid of nc[0] x nc[1] x nc[2] cells.
 * Cell of an atom along axis k: floor(x_k * inv[k]) clamped to [0, nc[k]-1];
 * linear index cx + nc0 (cy + nc1 cz).  Outputs: cell[n], cell_start
 * [ncells + 1] (exclusive prefix of the counts) and perm[n] = the atom ids
 * in cell order, ascending id inside a cell. */
void orc_cell_sort(int64_t n, const double *x, const double *inv,
                   const int32_t *nc, int32_t *cell, int32_t *cell_start,
                   int32_t *perm)
{
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t ck[3];
        for (int k = 0; k < 3; ++k) {
            double q = floor(x[3 * i + k] * inv[k]);
            int32_t ci = (int32_t)q;
            if (q < 0.0) ci = 0;
            if (q > (double)(nc[k] - 1)) ci = nc[k] - 1;
            ck[k] = ci;
        }
        cell[i] = ck[0] + nc[0] * (ck[1] + nc[1] * ck[2]);
        cell_start[cell[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
    int32_t *fill = (int32_t *)calloc((size_t)(ncell > 0 ? ncell : 1), sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = cell[i];
        perm[cell_start[c] + fill[c]] = (int32_t)i;
        fill[c] += 1;
    }
    free(fill);
}

/* Every vapour-vapour pair (i < j) and vapour-wall pair (i, w) whose
 * minimum-image squared distance is strictly below rc^2, in lexicographic
 * order.  Writes at most cap pairs of each kind; returns both totals. */
void orc_pairs(int64_t nv, const double *xv, int64_t nw, const double *xw,
               const double *box, double rc, int64_t cap, int32_t *vv,
               int64_t *n_vv, int32_t *vw, int64_t *n_vw)
{
    int64_t a = 0, b = 0;
    for (int64_t i = 0; i < nv; ++i) {
        for (int64_t j = i + 1; j < nv; ++j) {
            double d[3];
            min_image(xv + 3 * i, xv + 3 * j, box, d);
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rc * rc) {
                if (a < cap) {
                    vv[2 * a] = (int32_t)i;
                    vv[2 * a + 1] = (int32_t)j;
                }
                ++a;
            }
        }
        for (int64_t k = 0; k < nw; ++k) {
            double d[3];
            min_image(xv + 3 * i, xw + 3 * k, box, d);
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rc * rc) {
                if (b < cap) {
                    vw[2 * b] = (int32_t)i;
                    vw[2 * b + 1] = (int32_t)k;
                }
                ++b;
            }
        }
    }
    *n_vv = a;
    *n_vw = b;
}

/* All-pairs Lennard-Jones forces as the paper's force function states them
 * (Sec. 3): every pair i != j contributes, with no cutoff and no shift;
 * r_ij = x_i - x_j by the minimum image along each axis with box[k] > 0.
 * f_i = sum_j 24 eps (2 (s/r)^12 - (s/r)^6) r_ij / r^2; u_i = sum_j u(r_ij) / 2
 * with u(r) = 4 eps ((s/r)^12 - (s/r)^6); *e = sum_i u_i. */
void orc_allpairs(int64_t n, const double *x, const double *box, double eps, double sigma,
                  double *f, double *u, double *e)
{
    double tot = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0}, ui = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            for (int k = 0; k < 3; ++k) {
                d[k] = x[3 * i + k] - x[3 * j + k];
                if (box[k] > 0.0) d[k] -= box[k] * nearbyint(d[k] / box[k]);
            }
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const double sr2 = sigma * sigma / r2, sr6 = sr2 * sr2 * sr2;
            const double w = 24.0 * eps * sr6 * (2.0 * sr6 - 1.0) / r2;
            for (int k = 0; k < 3; ++k) fi[k] += w * d[k];
            ui += 4.0 * eps * sr6 * (sr6 - 1.0);
        }
        for (int k = 0; k < 3; ++k) f[3 * i + k] = fi[k];
        u[i] = 0.5 * ui;
        tot += u[i];
    }
    *e = tot;
}

/* ---------------------------------------------------------------------- */
/* The paper's pore model (Secs. 4-5): all-pairs forces, reflecting pore  */
/* walls, periodic outer space, in two or three dimensions                */
/* ---------------------------------------------------------------------- */

/* Geometry of the model, in the reading fixed for this repository (the
 * paper describes it in words and one figure; the reflection rule itself is
 * in a reference that is not at hand, so specular reflection is taken):
 *   pore   P = [0, lx) x [0, ly] (x [0, lz] in 3D): walls at x = 0, y = 0,
 *          y = ly (and z = 0, z = lz) reflect specularly; the face x = lx
 *          is open (the pore mouth, 0 <= y < ly, 0 <= z < lz);
 *   outer  O = [lx, (k+1) lx) x [-k ly, (k+1) ly) (x [-k lz, (k+1) lz)):
 *          periodic along y (and z) with period (2k+1) ly (lz) and along x
 *          with period k lx, except that a particle crossing x = lx
 *          leftwards inside the mouth (0 <= y < ly, 0 <= z < lz) enters the
 *          pore.  The outer space is k (2k+1)^(d-1) pore volumes: 21 for
 *          the 2D model's k = 3, 9 for the 3D model's k = 1 (Secs. 4, 5).
 * A particle belongs to the pore iff x < lx. */
typedef struct {
    int32_t dim;  /* 2 or 3 */
    int32_t pad_;
    double lx, ly, lz, k;
    double sigma, epsilon, mass, dt;
    double tau, t0; /* Berendsen thermostat (tau > 0), else NVE */
} orc_pm_model;

/* All-pairs forces in d dimensions with plain differences (no images: the
 * model's domain is not a torus): f_i = sum_j 24 eps (2 s^12 - s^6) r_ij / r^2
 * with s = sigma / r, per-atom energy shares u_i = sum_j u(r_ij) / 2 and,
 * if w is not NULL, per-atom virial shares w_i = sum_j r_ij . f_ij / 2 (the
 * pair term of the pressure formula of Sec. 2, split equally between the
 * two molecules).  Returns the total energy, summed in ascending atom
 * order. */
static double pm_forces(int d, int64_t n, const double *x, double sig, double eps, double *f,
                        double *u, double *w)
{
    double tot = 0.0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0}, ui = 0.0, wi = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dd[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
            for (int k = 0; k < d; ++k) {
                dd[k] = x[d * i + k] - x[d * j + k];
                r2 += dd[k] * dd[k];
            }
            const double sr2 = sig * sig / r2, sr6 = sr2 * sr2 * sr2;
            const double w = 24.0 * eps * sr6 * (2.0 * sr6 - 1.0) / r2;
            for (int k = 0; k < d; ++k) fi[k] += w * dd[k];
            ui += 4.0 * eps * sr6 * (sr6 - 1.0);
            wi += w * r2;
        }
        for (int k = 0; k < d; ++k) f[d * i + k] = fi[k];
        u[i] = 0.5 * ui;
        if (w) w[i] = 0.5 * wi;
    }
    for (int64_t i = 0; i < n; ++i) tot += u[i];
    return tot;
}

void orc_pm_forces(const orc_pm_model *m, int64_t n, const double *x, double *f, double *u,
                   double *e)
{
    *e = pm_forces(m->dim, n, x, m->sigma, m->epsilon, f, u, NULL);
}

/* Carry one particle along the straight drift of one step, p -> p + dl
 * (dl = v dt + a dt^2 / 2, the paper's F2), through the model's boundaries:
 * the segment is followed event by event, each event being the first plane
 * the remaining segment crosses:
 *   in the pore:  a wall plane (x = 0; y = 0 or ly; z = 0 or lz): the
 *                 particle stops on the plane, the normal components of the
 *                 remaining displacement and of v change sign (specular
 *                 reflection); the mouth plane x = lx crossed rightwards:
 *                 the particle passes into the outer space;
 *   in the outer: x = (k+1) lx crossed rightwards: the particle reappears at
 *                 x = lx; x = lx crossed leftwards: inside the mouth it
 *                 passes into the pore, elsewhere it reappears at
 *                 x = (k+1) lx; y (z) leaving [-k l, (k+1) l): it reappears
 *                 on the opposite face.
 * Ties between planes go to the lowest axis first.  Returns the number of
 * wall reflections. */
int orc_pm_trace(const orc_pm_model *m, double *p, const double *dl_in, double *v)
{
    const int d = m->dim;
    const double L[3] = {m->lx, m->ly, m->lz};
    double dl[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < d; ++k) dl[k] = dl_in[k];
    int in_pore = p[0] < m->lx, refl = 0;
    for (int it = 0; it < 64; ++it) {
        /* earliest plane crossing of the remaining segment, t in [0, 1] */
        double tb = 2.0;
        int ax = -1, kind = 0; /* kind: 1 reflect, 2 mouth out, 3 wrap x right,
                                  4 cross x = lx leftwards, 5 wrap y/z */
        double plane = 0.0;
        for (int k = 0; k < d; ++k) {
            if (dl[k] == 0.0) continue;
            double w;
            int kd;
            if (in_pore) {
                if (k == 0) {
                    if (dl[0] < 0.0) { w = 0.0; kd = 1; }
                    else { w = m->lx; kd = 2; }
                } else {
                    w = dl[k] < 0.0 ? 0.0 : L[k];
                    kd = 1;
                }
            } else {
                if (k == 0) {
                    if (dl[0] > 0.0) { w = (m->k + 1.0) * m->lx; kd = 3; }
                    else { w = m->lx; kd = 4; }
                } else {
                    w = dl[k] < 0.0 ? -m->k * L[k] : (m->k + 1.0) * L[k];
                    kd = 5;
                }
            }
            /* a segment ending exactly on a plane is an event only where the
             * plane is an excluded upper face (the outer space's periodic
             * ranges are half-open); the pore is closed in y and z */
            const int excl = !in_pore && dl[k] > 0.0;
            const double t = (w - p[k]) / dl[k];
            if ((t < 1.0 || (excl && t <= 1.0)) && t < tb) {
                tb = t < 0.0 ? 0.0 : t;
                ax = k;
                kind = kd;
                plane = w;
            }
        }
        if (ax < 0) {
            for (int k = 0; k < d; ++k) p[k] += dl[k];
            return refl;
        }
        for (int k = 0; k < d; ++k) {
            if (k == ax) {
                p[k] = plane;
            } else {
                p[k] += tb * dl[k];
            }
            dl[k] *= (1.0 - tb);
        }
        switch (kind) {
        case 1:
            dl[ax] = -dl[ax];
            v[ax] = -v[ax];
            ++refl;
            break;
        case 2:
            in_pore = 0;
            break;
        case 3:
            p[0] = m->lx;
            break;
        case 4: {
            int mouth = p[1] >= 0.0 && p[1] < m->ly;
            if (d == 3) mouth = mouth && p[2] >= 0.0 && p[2] < m->lz;
            if (mouth)
                in_pore = 1;
            else
                p[0] = (m->k + 1.0) * m->lx;
            break;
        }
        case 5:
            p[ax] = dl[ax] < 0.0 ? (m->k + 1.0) * L[ax] : -m->k * L[ax];
            break;
        }
    }
    return -1; /* more events than any step can hold: not a valid drift */
}

/* Advance n particles of the pore model by nsteps velocity-Verlet steps:
 *   F2: dl = v dt + a dt^2 / 2, v <- v + a dt / 2, the particle carried
 *       along dl by orc_pm_trace;
 *   F1: a = f / m from the all-pairs forces at the new positions;
 *   F3: v <- v + a dt / 2;
 *   F4 (tau > 0): v <- lambda v, lambda = sqrt(1 + (dt / tau) (t0 / T - 1)),
 *       T = 2 K / (d n) from the F3 velocities (the walls break momentum
 *       conservation, so every degree of freedom counts).
 * x, v: [n][d], updated in place.  rec, if not NULL, receives rows (step,
 * ke, pe, n_pore, reflections so far, pressure in the pore) for step 0,
 * every step that is a multiple of every, and the last step; returns the
 * rows written, or -1 if a drift could not be traced.
 * Pressure in the pore (Sec. 2: the pore volume V, the doubled kinetic
 * energy and the pair virial, in d dimensions):
 *   P = (2 K_pore + W_pore) / (d V),  V = lx ly (lz),
 * K_pore the kinetic energy (after F3) of the molecules in the pore and
 * W_pore the sum of their virial shares (every pair's r_ij . f_ij split
 * equally between its molecules, f_ij the force on i from j; the sign of
 * the printed formula fits the other convention, f = dU/dr). */
int64_t orc_pm_run(const orc_pm_model *m, int64_t n, double *x, double *v, int64_t nsteps,
                   int64_t every, double *rec)
{
    const int d = m->dim;
    const double dt = m->dt, ms = m->mass;
    double *f = (double *)malloc(sizeof(double) * (size_t)(d * (n > 0 ? n : 1)));
    double *u = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *a = (double *)malloc(sizeof(double) * (size_t)(d * (n > 0 ? n : 1)));
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    const double vol = d == 3 ? m->lx * m->ly * m->lz : m->lx * m->ly;
    int64_t rows = 0, refl = 0;
    double pe = pm_forces(d, n, x, m->sigma, m->epsilon, f, u, w);
    for (int64_t q = 0; q < d * n; ++q) a[q] = f[q] / ms;
    for (int64_t s = 0; s <= nsteps; ++s) {
        if (s > 0) {
            for (int64_t i = 0; i < n; ++i) {
                double p[3] = {0.0, 0.0, 0.0}, dl[3] = {0.0, 0.0, 0.0}, vv[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < d; ++k) {
                    p[k] = x[d * i + k];
                    dl[k] = v[d * i + k] * dt + 0.5 * a[d * i + k] * dt * dt;
                    vv[k] = v[d * i + k] + 0.5 * a[d * i + k] * dt;
                }
                const int r = orc_pm_trace(m, p, dl, vv);
                if (r < 0) {
                    rows = -1;
                    goto out;
                }
                refl += r;
                for (int k = 0; k < d; ++k) {
                    x[d * i + k] = p[k];
                    v[d * i + k] = vv[k];
                }
            }
            pe = pm_forces(d, n, x, m->sigma, m->epsilon, f, u, w);
            for (int64_t q = 0; q < d * n; ++q) {
                a[q] = f[q] / ms;
                v[q] += 0.5 * a[q] * dt;
            }
        }
        double ke = 0.0, kp = 0.0, wp = 0.0;
        int64_t np = 0;
        for (int64_t i = 0; i < n; ++i) {
            double s2 = 0.0;
            for (int k = 0; k < d; ++k) s2 += v[d * i + k] * v[d * i + k];
            ke += 0.5 * ms * s2;
            if (x[d * i] < m->lx) {
                ++np;
                kp += 0.5 * ms * s2;
                wp += w[i];
            }
        }
        if (rec && (s == 0 || s == nsteps || (every > 0 && s % every == 0))) {
            rec[6 * rows + 0] = (double)s;
            rec[6 * rows + 1] = ke;
            rec[6 * rows + 2] = pe;
            rec[6 * rows + 3] = (double)np;
            rec[6 * rows + 4] = (double)refl;
            rec[6 * rows + 5] = (2.0 * kp + wp) / ((double)d * vol);
            ++rows;
        }
        if (s > 0 && m->tau > 0.0 && n > 0) {
            const double T = 2.0 * ke / ((double)d * (double)n);
            const double lam = sqrt(1.0 + (dt / m->tau) * (m->t0 / T - 1.0));
            for (int64_t q = 0; q < d * n; ++q) v[q] *= lam;
        }
    }
out:
    free(f);
    free(u);
    free(a);
    free(w);
    return rows;
}

/* ---------------------------------------------------------------------- */
/* Pressure in the pore of the cell-list workloads (Sec. 2)               */
/* ---------------------------------------------------------------------- */

/* The pore's void, a continuous region (the reading fixed for this
 * repository: the hole cut through the slab, not the lattice sites):
 *   cylinder, cone, ink-bottle: z in [z_lo, z_lo + t) of the slab and
 *     (x - Lx/2)^2 + (y - Ly/2)^2 < r(z)^2, with r(z) the hole's radius at
 *     that height (the cone's radius linear in z from r0 at z_lo to r1 at
 *     z_lo + t; the ink-bottle's neck r0 where z - z_lo < t/4 or >= 3t/4,
 *     its cavity r1 between);
 *   slit: the gap between the two slabs, z in [c - gap/2, c + gap/2);
 *   none: the whole box.  A plain slab has no pore.
 * Returns 1 if the point lies in the pore. */
static int in_pore(const orc_pore *pp, const double *box, const double *p)
{
    const double t = pp->slab_thickness, c = pp->slab_center_z;
    if (pp->kind == 0) return 1;
    if (pp->kind == 1) return 0;
    if (pp->kind == 3) return p[2] >= c - 0.5 * pp->slit_gap && p[2] < c + 0.5 * pp->slit_gap;
    const double z_lo = c - 0.5 * t, h = p[2] - z_lo;
    if (h < 0.0 || h >= t) return 0;
    double r;
    if (pp->kind == 2)
        r = pp->r0;
    else if (pp->kind == 4)
        r = pp->r0 + (pp->r1 - pp->r0) * (h / t);
    else
        r = (h < 0.25 * t || h >= 0.75 * t) ? pp->r0 : pp->r1;
    const double dx = p[0] - 0.5 * box[0], dy = p[1] - 0.5 * box[1];
    return dx * dx + dy * dy < r * r;
}

/* Volume of that region: pi r^2 t (cylinder), the frustum
 * pi t (r0^2 + r0 r1 + r1^2) / 3 (cone), pi (t/2) (r0^2 + r1^2) (ink-bottle:
 * two neck quarters and the cavity half), Lx Ly gap (slit), Lx Ly Lz (none);
 * 0 for a plain slab. */
double orc_pore_volume(const orc_pore *pp, const double *box)
{
    const double t = pp->slab_thickness, pi = 3.14159265358979323846;
    switch (pp->kind) {
    case 0: return box[0] * box[1] * box[2];
    case 2: return pi * pp->r0 * pp->r0 * t;
    case 3: return box[0] * box[1] * pp->slit_gap;
    case 4: return pi * t * (pp->r0 * pp->r0 + pp->r0 * pp->r1 + pp->r1 * pp->r1) / 3.0;
    case 5: return pi * 0.5 * t * (pp->r0 * pp->r0 + pp->r1 * pp->r1);
    default: return 0.0;
    }
}

/* Pressure in the pore by the formula of Sec. 2 with V the pore volume:
 *   P = (2 K_pore + W_pore) / (3 V),
 * K_pore the kinetic energy of the vapour molecules in the pore and W_pore
 * their shares of the vapour pair virials (each pair's r_ij . f_ij inside the
 * cutoff split equally between its two molecules; f_ij the force on i from
 * j, minimum image; the wall atoms are not molecules of the formula).
 * out[5] = {K_pore, W_pore, n_pore, V, P}. */
void orc_pore_pressure(int64_t nv, const double *xv, const double *v, const orc_params *p,
                       const orc_pore *pp, double *out)
{
    double kp = 0.0, wp = 0.0;
    int64_t np = 0;
    const double rc2 = p->cutoff * p->cutoff;
    for (int64_t i = 0; i < nv; ++i) {
        if (!in_pore(pp, p->box, xv + 3 * i)) continue;
        ++np;
        kp += 0.5 * p->mass * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] +
                               v[3 * i + 2] * v[3 * i + 2]);
        double wi = 0.0;
        for (int64_t j = 0; j < nv; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(xv + 3 * i, xv + 3 * j, p->box, d);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 >= rc2) continue;
            double u, w;
            lj_pair(r2, p->sigma, p->epsilon, p->cutoff, &u, &w);
            wi += w * r2;
        }
        wp += 0.5 * wi;
    }
    const double V = orc_pore_volume(pp, p->box);
    out[0] = kp;
    out[1] = wp;
    out[2] = (double)np;
    out[3] = V;
    out[4] = V > 0.0 ? (2.0 * kp + wp) / (3.0 * V) : 0.0;
}

/* Number of the n points that lie in the pore (for the volume pins). */
int64_t orc_pore_count(int64_t n, const double *x, const double *box, const orc_pore *pp)
{
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i) c += in_pore(pp, box, x + 3 * i);
    return c;
}
