/*
 * poremd.h -- C interface of the MI355X (gfx950) pore molecular-dynamics
 * library.
 *
 * The library advances systems of vapour molecules interacting with each
 * other and with the fixed atoms of a pore wall, as in Korenkov, Nikonov,
 * Popovicova, arXiv:1812.07993:
 *   - equations of motion m_i d^2 r_i/dt^2 = f_i                (Sec. 2, eq. 1)
 *   - f_i = -dU/dr_i + f_i^ex: Lennard-Jones pairs between vapour molecules,
 *     and the field of the wall atoms as f^ex                    (Sec. 2, eq. 2)
 *   - velocity Verlet: drift and first half-kick (the paper's F2), forces at
 *     the new positions (F1), second half-kick (F3)             (Sec. 3)
 *   - periodic boundaries on the outer box (Secs. 4-5).
 * Model readings the paper leaves open (fixed here and in the tests): 12-6
 * Lennard-Jones truncated at r_c and energy-shifted (force not shifted);
 * vapour-wall pairs use (sigma_wall, epsilon_wall) with the same r_c; walls
 * are simple-cubic lattices that never move; reduced units, k_B = 1.
 *
 * Conventions for every function:
 *   - Return value: PMD_OK (0) or a negative pmd_status.  A message for the
 *     last failure on the calling thread is available from pmd_last_error().
 *     No C++ exception crosses this interface.
 *   - Host arrays are row-major [n][3] doubles, in the caller's particle order
 *     (index i of the array given to pmd_create_system).  The library copies
 *     inputs; the caller keeps ownership of every pointer it passes.
 *   - Positions are returned wrapped into [0, L) on each axis.
 *   - A handle is not thread-safe; distinct handles may be used from
 *     different threads.
 *   - Work is queued on a HIP stream (the one given at creation, or a
 *     library-owned stream if NULL) and runs asynchronously until a call
 *     that reads results, or pmd_sync, waits for it.
 */
#ifndef POREMD_H
#define POREMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PMD_OK = 0,
    PMD_EINVAL = -1,   /* invalid argument (message says which) */
    PMD_ENOMEM = -2,   /* device memory or budget exhausted */
    PMD_EHIP = -3,     /* a HIP runtime call failed */
    PMD_ENUMERIC = -4, /* a non-finite force, energy or position appeared */
    PMD_EAGAIN = -5,   /* no room now (batch full or over budget); retry */
    PMD_ESTATE = -6    /* call not allowed in the handle's current state */
} pmd_status;

typedef enum { PMD_FP64 = 0, PMD_MIXED = 1 } pmd_precision;

typedef enum {
    PMD_PORE_NONE = 0,      /* no wall atoms */
    PMD_PORE_SLAB = 1,      /* one slab, no hole */
    PMD_PORE_CYLINDER = 2,  /* one slab with a cylindrical hole of radius r0 */
    PMD_PORE_SLIT = 3,      /* two slabs whose facing surfaces are slit_gap apart */
    PMD_PORE_CONE = 4,      /* one slab, hole radius linear from r0 (lower face) to r1 (upper face) */
    PMD_PORE_INKBOTTLE = 5  /* one slab, neck r0 in its outer quarters, cavity r1 in between */
} pmd_pore_kind;

/* Model parameters, reduced Lennard-Jones units.  box[k] is the periodic
 * box edge L_k.  Constraints: every L_k >= 3 * (cutoff + skin), sigma,
 * epsilon, mass, dt > 0, cutoff > 0. */
typedef struct {
    double box[3];
    double sigma, epsilon, mass, cutoff, dt;
    double sigma_wall, epsilon_wall;
    int32_t precision;    /* pmd_precision: PMD_FP64 = all arithmetic in FP64;
                             PMD_MIXED = pair forces in FP32, per-particle
                             force sums, integration and energies in FP64 */
    int32_t reserved;
    /* Berendsen thermostat (Sec. 2; the F4 listing of Sec. 3): with
     * thermostat_tau > 0 every step ends with v <- lambda v, lambda =
     * sqrt(1 + (dt / tau) (t0 / T - 1)), T = 2 ke / (3 n - 3) measured on the
     * full-step velocities (the recorded ke is this one, before the
     * scaling).  0 = off (NVE).  Requires tau >= dt and t0 > 0. */
    double thermostat_tau;
    double thermostat_t0;
} pmd_params;

/* Pore geometry.  Wall sites sit on a simple cubic lattice of spacing
 * lattice_a at x = (i + 1/2) a, y = (j + 1/2) a over the whole box and
 * z = z_lo + (k + 1/2) a through each slab [z_lo, z_lo + slab_thickness).
 * A slab is centred at slab_center_z (for a slit, the gap is).  The pore
 * axis is the line x = L_x/2, y = L_y/2; a site is removed when its distance
 * from the axis is strictly below the pore radius of its layer (evaluated at
 * the layer's centre).  Wall sites are numbered layer by layer (lower slab
 * first), then by y, then by x. */
typedef struct {
    int32_t kind;         /* pmd_pore_kind */
    int32_t reserved;
    double lattice_a;
    double slab_center_z;
    double slab_thickness;
    double r0, r1;
    double slit_gap;
} pmd_pore;

/* Energies at one step (per system).  ke = (m/2) sum |v|^2 at the full
 * step; pe_vv = sum over vapour pairs i<j; pe_vw = sum over vapour-wall
 * pairs; temperature = 2 ke / (3 n - 3).  virial_vv = sum over vapour pairs
 * i<j inside the cutoff of r_ij . f_ij (r_ij = r_i - r_j, minimum image;
 * f_ij the force on i from j, positive when repulsive), virial_vw the same
 * over vapour-wall pairs.
 * The pressure in the pore by the formula of Sec. 2 (P from the doubled
 * kinetic energy and the pair virial over the pore volume V):
 *   pressure = (2 ke_pore + virial_pore) / (3 pore_volume),
 * over the molecules whose position lies in the pore's void (the hole
 * through the slab, evaluated at each height as the hole's radius there;
 * the slit's gap; the whole box without walls; nothing for a plain slab),
 * ke_pore their kinetic energy, virial_pore their shares of the vapour pair
 * virials (each pair's r_ij . f_ij split equally between its two molecules;
 * the wall atoms are not molecules of the formula), pore_volume the void's
 * volume (pmd_pore_volume).  The printed formula's minus sign fits the
 * other force convention (f = dU/dr). */
typedef struct {
    int64_t step;
    double ke, pe_vv, pe_vw, etotal, temperature;
    double virial_vv, virial_vw;  /* 0 unless the tuning asks for them */
    double ke_pore, virial_pore;  /* 0 unless the tuning asks for the virial */
    int64_t n_pore;               /* molecules in the pore (ditto) */
    double pore_volume;
    double pressure;              /* 0 unless the tuning asks for the virial */
} pmd_energies;

/* Performance knobs; zero fields take the library default.  skin: extra
 * radius of the neighbour lists beyond the cutoff; rebin_every: steps
 * between neighbour-list rebuilds (a rebuild also happens early whenever an
 * atom has moved more than skin/2 from its position at the last one); block: threads
 * per workgroup of the force kernels (a multiple of 64 from 64 to 1024; each
 * workgroup owns one brick of cells, sized to hold about 0.8 x block atoms
 * unless brick_atoms says otherwise); list_cap:
 * neighbour-list storage per atom in 32-bit words (a vapour partner takes
 * half a word, a wall partner a word, each part rounded up to four words);
 * energy_every: record energies every k steps (the last step of
 * every pmd_step call is always recorded). */
typedef struct {
    double skin;
    int32_t rebin_every;
    int32_t block;
    int32_t list_cap;
    int32_t energy_every;
    int32_t use_graph;    /* 1: replay captured HIP graphs; 0: plain launches */
    int32_t brick_atoms;  /* target atoms per brick (workgroup); 0 = 0.8 x block */
    int32_t brick_order;  /* workgroup order of the brick kernels: 1 = each XCD
                           * takes a contiguous run of bricks, 2 = bricks dealt
                           * round-robin over the XCDs; 0 = library default */
    int32_t virial;       /* 1: record the virial sums (virial_vv, virial_vw of
                           * pmd_energies) on recording steps; 0 (default): they
                           * read 0 and the step kernel is about 3% faster */
} pmd_tuning;

typedef struct pmd_system pmd_system;
typedef struct pmd_batch pmd_batch;

/* Message for the last failure on the calling thread (never NULL). */
const char *pmd_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int pmd_version(void);

/* Number of wall sites a pore would generate in a box (host arithmetic
 * only; no device work). */
int pmd_wall_count(const pmd_params *params, const pmd_pore *pore, int64_t *n_wall);

/* Volume of the pore's void (host arithmetic): pi r0^2 t (cylinder),
 * pi t (r0^2 + r0 r1 + r1^2) / 3 (cone), pi (t/2) (r0^2 + r1^2) (ink-bottle:
 * neck quarters and cavity half), Lx Ly slit_gap (slit), Lx Ly Lz (no walls),
 * 0 (plain slab): the V of the pressure in the pore (Sec. 2). */
int pmd_pore_volume(const pmd_params *params, const pmd_pore *pore, double *volume);

/* Device bytes a system of n_vapor molecules with this pore occupies in a
 * batch, with the given tuning (NULL = defaults): the figure pmd_batch_admit
 * charges against the batch's budget. */
int pmd_footprint_bytes(const pmd_params *params, const pmd_pore *pore,
                        int64_t n_vapor, const pmd_tuning *tuning, size_t *out);

/* Create a system (Sec. 2: N particles with positions, velocities and mass
 * in a pore).  pos, vel: host [n_vapor][3].  Walls: if wall_pos is NULL the
 * library generates them from pore (n_wall is ignored); otherwise wall_pos
 * is host [n_wall][3] and pore only describes the geometry.  hip_stream: a
 * hipStream_t to queue work on, or NULL for a library-owned stream.
 * tuning: NULL = defaults.  The initial forces and energies are computed
 * before the call returns.  Fails with PMD_EINVAL on a bad parameter,
 * non-finite input or a position outside [0, L) after wrapping. */
int pmd_create_system(const pmd_params *params, const pmd_pore *pore,
                      int64_t n_vapor, const double *pos, const double *vel,
                      int64_t n_wall, const double *wall_pos, void *hip_stream,
                      const pmd_tuning *tuning, pmd_system **out);

/* Queue nsteps velocity-Verlet steps (each: F2 drift and half-kick, F1
 * forces, F3 half-kick, and with a thermostat the F4 scaling, Sec. 3).
 * Asynchronous; pmd_sync or any readback waits. */
int pmd_step(pmd_system *sys, int64_t nsteps);

/* Wait until every queued step has been done.  Returns PMD_ENUMERIC if a
 * non-finite value appeared. */
int pmd_sync(pmd_system *sys);

/* Readbacks (wait for queued work).  n must equal the system's count.  The
 * quantities are the state the paper keeps per particle: coordinates,
 * velocities and forces (Sec. 3), and the kinetic and potential energies of
 * the model of Sec. 2.  Host out buffers, owned by the caller; PMD_EINVAL on
 * a count mismatch or NULL, PMD_ENUMERIC if a non-finite value appeared. */
int pmd_get_positions(pmd_system *sys, double *out, int64_t n);
int pmd_get_velocities(pmd_system *sys, double *out, int64_t n);
/* Forces on the vapour molecules at the current positions, [n][3]: f_i of
 * Sec. 2, eq. 2 (pairs with other molecules plus the wall field). */
int pmd_get_forces(pmd_system *sys, double *out, int64_t n);
/* Energies at the current step (ke, pe and their sum, Sec. 2). */
int pmd_get_energies(pmd_system *sys, pmd_energies *out);
/* Recorded energies, oldest first; at most cap rows; *n_out = rows written. */
int pmd_get_energy_history(pmd_system *sys, pmd_energies *out, int64_t cap,
                           int64_t *n_out);
/* Wall sites in the canonical order of pmd_pore, [n_wall][3] (the fixed
 * atoms whose field is f^ex of Sec. 2, eq. 2). */
int pmd_get_wall_positions(pmd_system *sys, double *out, int64_t n_wall);
int pmd_get_counts(pmd_system *sys, int64_t *n_vapor, int64_t *n_wall);
int64_t pmd_get_step(pmd_system *sys);

/* Positions into a device buffer dev_out ([n][3] doubles, caller order),
 * queued on `stream` (NULL = the system's stream) after the system's
 * queued work.  Does not wait. */
int pmd_get_positions_device(pmd_system *sys, double *dev_out, int64_t n,
                             void *stream);

/* Change the performance knobs of an existing system (takes effect at the
 * next pmd_step). */
int pmd_set_tuning(pmd_system *sys, const pmd_tuning *tuning);
int pmd_get_tuning(pmd_system *sys, pmd_tuning *out);

/* Replace the state of a system (not one resident in a batch) with
 * caller-order positions and velocities, host [n][3] each, n equal to the
 * system's vapour count, and set its step counter to `step`: the restart
 * from a checkpoint taken with pmd_get_positions / pmd_get_velocities /
 * pmd_get_step.  Forces and energies at the loaded positions are computed
 * before the call returns, and the energy history restarts at `step`.  The
 * continued trajectory equals the uninterrupted one to rounding (the force
 * sums are re-ordered by the fresh cell binning).  Same input checks as
 * pmd_create_system. */
int pmd_set_state(pmd_system *sys, const double *pos, const double *vel,
                  int64_t n, int64_t step);

/* ---- Autotuner (neighbour-list skin, rebuild period, brick size) --------
 * The skin and the rebuild period trade the cost of a rebuild against the
 * length of the neighbour lists the force pass walks; the best pair depends
 * on the density, the temperature and the device.  pmd_autotune times each
 * candidate on one trial copy of the system described by the same inputs as
 * pmd_create_system (the caller's arrays are not changed, no caller system
 * is touched): the trial copy first runs max(2 x trial_steps, 1000) steps
 * (a fresh placement is not typical of a run: adsorption onto the walls
 * changes local densities and speeds); per candidate it then reloads that
 * state, runs trial_steps / 4 untimed steps and times trial_steps steps
 * (wall clock, including rebuilds and early-rebuild round trips).
 * us_per_step [n_candidates] (may be NULL) receives each candidate's
 * microseconds per step (infinity for a candidate that cannot run, e.g. a
 * skin leaving fewer than 3 cells per axis); *best the index of the fastest,
 * or, when us_per_step is given, of the fastest candidate with the largest
 * skin among those within 2% of the fastest, since early rebuilds grow more
 * frequent as a run goes on.  Fails if none runs.  pmd_autotune_grid writes the built-in candidate grid (skin x
 * rebuild period, other knobs at their defaults) into out[cap]; with
 * out == NULL it only reports the count in *n_out. */
int pmd_autotune_grid(const pmd_params *params, int64_t n_vapor, pmd_tuning *out,
                      int32_t cap, int32_t *n_out);
int pmd_autotune(const pmd_params *params, const pmd_pore *pore, int64_t n_vapor,
                 const double *pos, const double *vel, int64_t n_wall,
                 const double *wall_pos, void *hip_stream,
                 const pmd_tuning *candidates, int32_t n_candidates,
                 int64_t trial_steps, double *us_per_step, int32_t *best);

/* Destroy a system (NULL-safe).  Waits for queued work. */
int pmd_destroy(pmd_system *sys);

/* ---- Kernel timing, for measurement ------------------------------------ */

/* When enabled, the system's steps are queued without graph capture and the
 * R back-to-back launches of the force-and-integrate kernel in each replay
 * (R = rebin_every) are bracketed by one pair of HIP events on the system's
 * stream; the host waits after each replay to read how many steps it did.
 * A replay cut short by an early rebuild also holds launches that return at
 * once; their duration is measured when timing is enabled (32 back-to-back
 * launches on the system at rest; the system must have no queued steps) and
 * subtracted.  pmd_kernel_time returns the number of launches that did a
 * step and the mean duration of one in milliseconds; pmd_kernel_times writes
 * one value per replay that did a step (its mean launch duration, oldest
 * first, at most cap values) and the number of such replays in *n_out.
 * Enabling or disabling clears earlier timings. */
int pmd_timing_enable(pmd_system *sys, int enable);
int pmd_kernel_time(pmd_system *sys, int64_t *launches, double *mean_ms);
int pmd_kernel_times(pmd_system *sys, double *out_ms, int64_t cap, int64_t *n_out);

/* ---- Test-only debug exports (same library; unstable) ------------------- */

/* Cell binning after the last rebuild.  cell_of_atom[n]: linear cell
 * cx + ncell_0 (cy + ncell_1 cz) of each atom (caller order); perm[n]: caller
 * indices in storage order (cells grouped in bricks, ascending caller index
 * inside a cell); cell_start[n_cells + 1]: storage position of the first
 * atom of each linear cell (the last entry is n); ncell[3] and inv[3] (cells
 * per unit length, inv_k = ncell_k / L_k) describe the grid.  Positions used
 * are those at the last rebuild. */
int pmd_debug_cells(pmd_system *sys, int32_t *cell_of_atom, int64_t n,
                    int32_t *cell_start, int64_t n_cells_p1, int32_t *perm,
                    int32_t *ncell, double *inv);
/* In-cutoff pairs found through the neighbour lists at the current
 * positions, tested in FP64: vv (i < j) and vw (i, wall index), caller
 * order, each sorted lexicographically.  Writes at most cap pairs of each
 * kind; *n_vv and *n_vw receive the totals. */
int pmd_debug_pairs(pmd_system *sys, int32_t *vv, int64_t cap, int64_t *n_vv,
                    int32_t *vw, int64_t *n_vw);
/* Number of neighbour-list rebuilds so far, and the longest list at the
 * last one (in 32-bit words, as list_cap counts them). */
int pmd_debug_lists(pmd_system *sys, int64_t *rebuilds, int64_t *max_len);

/* ---- Batching and serving ------------------------------------------------ */

/* A batch advances many systems together: one launch per phase covers all
 * resident systems, and the steps are replayed from captured HIP graphs.
 * Each resident system takes exactly the steps of Sec. 3 (F2, F1, F3 and,
 * with a thermostat, F4) that it would take alone, with bit-identical
 * results; the paper runs one system at a time, so batching is a scheduling
 * layer with no counterpart there.
 * hbm_budget bounds the device bytes the batch may hold (0 = no bound);
 * max_slots bounds the number of resident systems. */
int pmd_batch_create(size_t hbm_budget, int max_slots, void *hip_stream,
                     pmd_batch **out);
/* Move a system into the batch with nsteps steps to run.  Waits for the
 * work already queued on the batch (admission changes the batch's tables).
 * Returns
 * PMD_EAGAIN if no slot or budget is free, or if the batch's wall slots
 * would exceed the limit of pmd_batch_wall_room.  The system handle stays
 * valid but may not be stepped or read until released. */
int pmd_batch_admit(pmd_batch *b, pmd_system *sys, int64_t nsteps, int *slot);
/* Run chunk_steps steps (or fewer where a system finishes) on every resident
 * system.  Asynchronous. */
int pmd_batch_advance(pmd_batch *b, int64_t chunk_steps);
/* Slots whose systems have finished their steps (waits for queued work). */
int pmd_batch_poll(pmd_batch *b, int *done_slots, int cap, int *n_done);
/* Non-blocking variant: reports the systems that had finished by the end
 * of the newest chunk of pmd_batch_advance that the device has completed
 * (each chunk leaves a copy of the systems' states in pinned host memory,
 * with an event), while later chunks may still run; it waits for nothing.
 * Where that state shows a system needing the host (a list or tile to
 * grow), it does what pmd_batch_poll does. */
int pmd_batch_poll_async(pmd_batch *b, int *done_slots, int cap, int *n_done);
/* Take a system out of the batch; its handle becomes usable again. */
int pmd_batch_release(pmd_batch *b, int slot, pmd_system **sys_out);
int pmd_batch_info(pmd_batch *b, int *resident, size_t *bytes_used,
                   size_t *bytes_budget);
int pmd_batch_destroy(pmd_batch *b);
/* The admission rule for wall atoms (host arithmetic only, no device work):
 * a neighbour-list entry names a wall by its slot in the batch's pool in 26
 * bits, so a batch may hold at most 2^26 - 1 wall slots in total.  Returns
 * PMD_OK if resident_walls + new_walls fits, PMD_EAGAIN if it does not,
 * PMD_EINVAL for a negative count.  pmd_batch_admit applies it before
 * admitting a system. */
int pmd_batch_wall_room(int64_t resident_walls, int64_t new_walls);

/* ---- All-pairs forces (the paper's F1 as printed) ------------------------ */

/* Forces and potential energy of n atoms where every pair i != j interacts:
 * the force function of Sec. 3 with no cutoff and no shift,
 *   u(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6),
 *   f_i  = sum_j 24 eps (2 (sigma/r)^12 - (sigma/r)^6) r_ij / r^2,
 * with r_ij = x_i - x_j taken by the minimum image along each axis whose
 * box[k] > 0 (box[k] <= 0: that axis is open).
 *   precision  1 = FP32 pair terms (from FP64 differences) with FP64 sums,
 *              2 = FP64 throughout.
 *   x_dev      device, [n][3] doubles (read).
 *   box        host, 3 doubles.
 *   f_dev      device, [n][3] doubles (written).
 *   u_dev      device, [n] doubles (written): each atom's half share,
 *              sum_j u(r_ij) / 2.
 *   e_dev      device, 1 double (written): the sum of u_dev (0 for n = 0),
 *              in a fixed order that depends only on n (strided partial
 *              sums, then a fixed tree), not in index order.
 *   stream     hipStream_t (NULL = the default stream); queued, no wait.
 * The caller owns every buffer; the sums are in a fixed order, so repeated
 * calls give identical results.  Coincident atoms give non-finite values.
 * Returns PMD_EINVAL for n < 0 or n > 2^24, a null buffer with n > 0, a
 * precision other than 1 or 2, or a non-finite or non-positive sigma, a
 * non-finite epsilon or box. */
int pmd_allpairs_forces(int precision, int64_t n, const double *x_dev,
                        const double box[3], double epsilon, double sigma,
                        double *f_dev, double *u_dev, double *e_dev,
                        void *stream);

/* ---- The paper's pore model (Secs. 4-5) --------------------------------- */

/* The model the paper times: N molecules in two (Sec. 4) or three (Sec. 5)
 * dimensions; every pair interacts through u(r) = 4 eps ((sigma/r)^12 -
 * (sigma/r)^6) with no cutoff and plain differences r_ij = x_i - x_j (the
 * domain is not a torus, so no images); no wall atoms.  The domain:
 *   pore   [0, lx) x [0, ly] (x [0, lz] in 3D), whose walls x = 0, y = 0,
 *          y = ly (z = 0, z = lz) reflect molecules specularly (Secs. 4, 5:
 *          reflecting pore walls; the rule is specular reflection of the
 *          normal velocity component), open at x = lx (the mouth,
 *          0 <= y < ly, 0 <= z < lz);
 *   outer  [lx, (k+1) lx) x [-k ly, (k+1) ly) (x [-k lz, (k+1) lz)), its
 *          faces periodic (Secs. 4, 5), except that a molecule crossing
 *          x = lx leftwards inside the mouth enters the pore.  Its volume is
 *          k (2k+1)^(dim-1) pore volumes: 21 at k = 3 in 2D (Sec. 4), 9 at
 *          k = 1 in 3D (Sec. 5).
 * A molecule belongs to the pore iff x < lx.  Positions and velocities are
 * [n][dim] doubles. */
typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t precision;    /* 1 = FP32 pair terms (from FP64 differences) with
                             FP64 sums; 2 = FP64 throughout */
    double lx, ly, lz;    /* pore edges (lz unused in 2D) */
    double k;             /* outer-space scale, > 0 */
    double sigma, epsilon, mass, dt;
    double thermostat_tau, thermostat_t0;  /* Berendsen F4 if tau > 0 */
} pmd_pm_model;

/* One energy record of a pore-model run. */
typedef struct {
    int64_t step;
    double ke;            /* (m/2) sum |v|^2 after F3 (before the F4 scaling) */
    double pe;            /* sum over pairs i < j of u(r_ij) */
    double etotal;        /* ke + pe */
    double temperature;   /* 2 ke / (dim n): the reflecting walls break
                             momentum conservation, so every degree of
                             freedom counts */
    double pressure;      /* in the pore, Sec. 2's virial formula with the
                             pore volume V = lx ly (lz):
                             P = (2 K + W) / (dim V), K the kinetic energy of
                             the molecules with x < lx, W their shares of the
                             pair virials (each pair's r_ij . f_ij split
                             equally between its molecules, f_ij the force on
                             i from j, positive when repulsive) */
    int64_t n_pore;       /* molecules with x < lx */
    int64_t reflections;  /* wall reflections since the run started */
    int64_t n_outside;    /* molecules outside the domain, plus drifts that
                             could not be traced; 0 in a valid run */
} pmd_pm_record;

/* Rows a run of nsteps steps records with energy_every (host arithmetic):
 * step 0, every multiple of energy_every (if > 0) and the last step. */
int64_t pmd_pm_record_rows(int64_t nsteps, int64_t energy_every);

/* Advance n molecules of the pore model by nsteps velocity-Verlet steps in
 * the order of the paper's GPU functions (Sec. 3):
 *   F2  dl = v dt + a dt^2 / 2, v <- v + a dt / 2, and the molecule carried
 *       along dl through the walls, the mouth and the periodic faces;
 *   F1  a = f / m from the all-pairs forces at the new positions;
 *   F3  v <- v + a dt / 2;
 *   F4  with thermostat_tau > 0: v <- lambda v, lambda = sqrt(1 + (dt / tau)
 *       (t0 / T - 1)), T from the F3 velocities (Sec. 2's Berendsen
 *       thermostat; the paper gives its rise time, not the formula).
 * The accelerations at the start are computed from x (a run always starts
 * from positions and velocities alone).
 *   x_dev, v_dev  device, [n][dim] doubles, updated in place; positions
 *                 must lie in the domain (a record's n_outside counts any
 *                 that do not).
 *   a_dev         device, [n][dim] doubles (NULL = not wanted): receives
 *                 the accelerations f / m at the final positions.
 *   rec_dev       device, rec_cap records (NULL = none): step 0, every
 *                 energy_every-th step and the last step, in order.
 *   stream        hipStream_t (NULL = the default stream); queued, no wait.
 * Working memory ((dim + 4) n + 2 + 4 ceil(n / 256) doubles) is taken from the stream-ordered
 * allocator for the call and returned at its end.  Sums are in a fixed
 * order: repeated runs give identical results.  Returns PMD_EINVAL for a
 * dim other than 2 or 3, a precision other than 1 or 2, n outside 0..2^20,
 * a null buffer with n > 0, a non-positive or non-finite length, k, sigma,
 * mass or dt, a thermostat with tau < dt or t0 <= 0, or rec_cap below
 * pmd_pm_record_rows; PMD_ENOMEM if the working memory cannot be had. */
int pmd_pm_run(const pmd_pm_model *model, int64_t n, double *x_dev,
               double *v_dev, double *a_dev, int64_t nsteps,
               int64_t energy_every, pmd_pm_record *rec_dev, int64_t rec_cap,
               void *stream);

/* pmd_pm_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same arguments, steps and results, but the working memory is a static
 * device array of the library, one per GPU, held until the process ends,
 * sized for n <= 65536 molecules (3.7 MB).  Makes no allocation of any kind.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams, or from different threads) race and give wrong
 * results; calls queued on one stream are safe.  Returns PMD_EINVAL for
 * n > 65536 and for everything pmd_pm_run rejects. */
int pmd_pm_run_noalloc(const pmd_pm_model *model, int64_t n, double *x_dev,
                       double *v_dev, double *a_dev, int64_t nsteps,
                       int64_t energy_every, pmd_pm_record *rec_dev,
                       int64_t rec_cap, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* POREMD_H */
