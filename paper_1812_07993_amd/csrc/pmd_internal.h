// pmd_internal.h -- device-side data layout of the pore-MD library.
//
// A "pool" holds the state of one or more systems in shared device arrays.
// A stand-alone system is a pool with one resident system; a batch is a pool
// with many.  Every per-atom array is cell-sorted structure-of-arrays; each
// system owns a contiguous range of vapour slots padded to a multiple of
// the workgroup size, so that a workgroup never spans two systems.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmd {

constexpr int kPad = 256;            // vapour slots per system are padded to this
constexpr int kChunk = 16;           // atoms per entry of the chunk -> system table
constexpr int kTile = 4096;          // cells per workgroup of the cell-count scan
constexpr int kRebuildBlock = 256;   // threads per workgroup of the per-atom rebuild kernels
constexpr int kMaxBlock = 1024;      // largest workgroup of the brick kernels (multiple of 64)
constexpr unsigned kIndexBits = 26;  // wall list entry: wall slot | neighbour-cell code << 26
constexpr unsigned kIndexMask = (1u << kIndexBits) - 1u;
// Vapour list entries are 16 bits: the partner's staged-tile index relative
// to the atom's neighbourhood base (the first staged atom of its neighbour
// cell (-1, -1, -1); the 27 neighbour cells are consecutive tile ranges
// after it) in the low kRelBits bits, the neighbour-cell code above them.
constexpr unsigned kRelBits = 11;
constexpr unsigned kRelMask = (1u << kRelBits) - 1u;
// Neighbour-cell code q = (dx+1) + 3 (dy+1) + 9 (dz+1) in 0..26 of a list
// entry; kPadQ marks pad entries, whose shift -2h per axis puts the partner
// beyond the cutoff.
constexpr unsigned kPadQ = 31u;
constexpr unsigned kPadCode = kPadQ << kIndexBits;   // a wall pad entry's code bits

enum Phase : int {
    PH_INIT = 0,  // forces not yet computed
    PH_REST = 1,  // full-step state x(t), v(t), a(t)
    PH_RUN = 2    // leapfrog state inside a run: x(t), v(t - dt/2)
};

enum Status : int {
    ST_HALT = 1,       // an atom moved more than skin/2 away from its position at the last rebuild
    ST_OVERFLOW = 2,   // a neighbour list exceeded its capacity
    ST_NONFINITE = 4,  // a non-finite force or position appeared
    ST_TILE = 8,       // a brick's halo did not fit the LDS tile
    ST_STALL = 16,     // a rebuild overflowed: later rebuilds and steps wait
                       // until the host has grown the buffer and cleared this bit
    ST_SPAN = 32       // an atom's neighbourhood in the staged tile spans more
                       // than 2^kRelBits atoms: the bricks must shrink
};

// Per-system constants (set on the host at admission).
struct SysParams {
    double L[3];        // box edges
    double invL[3];
    double h[3];        // cell edges, L / nc
    double inv_h[3];    // nc / L, used to bin
    int nc[3];
    int ncell;          // nc0 * nc1 * nc2
    int bdim[3];        // cells per brick along each axis
    int nbk[3];         // bricks along each axis (edge bricks may be partial)
    int nbrick;         // nbk0 * nbk1 * nbk2
    int bcells;         // bdim0 * bdim1 * bdim2
    int nkey;           // nbrick * bcells: cells are numbered brick by brick
    int broff;          // first workgroup (brick) of this system in the pool
    int voff, nv, vcap; // vapour slots [voff, voff + vcap), real atoms first nv after sorting
    int woff, nw;       // wall slots [woff, woff + nw)
    int coff;           // vapour cell_start base: nkey + 2 entries (cells, padding cell, end)
    int wcoff;          // wall cell_start base: ncell + 1 entries (linear cell order)
    int choff;          // first chunk (kChunk atoms) of this system
    int pboff;          // energy partials base (one entry per brick)
    int toff, ntile;    // scan tiles [toff, toff + ntile)
    int ering_off, ering_cap;
    int energy_every;
    int active;         // 1 if the slot holds a system
    int pad0;
    double A, B, Aw, Bw;   // 4 eps sig^12, 4 eps sig^6 for vapour-vapour and vapour-wall
    double uc, ucw;        // energy shift u(r_c) of each pair kind
    double rc2, rl2;       // cutoff^2, neighbour-list radius^2
    double dt, mass, inv_mass;
    double rw2;            // wall-list radius^2, (r_c + skin/2)^2
    float half_skin;       // rebuild threshold on the displacement since the last rebuild
    int thermo;            // 1: Berendsen thermostat on
    int virial;            // 1: record the virial sums
    double tau_t, t0, dof; // its rise time, target temperature, 3 nv - 3
    // the pore's void, for the pressure in the pore: kind as pmd_pore_kind
    // (none: the whole box; plain slab: no pore), the z range [pz0, pz1) of
    // the slab (the gap for a slit), the radii of the hole and its volume
    int pkind;
    int pad1;
    double pz0, pz1, pr0, pr1, pvol;
    // reciprocals of the brick extents, for exact quotients by FP64
    // multiplication: 1/bdim per axis, 1/nbk0, 1/(nbk0 nbk1), 1/bcells
    double inv_bdim[3], inv_nbk0, inv_nbk01, inv_bcells;
};

// Quotient n / d for 0 <= n < 2^50 from inv = 1/d (rounded): (n + 1/2)/d lies
// at least 1/(2d) from an integer, far more than the rounding of the FP64
// product, so the truncation is exact.  Three instructions in place of the
// forty or so of an integer division by a value known only at run time.
__host__ __device__ __forceinline__ int quot(int n, double inv)
{
    return (int)(((double)n + 0.5) * inv);
}

// Per-system dynamic state, written by kernels.
struct SysState {
    int remaining;    // steps left in the current run
    int phase;        // Phase
    int status;       // Status bits seen by the current launch
    int status_next;  // bits raised during the current launch (merged at its end)
    int lbuf;         // current local-coordinate buffer (0/1)
    int sbuf;         // buffer holding the latest positions and velocities (0/1);
                      // every step reads one and writes the other
    int sbuf_prev;    // that buffer before the last rebuild (the placement's source)
    int ibuf;         // buffer holding the caller ids in the current storage order
    int ibuf_prev;    // that buffer before the last rebuild
    int nrec;         // energy records written
    int max_nbr;      // longest neighbour list at the last rebuild
    int rebins;       // rebuilds so far
    int steps_since;  // steps since the last rebuild
    int stop;         // first step of the current replay that raised a stop bit (INT_MAX: none)
    long long step;   // completed steps
    double lambda;    // Berendsen factor of the current step
};

struct EnergyRec {
    long long step;
    double ke, pe_vv, pe_vw;
    double w_vv, w_vw;  // virial sums r . f over vapour pairs and vapour-wall pairs
    double ke_pore, w_pore, n_pore;  // the molecules in the pore: kinetic energy,
                                     // shares of the vapour pair virials, count
};

// Energy partials per brick and step slot: ke, pe_vv, pe_vw, w_vv, w_vw,
// ke_pore, w_pore, n_pore.
constexpr int kPartial = 8;

typedef float f4 __attribute__((ext_vector_type(4)));   // 16 bytes, one 128-bit load
typedef double d4 __attribute__((ext_vector_type(4)));  // 32 bytes

template <typename T> struct V4;
template <> struct V4<float> { using type = f4; };
template <> struct V4<double> { using type = d4; };

// Device pointers of a pool, passed by value to every kernel.
struct PoolDev {
    SysParams* sp;
    SysState* st;
    const int* chunk_sys; // chunk of kChunk vapour slots -> system slot
    int nchunk;           // chunks in use
    const int* tile_sys;  // scan tile -> system slot
    int ntile;            // scan tiles in use
    const int* brick_sys; // brick (workgroup of the list and step kernels) -> system slot
    int nbrick;           // bricks in use
    int lds_atoms;        // capacity of the staged neighbour tile (atoms)
    int hmax;             // largest halo box (cells) of any resident system
    int block;            // threads per workgroup of the brick kernels
    int brick_order;      // 1: contiguous runs of bricks per XCD, 2: round-robin over XCDs
    int vt, wt;           // vapour and wall slot capacity
    int cap;              // neighbour-list capacity per atom
    int nbt;              // brick capacity (stride of the two energy-partial slots)
    int nslots;           // system slots
    int thermo;           // 1 if a resident system has the thermostat on
    int virial;           // 1 if a resident system records the virial sums
    // per-atom state, double buffered by SysState::sbuf; SoA with stride vt
    double* X[2];
    double* V[2];
    int* id[2];
    double* A;            // accelerations at rest (stride vt)
    f4* lref;             // FP32 cell-local position at the last rebuild (w unused):
                          // the displacement since then is the step's new local
                          // position minus this, both from the same cell origin
    int* cref;            // packed cell (cx | cy << 10 | cz << 20) at the last rebuild
    int* cell_lin;        // linear cell index cx + nx (cy + ny cz) at the last rebuild
    void* L[2];           // local coordinates (f4 or d4), vt + wt entries; walls at vt + w
    // binning scratch
    int* count;           // per cell (all systems' ranges)
    int* clocal;          // exclusive prefix of the counts inside each scan tile
    int* ctile;           // per scan tile: sum, then global slot offset
    int* cstart;          // per cell + padding + end: first slot (global)
    int* arr;             // arrival rank within the cell (per slot)
    int* tmp;             // slots in arrival order
    int* tmpid;           // caller index of the atom at each arrival position
    int* cell_tmp;        // cell key of each old slot
    // neighbour lists in 16-byte chunks, chunk c of slot i at bytes
    // (c * vt + i) * 16: first the vapour entries, eight 16-bit ones per
    // chunk (entry k at uint16 index ((k / 8) * vt + i) * 8 + k % 8), then,
    // from chunk ceil(n_vapour / 8), the wall entries, four 32-bit ones per
    // chunk; each part ends on a chunk boundary with pad entries.  The
    // capacity `cap` counts 32-bit words (four per chunk).
    // nlist = n_vapour | n_wall << 16
    unsigned* list;
    int* nlist;
    // walls
    double* WX;           // sorted wall positions, SoA stride wt
    int* wid;             // canonical wall index of each sorted wall slot
    int* wcstart;         // wall cell_start (global wall slots)
    // energies
    double* partial;      // kPartial doubles per brick, two slots (step parity)
    EnergyRec* erec;
};

struct PoreDev {
    int kind;
    int nslab;
    double a;
    double z_lo[2];
    double t;
    double r0, r1;
    int nx, ny, nz;       // sites per slab: nx * ny * nz
    int pad;
};

// ---- launchers (pmd_kernels.hip) -----------------------------------------
hipError_t launch_wall_generate(const PoreDev& pore, const double* L, double* out_xyz_soa,
                                int stride, int* block_counts, int* block_offsets,
                                int* total, hipStream_t s);
hipError_t launch_wall_bin(const PoolDev& P, int sys, const double* raw_soa, int raw_stride,
                           int nw, int precision, hipStream_t s);
hipError_t launch_rebuild(const PoolDev& P, int nslots, int precision, hipStream_t s);
hipError_t launch_set_run(const PoolDev& P, int slot, int add_steps, int clear_bits,
                          hipStream_t s);
hipError_t launch_reset_state(const PoolDev& P, int slot, long long step, hipStream_t s);
hipError_t launch_step(const PoolDev& P, int kk, int precision, hipStream_t s, hipEvent_t ev0,
                       hipEvent_t ev1);
hipError_t launch_commit(const PoolDev& P, int nslots, int R, hipStream_t s);
hipError_t launch_unpermute(const PoolDev& P, int slot, int which, double* out_aos,
                            int n, hipStream_t s);
hipError_t launch_wall_unpermute(const PoolDev& P, int slot, double* out_aos, int n,
                                 hipStream_t s);
hipError_t launch_debug_pairs(const PoolDev& P, int slot, int precision, int* out_triples,
                              int cap, int* counts, hipStream_t s);
hipError_t launch_copy_in(const PoolDev& P, int slot, const double* pos_aos,
                          const double* vel_aos, int n, int vcap, hipStream_t s);

}  // namespace pmd
