// The paper's pore model (all-pairs forces, reflecting pore walls, periodic
// outer space, 2D or 3D): launch of its steps, called by the C entry points
// pmd_pm_run and pmd_pm_run_noalloc.
#pragma once

#include <hip/hip_runtime.h>

namespace pmd {

struct PmArgs {
    int n, dim, precision;  // precision: 1 FP32 pair terms, 2 FP64
    double lx, ly, lz, k;
    double sig2, eps4, eps24, mass, inv_mass, dt, hdt, tau, t0;
    double vol;  // the pore's volume (area in 2D)
};

// Per-run working memory: accelerations [n][dim], per-molecule kinetic
// energy, pair-energy share, pair-virial share and place (1 in the pore, 2
// outside the domain) [n] each, two counters (wall reflections, drifts that
// could not be traced), and per workgroup of the update kernel its counts
// of reflections and failed traces, in two slots by step parity.
struct PmWork {
    double* acc;
    double* ke;
    double* u;
    double* vir;
    double* where;
    long long* counts;
    double* part;  // [2 parities][2 counts][nblk]
};

// Same layout as pmd_pm_record of the C interface.
struct PmRecord {
    long long step;
    double ke, pe, etotal, temperature, pressure;
    long long n_pore, reflections, n_outside;
};

constexpr int kPmDrift = 256;  // threads per workgroup of the update kernel

inline long long pm_drift_blocks(long long n) { return n > 0 ? (n + kPmDrift - 1) / kPmDrift : 1; }

// Doubles of working memory a run of n molecules in dim dimensions needs.
inline size_t pm_work_doubles(long long n, int dim)
{
    return (size_t)n * (dim + 4) + 2 + 4 * (size_t)pm_drift_blocks(n);
}

inline PmWork pm_work_at(double* base, long long n, int dim)
{
    PmWork w;
    w.acc = base;
    w.ke = base + (size_t)n * dim;
    w.u = w.ke + n;
    w.vir = w.u + n;
    w.where = w.vir + n;
    w.counts = (long long*)(w.where + n);
    w.part = w.where + n + 2;
    return w;
}

// The allocation-free entry point keeps its working memory in a static
// device array of this many doubles: runs of up to kPmScratchAtoms
// molecules in three dimensions (3.7 MB).
constexpr long long kPmScratchAtoms = 65536;
constexpr size_t kPmScratchDoubles = (size_t)kPmScratchAtoms * (3 + 4) + 2 + 4 * (size_t)(kPmScratchAtoms / kPmDrift);

// Device address of the current device's static working array (looked up
// with hipGetSymbolAddress on the first call per device, then cached).
hipError_t pm_scratch_ptr(double** out);

hipError_t launch_pm_run(const PmArgs& a, double* x, double* v, PmWork w, long long nsteps,
                         long long every, PmRecord* rec, hipStream_t s);

}  // namespace pmd
