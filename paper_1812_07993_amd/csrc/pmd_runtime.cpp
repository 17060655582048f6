// pmd_runtime.cpp -- host runtime behind poremd.h: device memory pools,
// system creation, the step driver (graph replay of a rebuild followed by R
// fused steps), readbacks, batching and errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <numeric>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/poremd.h"
#include "pmd_allpairs.h"
#include "pmd_internal.h"
#include "pmd_paper.h"

using namespace pmd;

namespace {

thread_local std::string g_err = "no error";

// One lock for the calls that capture HIP graphs, allocate or free device
// memory, or copy synchronously: HIP's thread-local capture mode does not
// keep such calls on other threads (a server creating systems on worker
// threads while its tick thread re-captures a batch's graph) from breaking
// the capture.  Recursive, because some of these calls make others.
std::recursive_mutex g_gpu_mu;
#define GPU_LOCK std::lock_guard<std::recursive_mutex> gpu_lock_(g_gpu_mu)

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess)                                                            \
            return fail(e_ == hipErrorOutOfMemory ? PMD_ENOMEM : PMD_EHIP, "%s: %s (%s:%d)", \
                        #x, hipGetErrorString(e_), __FILE__, __LINE__);                  \
    } while (0)

#define CHK(x)                 \
    do {                       \
        int r_ = (x);          \
        if (r_ != PMD_OK) return r_; \
    } while (0)

int round_up(int a, int b) { return ((a + b - 1) / b) * b; }

// Workgroup order of the brick kernels: 1 = each XCD takes a contiguous run
// of bricks (spatial neighbours share an L2), 2 = bricks dealt round-robin
// over the XCDs (a dense region of the box is spread over all of them).
constexpr int kDefaultBrickOrder = 2;

constexpr int kDefaultErings = 16384;

// ---------------------------------------------------------------------------
// Model constants
// ---------------------------------------------------------------------------

struct Grid {
    int nc[3];
    double h[3];
};

int grid_for(const pmd_params& p, double skin, Grid* g)
{
    const double rl = p.cutoff + skin;
    for (int k = 0; k < 3; ++k) {
        int n = (int)std::floor(p.box[k] / rl);
        if (n < 3)
            return fail(PMD_EINVAL, "box edge %g is below 3 (cutoff + skin) = %g", p.box[k], 3 * rl);
        if (n > 1023) n = 1023;
        g->nc[k] = n;
        g->h[k] = p.box[k] / n;
    }
    return PMD_OK;
}

int check_params(const pmd_params* p, const pmd_pore* q)
{
    if (!p || !q) return fail(PMD_EINVAL, "params and pore must not be NULL");
    for (int k = 0; k < 3; ++k)
        if (!(p->box[k] > 0) || !std::isfinite(p->box[k])) return fail(PMD_EINVAL, "box[%d] must be > 0", k);
    if (!(p->sigma > 0) || !(p->epsilon >= 0) || !(p->mass > 0) || !(p->cutoff > 0) || !(p->dt > 0))
        return fail(PMD_EINVAL, "sigma, mass, cutoff, dt must be > 0 and epsilon >= 0");
    if (!(p->sigma_wall > 0) || !(p->epsilon_wall >= 0))
        return fail(PMD_EINVAL, "sigma_wall must be > 0 and epsilon_wall >= 0");
    if (p->precision != PMD_FP64 && p->precision != PMD_MIXED)
        return fail(PMD_EINVAL, "precision must be PMD_FP64 or PMD_MIXED");
    if (!(p->thermostat_tau >= 0) || !std::isfinite(p->thermostat_tau))
        return fail(PMD_EINVAL, "thermostat_tau must be >= 0 (0: off)");
    if (p->thermostat_tau > 0 && (!(p->thermostat_tau >= p->dt) || !(p->thermostat_t0 > 0) ||
                                  !std::isfinite(p->thermostat_t0)))
        return fail(PMD_EINVAL, "a thermostat needs thermostat_tau >= dt and thermostat_t0 > 0");
    if (q->kind < PMD_PORE_NONE || q->kind > PMD_PORE_INKBOTTLE) return fail(PMD_EINVAL, "unknown pore kind %d", q->kind);
    if (q->kind != PMD_PORE_NONE) {
        if (!(q->lattice_a > 0)) return fail(PMD_EINVAL, "lattice_a must be > 0");
        if (!(q->slab_thickness > 0)) return fail(PMD_EINVAL, "slab_thickness must be > 0");
        double lo, hi;
        if (q->kind == PMD_PORE_SLIT) {
            lo = q->slab_center_z - 0.5 * q->slit_gap - q->slab_thickness;
            hi = q->slab_center_z + 0.5 * q->slit_gap + q->slab_thickness;
        } else {
            lo = q->slab_center_z - 0.5 * q->slab_thickness;
            hi = q->slab_center_z + 0.5 * q->slab_thickness;
        }
        if (lo < 0 || hi > p->box[2]) return fail(PMD_EINVAL, "pore slabs [%g, %g) leave the box", lo, hi);
    }
    return PMD_OK;
}

PoreDev pore_dev(const pmd_params& p, const pmd_pore& q)
{
    PoreDev d{};
    d.kind = q.kind;
    d.a = q.lattice_a > 0 ? q.lattice_a : 1.0;
    d.t = q.slab_thickness;
    d.r0 = q.r0;
    d.r1 = q.r1;
    d.nx = (int)std::floor(p.box[0] / d.a + 0.5);
    d.ny = (int)std::floor(p.box[1] / d.a + 0.5);
    d.nz = (int)std::floor(q.slab_thickness / d.a + 0.5);
    if (q.kind == PMD_PORE_NONE) {
        d.nslab = 0;
    } else if (q.kind == PMD_PORE_SLIT) {
        d.nslab = 2;
        d.z_lo[0] = q.slab_center_z - 0.5 * q.slit_gap - q.slab_thickness;
        d.z_lo[1] = q.slab_center_z + 0.5 * q.slit_gap;
    } else {
        d.nslab = 1;
        d.z_lo[0] = q.slab_center_z - 0.5 * q.slab_thickness;
    }
    return d;
}

// The pore's void (the region of the pressure in the pore): the hole through
// the slab (z range of the slab, radii r0, r1), the slit's gap, the whole box
// without walls, nothing for a plain slab; and its volume in closed form:
// pi r0^2 t, the cone's frustum pi t (r0^2 + r0 r1 + r1^2) / 3, the
// ink-bottle's pi (t/2) (r0^2 + r1^2), Lx Ly gap, Lx Ly Lz.
double pore_void_volume(const pmd_params& p, const pmd_pore& q)
{
    const double t = q.slab_thickness, pi = 3.14159265358979323846;
    switch (q.kind) {
    case PMD_PORE_NONE: return p.box[0] * p.box[1] * p.box[2];
    case PMD_PORE_CYLINDER: return pi * q.r0 * q.r0 * t;
    case PMD_PORE_SLIT: return p.box[0] * p.box[1] * q.slit_gap;
    case PMD_PORE_CONE: return pi * t * (q.r0 * q.r0 + q.r0 * q.r1 + q.r1 * q.r1) / 3.0;
    case PMD_PORE_INKBOTTLE: return pi * 0.5 * t * (q.r0 * q.r0 + q.r1 * q.r1);
    default: return 0.0;
    }
}

void set_pore_region(SysParams& sp, const pmd_params& p, const pmd_pore& q)
{
    sp.pkind = q.kind;
    if (q.kind == PMD_PORE_SLIT) {
        sp.pz0 = q.slab_center_z - 0.5 * q.slit_gap;
        sp.pz1 = q.slab_center_z + 0.5 * q.slit_gap;
    } else {
        sp.pz0 = q.slab_center_z - 0.5 * q.slab_thickness;
        sp.pz1 = q.slab_center_z + 0.5 * q.slab_thickness;
    }
    sp.pr0 = q.r0;
    sp.pr1 = q.r1;
    sp.pvol = pore_void_volume(p, q);
}

// Host count of the wall sites (used to size buffers before generation).
int64_t host_wall_count(const pmd_params& p, const pmd_pore& q)
{
    const PoreDev d = pore_dev(p, q);
    int64_t n = 0;
    for (int s = 0; s < d.nslab; ++s)
        for (int k = 0; k < d.nz; ++k) {
            const double hz = (k + 0.5) * d.a;
            double r = 0.0;
            if (d.kind == PMD_PORE_CYLINDER) r = d.r0;
            else if (d.kind == PMD_PORE_CONE) r = d.r0 + (d.r1 - d.r0) * (hz / d.t);
            else if (d.kind == PMD_PORE_INKBOTTLE) r = (hz < 0.25 * d.t || hz >= 0.75 * d.t) ? d.r0 : d.r1;
            for (int j = 0; j < d.ny; ++j)
                for (int i = 0; i < d.nx; ++i) {
                    const double dx = (i + 0.5) * d.a - 0.5 * p.box[0];
                    const double dy = (j + 0.5) * d.a - 0.5 * p.box[1];
                    if (!(dx * dx + dy * dy < r * r)) ++n;
                }
        }
    return n;
}

// Neighbour-list words per atom for a skin: room for 1.5 x the mean count in
// the list sphere (at least at density 0.3, adsorbed layers are denser than
// the mean) at two vapour entries per word, plus room for wall partners (a
// word each) and the chunk padding.
int default_list_cap(const pmd_params& p, int64_t nv, double skin)
{
    const double V = p.box[0] * p.box[1] * p.box[2];
    const double rho = std::max(0.3, (double)nv / V);
    const double rl = p.cutoff + skin;
    const double sphere = 4.0 / 3.0 * M_PI * rl * rl * rl;
    return round_up((int)std::ceil(0.75 * sphere * rho) + 48, 16);
}

pmd_tuning default_tuning(const pmd_params& p, int64_t nv)
{
    pmd_tuning t{};
    t.skin = 0.5;
    t.rebin_every = 7;
    t.block = 256;
    t.list_cap = default_list_cap(p, nv, t.skin);
    t.energy_every = 0;
    t.use_graph = 1;
    t.brick_atoms = 0;
    t.brick_order = kDefaultBrickOrder;
    t.virial = 0;
    return t;
}

int merge_tuning(const pmd_params& p, int64_t nv, const pmd_tuning* in, pmd_tuning* out)
{
    pmd_tuning d = default_tuning(p, nv);
    if (in) {
        if (in->skin > 0) {
            d.skin = in->skin;
            d.list_cap = default_list_cap(p, nv, d.skin);
        }
        if (in->rebin_every > 0) d.rebin_every = in->rebin_every;
        if (in->block > 0) d.block = in->block;
        if (in->list_cap > 0) d.list_cap = in->list_cap;
        if (in->energy_every >= 0) d.energy_every = in->energy_every;
        d.use_graph = in->use_graph;
        if (in->brick_atoms > 0) d.brick_atoms = in->brick_atoms;
        if (in->brick_order > 0) d.brick_order = in->brick_order;
        d.virial = in->virial ? 1 : 0;
    }
    if (d.block < 64 || d.block > kMaxBlock || d.block % 64)
        return fail(PMD_EINVAL, "block must be a multiple of 64 from 64 to %d (got %d)", kMaxBlock, d.block);
    if (d.rebin_every > 1000) return fail(PMD_EINVAL, "rebin_every must be <= 1000");
    if (d.brick_order != 1 && d.brick_order != 2)
        return fail(PMD_EINVAL, "brick_order must be 0, 1 or 2 (got %d)", d.brick_order);
    if (d.list_cap > 4096) return fail(PMD_EINVAL, "list_cap must be <= 4096");
    d.list_cap = round_up(d.list_cap, 16);  // the list layout groups entries by 4
    *out = d;
    return PMD_OK;
}

// ---------------------------------------------------------------------------
// Device memory pool
// ---------------------------------------------------------------------------

struct Pool {
    int precision = 0;
    int block = 256;
    int brick_order = kDefaultBrickOrder;
    int cap = 64;
    int vt = 0, wt = 0, ct = 0, wct = 0, nbt = 0, nslots = 0, ering_cap = kDefaultErings;
    int thermo = 0;  // a resident system has the thermostat on
    int virial = 0;  // a resident system records the virial sums
    size_t bytes = 0;
    // device arrays
    SysParams* d_sp = nullptr;
    SysState* d_st = nullptr;
    int* d_chunk = nullptr;
    int* d_tile = nullptr;
    int* d_brick = nullptr;
    double* X[2] = {nullptr, nullptr};
    double* V[2] = {nullptr, nullptr};
    int* id[2] = {nullptr, nullptr};
    double* A = nullptr;
    f4* lref = nullptr;
    int* cref = nullptr;
    int* cell_lin = nullptr;
    void* L[2] = {nullptr, nullptr};
    int* count = nullptr;
    int* clocal = nullptr;
    int* ctile = nullptr;
    int* cstart = nullptr;
    int* arr = nullptr;
    int* tmp = nullptr;
    int* tmpid = nullptr;
    int* cell_tmp = nullptr;
    unsigned* list = nullptr;
    int* nlist = nullptr;
    double* WX = nullptr;
    int* wid = nullptr;
    int* wcstart = nullptr;
    double* partial = nullptr;
    EnergyRec* erec = nullptr;
    double* stage = nullptr;
    int* dbg = nullptr;
    // host
    std::vector<SysParams> hsp;
    std::vector<int> hchunk, htile, hbrick;
    int nchunk = 0, ntile = 0, tcap = 0, nbrick = 0, lds_atoms = 0, hmax = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    // captured replays for the current rebuild period: gexec[0] holds one
    // replay, gexec[1] holds kGraphReps; a call of any length launches the
    // large one and then the small one as often as needed, so calls of
    // different lengths never capture again
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int g_R = 0;
    bool dirty = true;
    bool timing = false;
    double t_exit_ms = 0.0;  // duration of a step launch whose workgroups all return at once
    // timing mode: one event pair around the R step launches of each replay,
    // with the steps that replay did (a replay cut short by an early rebuild
    // also holds launches that returned at once)
    struct TimedReplay {
        hipEvent_t a, b;
        int R;
        int done;
    };
    std::vector<TimedReplay> events;
    std::vector<void*> allocs;

    ~Pool() { release(); }

    void release()
    {
        if (stream) hipStreamSynchronize(stream);
        for (auto& g : gexec) {
            if (g) hipGraphExecDestroy(g);
            g = nullptr;
        }
        for (auto& e : events) {
            hipEventDestroy(e.a);
            hipEventDestroy(e.b);
        }
        events.clear();
        for (void* p : allocs) hipFree(p);
        allocs.clear();
        if (cap_stream) hipStreamDestroy(cap_stream);
        cap_stream = nullptr;
        if (own_stream && stream) hipStreamDestroy(stream);
        stream = nullptr;
    }

    template <typename T>
    int alloc(T** p, size_t count_elems)
    {
        size_t b = std::max<size_t>(count_elems, 1) * sizeof(T);
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, b);
        if (e != hipSuccess)
            return fail(PMD_ENOMEM, "hipMalloc of %zu bytes failed: %s", b, hipGetErrorString(e));
        allocs.push_back(q);
        bytes += b;
        *p = (T*)q;
        return PMD_OK;
    }

    PoolDev dev() const
    {
        PoolDev d{};
        d.sp = d_sp;
        d.st = d_st;
        d.chunk_sys = d_chunk;
        d.nchunk = nchunk;
        d.tile_sys = d_tile;
        d.ntile = ntile;
        d.brick_sys = d_brick;
        d.nbrick = nbrick;
        d.lds_atoms = lds_atoms;
        d.hmax = hmax;
        d.block = block;
        d.brick_order = brick_order;
        d.vt = vt;
        d.wt = wt;
        d.cap = cap;
        d.nbt = nbt;
        d.nslots = nslots;
        d.thermo = thermo;
        d.virial = virial;
        for (int b = 0; b < 2; ++b) {
            d.X[b] = X[b];
            d.V[b] = V[b];
            d.id[b] = id[b];
            d.L[b] = L[b];
        }
        d.A = A;
        d.lref = lref;
        d.cref = cref;
        d.cell_lin = cell_lin;
        d.count = count;
        d.clocal = clocal;
        d.ctile = ctile;
        d.cstart = cstart;
        d.arr = arr;
        d.tmp = tmp;
        d.tmpid = tmpid;
        d.cell_tmp = cell_tmp;
        d.list = list;
        d.nlist = nlist;
        d.WX = WX;
        d.wid = wid;
        d.wcstart = wcstart;
        d.partial = partial;
        d.erec = erec;
        return d;
    }
};

size_t lsize(int precision) { return precision == PMD_MIXED ? sizeof(f4) : sizeof(d4); }

// Bytes for capacities (used for footprint and budgets).
size_t pool_bytes(int precision, int vt, int wt, int ct, int wct, int nbt, int nslots, int cap,
                  int erings)
{
    size_t s = 0;
    s += 2 * 2 * 3 * (size_t)vt * 8 + 3 * (size_t)vt * 8;  // X, V double-buffered, A
    s += 2 * (size_t)vt * 4 + 2 * (size_t)vt * 4;          // id x2, cref, cell_lin
    s += (size_t)vt * 16;                                  // reference positions
    s += 2 * (size_t)(vt + wt) * lsize(precision);         // local coordinates x2
    s += 3 * (size_t)ct * 4 + 4 * (size_t)std::max(vt, wt) * 4;
    s += (size_t)vt * cap * 4 + (size_t)vt * 4;            // lists
    s += 3 * (size_t)wt * 8 + (size_t)wt * 4 + (size_t)wct * 4;
    s += 2 * kPartial * (size_t)nbt * 8 + (size_t)nslots * erings * sizeof(EnergyRec);
    s += 3 * (size_t)std::max(vt, wt) * 8 + (size_t)nslots * (sizeof(SysParams) + sizeof(SysState));
    return s;
}

int pool_allocate(Pool& p)
{
    const int vt = p.vt, wt = std::max(p.wt, 1);
    p.wt = wt;
    CHK(p.alloc(&p.d_sp, p.nslots));
    CHK(p.alloc(&p.d_st, p.nslots));
    CHK(p.alloc(&p.d_chunk, std::max(vt / kChunk, 1)));
    p.tcap = p.ct / kTile + p.nslots + 1;
    CHK(p.alloc(&p.d_tile, p.tcap));
    CHK(p.alloc(&p.ctile, p.tcap));
    CHK(p.alloc(&p.d_brick, std::max(p.nbt, 1)));
    for (int b = 0; b < 2; ++b) {
        CHK(p.alloc(&p.X[b], 3 * (size_t)vt));
        CHK(p.alloc(&p.V[b], 3 * (size_t)vt));
        CHK(p.alloc(&p.id[b], vt));
        void* l = nullptr;
        if (p.precision == PMD_MIXED) {
            f4* q;
            CHK(p.alloc(&q, (size_t)vt + wt));
            l = q;
        } else {
            d4* q;
            CHK(p.alloc(&q, (size_t)vt + wt));
            l = q;
        }
        p.L[b] = l;
    }
    CHK(p.alloc(&p.A, 3 * (size_t)vt));
    CHK(p.alloc(&p.lref, vt));
    CHK(p.alloc(&p.cref, vt));
    CHK(p.alloc(&p.cell_lin, vt));
    CHK(p.alloc(&p.count, p.ct));
    CHK(p.alloc(&p.clocal, p.ct));
    CHK(p.alloc(&p.cstart, p.ct));
    const int sc = std::max(vt, wt);
    CHK(p.alloc(&p.arr, sc));
    CHK(p.alloc(&p.tmp, sc));
    CHK(p.alloc(&p.tmpid, sc));
    CHK(p.alloc(&p.cell_tmp, sc));
    CHK(p.alloc(&p.list, (size_t)vt * p.cap));
    CHK(p.alloc(&p.nlist, vt));
    CHK(p.alloc(&p.WX, 3 * (size_t)wt));
    CHK(p.alloc(&p.wid, wt));
    CHK(p.alloc(&p.wcstart, std::max(p.wct, 1)));
    HIPCHK(hipMemset(p.wcstart, 0, sizeof(int) * (size_t)std::max(p.wct, 1)));
    CHK(p.alloc(&p.partial, 2 * kPartial * (size_t)std::max(p.nbt, 1)));
    CHK(p.alloc(&p.erec, (size_t)p.nslots * p.ering_cap));
    CHK(p.alloc(&p.stage, 3 * (size_t)sc));
    CHK(p.alloc(&p.dbg, 16));
    HIPCHK(hipMemset(p.count, 0, sizeof(int) * (size_t)p.ct));
    HIPCHK(hipMemset(p.d_st, 0, sizeof(SysState) * (size_t)p.nslots));
    HIPCHK(hipMemset(p.d_sp, 0, sizeof(SysParams) * (size_t)p.nslots));
    HIPCHK(hipMemset(p.nlist, 0, sizeof(int) * (size_t)vt));
    HIPCHK(hipMemset(p.lref, 0, sizeof(f4) * (size_t)vt));
    for (int b = 0; b < 2; ++b) {
        HIPCHK(hipMemset(p.L[b], 0, lsize(p.precision) * ((size_t)vt + wt)));
        HIPCHK(hipMemset(p.X[b], 0, sizeof(double) * 3 * (size_t)vt));
        HIPCHK(hipMemset(p.V[b], 0, sizeof(double) * 3 * (size_t)vt));
    }
    HIPCHK(hipMemset(p.A, 0, sizeof(double) * 3 * (size_t)vt));
    return PMD_OK;
}

// Resize the neighbour lists (content is rebuilt at the next rebuild).
int pool_grow_lists(Pool& p, int new_cap)
{
    HIPCHK(hipStreamSynchronize(p.stream));
    auto it = std::find(p.allocs.begin(), p.allocs.end(), (void*)p.list);
    size_t old = (size_t)p.vt * p.cap * 4;
    unsigned* q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)p.vt * new_cap * 4);
    if (e != hipSuccess) return fail(PMD_ENOMEM, "growing neighbour lists to %d failed", new_cap);
    if (it != p.allocs.end()) {
        hipFree(*it);
        *it = q;
    }
    p.bytes = p.bytes - old + (size_t)p.vt * new_cap * 4;
    p.list = q;
    p.cap = new_cap;
    p.dirty = true;
    return PMD_OK;
}

constexpr size_t kTileBytesMax = 60 * 1024;  // dynamic LDS of the staged halo tile

size_t tile_atom_bytes(int precision) { return (precision == PMD_MIXED ? sizeof(f4) : 3 * sizeof(double)) + 4; }

int halo_cells(const SysParams& sp)
{
    return (std::min(sp.bdim[0], sp.nc[0]) + 2) * (std::min(sp.bdim[1], sp.nc[1]) + 2) *
           (std::min(sp.bdim[2], sp.nc[2]) + 2);
}

// Lay out the chunk, scan-tile and brick tables from the per-slot parameters,
// size the staged LDS tile, and upload.
int pool_layout(Pool& p)
{
    p.hchunk.clear();
    p.htile.clear();
    p.hbrick.clear();
    int pb = 0, hmax = 0;
    double lds_want = 0;
    for (int s = 0; s < p.nslots; ++s) {
        SysParams& sp = p.hsp[s];
        if (!sp.active) {
            sp.choff = 0;
            sp.ntile = 0;
            sp.broff = 0;
            continue;
        }
        if (sp.voff % kPad || sp.vcap % kPad) return fail(PMD_EHIP, "misaligned system slots");
        // chunks follow slot order; chunks of released ranges map to -1
        sp.choff = sp.voff / kChunk;
        const int end = sp.choff + sp.vcap / kChunk;
        if ((int)p.hchunk.size() < end) p.hchunk.resize(end, -1);
        for (int c = sp.choff; c < end; ++c) p.hchunk[c] = s;
        sp.toff = (int)p.htile.size();
        sp.ntile = (sp.nkey + 2 + kTile - 1) / kTile;
        for (int t = 0; t < sp.ntile; ++t) p.htile.push_back(s);
        sp.broff = (int)p.hbrick.size();
        sp.pboff = pb;
        pb += sp.nbrick;
        for (int t = 0; t < sp.nbrick; ++t) p.hbrick.push_back(s);
        const int H = halo_cells(sp);
        hmax = std::max(hmax, H);
        // room for 1.3 times the mean occupancy (the brick shapes are chosen
        // to fit that); a denser halo grows the tile.  A larger margin takes
        // LDS that more resident workgroups could use
        const double occ = (double)sp.nv / sp.ncell;
        lds_want = std::max(lds_want, 1.3 * H * occ + 128.0);
    }
    p.nchunk = (int)p.hchunk.size();
    p.ntile = (int)p.htile.size();
    p.nbrick = (int)p.hbrick.size();
    p.thermo = 0;
    p.virial = 0;
    for (int s = 0; s < p.nslots; ++s)
        if (p.hsp[s].active) {
            if (p.hsp[s].thermo) p.thermo = 1;
            if (p.hsp[s].virial) p.virial = 1;
        }
    p.hmax = std::max(hmax, 1);
    const size_t ab = tile_atom_bytes(p.precision);
    const size_t ints = (size_t)(2 * p.hmax + 1) * 4;
    const int lds_max = (int)((kTileBytesMax - std::min(ints, kTileBytesMax / 2)) / ab);
    p.lds_atoms = std::max(std::min((int)lds_want, lds_max), std::min(p.lds_atoms, lds_max));
    if (p.nchunk > p.vt / kChunk) return fail(PMD_ENOMEM, "pool chunk table too small");
    if (p.ntile > p.tcap) return fail(PMD_ENOMEM, "pool tile table too small");
    if (pb > p.nbt) return fail(PMD_ENOMEM, "pool brick table too small (%d > %d)", pb, p.nbt);
    if (p.nchunk)
        HIPCHK(hipMemcpy(p.d_chunk, p.hchunk.data(), sizeof(int) * p.hchunk.size(), hipMemcpyHostToDevice));
    if (p.ntile)
        HIPCHK(hipMemcpy(p.d_tile, p.htile.data(), sizeof(int) * p.htile.size(), hipMemcpyHostToDevice));
    if (p.nbrick)
        HIPCHK(hipMemcpy(p.d_brick, p.hbrick.data(), sizeof(int) * p.hbrick.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p.d_sp, p.hsp.data(), sizeof(SysParams) * p.nslots, hipMemcpyHostToDevice));
    p.dirty = true;
    return PMD_OK;
}

// Staged-tile range of one atom's 27 neighbour cells in a brick of halo
// dimensions hx x hy x hz: from cell (-1, -1, -1) to cell (1, 1, 1) in the
// halo's x-fastest order (two planes, two rows and three cells of the halo).
int span_cells(int hx, int hy) { return 2 * hx * hy + 2 * hx + 3; }

// Brick shape: the largest brick (at most 8 cells per axis) whose expected
// atom count fits `target`, whose halo box fits the LDS tile and whose
// neighbourhood range fits a vapour list entry's index field, both at 1.3
// times the mean occupancy (room for density fluctuations); near-cubic
// shapes (smallest halo per cell) are preferred.  `target` scales with the
// workgroup size.
void choose_bricks(SysParams& sp, double target, size_t atom_bytes)
{
    const double occ = std::max((double)sp.nv / sp.ncell, 1e-3);
    int best[3] = {1, 1, 1};
    double best_score = -1.0;
    for (int bx = 1; bx <= std::min(8, sp.nc[0]); ++bx)
        for (int by = 1; by <= std::min(8, sp.nc[1]); ++by)
            for (int bz = 1; bz <= std::min(8, sp.nc[2]); ++bz) {
                const int P = bx * by * bz;
                if (P * occ > target && P > 1) continue;
                const int H = (bx + 2) * (by + 2) * (bz + 2);
                const double fit = (double)(kTileBytesMax - (size_t)(2 * H + 1) * 4) / atom_bytes;
                if (1.3 * H * occ > fit && P > 1) continue;
                if (1.3 * span_cells(bx + 2, by + 2) * occ > kRelMask + 1 && P > 1) continue;
                const double halo = (double)(bx + 2) * (by + 2) * (bz + 2) / P;
                const double score = P - 0.01 * halo;
                if (score > best_score) {
                    best_score = score;
                    best[0] = bx;
                    best[1] = by;
                    best[2] = bz;
                }
            }
    sp.bcells = 1;
    sp.nbrick = 1;
    for (int k = 0; k < 3; ++k) {
        sp.bdim[k] = best[k];
        sp.nbk[k] = (sp.nc[k] + best[k] - 1) / best[k];
        sp.bcells *= best[k];
        sp.nbrick *= sp.nbk[k];
        sp.inv_bdim[k] = 1.0 / best[k];
    }
    sp.inv_nbk0 = 1.0 / sp.nbk[0];
    sp.inv_nbk01 = 1.0 / ((double)sp.nbk[0] * sp.nbk[1]);
    sp.inv_bcells = 1.0 / sp.bcells;
    sp.nkey = sp.nbrick * sp.bcells;
}

// Upper bound of nkey + 2 over every brick shape choose_bricks can pick.
int key_capacity(const Grid& g) { return (g.nc[0] + 7) * (g.nc[1] + 7) * (g.nc[2] + 7) + 2; }
int key_capacity(const SysParams& sp) { return (sp.nc[0] + 7) * (sp.nc[1] + 7) * (sp.nc[2] + 7) + 2; }

// A brick's halo overflowed the LDS tile: grow the tile up to its limit,
// then shrink the system's bricks.  An atom's neighbourhood range that
// overflowed a vapour list entry's index field (status ST_SPAN) shrinks the
// bricks at once.  The next rebuild uses the new layout.
int pool_fix_tile(Pool& p, int slot, int status)
{
    const size_t ab = tile_atom_bytes(p.precision);
    const size_t ints = (size_t)(2 * p.hmax + 1) * 4;
    const int lds_max = (int)((kTileBytesMax - std::min(ints, kTileBytesMax / 2)) / ab);
    if (p.lds_atoms < lds_max && !(status & ST_SPAN)) {
        p.lds_atoms = std::min(lds_max, 2 * p.lds_atoms);
        p.dirty = true;
        return PMD_OK;
    }
    SysParams& sp = p.hsp[slot];
    if (sp.bcells == 1) return fail(PMD_ENOMEM, "a single cell's neighbourhood exceeds the LDS tile");
    const double occ = std::max((double)sp.nv / sp.ncell, 1e-3);
    choose_bricks(sp, 0.5 * sp.bcells * occ, ab);
    return pool_layout(p);
}

void fill_sys_params(SysParams& sp, const pmd_params& p, const Grid& g, const pmd_tuning& t,
                     int nv, int nw, double brick_target = 0.0)
{
    for (int k = 0; k < 3; ++k) {
        sp.L[k] = p.box[k];
        sp.invL[k] = 1.0 / p.box[k];
        sp.nc[k] = g.nc[k];
        sp.h[k] = g.h[k];
        sp.inv_h[k] = (double)g.nc[k] / p.box[k];
    }
    sp.ncell = g.nc[0] * g.nc[1] * g.nc[2];
    sp.nv = nv;
    sp.vcap = round_up(std::max(nv, 1), kPad);
    sp.nw = nw;
    const double s2 = p.sigma * p.sigma, s6 = s2 * s2 * s2;
    const double w2 = p.sigma_wall * p.sigma_wall, w6 = w2 * w2 * w2;
    sp.A = 4.0 * p.epsilon * s6 * s6;
    sp.B = 4.0 * p.epsilon * s6;
    sp.Aw = 4.0 * p.epsilon_wall * w6 * w6;
    sp.Bw = 4.0 * p.epsilon_wall * w6;
    const double rc2 = p.cutoff * p.cutoff, irc6 = 1.0 / (rc2 * rc2 * rc2);
    sp.uc = sp.A * irc6 * irc6 - sp.B * irc6;
    sp.ucw = sp.Aw * irc6 * irc6 - sp.Bw * irc6;
    sp.rc2 = rc2;
    const double rl = p.cutoff + t.skin;
    sp.rl2 = rl * rl;
    const double rw = p.cutoff + 0.5 * t.skin;
    sp.rw2 = rw * rw;
    sp.dt = p.dt;
    sp.mass = p.mass;
    sp.inv_mass = 1.0 / p.mass;
    sp.half_skin = (float)(0.5 * t.skin * (1.0 - 1e-3));
    sp.energy_every = t.energy_every;
    sp.thermo = p.thermostat_tau > 0 ? 1 : 0;
    sp.virial = t.virial ? 1 : 0;
    sp.tau_t = p.thermostat_tau;
    sp.t0 = p.thermostat_t0;
    sp.dof = nv > 1 ? 3.0 * nv - 3.0 : 3.0;
    sp.active = 1;
    choose_bricks(sp, brick_target > 0 ? brick_target : t.brick_atoms > 0 ? t.brick_atoms : 0.8 * t.block,
                  tile_atom_bytes(p.precision));
}

constexpr int kGraphReps = 8;

// Capture the two graphs of the rebuild period R: one replay of [rebuild,
// R steps, commit], and kGraphReps of them.
int pool_capture(Pool& p, int R)
{
    GPU_LOCK;
    if (p.gexec[0] || p.gexec[1]) {
        // launches of the old graphs may still be queued on the stream
        HIPCHK(hipStreamSynchronize(p.stream));
        for (auto& g : p.gexec) {
            if (g) HIPCHK(hipGraphExecDestroy(g));
            g = nullptr;
        }
    }
    if (!p.cap_stream) HIPCHK(hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking));
    const PoolDev d = p.dev();
    for (int q = 0; q < 2; ++q) {
        const int reps = q == 0 ? 1 : kGraphReps;
        HIPCHK(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
        for (int r = 0; r < reps; ++r) {
            launch_rebuild(d, p.nslots, p.precision, p.cap_stream);
            for (int k = 0; k < R; ++k) launch_step(d, k, p.precision, p.cap_stream, nullptr, nullptr);
            launch_commit(d, p.nslots, R, p.cap_stream);
        }
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamEndCapture(p.cap_stream, &g));
        hipError_t e = hipGraphInstantiate(&p.gexec[q], g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        HIPCHK(e);
    }
    p.g_R = R;
    p.dirty = false;
    return PMD_OK;
}

int read_state(Pool& p, int slot, SysState* out)
{
    HIPCHK(hipMemcpyAsync(out, p.d_st + slot, sizeof(SysState), hipMemcpyDeviceToHost, p.stream));
    HIPCHK(hipStreamSynchronize(p.stream));
    return PMD_OK;
}

// Queue `replays` repetitions of [rebuild, R steps].
int pool_enqueue(Pool& p, int R, int use_graph, int64_t replays)
{
    if (replays <= 0) return PMD_OK;
    const PoolDev d = p.dev();
    if (use_graph && !p.timing) {
        if (p.dirty || !p.gexec[0] || !p.gexec[1] || p.g_R != R) CHK(pool_capture(p, R));
        for (int64_t g = 0; g < replays / kGraphReps; ++g) HIPCHK(hipGraphLaunch(p.gexec[1], p.stream));
        for (int64_t g = 0; g < replays % kGraphReps; ++g) HIPCHK(hipGraphLaunch(p.gexec[0], p.stream));
        return PMD_OK;
    }
    for (int64_t r = 0; r < replays; ++r) {
        HIPCHK(launch_rebuild(d, p.nslots, p.precision, p.stream));
        Pool::TimedReplay t{nullptr, nullptr, R, 0};
        long long before = 0;
        if (p.timing) {
            // the timed pool holds one system (slot 0); the step count before
            // and after the replay gives the steps it did
            SysState st;
            CHK(read_state(p, 0, &st));
            before = st.step;
            // no system-scope fence on the timing events: the kernels'
            // duration is wanted, not that of a cache flush behind them
            HIPCHK(hipEventCreateWithFlags(&t.a, hipEventDisableSystemFence));
            HIPCHK(hipEventCreateWithFlags(&t.b, hipEventDisableSystemFence));
            HIPCHK(hipEventRecord(t.a, p.stream));
        }
        for (int k = 0; k < R; ++k) HIPCHK(launch_step(d, k, p.precision, p.stream, nullptr, nullptr));
        if (p.timing) HIPCHK(hipEventRecord(t.b, p.stream));
        HIPCHK(launch_commit(d, p.nslots, R, p.stream));
        if (p.timing) {
            SysState st;
            CHK(read_state(p, 0, &st));
            t.done = (int)(st.step - before);
            p.events.push_back(t);
        }
    }
    return PMD_OK;
}


}  // namespace

// ---------------------------------------------------------------------------
// Handles
// ---------------------------------------------------------------------------

struct pmd_system {
    std::unique_ptr<Pool> own;  // stand-alone pool (null while admitted to a batch)
    Pool* pool = nullptr;       // pool holding the state
    int slot = 0;
    pmd_batch* batch = nullptr;
    int64_t nv = 0, nw = 0;
    pmd_params params{};
    pmd_pore pore{};
    pmd_tuning tuning{};
    Grid grid{};
};

// A copy of the per-system state taken after a chunk of steps: queued on
// the batch's stream behind the chunk, into pinned host memory, with an
// event, so that the host can learn which systems finished while later
// chunks run.
struct StateSnap {
    hipEvent_t ev = nullptr;
    SysState* host = nullptr;  // [max_slots], pinned
    long long seq = -1;        // issue number; -1 = unused
    bool done = false;         // its event has completed
};

constexpr int kSnaps = 4;

struct pmd_batch {
    std::unique_ptr<Pool> pool;
    size_t budget = 0;
    int max_slots = 0;
    std::vector<pmd_system*> resident;  // by slot
    std::vector<int64_t> steps_wanted;
    hipStream_t user_stream = nullptr;
    int R = 10;
    pmd_tuning tuning{};
    bool configured = false;
    StateSnap snap[kSnaps];
    long long snap_seq = 0;             // next issue number
    std::vector<long long> admit_seq;   // by slot: first snapshot that can see its system
};

namespace {

int sys_sync(pmd_system* s)
{
    Pool& p = *s->pool;
    for (int iter = 0; iter < 100000; ++iter) {
        SysState st;
        CHK(read_state(p, s->slot, &st));
        if (st.status & ST_NONFINITE)
            return fail(PMD_ENUMERIC, "non-finite force or position at step %lld", (long long)st.step);
        if (st.remaining <= 0) return PMD_OK;
        if (st.status & ST_TILE) {
            CHK(pool_fix_tile(p, s->slot, st.status));
        } else if (st.status & ST_OVERFLOW) {
            const int need = round_up(std::max(st.max_nbr + st.max_nbr / 4 + 8, p.cap + 16), 16);
            if (need > 4096) return fail(PMD_ENOMEM, "neighbour list needs %d entries per atom", need);
            CHK(pool_grow_lists(p, need));
            s->tuning.list_cap = need;
        }
        if (st.status & ST_STALL) HIPCHK(launch_set_run(p.dev(), s->slot, 0, ST_STALL, p.stream));
        const int R = s->tuning.rebin_every;
        CHK(pool_enqueue(p, R, s->tuning.use_graph, (st.remaining + R - 1) / R));
    }
    return fail(PMD_EHIP, "step driver made no progress");
}

int check_atoms(const pmd_params& p, int64_t n, const double* pos, const double* vel)
{
    for (int64_t i = 0; i < 3 * n; ++i) {
        const int k = (int)(i % 3);
        if (!std::isfinite(pos[i]) || !std::isfinite(vel[i]))
            return fail(PMD_EINVAL, "non-finite input at atom %lld", (long long)(i / 3));
        if (pos[i] < 0.0 || pos[i] >= p.box[k])
            return fail(PMD_EINVAL, "position of atom %lld outside [0, L)", (long long)(i / 3));
    }
    return PMD_OK;
}

// Load caller-order positions and velocities into the system's slot, reset
// its step counter and energy history, and evaluate the forces at the loaded
// positions (bin, build lists, one force pass), growing the neighbour lists or
// the LDS tile if the first attempt reports that they are too small.
int load_state(pmd_system* sys, const double* pos, const double* vel, int64_t step)
{
    Pool& q = *sys->pool;
    const int slot = sys->slot;
    const int64_t n = sys->nv;
    double* dpos = nullptr;
    HIPCHK(hipMalloc(&dpos, sizeof(double) * 6 * (size_t)n));
    hipError_t e = hipMemcpyAsync(dpos, pos, sizeof(double) * 3 * n, hipMemcpyHostToDevice, q.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dpos + 3 * n, vel, sizeof(double) * 3 * n, hipMemcpyHostToDevice, q.stream);
    if (e == hipSuccess)
        e = launch_copy_in(q.dev(), slot, dpos, dpos + 3 * n, (int)n, q.hsp[slot].vcap, q.stream);
    if (e == hipSuccess) e = launch_reset_state(q.dev(), slot, (long long)step, q.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(q.stream);
    hipFree(dpos);
    HIPCHK(e);
    for (int attempt = 0; attempt < 8; ++attempt) {
        HIPCHK(launch_rebuild(q.dev(), q.nslots, q.precision, q.stream));
        HIPCHK(launch_step(q.dev(), 0, q.precision, q.stream, nullptr, nullptr));
        HIPCHK(launch_commit(q.dev(), q.nslots, 1, q.stream));
        SysState st;
        CHK(read_state(q, slot, &st));
        if (st.status & ST_NONFINITE) return fail(PMD_ENUMERIC, "non-finite initial forces");
        if (st.phase == PH_REST) return PMD_OK;
        if (st.status & ST_TILE) {
            CHK(pool_fix_tile(q, slot, st.status));
        } else if (st.status & ST_OVERFLOW) {
            const int need = round_up(std::max(st.max_nbr + st.max_nbr / 4 + 8, q.cap), 16);
            if (need > 4096) return fail(PMD_ENOMEM, "neighbour list needs %d entries", need);
            CHK(pool_grow_lists(q, need));
            sys->tuning.list_cap = need;
        }
        if (st.status & ST_STALL) HIPCHK(launch_set_run(q.dev(), slot, 0, ST_STALL, q.stream));
    }
    return fail(PMD_EHIP, "initial force evaluation did not complete");
}

int check_free(pmd_system* s)
{
    if (!s) return fail(PMD_EINVAL, "NULL system");
    if (s->batch) return fail(PMD_ESTATE, "system is resident in a batch; release it first");
    return PMD_OK;
}

}  // namespace

namespace {

// Copy one system's state from (src, sslot) into (dst, dslot).  dst.hsp[dslot]
// must already hold the destination offsets.  Vapour order, velocities and
// accelerations are copied as they are; the neighbour lists and cell tables
// are rebuilt by the next replay's rebuild, and wall cell offsets are rebased.
int move_system(Pool& src, int sslot, Pool& dst, int dslot)
{
    HIPCHK(hipStreamSynchronize(src.stream));
    HIPCHK(hipStreamSynchronize(dst.stream));
    const SysParams& a = src.hsp[sslot];
    const SysParams& b = dst.hsp[dslot];
    SysState st;
    HIPCHK(hipMemcpy(&st, src.d_st + sslot, sizeof(SysState), hipMemcpyDeviceToHost));
    const int sb = st.sbuf;
    const size_t nv = (size_t)a.vcap;
    for (int k = 0; k < 3; ++k) {
        HIPCHK(hipMemcpy(dst.X[0] + (size_t)k * dst.vt + b.voff, src.X[sb] + (size_t)k * src.vt + a.voff,
                         nv * 8, hipMemcpyDeviceToDevice));
        HIPCHK(hipMemcpy(dst.V[0] + (size_t)k * dst.vt + b.voff, src.V[sb] + (size_t)k * src.vt + a.voff,
                         nv * 8, hipMemcpyDeviceToDevice));
        HIPCHK(hipMemcpy(dst.A + (size_t)k * dst.vt + b.voff, src.A + (size_t)k * src.vt + a.voff,
                         nv * 8, hipMemcpyDeviceToDevice));
        if (a.nw)
            HIPCHK(hipMemcpy(dst.WX + (size_t)k * dst.wt + b.woff, src.WX + (size_t)k * src.wt + a.woff,
                             (size_t)a.nw * 8, hipMemcpyDeviceToDevice));
    }
    HIPCHK(hipMemcpy(dst.id[0] + b.voff, src.id[st.ibuf] + a.voff, nv * 4, hipMemcpyDeviceToDevice));
    HIPCHK(hipMemcpy(dst.lref + b.voff, src.lref + a.voff, nv * sizeof(f4), hipMemcpyDeviceToDevice));
    HIPCHK(hipMemcpy(dst.cref + b.voff, src.cref + a.voff, nv * 4, hipMemcpyDeviceToDevice));
    HIPCHK(hipMemcpy(dst.cell_lin + b.voff, src.cell_lin + a.voff, nv * 4, hipMemcpyDeviceToDevice));
    HIPCHK(hipMemset(dst.nlist + b.voff, 0, nv * 4));
    const size_t ls = lsize(dst.precision);
    if (a.nw) {
        HIPCHK(hipMemcpy(dst.wid + b.woff, src.wid + a.woff, (size_t)a.nw * 4, hipMemcpyDeviceToDevice));
        for (int q = 0; q < 2; ++q)
            HIPCHK(hipMemcpy((char*)dst.L[q] + ((size_t)dst.vt + b.woff) * ls,
                             (const char*)src.L[0] + ((size_t)src.vt + a.woff) * ls, (size_t)a.nw * ls,
                             hipMemcpyDeviceToDevice));
    }
    std::vector<int> wcs((size_t)a.ncell + 1);
    HIPCHK(hipMemcpy(wcs.data(), src.wcstart + a.wcoff, sizeof(int) * wcs.size(), hipMemcpyDeviceToHost));
    for (auto& v : wcs) v = v - a.woff + b.woff;
    HIPCHK(hipMemcpy(dst.wcstart + b.wcoff, wcs.data(), sizeof(int) * wcs.size(), hipMemcpyHostToDevice));
    // vapour cell tables: copy so that debug readbacks of a resting system stay valid
    std::vector<int> cs((size_t)a.nkey + 2);
    HIPCHK(hipMemcpy(cs.data(), src.cstart + a.coff, sizeof(int) * cs.size(), hipMemcpyDeviceToHost));
    for (auto& v : cs) v = v - a.voff + b.voff;
    HIPCHK(hipMemcpy(dst.cstart + b.coff, cs.data(), sizeof(int) * cs.size(), hipMemcpyHostToDevice));
    // energy records
    const int nrec = std::min(a.ering_cap, b.ering_cap);
    std::vector<EnergyRec> rec((size_t)a.ering_cap);
    HIPCHK(hipMemcpy(rec.data(), src.erec + a.ering_off, sizeof(EnergyRec) * rec.size(), hipMemcpyDeviceToHost));
    std::vector<EnergyRec> out((size_t)b.ering_cap);
    const int have = std::min(st.nrec, a.ering_cap);
    const int keep = std::min(have, nrec);
    for (int r = 0; r < keep; ++r) {
        const int from = (st.nrec - keep + r) % a.ering_cap;
        out[(size_t)((st.nrec - keep + r) % b.ering_cap)] = rec[(size_t)from];
    }
    HIPCHK(hipMemcpy(dst.erec + b.ering_off, out.data(), sizeof(EnergyRec) * out.size(), hipMemcpyHostToDevice));
    SysState nst = st;
    nst.sbuf = 0;
    nst.sbuf_prev = 0;
    nst.ibuf = 0;
    nst.ibuf_prev = 0;
    nst.status_next = 0;
    HIPCHK(hipMemcpy(dst.d_st + dslot, &nst, sizeof(SysState), hipMemcpyHostToDevice));
    return PMD_OK;
}

struct Needs {
    int vt = 0, wt = 0, ct = 0, wct = 0, nbt = 0;
};

Needs needs_of(const SysParams& sp)
{
    Needs n;
    n.vt = sp.vcap;
    n.wt = sp.nw;
    n.ct = key_capacity(sp);
    n.wct = sp.ncell + 1;
    n.nbt = key_capacity(sp);
    return n;
}

constexpr int kBatchErings = 4096;

size_t system_bytes(int precision, const SysParams& sp, int cap)
{
    const Needs n = needs_of(sp);
    return pool_bytes(precision, n.vt, n.wt, n.ct, n.wct, n.nbt, 1, cap, kBatchErings);
}

// Make a stand-alone single-slot pool for a system leaving a batch.
int make_single_pool(const Pool& like, const SysParams& sp_in, hipStream_t stream, bool own_stream,
                     std::unique_ptr<Pool>* out)
{
    auto pool = std::make_unique<Pool>();
    Pool& p = *pool;
    p.precision = like.precision;
    p.block = like.block;
    p.brick_order = like.brick_order;
    p.cap = like.cap;
    p.nslots = 1;
    p.ering_cap = kDefaultErings;
    SysParams sp = sp_in;
    sp.voff = sp.woff = sp.coff = sp.wcoff = sp.ering_off = 0;
    sp.ering_cap = p.ering_cap;
    p.vt = sp.vcap;
    p.wt = std::max(sp.nw, 1);
    p.ct = key_capacity(sp);
    p.wct = sp.ncell + 1;
    p.nbt = key_capacity(sp);
    p.stream = stream;
    p.own_stream = own_stream;
    if (!p.stream) {
        HIPCHK(hipStreamCreateWithFlags(&p.stream, hipStreamNonBlocking));
        p.own_stream = true;
    }
    CHK(pool_allocate(p));
    p.hsp.assign(1, sp);
    CHK(pool_layout(p));
    *out = std::move(pool);
    return PMD_OK;
}

// A wall neighbour-list entry holds the wall's slot in the whole pool in
// kIndexBits bits (the neighbour cell's offset code sits above them), so a
// pool may hold at most kIndexMask wall slots; past that, slots would spill
// into the code bits and name the wrong wall.
constexpr int64_t kMaxPoolWalls = (int64_t)kIndexMask;

int check_pool_walls(int64_t resident_walls, int64_t new_walls)
{
    if (resident_walls < 0 || new_walls < 0) return fail(PMD_EINVAL, "negative wall count");
    if (resident_walls + new_walls > kMaxPoolWalls)
        return fail(PMD_EAGAIN, "wall slots would exceed %lld (%lld resident + %lld new)",
                    (long long)kMaxPoolWalls, (long long)resident_walls, (long long)new_walls);
    return PMD_OK;
}

// Rebuild the batch pool with capacity for its residents plus `extra`, moving
// every resident system into tightly packed ranges.
int batch_repack(pmd_batch* b, const Needs& extra, int extra_cap)
{
    Pool* old = b->pool.get();
    Needs tot = extra;
    for (size_t s = 0; s < b->resident.size(); ++s)
        if (b->resident[s]) {
            const Needs n = needs_of(old->hsp[s]);
            tot.vt += n.vt;
            tot.wt += n.wt;
            tot.ct += n.ct;
            tot.wct += n.wct;
            tot.nbt += n.nbt;
        }
    auto np = std::make_unique<Pool>();
    Pool& p = *np;
    p.precision = old->precision;
    p.block = old->block;
    p.brick_order = old->brick_order;
    p.cap = std::max(old->cap, extra_cap);
    p.nslots = b->max_slots;
    p.ering_cap = kBatchErings;
    // growth room so that a stream of admissions does not repack every time
    CHK(check_pool_walls(tot.wt - extra.wt, extra.wt));
    p.vt = round_up((int)(tot.vt * 1.25) + kPad, kPad);
    // growth room, but never past the slots a list entry can name
    p.wt = (int)std::min<int64_t>((int64_t)(tot.wt * 1.25) + 1, kMaxPoolWalls);
    p.ct = (int)(tot.ct * 1.25) + 8;
    p.wct = (int)(tot.wct * 1.25) + 8;
    p.nbt = (int)(tot.nbt * 1.25) + 8;
    if (b->budget) {
        size_t want = pool_bytes(p.precision, p.vt, p.wt, p.ct, p.wct, p.nbt, p.nslots, p.cap, p.ering_cap);
        if (want > b->budget) {
            p.vt = round_up(tot.vt, kPad);
            p.wt = std::max(tot.wt, 1);
            p.ct = tot.ct;
            p.wct = tot.wct;
            p.nbt = tot.nbt;
        }
    }
    p.stream = old->stream;
    p.own_stream = false;
    CHK(pool_allocate(p));
    p.hsp.assign(p.nslots, SysParams{});
    int vo = 0, wo = 0, co = 0, wco = 0;
    for (size_t s = 0; s < b->resident.size(); ++s) {
        if (!b->resident[s]) continue;
        SysParams sp = old->hsp[s];
        sp.voff = vo;
        sp.woff = wo;
        sp.coff = co;
        sp.wcoff = wco;
        sp.ering_off = (int)s * p.ering_cap;
        sp.ering_cap = p.ering_cap;
        const Needs n = needs_of(sp);
        vo += n.vt;
        wo += n.wt;
        co += n.ct;
        wco += n.wct;
        p.hsp[s] = sp;
    }
    CHK(pool_layout(p));
    for (size_t s = 0; s < b->resident.size(); ++s)
        if (b->resident[s]) CHK(move_system(*old, (int)s, p, (int)s));
    CHK(pool_layout(p));
    // hand the stream over: the old pool must not destroy it
    const bool owned = old->own_stream;
    old->own_stream = false;
    old->stream = nullptr;
    p.own_stream = owned;
    b->pool = std::move(np);
    for (auto* sys : b->resident)
        if (sys) sys->pool = b->pool.get();
    return PMD_OK;
}

// Next free ranges after the highest resident range (bump allocation).
bool batch_bump(pmd_batch* b, const Needs& n, SysParams* sp)
{
    Pool& p = *b->pool;
    int vo = 0, wo = 0, co = 0, wco = 0;
    for (size_t s = 0; s < b->resident.size(); ++s) {
        if (!b->resident[s]) continue;
        const SysParams& q = p.hsp[s];
        const Needs m = needs_of(q);
        vo = std::max(vo, q.voff + m.vt);
        wo = std::max(wo, q.woff + m.wt);
        co = std::max(co, q.coff + m.ct);
        wco = std::max(wco, q.wcoff + m.wct);
    }
    int nbt = 0;
    for (size_t s = 0; s < b->resident.size(); ++s)
        if (b->resident[s]) nbt += needs_of(p.hsp[s]).nbt;
    if ((int64_t)wo + n.wt > kMaxPoolWalls) return false;
    if (vo + n.vt > p.vt || wo + n.wt > p.wt || co + n.ct > p.ct || wco + n.wct > p.wct ||
        nbt + n.nbt > p.nbt)
        return false;
    sp->voff = vo;
    sp->woff = wo;
    sp->coff = co;
    sp->wcoff = wco;
    return true;
}

size_t batch_used(pmd_batch* b)
{
    size_t u = 0;
    for (size_t s = 0; s < b->resident.size(); ++s)
        if (b->resident[s]) u += system_bytes(b->pool->precision, b->pool->hsp[s], b->pool->cap);
    return u;
}

}  // namespace

extern "C" {

const char* pmd_last_error(void) { return g_err.c_str(); }

int pmd_version(void) { return 100; }

int pmd_pore_volume(const pmd_params* params, const pmd_pore* pore, double* volume)
{
    try {
        CHK(check_params(params, pore));
        if (!volume) return fail(PMD_EINVAL, "volume must not be NULL");
        *volume = pore_void_volume(*params, *pore);
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_batch_wall_room(int64_t resident_walls, int64_t new_walls)
{
    try {
        return check_pool_walls(resident_walls, new_walls);
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_allpairs_forces(int precision, int64_t n, const double* x_dev, const double box[3],
                        double epsilon, double sigma, double* f_dev, double* u_dev, double* e_dev,
                        void* stream)
{
    try {
        if (precision != 1 && precision != 2) return fail(PMD_EINVAL, "precision must be 1 or 2 (got %d)", precision);
        if (n < 0 || n > (int64_t)1 << 24) return fail(PMD_EINVAL, "n must be in 0..2^24 (got %lld)", (long long)n);
        if (!box || !e_dev || !u_dev || (n > 0 && (!x_dev || !f_dev)))
            return fail(PMD_EINVAL, "need box, e_dev, u_dev, and x_dev, f_dev for n > 0");
        if (!std::isfinite(sigma) || sigma <= 0 || !std::isfinite(epsilon))
            return fail(PMD_EINVAL, "need a finite sigma > 0 and a finite epsilon");
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(box[k])) return fail(PMD_EINVAL, "box edges must be finite");
        HIPCHK(launch_allpairs(precision, (int)n, x_dev, box, epsilon, sigma, f_dev, u_dev, e_dev,
                               (hipStream_t)stream));
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int64_t pmd_pm_record_rows(int64_t nsteps, int64_t energy_every)
{
    if (nsteps < 0) return 0;
    int64_t rows = 1 + (energy_every > 0 ? nsteps / energy_every : 0);
    if (nsteps > 0 && (energy_every <= 0 || nsteps % energy_every != 0)) ++rows;
    return rows;
}

}  // extern "C"

namespace {

static_assert(sizeof(PmRecord) == sizeof(pmd_pm_record), "record layouts differ");

// Checks shared by the pore-model entry points; fills the kernel arguments.
int pm_check(const pmd_pm_model* m, int64_t n, const double* x_dev, const double* v_dev,
             int64_t nsteps, int64_t energy_every, const pmd_pm_record* rec_dev, int64_t rec_cap,
             int64_t n_max, PmArgs* out)
{
    if (!m) return fail(PMD_EINVAL, "model must not be NULL");
    if (m->dim != 2 && m->dim != 3) return fail(PMD_EINVAL, "dim must be 2 or 3 (got %d)", m->dim);
    if (m->precision != 1 && m->precision != 2)
        return fail(PMD_EINVAL, "precision must be 1 or 2 (got %d)", m->precision);
    if (n < 0 || n > n_max) return fail(PMD_EINVAL, "n must be in 0..%lld (got %lld)", (long long)n_max, (long long)n);
    if (n > 0 && (!x_dev || !v_dev)) return fail(PMD_EINVAL, "need x_dev and v_dev for n > 0");
    if (nsteps < 0 || nsteps > ((int64_t)1 << 40)) return fail(PMD_EINVAL, "nsteps out of range");
    if (energy_every < 0) return fail(PMD_EINVAL, "energy_every must be >= 0");
    if (rec_dev && rec_cap < pmd_pm_record_rows(nsteps, energy_every))
        return fail(PMD_EINVAL, "rec_cap %lld < %lld records", (long long)rec_cap,
                    (long long)pmd_pm_record_rows(nsteps, energy_every));
    const double len[3] = {m->lx, m->ly, m->dim == 3 ? m->lz : 1.0};
    for (double l : len)
        if (!std::isfinite(l) || l <= 0.0) return fail(PMD_EINVAL, "pore edges must be finite and > 0");
    if (!std::isfinite(m->k) || m->k <= 0.0) return fail(PMD_EINVAL, "k must be finite and > 0");
    if (!std::isfinite(m->sigma) || m->sigma <= 0.0 || !std::isfinite(m->epsilon) ||
        !std::isfinite(m->mass) || m->mass <= 0.0 || !std::isfinite(m->dt) || m->dt <= 0.0)
        return fail(PMD_EINVAL, "need finite sigma, mass, dt > 0 and a finite epsilon");
    if (!std::isfinite(m->thermostat_tau) || m->thermostat_tau < 0.0)
        return fail(PMD_EINVAL, "thermostat_tau must be finite and >= 0");
    if (m->thermostat_tau > 0.0 &&
        (m->thermostat_tau < m->dt || !std::isfinite(m->thermostat_t0) || m->thermostat_t0 <= 0.0))
        return fail(PMD_EINVAL, "a thermostat needs tau >= dt and t0 > 0");
    PmArgs a{};
    a.n = (int)n;
    a.dim = m->dim;
    a.precision = m->precision;
    a.lx = m->lx;
    a.ly = m->ly;
    a.lz = m->dim == 3 ? m->lz : 0.0;
    a.k = m->k;
    a.sig2 = m->sigma * m->sigma;
    a.eps4 = 4.0 * m->epsilon;
    a.eps24 = 24.0 * m->epsilon;
    a.mass = m->mass;
    a.inv_mass = 1.0 / m->mass;
    a.dt = m->dt;
    a.hdt = 0.5 * m->dt;
    a.tau = m->thermostat_tau;
    a.t0 = m->thermostat_t0;
    a.vol = m->lx * m->ly * (m->dim == 3 ? m->lz : 1.0);
    *out = a;
    return PMD_OK;
}

constexpr int64_t kPmMaxAtoms = (int64_t)1 << 20;

}  // namespace

extern "C" {

int pmd_pm_run(const pmd_pm_model* model, int64_t n, double* x_dev, double* v_dev, double* a_dev,
               int64_t nsteps, int64_t energy_every, pmd_pm_record* rec_dev, int64_t rec_cap,
               void* stream)
{
    try {
        PmArgs a;
        CHK(pm_check(model, n, x_dev, v_dev, nsteps, energy_every, rec_dev, rec_cap, kPmMaxAtoms, &a));
        const hipStream_t s = (hipStream_t)stream;
        void* ws = nullptr;
        HIPCHK(hipMallocAsync(&ws, sizeof(double) * pm_work_doubles(n, a.dim), s));
        PmWork w = pm_work_at((double*)ws, n, a.dim);
        if (a_dev) w.acc = a_dev;  // the caller's buffer serves as the accelerations
        const hipError_t e = launch_pm_run(a, x_dev, v_dev, w, nsteps, energy_every,
                                           (PmRecord*)rec_dev, s);
        const hipError_t f = hipFreeAsync(ws, s);
        HIPCHK(e);
        HIPCHK(f);
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_pm_run_noalloc(const pmd_pm_model* model, int64_t n, double* x_dev, double* v_dev,
                       double* a_dev, int64_t nsteps, int64_t energy_every, pmd_pm_record* rec_dev,
                       int64_t rec_cap, void* stream)
{
    try {
        PmArgs a;
        if (n > kPmScratchAtoms)
            return fail(PMD_EINVAL, "n = %lld exceeds the static working memory (%lld molecules)",
                        (long long)n, (long long)kPmScratchAtoms);
        CHK(pm_check(model, n, x_dev, v_dev, nsteps, energy_every, rec_dev, rec_cap, kPmScratchAtoms,
                     &a));
        double* base = nullptr;
        HIPCHK(pm_scratch_ptr(&base));
        PmWork w = pm_work_at(base, n, a.dim);
        if (a_dev) w.acc = a_dev;
        HIPCHK(launch_pm_run(a, x_dev, v_dev, w, nsteps, energy_every, (PmRecord*)rec_dev,
                             (hipStream_t)stream));
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_wall_count(const pmd_params* params, const pmd_pore* pore, int64_t* n_wall)
{
    try {
        CHK(check_params(params, pore));
        if (!n_wall) return fail(PMD_EINVAL, "n_wall must not be NULL");
        *n_wall = host_wall_count(*params, *pore);
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_footprint_bytes(const pmd_params* params, const pmd_pore* pore, int64_t n_vapor,
                        const pmd_tuning* tuning, size_t* out)
{
    try {
        CHK(check_params(params, pore));
        if (!out || n_vapor < 1) return fail(PMD_EINVAL, "n_vapor must be >= 1 and out not NULL");
        pmd_tuning t;
        CHK(merge_tuning(*params, n_vapor, tuning, &t));
        Grid g;
        CHK(grid_for(*params, t.skin, &g));
        SysParams sp{};
        fill_sys_params(sp, *params, g, t, (int)n_vapor, (int)host_wall_count(*params, *pore));
        // the same accounting a batch uses when it admits the system
        *out = system_bytes(params->precision, sp, t.list_cap);
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_create_system(const pmd_params* params, const pmd_pore* pore, int64_t n_vapor,
                      const double* pos, const double* vel, int64_t n_wall,
                      const double* wall_pos, void* hip_stream, const pmd_tuning* tuning,
                      pmd_system** out)
{
    try {
        GPU_LOCK;
        if (!out) return fail(PMD_EINVAL, "out must not be NULL");
        *out = nullptr;
        CHK(check_params(params, pore));
        if (n_vapor < 1 || !pos || !vel) return fail(PMD_EINVAL, "need n_vapor >= 1 and pos, vel");
        const int64_t nw = wall_pos ? n_wall : host_wall_count(*params, *pore);
        if (nw < 0) return fail(PMD_EINVAL, "n_wall must be >= 0");
        if (n_vapor + nw + 2 * kPad >= (int64_t)kIndexMask)
            return fail(PMD_EINVAL, "too many atoms for one system (%lld)", (long long)(n_vapor + nw));
        CHK(check_atoms(*params, n_vapor, pos, vel));
        if (wall_pos)
            for (int64_t i = 0; i < 3 * nw; ++i) {
                const int k = (int)(i % 3);
                if (!std::isfinite(wall_pos[i]) || wall_pos[i] < 0.0 || wall_pos[i] >= params->box[k])
                    return fail(PMD_EINVAL, "wall atom %lld outside [0, L)", (long long)(i / 3));
            }

        auto sys = std::make_unique<pmd_system>();
        sys->params = *params;
        sys->pore = *pore;
        sys->nv = n_vapor;
        sys->nw = nw;
        CHK(merge_tuning(*params, n_vapor, tuning, &sys->tuning));
        CHK(grid_for(*params, sys->tuning.skin, &sys->grid));

        auto pool = std::make_unique<Pool>();
        Pool& p = *pool;
        p.precision = params->precision;
        p.block = sys->tuning.block;
        p.brick_order = sys->tuning.brick_order;
        p.cap = sys->tuning.list_cap;
        p.nslots = 1;
        SysParams sp{};
        fill_sys_params(sp, *params, sys->grid, sys->tuning, (int)n_vapor, (int)nw);
        set_pore_region(sp, *params, *pore);
        p.vt = sp.vcap;
        p.wt = (int)std::max<int64_t>(nw, 1);
        p.ct = key_capacity(sys->grid);
        p.wct = sp.ncell + 1;
        p.nbt = key_capacity(sys->grid);
        sp.voff = 0;
        sp.woff = 0;
        sp.coff = 0;
        sp.wcoff = 0;
        sp.ering_off = 0;
        sp.ering_cap = p.ering_cap;
        if (hip_stream) {
            p.stream = (hipStream_t)hip_stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&p.stream, hipStreamNonBlocking));
            p.own_stream = true;
        }
        CHK(pool_allocate(p));
        p.hsp.assign(1, sp);
        CHK(pool_layout(p));

        // walls: generate (or take) the lattice, then bin it once
        double* raw = p.stage;  // SoA, stride wt
        if (nw > 0) {
            if (wall_pos) {
                std::vector<double> soa(3 * (size_t)nw);
                for (int64_t w = 0; w < nw; ++w)
                    for (int k = 0; k < 3; ++k) soa[(size_t)k * nw + w] = wall_pos[3 * w + k];
                HIPCHK(hipMemcpy(raw, soa.data(), sizeof(double) * soa.size(), hipMemcpyHostToDevice));
            } else {
                const PoreDev pd = pore_dev(*params, *pore);
                const long long nsites = (long long)pd.nslab * pd.nx * pd.ny * pd.nz;
                const int G = (int)((nsites + 255) / 256);
                int* counts = nullptr;
                HIPCHK(hipMalloc(&counts, sizeof(int) * (2 * (size_t)G + 1)));
                hipError_t e = launch_wall_generate(pd, params->box, raw, (int)nw, counts, counts + G,
                                                    counts + 2 * G, p.stream);
                int total = -1;
                if (e == hipSuccess)
                    e = hipMemcpyAsync(&total, counts + 2 * G, sizeof(int), hipMemcpyDeviceToHost, p.stream);
                if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
                hipFree(counts);
                HIPCHK(e);
                if (total != nw)
                    return fail(PMD_EHIP, "wall generation produced %d sites, expected %lld", total,
                                (long long)nw);
            }
        }
        HIPCHK(launch_wall_bin(p.dev(), 0, raw, (int)nw, (int)nw, p.precision, p.stream));
        HIPCHK(hipStreamSynchronize(p.stream));

        // vapour: copy in (caller order), then bin, build lists and compute a(0)
        sys->own = std::move(pool);
        sys->pool = sys->own.get();
        sys->slot = 0;
        CHK(load_state(sys.get(), pos, vel, 0));
        *out = sys.release();
        return PMD_OK;
    } catch (const std::bad_alloc&) {
        return fail(PMD_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_step(pmd_system* sys, int64_t nsteps)
{
    try {
        CHK(check_free(sys));
        if (nsteps < 0 || nsteps > (int64_t)1 << 30) return fail(PMD_EINVAL, "nsteps out of range");
        if (nsteps == 0) return PMD_OK;
        Pool& p = *sys->pool;
        HIPCHK(launch_set_run(p.dev(), sys->slot, (int)nsteps, 0, p.stream));
        const int R = sys->tuning.rebin_every;
        CHK(pool_enqueue(p, R, sys->tuning.use_graph, (nsteps + R - 1) / R));
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_sync(pmd_system* sys)
{
    try {
        CHK(check_free(sys));
        return sys_sync(sys);
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

static int readback(pmd_system* sys, int which, double* out, int64_t n)
{
    CHK(check_free(sys));
    if (!out || n != sys->nv) return fail(PMD_EINVAL, "need out and n == %lld", (long long)sys->nv);
    CHK(sys_sync(sys));
    Pool& p = *sys->pool;
    HIPCHK(launch_unpermute(p.dev(), sys->slot, which, p.stage, (int)n, p.stream));
    HIPCHK(hipMemcpyAsync(out, p.stage, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, p.stream));
    HIPCHK(hipStreamSynchronize(p.stream));
    return PMD_OK;
}

int pmd_get_positions(pmd_system* sys, double* out, int64_t n)
{
    try { return readback(sys, 0, out, n); } catch (...) { return fail(PMD_EHIP, "unexpected exception"); }
}

int pmd_get_velocities(pmd_system* sys, double* out, int64_t n)
{
    try { return readback(sys, 1, out, n); } catch (...) { return fail(PMD_EHIP, "unexpected exception"); }
}

int pmd_get_forces(pmd_system* sys, double* out, int64_t n)
{
    try { return readback(sys, 2, out, n); } catch (...) { return fail(PMD_EHIP, "unexpected exception"); }
}

static void to_energies(const EnergyRec& r, int64_t nv, bool virial, double pore_volume,
                        pmd_energies* e)
{
    e->step = r.step;
    e->ke = r.ke;
    e->pe_vv = r.pe_vv;
    e->pe_vw = r.pe_vw;
    e->etotal = r.ke + r.pe_vv + r.pe_vw;
    e->temperature = nv > 1 ? 2.0 * r.ke / (3.0 * nv - 3.0) : 0.0;
    // a pool runs the summing kernel when any of its systems asks for it
    e->virial_vv = virial ? r.w_vv : 0.0;
    e->virial_vw = virial ? r.w_vw : 0.0;
    e->ke_pore = virial ? r.ke_pore : 0.0;
    e->virial_pore = virial ? r.w_pore : 0.0;
    e->n_pore = virial ? (int64_t)r.n_pore : 0;
    e->pore_volume = pore_volume;
    e->pressure = virial && pore_volume > 0.0 ? (2.0 * r.ke_pore + r.w_pore) / (3.0 * pore_volume) : 0.0;
}

int pmd_get_energy_history(pmd_system* sys, pmd_energies* out, int64_t cap, int64_t* n_out)
{
    try {
        CHK(check_free(sys));
        if (!n_out || (cap > 0 && !out)) return fail(PMD_EINVAL, "need out and n_out");
        CHK(sys_sync(sys));
        Pool& p = *sys->pool;
        SysState st;
        CHK(read_state(p, sys->slot, &st));
        const int ring = p.hsp[sys->slot].ering_cap;
        const int64_t avail = std::min<int64_t>(st.nrec, ring);
        const int64_t first = st.nrec - avail;
        std::vector<EnergyRec> buf((size_t)ring);
        HIPCHK(hipMemcpy(buf.data(), p.erec + p.hsp[sys->slot].ering_off, sizeof(EnergyRec) * ring,
                         hipMemcpyDeviceToHost));
        const int64_t take = std::min(avail, cap);
        for (int64_t r = 0; r < take; ++r)
            to_energies(buf[(size_t)((first + (avail - take) + r) % ring)], sys->nv, sys->tuning.virial != 0,
                        pore_void_volume(sys->params, sys->pore), out + r);
        *n_out = take;
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_get_energies(pmd_system* sys, pmd_energies* out)
{
    if (!out) return fail(PMD_EINVAL, "out must not be NULL");
    int64_t n = 0;
    CHK(pmd_get_energy_history(sys, out, 1, &n));
    if (n != 1) return fail(PMD_ESTATE, "no energies recorded");
    return PMD_OK;
}

int pmd_get_wall_positions(pmd_system* sys, double* out, int64_t n_wall)
{
    try {
        CHK(check_free(sys));
        if (n_wall != sys->nw || (n_wall > 0 && !out)) return fail(PMD_EINVAL, "need n_wall == %lld", (long long)sys->nw);
        if (n_wall == 0) return PMD_OK;
        Pool& p = *sys->pool;
        HIPCHK(launch_wall_unpermute(p.dev(), sys->slot, p.stage, (int)n_wall, p.stream));
        HIPCHK(hipMemcpyAsync(out, p.stage, sizeof(double) * 3 * n_wall, hipMemcpyDeviceToHost, p.stream));
        HIPCHK(hipStreamSynchronize(p.stream));
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_get_counts(pmd_system* sys, int64_t* n_vapor, int64_t* n_wall)
{
    if (!sys) return fail(PMD_EINVAL, "NULL system");
    if (n_vapor) *n_vapor = sys->nv;
    if (n_wall) *n_wall = sys->nw;
    return PMD_OK;
}

int64_t pmd_get_step(pmd_system* sys)
{
    if (!sys || !sys->pool) return -1;
    SysState st;
    if (read_state(*sys->pool, sys->slot, &st) != PMD_OK) return -1;
    return st.step;
}

int pmd_get_positions_device(pmd_system* sys, double* dev_out, int64_t n, void* stream)
{
    try {
        CHK(check_free(sys));
        if (!dev_out || n != sys->nv) return fail(PMD_EINVAL, "need dev_out and n == %lld", (long long)sys->nv);
        CHK(sys_sync(sys));
        Pool& p = *sys->pool;
        hipStream_t s = stream ? (hipStream_t)stream : p.stream;
        HIPCHK(launch_unpermute(p.dev(), sys->slot, 0, dev_out, (int)n, s));
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_set_tuning(pmd_system* sys, const pmd_tuning* tuning)
{
    try {
        GPU_LOCK;
        CHK(check_free(sys));
        CHK(sys_sync(sys));
        pmd_tuning t;
        CHK(merge_tuning(sys->params, sys->nv, tuning, &t));
        Grid g;
        CHK(grid_for(sys->params, t.skin, &g));
        if (g.nc[0] != sys->grid.nc[0] || g.nc[1] != sys->grid.nc[1] || g.nc[2] != sys->grid.nc[2]) {
            // a different cell grid needs larger cell arrays: only allow grids
            // that fit the allocated ones
            if (key_capacity(g) > sys->pool->ct || g.nc[0] * g.nc[1] * g.nc[2] + 1 > sys->pool->wct)
                return fail(PMD_EINVAL, "skin too small for the allocated cell grid");
        }
        Pool& p = *sys->pool;
        if (t.list_cap > p.cap) CHK(pool_grow_lists(p, t.list_cap));
        t.list_cap = p.cap;
        sys->tuning = t;
        sys->grid = g;
        SysParams& sp = p.hsp[sys->slot];
        SysParams keep = sp;
        fill_sys_params(sp, sys->params, g, t, (int)sys->nv, (int)sys->nw);
        set_pore_region(sp, sys->params, sys->pore);
        sp.voff = keep.voff;
        sp.woff = keep.woff;
        sp.coff = keep.coff;
        sp.wcoff = keep.wcoff;
        sp.ering_off = keep.ering_off;
        sp.ering_cap = keep.ering_cap;
        p.block = t.block;
        p.brick_order = t.brick_order;
        CHK(pool_layout(p));
        if (g.nc[0] != keep.nc[0] || g.nc[1] != keep.nc[1] || g.nc[2] != keep.nc[2]) {
            // re-bin the walls on the new grid from their sorted positions
            HIPCHK(launch_wall_unpermute(p.dev(), sys->slot, p.stage, (int)sys->nw, p.stream));
            std::vector<double> aos(3 * (size_t)sys->nw), soa(3 * (size_t)sys->nw);
            HIPCHK(hipMemcpyAsync(aos.data(), p.stage, sizeof(double) * aos.size(), hipMemcpyDeviceToHost, p.stream));
            HIPCHK(hipStreamSynchronize(p.stream));
            for (int64_t w = 0; w < sys->nw; ++w)
                for (int k = 0; k < 3; ++k) soa[(size_t)k * sys->nw + w] = aos[3 * w + k];
            if (sys->nw)
                HIPCHK(hipMemcpy(p.stage, soa.data(), sizeof(double) * soa.size(), hipMemcpyHostToDevice));
            HIPCHK(launch_wall_bin(p.dev(), sys->slot, p.stage, (int)sys->nw, (int)sys->nw, p.precision, p.stream));
            HIPCHK(hipStreamSynchronize(p.stream));
        }
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_get_tuning(pmd_system* sys, pmd_tuning* out)
{
    if (!sys || !out) return fail(PMD_EINVAL, "NULL argument");
    *out = sys->tuning;
    return PMD_OK;
}

int pmd_set_state(pmd_system* sys, const double* pos, const double* vel, int64_t n, int64_t step)
{
    try {
        GPU_LOCK;
        CHK(check_free(sys));
        if (!pos || !vel) return fail(PMD_EINVAL, "pos and vel must not be NULL");
        if (n != sys->nv) return fail(PMD_EINVAL, "n = %lld, system has %lld vapour atoms",
                                      (long long)n, (long long)sys->nv);
        if (step < 0) return fail(PMD_EINVAL, "step must be >= 0");
        CHK(check_atoms(sys->params, n, pos, vel));
        CHK(sys_sync(sys));
        return load_state(sys, pos, vel, step);
    } catch (const std::bad_alloc&) {
        return fail(PMD_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_autotune_grid(const pmd_params* params, int64_t n_vapor, pmd_tuning* out, int32_t cap,
                      int32_t* n_out)
{
    try {
        if (!params || !n_out) return fail(PMD_EINVAL, "NULL argument");
        static const double skins[] = {0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 1.0};
        static const int periods[] = {4, 6, 8, 10, 12, 15, 20};
        const int total = (int)(sizeof(skins) / sizeof(skins[0]) * sizeof(periods) / sizeof(periods[0]));
        *n_out = total;
        if (!out) return PMD_OK;
        if (cap < total) return fail(PMD_EINVAL, "need room for %d candidates", total);
        const pmd_tuning base = default_tuning(*params, n_vapor);
        int k = 0;
        for (double sk : skins)
            for (int R : periods) {
                pmd_tuning t = base;
                t.skin = sk;
                t.rebin_every = R;
                t.list_cap = 0;  // sized from the density at the new skin
                out[k++] = t;
            }
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_autotune(const pmd_params* params, const pmd_pore* pore, int64_t n_vapor, const double* pos,
                 const double* vel, int64_t n_wall, const double* wall_pos, void* hip_stream,
                 const pmd_tuning* candidates, int32_t n_candidates, int64_t trial_steps,
                 double* us_per_step, int32_t* best)
{
    try {
        GPU_LOCK;
        if (!candidates || n_candidates < 1 || !best)
            return fail(PMD_EINVAL, "need candidates and best");
        if (trial_steps < 1 || trial_steps > 100000) return fail(PMD_EINVAL, "trial_steps out of range");
        for (int32_t c = 0; c < n_candidates; ++c) {
            pmd_tuning t;
            CHK(merge_tuning(*params, n_vapor, candidates + c, &t));
        }
        // one trial system, created at the smallest skin so that its cell
        // arrays also hold every coarser grid the later candidates use
        std::vector<int32_t> order(n_candidates);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return candidates[a].skin < candidates[b].skin;
        });
        pmd_system* trial = nullptr;
        CHK(pmd_create_system(params, pore, n_vapor, pos, vel, n_wall, wall_pos, hip_stream,
                              candidates + order[0], &trial));
        std::unique_ptr<pmd_system, int (*)(pmd_system*)> guard(trial, pmd_destroy);
        // the first steps of a freshly placed system are not typical of a
        // run (adsorption onto the walls changes densities and speeds), so
        // every candidate starts from the state 2 x trial_steps steps later
        CHK(pmd_step(trial, std::max<int64_t>(2 * trial_steps, 1000)));
        CHK(sys_sync(trial));
        std::vector<double> x0(3 * (size_t)n_vapor), v0(3 * (size_t)n_vapor);
        CHK(pmd_get_positions(trial, x0.data(), n_vapor));
        CHK(pmd_get_velocities(trial, v0.data(), n_vapor));
        const int64_t warm = std::max<int64_t>(trial_steps / 4, 1);
        double best_us = std::numeric_limits<double>::infinity();
        *best = -1;
        for (int32_t c : order) {
            double us = std::numeric_limits<double>::infinity();
            int rc = pmd_set_tuning(trial, candidates + c);
            if (rc == PMD_OK) rc = load_state(trial, x0.data(), v0.data(), 0);
            if (rc == PMD_OK) rc = pmd_step(trial, warm);
            if (rc == PMD_OK) rc = sys_sync(trial);
            if (rc == PMD_OK) {
                const auto t0 = std::chrono::steady_clock::now();
                rc = pmd_step(trial, trial_steps);
                if (rc == PMD_OK) rc = sys_sync(trial);
                const auto t1 = std::chrono::steady_clock::now();
                if (rc == PMD_OK)
                    us = std::chrono::duration<double, std::micro>(t1 - t0).count() / (double)trial_steps;
            }
            // a failing candidate (numerics aside) is only a slow one
            if (rc == PMD_ENUMERIC) return rc;
            if (us_per_step) us_per_step[c] = us;
            if (us < best_us) {
                best_us = us;
                *best = c;
            }
        }
        if (*best < 0) return fail(PMD_EHIP, "no candidate tuning completed its trial");
        // among candidates within 2% of the fastest, take the largest skin
        // (the fastest of those): early rebuilds become more frequent as a
        // run goes on, and a larger skin keeps them rare
        if (us_per_step) {
            for (int32_t c = 0; c < n_candidates; ++c) {
                if (!(us_per_step[c] <= 1.02 * best_us)) continue;
                const pmd_tuning& a = candidates[c];
                const pmd_tuning& b = candidates[*best];
                if (a.skin > b.skin || (a.skin == b.skin && us_per_step[c] < us_per_step[*best])) *best = c;
            }
        }
        return PMD_OK;
    } catch (const std::bad_alloc&) {
        return fail(PMD_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_destroy(pmd_system* sys)
{
    if (!sys) return PMD_OK;
    try {
        GPU_LOCK;
        if (sys->batch) return fail(PMD_ESTATE, "system is resident in a batch; release it first");
        delete sys;
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_timing_enable(pmd_system* sys, int enable)
{
    try {
        CHK(check_free(sys));
        Pool& p = *sys->pool;
        HIPCHK(hipStreamSynchronize(p.stream));
        for (auto& e : p.events) {
            hipEventDestroy(e.a);
            hipEventDestroy(e.b);
        }
        p.events.clear();
        p.timing = enable != 0;
        p.t_exit_ms = 0.0;
        if (p.timing) {
            // duration of a launch whose workgroups all return at once (the
            // launches after an early-rebuild halt): 32 back-to-back launches
            // on the system at rest
            SysState st;
            CHK(read_state(p, sys->slot, &st));
            if (st.remaining != 0) return fail(PMD_ESTATE, "system has queued steps");
            hipEvent_t a, b;
            HIPCHK(hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
            HIPCHK(hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
            const PoolDev d = p.dev();
            hipError_t e = launch_step(d, 0, p.precision, p.stream, nullptr, nullptr);  // warm
            if (e == hipSuccess) e = hipEventRecord(a, p.stream);
            for (int k = 0; k < 32 && e == hipSuccess; ++k)
                e = launch_step(d, 0, p.precision, p.stream, nullptr, nullptr);
            if (e == hipSuccess) e = hipEventRecord(b, p.stream);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            hipEventDestroy(a);
            hipEventDestroy(b);
            HIPCHK(e);
            p.t_exit_ms = ms / 32.0;
        }
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_kernel_time(pmd_system* sys, int64_t* launches, double* mean_ms)
{
    try {
        CHK(check_free(sys));
        Pool& p = *sys->pool;
        HIPCHK(hipStreamSynchronize(p.stream));
        double tot = 0.0;
        int64_t n = 0;
        for (auto& e : p.events) {
            float ms = 0.0f;
            if (e.done <= 0 || hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) continue;
            tot += ms - (e.R - e.done) * p.t_exit_ms;
            n += e.done;
        }
        if (launches) *launches = n;
        if (mean_ms) *mean_ms = n ? tot / n : 0.0;
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_kernel_times(pmd_system* sys, double* out_ms, int64_t cap, int64_t* n_out)
{
    try {
        CHK(check_free(sys));
        if (!n_out || (cap > 0 && !out_ms)) return fail(PMD_EINVAL, "NULL argument");
        Pool& p = *sys->pool;
        HIPCHK(hipStreamSynchronize(p.stream));
        int64_t n = 0;
        for (auto& e : p.events) {
            float ms = 0.0f;
            if (e.done <= 0 || hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) continue;
            if (n < cap) out_ms[n] = (ms - (e.R - e.done) * p.t_exit_ms) / e.done;
            ++n;
        }
        *n_out = n;
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_debug_cells(pmd_system* sys, int32_t* cell_of_atom, int64_t n, int32_t* cell_start,
                    int64_t n_cells_p1, int32_t* perm, int32_t* ncell, double* inv)
{
    try {
        CHK(check_free(sys));
        CHK(sys_sync(sys));
        Pool& p = *sys->pool;
        const SysParams& sp = p.hsp[sys->slot];
        if (ncell)
            for (int k = 0; k < 3; ++k) ncell[k] = sp.nc[k];
        if (inv)
            for (int k = 0; k < 3; ++k) inv[k] = sp.inv_h[k];
        if (!cell_of_atom && !cell_start && !perm) return PMD_OK;
        if (n != sys->nv || n_cells_p1 != sp.ncell + 1) return fail(PMD_EINVAL, "size mismatch");
        SysState st;
        CHK(read_state(p, sys->slot, &st));
        std::vector<int> ids(sp.vcap), cl(sp.vcap), cs(sp.nkey + 2);
        HIPCHK(hipMemcpy(ids.data(), p.id[st.ibuf] + sp.voff, sizeof(int) * sp.vcap, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(cl.data(), p.cell_lin + sp.voff, sizeof(int) * sp.vcap, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(cs.data(), p.cstart + sp.coff, sizeof(int) * (sp.nkey + 2), hipMemcpyDeviceToHost));
        // first storage position of each cell (cells are stored brick by brick)
        for (int c = 0; c < sp.ncell; ++c) {
            const int cx = c % sp.nc[0], cy = (c / sp.nc[0]) % sp.nc[1], cz = c / (sp.nc[0] * sp.nc[1]);
            const int Bx = cx / sp.bdim[0], By = cy / sp.bdim[1], Bz = cz / sp.bdim[2];
            const int key = (Bx + sp.nbk[0] * (By + sp.nbk[1] * Bz)) * sp.bcells +
                            (cx - Bx * sp.bdim[0]) + sp.bdim[0] * ((cy - By * sp.bdim[1]) + sp.bdim[1] * (cz - Bz * sp.bdim[2]));
            cell_start[c] = cs[key] - sp.voff;
        }
        cell_start[sp.ncell] = sp.nv;
        for (int q = 0; q < sp.nv; ++q) {
            perm[q] = ids[q];
            cell_of_atom[ids[q]] = cl[q];
        }
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_debug_pairs(pmd_system* sys, int32_t* vv, int64_t cap, int64_t* n_vv, int32_t* vw,
                    int64_t* n_vw)
{
    try {
        CHK(check_free(sys));
        if (!n_vv || !n_vw) return fail(PMD_EINVAL, "need n_vv and n_vw");
        CHK(sys_sync(sys));
        Pool& p = *sys->pool;
        const SysParams& sp = p.hsp[sys->slot];
        const int maxp = (int)std::min<int64_t>((int64_t)sp.nv * p.cap, 1 << 26);
        int* out = nullptr;
        HIPCHK(hipMalloc(&out, sizeof(int) * (3 * (size_t)maxp + 1)));
        int* counts = out + 3 * (size_t)maxp;
        hipError_t e = hipMemsetAsync(counts, 0, sizeof(int), p.stream);
        if (e == hipSuccess) e = launch_debug_pairs(p.dev(), sys->slot, p.precision, out, maxp, counts, p.stream);
        int total = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&total, counts, sizeof(int), hipMemcpyDeviceToHost, p.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
        std::vector<int> h;
        if (e == hipSuccess) {
            h.resize(3 * (size_t)std::min(total, maxp));
            if (!h.empty()) e = hipMemcpy(h.data(), out, sizeof(int) * h.size(), hipMemcpyDeviceToHost);
        }
        hipFree(out);
        HIPCHK(e);
        std::vector<std::pair<int, int>> a, b;
        for (size_t q = 0; q < h.size(); q += 3) (h[q] == 0 ? a : b).emplace_back(h[q + 1], h[q + 2]);
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        *n_vv = (int64_t)a.size();
        *n_vw = (int64_t)b.size();
        for (int64_t q = 0; q < std::min<int64_t>(cap, a.size()); ++q) {
            vv[2 * q] = a[q].first;
            vv[2 * q + 1] = a[q].second;
        }
        for (int64_t q = 0; q < std::min<int64_t>(cap, b.size()); ++q) {
            vw[2 * q] = b[q].first;
            vw[2 * q + 1] = b[q].second;
        }
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_debug_lists(pmd_system* sys, int64_t* rebuilds, int64_t* max_len)
{
    try {
        if (!sys || !sys->pool) return fail(PMD_EINVAL, "NULL system");
        SysState st;
        CHK(read_state(*sys->pool, sys->slot, &st));
        if (rebuilds) *rebuilds = st.rebins;
        if (max_len) *max_len = st.max_nbr;
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}


int pmd_batch_create(size_t hbm_budget, int max_slots, void* hip_stream, pmd_batch** out)
{
    try {
        if (!out) return fail(PMD_EINVAL, "out must not be NULL");
        if (max_slots < 1 || max_slots > 65536) return fail(PMD_EINVAL, "max_slots must be in [1, 65536]");
        auto b = std::make_unique<pmd_batch>();
        b->budget = hbm_budget;
        b->max_slots = max_slots;
        b->resident.assign(max_slots, nullptr);
        b->steps_wanted.assign(max_slots, 0);
        b->admit_seq.assign(max_slots, 0);
        b->user_stream = (hipStream_t)hip_stream;
        for (auto& sn : b->snap) {
            HIPCHK(hipEventCreateWithFlags(&sn.ev, hipEventDisableTiming));
            HIPCHK(hipHostMalloc((void**)&sn.host, sizeof(SysState) * (size_t)max_slots));
        }
        *out = b.release();
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_batch_admit(pmd_batch* b, pmd_system* sys, int64_t nsteps, int* slot)
{
    try {
        GPU_LOCK;
        if (!b || !sys || !slot) return fail(PMD_EINVAL, "NULL argument");
        if (sys->batch) return fail(PMD_ESTATE, "system already resident in a batch");
        if (nsteps < 0 || nsteps > (int64_t)1 << 30) return fail(PMD_EINVAL, "nsteps out of range");
        CHK(sys_sync(sys));
        // admission rewrites the pool's tables (and a repack frees the old
        // pool): the chunks still queued on the batch's stream read them, so
        // they must have finished first
        if (b->configured) HIPCHK(hipStreamSynchronize(b->pool->stream));
        Pool& sp0 = *sys->own;
        if (b->configured) {
            if (sp0.precision != b->pool->precision) return fail(PMD_EINVAL, "precision differs from the batch's");
            if (sys->tuning.block != b->tuning.block || sys->tuning.rebin_every != b->tuning.rebin_every)
                return fail(PMD_EINVAL, "block and rebin_every must match the batch's (%d, %d)",
                            b->tuning.block, b->tuning.rebin_every);
        }
        int free_slot = -1;
        for (int s = 0; s < b->max_slots; ++s)
            if (!b->resident[s]) {
                free_slot = s;
                break;
            }
        if (free_slot < 0) return fail(PMD_EAGAIN, "no free slot");
        const SysParams& src_sp = sp0.hsp[sys->slot];
        const int cap = std::max(sp0.cap, b->configured ? b->pool->cap : 0);
        const size_t need = system_bytes(sp0.precision, src_sp, cap);
        if (b->budget && batch_used(b) + need > b->budget)
            return fail(PMD_EAGAIN, "over the batch's device budget");
        if (!b->configured) {
            b->tuning = sys->tuning;
            b->R = sys->tuning.rebin_every;
            auto np = std::make_unique<Pool>();
            np->precision = sp0.precision;
            np->block = sys->tuning.block;
            np->brick_order = sys->tuning.brick_order;
            np->cap = sp0.cap;
            np->nslots = b->max_slots;
            np->ering_cap = kBatchErings;
            if (b->user_stream) {
                np->stream = b->user_stream;
            } else {
                HIPCHK(hipStreamCreateWithFlags(&np->stream, hipStreamNonBlocking));
                np->own_stream = true;
            }
            np->vt = kPad;
            np->wt = 1;
            np->ct = np->wct = 8;
            np->nbt = kPad / kChunk;
            CHK(pool_allocate(*np));
            np->hsp.assign(np->nslots, SysParams{});
            CHK(pool_layout(*np));
            b->pool = std::move(np);
            b->configured = true;
        }
        SysParams sp = src_sp;
        const Needs n = needs_of(sp);
        {
            int64_t resident_walls = 0;
            for (size_t s = 0; s < b->resident.size(); ++s)
                if (b->resident[s]) resident_walls += needs_of(b->pool->hsp[s]).wt;
            CHK(check_pool_walls(resident_walls, n.wt));
        }
        if (cap > b->pool->cap || !batch_bump(b, n, &sp)) {
            CHK(batch_repack(b, n, cap));
            if (!batch_bump(b, n, &sp)) return fail(PMD_ENOMEM, "batch repack left no room");
        }
        Pool& p = *b->pool;
        sp.ering_off = free_slot * p.ering_cap;
        sp.ering_cap = p.ering_cap;
        sp.active = 1;
        p.hsp[free_slot] = sp;
        CHK(pool_layout(p));
        CHK(move_system(sp0, sys->slot, p, free_slot));
        CHK(pool_layout(p));
        b->resident[free_slot] = sys;
        b->steps_wanted[free_slot] = nsteps;
        b->admit_seq[free_slot] = b->snap_seq;
        sys->own.reset();
        sys->pool = &p;
        sys->slot = free_slot;
        sys->batch = b;
        if (nsteps > 0) HIPCHK(launch_set_run(p.dev(), free_slot, (int)nsteps, 0, p.stream));
        *slot = free_slot;
        return PMD_OK;
    } catch (const std::bad_alloc&) {
        return fail(PMD_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_batch_advance(pmd_batch* b, int64_t chunk_steps)
{
    try {
        if (!b) return fail(PMD_EINVAL, "NULL batch");
        if (!b->configured || chunk_steps <= 0) return PMD_OK;
        const int R = b->R;
        CHK(pool_enqueue(*b->pool, R, b->tuning.use_graph, (chunk_steps + R - 1) / R));
        // the state after this chunk, for pmd_batch_poll_async; the ring's
        // oldest entry is reused (waiting for it only if four chunks are
        // still queued ahead of this one)
        StateSnap& sn = b->snap[b->snap_seq % kSnaps];
        if (sn.seq >= 0 && !sn.done) HIPCHK(hipEventSynchronize(sn.ev));
        Pool& p = *b->pool;
        HIPCHK(hipMemcpyAsync(sn.host, p.d_st, sizeof(SysState) * (size_t)p.nslots, hipMemcpyDeviceToHost,
                              p.stream));
        HIPCHK(hipEventRecord(sn.ev, p.stream));
        sn.seq = b->snap_seq++;
        sn.done = false;
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

// Non-blocking poll: the newest state snapshot whose chunk has completed
// names the systems that finished (a snapshot taken before a system was
// admitted says nothing about it).  A snapshot that shows a system needing
// the host (list overflow, tile overflow, a stall) hands over to the
// blocking poll, which fixes it.
static int batch_poll_snap(pmd_batch* b, int* done, int cap, int* n_done, bool* need_host)
{
    *need_host = false;
    const StateSnap* best = nullptr;
    for (auto& sn : b->snap) {
        if (sn.seq < 0) continue;
        if (!sn.done) {
            const hipError_t q = hipEventQuery(sn.ev);
            if (q == hipErrorNotReady) continue;
            HIPCHK(q);
            sn.done = true;
        }
        if (!best || sn.seq > best->seq) best = &sn;
    }
    if (!best) return PMD_OK;
    const Pool& p = *b->pool;
    for (int s = 0; s < p.nslots; ++s) {
        if (!b->resident[s] || best->seq < b->admit_seq[s]) continue;
        const SysState& st = best->host[s];
        if (st.status & (ST_TILE | ST_OVERFLOW | ST_STALL)) *need_host = true;
        const bool finished = st.remaining <= 0 || (st.status & ST_NONFINITE);
        if (finished && *n_done < cap) done[(*n_done)++] = s;
    }
    return PMD_OK;
}

static int batch_poll_impl(pmd_batch* b, int* done, int cap, int* n_done, bool wait)
{
    if (!b || !n_done || (cap > 0 && !done)) return fail(PMD_EINVAL, "NULL argument");
    *n_done = 0;
    if (!b->configured) return PMD_OK;
    Pool& p = *b->pool;
    if (!wait) {
        bool need_host = false;
        CHK(batch_poll_snap(b, done, cap, n_done, &need_host));
        if (!need_host) return PMD_OK;
        *n_done = 0;
    }
    std::vector<SysState> st((size_t)p.nslots);
    HIPCHK(hipMemcpyAsync(st.data(), p.d_st, sizeof(SysState) * st.size(), hipMemcpyDeviceToHost, p.stream));
    HIPCHK(hipStreamSynchronize(p.stream));
    bool grow = false;
    int need = p.cap;
    for (int s = 0; s < p.nslots; ++s) {
        if (!b->resident[s]) continue;
        if (st[s].status & ST_TILE) {
            CHK(pool_fix_tile(p, s, st[s].status));
        } else if (st[s].status & ST_OVERFLOW) {
            grow = true;
            need = std::max(need, st[s].max_nbr + st[s].max_nbr / 4 + 8);
        }
        const bool finished = st[s].remaining <= 0 || (st[s].status & ST_NONFINITE);
        if (finished && *n_done < cap) done[(*n_done)++] = s;
    }
    if (grow) {
        need = round_up(need, 16);
        if (need > 4096) return fail(PMD_ENOMEM, "neighbour list needs %d entries", need);
        CHK(pool_grow_lists(p, need));
    }
    for (int s = 0; s < p.nslots; ++s)
        if (b->resident[s] && (st[s].status & ST_STALL))
            HIPCHK(launch_set_run(p.dev(), s, 0, ST_STALL, p.stream));
    return PMD_OK;
}

int pmd_batch_poll(pmd_batch* b, int* done_slots, int cap, int* n_done)
{
    try { return batch_poll_impl(b, done_slots, cap, n_done, true); } catch (...) { return fail(PMD_EHIP, "unexpected exception"); }
}

int pmd_batch_poll_async(pmd_batch* b, int* done_slots, int cap, int* n_done)
{
    try { return batch_poll_impl(b, done_slots, cap, n_done, false); } catch (...) { return fail(PMD_EHIP, "unexpected exception"); }
}

int pmd_batch_release(pmd_batch* b, int slot, pmd_system** sys_out)
{
    try {
        GPU_LOCK;
        if (!b || slot < 0 || slot >= b->max_slots || !b->resident[slot])
            return fail(PMD_EINVAL, "no system in slot %d", slot);
        pmd_system* sys = b->resident[slot];
        Pool& p = *b->pool;
        HIPCHK(hipStreamSynchronize(p.stream));
        std::unique_ptr<Pool> own;
        CHK(make_single_pool(p, p.hsp[slot], nullptr, false, &own));
        CHK(move_system(p, slot, *own, 0));
        own->cap = p.cap;
        CHK(pool_layout(*own));
        b->resident[slot] = nullptr;
        b->steps_wanted[slot] = 0;
        p.hsp[slot] = SysParams{};
        CHK(pool_layout(p));
        sys->own = std::move(own);
        sys->pool = sys->own.get();
        sys->slot = 0;
        sys->batch = nullptr;
        sys->tuning.list_cap = sys->pool->cap;
        if (sys_out) *sys_out = sys;
        return PMD_OK;
    } catch (const std::bad_alloc&) {
        return fail(PMD_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

int pmd_batch_info(pmd_batch* b, int* resident, size_t* bytes_used, size_t* bytes_budget)
{
    if (!b) return fail(PMD_EINVAL, "NULL batch");
    int r = 0;
    for (auto* s : b->resident) r += s != nullptr;
    if (resident) *resident = r;
    if (bytes_used) *bytes_used = b->configured ? batch_used(b) : 0;
    if (bytes_budget) *bytes_budget = b->budget;
    return PMD_OK;
}

int pmd_batch_destroy(pmd_batch* b)
{
    if (!b) return PMD_OK;
    try {
        GPU_LOCK;
        for (int s = 0; s < b->max_slots; ++s)
            if (b->resident[s]) CHK(pmd_batch_release(b, s, nullptr));
        for (auto& sn : b->snap) {
            if (sn.ev) (void)hipEventDestroy(sn.ev);
            if (sn.host) (void)hipHostFree(sn.host);
        }
        delete b;
        return PMD_OK;
    } catch (...) {
        return fail(PMD_EHIP, "unexpected exception");
    }
}

}  // extern "C"
