// pmd_kernels.hip -- gfx950 kernels of the pore-MD hot path.
//
// One time step is velocity Verlet (arXiv:1812.07993, Sec. 3: F2 drift and
// first half-kick, F1 forces from the new positions, F3 second half-kick).
// Inside a run the step kernel fuses F1 and F3 of step n with F2 of step
// n + 1 (the leapfrog form of the same update), so one launch per step reads
// and writes each atom's state once.
//
// Forces (Sec. 2, eq. 2) are short-ranged Lennard-Jones sums over Verlet
// neighbour lists of radius r_c + skin, rebuilt from a cell grid (cells of
// edge >= r_c + skin) at the start of every graph replay and whenever an
// atom has moved more than skin/2 away from its position at the last
// rebuild (then every pair within r_c is still in the lists).  The rebuild is five launches: drift
// and bin count, per-system scan, arrival scatter, stable placement (atoms
// ordered by cell, then by caller index), list build.
//
// Precision: FP64 keeps every operation in double.  Mixed computes the pair
// terms in FP32 on cell-local coordinates (|x| <= cell edge, so the FP32
// rounding of a separation is ~1e-7 of the cell edge) and accumulates each
// atom's force, the integration and the energies in FP64.  A pair whose FP32
// r^2 lies within a narrow band of r_c^2 is re-tested in FP64 so that the
// cutoff decision matches an FP64 evaluation.
#include <hip/hip_ext.h>

#include "pmd_internal.h"

namespace pmd {

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs of the device.  Map
// the hardware index so each XCD receives a contiguous run of logical
// workgroups: cell-sorted neighbours then share that XCD's L2.  The grid is
// padded to a multiple of 8.
__device__ __forceinline__ int logical_block()
{
    const int q = gridDim.x >> 3;
    const int b = blockIdx.x;
    return (b & 7) * q + (b >> 3);
}

// Storage of the neighbour lists.  Entries are kept in 16-byte chunks of
// consecutive entries of one atom; chunk c of every slot is contiguous (16
// bytes per slot, stride vt), so a lane's chunk is one 16-byte load, a
// wave's chunk loads cover one contiguous 1 KB, and the list build's writes
// of one atom fill 16-byte pieces.  Vapour entries come first, eight 16-bit
// entries per chunk (two per 32-bit word, the lower half first); the wall
// entries follow from the next chunk boundary, four 32-bit entries per chunk.

// uint32 index of 32-bit word kw of slot i's list (four words per chunk).
__device__ __forceinline__ size_t list_at(int vt, int i, int kw)
{
    return (((size_t)(kw >> 2) * vt + i) << 2) + (kw & 3);
}

// uint16 index of vapour entry k of slot i.
__device__ __forceinline__ size_t vlist_at(int vt, int i, int k)
{
    return (((size_t)(k >> 3) * vt + i) << 3) + (k & 7);
}

// Shift -d h of neighbour-cell code q (d = offset of the neighbour cell,
// exactly h, 0 or -h per axis) that moves the neighbour's cell-local
// coordinate into the frame of the atom's cell; the pad code gives -2h per
// axis.
template <typename T>
__device__ __forceinline__ typename V4<T>::type shift_q(int q, T hx, T hy, T hz)
{
    const int fx = q >= 27 ? 3 : q % 3, fy = q >= 27 ? 3 : (q / 3) % 3, fz = q >= 27 ? 3 : q / 9;
    typename V4<T>::type v;
    v.x = (T)(1 - fx) * hx;
    v.y = (T)(1 - fy) * hy;
    v.z = (T)(1 - fz) * hz;
    v.w = (T)0;
    return v;
}

__device__ __forceinline__ int wrap_cell(int c, int n)
{
    c += (c < 0) ? n : 0;
    c -= (c >= n) ? n : 0;
    return c;
}

// Periodic image in [0, L) of a coordinate at most one box length outside it
// (an atom moves far less than L in a step): one add or subtract, no
// division; x + L rounding up to L for a tiny negative x gives 0.
__device__ __forceinline__ double wrap_box(double x, double L)
{
    x = (x < 0.0) ? x + L : (x >= L) ? x - L : x;
    return (x >= L) ? 0.0 : x;
}

__device__ __forceinline__ int cell_axis(double x, double inv, int n)
{
    double q = floor(x * inv);
    int c = (int)q;
    c = (q < 0.0) ? 0 : c;
    c = (q > (double)(n - 1)) ? n - 1 : c;
    return c;
}

// Minimum-image offset of x from the origin of cell index c along one axis.
__device__ __forceinline__ double local_axis(double x, int c, double h, double L, double invL)
{
    double l = x - (double)c * h;
    return l - L * rint(l * invL);
}

template <typename T>
__device__ __forceinline__ typename V4<T>::type make4(double x, double y, double z)
{
    typename V4<T>::type v;
    v.x = (T)x;
    v.y = (T)y;
    v.z = (T)z;
    v.w = (T)0;
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_or(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Exclusive scan over the workgroup (any size up to 1024, multiple of 64).
// Returns the exclusive prefix; *total receives the workgroup sum.
__device__ int block_exclusive_scan(int v, int* lds /* >= 16 ints */, int* total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    // every thread sums the wave totals itself (at most 16 broadcast reads)
    // instead of waiting for one thread to prefix them: one barrier, and lds
    // is not written again, so a kernel may call this once without another
    int pre = 0, all = 0;
    for (int w = 0; w < nw; ++w) {
        const int t = lds[w];
        pre += w < wave ? t : 0;
        all += t;
    }
    *total = all;
    return pre + x - v;
}

__device__ __forceinline__ double atomic_load_f64(const double* p)
{
    unsigned long long u = __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)u);
}

// ---------------------------------------------------------------------------
// Wall lattice (boundary treatment, part 1: fixed atoms of the pore walls)
// ---------------------------------------------------------------------------

__device__ double layer_radius(const PoreDev& p, double hz)
{
    switch (p.kind) {
    case 2: return p.r0;
    case 4: return p.r0 + (p.r1 - p.r0) * (hz / p.t);
    case 5: return (hz < 0.25 * p.t || hz >= 0.75 * p.t) ? p.r0 : p.r1;
    default: return 0.0;
    }
}

__device__ bool wall_site(const PoreDev& p, const double* L, long long s, double* xyz)
{
    const long long per_slab = (long long)p.nx * p.ny * p.nz;
    const int slab = (int)(s / per_slab);
    long long r = s - (long long)slab * per_slab;
    const int k = (int)(r / ((long long)p.nx * p.ny));
    r -= (long long)k * p.nx * p.ny;
    const int j = (int)(r / p.nx);
    const int i = (int)(r - (long long)j * p.nx);
    const double hz = (k + 0.5) * p.a;
    const double x = (i + 0.5) * p.a, y = (j + 0.5) * p.a;
    xyz[0] = x;
    xyz[1] = y;
    xyz[2] = p.z_lo[slab] + hz;
    const double rad = layer_radius(p, hz);
    const double dx = x - 0.5 * L[0], dy = y - 0.5 * L[1];
    return !(dx * dx + dy * dy < rad * rad);
}

struct Box3 { double L[3]; };

__global__ void k_wall_count(PoreDev p, Box3 b, long long nsites, int* block_counts)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double xyz[3];
    const bool keep = s < nsites && wall_site(p, b.L, s, xyz);
    const int c = __syncthreads_count(keep);
    if (threadIdx.x == 0) block_counts[blockIdx.x] = c;
}

__global__ void k_scan_small(const int* in, int n, int* out, int* total)
{
    __shared__ int lds[17];
    const int T = blockDim.x;
    const int per = (n + T - 1) / T;
    const int lo = threadIdx.x * per, hi = min(n, lo + per);
    int sum = 0;
    for (int c = lo; c < hi; ++c) sum += in[c];
    int tot;
    int run = block_exclusive_scan(sum, lds, &tot);
    for (int c = lo; c < hi; ++c) {
        int k = in[c];
        out[c] = run;
        run += k;
    }
    if (threadIdx.x == 0) *total = tot;
}

__global__ void k_wall_emit(PoreDev p, Box3 b, long long nsites, const int* block_offsets,
                            double* out, int stride)
{
    __shared__ int wave_base[16];
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double xyz[3];
    const bool keep = s < nsites && wall_site(p, b.L, s, xyz);
    const unsigned long long m = __ballot(keep);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wave_base[wave] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            int t = wave_base[w];
            wave_base[w] = run;
            run += t;
        }
    }
    __syncthreads();
    if (keep) {
        const int rank = wave_base[wave] + __popcll(m & ((1ull << lane) - 1ull));
        const int o = block_offsets[blockIdx.x] + rank;
        out[o] = xyz[0];
        out[stride + o] = xyz[1];
        out[2 * stride + o] = xyz[2];
    }
}

hipError_t launch_wall_generate(const PoreDev& pore, const double* L, double* out, int stride,
                                int* block_counts, int* block_offsets, int* total, hipStream_t s)
{
    const long long nsites = (long long)pore.nslab * pore.nx * pore.ny * pore.nz;
    if (nsites <= 0) return hipSuccess;
    const int B = 256;
    const int G = (int)((nsites + B - 1) / B);
    Box3 b;
    for (int k = 0; k < 3; ++k) b.L[k] = L[k];
    hipLaunchKernelGGL(k_wall_count, dim3(G), dim3(B), 0, s, pore, b, nsites, block_counts);
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, block_counts, G, block_offsets,
                       total);
    hipLaunchKernelGGL(k_wall_emit, dim3(G), dim3(B), 0, s, pore, b, nsites, block_offsets, out,
                       stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wall binning (once per system): walls sorted by cell, then by canonical
// index; local coordinates written into both coordinate buffers.
// ---------------------------------------------------------------------------

__global__ void k_wall_bin_count(PoolDev P, int sys, const double* raw, int rs)
{
    const SysParams& sp = P.sp[sys];
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= sp.nw) return;
    const int cx = cell_axis(raw[w], sp.inv_h[0], sp.nc[0]);
    const int cy = cell_axis(raw[rs + w], sp.inv_h[1], sp.nc[1]);
    const int cz = cell_axis(raw[2 * rs + w], sp.inv_h[2], sp.nc[2]);
    const int c = cx + sp.nc[0] * (cy + sp.nc[1] * cz);
    P.cell_tmp[w] = c;
    P.arr[w] = atomicAdd(&P.count[sp.coff + c], 1);
}

__global__ void k_wall_bin_scan(PoolDev P, int sys)
{
    __shared__ int lds[17];
    const SysParams& sp = P.sp[sys];
    const int M = sp.ncell;
    int* cnt = P.count + sp.coff;
    int* cs = P.wcstart + sp.wcoff;
    const int T = blockDim.x;
    const int per = (M + T - 1) / T;
    const int lo = threadIdx.x * per, hi = min(M, lo + per);
    int sum = 0;
    for (int c = lo; c < hi; ++c) sum += cnt[c];
    int tot;
    int run = sp.woff + block_exclusive_scan(sum, lds, &tot);
    for (int c = lo; c < hi; ++c) {
        int k = cnt[c];
        cs[c] = run;
        run += k;
        cnt[c] = 0;
    }
    if (threadIdx.x == 0) cs[M] = sp.woff + tot;
}

__global__ void k_wall_bin_scatter(PoolDev P, int sys)
{
    const SysParams& sp = P.sp[sys];
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= sp.nw) return;
    const int c = P.cell_tmp[w];
    P.tmp[P.wcstart[sp.wcoff + c] - sp.woff + P.arr[w]] = w;
}

template <typename T>
__global__ void k_wall_bin_place(PoolDev P, int sys, const double* raw, int rs)
{
    using V = typename V4<T>::type;
    const SysParams& sp = P.sp[sys];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.nw) return;
    const int o = P.tmp[p];
    const int c = P.cell_tmp[o];
    const int b0 = P.wcstart[sp.wcoff + c] - sp.woff, b1 = P.wcstart[sp.wcoff + c + 1] - sp.woff;
    int rank = 0;
    for (int q = b0; q < b1; ++q) rank += (P.tmp[q] < o);
    const int d = sp.woff + b0 + rank;
    const double x = raw[o], y = raw[rs + o], z = raw[2 * rs + o];
    P.WX[d] = x;
    P.WX[P.wt + d] = y;
    P.WX[2 * P.wt + d] = z;
    P.wid[d] = o;
    const int cx = c % sp.nc[0], cy = (c / sp.nc[0]) % sp.nc[1], cz = c / (sp.nc[0] * sp.nc[1]);
    const V l = make4<T>(local_axis(x, cx, sp.h[0], sp.L[0], sp.invL[0]),
                         local_axis(y, cy, sp.h[1], sp.L[1], sp.invL[1]),
                         local_axis(z, cz, sp.h[2], sp.L[2], sp.invL[2]));
    ((V*)P.L[0])[P.vt + d] = l;
    ((V*)P.L[1])[P.vt + d] = l;
}

hipError_t launch_wall_bin(const PoolDev& P, int sys, const double* raw, int rs, int nw,
                           int precision, hipStream_t s)
{
    if (nw <= 0) {
        hipLaunchKernelGGL(k_wall_bin_scan, dim3(1), dim3(1024), 0, s, P, sys);
        return hipGetLastError();
    }
    const int B = 256, G = (nw + B - 1) / B;
    hipLaunchKernelGGL(k_wall_bin_count, dim3(G), dim3(B), 0, s, P, sys, raw, rs);
    hipLaunchKernelGGL(k_wall_bin_scan, dim3(1), dim3(1024), 0, s, P, sys);
    hipLaunchKernelGGL(k_wall_bin_scatter, dim3(G), dim3(B), 0, s, P, sys);
    if (precision == 1)
        hipLaunchKernelGGL(k_wall_bin_place<float>, dim3(G), dim3(B), 0, s, P, sys, raw, rs);
    else
        hipLaunchKernelGGL(k_wall_bin_place<double>, dim3(G), dim3(B), 0, s, P, sys, raw, rs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rebuild: drift (run start) + bin count, scan, scatter, place, list build
// ---------------------------------------------------------------------------

// Cells are numbered brick by brick (bricks of bdim cells, x fastest inside
// a brick and between bricks), so the atoms of one brick are contiguous
// slots after sorting.
__device__ __forceinline__ int cell_key(const SysParams& sp, int cx, int cy, int cz)
{
    const int Bx = quot(cx, sp.inv_bdim[0]), By = quot(cy, sp.inv_bdim[1]), Bz = quot(cz, sp.inv_bdim[2]);
    const int lx = cx - Bx * sp.bdim[0], ly = cy - By * sp.bdim[1], lz = cz - Bz * sp.bdim[2];
    const int b = Bx + sp.nbk[0] * (By + sp.nbk[1] * Bz);
    return b * sp.bcells + lx + sp.bdim[0] * (ly + sp.bdim[1] * lz);
}

__device__ __forceinline__ void key_cell(const SysParams& sp, int key, int& cx, int& cy, int& cz)
{
    const int b = quot(key, sp.inv_bcells), l = key - b * sp.bcells;
    const int Bz = quot(b, sp.inv_nbk01), b2 = b - Bz * sp.nbk[0] * sp.nbk[1];
    const int By = quot(b2, sp.inv_nbk0), Bx = b2 - By * sp.nbk[0];
    const int lz = quot(l, sp.inv_bdim[0] * sp.inv_bdim[1]), l2 = l - lz * sp.bdim[0] * sp.bdim[1];
    const int ly = quot(l2, sp.inv_bdim[0]), lx = l2 - ly * sp.bdim[0];
    cx = Bx * sp.bdim[0] + lx;
    cy = By * sp.bdim[1] + ly;
    cz = Bz * sp.bdim[2] + lz;
}

struct SlotCtx {
    int s, li, i;
};

// Per-atom kernels: kRebuildBlock threads = kRebuildBlock slots of one system.
__device__ __forceinline__ bool rebuild_ctx(const PoolDev& P, SlotCtx& c)
{
    const int lb = logical_block();
    const int chunk = lb * (kRebuildBlock / kChunk);
    if (chunk >= P.nchunk) return false;
    const int s = P.chunk_sys[chunk];
    if (s < 0) return false;
    const SysState* st = P.st + s;
    if (st->remaining <= 0 || (st->status & (ST_NONFINITE | ST_STALL))) return false;
    const SysParams* sp = P.sp + s;
    c.s = s;
    c.li = (chunk - sp->choff) * kChunk + (int)threadIdx.x;
    c.i = sp->voff + c.li;
    return true;
}

// First slot of cell c of a system between the scan and the placement
// (tile offset + prefix inside the tile).
__device__ __forceinline__ int cell_begin(const PoolDev& P, const SysParams& sp, int c)
{
    return P.ctile[sp.toff + c / kTile] + P.clocal[sp.coff + c];
}

__global__ void k_bin_count(PoolDev P)
{
    SlotCtx c;
    if (!rebuild_ctx(P, c)) return;
    const SysParams& sp = P.sp[c.s];
    const SysState& st = P.st[c.s];
    const int vt = P.vt;
    int cell;
    if (c.li < sp.nv) {
        const int b = st.sbuf;
        double* X = P.X[b];
        double x = X[c.i], y = X[vt + c.i], z = X[2 * vt + c.i];
        if (st.phase == PH_REST) {
            // first half of the run's first step (F2): v += a dt/2, x += v dt
            double* Vv = P.V[b];
            const double hdt = 0.5 * sp.dt;
            double vx = Vv[c.i] + hdt * P.A[c.i];
            double vy = Vv[vt + c.i] + hdt * P.A[vt + c.i];
            double vz = Vv[2 * vt + c.i] + hdt * P.A[2 * vt + c.i];
            x = wrap_box(x + vx * sp.dt, sp.L[0]);
            y = wrap_box(y + vy * sp.dt, sp.L[1]);
            z = wrap_box(z + vz * sp.dt, sp.L[2]);
            Vv[c.i] = vx;
            Vv[vt + c.i] = vy;
            Vv[2 * vt + c.i] = vz;
            X[c.i] = x;
            X[vt + c.i] = y;
            X[2 * vt + c.i] = z;
        }
        const int cx = cell_axis(x, sp.inv_h[0], sp.nc[0]);
        const int cy = cell_axis(y, sp.inv_h[1], sp.nc[1]);
        const int cz = cell_axis(z, sp.inv_h[2], sp.nc[2]);
        cell = cell_key(sp, cx, cy, cz);
    } else {
        cell = sp.nkey;  // padding slots gather in one extra cell
    }
    P.cell_tmp[c.i] = cell;
    // One atomic per distinct cell of the wave (atoms arrive cell-sorted from
    // the last rebuild, so a wave holds a few cells): the lowest lane of each
    // cell adds the cell's lane count, and each lane's arrival rank is the
    // returned base plus its rank among the cell's lanes.  The ranks are
    // unique within a cell, which is all the placement needs.
    const int g = sp.coff + cell;  // count index, distinct across systems
    const int lane = (int)(threadIdx.x & 63);
    unsigned long long todo = __ballot(1);
    int base = 0, rank = 0, lead = lane;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int key = __shfl(g, leader, 64);
        const unsigned long long m = __ballot(g == key);
        if (g == key) {
            rank = __popcll(m & ((1ull << lane) - 1ull));
            lead = leader;
            if (lane == leader) base = atomicAdd(&P.count[key], __popcll(m));
        }
        todo &= ~m;
    }
    P.arr[c.i] = __shfl(base, lead, 64) + rank;
}

// One workgroup (1024 threads x 4 cells) per scan tile writes the exclusive
// prefix of its tile and the tile sum.  Counts run over nkey + 2 entries
// (cells, padding cell, a zero end entry), so the prefix at nkey + 1 is the
// system's slot count.
__global__ void __launch_bounds__(1024) k_bin_scan(PoolDev P)
{
    __shared__ int lds[17];
    const int tile = blockIdx.x;
    if (tile >= P.ntile) return;
    const int s = P.tile_sys[tile];
    const SysParams& sp = P.sp[s];
    const SysState* st = P.st + s;
    if (!sp.active || st->remaining <= 0 || (st->status & (ST_NONFINITE | ST_STALL))) return;
    const int lt = tile - sp.toff;
    const int M = sp.nkey + 2;
    const int c0 = lt * kTile + 4 * (int)threadIdx.x;
    int* cnt = P.count + sp.coff;
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (c0 + k < M) ? cnt[c0 + k] : 0;
    const int sum = v[0] + v[1] + v[2] + v[3];
    int tot;
    int run = block_exclusive_scan(sum, lds, &tot);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (c0 + k < M) {
            P.clocal[sp.coff + c0 + k] = run;
            run += v[k];
            cnt[c0 + k] = 0;
        }
    if (threadIdx.x == 0) P.ctile[sp.toff + lt] = tot;
}

// One workgroup per system: tile sums -> slot offsets; advance the rebuild
// state (swap the state buffers, clear halts, start the run).
__global__ void k_bin_scan_finish(PoolDev P, int nslots)
{
    const int s = blockIdx.x;
    if (s >= nslots || threadIdx.x != 0) return;
    const SysParams& sp = P.sp[s];
    SysState* st = P.st + s;
    if (!sp.active || st->remaining <= 0 || (st->status & (ST_NONFINITE | ST_STALL))) return;
    int off = sp.voff;
    for (int t = 0; t < sp.ntile; ++t) {
        const int q = P.ctile[sp.toff + t];
        P.ctile[sp.toff + t] = off;
        off += q;
    }
    st->sbuf_prev = st->sbuf;
    st->sbuf ^= 1;
    st->ibuf_prev = st->ibuf;
    st->ibuf ^= 1;
    st->status &= ~(ST_HALT | ST_OVERFLOW | ST_TILE | ST_SPAN);
    if (st->phase == PH_REST) st->phase = PH_RUN;
    st->rebins += 1;
    st->max_nbr = 0;
    st->steps_since = 0;
}

__global__ void k_bin_scatter(PoolDev P)
{
    SlotCtx c;
    if (!rebuild_ctx(P, c)) return;
    const SysParams& sp = P.sp[c.s];
    const int cell = P.cell_tmp[c.i];
    const int q = cell_begin(P, sp, cell) + P.arr[c.i];
    P.tmp[q] = c.i;
    // the caller index beside it, so the placement ranks a cell's arrivals
    // from one contiguous range instead of a gather per arrival
    P.tmpid[q] = P.id[P.st[c.s].ibuf_prev][c.i];
}

template <typename T>
__global__ void k_bin_place(PoolDev P)
{
    using V = typename V4<T>::type;
    SlotCtx c;
    if (!rebuild_ctx(P, c)) return;
    const SysParams& sp = P.sp[c.s];
    const SysState& st = P.st[c.s];
    const int vt = P.vt;
    const int src = st.sbuf_prev, dst = st.sbuf;
    const int o = P.tmp[c.i];
    const int cell = P.cell_tmp[o];
    const int b0 = cell_begin(P, sp, cell), b1 = cell_begin(P, sp, cell + 1);
    const int myid = P.tmpid[c.i];
    int rank = 0;
    // the caller indices of the cell's arrivals eight at a time, loads
    // issued together (indices clamped to the cell's last arrival)
    for (int q = b0; q < b1; q += 8) {
        int idq[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) idq[u] = P.tmpid[min(q + u, b1 - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) rank += (q + u < b1 && idq[u] < myid) ? 1 : 0;
    }
    const int d = b0 + rank;
    const double* Xs = P.X[src];
    const double* Vs = P.V[src];
    double* Xd = P.X[dst];
    double* Vd = P.V[dst];
    const double x = Xs[o], y = Xs[vt + o], z = Xs[2 * vt + o];
    Xd[d] = x;
    Xd[vt + d] = y;
    Xd[2 * vt + d] = z;
    Vd[d] = Vs[o];
    Vd[vt + d] = Vs[vt + o];
    Vd[2 * vt + d] = Vs[2 * vt + o];
    P.id[st.ibuf][d] = myid;
    V* Lc = (V*)P.L[st.lbuf];
    if (cell < sp.nkey) {
        int cx, cy, cz;
        key_cell(sp, cell, cx, cy, cz);
        P.cref[d] = cx | (cy << 10) | (cz << 20);
        P.cell_lin[d] = cx + sp.nc[0] * (cy + sp.nc[1] * cz);
        const double lx = local_axis(x, cx, sp.h[0], sp.L[0], sp.invL[0]);
        const double ly = local_axis(y, cy, sp.h[1], sp.L[1], sp.invL[1]);
        const double lz = local_axis(z, cz, sp.h[2], sp.L[2], sp.invL[2]);
        Lc[d] = make4<T>(lx, ly, lz);
        P.lref[d] = make4<float>(lx, ly, lz);
    } else {
        P.cref[d] = 0;
        P.cell_lin[d] = -1;
        Lc[d] = make4<T>(0.0, 0.0, 0.0);
        P.lref[d] = make4<float>(0.0, 0.0, 0.0);
    }
    // final cell table for the list build and the readbacks
    for (int q = c.li; q < sp.nkey + 2; q += sp.vcap) P.cstart[sp.coff + q] = cell_begin(P, sp, q);
}

// ---------------------------------------------------------------------------
// Brick kernels: one workgroup per brick of cells.  The brick's halo box
// (the brick plus one cell on every side, (bx+2)(by+2)(bz+2) cells, periodic)
// is staged in LDS; every neighbour cell of an atom of the brick lies inside
// it, so the list build and the step kernel read neighbours from LDS.
// ---------------------------------------------------------------------------

struct BrickCtx {
    int s, b;  // system slot, brick index within the system
};

__device__ __forceinline__ bool brick_ctx(const PoolDev& P, BrickCtx& c, int bad_bits)
{
    const int lb = P.brick_order == 2 ? (int)blockIdx.x : logical_block();
    if (lb >= P.nbrick) return false;
    const int s = P.brick_sys[lb];
    if (s < 0) return false;
    const SysState* st = P.st + s;
    if (st->remaining <= 0 || (st->status & bad_bits)) return false;
    c.s = s;
    c.b = lb - P.sp[s].broff;
    return true;
}

struct HaloGeo {
    int start[3];  // first cell of the brick along each axis
    int hd[3];     // halo box extent (brick extent + 2)
    int H;         // halo cells
    double inv0, inv01;  // 1 / hd[0], 1 / (hd[0] hd[1])
};

// Halo cell h as (hx, hy, hz), x fastest (exact quotients, see quot).
__device__ __forceinline__ void halo_xyz(const HaloGeo& g, int h, int& hx, int& hy, int& hz)
{
    hz = quot(h, g.inv01);
    const int r = h - hz * g.hd[0] * g.hd[1];
    hy = quot(r, g.inv0);
    hx = r - hy * g.hd[0];
}

__device__ __forceinline__ HaloGeo halo_geo(const SysParams& sp, int b)
{
    HaloGeo g;
    const int B[3] = {b % sp.nbk[0], (b / sp.nbk[0]) % sp.nbk[1], b / (sp.nbk[0] * sp.nbk[1])};
    g.H = 1;
    for (int k = 0; k < 3; ++k) {
        g.start[k] = B[k] * sp.bdim[k];
        const int end = min(sp.nc[k], g.start[k] + sp.bdim[k]);
        g.hd[k] = end - g.start[k] + 2;
        g.H *= g.hd[k];
    }
    g.inv0 = 1.0 / g.hd[0];
    g.inv01 = 1.0 / (g.hd[0] * g.hd[1]);
    return g;
}

// A staged position in the LDS tile: the float4 itself in FP32 (one 16-byte
// access), x, y, z in FP64 (24 bytes instead of 32, so that more workgroups
// fit a compute unit's LDS).
struct d3t {
    double x, y, z;
};
template <typename T> struct TileAtom;
template <> struct TileAtom<float> { using type = f4; };
template <> struct TileAtom<double> { using type = d3t; };

__device__ __forceinline__ f4 tile_get(const f4* p) { return *p; }
__device__ __forceinline__ d4 tile_get(const d3t* p)
{
    d4 v;
    v.x = p->x;
    v.y = p->y;
    v.z = p->z;
    v.w = 0.0;
    return v;
}
__device__ __forceinline__ void tile_put(f4* p, const f4& v) { *p = v; }
__device__ __forceinline__ void tile_put(d3t* p, const d4& v)
{
    p->x = v.x;
    p->y = v.y;
    p->z = v.z;
}

// LDS tile: staged positions, their slots, and per halo cell the first slot
// and the first staged index.
template <typename T>
struct Tile {
    typename TileAtom<T>::type* pos;
    int* slot;
    int* hbeg;   // [hmax] first slot of the halo cell
    int* hoff;   // [hmax + 1] first staged index of the halo cell
};

// Vapour tile of `cap` atoms at smem + offset.
template <typename T>
__device__ __forceinline__ Tile<T> tile_at(unsigned char* smem, size_t offset, int cap, int hmax)
{
    Tile<T> t;
    t.pos = (typename TileAtom<T>::type*)(smem + offset);
    t.slot = (int*)(smem + offset + (size_t)cap * sizeof(typename TileAtom<T>::type));
    t.hbeg = t.slot + cap;
    t.hoff = t.hbeg + hmax;
    return t;
}

template <typename T>
__device__ __forceinline__ size_t tile_size(int cap, int hmax)
{
    return ((size_t)cap * (sizeof(typename TileAtom<T>::type) + 4) + (size_t)(2 * hmax + 1) * 4 + 31) & ~(size_t)31;
}

template <typename T>
__device__ __forceinline__ Tile<T> tile_of(unsigned char* smem, const PoolDev& P)
{
    return tile_at<T>(smem, 0, P.lds_atoms, P.hmax);
}

template <typename T>
__device__ __forceinline__ size_t tile_bytes_of(const PoolDev& P)
{
    return tile_size<T>(P.lds_atoms, P.hmax);
}

// Stage the halo box of brick g into LDS.  Returns the number of staged
// atoms, or -1 if it exceeds the tile capacity.  with_pos = false stages
// only the slots.
template <typename T>
__device__ int stage_halo(const PoolDev& P, const SysParams& sp, const HaloGeo& g, Tile<T>& t,
                          const typename V4<T>::type* Lc, bool with_pos, int* lds_scan,
                          int cap = -1)
{
    if (cap < 0) cap = P.lds_atoms;
    const int T_ = blockDim.x;
    const int per = (g.H + T_ - 1) / T_;
    const int lo = threadIdx.x * per, hi = min(g.H, lo + per);
    int sum = 0;
    for (int h = lo; h < hi; ++h) {
        int hx, hy, hz;
        halo_xyz(g, h, hx, hy, hz);
        const int cx = wrap_cell(g.start[0] - 1 + hx, sp.nc[0]);
        const int cy = wrap_cell(g.start[1] - 1 + hy, sp.nc[1]);
        const int cz = wrap_cell(g.start[2] - 1 + hz, sp.nc[2]);
        const int key = cell_key(sp, cx, cy, cz);
        const int b0 = P.cstart[sp.coff + key];
        const int n = P.cstart[sp.coff + key + 1] - b0;
        t.hbeg[h] = b0;
        t.hoff[h] = n;  // count for now
        sum += n;
    }
    int tot;
    int run = block_exclusive_scan(sum, lds_scan, &tot);
    if (tot > cap) return -1;  // (tot is the same in every thread)
    // the thread owning a halo cell writes its first staged index and the
    // storage slots of its staged atoms (a cell's atoms are consecutive
    // slots)
    for (int h = lo; h < hi; ++h) {
        const int n = t.hoff[h], b0 = t.hbeg[h];
        t.hoff[h] = run;
        for (int k = 0; k < n; ++k) t.slot[run + k] = b0 + k;
        run += n;
    }
    if (threadIdx.x == 0) t.hoff[g.H] = tot;
    __syncthreads();
    if (with_pos) {
        // each thread issues 4 independent loads (indices clamped to a valid
        // staged atom) before storing the ones in range
        for (int a0 = threadIdx.x; a0 < tot; a0 += 4 * T_) {
            const int a1 = a0 + T_, a2 = a0 + 2 * T_, a3 = a0 + 3 * T_;
            const typename V4<T>::type v0 = Lc[t.slot[a0]];
            const typename V4<T>::type v1 = Lc[t.slot[min(a1, tot - 1)]];
            const typename V4<T>::type v2 = Lc[t.slot[min(a2, tot - 1)]];
            const typename V4<T>::type v3 = Lc[t.slot[min(a3, tot - 1)]];
            tile_put(t.pos + a0, v0);
            if (a1 < tot) tile_put(t.pos + a1, v1);
            if (a2 < tot) tile_put(t.pos + a2, v2);
            if (a3 < tot) tile_put(t.pos + a3, v3);
        }
    }
    __syncthreads();
    return tot;
}

// Halo cell of neighbour t (0..26) of an atom whose cell is (cx, cy, cz).
__device__ __forceinline__ int halo_cell(const HaloGeo& g, int cx, int cy, int cz, int t)
{
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const int hx = cx - g.start[0] + 1 + dx;
    const int hy = cy - g.start[1] + 1 + dy;
    const int hz = cz - g.start[2] + 1 + dz;
    return hx + g.hd[0] * (hy + g.hd[1] * hz);
}

// Squared distance from a point at local offset l (from its cell's origin,
// 0 <= l < h) to the box of the neighbour cell at offset d (-1, 0, 1).
__device__ __forceinline__ double box_gap(double l, int d, double h)
{
    return d < 0 ? l : d > 0 ? h - l : 0.0;
}

// Neighbour lists (radius r_c + skin for vapour, r_c + skin/2 for the fixed
// walls) of the atoms of one brick, in a fixed order: neighbour cells 0..26,
// staged order inside a cell; vapour entries first (16 bits each), then
// walls (32 bits each), each part padded to whole 16-byte chunks.  Vapour
// entries index the brick's staged tile, which the step kernel rebuilds
// identically from the same cell tables; wall entries are wall slots.  Wall
// candidates are read from global memory (the static wall coordinates stay
// in L2): staging them would size every brick's LDS for the densest wall
// halo and leave one workgroup per CU.
template <typename T>
__global__ void __launch_bounds__(kMaxBlock) k_list_build(PoolDev P)
{
    using V = typename V4<T>::type;
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ int lds_scan[17];
    BrickCtx c;
    if (!brick_ctx(P, c, ST_NONFINITE | ST_STALL)) return;
    const SysParams& sp = P.sp[c.s];
    const SysState& st = P.st[c.s];
    const int vt = P.vt;
    const V* Lc = (const V*)P.L[st.lbuf];
    const HaloGeo g = halo_geo(sp, c.b);
    Tile<T> t = tile_of<T>(smem, P);
    // wall slot range of every halo cell, next to the staged tile, so the
    // wall search reads its cell ranges from LDS
    int* wrange = (int*)(smem + tile_bytes_of<T>(P));
    {
        const int* wcs = P.wcstart + sp.wcoff;
        for (int h = threadIdx.x; h < g.H; h += blockDim.x) {
            int hx, hy, hz;
            halo_xyz(g, h, hx, hy, hz);
            const int cl = wrap_cell(g.start[0] - 1 + hx, sp.nc[0]) +
                           sp.nc[0] * (wrap_cell(g.start[1] - 1 + hy, sp.nc[1]) +
                                       sp.nc[1] * wrap_cell(g.start[2] - 1 + hz, sp.nc[2]));
            wrange[2 * h] = wcs[cl];
            wrange[2 * h + 1] = wcs[cl + 1];
        }
    }
    const int tot = stage_halo<T>(P, sp, g, t, Lc, true, lds_scan);
    const int key0 = c.b * sp.bcells;
    const int i0 = P.cstart[sp.coff + key0], i1 = P.cstart[sp.coff + key0 + sp.bcells];
    const V* Lw = Lc + vt;
    if (tot < 0) {
        for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) P.nlist[i] = 0;
        if (threadIdx.x == 0) atomicOr(&P.st[c.s].status, ST_OVERFLOW | ST_TILE);
        return;
    }
    const T rl2 = (T)sp.rl2, rw2 = (T)sp.rw2;
    // cells farther than the radius cannot hold a partner (with a margin for
    // the rounding of the local coordinates)
    const double cull_v = sp.rl2 * (1.0 + 1e-6), cull_w = sp.rw2 * (1.0 + 1e-6);
    const int cap = P.cap;
    // wall candidates per load round (a window is two rounds): four in both
    // precisions (rounds of 12 FP32 positions held 20 more registers and
    // made the rebuild slower)
    constexpr int kWallRound = 4;
    int mx = 0;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) {
        const V me = Lc[i];
        const int cr = P.cref[i];
        const int cx = cr & 1023, cy = (cr >> 10) & 1023, cz = cr >> 20;
        const double lx = (double)me.x, ly = (double)me.y, lz = (double)me.z;
        // the atom's own staged index (its cell's atoms are staged in slot
        // order; with at least 3 cells per axis the 27 cells are distinct, so
        // this is its only copy in the tile)
        const int hs = halo_cell(g, cx, cy, cz, 13);
        const int aself = t.hoff[hs] + (i - t.hbeg[hs]);
        // neighbour cells in the order q = (dx+1) + 3 (dy+1) + 9 (dz+1), as
        // nested z, y loops over rows of three cells: each level culls with
        // the partial box gap of the levels above it (a whole plane or row of
        // cells at once) and carries the atom's coordinate shifted into the
        // neighbour cell's frame (px = me.x - dx h_x, and so on)
        const int hstr1 = g.hd[0], hstr2 = g.hd[0] * g.hd[1];
        const T hx = (T)sp.h[0], hy = (T)sp.h[1], hz = (T)sp.h[2];
        // vapour entries are 16-bit: the partner's staged index relative to
        // the first staged atom of neighbour cell (-1, -1, -1) (the 27 cells
        // lie in the tile range from there to the end of cell (1, 1, 1)),
        // with the neighbour-cell code above; a range longer than the index
        // field stops the system until the host has shrunk its bricks
        const int base = t.hoff[halo_cell(g, cx, cy, cz, 0)];
        if (t.hoff[halo_cell(g, cx, cy, cz, 26) + 1] - base > (int)kRelMask + 1) {
            P.nlist[i] = 0;
            atomicOr(&P.st[c.s].status, ST_OVERFLOW | ST_TILE | ST_SPAN);
            continue;
        }
        // two entries per 32-bit store: an even entry waits in `pend`
        int nv = 0;
        unsigned pend = 0u;
        auto emit = [&](unsigned v) {
            if (nv & 1) {
                if ((nv >> 1) < cap) P.list[list_at(vt, i, nv >> 1)] = pend | (v << 16);
            } else {
                pend = v;
            }
            ++nv;
        };
#pragma unroll 1
        for (int dz = -1; dz <= 1; ++dz) {
            const double gz = box_gap(lz, dz, sp.h[2]), gz2 = gz * gz;
            if (gz2 >= cull_v) continue;
            const T pz = me.z - (T)dz * hz;
#pragma unroll 1
            for (int dy = -1; dy <= 1; ++dy) {
                const double gy = box_gap(ly, dy, sp.h[1]), gyz = fma(gy, gy, gz2);
                if (gyz >= cull_v) continue;
                const T py = me.y - (T)dy * hy;
                // the row's cells dx = -1, 0, 1 are consecutive in the tile
                // (x-fastest halo order): one candidate range, less the end
                // cells that lie beyond the radius; a candidate's x frame
                // follows from which cell's range holds it
                const int hrow = hs + dy * hstr1 + dz * hstr2;
                const int b1 = t.hoff[hrow], b2 = t.hoff[hrow + 1];
                const double gxm = box_gap(lx, -1, sp.h[0]), gxp = box_gap(lx, 1, sp.h[0]);
                const int lo = fma(gxm, gxm, gyz) >= cull_v ? b1 : t.hoff[hrow - 1];
                const int hi = fma(gxp, gxp, gyz) >= cull_v ? b2 : t.hoff[hrow + 2];
                const T pxm = me.x + hx, pxp = me.x - hx;  // frames of cells dx = -1, +1
                const unsigned qrow = (unsigned)(3 * (dy + 1) + 9 * (dz + 1));
                // windows of 32 candidates: the tests of a window set bits of
                // a mask (no branch per candidate), then only the hits are
                // written, in candidate order
                for (int w0 = lo; w0 < hi; w0 += 32) {
                    const int wend = min(hi, w0 + 32);
                    unsigned bits = 0u;
                    for (int a = w0; a < wend; a += 4) {
                        // four candidates through one pointer; the reads past
                        // the range's last atom (at most three, a + 3 <=
                        // cap + 2) stay inside the workgroup's LDS (the slot
                        // table follows the positions) and their bits are
                        // dropped below
                        const auto* pa = t.pos + a;
                        V o[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) o[u] = tile_get(pa + u);
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int ac = a + u;
                            const T px = ac < b1 ? pxm : (ac < b2 ? me.x : pxp);
                            const T ex = px - o[u].x, ey = py - o[u].y, ez = pz - o[u].z;
                            bits |= (unsigned)(ex * ex + ey * ey + ez * ez < rl2) << (a - w0 + u);
                        }
                    }
                    // candidates past the range's end, and the atom itself
                    const int nwin = wend - w0, dself = aself - w0;
                    bits &= nwin >= 32 ? ~0u : ((1u << nwin) - 1u);
                    bits &= ~((unsigned)(dself >= 0 && dself < 32) << (dself & 31));
                    while (bits) {
                        const int u = __builtin_ctz(bits);
                        bits &= bits - 1u;
                        const int ac = w0 + u;
                        const unsigned q = qrow + (unsigned)(ac >= b1) + (unsigned)(ac >= b2);
                        emit((unsigned)(ac - base) | (q << kRelBits));
                    }
                }
            }
        }
        // the vapour entries end on a chunk boundary: the rest of the last
        // chunk holds pad entries (the atom itself under the pad code), so the
        // step kernel reads whole groups with no per-entry length test
        const int nvap = nv;
        const int nvw = ((nv + 7) >> 3) << 2;  // 32-bit words of the vapour part
        while (nv < 2 * nvw) emit((unsigned)(aself - base) | (kPadQ << kRelBits));
        int nw = 0;
        unsigned lastw = 0;
#pragma unroll 1
        for (int dz = -1; dz <= 1; ++dz) {
            const double gz = box_gap(lz, dz, sp.h[2]), gz2 = gz * gz;
            if (gz2 >= cull_w) continue;
            const T pz = me.z - (T)dz * hz;
#pragma unroll 1
            for (int dy = -1; dy <= 1; ++dy) {
                const double gy = box_gap(ly, dy, sp.h[1]), gyz = fma(gy, gy, gz2);
                if (gyz >= cull_w) continue;
                const T py = me.y - (T)dy * hy;
#pragma unroll 1
                for (int dx = -1; dx <= 1; ++dx) {
                    const double gx = box_gap(lx, dx, sp.h[0]);
                    if (fma(gx, gx, gyz) >= cull_w) continue;
                    const int h = hs + dx + dy * hstr1 + dz * hstr2;
                    const int w0c = wrange[2 * h], w1 = wrange[2 * h + 1];
                    if (w0c >= w1) continue;
                    const T px = me.x - (T)dx * hx;
                    const unsigned code = (unsigned)((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)) << kIndexBits;
                    // windows of two rounds of kWallRound candidates (loads
                    // of a round issued together, indices clamped to the
                    // cell's last wall): tests into a mask, then the hits
                    for (int w0 = w0c; w0 < w1; w0 += 2 * kWallRound) {
                        unsigned bits = 0u;
#pragma unroll
                        for (int rd = 0; rd < 2; ++rd) {
                            const int wr = w0 + rd * kWallRound;
                            V o[kWallRound];
#pragma unroll
                            for (int u = 0; u < kWallRound; ++u) o[u] = Lw[min(wr + u, w1 - 1)];
#pragma unroll
                            for (int u = 0; u < kWallRound; ++u) {
                                const T ex = px - o[u].x, ey = py - o[u].y, ez = pz - o[u].z;
                                bits |= (unsigned)(ex * ex + ey * ey + ez * ez < rw2) << (rd * kWallRound + u);
                            }
                        }
                        const int nwin = w1 - w0;
                        bits &= nwin >= 2 * kWallRound ? ~0u : ((1u << nwin) - 1u);
                        while (bits) {
                            const int u = __builtin_ctz(bits);
                            bits &= bits - 1u;
                            const unsigned w = (unsigned)(w0 + u);
                            if (nvw + nw < cap) P.list[list_at(vt, i, nvw + nw)] = w | code;
                            lastw = w;
                            ++nw;
                        }
                    }
                }
            }
        }
        // the wall entries start at word nvw (a chunk boundary) and end on a
        // chunk boundary too (pads: the last wall entry's slot under the pad
        // code); nt counts 32-bit words
        const int nt = nvw + ((nw + 3) & ~3);
        for (int k = nvw + nw; k < min(nt, cap); ++k) P.list[list_at(vt, i, k)] = lastw | kPadCode;
        const bool ok = nt <= cap;
        P.nlist[i] = ok ? (nvap | (nw << 16)) : 0;
        mx = max(mx, nt);
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0 && mx > 0) {
        atomicMax(&P.st[c.s].max_nbr, mx);
        if (mx > cap) atomicOr(&P.st[c.s].status, ST_OVERFLOW);
    }
}

size_t tile_bytes(const PoolDev& P, int precision)
{
    const size_t v = precision == 1 ? sizeof(f4) : 3 * sizeof(double);
    return ((size_t)P.lds_atoms * (v + 4) + (size_t)(2 * P.hmax + 1) * 4 + 31) & ~(size_t)31;
}

hipError_t launch_rebuild(const PoolDev& P, int nslots, int precision, hipStream_t s)
{
    const int nrb = P.nchunk / (kRebuildBlock / kChunk);
    const int G = ((nrb + 7) / 8) * 8;
    const int GB = ((P.nbrick + 7) / 8) * 8;
    if (G == 0) return hipSuccess;
    const size_t lds = tile_bytes(P, precision) + 8 * (size_t)P.hmax;  // tile + wall ranges
    hipLaunchKernelGGL(k_bin_count, dim3(G), dim3(kRebuildBlock), 0, s, P);
    hipLaunchKernelGGL(k_bin_scan, dim3(P.ntile), dim3(1024), 0, s, P);
    hipLaunchKernelGGL(k_bin_scan_finish, dim3(nslots), dim3(64), 0, s, P, nslots);
    hipLaunchKernelGGL(k_bin_scatter, dim3(G), dim3(kRebuildBlock), 0, s, P);
    if (precision == 1) {
        hipLaunchKernelGGL(k_bin_place<float>, dim3(G), dim3(kRebuildBlock), 0, s, P);
        hipLaunchKernelGGL(k_list_build<float>, dim3(GB), dim3(P.block), lds, s, P);
    } else {
        hipLaunchKernelGGL(k_bin_place<double>, dim3(G), dim3(kRebuildBlock), 0, s, P);
        hipLaunchKernelGGL(k_list_build<double>, dim3(GB), dim3(P.block), lds, s, P);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step: forces (F1) + second half-kick (F3) [+ next drift and half-kick (F2)]
// ---------------------------------------------------------------------------

// Whether the energies of step kstep are recorded: the initial evaluation,
// the last step of a run and every energy_every-th step.
__device__ __forceinline__ bool step_records(const SysParams& sp, bool init, bool last, long long kstep)
{
    return init || last || (sp.energy_every > 0 && (kstep % sp.energy_every) == 0);
}

// Sum one step's per-brick energy partials in brick order (fixed, so the
// total is deterministic) and append the record.  Called by a whole
// workgroup; the partials were written by an earlier launch.
// red: workgroup scratch of kPartial x (waves) doubles.
typedef double Red[kPartial][kMaxBlock / 64];

__device__ void record_energies(const PoolDev& P, const SysParams& sp, int s, int ring, long long kstep,
                                Red& red)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    const double* pp = P.partial + kPartial * ((size_t)ring * P.nbt + sp.pboff);
    double v[kPartial];
#pragma unroll
    for (int q = 0; q < kPartial; ++q) v[q] = 0.0;
    for (int b = tid; b < sp.nbrick; b += blockDim.x) {
#pragma unroll
        for (int q = 0; q < kPartial; ++q) v[q] += pp[kPartial * b + q];
    }
#pragma unroll
    for (int q = 0; q < kPartial; ++q) {
        const double t = wave_sum(v[q]);
        if (lane == 0) red[q][wave] = t;
    }
    __syncthreads();
    if (tid == 0) {
        double t[kPartial];
        for (int q = 0; q < kPartial; ++q) {
            t[q] = 0.0;
            for (int w = 0; w < nwave; ++w) t[q] += red[q][w];
        }
        SysState* sw = P.st + s;
        const int n = sw->nrec;
        EnergyRec r;
        r.step = kstep;
        r.ke = t[0];
        r.pe_vv = t[1];
        r.pe_vw = t[2];
        r.w_vv = t[3];
        r.w_vw = t[4];
        r.ke_pore = t[5];
        r.w_pore = t[6];
        r.n_pore = t[7];
        P.erec[sp.ering_off + (n % sp.ering_cap)] = r;
        sw->nrec = n + 1;
    }
    __syncthreads();
}

constexpr int kGroupV = 4;  // vapour list entries fetched together in the step kernel (multiple of 4)
// wall list entries (and wall positions) fetched together: one chunk of four
// in both precisions (groups of eight FP32 positions held four more
// registers and made the step about 1% slower)
template <typename T> constexpr int kGroupW = 4;



template <typename T>
__device__ __forceinline__ T inv_of(T r2);
template <>
__device__ __forceinline__ float inv_of<float>(float r2) { return __builtin_amdgcn_rcpf(r2); }
template <>
__device__ __forceinline__ double inv_of<double>(double r2) { return 1.0 / r2; }

// Per-workgroup context of one step of one system.
template <typename T>
struct StepCtx {
    using V = typename V4<T>::type;
    bool init, last, doE;
    bool thermo;           // Berendsen thermostat: the step ends in k_thermo
    int lbuf;
    const V* Lc;           // local coordinates read this step (walls at vt + w)
    const double* X;       // positions and velocities at the start of the step
    const double* Vv;
    double* Xn;            // ... and after it (the other buffer)
    double* Vn;
    T rc2, Av, Bv, Aw, Bw, A12v, B6v, A12w, B6w, ucv, ucw, band, hx, hy, hz;
    // FP64 constants of the integration, held in scalar registers
    double L[3], invL[3], h[3], dt, hdt, mass, inv_mass;
    float half_skin;
};

// A workgroup-uniform value moved into scalar registers, which frees the
// vector registers a per-lane copy would hold through the kernel.
__device__ __forceinline__ double uniform_f64(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ float uniform_f32(float v)
{
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}

template <typename T>
__device__ __forceinline__ StepCtx<T> step_ctx(const PoolDev& P, const SysParams& sp, const SysState& st, int kk)
{
    StepCtx<T> x;
    x.init = st.phase == PH_INIT;
    x.last = !x.init && kk == st.remaining - 1;
    const long long kstep = x.init ? st.step : st.step + kk + 1;
    x.thermo = !x.init && sp.thermo;
    // the thermostat needs every step's kinetic energy
    x.doE = step_records(sp, x.init, x.last, kstep) || x.thermo;
    x.lbuf = st.lbuf ^ (kk & 1);
    x.Lc = (const typename V4<T>::type*)P.L[x.lbuf];
    // positions and velocities: read from one buffer, written to the other,
    // so every workgroup (the cutoff-edge re-test reads partners' positions)
    // sees the positions at the start of the step
    const int xb = x.init ? st.sbuf : st.sbuf ^ (kk & 1);
    x.X = P.X[xb];
    x.Vv = P.V[xb];
    x.Xn = P.X[xb ^ 1];
    x.Vn = P.V[xb ^ 1];
    x.rc2 = (T)sp.rc2;
    x.Av = (T)sp.A;
    x.Bv = (T)sp.B;
    x.Aw = (T)sp.Aw;
    x.Bw = (T)sp.Bw;
    x.A12v = (T)12 * x.Av;
    x.B6v = (T)6 * x.Bv;
    x.A12w = (T)12 * x.Aw;
    x.B6w = (T)6 * x.Bw;
    x.ucv = (T)sp.uc;
    x.ucw = (T)sp.ucw;
    x.band = (T)(4.0e-6 * sp.rc2);
    x.hx = (T)sp.h[0];
    x.hy = (T)sp.h[1];
    x.hz = (T)sp.h[2];
    for (int k = 0; k < 3; ++k) {
        x.L[k] = uniform_f64(sp.L[k]);
        x.invL[k] = uniform_f64(sp.invL[k]);
        x.h[k] = uniform_f64(sp.h[k]);
    }
    x.dt = uniform_f64(sp.dt);
    x.hdt = uniform_f64(0.5 * sp.dt);
    x.mass = uniform_f64(sp.mass);
    x.inv_mass = uniform_f64(sp.inv_mass);
    x.half_skin = uniform_f32(sp.half_skin);
    return x;
}

// Per-atom force and energy sums (FP64).
struct Acc {
    double fx, fy, fz, ev, ew;
    double wv, ww;  // virial sums r . f (vapour and wall partners)
};

// One in-cutoff pair: FP32 (mixed) or FP64 LJ, FP64 sums; on recording
// steps also its energy and, with VIR, its r . f.
template <typename T, bool VIR>
__device__ __forceinline__ void pair_term(const StepCtx<T>& x, Acc& a, T dx, T dy, T dz, T r2, bool wall)
{
    const T A = wall ? x.Aw : x.Av, B = wall ? x.Bw : x.Bv;
    const T sr2 = inv_of<T>(r2);
    const T sr6 = sr2 * sr2 * sr2;
    const double w = (double)(sr2 * sr6 * ((wall ? x.A12w : x.A12v) * sr6 - (wall ? x.B6w : x.B6v)));
    a.fx = fma(w, (double)dx, a.fx);
    a.fy = fma(w, (double)dy, a.fy);
    a.fz = fma(w, (double)dz, a.fz);
    if (x.doE) {
        const double u_ = (double)(sr6 * (A * sr6 - B) - (wall ? x.ucw : x.ucv));
        if (wall)
            a.ew += u_;
        else
            a.ev += u_;
        if constexpr (VIR) {
            const double v_ = w * (double)r2;  // r . f of the pair
            if (wall)
                a.ww += v_;
            else
                a.wv += v_;
        }
    }
}

// List entry k of atom i if its FP32 r^2 lies within the band around the
// cutoff: the pair is decided on the FP64 master positions.
// List position k of atom i: vapour entry k for k < nvap, else wall entry
// k - nvap (whose words start at word nvw); base is the atom's neighbourhood
// base in the staged tile.
template <typename T, bool VIR>
__device__ __forceinline__ void edge_entry(const PoolDev& P, const SysParams& sp, const StepCtx<T>& x,
                                           const Tile<T>& tl, const typename V4<T>::type* lut, int i,
                                           int k, int nvap, int base, const typename V4<T>::type& me,
                                           double xi, double yi, double zi, Acc& a)
{
    using V = typename V4<T>::type;
    const int vt = P.vt;
    const bool wall = k >= nvap;
    int ai, q;
    if (wall) {
        const int nvw = ((nvap + 7) >> 3) << 2;
        const unsigned e = P.list[list_at(vt, i, nvw + k - nvap)];
        ai = (int)(e & kIndexMask);
        q = (int)(e >> kIndexBits);
    } else {
        const unsigned e = ((const unsigned short*)P.list)[vlist_at(vt, i, k)];
        ai = base + (int)(e & kRelMask);
        q = (int)(e >> kRelBits);
    }
    const V o = wall ? x.Lc[vt + ai] : tile_get(tl.pos + ai);
    const V sh = lut[q];
    const T dx = me.x - o.x + sh.x;
    const T dy = me.y - o.y + sh.y;
    const T dz = me.z - o.z + sh.z;
    const T r2 = dx * dx + dy * dy + dz * dz;
    if (!(fabs(r2 - x.rc2) < x.band)) return;
    double ox, oy, oz;
    if (wall) {
        ox = P.WX[ai];
        oy = P.WX[P.wt + ai];
        oz = P.WX[2 * P.wt + ai];
    } else {
        const int j = tl.slot[ai];
        ox = x.X[j];
        oy = x.X[vt + j];
        oz = x.X[2 * vt + j];
    }
    double ex = xi - ox, ey = yi - oy, ez = zi - oz;
    ex -= sp.L[0] * rint(ex * sp.invL[0]);
    ey -= sp.L[1] * rint(ey * sp.invL[1]);
    ez -= sp.L[2] * rint(ez * sp.invL[2]);
    if (ex * ex + ey * ey + ez * ez < sp.rc2) pair_term<T, VIR>(x, a, dx, dy, dz, r2, wall);
}

// The pairs of atom i that the pair loops left out (FP32 r^2 within the band
// around the cutoff), decided on the FP64 master positions and added in list
// order.  The loops record the list positions of the last two such entries
// (k0 the later one; ne counts them all); only an atom with more than two
// rescans its list (positions 0 .. nvap - 1 for the vapour entries, nvap on
// for the wall entries).
template <typename T, bool VIR>
__device__ void edge_pass(const PoolDev& P, const SysParams& sp, const StepCtx<T>& x,
                          const Tile<T>& tl, const typename V4<T>::type* lut, int i, int nvap, int nwal,
                          int base, int ne, int k0, int k1, Acc& a)
{
    const int vt = P.vt;
    const typename V4<T>::type me = x.Lc[i];
    const double xi = x.X[i], yi = x.X[vt + i], zi = x.X[2 * vt + i];
    if (ne <= 2) {
        if (ne == 2) edge_entry<T, VIR>(P, sp, x, tl, lut, i, k1, nvap, base, me, xi, yi, zi, a);
        edge_entry<T, VIR>(P, sp, x, tl, lut, i, k0, nvap, base, me, xi, yi, zi, a);
        return;
    }
    for (int k = 0; k < nvap + nwal; ++k)
        edge_entry<T, VIR>(P, sp, x, tl, lut, i, k, nvap, base, me, xi, yi, zi, a);
}

// What a lane reads of its atom before the pair loops: the local position,
// the list lengths and the first list chunk.  They are independent loads,
// issued together; for a lane's first atom they are issued before the halo
// staging and arrive while it runs.  (Preloading the epilogue's position and
// velocity too holds 12 more registers through the pair loops, which spill.)
template <typename T>
struct AtomIn {
    typename V4<T>::type me;
    int nl;
    int cr;  // packed cell coordinates (the neighbourhood base in the tile follows from them)
    uint4 c0;
};

template <typename T>
__device__ __forceinline__ AtomIn<T> atom_in(const PoolDev& P, const StepCtx<T>& x, int i)
{
    const int vt = P.vt;
    AtomIn<T> r;
    r.me = x.Lc[i];
    r.nl = P.nlist[i];
    r.cr = P.cref[i];
    r.c0 = ((const uint4*)P.list)[i];  // chunk 0 of slot i
    (void)vt;
    return r;
}

// F3 (second half-kick) and, unless the run ends, F2 of the next step (first
// half-kick, drift, wrap, local coordinates, displacement since the last
// rebuild).  Returns the kinetic energy at the full step; raises halt and
// non-finite bits.
template <typename T>
__device__ double atom_epilogue(const PoolDev& P, const StepCtx<T>& x, int i,
                                const Acc& a, int& flags)
{
    using V = typename V4<T>::type;
    const int vt = P.vt;
    const double xi = x.X[i], yi = x.X[vt + i], zi = x.X[2 * vt + i];
    double vx = x.Vv[i], vy = x.Vv[vt + i], vz = x.Vv[2 * vt + i];
    const double ax = a.fx * x.inv_mass, ay = a.fy * x.inv_mass, az = a.fz * x.inv_mass;
    if (x.init) {
        P.A[i] = ax;
        P.A[vt + i] = ay;
        P.A[2 * vt + i] = az;
    } else {
        const double hdt = x.hdt;
        vx += hdt * ax;  // F3: v(t) = v(t - dt/2) + a(t) dt/2
        vy += hdt * ay;
        vz += hdt * az;
    }
    const double kei = 0.5 * x.mass * (vx * vx + vy * vy + vz * vz);
    if (!x.init) {
        // the last step of a run, and every step under the thermostat (whose
        // scaling needs the whole system's temperature first), stores the
        // full-step state; k_thermo then scales v and drifts
        if (x.last || x.thermo) {
            x.Xn[i] = xi;
            x.Xn[vt + i] = yi;
            x.Xn[2 * vt + i] = zi;
            x.Vn[i] = vx;
            x.Vn[vt + i] = vy;
            x.Vn[2 * vt + i] = vz;
            P.A[i] = ax;
            P.A[vt + i] = ay;
            P.A[2 * vt + i] = az;
        } else {
            const double hdt = x.hdt;
            vx += hdt * ax;  // F2 of the next step: v(t + dt/2) = v(t) + a(t) dt/2
            vy += hdt * ay;
            vz += hdt * az;
            const double xx = wrap_box(xi + vx * x.dt, x.L[0]);
            const double yy = wrap_box(yi + vy * x.dt, x.L[1]);
            const double zz = wrap_box(zi + vz * x.dt, x.L[2]);
            x.Vn[i] = vx;
            x.Vn[vt + i] = vy;
            x.Vn[2 * vt + i] = vz;
            x.Xn[i] = xx;
            x.Xn[vt + i] = yy;
            x.Xn[2 * vt + i] = zz;
            const int cr = P.cref[i];
            const int cx = cr & 1023, cy = (cr >> 10) & 1023, cz = cr >> 20;
            V* Ln = (V*)P.L[x.lbuf ^ 1];
            const double lx = local_axis(xx, cx, x.h[0], x.L[0], x.invL[0]);
            const double ly = local_axis(yy, cy, x.h[1], x.L[1], x.invL[1]);
            const double lz = local_axis(zz, cz, x.h[2], x.L[2], x.invL[2]);
            Ln[i] = make4<T>(lx, ly, lz);
            // displacement since the last rebuild: both local positions are
            // measured from the same cell origin (minimum image)
            const f4 r = P.lref[i];
            const float ex = (float)lx - r.x, ey = (float)ly - r.y, ez = (float)lz - r.z;
            if (ex * ex + ey * ey + ez * ez > x.half_skin * x.half_skin) flags |= ST_HALT;
        }
    }
    if (!isfinite(a.fx + a.fy + a.fz) || !isfinite(kei)) flags |= ST_NONFINITE;
    return kei;
}

// Whether a position lies in the pore's void (the hole through the slab, the
// slit's gap, the whole box without walls; nothing for a plain slab): the
// region of the pressure in the pore.
__device__ __forceinline__ bool in_pore(const SysParams& sp, double x, double y, double z)
{
    if (sp.pkind == 0) return true;
    if (sp.pkind == 1 || z < sp.pz0 || z >= sp.pz1) return false;
    if (sp.pkind == 3) return true;
    const double t = sp.pz1 - sp.pz0, h = z - sp.pz0;
    double r = sp.pr0;
    if (sp.pkind == 4) r = sp.pr0 + (sp.pr1 - sp.pr0) * (h / t);
    if (sp.pkind == 5) r = (h < 0.25 * t || h >= 0.75 * t) ? sp.pr0 : sp.pr1;
    const double dx = x - 0.5 * sp.L[0], dy = y - 0.5 * sp.L[1];
    return dx * dx + dy * dy < r * r;
}

// Workgroup reductions in a fixed order (lane tree, then waves in order):
// status bits to the system, energies to the brick's partial of slot kk & 1.
__device__ void step_reduce(const PoolDev& P, const SysParams& sp, int s, int b, int kk, bool doE,
                            int flags, double ke, double evv, double evw, double wvv, double wvw,
                            double kp, double wp, double np, Red& red)
{
    __shared__ int flag_or[kMaxBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    flags = wave_or(flags);
    if (lane == 0) flag_or[wave] = flags;
    if (doE) {
        const double v[kPartial] = {ke, evv, evw, wvv, wvw, kp, wp, np};
#pragma unroll
        for (int q = 0; q < kPartial; ++q) {
            const double t = wave_sum(v[q]);
            if (lane == 0) red[q][wave] = t;
        }
    }
    __syncthreads();
    if (tid == 0) {
        int f = 0;
        for (int w = 0; w < nwave; ++w) f |= flag_or[w];
        if (f) {
            atomicOr(&P.st[s].status_next, f);
            if (f & (ST_HALT | ST_NONFINITE | ST_OVERFLOW)) atomicMin(&P.st[s].stop, kk);
        }
        if (doE) {
            double* pp = P.partial + kPartial * ((size_t)(kk & 1) * P.nbt + sp.pboff + b);
            for (int q = 0; q < kPartial; ++q) {
                double t = 0.0;
                for (int w = 0; w < nwave; ++w) t += red[q][w];
                pp[q] = t;
            }
        }
    }
}

// A list entry in the band around the cutoff: counted, and the list
// positions of the last two kept (k0 the latest) for the pass that decides
// them in FP64.
__device__ __forceinline__ void note_edge(int& ne, int& k0, int& k1, int k, bool near)
{
    k1 = near ? k0 : k1;
    k0 = near ? k : k0;
    ne += near;
}

// The cutoff-band entries of one group of G list entries starting at list
// position k: a branch on the whole wave (band entries are rare, about one
// group in a thousand holds one in any lane), so the common case costs a few
// scalar instructions instead of the bookkeeping per entry; the empty asm
// keeps the compiler from turning the branch back into selects.
template <int G>
__device__ __forceinline__ void note_group(const bool (&nr)[G], int& ne, int& k0, int& k1, int k)
{
    bool any = false;
#pragma unroll
    for (int u = 0; u < G; ++u) any |= nr[u];
    if (__builtin_amdgcn_ballot_w64(any) != 0) {
        asm volatile("");
#pragma unroll
        for (int u = 0; u < G; ++u) note_edge(ne, k0, k1, k + u, nr[u]);
    }
}

// One list entry's pair with no branch: w (and the energy) is masked to 0
// unless `in` (a live entry inside the cutoff and outside the band), and r^2
// is replaced by 1 where masked, so no infinity or NaN is formed; adding
// the masked zero leaves every sum exactly as a skipped pair would.
template <typename T, bool VIR, bool DOE>
__device__ __forceinline__ void pair_masked(const StepCtx<T>& x, Acc& a, T dx, T dy, T dz, T r2, bool in,
                                            bool wall)
{
    const T sr2 = inv_of<T>(in ? r2 : (T)1);
    const T sr6 = sr2 * sr2 * sr2;
    const T wf = sr2 * sr6 * ((wall ? x.A12w : x.A12v) * sr6 - (wall ? x.B6w : x.B6v));
    // w d added in FP64 (one rounding: the FP64 product of two FP32 values is
    // exact); the pair's two atoms add exact negatives
    const double w = (double)(in ? wf : (T)0);
    a.fx = fma(w, (double)dx, a.fx);
    a.fy = fma(w, (double)dy, a.fy);
    a.fz = fma(w, (double)dz, a.fz);
    if constexpr (DOE) {
        const T u = sr6 * ((wall ? x.Aw : x.Av) * sr6 - (wall ? x.Bw : x.Bv)) - (wall ? x.ucw : x.ucv);
        const double ud = (double)(in ? u : (T)0);
        if (wall)
            a.ew += ud;
        else
            a.ev += ud;
        if constexpr (VIR) {
            const double vd = w * (double)r2;  // r . f of the pair
            if (wall)
                a.ww += vd;
            else
                a.wv += vd;
        }
    }
}

// The brick's atoms, one lane each: the pair loops, the rare cutoff-band
// pass, the epilogue (F3 and the next F2); DOE: a recording step (energies,
// with VIR the virial sums and the pore's sums too).
template <typename T, bool VIR, bool DOE>
__device__ __forceinline__ void step_atoms(PoolDev& P, const SysParams& sp, const StepCtx<T>& x,
                                           const HaloGeo& g, const Tile<T>& tl,
                                           const typename V4<T>::type* lut, int i0, int i1,
                                           const AtomIn<T>& first, Acc& a, double& ke, double& lwv,
                                           double& lkp, double& lwp, double& lnp, int& flags)
{
    using V = typename V4<T>::type;
    const int vt = P.vt;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) {
        const AtomIn<T> in = i == i0 + (int)threadIdx.x ? first : atom_in<T>(P, x, i);
        const V me = in.me;
        const int nl = in.nl;
        const int nvap = nl & 0xFFFF;
        a.fx = a.fy = a.fz = 0.0;
        if constexpr (VIR) a.wv = 0.0;
        // entries come in 16-byte chunks (one load each): eight 16-bit
        // vapour entries (two groups) or four 32-bit wall entries per chunk,
        // kGroupW<T> / 4 chunks per wall group; the next chunk is in flight
        // while the current one is evaluated, and a group's partner
        // positions (from LDS for vapour, from global memory for walls) and
        // shifts are all read before any is used.  Each part of the list
        // ends on a chunk boundary with pad entries whose shift puts the
        // partner beyond the cutoff, so no entry needs a length test.  Pairs
        // whose FP32 r^2 lies within a narrow band around the cutoff are left
        // out here and decided in FP64 after the whole list (a rare slow
        // path: a few atoms per step).  Chunk loads past the end of this
        // atom's list are clamped to the capacity and their values are not
        // used, so the code is straight-line and each wait covers only the
        // loads it needs
        int ne = 0, ke0 = 0, ke1 = 0;  // cutoff-band entries: count, last two list positions
        const int nwal = nl >> 16;
        const int lastchunk = P.cap / 4 - 1;
        const uint4* lst4 = (const uint4*)P.list + i;  // chunk c of this atom at lst4[c * vt]
        // the atom's neighbourhood in the tile starts at the first staged
        // atom of its neighbour cell (-1, -1, -1)
        const auto* posb = tl.pos + tl.hoff[halo_cell(g, in.cr & 1023, (in.cr >> 10) & 1023, in.cr >> 20, 0)];
        static_assert(kGroupV == 4, "the vapour loop takes half a 16-byte chunk per group");
        // one group of four vapour entries (two 32-bit words of a chunk) at
        // list position k
        auto vapour_group = [&](const unsigned w0, const unsigned w1, int k) {
            const unsigned ec[4] = {w0 & 0xFFFFu, w0 >> 16, w1 & 0xFFFFu, w1 >> 16};
            V o[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) o[u] = tile_get(posb + (ec[u] & kRelMask));
            V sh[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) sh[u] = lut[ec[u] >> kRelBits];
            bool nr[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const T dx = me.x - o[u].x + sh[u].x;
                const T dy = me.y - o[u].y + sh[u].y;
                const T dz = me.z - o[u].z + sh[u].z;
                const T r2 = dx * dx + dy * dy + dz * dz;
                nr[u] = sizeof(T) == 4 && fabs(r2 - x.rc2) < x.band;
                pair_masked<T, VIR, DOE>(x, a, dx, dy, dz, r2, r2 < x.rc2 && !nr[u], false);
            }
            note_group<4>(nr, ne, ke0, ke1, k);
        };
        // two chunks per trip in alternating registers: the next chunk's
        // load is in flight while the current one is evaluated (the empty
        // asm with a memory clobber keeps the compiler from folding the
        // prefetched load and the first one into a single load at the top)
        uint4 ca = in.c0, cb;
        for (int k0 = 0; k0 < nvap; k0 += 16) {
            cb = lst4[(size_t)min((k0 >> 3) + 1, lastchunk) * vt];
            asm volatile("" ::: "memory");
            vapour_group(ca.x, ca.y, k0);
            if (k0 + 4 >= nvap) break;
            vapour_group(ca.z, ca.w, k0 + 4);
            if (k0 + 8 >= nvap) break;
            ca = lst4[(size_t)min((k0 >> 3) + 2, lastchunk) * vt];
            asm volatile("" ::: "memory");
            vapour_group(cb.x, cb.y, k0 + 8);
            if (k0 + 12 >= nvap) break;
            vapour_group(cb.z, cb.w, k0 + 12);
        }
        if (nwal > 0) {
            // wall chunks c0 .. c0 + ncw - 1 (c0: the first chunk after the
            // vapour part); a group's chunks past the last one take the
            // group's first entry under the pad code
            constexpr int G = kGroupW<T> / 4;
            const int c0 = (nvap + 7) >> 3, ncw = (nwal + 3) >> 2;
            const V* Lw = x.Lc + vt;
            uint4 cw[G];
#pragma unroll
            for (int q = 0; q < G; ++q) cw[q] = lst4[(size_t)min(c0 + q, lastchunk) * vt];
            for (int c = 0; c < ncw; c += G) {
                unsigned e[kGroupW<T>];
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    const bool live = q == 0 || c + q < ncw;
                    e[4 * q] = live ? cw[q].x : (cw[0].x | kPadCode);
                    e[4 * q + 1] = live ? cw[q].y : (cw[0].x | kPadCode);
                    e[4 * q + 2] = live ? cw[q].z : (cw[0].x | kPadCode);
                    e[4 * q + 3] = live ? cw[q].w : (cw[0].x | kPadCode);
                }
                V ow[kGroupW<T>];
#pragma unroll
                for (int u = 0; u < kGroupW<T>; ++u) ow[u] = Lw[e[u] & kIndexMask];
#pragma unroll
                for (int q = 0; q < G; ++q) cw[q] = lst4[(size_t)min(c0 + c + G + q, lastchunk) * vt];
                bool nr[kGroupW<T>];
#pragma unroll
                for (int u = 0; u < kGroupW<T>; ++u) {
                    const V sw = lut[e[u] >> kIndexBits];
                    const T dx = me.x - ow[u].x + sw.x;
                    const T dy = me.y - ow[u].y + sw.y;
                    const T dz = me.z - ow[u].z + sw.z;
                    const T r2 = dx * dx + dy * dy + dz * dz;
                    nr[u] = sizeof(T) == 4 && fabs(r2 - x.rc2) < x.band;
                    pair_masked<T, VIR, DOE>(x, a, dx, dy, dz, r2, r2 < x.rc2 && !nr[u], true);
                }
                note_group<kGroupW<T>>(nr, ne, ke0, ke1, nvap + 4 * c);
            }
        }
        if (ne)
            edge_pass<T, VIR>(P, sp, x, tl, lut, i, nvap, nwal, (int)(posb - tl.pos), ne, ke0, ke1, a);
        const double kei = atom_epilogue<T>(P, x, i, a, flags);
        ke += kei;
        if constexpr (VIR && DOE) {
            lwv += a.wv;
            if (in_pore(sp, x.X[i], x.X[vt + i], x.X[2 * vt + i])) {
                lkp += kei;
                lwp += a.wv;
                lnp += 1.0;
            }
        }
    }
}

template <typename T, bool VIR>
__device__ __forceinline__ void step_body(PoolDev& P, int kk)
{
    using V = typename V4<T>::type;
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ int lds_scan[17];
    __shared__ Red red;  // the energy reductions at the start and the end

    BrickCtx c;
    if (!brick_ctx(P, c, ST_OVERFLOW | ST_NONFINITE)) return;
    const int s = c.s;
    const SysParams& sp = P.sp[s];
    const SysState st = P.st[s];
    // step kk of the replay runs unless the run ends earlier or an earlier
    // step of the replay raised a stop (displacement beyond skin/2, non-finite)
    if (kk >= st.remaining || kk > st.stop) return;
    const int tid = threadIdx.x;
    const StepCtx<T> x = step_ctx<T>(P, sp, st, kk);
    // the system's first brick records the previous step's energies
    if (c.b == 0 && kk > 0) {
        const long long kprev = st.step + kk;
        if (step_records(sp, false, false, kprev)) record_energies(P, sp, s, (kk - 1) & 1, kprev, red);
    }
    const HaloGeo g = halo_geo(sp, c.b);
    Tile<T> tl = tile_of<T>(smem, P);
    // shift of each neighbour-cell code (made visible by the staging's
    // barriers): one LDS read per list entry instead of decoding the code
    __shared__ V lut[32];
    if (tid < 32) lut[tid] = shift_q<T>(tid, x.hx, x.hy, x.hz);
    const int key0 = c.b * sp.bcells;
    const int i0 = P.cstart[sp.coff + key0], i1 = P.cstart[sp.coff + key0 + sp.bcells];
    // the lane's first atom: its loads are in flight during the staging
    AtomIn<T> first{};
    if (i0 + tid < i1) first = atom_in<T>(P, x, i0 + tid);
    const int tot = stage_halo<T>(P, sp, g, tl, x.Lc, true, lds_scan);

    double ke = 0.0;
    // force fields per atom; the energy and virial fields run over all of
    // this lane's atoms (no second set of sums to keep live in the loops),
    // except that the vapour virial is per atom with VIR (its share goes to
    // the pore's sum when the atom lies in the pore)
    Acc a{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double lwv = 0.0, lkp = 0.0, lwp = 0.0, lnp = 0.0;
    int flags = tot < 0 ? (ST_OVERFLOW | ST_TILE) : 0;
    // energies (and virial sums) only on recording steps: a workgroup-uniform
    // choice between two builds of the pair loops
    if (tot >= 0) {
        if (x.doE)
            step_atoms<T, VIR, true>(P, sp, x, g, tl, lut, i0, i1, first, a, ke, lwv, lkp, lwp, lnp, flags);
        else
            step_atoms<T, VIR, false>(P, sp, x, g, tl, lut, i0, i1, first, a, ke, lwv, lkp, lwp, lnp, flags);
    }
    // vapour pairs were met from both atoms: half of each sum (and each
    // pair's virial is shared equally by its two molecules)
    step_reduce(P, sp, s, c.b, kk, x.doE, flags, ke, 0.5 * a.ev, a.ew, 0.5 * (VIR ? lwv : a.wv), a.ww,
                lkp, 0.5 * lwp, lnp, red);
}

// The step kernel (F1 + F3 + the next F2, see step_body); k_step_virial
// also sums r . f on recording steps (a pool with a system that asks for
// the virial), which costs the plain kernel's registers and about 3%.
template <typename T>
__global__ void __launch_bounds__(kMaxBlock) k_step(PoolDev P, int kk)
{
    step_body<T, false>(P, kk);
}

template <typename T>
__global__ void __launch_bounds__(kMaxBlock) k_step_virial(PoolDev P, int kk)
{
    step_body<T, true>(P, kk);
}

// End of a replay, one workgroup per system: count the steps the replay
// did, record the last one's energies if due, and advance the state.
__global__ void __launch_bounds__(256) k_commit(PoolDev P, int nslots, int R)
{
    const int s = blockIdx.x;
    if (s >= nslots) return;
    const SysParams& sp = P.sp[s];
    const SysState st = P.st[s];
    if (!sp.active || st.remaining <= 0 || (st.status & (ST_OVERFLOW | ST_NONFINITE))) {
        if (threadIdx.x == 0 && sp.active) {
            // a failed rebuild stalls the system: the replays queued behind
            // this one skip their rebuilds and steps until the host has
            // grown the buffer
            const int f = st.status | st.status_next;
            P.st[s].status = f | ((f & ST_OVERFLOW) ? ST_STALL : 0);
            P.st[s].status_next = 0;
            P.st[s].stop = 0x7fffffff;
        }
        return;
    }
    const bool init = st.phase == PH_INIT;
    const int done = min(min(R, st.remaining), st.stop == 0x7fffffff ? R : st.stop + 1);
    const int kl = done - 1;  // last step of the replay
    const bool last = !init && kl == st.remaining - 1;
    const long long kstep = init ? st.step : st.step + kl + 1;
    __shared__ Red red;
    if (step_records(sp, init, last, kstep)) record_energies(P, sp, s, kl & 1, kstep, red);
    if (threadIdx.x != 0) return;
    SysState* sw = P.st + s;
    sw->status = st.status | st.status_next;
    sw->status_next = 0;
    sw->stop = 0x7fffffff;
    if (init) {
        sw->phase = PH_REST;
        sw->remaining = 0;
        return;
    }
    sw->step = st.step + done;
    sw->remaining = st.remaining - done;
    sw->steps_since = st.steps_since + done;
    // every step but the run's last one moved the positions into the other
    // local-coordinate buffer
    sw->lbuf = st.lbuf ^ ((done - (last ? 1 : 0)) & 1);
    // every step wrote its positions and velocities into the other buffer
    sw->sbuf = st.sbuf ^ (done & 1);
    if (last) sw->phase = PH_REST;
}

// ---------------------------------------------------------------------------
// Berendsen thermostat (F4): after step kk's forces and second half-kick,
// lambda from the step's temperature, then v <- lambda v and, unless the run
// ends, the next step's first half-kick and drift.
// ---------------------------------------------------------------------------

// One workgroup per system: the temperature of step kk from its kinetic
// energy partials (summed in brick order), and the factor
// lambda = sqrt(1 + (dt / tau) (t0 / T - 1)).
__global__ void __launch_bounds__(256) k_lambda(PoolDev P, int kk)
{
    __shared__ double red[kMaxBlock / 64];
    const int s = blockIdx.x;
    if (s >= P.nslots) return;
    const SysParams& sp = P.sp[s];
    const SysState st = P.st[s];
    if (!sp.active || !sp.thermo || st.phase == PH_INIT || kk >= st.remaining || kk > st.stop ||
        (st.status & (ST_OVERFLOW | ST_NONFINITE | ST_STALL)))
        return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    const double* pp = P.partial + kPartial * ((size_t)(kk & 1) * P.nbt + sp.pboff);
    double ke = 0.0;
    for (int q = tid; q < sp.nbrick; q += blockDim.x) ke += pp[kPartial * q];
    ke = wave_sum(ke);
    if (lane == 0) red[wave] = ke;
    __syncthreads();
    if (tid != 0) return;
    ke = 0.0;
    for (int w = 0; w < nwave; ++w) ke += red[w];
    const double T = 2.0 * ke / sp.dof;
    const double l2 = 1.0 + (sp.dt / sp.tau_t) * (sp.t0 / T - 1.0);
    P.st[s].lambda = sqrt(l2 > 0.0 ? l2 : 0.0);
}

// Per atom: v <- lambda v on the full-step velocities that k_step stored,
// then (unless this is the run's last step) v += a dt/2, x += v dt, wrap, new
// local coordinates and displacement test, exactly as the fused step epilogue
// does without the thermostat.
template <typename T>
__global__ void k_thermo(PoolDev P, int kk)
{
    using V = typename V4<T>::type;
    SlotCtx c;
    if (!rebuild_ctx(P, c)) return;
    const SysParams& sp = P.sp[c.s];
    const SysState st = P.st[c.s];
    if (!sp.thermo || st.phase == PH_INIT || kk >= st.remaining || kk > st.stop ||
        (st.status & ST_OVERFLOW) || c.li >= sp.nv)
        return;
    const int vt = P.vt, i = c.i;
    const int xb = st.sbuf ^ (kk & 1) ^ 1;  // the buffer k_step wrote this step
    double* X = P.X[xb];
    double* Vv = P.V[xb];
    const double lam = st.lambda;
    double vx = lam * Vv[i], vy = lam * Vv[vt + i], vz = lam * Vv[2 * vt + i];
    if (kk == st.remaining - 1) {
        Vv[i] = vx;
        Vv[vt + i] = vy;
        Vv[2 * vt + i] = vz;
        return;
    }
    const double hdt = 0.5 * sp.dt;
    vx += hdt * P.A[i];
    vy += hdt * P.A[vt + i];
    vz += hdt * P.A[2 * vt + i];
    const double xx = wrap_box(X[i] + vx * sp.dt, sp.L[0]);
    const double yy = wrap_box(X[vt + i] + vy * sp.dt, sp.L[1]);
    const double zz = wrap_box(X[2 * vt + i] + vz * sp.dt, sp.L[2]);
    Vv[i] = vx;
    Vv[vt + i] = vy;
    Vv[2 * vt + i] = vz;
    X[i] = xx;
    X[vt + i] = yy;
    X[2 * vt + i] = zz;
    const int cr = P.cref[i];
    const int cx = cr & 1023, cy = (cr >> 10) & 1023, cz = cr >> 20;
    V* Ln = (V*)P.L[st.lbuf ^ (kk & 1) ^ 1];
    const double lx = local_axis(xx, cx, sp.h[0], sp.L[0], sp.invL[0]);
    const double ly = local_axis(yy, cy, sp.h[1], sp.L[1], sp.invL[1]);
    const double lz = local_axis(zz, cz, sp.h[2], sp.L[2], sp.invL[2]);
    Ln[i] = make4<T>(lx, ly, lz);
    const f4 r = P.lref[i];
    const float ex = (float)lx - r.x, ey = (float)ly - r.y, ez = (float)lz - r.z;
    int f = ex * ex + ey * ey + ez * ez > sp.half_skin * sp.half_skin ? ST_HALT : 0;
    if (!isfinite(xx + yy + zz + vx + vy + vz)) f |= ST_NONFINITE;
    if (f) {
        // rare: an early rebuild (or a failure) after this step
        atomicOr(&P.st[c.s].status_next, f);
        atomicMin(&P.st[c.s].stop, kk);
    }
}

hipError_t launch_step(const PoolDev& P, int kk, int precision, hipStream_t s, hipEvent_t ev0,
                       hipEvent_t ev1)
{
    const int G = ((P.nbrick + 7) / 8) * 8;
    const int B = P.block;
    if (G == 0) return hipSuccess;
    const size_t lds = tile_bytes(P, precision);
    auto kf = P.virial ? k_step_virial<float> : k_step<float>;
    auto kd = P.virial ? k_step_virial<double> : k_step<double>;
    if (ev0 && ev1) {
        if (precision == 1)
            hipExtLaunchKernelGGL(kf, dim3(G), dim3(B), lds, s, ev0, ev1, 0, P, kk);
        else
            hipExtLaunchKernelGGL(kd, dim3(G), dim3(B), lds, s, ev0, ev1, 0, P, kk);
    } else {
        if (precision == 1)
            hipLaunchKernelGGL(kf, dim3(G), dim3(B), lds, s, P, kk);
        else
            hipLaunchKernelGGL(kd, dim3(G), dim3(B), lds, s, P, kk);
    }
    if (P.thermo) {
        hipLaunchKernelGGL(k_lambda, dim3(P.nslots), dim3(256), 0, s, P, kk);
        const int GT = ((P.nchunk / (kRebuildBlock / kChunk) + 7) / 8) * 8;
        if (precision == 1)
            hipLaunchKernelGGL(k_thermo<float>, dim3(GT), dim3(kRebuildBlock), 0, s, P, kk);
        else
            hipLaunchKernelGGL(k_thermo<double>, dim3(GT), dim3(kRebuildBlock), 0, s, P, kk);
    }
    return hipGetLastError();
}

hipError_t launch_commit(const PoolDev& P, int nslots, int R, hipStream_t s)
{
    hipLaunchKernelGGL(k_commit, dim3(nslots), dim3(256), 0, s, P, nslots, R);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host-requested state changes and readbacks
// ---------------------------------------------------------------------------

__global__ void k_set_run(PoolDev P, int slot, int add_steps, int clear_bits)
{
    P.st[slot].remaining += add_steps;
    P.st[slot].status &= ~clear_bits;
}

hipError_t launch_set_run(const PoolDev& P, int slot, int add_steps, int clear_bits, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_run, dim3(1), dim3(1), 0, s, P, slot, add_steps, clear_bits);
    return hipGetLastError();
}

// Start over from freshly loaded positions and velocities at step `step`:
// the next run is the initial force evaluation, the energy history restarts.
__global__ void k_reset_state(PoolDev P, int slot, long long step)
{
    SysState* st = P.st + slot;
    st->remaining = 1;
    st->phase = PH_INIT;
    st->status = 0;
    st->status_next = 0;
    st->nrec = 0;
    st->max_nbr = 0;
    st->steps_since = 0;
    st->stop = 0x7fffffff;
    st->step = step;
}

hipError_t launch_reset_state(const PoolDev& P, int slot, long long step, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(1), 0, s, P, slot, step);
    return hipGetLastError();
}

// which: 0 positions, 1 velocities, 2 forces (m a)
__global__ void k_unpermute(PoolDev P, int slot, int which, double* out, int n)
{
    const SysParams& sp = P.sp[slot];
    const SysState& st = P.st[slot];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.nv || p >= n) return;
    const int i = sp.voff + p;
    const int vt = P.vt;
    const int id = P.id[st.ibuf][i];
    if (id < 0 || id >= n) return;
    const double* src = which == 0 ? P.X[st.sbuf] : which == 1 ? P.V[st.sbuf] : P.A;
    const double m = which == 2 ? sp.mass : 1.0;
    out[3 * (size_t)id] = m * src[i];
    out[3 * (size_t)id + 1] = m * src[vt + i];
    out[3 * (size_t)id + 2] = m * src[2 * vt + i];
}

hipError_t launch_unpermute(const PoolDev& P, int slot, int which, double* out, int n,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpermute, dim3((n + 255) / 256), dim3(256), 0, s, P, slot, which, out, n);
    return hipGetLastError();
}

__global__ void k_wall_unpermute(PoolDev P, int slot, double* out, int n)
{
    const SysParams& sp = P.sp[slot];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.nw || p >= n) return;
    const int w = sp.woff + p;
    const int id = P.wid[w];
    if (id < 0 || id >= n) return;
    out[3 * (size_t)id] = P.WX[w];
    out[3 * (size_t)id + 1] = P.WX[P.wt + w];
    out[3 * (size_t)id + 2] = P.WX[2 * P.wt + w];
}

hipError_t launch_wall_unpermute(const PoolDev& P, int slot, double* out, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wall_unpermute, dim3((n + 255) / 256), dim3(256), 0, s, P, slot, out, n);
    return hipGetLastError();
}

// Pairs within the cutoff found through the lists, tested in FP64 on the
// master positions: out holds (kind, a, b) triples; counts[0] = total.
template <typename T>
__global__ void k_debug_pairs(PoolDev P, int slot, int* out, int cap, int* counts)
{
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ int lds_scan[17];
    const SysParams& sp = P.sp[slot];
    const SysState& st = P.st[slot];
    const int b = blockIdx.x;
    if (b >= sp.nbrick) return;
    const HaloGeo g = halo_geo(sp, b);
    Tile<T> t = tile_of<T>(smem, P);
    const typename V4<T>::type* Lc = (const typename V4<T>::type*)P.L[st.lbuf];
    const int tot = stage_halo<T>(P, sp, g, t, Lc, false, lds_scan);
    if (tot < 0) return;
    const int vt = P.vt;
    const double* X = P.X[st.sbuf];
    const int* ids = P.id[st.ibuf];
    const int key0 = b * sp.bcells;
    const int i0 = P.cstart[sp.coff + key0], i1 = P.cstart[sp.coff + key0 + sp.bcells];
    for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) {
        const int nl = P.nlist[i];
        const int nvap = nl & 0xFFFF, nvw = ((nvap + 7) >> 3) << 2, n = nvap + (nl >> 16);
        const double xi = X[i], yi = X[vt + i], zi = X[2 * vt + i];
        const int cr = P.cref[i];
        const int base = t.hoff[halo_cell(g, cr & 1023, (cr >> 10) & 1023, cr >> 20, 0)];
        for (int k = 0; k < n; ++k) {
            const int a = k >= nvap
                ? (int)(P.list[list_at(vt, i, nvw + k - nvap)] & kIndexMask)
                : base + (int)(((const unsigned short*)P.list)[vlist_at(vt, i, k)] & kRelMask);
            double ox, oy, oz;
            int kind, bb;
            if (k >= nvap) {
                ox = P.WX[a];
                oy = P.WX[P.wt + a];
                oz = P.WX[2 * P.wt + a];
                kind = 1;
                bb = P.wid[a];
            } else {
                const int j = t.slot[a];
                ox = X[j];
                oy = X[vt + j];
                oz = X[2 * vt + j];
                kind = 0;
                bb = ids[j];
                if (!(ids[i] < bb)) continue;
            }
            double ex = xi - ox, ey = yi - oy, ez = zi - oz;
            ex -= sp.L[0] * rint(ex * sp.invL[0]);
            ey -= sp.L[1] * rint(ey * sp.invL[1]);
            ez -= sp.L[2] * rint(ez * sp.invL[2]);
            if (ex * ex + ey * ey + ez * ez < sp.rc2) {
                const int q = atomicAdd(counts, 1);
                if (q < cap) {
                    out[3 * q] = kind;
                    out[3 * q + 1] = ids[i];
                    out[3 * q + 2] = bb;
                }
            }
        }
    }
}

hipError_t launch_debug_pairs(const PoolDev& P, int slot, int precision, int* out, int cap,
                              int* counts, hipStream_t s)
{
    SysParams sp;
    hipError_t e = hipMemcpy(&sp, P.sp + slot, sizeof(SysParams), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    if (sp.nbrick <= 0) return hipSuccess;
    const size_t lds = tile_bytes(P, precision);
    if (precision == 1)
        hipLaunchKernelGGL(k_debug_pairs<float>, dim3(sp.nbrick), dim3(P.block), lds, s, P, slot, out,
                           cap, counts);
    else
        hipLaunchKernelGGL(k_debug_pairs<double>, dim3(sp.nbrick), dim3(P.block), lds, s, P, slot,
                           out, cap, counts);
    return hipGetLastError();
}

// Caller-order AoS positions/velocities -> the system's SoA slots (unsorted;
// id = caller index); padding slots get ids nv .. vcap-1 and zero state.
__global__ void k_copy_in(PoolDev P, int slot, const double* pos, const double* vel, int n)
{
    const SysParams& sp = P.sp[slot];
    const SysState& st = P.st[slot];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= sp.vcap) return;
    const int i = sp.voff + p;
    const int vt = P.vt;
    double* X = P.X[st.sbuf];
    double* Vv = P.V[st.sbuf];
    if (p < n) {
        X[i] = pos[3 * (size_t)p];
        X[vt + i] = pos[3 * (size_t)p + 1];
        X[2 * vt + i] = pos[3 * (size_t)p + 2];
        Vv[i] = vel[3 * (size_t)p];
        Vv[vt + i] = vel[3 * (size_t)p + 1];
        Vv[2 * vt + i] = vel[3 * (size_t)p + 2];
    } else {
        X[i] = X[vt + i] = X[2 * vt + i] = 0.0;
        Vv[i] = Vv[vt + i] = Vv[2 * vt + i] = 0.0;
    }
    P.A[i] = P.A[vt + i] = P.A[2 * vt + i] = 0.0;
    P.id[st.ibuf][i] = p;
    P.lref[i] = make4<float>(0.0, 0.0, 0.0);
}

hipError_t launch_copy_in(const PoolDev& P, int slot, const double* pos, const double* vel, int n,
                          int vcap, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_in, dim3((vcap + 255) / 256), dim3(256), 0, s, P, slot, pos, vel, n);
    return hipGetLastError();
}

}  // namespace pmd
