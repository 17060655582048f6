// The paper's own pore model (Secs. 4-5) on the GPU: N molecules in two or
// three dimensions, every pair interacting through the Lennard-Jones
// potential with no cutoff, a pore whose walls reflect molecules specularly
// and whose open face leads into a periodic outer space; velocity Verlet in
// the order of the paper's GPU functions (F2 drift and half-kick, F1 forces,
// F3 half-kick) and the Berendsen F4.
//
// One step is two launches:
//   k_pm_forces  one wave per molecule, its partners split over the 64 lanes
//                and read straight from memory (a few hundred KB at the
//                paper's sizes, L2-resident), the lane sums combined by a
//                fixed tree of shuffles; lane 0 forms the acceleration, the
//                F3 half-kick, the kinetic energy, the energy share and
//                whether the molecule is in the pore;
//   k_pm_update  one workgroup per 256 molecules: each sums the step's
//                energies and the pore's sums in the same fixed order (so
//                all find the same Berendsen factor), workgroup 0 writes the
//                record, and each does F4 and the next step's F2 with the
//                boundary trace for its molecules.
// (One workgroup doing the per-molecule work for all molecules took 14-25 us
// a step; a third launch for it cost more in launch rate than it saved.)
// This file shares nothing with the cell-list path or the all-pairs entry.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pmd_paper.h"

namespace pmd {

// Working memory of the allocation-free entry point: one array per GPU,
// held until the process ends.  Host code never uses this name as an
// address (on the host it is only a stand-in); it uses the device address
// that pm_scratch_ptr obtains for the current device.
static __device__ __align__(256) double scratch[kPmScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t pm_scratch_ptr(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

constexpr int kPmLanes = 64;

// 1 / r^2: in FP32 the hardware estimate refined by one Newton-Raphson step
// for the reciprocal (y + y (1 - a y)), in FP64 one division.
template <typename T>
__device__ __forceinline__ T pm_recip(T a);
template <>
__device__ __forceinline__ float pm_recip<float>(float a)
{
    const float y = __builtin_amdgcn_rcpf(a);
    return fmaf(y, fmaf(-a, y, 1.0f), y);
}
template <>
__device__ __forceinline__ double pm_recip<double>(double a)
{
    return 1.0 / a;
}

// Whether a position lies in the model's domain (pore or outer space).
template <int D>
__device__ bool pm_inside(const PmArgs& a, const double* p)
{
    const double Lw[3] = {a.lx, a.ly, a.lz};
    bool in;
    if (p[0] >= 0.0 && p[0] < a.lx) {
        in = true;
#pragma unroll
        for (int k = 1; k < D; ++k) in = in && p[k] >= 0.0 && p[k] <= Lw[k];
    } else {
        in = p[0] >= a.lx && p[0] < (a.k + 1.0) * a.lx;
#pragma unroll
        for (int k = 1; k < D; ++k) in = in && p[k] >= -a.k * Lw[k] && p[k] < (a.k + 1.0) * Lw[k];
    }
    return in;
}

// Forces (F1) at the current positions, then with KICK the F3 half-kick;
// writes each molecule's acceleration, kinetic energy and half shares of the
// pair energies and of the pair virials r_ij . f_ij.
template <typename T, int D, bool KICK>
__global__ void __launch_bounds__(kPmLanes) k_pm_forces(const double* __restrict__ x,
                                                       double* __restrict__ v, PmWork w, PmArgs a)
{
    const int lane = threadIdx.x;
    const int i = blockIdx.x;  // the grid has exactly n workgroups
    double xi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xi[k] = x[(size_t)D * i + k];
    double f[D], us = 0.0, ws = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) f[k] = 0.0;
    const T sig2 = (T)a.sig2, eps4 = (T)a.eps4, eps24 = (T)a.eps24;
#pragma unroll 2
    for (int j = lane; j < a.n; j += kPmLanes) {
        double d[D];
        double r2d = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            d[k] = xi[k] - x[(size_t)D * j + k];
            r2d += d[k] * d[k];
        }
        if (j != i) {
            const T ir2 = pm_recip<T>((T)r2d);
            const T s2 = sig2 * ir2;
            const T s6 = s2 * s2 * s2;
            const T wf = eps24 * s6 * ((T)2 * s6 - (T)1) * ir2;
#pragma unroll
            for (int k = 0; k < D; ++k) f[k] += (double)(wf * (T)d[k]);
            us += (double)(eps4 * s6 * (s6 - (T)1));
            ws += (double)(wf * (T)r2d);  // r_ij . f_ij of the pair
        }
    }
#pragma unroll
    for (int o = kPmLanes / 2; o >= 1; o /= 2) {
#pragma unroll
        for (int k = 0; k < D; ++k) f[k] += __shfl_down(f[k], o);
        us += __shfl_down(us, o);
        ws += __shfl_down(ws, o);
    }
    if (lane == 0) {
        double ke = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double ak = f[k] * a.inv_mass;
            w.acc[(size_t)D * i + k] = ak;
            double vk = v[(size_t)D * i + k];
            if (KICK) {
                vk += a.hdt * ak;
                v[(size_t)D * i + k] = vk;
            }
            ke += vk * vk;
        }
        w.ke[i] = 0.5 * a.mass * ke;
        w.u[i] = 0.5 * us;
        w.vir[i] = 0.5 * ws;
        w.where[i] = (xi[0] < a.lx ? 1.0 : 0.0) + (pm_inside<D>(a, xi) ? 0.0 : 2.0);
    }
}

// The drift of one step, p -> p + dl, carried through the model's
// boundaries event by event (each event the first plane the rest of the
// segment meets): in the pore, the walls x = 0, y = 0, y = ly (z = 0, z = lz)
// reflect (the normal components of the rest of dl and of v flip) and the
// mouth x = lx lets the molecule out; in the outer space, leaving through
// x = (k+1) lx brings it back at x = lx, crossing x = lx leftwards takes it
// into the pore inside the mouth and back to x = (k+1) lx elsewhere, and the
// transverse faces are periodic.  A segment that ends exactly on a plane
// makes an event only on the outer space's excluded upper faces.  Ties go to
// the lowest axis.  Returns the reflections, or -1 if the events do not end.
template <int D>
__device__ int pm_trace(const PmArgs& a, double* p, double* dl, double* v)
{
    const double Lw[3] = {a.lx, a.ly, a.lz};
    bool pore = p[0] < a.lx;
    int refl = 0;
    for (int it = 0; it < 64; ++it) {
        double tb = 2.0, plane = 0.0;
        int ax = -1, kind = 0;  // 1 reflect, 2 out of the mouth, 3 wrap x, 4 x = lx leftwards, 5 wrap y/z
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (dl[k] == 0.0) continue;
            double wpl;
            int kd;
            if (pore) {
                if (k == 0) {
                    wpl = dl[0] < 0.0 ? 0.0 : a.lx;
                    kd = dl[0] < 0.0 ? 1 : 2;
                } else {
                    wpl = dl[k] < 0.0 ? 0.0 : Lw[k];
                    kd = 1;
                }
            } else {
                if (k == 0) {
                    wpl = dl[0] > 0.0 ? (a.k + 1.0) * a.lx : a.lx;
                    kd = dl[0] > 0.0 ? 3 : 4;
                } else {
                    wpl = dl[k] < 0.0 ? -a.k * Lw[k] : (a.k + 1.0) * Lw[k];
                    kd = 5;
                }
            }
            const bool excl = !pore && dl[k] > 0.0;
            const double t = (wpl - p[k]) / dl[k];
            if ((t < 1.0 || (excl && t <= 1.0)) && t < tb) {
                tb = t < 0.0 ? 0.0 : t;
                ax = k;
                kind = kd;
                plane = wpl;
            }
        }
        if (ax < 0) {
#pragma unroll
            for (int k = 0; k < D; ++k) p[k] += dl[k];
            return refl;
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            p[k] = k == ax ? plane : p[k] + tb * dl[k];
            dl[k] *= 1.0 - tb;
        }
        if (kind == 1) {
            dl[ax] = -dl[ax];
            v[ax] = -v[ax];
            ++refl;
        } else if (kind == 2) {
            pore = false;
        } else if (kind == 3) {
            p[0] = a.lx;
        } else if (kind == 4) {
            bool mouth = p[1] >= 0.0 && p[1] < a.ly;
            if (D == 3) mouth = mouth && p[D - 1] >= 0.0 && p[D - 1] < a.lz;
            if (mouth)
                pore = true;
            else
                p[0] = (a.k + 1.0) * a.lx;
        } else {
            p[ax] = dl[ax] < 0.0 ? (a.k + 1.0) * Lw[ax] : -a.k * Lw[ax];
        }
    }
    return -1;
}

// Fixed-order workgroup sums of K values at once: each wave combines its
// lanes by a fixed tree of shuffles, then the waves' sums are added in wave
// order; every thread receives the K totals.
template <int K, int B = kPmDrift>
__device__ void pm_block_sums(double (&v)[K], double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kWaves = B / 64;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] += __shfl_down(v[q], o);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) red[q * kWaves + wave] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += red[q * kWaves + w];
        v[q] = t;
    }
    __syncthreads();
}

// End of step `step` (0 = the initial state), one workgroup per 256
// molecules.  Every workgroup sums, in the same fixed order, the step's
// energies (kinetic energy of the F3 velocities, pair energy at the current
// positions), the pore's K and W (Sec. 2: P = (2 K + W) / (d V) over the
// molecules in the pore, V the pore's volume, W their shares of the pair
// virials) and the previous step's drift counts, so each finds the same
// Berendsen factor without another launch; workgroup 0 writes the record
// and the run's counters.  Then each workgroup does, for its molecules, F4
// (v <- lambda v, steps >= 1 with a thermostat) and, with drift, the next
// step's F2: dl = v dt + a dt^2 / 2, v <- v + a dt / 2, the molecule carried
// along dl through the boundaries; its counts of reflections and failed
// traces go to the slot of this step's parity.  nprev: workgroups of the
// previous launch (0 at step 0).
template <int D>
__global__ void __launch_bounds__(kPmDrift) k_pm_update(double* __restrict__ x, double* __restrict__ v, PmWork w,
                                                       PmArgs a, long long step, int rec_row, int thermo,
                                                       int drift, int nprev, PmRecord* __restrict__ rec)
{
    __shared__ double red[8 * (kPmDrift / 64)];
    const int tid = threadIdx.x, nb = (int)gridDim.x;
    double ke = 0.0, pe = 0.0, np = 0.0, out = 0.0, kp = 0.0, wp = 0.0;
    for (int i = tid; i < a.n; i += kPmDrift) {
        const double kei = w.ke[i], wh = w.where[i];
        ke += kei;
        pe += w.u[i];
        const bool pore = wh == 1.0 || wh == 3.0;
        np += pore ? 1.0 : 0.0;
        kp += pore ? kei : 0.0;
        wp += pore ? w.vir[i] : 0.0;
        out += wh >= 2.0 ? 1.0 : 0.0;
    }
    double refl = 0.0, bad = 0.0;
    const double* prev = w.part + 2 * (size_t)nprev * ((step + 1) & 1);
    for (int b = tid; b < nprev; b += kPmDrift) {
        refl += prev[b];
        bad += prev[nprev + b];
    }
    double sums[8] = {ke, pe, np, out, kp, wp, refl, bad};
    pm_block_sums<8>(sums, red);
    const double T = a.n > 0 ? 2.0 * sums[0] / ((double)D * (double)a.n) : 0.0;
    if (blockIdx.x == 0 && tid == 0) {
        // the counts start with the run (no memset node: callers may capture)
        const long long r0 = step == 0 ? 0LL : w.counts[0] + (long long)sums[6];
        const long long r1 = step == 0 ? 0LL : w.counts[1] + (long long)sums[7];
        w.counts[0] = r0;
        w.counts[1] = r1;
        if (rec_row >= 0) {
            PmRecord r;
            r.step = step;
            r.ke = sums[0];
            r.pe = sums[1];
            r.etotal = sums[0] + sums[1];
            r.temperature = T;
            r.pressure = (2.0 * sums[4] + sums[5]) / ((double)D * a.vol);
            r.n_pore = (long long)sums[2];
            r.reflections = r0;
            r.n_outside = (long long)sums[3] + r1;
            rec[rec_row] = r;
        }
    }
    if (!thermo && !drift) return;
    const double lam = thermo && a.n > 0 ? sqrt(1.0 + (a.dt / a.tau) * (a.t0 / T - 1.0)) : 1.0;
    const int i = blockIdx.x * kPmDrift + tid;
    double cnt[2] = {0.0, 0.0};
    if (i < a.n) {
        double p[D], vv[D], dl[D];
#pragma unroll
        for (int k = 0; k < D; ++k) vv[k] = lam * v[(size_t)D * i + k];
        if (drift) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double ak = w.acc[(size_t)D * i + k];
                p[k] = x[(size_t)D * i + k];
                dl[k] = vv[k] * a.dt + 0.5 * ak * a.dt * a.dt;
                vv[k] += a.hdt * ak;
            }
            const int r = pm_trace<D>(a, p, dl, vv);
            if (r < 0)
                cnt[1] = 1.0;
            else
                cnt[0] = (double)r;
#pragma unroll
            for (int k = 0; k < D; ++k) x[(size_t)D * i + k] = p[k];
        }
#pragma unroll
        for (int k = 0; k < D; ++k) v[(size_t)D * i + k] = vv[k];
    }
    if (!drift) return;
    pm_block_sums<2>(cnt, red);
    if (tid == 0) {
        double* cur = w.part + 2 * (size_t)nb * (step & 1);
        cur[blockIdx.x] = cnt[0];
        cur[nb + blockIdx.x] = cnt[1];
    }
}

template <int D>
static hipError_t pm_run_dim(const PmArgs& a, double* x, double* v, PmWork w, long long nsteps,
                             long long every, PmRecord* rec, hipStream_t s)
{
    const dim3 gf((unsigned)a.n), bf(kPmLanes);
    const int nb = (int)pm_drift_blocks(a.n);
    const dim3 gu((unsigned)nb), bu(kPmDrift);
    const bool thermo = a.tau > 0.0;
    int row = 0;
    if (a.n > 0) {
        if (a.precision == 1)
            hipLaunchKernelGGL((k_pm_forces<float, D, false>), gf, bf, 0, s, x, v, w, a);
        else
            hipLaunchKernelGGL((k_pm_forces<double, D, false>), gf, bf, 0, s, x, v, w, a);
    }
    hipLaunchKernelGGL(k_pm_update<D>, gu, bu, 0, s, x, v, w, a, 0LL, rec ? row++ : -1, 0,
                       nsteps > 0 ? 1 : 0, 0, rec);
    for (long long st = 1; st <= nsteps; ++st) {
        if (a.n > 0) {
            if (a.precision == 1)
                hipLaunchKernelGGL((k_pm_forces<float, D, true>), gf, bf, 0, s, x, v, w, a);
            else
                hipLaunchKernelGGL((k_pm_forces<double, D, true>), gf, bf, 0, s, x, v, w, a);
        }
        const bool record = rec && (st == nsteps || (every > 0 && st % every == 0));
        hipLaunchKernelGGL(k_pm_update<D>, gu, bu, 0, s, x, v, w, a, st, record ? row++ : -1,
                           thermo ? 1 : 0, st < nsteps ? 1 : 0, nb, rec);
    }
    return hipGetLastError();
}

hipError_t launch_pm_run(const PmArgs& a, double* x, double* v, PmWork w, long long nsteps,
                         long long every, PmRecord* rec, hipStream_t s)
{
    return a.dim == 2 ? pm_run_dim<2>(a, x, v, w, nsteps, every, rec, s)
                      : pm_run_dim<3>(a, x, v, w, nsteps, every, rec, s);
}

}  // namespace pmd
