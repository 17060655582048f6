// All-pairs Lennard-Jones forces: the force function as the paper states it
// (Sec. 3), every pair interacting with no cutoff and no shift, minimum
// image on the periodic axes.  The cell-list path lives in pmd_kernels.hip;
// this file shares nothing with it.
#include <hip/hip_runtime.h>

#include "pmd_allpairs.h"

namespace pmd {

struct AllPairsArgs {
    double L[3], iL[3];  // box edges (0 on open axes) and their inverses
    double sig2, eps4, eps24;
    int n;
};

// One workgroup = one wave = 4 atoms x 16 slices of the partners: lane l
// owns atom 4 b + (l & 3) and the partners k = l >> 2 (mod 16) of each
// 64-atom tile staged in LDS, so the paper's sizes (a few thousand atoms)
// still give the chip thousands of waves.  The sixteen partial sums of an
// atom are combined in a fixed order by four shuffles, so results do not
// depend on timing.
constexpr int kApAtoms = 4, kApParts = 16, kApTile = kApAtoms * kApParts;

template <typename T>
__global__ void __launch_bounds__(kApTile) k_allpairs(const double* __restrict__ x, AllPairsArgs a,
                                                     double* __restrict__ f, double* __restrict__ u)
{
    __shared__ double4 tile[kApTile];
    const int lane = threadIdx.x;
    const int part = lane / kApAtoms;
    const int i = blockIdx.x * kApAtoms + lane % kApAtoms;
    const bool live = i < a.n;
    const int ic = live ? i : a.n - 1;  // the grid only exists for n >= 1
    const double xi = x[3 * (size_t)ic], yi = x[3 * (size_t)ic + 1], zi = x[3 * (size_t)ic + 2];
    double fx = 0.0, fy = 0.0, fz = 0.0, us = 0.0;
    const T sig2 = (T)a.sig2, eps4 = (T)a.eps4, eps24 = (T)a.eps24;
    for (int j0 = 0; j0 < a.n; j0 += kApTile) {
        const int j = j0 + lane;
        if (j < a.n) tile[lane] = make_double4(x[3 * (size_t)j], x[3 * (size_t)j + 1], x[3 * (size_t)j + 2], 0.0);
        __syncthreads();
        const int m = min(kApTile, a.n - j0);
        for (int k = part; k < m; k += kApParts) {
            const double4 o = tile[k];
            double dx = xi - o.x, dy = yi - o.y, dz = zi - o.z;
            if (a.L[0] > 0.0) dx -= a.L[0] * rint(dx * a.iL[0]);
            if (a.L[1] > 0.0) dy -= a.L[1] * rint(dy * a.iL[1]);
            if (a.L[2] > 0.0) dz -= a.L[2] * rint(dz * a.iL[2]);
            if (j0 + k != i) {
                const T r2 = (T)(dx * dx + dy * dy + dz * dz);
                const T s2 = sig2 / r2;
                const T s6 = s2 * s2 * s2;
                const T w = eps24 * s6 * ((T)2 * s6 - (T)1) / r2;
                fx += (double)(w * (T)dx);
                fy += (double)(w * (T)dy);
                fz += (double)(w * (T)dz);
                us += (double)(eps4 * s6 * (s6 - (T)1));
            }
        }
        __syncthreads();
    }
    // the partial sums of lanes l, l + 4, ..., l + 60, halved four times
#pragma unroll
    for (int o = kApTile / 2; o >= kApAtoms; o /= 2) {
        fx += __shfl_down(fx, o);
        fy += __shfl_down(fy, o);
        fz += __shfl_down(fz, o);
        us += __shfl_down(us, o);
    }
    if (part == 0 && live) {
        f[3 * (size_t)i] = fx;
        f[3 * (size_t)i + 1] = fy;
        f[3 * (size_t)i + 2] = fz;
        u[i] = 0.5 * us;
    }
}

// Total energy: one workgroup sums the per-atom shares, each thread over a
// fixed stride, then a fixed tree.
__global__ void __launch_bounds__(256) k_allpairs_sum(const double* __restrict__ u, int n, double* __restrict__ e)
{
    __shared__ double part[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += u[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) e[0] = part[0];
}

hipError_t launch_allpairs(int precision, int n, const double* x, const double box[3], double eps,
                           double sigma, double* f, double* u, double* e, hipStream_t s)
{
    AllPairsArgs a;
    for (int k = 0; k < 3; ++k) {
        a.L[k] = box[k] > 0.0 ? box[k] : 0.0;
        a.iL[k] = box[k] > 0.0 ? 1.0 / box[k] : 0.0;
    }
    a.sig2 = sigma * sigma;
    a.eps4 = 4.0 * eps;
    a.eps24 = 24.0 * eps;
    a.n = n;
    if (n > 0) {
        const int G = (n + kApAtoms - 1) / kApAtoms;
        if (precision == 1)
            hipLaunchKernelGGL(k_allpairs<float>, dim3(G), dim3(kApTile), 0, s, x, a, f, u);
        else
            hipLaunchKernelGGL(k_allpairs<double>, dim3(G), dim3(kApTile), 0, s, x, a, f, u);
    }
    hipLaunchKernelGGL(k_allpairs_sum, dim3(1), dim3(256), 0, s, u, n, e);
    return hipGetLastError();
}


}  // namespace pmd
