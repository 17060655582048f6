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

// One workgroup = one wave per atom: lane l takes the partners j = l, l + 64,
// ... in order, read straight from memory (the positions of the paper's
// sizes, a few hundred KB, stay in L2), so the chip gets N waves and no
// barrier.  The 64 partial sums of the atom are combined in a fixed tree of
// shuffles, so results do not depend on timing.
constexpr int kApLanes = 64;

// 1 / r^2, the one reciprocal a pair needs: in FP32 the hardware estimate
// refined by one Newton-Raphson step for the reciprocal (y <- y + y (1 - a y),
// which roughly doubles the correct bits of the estimate), in FP64 one
// division.
template <typename T>
__device__ __forceinline__ T ap_recip(T a);
template <>
__device__ __forceinline__ float ap_recip<float>(float a)
{
    const float y = __builtin_amdgcn_rcpf(a);
    return fmaf(y, fmaf(-a, y, 1.0f), y);
}
template <>
__device__ __forceinline__ double ap_recip<double>(double a)
{
    return 1.0 / a;
}

template <typename T>
__global__ void __launch_bounds__(kApLanes) k_allpairs(const double* __restrict__ x, AllPairsArgs a,
                                                      double* __restrict__ f, double* __restrict__ u)
{
    const int lane = threadIdx.x;
    const int i = blockIdx.x;  // the grid has exactly n workgroups
    const double xi = x[3 * (size_t)i], yi = x[3 * (size_t)i + 1], zi = x[3 * (size_t)i + 2];
    double fx = 0.0, fy = 0.0, fz = 0.0, us = 0.0;
    const T sig2 = (T)a.sig2, eps4 = (T)a.eps4, eps24 = (T)a.eps24;
#pragma unroll 2
    for (int j = lane; j < a.n; j += kApLanes) {
        double dx = xi - x[3 * (size_t)j], dy = yi - x[3 * (size_t)j + 1], dz = zi - x[3 * (size_t)j + 2];
        if (a.L[0] > 0.0) dx -= a.L[0] * rint(dx * a.iL[0]);
        if (a.L[1] > 0.0) dy -= a.L[1] * rint(dy * a.iL[1]);
        if (a.L[2] > 0.0) dz -= a.L[2] * rint(dz * a.iL[2]);
        if (j != i) {
            const T r2 = (T)(dx * dx + dy * dy + dz * dz);
            const T ir2 = ap_recip<T>(r2);
            const T s2 = sig2 * ir2;
            const T s6 = s2 * s2 * s2;
            const T w = eps24 * s6 * ((T)2 * s6 - (T)1) * ir2;
            fx += (double)(w * (T)dx);
            fy += (double)(w * (T)dy);
            fz += (double)(w * (T)dz);
            us += (double)(eps4 * s6 * (s6 - (T)1));
        }
    }
#pragma unroll
    for (int o = kApLanes / 2; o >= 1; o /= 2) {
        fx += __shfl_down(fx, o);
        fy += __shfl_down(fy, o);
        fz += __shfl_down(fz, o);
        us += __shfl_down(us, o);
    }
    if (lane == 0) {
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
        if (precision == 1)
            hipLaunchKernelGGL(k_allpairs<float>, dim3(n), dim3(kApLanes), 0, s, x, a, f, u);
        else
            hipLaunchKernelGGL(k_allpairs<double>, dim3(n), dim3(kApLanes), 0, s, x, a, f, u);
    }
    hipLaunchKernelGGL(k_allpairs_sum, dim3(1), dim3(256), 0, s, u, n, e);
    return hipGetLastError();
}


}  // namespace pmd
