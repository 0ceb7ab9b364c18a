// Device helpers shared by the sweep and auxiliary kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>

#include "ep_internal.h"

namespace ep {

__device__ __forceinline__ double nan_to_inf(double v) { return (v <= DBL_MAX) ? v : INFINITY; }

// Max over a wave64 (all lanes get the result).
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide max of non-negative values folded into *dst with one atomicMax
// per block.  All threads of the block must call it.
template <int NT>
__device__ __forceinline__ void block_max_to(double v, unsigned long long* dst, double* sh)
{
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    v = wave_max(nan_to_inf(v));
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    if (tid < 64) {
        double w = tid < NT / 64 ? sh[tid] : 0.0;
        w = wave_max(w);
        if (tid == 0 && w > 0.0) atomicMax(dst, (unsigned long long)__double_as_longlong(w));
    }
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ void block_sum_to(double v, unsigned long long* dst, double* sh)
{
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    v = wave_sum(v);
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    if (tid < 64) {
        double w = tid < NT / 64 ? sh[tid] : 0.0;
        w = wave_sum(w);
        if (tid == 0 && w != 0.0) atomicAdd(dst, (unsigned long long)w);
    }
    __syncthreads();
}

// Return mapping at a centre.  J2 is of the trial sums T; returns Lambda
// (0 when elastic, +inf at the apex) and writes the plastic rate
// D (tauII_tr - Y), the returned tauII and the bound Y.
template <typename R>
__device__ __forceinline__ R centre_lambda(R J2, R D, R p, R c, R A, R B, R& lamdot, R& tii, R& Y)
{
    R tii_tr = sqrt(J2) / D;
    Y = A * p + B * c;
    Y = Y > R(0) ? Y : R(0);
    R lam = R(0);
    lamdot = R(0);
    tii = tii_tr;
    if (tii_tr > Y) {
        lam = D * (tii_tr / Y - R(1));
        lamdot = D * (tii_tr - Y);
        tii = Y;
    }
    return lam;
}

}  // namespace ep
