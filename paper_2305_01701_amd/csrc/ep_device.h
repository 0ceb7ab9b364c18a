// Device helpers shared by the sweep and auxiliary kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>

#include "ep_internal.h"

namespace ep {

// Block index -> logical tile so that consecutive logical tiles run on the
// same XCD (dispatch is round-robin over the 8 XCDs).  Bijective for any nb.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb / 8, r = nb % 8;
    const int x = b % 8, s = b / 8;
    return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

__device__ __forceinline__ double nan_to_inf(double v) { return (v <= DBL_MAX) ? v : INFINITY; }

// Running maximum that keeps a NaN once it has seen one (fmax drops NaN
// arguments, which would hide a diverging state from the residual check).
template <typename T>
__device__ __forceinline__ T nmax(T acc, T x) { return (x > acc || x != x) ? x : acc; }

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
        if (tid == 0 && w > 0.0) {
            // skip the atomic when the running maximum is already larger: a
            // stale read only costs an unnecessary atomic, never a wrong max
            const unsigned long long bits = (unsigned long long)__double_as_longlong(w);
            if (bits > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dst, bits);
        }
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

// Plastic rate of a dilatant or regularised return.  Dilatancy (psi > 0,
// potential sqrt(J2) - C p): the plastic rate lamdot adds lamdot * Cik to the
// pressure of the update.  Consistency regularisation: the returned tauII
// exceeds the bound by vp * lamdot.  With tauII D + lamdot = sqrt(J2) and
// tauII = max(0, A p + B c) + vp lamdot, lamdot is
//     (sqrt(J2) - D (A p + B c)) / (1 + D A Cik + D vp)
// (p before the correction) when the corrected bound is non-negative, else
// the apex root sqrt(J2) / (1 + D vp).  Returns lamdot; p is corrected.
template <typename R>
__device__ __forceinline__ R consistent_rate(R sq, R D, R& p, R c, R A, R B, R Cik, R vp)
{
#pragma clang fp contract(on)
    R ld = (sq - D * (A * p + B * c)) / (R(1) + D * A * Cik + D * vp);
    if (A * (p + ld * Cik) + B * c < R(0)) ld = sq / (R(1) + D * vp);
    p = p + ld * Cik;
    return ld;
}

// Compliance 1/(G dt) of the interior 2D vertex at element e when G is given
// per cell: the mean over its four cells (cells and vertices share the
// element stride sy).
template <typename R>
__device__ __forceinline__ R vertex_compliance(const R* __restrict__ igdc, long e, long sy)
{
#pragma clang fp contract(on)
    return R(0.25) * (igdc[e - 1 - sy] + igdc[e - sy] + igdc[e - 1] + igdc[e]);
}

// Compliance of an interior 3D edge (or 2D vertex): the mean over the four
// cells around it, e - s1 - s2, e - s2, e - s1 and e (xy edges: s1 = 1,
// s2 = sy; xz: 1, sz; yz: sy, sz).
template <typename R>
__device__ __forceinline__ R edge_compliance(const R* __restrict__ igdc, long e, long s1, long s2)
{
#pragma clang fp contract(on)
    return R(0.25) * (igdc[e - s1 - s2] + igdc[e - s2] + igdc[e - s1] + igdc[e]);
}

// Return mapping at a centre.  J2 is of the trial sums T; returns Lambda
// (0 when elastic, +inf at the apex) and writes the plastic rate
// D (tauII_tr - tauII), the returned tauII and the bound Y; p gets the
// dilatant pressure correction when Cik != 0, and tauII the overstress
// vp lamdot when vp != 0.
template <typename R>
__device__ __forceinline__ R centre_lambda(R J2, R D, R& p, R c, R A, R B, R Cik, R vp, R& lamdot, R& tii,
                                           R& Y)
{
#pragma clang fp contract(on)
    R tii_tr = sqrt(J2) / D;
    Y = A * p + B * c;
    Y = Y > R(0) ? Y : R(0);
    R lam = R(0);
    lamdot = R(0);
    tii = tii_tr;
    if (tii_tr > Y) {
        R ld = R(0);
        if (Cik != R(0) || vp != R(0)) {
            ld = consistent_rate(sqrt(J2), D, p, c, A, B, Cik, vp);
            Y = A * p + B * c;
            Y = Y > R(0) ? Y : R(0);
        }
        tii = Y + vp * ld;
        lam = D * (tii_tr / tii - R(1));
        lamdot = D * (tii_tr - tii);
    }
    return lam;
}

// Reciprocal and square root of the fused sweeps: the hardware
// approximations (about 1 ulp) in FP32, IEEE operations in FP64.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }

// Return mapping at a centre (the return-mapping section, Lambda form on the
// staggered grid).  The deviator of the iteration is tau = T / (D + Lambda)
// with T = tau_k/(G~ dtau) + S, S = tau^/(G dt) + 2 e' the physical trial,
// D = 1/(G~ dtau) + Dp, Dp = 1/(G dt) + 1/mu_s.  Lambda is the radial return
// of the physical trial S (shear parts averaged from the four shear points)
// against the bound: sqrt(J2(S)) = (Dp + Lambda) tauII, tauII = max(0, A p +
// B c) (+ vp lamdot, with the pressure's dilatant correction).  With it the
// fixed point tau = S / (Dp + Lambda) solves the increment's equations with
// the pseudo-time terms removed, whatever the pseudo-time steps.  During the
// iteration Lambda is blended with the return of the pseudo-time trial
// (normal parts of T, averaged shear parts of S scaled to their pseudo-time
// form at the fixed point, f = (D + Lambda) / (Dp + Lambda)) against D:
// Lambda + blend (Lambda_T - Lambda), and the pressure likewise; both returns
// agree at the fixed point.
//   nT2, nS2: (1/2) sum of the squared normal components of T and of S;
//   sh2: sum of the squared averaged shear components of S;
//   p: the pressure update on entry, with its dilatant correction on exit.
// Returns Lambda (0 elastic, +inf at the apex).
template <typename R>
__device__ __forceinline__ R centre_return(R nT2, R nS2, R sh2, R Dp, R invDp, R D, R invD, R& p, R c, R A,
                                           R B, R Cik, R vp, R blend)
{
#pragma clang fp contract(on)   // same rounding in every kernel that inlines it
    R Y0 = A * p + B * c;
    Y0 = Y0 > R(0) ? Y0 : R(0);
    const R sqS = fast_sqrt(nS2 + sh2);
    if (!(sqS * invDp > Y0)) return R(0);
    const R ptr = p;
    R tii = Y0;
    if (Cik != R(0) || vp != R(0)) {             // dilatant and/or regularised return
        const R ld = consistent_rate(sqS, Dp, p, c, A, B, Cik, vp);
        tii = A * p + B * c;
        tii = (tii > R(0) ? tii : R(0)) + vp * ld;
    }
    R lam = sqS * fast_rcp(tii) - Dp;
    if (blend != R(0) && D != Dp && lam < R(INFINITY)) {
        const R f = (D + lam) * fast_rcp(Dp + lam);
        const R sqT = fast_sqrt(nT2 + f * f * sh2);
        R lt = R(0), pt = ptr;
        if (sqT * invD > Y0) {
            R tt = Y0;
            if (Cik != R(0) || vp != R(0)) {
                const R ld = consistent_rate(sqT, D, pt, c, A, B, Cik, vp);
                tt = A * pt + B * c;
                tt = (tt > R(0) ? tt : R(0)) + vp * ld;
            }
            lt = sqT * fast_rcp(tt) - D;
        }
        if (lt < R(INFINITY)) {
            lam = lam + blend * (lt - lam);
            p = p + blend * (pt - p);
        }
    }
    return lam;
}

}  // namespace ep
