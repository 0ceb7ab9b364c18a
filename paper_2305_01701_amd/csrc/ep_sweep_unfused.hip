// Unfused PT sweep: three kernels per iteration (centres, shear points,
// velocities), each a plain one-thread-per-point stencil.  It is the
// straightforward form of the Jacobi iteration and the fallback of the fused
// kernels; one sweep moves about 44 (3D) / 30 (2D) field accesses per cell
// instead of the 25 / 17 of a fused sweep.
//
// One iteration (paper: accelerated pseudo-transient method; return mapping):
//   centres   div v, p^{k+1} = (p^k/K~dtau + p^/(K dt) - div)/(1/K~dtau + 1/(K dt)),
//             S = tau^/(G dt) + 2 e'(v), T = tau^k/G~dtau + S, Lambda from the
//             return of centre_return (physical trial S with the 4-point means of
//             the shear-point S, blended with the pseudo-time trial), tau = T/(D+Lambda)
//   shear     T at vertices (2D) / edges (3D), Lambda = mean of the 4 adjacent
//             centres, tau = T/(D+Lambda); zero on the walls (free slip)
//   faces     R = div(tau - p I), v^{k+1} = v^k + dtau/rho~ R; wall faces keep
//             their prescribed normal velocity.
#include "ep_device.h"

namespace ep {

namespace {

constexpr int BX = 64, BY = 4, NT = BX * BY;

// Physical shear trial S = tau^/(G dt) + 2 e at the vertex e (zero on walls).
template <typename R>
__device__ __forceinline__ R vertex_S2(const SweepArgs<R>& a, long e, int i, int j)
{
    if (i <= 0 || i >= a.nx || j <= 0 || j >= a.ny) return R(0);
    const R* vx = a.it[F_VX];
    const R* vy = a.it[F_VY];
    R e2 = (vx[e] - vx[e - a.sy]) * a.idy + (vy[e] - vy[e - 1]) * a.idx;
    const R ig = a.igdc ? vertex_compliance(a.igdc, e, (long)a.sy) : a.igd;
    return a.old[O_TXY][e] * ig + e2;
}
// Pseudo-time trial T = tau^k/(G~ dtau) + S.
template <typename R>
__device__ __forceinline__ R vertex_T2(const SweepArgs<R>& a, long e, int i, int j)
{
    if (i <= 0 || i >= a.nx || j <= 0 || j >= a.ny) return R(0);
    return a.it[F_TXY][e] * a.igt + vertex_S2(a, e, i, j);
}

// ------------------------------------------------------------------ 2D
template <typename R, int MODE>
__global__ __launch_bounds__(NT) void k_centre_2d(SweepArgs<R> a)
{
    __shared__ double sh[NT / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double rmax = 0.0, smax = 0.0;
    if (i < a.nx && j < a.ny) {
        const long c = i + (long)a.sy * j;
        const R* vx = a.it[F_VX];
        const R* vy = a.it[F_VY];
        R dvx = (vx[c + 1] - vx[c]) * a.idx + a.ebx;
        R dvy = (vy[c + a.sy] - vy[c]) * a.idy + a.eby;
        R div = dvx + dvy;
        R pn = (a.it[F_P][c] * a.ikt + a.old[O_P][c] * a.ikd - div) / (a.ikt + a.ikd);
        const R igc = a.igdc ? a.igdc[c] : a.igd;        // per-cell G: the cell's compliance, Dp and D
        const R Dp = a.igdc ? igc + a.imus : a.Dp;
        const R Dc = a.igdc ? a.igt + Dp : a.D;
        const R Sxx = a.old[O_TXX][c] * igc + R(2) * (dvx - div / R(3));
        const R Syy = a.old[O_TYY][c] * igc + R(2) * (dvy - div / R(3));
        const R Txx = a.it[F_TXX][c] * a.igt + Sxx;
        const R Tyy = a.it[F_TYY][c] * a.igt + Syy;
        const R Sb = R(0.25) * (vertex_S2(a, c, i, j) + vertex_S2(a, c + 1, i + 1, j)
                              + vertex_S2(a, c + a.sy, i, j + 1) + vertex_S2(a, c + a.sy + 1, i + 1, j + 1));
        const R nS2 = R(0.5) * (Sxx * Sxx + Syy * Syy), sh2 = Sb * Sb;
        const R ptr = pn;
        R lam = centre_return(R(0.5) * (Txx * Txx + Tyy * Tyy), nS2, sh2, Dp, R(1) / Dp, Dc, R(1) / Dc, pn, a.coh[c],
                              a.A, a.B, a.Cik, a.vp, a.blend);
        if (a.lam_mode == LAM_FROZEN) {                  // frozen plasticity: Lambda held fixed
            lam = a.lam[c];
            if (a.Cik != R(0)) pn = ptr + lam * sqrt(nS2 + sh2) / (Dp + lam) * a.Cik;   // its dilatancy
        } else {
            a.lam[c] = lam;                              // read by the shear-point kernel
        }
        R txx = Txx / (Dc + lam), tyy = Tyy / (Dc + lam);
        a.nx_[F_P][c] = pn;
        a.nx_[F_TXX][c] = txx;
        a.nx_[F_TYY][c] = tyy;
        if (MODE == MODE_CHECK) {
            R dp = fabs(pn - a.it[F_P][c]) * a.rK;
            R dt = nmax(fabs(txx - a.it[F_TXX][c]), fabs(tyy - a.it[F_TYY][c])) * a.rG;
            rmax = nmax((double)dp, (double)dt);
            smax = (double)nmax(nmax(fabs(pn), fabs(txx)), fabs(tyy));
        }
    }
    if (MODE == MODE_CHECK) {
        block_max_to<NT>(rmax, a.red + RED_RESID, sh);
        block_max_to<NT>(smax, a.red + RED_SMAX, sh);
    }
}

template <typename R, int MODE>
__global__ __launch_bounds__(NT) void k_vertex_2d(SweepArgs<R> a)
{
    __shared__ double sh[NT / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double rmax = 0.0;
    if (i <= a.nx && j <= a.ny) {
        const long e = i + (long)a.sy * j;
        R t = R(0);
        if (i > 0 && i < a.nx && j > 0 && j < a.ny) {
            R T = vertex_T2(a, e, i, j);
            R lv = R(0.25) * (a.lam[e - a.sy - 1] + a.lam[e - a.sy] + a.lam[e - 1] + a.lam[e]);
            const R Dv = a.igdc ? a.igt + vertex_compliance(a.igdc, e, (long)a.sy) + a.imus : a.D;
            t = T / (Dv + lv);
        }
        a.nx_[F_TXY][e] = t;
        if (MODE == MODE_CHECK) rmax = (double)(fabs(t - a.it[F_TXY][e]) * a.rG);
    }
    if (MODE == MODE_CHECK) block_max_to<NT>(rmax, a.red + RED_RESID, sh);
}

template <typename R, int MODE>
__global__ __launch_bounds__(NT) void k_velocity_2d(SweepArgs<R> a)
{
    __shared__ double sh[NT / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double rmax = 0.0, vmax = 0.0;
    const R* p = a.nx_[F_P];
    const R* txx = a.nx_[F_TXX];
    const R* tyy = a.nx_[F_TYY];
    const R* txy = a.nx_[F_TXY];
    const long e = i + (long)a.sy * j;
    if (i <= a.nx && j < a.ny) {                    // x-faces
        R v = a.it[F_VX][e];
        if (i > 0 && i < a.nx) {
            R Rx = ((txx[e] - p[e]) - (txx[e - 1] - p[e - 1])) * a.idx + (txy[e + a.sy] - txy[e]) * a.idy;
            v = v + a.dtrho * Rx;
            rmax = nmax(rmax, (double)fabs(Rx));
        }
        if (MODE != MODE_PHYS) a.nx_[F_VX][e] = v;
        vmax = nmax(vmax, (double)fabs(v));
    }
    if (i < a.nx && j <= a.ny) {                    // y-faces
        R v = a.it[F_VY][e];
        if (j > 0 && j < a.ny) {
            R Ry = ((tyy[e] - p[e]) - (tyy[e - a.sy] - p[e - a.sy])) * a.idy + (txy[e + 1] - txy[e]) * a.idx;
            v = v + a.dtrho * Ry;
            rmax = nmax(rmax, (double)fabs(Ry));
        }
        if (MODE != MODE_PHYS) a.nx_[F_VY][e] = v;
        vmax = nmax(vmax, (double)fabs(v));
    }
    if (MODE != MODE_UPDATE) {
        block_max_to<NT>(rmax, a.red + RED_MOM, sh);
        if (MODE == MODE_CHECK) {
            block_max_to<NT>(rmax, a.red + RED_RESID, sh);
            block_max_to<NT>(vmax, a.red + RED_VMAX, sh);
        }
    }
}

// ------------------------------------------------------------------ 3D
// Physical shear trials S = tau^/(G dt) + 2 e at the three edge families,
// zero on walls; the pseudo-time trials T = tau^k/(G~ dtau) + S.
template <typename R>
__device__ __forceinline__ R S_xy(const SweepArgs<R>& a, long e, int i, int j)
{
    if (i <= 0 || i >= a.nx || j <= 0 || j >= a.ny) return R(0);
    R e2 = (a.it[F_VX][e] - a.it[F_VX][e - a.sy]) * a.idy + (a.it[F_VY][e] - a.it[F_VY][e - 1]) * a.idx;
    const R ig = a.igdc ? edge_compliance(a.igdc, e, 1L, (long)a.sy) : a.igd;
    return a.old[O_TXY][e] * ig + e2;
}
template <typename R>
__device__ __forceinline__ R S_xz(const SweepArgs<R>& a, long e, int i, int k)
{
    if (i <= 0 || i >= a.nx || k <= 0 || k >= a.nz) return R(0);
    R e2 = (a.it[F_VX][e] - a.it[F_VX][e - a.sz]) * a.idz + (a.it[F_VZ][e] - a.it[F_VZ][e - 1]) * a.idx;
    const R ig = a.igdc ? edge_compliance(a.igdc, e, 1L, a.sz) : a.igd;
    return a.old[O_TXZ][e] * ig + e2;
}
template <typename R>
__device__ __forceinline__ R S_yz(const SweepArgs<R>& a, long e, int j, int k)
{
    if (j <= 0 || j >= a.ny || k <= 0 || k >= a.nz) return R(0);
    R e2 = (a.it[F_VY][e] - a.it[F_VY][e - a.sz]) * a.idz + (a.it[F_VZ][e] - a.it[F_VZ][e - a.sy]) * a.idy;
    const R ig = a.igdc ? edge_compliance(a.igdc, e, (long)a.sy, a.sz) : a.igd;
    return a.old[O_TYZ][e] * ig + e2;
}
template <typename R>
__device__ __forceinline__ R T_xy(const SweepArgs<R>& a, long e, int i, int j)
{
    if (i <= 0 || i >= a.nx || j <= 0 || j >= a.ny) return R(0);
    return a.it[F_TXY][e] * a.igt + S_xy(a, e, i, j);
}
template <typename R>
__device__ __forceinline__ R T_xz(const SweepArgs<R>& a, long e, int i, int k)
{
    if (i <= 0 || i >= a.nx || k <= 0 || k >= a.nz) return R(0);
    return a.it[F_TXZ][e] * a.igt + S_xz(a, e, i, k);
}
template <typename R>
__device__ __forceinline__ R T_yz(const SweepArgs<R>& a, long e, int j, int k)
{
    if (j <= 0 || j >= a.ny || k <= 0 || k >= a.nz) return R(0);
    return a.it[F_TYZ][e] * a.igt + S_yz(a, e, j, k);
}

template <typename R, int MODE>
__global__ __launch_bounds__(NT) void k_centre_3d(SweepArgs<R> a)
{
    __shared__ double sh[NT / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    double rmax = 0.0, smax = 0.0;
    if (i < a.nx && j < a.ny) {
        const long c = i + (long)a.sy * j + a.sz * k;
        const long sy = a.sy, sz = a.sz;
        R dvx = (a.it[F_VX][c + 1] - a.it[F_VX][c]) * a.idx + a.ebx;
        R dvy = (a.it[F_VY][c + sy] - a.it[F_VY][c]) * a.idy + a.eby;
        R dvz = (a.it[F_VZ][c + sz] - a.it[F_VZ][c]) * a.idz + a.ebz;
        R div = dvx + dvy + dvz;
        R pn = (a.it[F_P][c] * a.ikt + a.old[O_P][c] * a.ikd - div) / (a.ikt + a.ikd);
        const R igc = a.igdc ? a.igdc[c] : a.igd;        // per-cell G: the cell's compliance, Dp and D
        const R Dp = a.igdc ? igc + a.imus : a.Dp;
        const R Dc = a.igdc ? a.igt + Dp : a.D;
        const R Sxx = a.old[O_TXX][c] * igc + R(2) * (dvx - div / R(3));
        const R Syy = a.old[O_TYY][c] * igc + R(2) * (dvy - div / R(3));
        const R Szz = -(Sxx + Syy);
        const R Txx = a.it[F_TXX][c] * a.igt + Sxx;
        const R Tyy = a.it[F_TYY][c] * a.igt + Syy;
        const R Tzz = -(Txx + Tyy);
        const R Sxy = R(0.25) * (S_xy(a, c, i, j) + S_xy(a, c + 1, i + 1, j) + S_xy(a, c + sy, i, j + 1)
                               + S_xy(a, c + sy + 1, i + 1, j + 1));
        const R Sxz = R(0.25) * (S_xz(a, c, i, k) + S_xz(a, c + 1, i + 1, k) + S_xz(a, c + sz, i, k + 1)
                               + S_xz(a, c + sz + 1, i + 1, k + 1));
        const R Syz = R(0.25) * (S_yz(a, c, j, k) + S_yz(a, c + sy, j + 1, k) + S_yz(a, c + sz, j, k + 1)
                               + S_yz(a, c + sy + sz, j + 1, k + 1));
        const R nS2 = R(0.5) * (Sxx * Sxx + Syy * Syy + Szz * Szz), sh2 = Sxy * Sxy + Sxz * Sxz + Syz * Syz;
        const R ptr = pn;
        R lam = centre_return(R(0.5) * (Txx * Txx + Tyy * Tyy + Tzz * Tzz), nS2, sh2, Dp, R(1) / Dp, Dc, R(1) / Dc,
                              pn, a.coh[c], a.A, a.B, a.Cik, a.vp, a.blend);
        if (a.lam_mode == LAM_FROZEN) {                  // frozen plasticity: Lambda held fixed
            lam = a.lam[c];
            if (a.Cik != R(0)) pn = ptr + lam * sqrt(nS2 + sh2) / (Dp + lam) * a.Cik;   // its dilatancy
        } else {
            a.lam[c] = lam;                              // read by the shear-point kernel
        }
        R txx = Txx / (Dc + lam), tyy = Tyy / (Dc + lam);
        a.nx_[F_P][c] = pn;
        a.nx_[F_TXX][c] = txx;
        a.nx_[F_TYY][c] = tyy;
        if (MODE == MODE_CHECK) {
            R dp = fabs(pn - a.it[F_P][c]) * a.rK;
            R dtx = fabs(txx - a.it[F_TXX][c]), dty = fabs(tyy - a.it[F_TYY][c]);
            R dtz = fabs((txx + tyy) - (a.it[F_TXX][c] + a.it[F_TYY][c]));
            rmax = nmax(nmax((double)dp, (double)(nmax(nmax(dtx, dty), dtz) * a.rG)), 0.0);
            smax = (double)nmax(nmax(fabs(pn), fabs(txx)), nmax(fabs(tyy), fabs(txx + tyy)));
        }
    }
    if (MODE == MODE_CHECK) {
        block_max_to<NT>(rmax, a.red + RED_RESID, sh);
        block_max_to<NT>(smax, a.red + RED_SMAX, sh);
    }
}

template <typename R, int MODE>
__global__ __launch_bounds__(NT) void k_edge_3d(SweepArgs<R> a)
{
    __shared__ double sh[NT / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    double rmax = 0.0;
    if (i <= a.nx && j <= a.ny) {
        const long e = i + (long)a.sy * j + a.sz * k;
        const long sy = a.sy, sz = a.sz;
        const R* lam = a.lam;
        if (k < a.nz) {                                   // xy edges
            R t = R(0);
            if (i > 0 && i < a.nx && j > 0 && j < a.ny) {
                R lv = R(0.25) * (lam[e - sy - 1] + lam[e - sy] + lam[e - 1] + lam[e]);
                t = T_xy(a, e, i, j) / ((a.igdc ? a.igt + edge_compliance(a.igdc, e, 1L, sy) + a.imus : a.D) + lv);
            }
            a.nx_[F_TXY][e] = t;
            if (MODE == MODE_CHECK) rmax = nmax(rmax, (double)fabs(t - a.it[F_TXY][e]));
        }
        if (j < a.ny) {                                   // xz edges
            R t = R(0);
            if (i > 0 && i < a.nx && k > 0 && k < a.nz) {
                R lv = R(0.25) * (lam[e - sz - 1] + lam[e - sz] + lam[e - 1] + lam[e]);
                t = T_xz(a, e, i, k) / ((a.igdc ? a.igt + edge_compliance(a.igdc, e, 1L, sz) + a.imus : a.D) + lv);
            }
            a.nx_[F_TXZ][e] = t;
            if (MODE == MODE_CHECK) rmax = nmax(rmax, (double)fabs(t - a.it[F_TXZ][e]));
        }
        if (i < a.nx) {                                   // yz edges
            R t = R(0);
            if (j > 0 && j < a.ny && k > 0 && k < a.nz) {
                R lv = R(0.25) * (lam[e - sz - sy] + lam[e - sz] + lam[e - sy] + lam[e]);
                t = T_yz(a, e, j, k) / ((a.igdc ? a.igt + edge_compliance(a.igdc, e, (long)sy, sz) + a.imus : a.D) + lv);
            }
            a.nx_[F_TYZ][e] = t;
            if (MODE == MODE_CHECK) rmax = nmax(rmax, (double)fabs(t - a.it[F_TYZ][e]));
        }
    }
    if (MODE == MODE_CHECK) block_max_to<NT>(rmax * (double)a.rG, a.red + RED_RESID, sh);
}

template <typename R, int MODE>
__global__ __launch_bounds__(NT) void k_velocity_3d(SweepArgs<R> a)
{
    __shared__ double sh[NT / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    double rmax = 0.0, vmax = 0.0;
    const R* p = a.nx_[F_P];
    const R* txx = a.nx_[F_TXX];
    const R* tyy = a.nx_[F_TYY];
    const R* txy = a.nx_[F_TXY];
    const R* txz = a.nx_[F_TXZ];
    const R* tyz = a.nx_[F_TYZ];
    const long sy = a.sy, sz = a.sz;
    const long e = i + sy * j + sz * k;
    if (i <= a.nx && j < a.ny && k < a.nz) {         // x-faces
        R v = a.it[F_VX][e];
        if (i > 0 && i < a.nx) {
            R Rx = ((txx[e] - p[e]) - (txx[e - 1] - p[e - 1])) * a.idx
                 + (txy[e + sy] - txy[e]) * a.idy + (txz[e + sz] - txz[e]) * a.idz;
            v = v + a.dtrho * Rx;
            rmax = nmax(rmax, (double)fabs(Rx));
        }
        if (MODE != MODE_PHYS) a.nx_[F_VX][e] = v;
        vmax = nmax(vmax, (double)fabs(v));
    }
    if (i < a.nx && j <= a.ny && k < a.nz) {         // y-faces
        R v = a.it[F_VY][e];
        if (j > 0 && j < a.ny) {
            R Ry = (txy[e + 1] - txy[e]) * a.idx
                 + ((tyy[e] - p[e]) - (tyy[e - sy] - p[e - sy])) * a.idy + (tyz[e + sz] - tyz[e]) * a.idz;
            v = v + a.dtrho * Ry;
            rmax = nmax(rmax, (double)fabs(Ry));
        }
        if (MODE != MODE_PHYS) a.nx_[F_VY][e] = v;
        vmax = nmax(vmax, (double)fabs(v));
    }
    if (i < a.nx && j < a.ny && k <= a.nz) {         // z-faces
        R v = a.it[F_VZ][e];
        if (k > 0 && k < a.nz) {
            R szu = -(txx[e] + tyy[e]) - p[e];
            R szd = -(txx[e - sz] + tyy[e - sz]) - p[e - sz];
            R Rz = (txz[e + 1] - txz[e]) * a.idx + (tyz[e + sy] - tyz[e]) * a.idy + (szu - szd) * a.idz;
            v = v + a.dtrho * Rz;
            rmax = nmax(rmax, (double)fabs(Rz));
        }
        if (MODE != MODE_PHYS) a.nx_[F_VZ][e] = v;
        vmax = nmax(vmax, (double)fabs(v));
    }
    if (MODE != MODE_UPDATE) {
        block_max_to<NT>(rmax, a.red + RED_MOM, sh);
        if (MODE == MODE_CHECK) {
            block_max_to<NT>(rmax, a.red + RED_RESID, sh);
            block_max_to<NT>(vmax, a.red + RED_VMAX, sh);
        }
    }
}

template <typename R, int MODE>
void run_2d(const SweepArgs<R>& a, hipStream_t s)
{
    dim3 blk(BX, BY);
    dim3 gc((a.nx + BX - 1) / BX, (a.ny + BY - 1) / BY);
    dim3 gv((a.nx + 1 + BX - 1) / BX, (a.ny + 1 + BY - 1) / BY);
    k_centre_2d<R, MODE><<<gc, blk, 0, s>>>(a);
    k_vertex_2d<R, MODE><<<gv, blk, 0, s>>>(a);
    k_velocity_2d<R, MODE><<<gv, blk, 0, s>>>(a);
}

template <typename R, int MODE>
void run_3d(const SweepArgs<R>& a, hipStream_t s)
{
    dim3 blk(BX, BY);
    dim3 gc((a.nx + BX - 1) / BX, (a.ny + BY - 1) / BY, a.nz);
    dim3 gv((a.nx + 1 + BX - 1) / BX, (a.ny + 1 + BY - 1) / BY, a.nz + 1);
    k_centre_3d<R, MODE><<<gc, blk, 0, s>>>(a);
    k_edge_3d<R, MODE><<<gv, blk, 0, s>>>(a);
    k_velocity_3d<R, MODE><<<gv, blk, 0, s>>>(a);
}

}  // namespace

template <typename R>
void launch_sweep_unfused_2d(const SweepArgs<R>& a, int mode, hipStream_t s)
{
    if (mode == MODE_UPDATE) run_2d<R, MODE_UPDATE>(a, s);
    else if (mode == MODE_CHECK) run_2d<R, MODE_CHECK>(a, s);
    else run_2d<R, MODE_PHYS>(a, s);
}

template <typename R>
void launch_sweep_unfused_3d(const SweepArgs<R>& a, int mode, hipStream_t s)
{
    if (mode == MODE_UPDATE) run_3d<R, MODE_UPDATE>(a, s);
    else if (mode == MODE_CHECK) run_3d<R, MODE_CHECK>(a, s);
    else run_3d<R, MODE_PHYS>(a, s);
}

template void launch_sweep_unfused_2d<double>(const SweepArgs<double>&, int, hipStream_t);
template void launch_sweep_unfused_2d<float>(const SweepArgs<float>&, int, hipStream_t);
template void launch_sweep_unfused_3d<double>(const SweepArgs<double>&, int, hipStream_t);
template void launch_sweep_unfused_3d<float>(const SweepArgs<float>&, int, hipStream_t);

}  // namespace ep
