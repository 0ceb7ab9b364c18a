// Per-increment kernels around the PT loop: copies and precision
// conversions, wall velocities, FP64 accumulators (displacement, strain,
// plastic strain), diagnostics of the accepted state and column integrals of
// sigma_xx.  All run once per increment (or per precision switch), so they
// are simple grid-stride / one-thread-per-point kernels.
#include "ep_device.h"

namespace ep {

namespace {

constexpr int NT1 = 256;

inline int blocks_for(long n) { long b = (n + NT1 - 1) / NT1; return (int)(b > 65535L * 8 ? 65535L * 8 : b); }

__global__ void k_fill(double* p, double v, long n)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) p[q] = v;
}
__global__ void k_copy(double* d, const double* s, long n)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) d[q] = s[q];
}
// compact (x fastest) guess array -> padded FP64 field, optionally added to a
// base field of the padded layout; src == nullptr gives the base (or zero)
template <typename T>
__global__ void k_guess_in(double* d, const T* __restrict__ src, const double* __restrict__ base, int e0, int e1,
                           int e2, long sy, long sz)
{
    const long n = (long)e0 * e1 * e2;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int i = (int)(q % e0);
        const long r = q / e0;
        const int j = (int)(r % e1), k = (int)(r / e1);
        const long e = i + sy * j + sz * k;
        d[e] = (base ? base[e] : 0.0) + (src ? (double)src[q] : 0.0);
    }
}
__global__ void k_to_f32(float* d, const double* s, long n)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) d[q] = (float)s[q];
}
__global__ void k_to_f64(double* d, const float* s, long n)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) d[q] = (double)s[q];
}
__device__ __forceinline__ double face_bg(const AuxGrid& g, int d, long q, double erate, double len, double sp)
{
    const long i = q % g.sy, j = (q / g.sy) % (g.ny + 1), k = q / g.sz;
    const long n = d == 0 ? i : d == 1 ? j : k;
    return erate * (-0.5 * len + n * sp);
}
__global__ void k_vel_to_f32(AuxGrid g, int d, float* dst, const double* src, double er, double len, double sp)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < g.nelem; q += (long)gridDim.x * blockDim.x)
        dst[q] = (float)(src[q] - face_bg(g, d, q, er, len, sp));
}
__global__ void k_vel_to_f64(AuxGrid g, int d, double* dst, const float* src, double er, double len, double sp)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < g.nelem; q += (long)gridDim.x * blockDim.x)
        dst[q] = (double)src[q] + face_bg(g, d, q, er, len, sp);
}
__global__ void k_incr_to_f64(double* d, const double* b64, const float* x, const float* b32, long n)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x)
        d[q] = b64[q] + ((double)x[q] - (double)b32[q]);
}
__global__ void k_reset(unsigned long long* r)
{
    if (threadIdx.x < RED_N) r[threadIdx.x] = 0ull;
}
__global__ void k_reset_n(unsigned long long* r, int n)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) r[q] = 0ull;
}

__global__ void k_walls(AuxGrid g, double* vx, double* vy, double* vz, double ex, double ey, double ez,
                        double lx, double ly, double lz)
{
    // thread (a, b) over the largest wall face; each writes the matching
    // points of the walls it covers
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    const int nz = g.ndim == 3 ? g.nz : 1;
    // x-walls: (j, k) = (a, b)
    if (a < g.ny && b < nz) {
        long e = (long)g.sy * a + g.sz * b;
        vx[e] = -0.5 * lx * ex;
        vx[e + g.nx] = 0.5 * lx * ex;
    }
    // y-walls: (i, k) = (a, b)
    if (a < g.nx && b < nz) {
        long e = a + g.sz * b;
        vy[e] = -0.5 * ly * ey;
        vy[e + (long)g.sy * g.ny] = 0.5 * ly * ey;
    }
    // z-walls: (i, j) = (a % nx, ...): handled by a second launch dimension
    if (g.ndim == 3 && a < g.nx && b < g.ny) {
        long e = a + (long)g.sy * b;
        vz[e] = -0.5 * lz * ez;
        vz[e + g.sz * g.nz] = 0.5 * lz * ez;
    }
}

__global__ void k_accumulate(AuxGrid g, double dt, double idx, double idy, double idz,
                             const double* vx, const double* vy, const double* vz,
                             double* ux, double* uy, double* uz,
                             double* exx, double* eyy, double* ezz, double* exy, double* exz, double* eyz,
                             double* epsp, const double* lamdot)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    if (i > g.nx || j > g.ny) return;
    const bool d3 = g.ndim == 3;
    if (!d3 && k > 0) return;
    const long sy = g.sy, sz = g.sz;
    const long e = i + sy * j + sz * k;
    const int nz = d3 ? g.nz : 1;
    // displacements at faces
    if (j < g.ny && k < nz) ux[e] += dt * vx[e];
    if (i < g.nx && k < nz) uy[e] += dt * vy[e];
    if (d3 && i < g.nx && j < g.ny) uz[e] += dt * vz[e];
    // centres
    if (i < g.nx && j < g.ny && k < nz) {
        exx[e] += dt * (vx[e + 1] - vx[e]) * idx;
        eyy[e] += dt * (vy[e + sy] - vy[e]) * idy;
        if (d3) ezz[e] += dt * (vz[e + sz] - vz[e]) * idz;
        epsp[e] += dt * 0.5 * lamdot[e];
    }
    // interior shear points
    if (i > 0 && i < g.nx && j > 0 && j < g.ny && k < nz)
        exy[e] += dt * 0.5 * ((vx[e] - vx[e - sy]) * idy + (vy[e] - vy[e - 1]) * idx);
    if (d3 && i > 0 && i < g.nx && j < g.ny && k > 0 && k < g.nz)
        exz[e] += dt * 0.5 * ((vx[e] - vx[e - sz]) * idz + (vz[e] - vz[e - 1]) * idx);
    if (d3 && i < g.nx && j > 0 && j < g.ny && k > 0 && k < g.nz)
        eyz[e] += dt * 0.5 * ((vy[e] - vy[e - sz]) * idz + (vz[e] - vz[e - sy]) * idy);
}

// Centre diagnostics: one PT evaluation of the accepted state without writes
// of the state.  Mirrors the centre computation of the sweep.
template <typename R>
__device__ R shear_T(const SweepArgs<R>& a, int f, int of, long e, long s1, long s2, R i1, R i2,
                     const R* v1, const R* v2)
{
    R e2 = (v1[e] - v1[e - s1]) * i1 + (v2[e] - v2[e - s2]) * i2;
    // per-cell G: the mean compliance of the four cells around the shear point
    const R ig = !a.igdc ? a.igd
               : f == F_TXY ? edge_compliance(a.igdc, e, 1L, (long)a.sy)
               : f == F_TXZ ? edge_compliance(a.igdc, e, 1L, a.sz)
                            : edge_compliance(a.igdc, e, (long)a.sy, a.sz);
    return a.it[f][e] * a.igt + a.old[of][e] * ig + e2;
}

template <typename R>
__global__ __launch_bounds__(256) void k_diag(SweepArgs<R> a, double* lamdot, double* tii_out, double* yld)
{
    __shared__ double sh[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    const bool d3 = a.nz > 0;
    double cnt = 0.0, viol = -INFINITY;
    if (i < a.nx && j < a.ny) {
        const long sy = a.sy, sz = a.sz;
        const long c = i + sy * j + sz * k;
        const R* vx = a.it[F_VX];
        const R* vy = a.it[F_VY];
        R dvx = (vx[c + 1] - vx[c]) * a.idx;
        R dvy = (vy[c + sy] - vy[c]) * a.idy;
        R dvz = d3 ? (a.it[F_VZ][c + sz] - a.it[F_VZ][c]) * a.idz : R(0);
        R div = dvx + dvy + dvz;
        R pn = (a.it[F_P][c] * a.ikt + a.old[O_P][c] * a.ikd - div) / (a.ikt + a.ikd);
        const R igc = a.igdc ? a.igdc[c] : a.igd;        // per-cell G: compliance and D
        const R Dc = a.igdc ? a.igt + igc + a.imus : a.D;
        R Txx = a.it[F_TXX][c] * a.igt + a.old[O_TXX][c] * igc + R(2) * (dvx - div / R(3));
        R Tyy = a.it[F_TYY][c] * a.igt + a.old[O_TYY][c] * igc + R(2) * (dvy - div / R(3));
        auto Txy = [&](long e, int ii, int jj) -> R {
            if (ii <= 0 || ii >= a.nx || jj <= 0 || jj >= a.ny) return R(0);
            return shear_T(a, F_TXY, O_TXY, e, sy, 1, a.idy, a.idx, vx, vy);
        };
        R Tb = R(0.25) * (Txy(c, i, j) + Txy(c + 1, i + 1, j) + Txy(c + sy, i, j + 1) + Txy(c + sy + 1, i + 1, j + 1));
        R J2;
        // stored-stress tauII at the centre (shear averaged from the shear points)
        const R* sxy = a.it[F_TXY];
        R bxy = R(0.25) * (sxy[c] + sxy[c + 1] + sxy[c + sy] + sxy[c + sy + 1]);
        R txx_s = a.it[F_TXX][c], tyy_s = a.it[F_TYY][c];
        R tii_s;
        if (d3) {
            const R* vz = a.it[F_VZ];
            auto Txz = [&](long e, int ii, int kk) -> R {
                if (ii <= 0 || ii >= a.nx || kk <= 0 || kk >= a.nz) return R(0);
                return shear_T(a, F_TXZ, O_TXZ, e, sz, 1, a.idz, a.idx, vx, vz);
            };
            auto Tyz = [&](long e, int jj, int kk) -> R {
                if (jj <= 0 || jj >= a.ny || kk <= 0 || kk >= a.nz) return R(0);
                return shear_T(a, F_TYZ, O_TYZ, e, sz, sy, a.idz, a.idy, vy, vz);
            };
            R Tzz = -(Txx + Tyy);
            R Txzb = R(0.25) * (Txz(c, i, k) + Txz(c + 1, i + 1, k) + Txz(c + sz, i, k + 1) + Txz(c + sz + 1, i + 1, k + 1));
            R Tyzb = R(0.25) * (Tyz(c, j, k) + Tyz(c + sy, j + 1, k) + Tyz(c + sz, j, k + 1) + Tyz(c + sy + sz, j + 1, k + 1));
            J2 = R(0.5) * (Txx * Txx + Tyy * Tyy + Tzz * Tzz) + Tb * Tb + Txzb * Txzb + Tyzb * Tyzb;
            const R* sxz = a.it[F_TXZ];
            const R* syz = a.it[F_TYZ];
            R bxz = R(0.25) * (sxz[c] + sxz[c + 1] + sxz[c + sz] + sxz[c + sz + 1]);
            R byz = R(0.25) * (syz[c] + syz[c + sy] + syz[c + sz] + syz[c + sy + sz]);
            R tzz_s = -(txx_s + tyy_s);
            tii_s = sqrt(R(0.5) * (txx_s * txx_s + tyy_s * tyy_s + tzz_s * tzz_s) + bxy * bxy + bxz * bxz + byz * byz);
        } else {
            J2 = R(0.5) * (Txx * Txx + Tyy * Tyy) + Tb * Tb;
            tii_s = sqrt(R(0.5) * (txx_s * txx_s + tyy_s * tyy_s) + bxy * bxy);
        }
        R ld, tii, Y;
        R lam = centre_lambda(J2, Dc, pn, a.coh[c], a.A, a.B, a.Cik, a.vp, ld, tii, Y);
        lamdot[c] = (double)ld;
        tii_out[c] = (double)tii;
        yld[c] = (double)Y;
        cnt = lam > R(0) ? 1.0 : 0.0;
        // violation of the stored state against its own bound
        R Ys = a.A * a.it[F_P][c] + a.B * a.coh[c];
        Ys = Ys > R(0) ? Ys : R(0);
        viol = (double)(tii_s - Ys);
    }
    block_sum_to<256>(cnt, a.red + RED_NYIELD, sh);
    // the violation can be negative: shift by a large constant so that the
    // unsigned max of the bit patterns orders it correctly
    block_max_to<256>(i < a.nx && j < a.ny ? viol + 1.0 : 0.0, a.red + RED_VIOL, sh);
}

// Continuity residual of the current state: max over cells of
// |(p - p^)/(K dt) + div v| (ikd = 1/(K dt), 0 in the incompressible limit).
__global__ void k_continuity(AuxGrid g, const double* vx, const double* vy, const double* vz, const double* p,
                             const double* p_old, double ikd, double idx, double idy, double idz,
                             unsigned long long* red)
{
    __shared__ double sh[NT1 / 64];
    const int nz = g.ndim == 3 ? g.nz : 1;
    const long n = (long)g.nx * g.ny * nz;
    double m = 0.0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const long i = t % g.nx, j = (t / g.nx) % g.ny, k = t / ((long)g.nx * g.ny);
        const long c = i + g.sy * j + g.sz * k;
        double div = (vx[c + 1] - vx[c]) * idx + (vy[c + g.sy] - vy[c]) * idy;
        if (g.ndim == 3) div += (vz[c + g.sz] - vz[c]) * idz;
        m = nmax(m, fabs((p[c] - p_old[c]) * ikd + div));
    }
    block_max_to<NT1>(m, red, sh);
}

__global__ void k_columns(AuxGrid g, const double* p, const double* txx, double w, double* out)
{
    // one block per column (0, nx/2, nx-1); threads stride over (j, k)
    __shared__ double sh[4];
    const int col = blockIdx.x == 0 ? 0 : (blockIdx.x == 1 ? g.nx / 2 : g.nx - 1);
    const int nz = g.ndim == 3 ? g.nz : 1;
    const long n = (long)g.ny * nz;
    double s = 0.0;
    for (long q = threadIdx.x; q < n; q += blockDim.x) {
        long j = q % g.ny, k = q / g.ny;
        long e = col + g.sy * j + g.sz * k;
        s += (txx[e] - p[e]) * w;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// ------------------------------------------------ objective stress update
// tau^R in the component form of the paper's appendix with the vorticity
// w_ab = (dv_a/dx_b - dv_b/dx_a)/2 at its natural shear points (2D
// vertices, 3D xy/xz/yz edges), zero on wall points; centre terms are
// 4-point means of the shear products, shear-point terms use 4-point means
// of the centre stresses and of the other shear components; first-order
// upwind advection with the velocity averaged to the point, zero gradient
// where the upwind neighbour lies outside the field's grid.  Wall shear
// points keep their stresses.  All points share the padded index
// i + sy j + sz k.

// first-order upwind derivative along one axis: n = extent of the field on
// that axis, st = index stride, idx = the point's index on the axis
__device__ __forceinline__ double upwind(const double* f, long e, int idx, int n, long st, double u, double h)
{
    const int m = idx + (u > 0.0 ? -1 : 1);
    if (m < 0 || m >= n) return 0.0;
    const double f0 = f[e], f1 = f[e + (m - idx) * st];
    return u > 0.0 ? (f0 - f1) / h : (f1 - f0) / h;
}

__global__ void k_objective_2d(AuxGrid g, ObjectiveArgs a)
{
    const int nx = g.nx, ny = g.ny;
    const long sy = g.sy;
    const double *vx = a.in[F_VX], *vy = a.in[F_VY], *p = a.in[F_P], *txx = a.in[F_TXX], *tyy = a.in[F_TYY],
                 *txy = a.in[F_TXY];
    const double dx = a.dx, dy = a.dy, dt = a.dt;
    auto w = [&](int i, int j) -> double {        // vertex vorticity, 0 on walls
        if (i <= 0 || i >= nx || j <= 0 || j >= ny) return 0.0;
        const long q = i + sy * j;
        return 0.5 * ((vx[q] - vx[q - sy]) / dy - (vy[q] - vy[q - 1]) / dx);
    };
    const long n = (long)(nx + 1) * (ny + 1);
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int i = (int)(t % (nx + 1)), j = (int)(t / (nx + 1));
        const long e = i + sy * j;
        if (i < nx && j < ny) {                   // centre
            const double ux = 0.5 * (vx[e] + vx[e + 1]), uy = 0.5 * (vy[e] + vy[e + sy]);
            const double pxy = 0.25 * (txy[e] * w(i, j) + txy[e + 1] * w(i + 1, j) + txy[e + sy] * w(i, j + 1)
                                       + txy[e + sy + 1] * w(i + 1, j + 1));
            auto adv = [&](const double* f) {
                return ux * upwind(f, e, i, nx, 1, ux, dx) + uy * upwind(f, e, j, ny, sy, uy, dy);
            };
            a.out[F_P][e] = p[e] - dt * adv(p);
            a.out[F_TXX][e] = txx[e] + dt * (2.0 * pxy - adv(txx));
            a.out[F_TYY][e] = tyy[e] + dt * (-2.0 * pxy - adv(tyy));
        }
        if (i == 0 || i == nx || j == 0 || j == ny) {
            a.out[F_TXY][e] = txy[e];
        } else {                                  // interior vertex
            const double ux = 0.5 * (vx[e - sy] + vx[e]), uy = 0.5 * (vy[e - 1] + vy[e]);
            const double d = 0.25 * ((tyy[e - sy - 1] - txx[e - sy - 1]) + (tyy[e - sy] - txx[e - sy])
                                     + (tyy[e - 1] - txx[e - 1]) + (tyy[e] - txx[e]));
            const double adv = ux * upwind(txy, e, i, nx + 1, 1, ux, dx) + uy * upwind(txy, e, j, ny + 1, sy, uy, dy);
            a.out[F_TXY][e] = txy[e] + dt * (w(i, j) * d - adv);
        }
    }
}

__global__ void k_objective_3d(AuxGrid g, ObjectiveArgs a)
{
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const long sy = g.sy, sz = g.sz;
    const double *vx = a.in[F_VX], *vy = a.in[F_VY], *vz = a.in[F_VZ], *p = a.in[F_P], *txx = a.in[F_TXX],
                 *tyy = a.in[F_TYY], *txy = a.in[F_TXY], *txz = a.in[F_TXZ], *tyz = a.in[F_TYZ];
    const double dx = a.dx, dy = a.dy, dz = a.dz, dt = a.dt;
    // vorticity at the shear points, 0 on wall points
    auto wxy = [&](int i, int j, int k) -> double {
        if (i <= 0 || i >= nx || j <= 0 || j >= ny) return 0.0;
        const long q = i + sy * j + sz * k;
        return 0.5 * ((vx[q] - vx[q - sy]) / dy - (vy[q] - vy[q - 1]) / dx);
    };
    auto wxz = [&](int i, int j, int k) -> double {
        if (i <= 0 || i >= nx || k <= 0 || k >= nz) return 0.0;
        const long q = i + sy * j + sz * k;
        return 0.5 * ((vx[q] - vx[q - sz]) / dz - (vz[q] - vz[q - 1]) / dx);
    };
    auto wyz = [&](int i, int j, int k) -> double {
        if (j <= 0 || j >= ny || k <= 0 || k >= nz) return 0.0;
        const long q = i + sy * j + sz * k;
        return 0.5 * ((vy[q] - vy[q - sz]) / dz - (vz[q] - vz[q - sy]) / dy);
    };
    auto tzz = [&](long q) { return -(txx[q] + tyy[q]); };
    auto at = [&](int i, int j, int k) -> long { return i + sy * j + sz * k; };
    const long n = (long)(nx + 1) * (ny + 1) * (nz + 1);
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int i = (int)(t % (nx + 1)), j = (int)((t / (nx + 1)) % (ny + 1)), k = (int)(t / ((long)(nx + 1) * (ny + 1)));
        const long e = at(i, j, k);
        if (i < nx && j < ny && k < nz) {         // centre
            const double ux = 0.5 * (vx[e] + vx[e + 1]), uy = 0.5 * (vy[e] + vy[e + sy]), uz = 0.5 * (vz[e] + vz[e + sz]);
            double pxy = 0.0, pxz = 0.0, pyz = 0.0;
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    pxy += txy[at(i + c, j + b, k)] * wxy(i + c, j + b, k);
                    pxz += txz[at(i + c, j, k + b)] * wxz(i + c, j, k + b);
                    pyz += tyz[at(i, j + c, k + b)] * wyz(i, j + c, k + b);
                }
            pxy *= 0.25;
            pxz *= 0.25;
            pyz *= 0.25;
            auto adv = [&](const double* f) {
                return ux * upwind(f, e, i, nx, 1, ux, dx) + uy * upwind(f, e, j, ny, sy, uy, dy)
                     + uz * upwind(f, e, k, nz, sz, uz, dz);
            };
            a.out[F_P][e] = p[e] - dt * adv(p);
            a.out[F_TXX][e] = txx[e] + dt * (2.0 * (pxy + pxz) - adv(txx));
            a.out[F_TYY][e] = tyy[e] + dt * (-2.0 * (pxy - pyz) - adv(tyy));
        }
        if (k < nz) {                             // xy edge (x_i, y_j, z_k+1/2)
            if (i == 0 || i == nx || j == 0 || j == ny) {
                a.out[F_TXY][e] = txy[e];
            } else {
                const double ux = 0.5 * (vx[e - sy] + vx[e]), uy = 0.5 * (vy[e - 1] + vy[e]);
                double uz = 0.0, d = 0.0, tb = 0.0, wb = 0.0, sb = 0.0, vb = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = -1; b < 1; ++b)
                        for (int a2 = -1; a2 < 1; ++a2) uz += vz[at(i + a2, j + b, k + c)];
                for (int b = -1; b < 1; ++b)
                    for (int a2 = -1; a2 < 1; ++a2) d += tyy[at(i + a2, j + b, k)] - txx[at(i + a2, j + b, k)];
                for (int c = 0; c < 2; ++c)
                    for (int a2 = -1; a2 < 1; ++a2) {   // yz edges around
                        tb += tyz[at(i + a2, j, k + c)];
                        wb += wyz(i + a2, j, k + c);
                    }
                for (int c = 0; c < 2; ++c)
                    for (int b = -1; b < 1; ++b) {      // xz edges around
                        sb += txz[at(i, j + b, k + c)];
                        vb += wxz(i, j + b, k + c);
                    }
                uz *= 0.125;
                d *= 0.25; tb *= 0.25; wb *= 0.25; sb *= 0.25; vb *= 0.25;
                const double r = wxy(i, j, k) * d + tb * vb + sb * wb;
                const double adv = ux * upwind(txy, e, i, nx + 1, 1, ux, dx) + uy * upwind(txy, e, j, ny + 1, sy, uy, dy)
                                 + uz * upwind(txy, e, k, nz, sz, uz, dz);
                a.out[F_TXY][e] = txy[e] + dt * (r - adv);
            }
        }
        if (j < ny) {                             // xz edge (x_i, y_j+1/2, z_k)
            if (i == 0 || i == nx || k == 0 || k == nz) {
                a.out[F_TXZ][e] = txz[e];
            } else {
                const double ux = 0.5 * (vx[e - sz] + vx[e]), uz = 0.5 * (vz[e - 1] + vz[e]);
                double uy = 0.0, d = 0.0, tb = 0.0, wb = 0.0, sb = 0.0, vb = 0.0;
                for (int c = -1; c < 1; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a2 = -1; a2 < 1; ++a2) uy += vy[at(i + a2, j + b, k + c)];
                for (int c = -1; c < 1; ++c)
                    for (int a2 = -1; a2 < 1; ++a2) d += tzz(at(i + a2, j, k + c)) - txx[at(i + a2, j, k + c)];
                for (int b = 0; b < 2; ++b)
                    for (int a2 = -1; a2 < 1; ++a2) {   // yz edges around
                        tb += tyz[at(i + a2, j + b, k)];
                        wb += wyz(i + a2, j + b, k);
                    }
                for (int c = -1; c < 1; ++c)
                    for (int b = 0; b < 2; ++b) {       // xy edges around
                        sb += txy[at(i, j + b, k + c)];
                        vb += wxy(i, j + b, k + c);
                    }
                uy *= 0.125;
                d *= 0.25; tb *= 0.25; wb *= 0.25; sb *= 0.25; vb *= 0.25;
                const double r = wxz(i, j, k) * d + tb * vb - sb * wb;
                const double adv = ux * upwind(txz, e, i, nx + 1, 1, ux, dx) + uy * upwind(txz, e, j, ny, sy, uy, dy)
                                 + uz * upwind(txz, e, k, nz + 1, sz, uz, dz);
                a.out[F_TXZ][e] = txz[e] + dt * (r - adv);
            }
        }
        if (i < nx) {                             // yz edge (x_i+1/2, y_j, z_k)
            if (j == 0 || j == ny || k == 0 || k == nz) {
                a.out[F_TYZ][e] = tyz[e];
            } else {
                const double uy = 0.5 * (vy[e - sz] + vy[e]), uz = 0.5 * (vz[e - sy] + vz[e]);
                double ux = 0.0, d = 0.0, sb = 0.0, vb = 0.0, tb = 0.0, wb = 0.0;
                for (int c = -1; c < 1; ++c)
                    for (int b = -1; b < 1; ++b)
                        for (int a2 = 0; a2 < 2; ++a2) ux += vx[at(i + a2, j + b, k + c)];
                for (int c = -1; c < 1; ++c)
                    for (int b = -1; b < 1; ++b) d += tzz(at(i, j + b, k + c)) - tyy[at(i, j + b, k + c)];
                for (int c = -1; c < 1; ++c)
                    for (int a2 = 0; a2 < 2; ++a2) {    // xy edges around
                        sb += txy[at(i + a2, j, k + c)];
                        vb += wxy(i + a2, j, k + c);
                    }
                for (int b = -1; b < 1; ++b)
                    for (int a2 = 0; a2 < 2; ++a2) {    // xz edges around
                        tb += txz[at(i + a2, j + b, k)];
                        wb += wxz(i + a2, j + b, k);
                    }
                ux *= 0.125;
                d *= 0.25; sb *= 0.25; vb *= 0.25; tb *= 0.25; wb *= 0.25;
                const double r = wyz(i, j, k) * d - sb * wb - tb * vb;
                const double adv = ux * upwind(tyz, e, i, nx, 1, ux, dx) + uy * upwind(tyz, e, j, ny + 1, sy, uy, dy)
                                 + uz * upwind(tyz, e, k, nz + 1, sz, uz, dz);
                a.out[F_TYZ][e] = tyz[e] + dt * (r - adv);
            }
        }
    }
}

}  // namespace

void launch_fill(double* p, double v, long n, hipStream_t s) { k_fill<<<blocks_for(n), NT1, 0, s>>>(p, v, n); }
void launch_guess_in(double* d, const void* src, bool f32, const double* base, const int ext[3], long sy, long sz,
                     hipStream_t s)
{
    const long n = (long)ext[0] * ext[1] * ext[2];
    if (f32)
        k_guess_in<float><<<blocks_for(n), NT1, 0, s>>>(d, (const float*)src, base, ext[0], ext[1], ext[2], sy, sz);
    else
        k_guess_in<double><<<blocks_for(n), NT1, 0, s>>>(d, (const double*)src, base, ext[0], ext[1], ext[2], sy, sz);
}
void launch_copy(double* d, const double* src, long n, hipStream_t s) { k_copy<<<blocks_for(n), NT1, 0, s>>>(d, src, n); }
void launch_to_f32(float* d, const double* src, long n, hipStream_t s) { k_to_f32<<<blocks_for(n), NT1, 0, s>>>(d, src, n); }
void launch_to_f64(double* d, const float* src, long n, hipStream_t s) { k_to_f64<<<blocks_for(n), NT1, 0, s>>>(d, src, n); }
void launch_vel_to_f32(const AuxGrid& g, int d, float* dst, const double* src, double erate, double len,
                       double spacing, hipStream_t s)
{
    k_vel_to_f32<<<blocks_for(g.nelem), NT1, 0, s>>>(g, d, dst, src, erate, len, spacing);
}
void launch_vel_to_f64(const AuxGrid& g, int d, double* dst, const float* src, double erate, double len,
                       double spacing, hipStream_t s)
{
    k_vel_to_f64<<<blocks_for(g.nelem), NT1, 0, s>>>(g, d, dst, src, erate, len, spacing);
}
void launch_incr_to_f64(double* d, const double* b64, const float* x, const float* b32, long n, hipStream_t s)
{
    k_incr_to_f64<<<blocks_for(n), NT1, 0, s>>>(d, b64, x, b32, n);
}
void launch_reset_red(unsigned long long* red, hipStream_t s) { k_reset<<<1, 64, 0, s>>>(red); }
void launch_reset_red_n(unsigned long long* red, int n_models, hipStream_t s)
{
    const int n = n_models * RED_N;
    k_reset_n<<<(n + 255) / 256, 256, 0, s>>>(red, n);
}

void launch_set_walls(const AuxGrid& g, double* vx, double* vy, double* vz, const double erate[3],
                      double lx, double ly, double lz, hipStream_t s)
{
    int na = g.nx > g.ny ? g.nx : g.ny;
    int nb = g.ndim == 3 ? (g.nz > g.ny ? g.nz : g.ny) : 1;
    dim3 grid((na + 127) / 128, nb);
    k_walls<<<grid, 128, 0, s>>>(g, vx, vy, vz, erate[0], erate[1], erate[2], lx, ly, lz);
}

void launch_accumulate(const AuxGrid& g, double dt, double idx, double idy, double idz,
                       const double* const v[3], double* const u[3], double* const e[6],
                       double* epsp, const double* lamdot, hipStream_t s)
{
    dim3 grid((g.nx + 1 + 127) / 128, g.ny + 1, g.ndim == 3 ? g.nz + 1 : 1);
    k_accumulate<<<grid, 128, 0, s>>>(g, dt, idx, idy, idz, v[0], v[1], v[2], u[0], u[1], u[2],
                                      e[0], e[1], e[2], e[3], e[4], e[5], epsp, lamdot);
}

template <typename R>
void launch_diagnostics(const SweepArgs<R>& a, double* lamdot, double* tii, double* yld, hipStream_t s)
{
    dim3 grid((a.nx + 255) / 256, a.ny, a.nz > 0 ? a.nz : 1);
    k_diag<R><<<grid, 256, 0, s>>>(a, lamdot, tii, yld);
}
template void launch_diagnostics<double>(const SweepArgs<double>&, double*, double*, double*, hipStream_t);
template void launch_diagnostics<float>(const SweepArgs<float>&, double*, double*, double*, hipStream_t);

void launch_continuity(const AuxGrid& g, const double* const v[3], const double* p, const double* p_old, double ikd,
                       double idx, double idy, double idz, unsigned long long* red_slot, hipStream_t s)
{
    const int nz = g.ndim == 3 ? g.nz : 1;
    k_continuity<<<blocks_for((long)g.nx * g.ny * nz), NT1, 0, s>>>(g, v[0], v[1], v[2], p, p_old, ikd, idx, idy,
                                                                   idz, red_slot);
}

void launch_column_integrals(const AuxGrid& g, const double* p, const double* txx, double dy, double dz,
                             double* out3, hipStream_t s)
{
    k_columns<<<3, 256, 0, s>>>(g, p, txx, g.ndim == 3 ? dy * dz : dy, out3);
}

void launch_objective(const AuxGrid& g, const ObjectiveArgs& a, hipStream_t s)
{
    const long n = (long)(g.nx + 1) * (g.ny + 1) * (g.ndim == 3 ? g.nz + 1 : 1);
    if (g.ndim == 3) k_objective_3d<<<blocks_for(n), NT1, 0, s>>>(g, a);
    else k_objective_2d<<<blocks_for(n), NT1, 0, s>>>(g, a);
}

}  // namespace ep
