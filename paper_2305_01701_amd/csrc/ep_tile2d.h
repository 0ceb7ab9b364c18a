// One fused 2D PT sweep over a TX x TY tile of cells (shared by the
// single-model kernel and the batched persistent kernel).
//
// The workgroup loads velocities, shear stresses (iteration k and increment
// start) over a 2-point halo and the centre data over a 1-point halo, all
// global loads issued before the first stage; then in LDS: shear trials at
// vertices (the physical trial S and the pseudo-time trial T), centre update
// (pressure, deviatoric trial, return mapping of centre_return), vertex
// stresses from the averaged centre Lambda, velocities.  Halo points
// are recomputed, so tiles are independent within a sweep.  A caller that
// runs several tiles in one workgroup must put a barrier between them (the
// last stage reads LDS that the next tile's first stage overwrites).
#pragma once
#include "ep_device.h"

namespace ep {

// Workgroup size of a tile: enough threads for one pass over the halo plane
// (W x H points), so that no wave does a second round of a stage while the
// others wait at its barrier; two balanced passes when that exceeds 1024.
template <int TX, int TY>
constexpr int tile_threads_2d()
{
    constexpr int n = (TX + 4) * (TY + 4);
    return n <= 1024 ? (n + 63) / 64 * 64 : ((n + 1) / 2 + 63) / 64 * 64;
}

template <typename R, int TX, int TY, int MODE, int NT>
__device__ __forceinline__ void sweep_tile_2d(const SweepArgs<R>& a, int bx, int by)
{
    // multiply-adds are fused only within one expression, so that every
    // caller (single-model or batched kernel) rounds each point identically
#pragma clang fp contract(on)
    constexpr int W = TX + 4, H = TY + 4, N = W * H;
    __shared__ R s_vx[N], s_vy[N], s_Txy[N], s_Sxy[N], s_lam[N], s_p[N], s_sxx[N], s_syy[N], s_nxy[N];
    __shared__ double s_red[NT / 64 > 0 ? NT / 64 : 1];

    const int i0 = bx * TX, j0 = by * TY;
    const int nx = a.nx, ny = a.ny;
    const long sy = a.sy;
    const int tid = threadIdx.x;
    const int hx = (i0 + TX == nx) ? 1 : 0;
    const int hy = (j0 + TY == ny) ? 1 : 0;
    const R idx = a.idx, idy = a.idy, igt = a.igt, igd = a.igd, ikt = a.ikt, ikd = a.ikd, D = a.D;
    double rmax = 0.0, mmax = 0.0, vmax = 0.0, smax = 0.0;   // combined, momentum-only, |v|, |stress|

    // issue every global load of the tile up front (velocities, shear stresses
    // of iteration k and of the increment start, centre data), then the stages
    constexpr int NQ = (N + NT - 1) / NT;
    constexpr int CW = TX + 2, CN = (TX + 2) * (TY + 2), NR = (CN + NT - 1) / NT;
    R gvx[NQ], gvy[NQ], gxy[NQ], gxyo[NQ];
    R gp[NR], gpo[NR], gsx[NR], gsxo[NR], gsy[NR], gsyo[NR], gc[NR];
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int q = tid + NT * u;
        const int i = i0 - 2 + q % W, j = j0 - 2 + q / W;
        const long e = i + sy * j;
        const bool ok = q < N;
        gvx[u] = (ok && i >= 0 && i <= nx && j >= 0 && j < ny) ? a.it[F_VX][e] : R(0);
        gvy[u] = (ok && i >= 0 && i < nx && j >= 0 && j <= ny) ? a.it[F_VY][e] : R(0);
        const bool exy = ok && i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1;
        gxy[u] = exy ? a.it[F_TXY][e] : R(0);
        gxyo[u] = exy ? a.old[O_TXY][e] : R(0);
    }
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int r = tid + NT * u;
        const int i = i0 - 1 + r % CW, j = j0 - 1 + r / CW;
        const long e = i + sy * j;
        const bool ok = r < CN && i >= 0 && i < nx && j >= 0 && j < ny;
        gp[u] = ok ? a.it[F_P][e] : R(0);
        gpo[u] = ok ? a.old[O_P][e] : R(0);
        gsx[u] = ok ? a.it[F_TXX][e] : R(0);
        gsxo[u] = ok ? a.old[O_TXX][e] : R(0);
        gsy[u] = ok ? a.it[F_TYY][e] : R(0);
        gsyo[u] = ok ? a.old[O_TYY][e] : R(0);
        gc[u] = ok ? a.coh[e] : R(0);
    }
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int q = tid + NT * u;
        if (q < N) {
            s_vx[q] = gvx[u];
            s_vy[q] = gvy[u];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int q = tid + NT * u;
        if (q >= N) continue;
        const int la = q % W, lbb = q / W;
        if (la < 1 || lbb < 1) continue;
        const int i = i0 - 2 + la, j = j0 - 2 + lbb;
        R t = R(0), sv = R(0);
        if (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1) {
            R e2 = (s_vx[q] - s_vx[q - W]) * idy + (s_vy[q] - s_vy[q - 1]) * idx;
            const R ig = a.igdc ? vertex_compliance(a.igdc, i + sy * j, sy) : igd;
            sv = gxyo[u] * ig + e2;
            t = gxy[u] * igt + sv;
        }
        s_Txy[q] = t;
        s_Sxy[q] = sv;
    }
    __syncthreads();
    {
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int r = tid + NT * u;
            if (r >= CN) continue;
            const int la = 1 + r % CW, lbb = 1 + r / CW;
            const int q = la + W * lbb;
            const int i = i0 - 2 + la, j = j0 - 2 + lbb;
            if (!(i >= 0 && i < nx && j >= 0 && j < ny)) {
                s_lam[q] = R(0);
                s_p[q] = R(0);
                s_sxx[q] = R(0);
                s_syy[q] = R(0);
                continue;
            }
            const long e = i + sy * j;
            R dvx = (s_vx[q + 1] - s_vx[q]) * idx + a.ebx;
            R dvy = (s_vy[q + W] - s_vy[q]) * idy + a.eby;
            R div = dvx + dvy;
            const R pk = gp[u], txk = gsx[u], tyk = gsy[u];
            R pn = (pk * ikt + gpo[u] * ikd - div) * a.ikk;
            // per-cell G: the cell's compliance, its physical Dp and its D
            const R igc = a.igdc ? a.igdc[e] : igd;
            const R Dp = a.igdc ? igc + a.imus : a.Dp;
            const R invDp = a.igdc ? R(1) / Dp : a.invDp;
            const R Dc = a.igdc ? igt + Dp : D;
            const R invDc = a.igdc ? R(1) / Dc : a.invD;
            const R Sxx = gsxo[u] * igc + R(2) * (dvx - div / R(3));
            const R Syy = gsyo[u] * igc + R(2) * (dvy - div / R(3));
            const R Txx = txk * igt + Sxx, Tyy = tyk * igt + Syy;
            const R Sb = R(0.25) * (s_Sxy[q] + s_Sxy[q + 1] + s_Sxy[q + W] + s_Sxy[q + W + 1]);
            const R nS2 = R(0.5) * (Sxx * Sxx + Syy * Syy), sh2 = Sb * Sb;
            const R ptr = pn;
            const bool own = la >= 2 && la < TX + 2 && lbb >= 2 && lbb < TY + 2;
            R lam;
            if (a.lam_mode == LAM_FROZEN) {               // frozen plasticity: the held Lambda
                lam = a.lam[e];
                // dilatancy of the held Lambda: lamdot = Lambda sqrt(J2(S)) / (Dp + Lambda)
                if (a.Cik != R(0)) pn = ptr + lam * fast_sqrt(nS2 + sh2) * fast_rcp(Dp + lam) * a.Cik;
            } else {
                lam = centre_return(R(0.5) * (Txx * Txx + Tyy * Tyy), nS2, sh2, Dp, invDp, Dc, invDc, pn, gc[u], a.A,
                                    a.B, a.Cik, a.vp, a.blend);
                if (a.lam_mode == LAM_STORE && own) a.lam[e] = lam;    // stored for freezing
            }
            const R sc_ = fast_rcp(Dc + lam);
            R txx = Txx * sc_, tyy = Tyy * sc_;
            s_lam[q] = lam;
            s_p[q] = pn;
            s_sxx[q] = txx;
            s_syy[q] = tyy;
            if (own) {
                a.nx_[F_P][e] = pn;
                a.nx_[F_TXX][e] = txx;
                a.nx_[F_TYY][e] = tyy;
                if (MODE == MODE_CHECK) {
                    R dp = fabs(pn - pk) * a.rK;
                    R dt = nmax(fabs(txx - txk), fabs(tyy - tyk)) * a.rG;
                    rmax = nmax(rmax, nmax((double)dp, (double)dt));
                    smax = nmax(smax, (double)nmax(nmax(fabs(pn), fabs(txx)), fabs(tyy)));
                }
            }
        }
    }
    __syncthreads();
    {
        constexpr int EW = TX + 1, EN = (TX + 1) * (TY + 1);
        for (int r = tid; r < EN; r += NT) {
            const int la = 2 + r % EW, lbb = 2 + r / EW;
            const int q = la + W * lbb;
            const int i = i0 - 2 + la, j = j0 - 2 + lbb;
            R t = R(0);
            if (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1) {
                R lv = R(0.25) * (s_lam[q - W - 1] + s_lam[q - W] + s_lam[q - 1] + s_lam[q]);
                const R Dv = a.igdc ? igt + vertex_compliance(a.igdc, i + sy * j, sy) + a.imus : D;
                t = s_Txy[q] * fast_rcp(Dv + lv);
            }
            s_nxy[q] = t;
            if (la < TX + 2 + hx && lbb < TY + 2 + hy && i <= nx && j <= ny) {
                const long e = i + sy * j;
                a.nx_[F_TXY][e] = t;
                if (MODE == MODE_CHECK) rmax = nmax(rmax, (double)(fabs(t - a.it[F_TXY][e]) * a.rG));
            }
        }
    }
    __syncthreads();
    {
        constexpr int FW = TX + 1, FN = (TX + 1) * (TY + 1);
        for (int r = tid; r < FN; r += NT) {
            const int la = 2 + r % FW, lbb = 2 + r / FW;
            const int q = la + W * lbb;
            const int i = i0 - 2 + la, j = j0 - 2 + lbb;
            const long e = i + sy * j;
            if (la < TX + 2 + hx && lbb < TY + 2 && i <= nx && j < ny) {
                R v = s_vx[q];
                if (i >= 1 && i <= nx - 1) {
                    R Rx = ((s_sxx[q] - s_p[q]) - (s_sxx[q - 1] - s_p[q - 1])) * idx + (s_nxy[q + W] - s_nxy[q]) * idy;
                    v = v + a.dtrho * Rx;
                    mmax = nmax(mmax, (double)fabs(Rx));
                }
                if (MODE != MODE_PHYS) a.nx_[F_VX][e] = v;
                vmax = nmax(vmax, (double)fabs(v));
            }
            if (la < TX + 2 && lbb < TY + 2 + hy && i < nx && j <= ny) {
                R v = s_vy[q];
                if (j >= 1 && j <= ny - 1) {
                    R Ry = ((s_syy[q] - s_p[q]) - (s_syy[q - W] - s_p[q - W])) * idy + (s_nxy[q + 1] - s_nxy[q]) * idx;
                    v = v + a.dtrho * Ry;
                    mmax = nmax(mmax, (double)fabs(Ry));
                }
                if (MODE != MODE_PHYS) a.nx_[F_VY][e] = v;
                vmax = nmax(vmax, (double)fabs(v));
            }
        }
    }
    if (MODE != MODE_UPDATE) {
        block_max_to<NT>(mmax, a.red + RED_MOM, s_red);
        if (MODE == MODE_CHECK) {
            block_max_to<NT>(fmax(rmax, mmax), a.red + RED_RESID, s_red);
            block_max_to<NT>(vmax, a.red + RED_VMAX, s_red);
            block_max_to<NT>(smax, a.red + RED_SMAX, s_red);
        }
    }
}

}  // namespace ep
