// Fused PT sweep: one kernel per pseudo-transient iteration.
//
// One iteration couples points up to two cells apart (v -> shear trial at
// edges -> 4-point mean at centres -> Lambda at centres -> mean back to
// edges -> velocity), so a workgroup that owns a tile recomputes a halo:
//
//   3D: a workgroup owns a TX x TY column of cells over a chunk of ZC
//   z-planes and marches up the chunk.  Every quantity lives in LDS as 2D
//   planes of (TX+4) x (TY+4) points (a 2-point x-y halo) in two-slot ring
//   buffers over z.  Step f of the march forms the shear trials on the
//   z-level f (xz, yz edges) and the plane f-1 (xy edges), the centre update
//   of plane f-1 (pressure, deviator, return mapping), the new edge stresses
//   of plane/level f-1, and the new velocities of plane f-2 (vx, vy) and
//   level f-1 (vz), then stores the velocity planes of step f+1 to LDS: four
//   workgroup barriers per step.  The velocity stage updates each thread's
//   own plane points, whose old values the thread keeps in registers.  Each
//   field is read from and written to HBM once per sweep; the halo reads of
//   neighbouring tiles are served by L2 (blocks are remapped so that spatial
//   neighbours run on the same XCD).
//   2D: the same stages on a single TX x TY tile (ep_tile2d.h, run by the
//   tile-list kernel of ep_sweep_batch.hip for single models and batches).
//
// The arithmetic of every point is that of the unfused sweep (same formulas,
// same Jacobi order: all reads are of iteration k, all writes iteration k+1).
#include <type_traits>

#include "ep_device.h"

namespace ep {

namespace {

__device__ __forceinline__ int mod2(int f) { return f & 1; }

// Tile grid of a 3D sweep and its interior rectangle [bx0, bx1) x [by0,
// by1): tiles whose points, 2-point halo included, lie strictly inside the
// domain in x and y.
struct TileSet {
    int nbx, nby, nbz;
    int bx0, bx1, by0, by1;
};

// ----------------------------------------------------------------------- 3D
// Global data a march step needs is prefetched into registers one step
// ahead (velocities of plane f+1, edge stresses of level f+1 and plane f,
// centre data of plane f, and with a per-cell G the compliances of plane
// f+1), so that HBM latency overlaps the LDS work of the current step.  Each
// thread owns the same plane positions in every step; the edge stage (S4)
// works on the edge points among them, so the edge stresses of iteration k
// it needs (for the pseudo-time trial and the residual) are the thread's own
// prefetched values, and only the physical trials S (which the centres
// average) go through LDS.
template <typename R, int TX, int TY, int ZC, int MODE, int NT, int WPE, bool HG>
__global__ __attribute__((amdgpu_flat_work_group_size(1, NT), amdgpu_waves_per_eu(WPE)))
void k_fused_3d(SweepArgs<R> a, TileSet ts)
{
    constexpr int W = TX + 4, H = TY + 4, N = W * H;
    constexpr int NQ = (N + NT - 1) / NT;                  // plane positions per thread
    constexpr int CW = TX + 2, CN = (TX + 2) * (TY + 2);   // centre region (1-cell halo)
    constexpr int NR = (CN + NT - 1) / NT;
    constexpr int NG = HG ? 2 : 1;
    __shared__ R s_vx[2][N], s_vy[2][N], s_vz[2][N];
    __shared__ R s_Sxy[N], s_Sxz[2][N], s_Syz[2][N];
    __shared__ R s_lam[2][N], s_p[2][N], s_sxx[2][N], s_syy[2][N];
    __shared__ R s_nxy[2][N], s_nxz[2][N], s_nyz[2][N];
    __shared__ R s_ig[NG][HG ? N : 1];                    // per-cell 1/(G dt), two planes
    __shared__ double s_red[NT / 64 > 0 ? NT / 64 : 1];

    const int lb = xcd_remap(blockIdx.x, ts.nbx * ts.nby * ts.nbz);
    const int bx = lb % ts.nbx, by = (lb / ts.nbx) % ts.nby, bz = lb / (ts.nbx * ts.nby);
    // the same sweep, compiled twice: for tiles strictly inside the domain in
    // x and y no point needs a boundary test
    auto body = [&](auto interior) {
    constexpr bool INT = decltype(interior)::value;
    const int i0 = bx * TX, j0 = by * TY;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int k0 = bz * ZC, k1 = min(k0 + ZC, nz);
    const long sz = a.sz;
    const int tid = threadIdx.x;
    const int hx = (i0 + TX == nx) ? 1 : 0;     // owns the x = nx row when nx % TX == 0
    const int hy = (j0 + TY == ny) ? 1 : 0;
    const bool last_z = (k1 == nz);

    // Fields are addressed from the first field of their group (iteration
    // k, k+1, increment start) and the uniform field stride fs, and points
    // as a uniform plane address plus a 32-bit in-plane byte offset: the
    // loads and stores take a scalar base and one vector offset, and the 26
    // field pointers need not stay in scalar registers.  fs is made opaque
    // to the compiler once per march step so that the field addresses are
    // formed where they are used rather than hoisted out of the loop and
    // kept live (spilled) over it.
    const R* const itb = a.it[0];
    R* const nxb = a.nx_[0];
    const R* const olb = a.old[0];
    long fs = a.fs;
    auto ld = [](const R* pl, unsigned o) -> R { return *(const R*)((const char*)pl + o); };
    auto st = [](R* pl, unsigned o, R v) { *(R*)((char*)pl + o) = v; };
    auto off = [&](int i, int j) -> unsigned { return (unsigned)(i + a.sy * j) * (unsigned)sizeof(R); };
    const R idx = a.idx, idy = a.idy, idz = a.idz, igt = a.igt, igd = a.igd, ikt = a.ikt, ikd = a.ikd;
    const R D = a.D;

    // per-thread positions: plane points q (S1, S2, S4, S5) and centre points r (S3)
    int qi[NQ], qj[NQ];
    unsigned qo[NQ];
    bool qok[NQ];
    for (int u = 0; u < NQ; ++u) {
        const int q = tid + NT * u;
        qok[u] = q < N;
        qi[u] = i0 - 2 + q % W;
        qj[u] = j0 - 2 + q / W;
        qo[u] = off(qi[u], qj[u]);
    }
    int ri[NR], rj[NR];
    unsigned ro[NR];
    bool rok[NR];
    for (int u = 0; u < NR; ++u) {
        const int r = tid + NT * u;
        rok[u] = r < CN;
        ri[u] = i0 - 1 + r % CW;
        rj[u] = j0 - 1 + r / CW;
        ro[u] = off(ri[u], rj[u]);
    }

    // prefetch registers (step g)
    R fvx[NQ], fvy[NQ], fvz[NQ], fxz[NQ], fxzo[NQ], fyz[NQ], fyzo[NQ], fxy[NQ], fxyo[NQ], fig[NQ];
    R fp[NR], fpo[NR], fsx[NR], fsxo[NR], fsy[NR], fsyo[NR], fc[NR];
    auto prefetch = [&](int g) {
        const bool pl = g >= 0 && g < nz, lv = g >= 0 && g <= nz, inner = g >= 1 && g <= nz - 1;
        const bool pm = g - 1 >= 0 && g - 1 < nz;
        const long pg = sz * g, pg1 = pg - sz;
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int i = qi[u], j = qj[u];
            const unsigned o = qo[u];
            const bool ok = qok[u];
            fvx[u] = (ok && pl && (INT || (i >= 0 && i <= nx && j >= 0 && j < ny))) ? ld(itb + F_VX * fs + pg, o) : R(0);
            fvy[u] = (ok && pl && (INT || (i >= 0 && i < nx && j >= 0 && j <= ny))) ? ld(itb + F_VY * fs + pg, o) : R(0);
            fvz[u] = (ok && lv && (INT || (i >= 0 && i < nx && j >= 0 && j < ny))) ? ld(itb + F_VZ * fs + pg, o) : R(0);
            // edge stresses of iteration k wherever the edge exists (wall
            // values enter the residual), increment-start values inside
            const bool xz_in = INT || (i >= 0 && i <= nx && j >= 0 && j < ny);
            const bool yz_in = INT || (i >= 0 && i < nx && j >= 0 && j <= ny);
            const bool xy_in = INT || (i >= 0 && i <= nx && j >= 0 && j <= ny);
            fxz[u] = (ok && lv && xz_in) ? ld(itb + F_TXZ * fs + pg, o) : R(0);
            fyz[u] = (ok && lv && yz_in) ? ld(itb + F_TYZ * fs + pg, o) : R(0);
            fxy[u] = (ok && pm && xy_in) ? ld(itb + F_TXY * fs + pg1, o) : R(0);
            const bool exz = ok && inner && (INT || (i >= 1 && i <= nx - 1 && j >= 0 && j < ny));
            const bool eyz = ok && inner && (INT || (j >= 1 && j <= ny - 1 && i >= 0 && i < nx));
            fxzo[u] = exz ? ld(olb + O_TXZ * fs + pg, o) : R(0);
            fyzo[u] = eyz ? ld(olb + O_TYZ * fs + pg, o) : R(0);
            const bool exy = ok && pm && (INT || (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1));
            fxyo[u] = exy ? ld(olb + O_TXY * fs + pg1, o) : R(0);
            if (HG)
                fig[u] = (ok && pl && (INT || (i >= 0 && i < nx && j >= 0 && j < ny))) ? ld(a.igdc + pg, o) : R(0);
        }
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int i = ri[u], j = rj[u];
            const unsigned o = ro[u];
            const bool ok = rok[u] && pm && (INT || (i >= 0 && i < nx && j >= 0 && j < ny));
            fp[u] = ok ? ld(itb + F_P * fs + pg1, o) : R(0);
            fpo[u] = ok ? ld(olb + O_P * fs + pg1, o) : R(0);
            fsx[u] = ok ? ld(itb + F_TXX * fs + pg1, o) : R(0);
            fsxo[u] = ok ? ld(olb + O_TXX * fs + pg1, o) : R(0);
            fsy[u] = ok ? ld(itb + F_TYY * fs + pg1, o) : R(0);
            fsyo[u] = ok ? ld(olb + O_TYY * fs + pg1, o) : R(0);
            fc[u] = ok ? ld(a.coh + pg1, o) : R(0);
        }
    };

    // combined, momentum-only, |v|, |stress| maxima, kept in the field type
    // (maxima are exact) and widened for the block reduction
    R rmax = R(0), mmax = R(0), vmax = R(0), smax = R(0);

    // S1 of step g: the prefetched velocities of plane g (vx, vy) and level
    // g (vz), and the compliances of plane g, go to LDS and the velocities
    // into this thread's register history, from which S5 takes the old
    // velocities of its own points (vx, vy of plane g-2, vz of level g-1 at
    // step g)
    R hvx1[NQ], hvx2[NQ], hvx3[NQ], hvy1[NQ], hvy2[NQ], hvy3[NQ], hvz1[NQ], hvz2[NQ];
    auto stage_velocities = [&](int g) {
        const bool ld_xy = g >= 0 && g < nz;
        const bool ld_z = g >= 0 && g <= nz;
        const int s2 = mod2(g);
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            hvx3[u] = hvx2[u]; hvx2[u] = hvx1[u]; hvx1[u] = fvx[u];
            hvy3[u] = hvy2[u]; hvy2[u] = hvy1[u]; hvy1[u] = fvy[u];
            hvz2[u] = hvz1[u]; hvz1[u] = fvz[u];
            if (!qok[u]) continue;
            const int q = tid + NT * u;
            if (ld_xy) {
                s_vx[s2][q] = fvx[u];
                s_vy[s2][q] = fvy[u];
                if (HG) s_ig[s2 & (NG - 1)][q] = fig[u];
            }
            if (ld_z) s_vz[s2][q] = fvz[u];
        }
    };
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        hvx1[u] = hvx2[u] = hvx3[u] = R(0);
        hvy1[u] = hvy2[u] = hvy3[u] = R(0);
        hvz1[u] = hvz2[u] = R(0);
    }
    // edge stresses of iteration k at the level of the previous step (xz,
    // yz), and with a per-cell G the edge compliances of this step (xy at
    // plane f-1; xz, yz at level f) and of the previous step (xz, yz)
    R pcxz[NQ], pcyz[NQ], gxy[NQ], gxz[NQ], gyz[NQ], pgxz[NQ], pgyz[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        pcxz[u] = pcyz[u] = R(0);
        gxy[u] = gxz[u] = gyz[u] = pgxz[u] = pgyz[u] = igd;
    }
    prefetch(k0 - 2);
    stage_velocities(k0 - 2);
    __syncthreads();
    for (int f = k0 - 2; f <= k1 + 1; ++f) {
        asm volatile("" : "+s"(fs));
        // take over the data of step f, start loading step f+1
        R cxz[NQ], cxzo[NQ], cyz[NQ], cyzo[NQ], cxy[NQ], cxyo[NQ];
        R cp[NR], cpo[NR], csx[NR], csxo[NR], csy[NR], csyo[NR], cc[NR];
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            cxz[u] = fxz[u]; cxzo[u] = fxzo[u]; cyz[u] = fyz[u]; cyzo[u] = fyzo[u];
            cxy[u] = fxy[u]; cxyo[u] = fxyo[u];
            if (HG) { pgxz[u] = gxz[u]; pgyz[u] = gyz[u]; }
        }
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            cp[u] = fp[u]; cpo[u] = fpo[u]; csx[u] = fsx[u]; csxo[u] = fsxo[u];
            csy[u] = fsy[u]; csyo[u] = fsyo[u]; cc[u] = fc[u];
        }
        if (f + 1 <= k1 + 1) prefetch(f + 1);

        // ---- S2: physical shear trials: xz, yz at level f; xy at plane f-1 --
        {
            const bool do_l = f >= k0 - 1 && f >= 0 && f <= nz;
            const bool do_p = f - 1 >= k0 - 1 && f - 1 >= 0 && f - 1 < nz;
            const int l = f, sl = mod2(l), cm = mod2(l), cp3 = mod2(l - 1), pm = mod2(f - 1);
            const bool inner_l = l >= 1 && l <= nz - 1;
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int q = tid + NT * u;
                if (!qok[u] || q % W < 1 || q / W < 1) continue;
                const int i = qi[u], j = qj[u];
                if (do_l) {
                    R sxz = R(0), syz = R(0);
                    if (HG) {       // compliance of an edge: mean of its four cells
                        const int a0 = sl & (NG - 1), a1 = cp3 & (NG - 1);
                        gxz[u] = inner_l ? R(0.25) * (s_ig[a1][q - 1] + s_ig[a1][q] + s_ig[a0][q - 1] + s_ig[a0][q]) : igd;
                        gyz[u] = inner_l ? R(0.25) * (s_ig[a1][q - W] + s_ig[a1][q] + s_ig[a0][q - W] + s_ig[a0][q]) : igd;
                    }
                    if (inner_l && (INT || (i >= 1 && i <= nx - 1 && j >= 0 && j < ny))) {
                        R e2 = (s_vx[cm][q] - s_vx[cp3][q]) * idz + (s_vz[sl][q] - s_vz[sl][q - 1]) * idx;
                        sxz = cxzo[u] * (HG ? gxz[u] : igd) + e2;
                    }
                    if (inner_l && (INT || (j >= 1 && j <= ny - 1 && i >= 0 && i < nx))) {
                        R e2 = (s_vy[cm][q] - s_vy[cp3][q]) * idz + (s_vz[sl][q] - s_vz[sl][q - W]) * idy;
                        syz = cyzo[u] * (HG ? gyz[u] : igd) + e2;
                    }
                    s_Sxz[sl][q] = sxz;
                    s_Syz[sl][q] = syz;
                }
                if (do_p) {
                    R t = R(0);
                    if (HG) {
                        const int a0 = pm & (NG - 1);
                        gxy[u] = R(0.25) * (s_ig[a0][q - W - 1] + s_ig[a0][q - W] + s_ig[a0][q - 1] + s_ig[a0][q]);
                    }
                    if (INT || (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1)) {
                        R e2 = (s_vx[pm][q] - s_vx[pm][q - W]) * idy + (s_vy[pm][q] - s_vy[pm][q - 1]) * idx;
                        t = cxyo[u] * (HG ? gxy[u] : igd) + e2;
                    }
                    s_Sxy[q] = t;
                }
            }
        }
        __syncthreads();
        // ---- S3: centres of plane c = f-1 -----------------------------------
        const int c = f - 1;
        if (c >= k0 - 1 && c >= 0 && c < nz && c <= k1) {
            const int cm = mod2(c), sc = mod2(c), sc1 = mod2(c + 1);
#pragma unroll
            for (int u = 0; u < NR; ++u) {
                if (!rok[u]) continue;
                const int r = tid + NT * u;
                const int la = 1 + r % CW, lbb = 1 + r / CW;
                const int q = la + W * lbb;
                const int i = ri[u], j = rj[u];
                if (!INT && !(i >= 0 && i < nx && j >= 0 && j < ny)) {
                    s_lam[sc][q] = R(0);
                    s_p[sc][q] = R(0);
                    s_sxx[sc][q] = R(0);
                    s_syy[sc][q] = R(0);
                    continue;
                }
                R dvx = (s_vx[cm][q + 1] - s_vx[cm][q]) * idx + a.ebx;
                R dvy = (s_vy[cm][q + W] - s_vy[cm][q]) * idy + a.eby;
                R dvz = (s_vz[sc1][q] - s_vz[sc][q]) * idz + a.ebz;
                R div = dvx + dvy + dvz;
                const R pk = cp[u], txk = csx[u], tyk = csy[u];
                R pn = (pk * ikt + cpo[u] * ikd - div) * a.ikk;
                // per-cell G: the cell's compliance, its physical Dp and its D
                const R igc = HG ? s_ig[cm & (NG - 1)][q] : igd;
                const R Dp = HG ? igc + a.imus : a.Dp;
                const R invDp = HG ? fast_rcp(Dp) : a.invDp;
                const R Dc = HG ? igt + Dp : D;
                const R invDc = HG ? fast_rcp(Dc) : a.invD;
                const R Sxx = csxo[u] * igc + R(2) * (dvx - div * R(1.0 / 3.0));
                const R Syy = csyo[u] * igc + R(2) * (dvy - div * R(1.0 / 3.0));
                const R Szz = -(Sxx + Syy);
                const R Txx = txk * igt + Sxx, Tyy = tyk * igt + Syy, Tzz = -(Txx + Tyy);
                const R Sxyb = R(0.25) * (s_Sxy[q] + s_Sxy[q + 1] + s_Sxy[q + W] + s_Sxy[q + W + 1]);
                const R Sxzb = R(0.25) * (s_Sxz[sc][q] + s_Sxz[sc][q + 1] + s_Sxz[sc1][q] + s_Sxz[sc1][q + 1]);
                const R Syzb = R(0.25) * (s_Syz[sc][q] + s_Syz[sc][q + W] + s_Syz[sc1][q] + s_Syz[sc1][q + W]);
                const R nS2 = R(0.5) * (Sxx * Sxx + Syy * Syy + Szz * Szz);
                const R sh2 = Sxyb * Sxyb + Sxzb * Sxzb + Syzb * Syzb;
                const R ptr = pn;
                const bool own = la >= 2 && la < TX + 2 && lbb >= 2 && lbb < TY + 2 && c >= k0 && c < k1;
                R lam;
                if (a.lam_mode == LAM_FROZEN) {                  // frozen plasticity: the held Lambda
                    lam = ld(a.lam + sz * c, ro[u]);
                    // dilatancy of the held Lambda: lamdot = Lambda sqrt(J2(S)) / (Dp + Lambda)
                    if (a.Cik != R(0)) pn = ptr + lam * fast_sqrt(nS2 + sh2) * fast_rcp(Dp + lam) * a.Cik;
                } else {
                    lam = centre_return(R(0.5) * (Txx * Txx + Tyy * Tyy + Tzz * Tzz), nS2, sh2, Dp, invDp, Dc, invDc,
                                        pn, cc[u], a.A, a.B, a.Cik, a.vp, a.blend);
                    if (a.lam_mode != LAM_COMPUTE && own) st(a.lam + sz * c, ro[u], lam);     // stored for freezing
                }
                const R sc_ = fast_rcp(Dc + lam);
                R txx = Txx * sc_, tyy = Tyy * sc_;
                s_lam[sc][q] = lam;
                s_p[sc][q] = pn;
                s_sxx[sc][q] = txx;
                s_syy[sc][q] = tyy;
                if (own) {
                    const long pc = sz * c;
                    st(nxb + F_P * fs + pc, ro[u], pn);
                    st(nxb + F_TXX * fs + pc, ro[u], txx);
                    st(nxb + F_TYY * fs + pc, ro[u], tyy);
                    if (MODE == MODE_CHECK) {
                        R dp = fabs(pn - pk) * a.rK;
                        R dtx = fabs(txx - txk), dty = fabs(tyy - tyk), dtz = fabs((txx + tyy) - (txk + tyk));
                        rmax = nmax(rmax, nmax(dp, nmax(nmax(dtx, dty), dtz) * a.rG));
                        smax = nmax(smax, nmax(nmax(fabs(pn), fabs(txx)), nmax(fabs(tyy), fabs(txx + tyy))));
                    }
                }
            }
        }
        __syncthreads();
        // ---- S4: new edge stresses: xy at plane f-1, xz / yz at level f-1,
        //      at this thread's own edge points: T = tau_k/(G~ dtau) + S ------
        {
            const int p = f - 1, l = f - 1;
            const bool do_p = p >= k0 && p < k1;
            const bool do_l = l >= k0 && l <= k1 && l >= 0 && l <= nz;
            const int sp = mod2(p), sl = mod2(l), sm = mod2(l - 1);
            const bool inner_l = l >= 1 && l <= nz - 1;
            const bool own_l = l < k1 || (l == nz && last_z);
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int q = tid + NT * u;
                const int la = q % W, lbb = q / W;
                if (!qok[u] || la < 2 || la > TX + 2 || lbb < 2 || lbb > TY + 2) continue;
                const int i = qi[u], j = qj[u];
                const unsigned o = qo[u];
                if (do_p) {
                    R t = R(0);
                    if (INT || (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1)) {
                        R lv = R(0.25) * (s_lam[sp][q - W - 1] + s_lam[sp][q - W] + s_lam[sp][q - 1] + s_lam[sp][q]);
                        const R De = HG ? igt + gxy[u] + a.imus : D;
                        t = (cxy[u] * igt + s_Sxy[q]) * fast_rcp(De + lv);
                    }
                    s_nxy[sp][q] = t;
                    if (la < TX + 2 + hx && lbb < TY + 2 + hy && (INT || (i <= nx && j <= ny))) {
                        st(nxb + F_TXY * fs + sz * p, o, t);
                        if (MODE == MODE_CHECK) rmax = nmax(rmax, fabs(t - cxy[u]) * a.rG);
                    }
                }
                if (do_l) {
                    const long pl = sz * l;
                    // xz edge (i, j) at level l: x-extent nx+1, y-extent ny
                    if (lbb < TY + 2) {
                        R t = R(0);
                        if (inner_l && (INT || (i >= 1 && i <= nx - 1 && j < ny))) {
                            R lv = R(0.25) * (s_lam[sm][q - 1] + s_lam[sm][q] + s_lam[sl][q - 1] + s_lam[sl][q]);
                            const R De = HG ? igt + pgxz[u] + a.imus : D;
                            t = (pcxz[u] * igt + s_Sxz[sl][q]) * fast_rcp(De + lv);
                        }
                        s_nxz[sl][q] = t;
                        if (own_l && la < TX + 2 + hx && (INT || (i <= nx && j < ny))) {
                            st(nxb + F_TXZ * fs + pl, o, t);
                            if (MODE == MODE_CHECK) rmax = nmax(rmax, fabs(t - pcxz[u]) * a.rG);
                        }
                    }
                    // yz edge (i, j) at level l: x-extent nx, y-extent ny+1
                    if (la < TX + 2) {
                        R t = R(0);
                        if (inner_l && (INT || (j >= 1 && j <= ny - 1 && i < nx))) {
                            R lv = R(0.25) * (s_lam[sm][q - W] + s_lam[sm][q] + s_lam[sl][q - W] + s_lam[sl][q]);
                            const R De = HG ? igt + pgyz[u] + a.imus : D;
                            t = (pcyz[u] * igt + s_Syz[sl][q]) * fast_rcp(De + lv);
                        }
                        s_nyz[sl][q] = t;
                        if (own_l && lbb < TY + 2 + hy && (INT || (i < nx && j <= ny))) {
                            st(nxb + F_TYZ * fs + pl, o, t);
                            if (MODE == MODE_CHECK) rmax = nmax(rmax, fabs(t - pcyz[u]) * a.rG);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NQ; ++u) {      // this step's level becomes the previous one
            pcxz[u] = cxz[u];
            pcyz[u] = cyz[u];
        }
        __syncthreads();
        // ---- S5: velocities: vx, vy at plane f-2, vz at level f-1, at this
        //      thread's own plane points; then S1 of step f+1 ----------------
        {
            const int p = f - 2, l = f - 1;
            const bool do_xy = p >= k0 && p < k1;
            const bool do_z = l >= 0 && ((l >= k0 && l < k1) || (l == nz && last_z));
            const int sp = mod2(p), sp1 = mod2(p + 1), sl = mod2(l), sm = mod2(l - 1);
            const bool inner_l = l >= 1 && l <= nz - 1;
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int q = tid + NT * u;
                const int la = q % W, lbb = q / W, i = qi[u], j = qj[u];
                if (!qok[u] || la < 2 || lbb < 2) continue;
                if (do_xy) {
                    const long pp = sz * p;
                    if (la < TX + 2 + hx && lbb < TY + 2 && (INT || (i <= nx && j < ny))) {      // x-face
                        R v = hvx3[u];
                        if (INT || (i >= 1 && i <= nx - 1)) {
                            R Rx = ((s_sxx[sp][q] - s_p[sp][q]) - (s_sxx[sp][q - 1] - s_p[sp][q - 1])) * idx
                                 + (s_nxy[sp][q + W] - s_nxy[sp][q]) * idy + (s_nxz[sp1][q] - s_nxz[sp][q]) * idz;
                            v = v + a.dtrho * Rx;
                            mmax = nmax(mmax, fabs(Rx));
                        }
                        if (MODE != MODE_PHYS) st(nxb + F_VX * fs + pp, qo[u], v);
                        vmax = nmax(vmax, fabs(v));
                    }
                    if (la < TX + 2 && lbb < TY + 2 + hy && (INT || (i < nx && j <= ny))) {      // y-face
                        R v = hvy3[u];
                        if (INT || (j >= 1 && j <= ny - 1)) {
                            R Ry = (s_nxy[sp][q + 1] - s_nxy[sp][q]) * idx
                                 + ((s_syy[sp][q] - s_p[sp][q]) - (s_syy[sp][q - W] - s_p[sp][q - W])) * idy
                                 + (s_nyz[sp1][q] - s_nyz[sp][q]) * idz;
                            v = v + a.dtrho * Ry;
                            mmax = nmax(mmax, fabs(Ry));
                        }
                        if (MODE != MODE_PHYS) st(nxb + F_VY * fs + pp, qo[u], v);
                        vmax = nmax(vmax, fabs(v));
                    }
                }
                if (do_z && la < TX + 2 && lbb < TY + 2 && (INT || (i < nx && j < ny))) {
                    R v = hvz2[u];
                    if (inner_l) {
                        R szu = -(s_sxx[sl][q] + s_syy[sl][q]) - s_p[sl][q];
                        R szd = -(s_sxx[sm][q] + s_syy[sm][q]) - s_p[sm][q];
                        R Rz = (s_nxz[sl][q + 1] - s_nxz[sl][q]) * idx + (s_nyz[sl][q + W] - s_nyz[sl][q]) * idy
                             + (szu - szd) * idz;
                        v = v + a.dtrho * Rz;
                        mmax = nmax(mmax, fabs(Rz));
                    }
                    if (MODE != MODE_PHYS) st(nxb + F_VZ * fs + sz * l, qo[u], v);
                    vmax = nmax(vmax, fabs(v));
                }
            }
        }
        if (f + 1 <= k1 + 1) stage_velocities(f + 1);
        __syncthreads();
    }
    if (MODE != MODE_UPDATE) {
        block_max_to<NT>((double)mmax, a.red + RED_MOM, s_red);
        if (MODE == MODE_CHECK) {
            block_max_to<NT>((double)fmax(rmax, mmax), a.red + RED_RESID, s_red);
            block_max_to<NT>((double)vmax, a.red + RED_VMAX, s_red);
            block_max_to<NT>((double)smax, a.red + RED_SMAX, s_red);
        }
    }
    };
    if (bx >= ts.bx0 && bx < ts.bx1 && by >= ts.by0 && by < ts.by1) body(std::true_type{});
    else body(std::false_type{});
}

// Tile shapes and workgroup sizes (X, Y: column; Z: planes per chunk; T:
// threads; E: waves per SIMD to fit in registers, two FP32 workgroups per
// CU).  FP32 has two shapes, both with 768 threads covering the halo plane
// and every later stage in a single pass (no wave does a second round while
// the others wait at a stage barrier), 72-73 KB of LDS:
//  - 48 x 10 (52 x 14 = 728 plane points): rows of 52 values touch fewer
//    partly used 128-byte lines per value than the 36 of a 32-wide tile
//    (measured at 511^3: 2.14x against 2.35x the algorithmic reads, 4.10
//    against 4.30 ms per sweep; 64 x 7, 56 x 8, 40 x 13 and 48 x 9 slower);
//  - 32 x 16 (36 x 20 = 720 points), which fits grids of 32-cell multiples
//    with fewer workgroups (255^3: 1024 workgroups, two full rounds of 512,
//    0.585 ms, against 1248 and 0.618 ms for 48 x 10).
// FP64: 32 x 16 tiles with 768 threads as well (144-154 KB of LDS, one
// workgroup and three waves per SIMD per CU, the occupancy three 256-thread
// 16 x 8 workgroups had): the wider halo plane cuts the re-read halo (the
// FP64 sweep moves 2.06x its algorithmic bytes on 16 x 8 tiles), 511^3:
// 8.42 against 9.39 ms per sweep (48 x 10: 8.77 ms).
template <int X_, int Y_, int Z_, int T_, int E_> struct Tile {
    static constexpr int X = X_, Y = Y_, Z = Z_, T = T_, E = E_;
};
using TileF_wide = Tile<48, 10, 32, 768, 6>;
using TileF_square = Tile<32, 16, 32, 768, 6>;
using TileD = Tile<32, 16, 32, 768, 3>;

// first and one-past-last tile index along an axis whose tiles lie strictly
// inside with their 2-point halo: 3 <= i0 and i0 + T + 2 <= n
inline void interior_range(int n, int T, int nb, int& b0, int& b1)
{
    b0 = (3 + T - 1) / T;
    b1 = (n - T - 2) >= 0 ? (n - T - 2) / T + 1 : 0;
    if (b1 > nb) b1 = nb;
    if (b1 < b0) b1 = b0;
}

template <typename S>
long tile_count(int nx, int ny, int nz)
{
    return (long)((nx + S::X - 1) / S::X) * ((ny + S::Y - 1) / S::Y) * ((nz + S::Z - 1) / S::Z);
}

template <typename S, typename R, int MODE>
void run_3d(const SweepArgs<R>& a, hipStream_t s)
{
    constexpr int TX = S::X, TY = S::Y, ZC = S::Z, NT = S::T, WPE = S::E;
    TileSet ts;
    ts.nbx = (a.nx + TX - 1) / TX;
    ts.nby = (a.ny + TY - 1) / TY;
    ts.nbz = (a.nz + ZC - 1) / ZC;
    interior_range(a.nx, TX, ts.nbx, ts.bx0, ts.bx1);
    interior_range(a.ny, TY, ts.nby, ts.by0, ts.by1);
    const int nb = ts.nbx * ts.nby * ts.nbz;
    if (a.igdc) k_fused_3d<R, TX, TY, ZC, MODE, NT, WPE, true><<<nb, NT, 0, s>>>(a, ts);
    else k_fused_3d<R, TX, TY, ZC, MODE, NT, WPE, false><<<nb, NT, 0, s>>>(a, ts);
}

// Compute units of the current device (two FP32 workgroups run on each).
int device_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return 256;
    }
    return n;
}

// FP32 tile shape of a grid: rounds of resident workgroups times the cost of
// a round, a 48 x 10 round costing 0.85 of a 32 x 16 one (measured at 511^3:
// 18 rounds in 4.10 ms against 16 in 4.30 ms).
bool wide_tile(int nx, int ny, int nz)
{
    static const int resident = 2 * device_cus();
    const long rw = (tile_count<TileF_wide>(nx, ny, nz) + resident - 1) / resident;
    const long rs = (tile_count<TileF_square>(nx, ny, nz) + resident - 1) / resident;
    return 0.85 * (double)rw <= (double)rs;
}

template <typename R, int MODE>
void run_3d(const SweepArgs<R>& a, hipStream_t s)
{
    if constexpr (sizeof(R) == 8) run_3d<TileD, R, MODE>(a, s);
    else if (wide_tile(a.nx, a.ny, a.nz)) run_3d<TileF_wide, R, MODE>(a, s);
    else run_3d<TileF_square, R, MODE>(a, s);
}


}  // namespace

// Measured on MI355X at 255^3: fused 0.55 ms (FP32) and 1.14 ms (FP64) per
// sweep against 1.57 ms for the three unfused FP64 kernels.
bool fused_preferred(int, bool) { return true; }

template <typename R>
void launch_sweep_fused_3d(const SweepArgs<R>& a, int mode, hipStream_t s)
{
    if (mode == MODE_UPDATE) run_3d<R, MODE_UPDATE>(a, s);
    else if (mode == MODE_CHECK) run_3d<R, MODE_CHECK>(a, s);
    else run_3d<R, MODE_PHYS>(a, s);
}


template void launch_sweep_fused_3d<double>(const SweepArgs<double>&, int, hipStream_t);
template void launch_sweep_fused_3d<float>(const SweepArgs<float>&, int, hipStream_t);

}  // namespace ep
