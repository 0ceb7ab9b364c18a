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
// centre data of plane f), so that HBM latency overlaps the LDS work of the
// current step.  Each thread owns the same plane positions in every step.
template <typename R, int TX, int TY, int ZC, int MODE, int NT, int WPE>
__global__ __attribute__((amdgpu_flat_work_group_size(1, NT), amdgpu_waves_per_eu(WPE)))
void k_fused_3d(SweepArgs<R> a, TileSet ts)
{
    constexpr int W = TX + 4, H = TY + 4, N = W * H;
    constexpr int NQ = (N + NT - 1) / NT;                  // plane positions per thread
    constexpr int CW = TX + 2, CN = (TX + 2) * (TY + 2);   // centre region (1-cell halo)
    constexpr int NR = (CN + NT - 1) / NT;
    __shared__ R s_vx[2][N], s_vy[2][N], s_vz[2][N];
    __shared__ R s_Txy[N], s_Txz[2][N], s_Tyz[2][N];
    __shared__ R s_lam[2][N], s_p[2][N], s_sxx[2][N], s_syy[2][N];
    __shared__ R s_nxy[2][N], s_nxz[2][N], s_nyz[2][N];
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

    // per-thread positions: plane points q (S1, S2) and centre points r (S3)
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
    R fvx[NQ], fvy[NQ], fvz[NQ], fxz[NQ], fxzo[NQ], fyz[NQ], fyzo[NQ], fxy[NQ], fxyo[NQ];
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
            const bool exz = ok && inner && (INT || (i >= 1 && i <= nx - 1 && j >= 0 && j < ny));
            const bool eyz = ok && inner && (INT || (j >= 1 && j <= ny - 1 && i >= 0 && i < nx));
            fxz[u] = exz ? ld(itb + F_TXZ * fs + pg, o) : R(0);
            fxzo[u] = exz ? ld(olb + O_TXZ * fs + pg, o) : R(0);
            fyz[u] = eyz ? ld(itb + F_TYZ * fs + pg, o) : R(0);
            fyzo[u] = eyz ? ld(olb + O_TYZ * fs + pg, o) : R(0);
            const bool exy = ok && pm && (INT || (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1));
            fxy[u] = exy ? ld(itb + F_TXY * fs + pg1, o) : R(0);
            fxyo[u] = exy ? ld(olb + O_TXY * fs + pg1, o) : R(0);
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
    // g (vz) go to LDS and into this thread's register history, from which
    // S5 takes the old velocities of its own points (vx, vy of plane g-2, vz
    // of level g-1 at step g)
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
        }
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            cp[u] = fp[u]; cpo[u] = fpo[u]; csx[u] = fsx[u]; csxo[u] = fsxo[u];
            csy[u] = fsy[u]; csyo[u] = fsyo[u]; cc[u] = fc[u];
        }
        if (f + 1 <= k1 + 1) prefetch(f + 1);

        // ---- S2: shear trials: xz, yz at level f; xy at plane f-1 ----------
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
                    R txz = R(0), tyz = R(0);
                    if (inner_l && (INT || (i >= 1 && i <= nx - 1 && j >= 0 && j < ny))) {
                        R e2 = (s_vx[cm][q] - s_vx[cp3][q]) * idz + (s_vz[sl][q] - s_vz[sl][q - 1]) * idx;
                        txz = cxz[u] * igt + cxzo[u] * igd + e2;
                    }
                    if (inner_l && (INT || (j >= 1 && j <= ny - 1 && i >= 0 && i < nx))) {
                        R e2 = (s_vy[cm][q] - s_vy[cp3][q]) * idz + (s_vz[sl][q] - s_vz[sl][q - W]) * idy;
                        tyz = cyz[u] * igt + cyzo[u] * igd + e2;
                    }
                    s_Txz[sl][q] = txz;
                    s_Tyz[sl][q] = tyz;
                }
                if (do_p) {
                    R t = R(0);
                    if (INT || (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1)) {
                        R e2 = (s_vx[pm][q] - s_vx[pm][q - W]) * idy + (s_vy[pm][q] - s_vy[pm][q - 1]) * idx;
                        t = cxy[u] * igt + cxyo[u] * igd + e2;
                    }
                    s_Txy[q] = t;
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
                R Txx = txk * igt + csxo[u] * igd + R(2) * (dvx - div * R(1.0 / 3.0));
                R Tyy = tyk * igt + csyo[u] * igd + R(2) * (dvy - div * R(1.0 / 3.0));
                R Tzz = -(Txx + Tyy);
                R Txyb = R(0.25) * (s_Txy[q] + s_Txy[q + 1] + s_Txy[q + W] + s_Txy[q + W + 1]);
                R Txzb = R(0.25) * (s_Txz[sc][q] + s_Txz[sc][q + 1] + s_Txz[sc1][q] + s_Txz[sc1][q + 1]);
                R Tyzb = R(0.25) * (s_Tyz[sc][q] + s_Tyz[sc][q + W] + s_Tyz[sc1][q] + s_Tyz[sc1][q + W]);
                R J2 = R(0.5) * (Txx * Txx + Tyy * Tyy + Tzz * Tzz) + Txyb * Txyb + Txzb * Txzb + Tyzb * Tyzb;
                R lam;
                const R ptr = pn;
                R sc_ = return_scale(J2, D, a.invD, pn, cc[u], a.A, a.B, a.Cik, a.vp, lam);
                const bool own = la >= 2 && la < TX + 2 && lbb >= 2 && lbb < TY + 2 && c >= k0 && c < k1;
                if (a.lam_mode != LAM_COMPUTE) {                 // frozen plasticity
                    if (a.lam_mode == LAM_FROZEN) {
                        lam = ld(a.lam + sz * c, ro[u]);
                        sc_ = R(1) / (D + lam);
                        // dilatancy of the held Lambda: lamdot = Lambda sqrt(J2) / (D + Lambda)
                        if (a.Cik != R(0)) pn = ptr + lam * fast_sqrt(J2) * sc_ * a.Cik;
                    } else if (own) {
                        st(a.lam + sz * c, ro[u], lam);
                    }
                }
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
        // ---- S4: new edge stresses: xy at plane f-1, xz / yz at level f-1 ---
        {
            const int p = f - 1;
            if (p >= k0 && p < k1) {
                const int sp = mod2(p);
                constexpr int EW = TX + 1, EN = (TX + 1) * (TY + 1);
                for (int r = tid; r < EN; r += NT) {
                    const int la = 2 + r % EW, lbb = 2 + r / EW;
                    const int q = la + W * lbb;
                    const int i = i0 - 2 + la, j = j0 - 2 + lbb;
                    R t = R(0);
                    if (INT || (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1)) {
                        R lv = R(0.25) * (s_lam[sp][q - W - 1] + s_lam[sp][q - W] + s_lam[sp][q - 1] + s_lam[sp][q]);
                        t = s_Txy[q] * fast_rcp(D + lv);
                    }
                    s_nxy[sp][q] = t;
                    if (la < TX + 2 + hx && lbb < TY + 2 + hy && (INT || (i <= nx && j <= ny))) {
                        const unsigned o = off(i, j);
                        st(nxb + F_TXY * fs + sz * p, o, t);
                        if (MODE == MODE_CHECK) rmax = nmax(rmax, fabs(t - ld(itb + F_TXY * fs + sz * p, o)) * a.rG);
                    }
                }
            }
            const int l = f - 1;
            if (l >= k0 && l <= k1 && l >= 0 && l <= nz) {
                const int sl = mod2(l), sm = mod2(l - 1);
                const bool inner_l = l >= 1 && l <= nz - 1;
                const bool own_l = l < k1 || (l == nz && last_z);
                constexpr int EW = TX + 1, EN = (TX + 1) * (TY + 1);
                for (int r = tid; r < EN; r += NT) {
                    const int la = 2 + r % EW, lbb = 2 + r / EW;
                    const int q = la + W * lbb;
                    const int i = i0 - 2 + la, j = j0 - 2 + lbb;
                    const unsigned o = off(i, j);
                    const long pl = sz * l;
                    // xz edge (i, j) at level l: x-extent nx+1, y-extent ny
                    if (lbb < TY + 2) {
                        R t = R(0);
                        if (inner_l && (INT || (i >= 1 && i <= nx - 1 && j < ny))) {
                            R lv = R(0.25) * (s_lam[sm][q - 1] + s_lam[sm][q] + s_lam[sl][q - 1] + s_lam[sl][q]);
                            t = s_Txz[sl][q] * fast_rcp(D + lv);
                        }
                        s_nxz[sl][q] = t;
                        if (own_l && la < TX + 2 + hx && (INT || (i <= nx && j < ny))) {
                            st(nxb + F_TXZ * fs + pl, o, t);
                            if (MODE == MODE_CHECK) rmax = nmax(rmax, fabs(t - ld(itb + F_TXZ * fs + pl, o)) * a.rG);
                        }
                    }
                    // yz edge (i, j) at level l: x-extent nx, y-extent ny+1
                    if (la < TX + 2) {
                        R t = R(0);
                        if (inner_l && (INT || (j >= 1 && j <= ny - 1 && i < nx))) {
                            R lv = R(0.25) * (s_lam[sm][q - W] + s_lam[sm][q] + s_lam[sl][q - W] + s_lam[sl][q]);
                            t = s_Tyz[sl][q] * fast_rcp(D + lv);
                        }
                        s_nyz[sl][q] = t;
                        if (own_l && lbb < TY + 2 + hy && (INT || (i < nx && j <= ny))) {
                            st(nxb + F_TYZ * fs + pl, o, t);
                            if (MODE == MODE_CHECK) rmax = nmax(rmax, fabs(t - ld(itb + F_TYZ * fs + pl, o)) * a.rG);
                        }
                    }
                }
            }
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

// Tile shapes and workgroup sizes.  FP32: 768 threads cover the 36 x 20
// halo plane (720 points) and every later stage in a single pass, so no
// wave does a second round while the others wait at the stage barrier.
template <typename R> struct Tile3;
// E: waves per SIMD to fit in registers (two FP32 workgroups per CU).
template <> struct Tile3<float> { static constexpr int X = 32, Y = 16, Z = 32, T = 768, E = 6; };
// FP64: 16 x 8 tiles (52 KB of LDS, three workgroups per CU).
template <> struct Tile3<double> { static constexpr int X = 16, Y = 8, Z = 32, T = 256, E = 3; };

// first and one-past-last tile index along an axis whose tiles lie strictly
// inside with their 2-point halo: 3 <= i0 and i0 + T + 2 <= n
inline void interior_range(int n, int T, int nb, int& b0, int& b1)
{
    b0 = (3 + T - 1) / T;
    b1 = (n - T - 2) >= 0 ? (n - T - 2) / T + 1 : 0;
    if (b1 > nb) b1 = nb;
    if (b1 < b0) b1 = b0;
}

template <typename R, int MODE>
void run_3d(const SweepArgs<R>& a, hipStream_t s)
{
    constexpr int TX = Tile3<R>::X, TY = Tile3<R>::Y, ZC = Tile3<R>::Z, NT = Tile3<R>::T, WPE = Tile3<R>::E;
    TileSet ts;
    ts.nbx = (a.nx + TX - 1) / TX;
    ts.nby = (a.ny + TY - 1) / TY;
    ts.nbz = (a.nz + ZC - 1) / ZC;
    interior_range(a.nx, TX, ts.nbx, ts.bx0, ts.bx1);
    interior_range(a.ny, TY, ts.nby, ts.by0, ts.by1);
    k_fused_3d<R, TX, TY, ZC, MODE, NT, WPE><<<ts.nbx * ts.nby * ts.nbz, NT, 0, s>>>(a, ts);
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
