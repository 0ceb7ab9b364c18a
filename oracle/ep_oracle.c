/*
 * CPU oracle for the per-increment elasto-plastic pseudo-transient solve.
 *
 * TEST INFRASTRUCTURE ONLY (see ep_oracle.h).  Plain FP64, unfused full-grid
 * loops, every intermediate in its own array, Jacobi order.  Built with
 * -ffp-contract=off.
 *
 * What it computes, per load increment (paper, "Accelerated pseudo-transient
 * method" and "Return mapping algorithm for plasticity"):
 *
 *   pseudo-transient momentum   rho~ dv/dt~ = div(tau - p I)
 *   pseudo-transient pressure   (1/K~) dp/dt~ + (p - p^)/(K dt) = -div v
 *   pseudo-transient deviator   (1/2G~) dtau/dt~ + (tau - tau^)/(2G dt)
 *                               + tau/(2 mu_s) = -lambda dQ/dsigma + e'(v)
 *
 * discretised on the conservative staggered grid (Discretization section),
 * backward Euler in pseudo-time for p and tau, explicit for v.  With
 * Q = sqrt(J2) (psi = 0) the plastic term is Lambda * tau with
 * Lambda = lambda_dot / tauII, so the stress update is tau = T / (D + Lambda)
 * with T = tau_old/(G~dtau) + S, S = tau^/(G dt) + 2 e' the physical trial,
 * D = 1/(G~dtau) + Dp, Dp = 1/(G dt) + 1/mu_s.  Lambda is set at cell
 * centres by the radial return of the physical trial S (its shear
 * components averaged from the four shear points) against the
 * Drucker-Prager bound A p + B c, so that the fixed point tau = S/(Dp + Lambda)
 * is the solution of the increment's equations with the pseudo-time terms
 * removed (the paper: the quasi-static solution is the attractor of the
 * pseudo-time iteration; Re and r only set its convergence).  The iteration
 * blends that Lambda with the return of the pseudo-time trial (centre_return),
 * which changes the path, not the fixed point.  Vertices / edges take the
 * mean Lambda of their four centres.
 *
 * Residual (Convergence study section): the L-inf momentum residual
 * max|div(tau) - grad p| over interior faces, combined (max) with the
 * pressure and deviator pseudo-rates expressed as the distance of p and tau
 * from their local fixed point per unit length,
 *   |p^{k+1}-p^k| K dt / (K~dtau L)  and  |tau^{k+1}-tau^k| eta / (G~dtau L),
 * so that a homogeneous state whose stresses are still relaxing in pseudo-time
 * is not taken as converged.  When this is at most
 * tol * max(R_ref, 2 G max|erate| dt / L) at a check, the physical stresses of
 * the current velocities (pseudo-time terms removed) are evaluated; their
 * momentum residual must meet the same bound (the certificate), and they are
 * the accepted stresses.  R_ref is the momentum residual of the physical
 * stresses of the plain guess (the previous increment's velocities); those
 * stresses are also the pseudo-time starting point of p and tau, and a
 * starting state that already meets the bound is accepted as it is.
 *
 * PT parameters (equations for rho~, G~, K~, Vp and the optimal Re, r): the
 * viscosity in rho~ is the visco-elastic eta = 1/(1/(G dt) + 1/mu_s),
 * L = max extent, V~ dtau = cfl * min spacing.  Then
 *   G~dtau = Re eta cfl h / (L (r + 4/3)),  K~dtau = r G~dtau,
 *   dtau/rho~ = cfl h L / (Re eta).
 *
 * Options, each documented where it is computed: the dilatant return
 * (psi > 0) and the consistency-regularised return (eta_vp > 0) in
 * plastic_lambda; the incompressible limit (K = +inf) in the pressure
 * update and p_res_visc; frozen plasticity (freeze_iter) in the sweeps; the
 * objective stress update (objective) in objective2d/3d; a per-cell shear
 * modulus in orc_set_shear_modulus, igd_vertex and igd_edge; loading schedules in
 * orc_set_strain_rate.
 */
#include "ep_oracle.h"

#include <float.h>
#include <stdio.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI_D 3.14159265358979323846

struct orc_state {
    orc_params prm;
    int nx, ny, nz, ndim;
    double dx, dy, dz;
    double gdtau, kdtau, dtrho, eta, A, B, h, L, inv_mus;
    double C;                 /* plastic potential Q = sqrt(J2) - C p (dilatancy) */
    /* state */
    double *vx, *vy, *vz;
    double *p, *txx, *tyy, *tzz, *txy, *txz, *tyz;
    double *p_old, *txx_old, *tyy_old, *tzz_old, *txy_old, *txz_old, *tyz_old;
    double *coh;
    double *igdc;             /* per-cell 1/(G dt) (NULL: uniform G = prm.shear) */
    /* accumulators and diagnostics */
    double *ux, *uy, *uz;
    double *exx, *eyy, *ezz, *exy, *exz, *eyz;
    double *eps_p;
    double *lam, *tII, *yld, *lamdot;
    /* scratch: new values, trial stresses, divergence */
    double *vxn, *vyn, *vzn;
    double *pn, *txxn, *tyyn, *tzzn, *txyn, *txzn, *tyzn;
    double *Txy, *Txz, *Tyz, *dv;
    double *Sxy, *Sxz, *Syz;  /* physical shear trials (pseudo-time terms removed) */
    double *vx0, *vy0, *vz0;  /* velocities at the start of the increment */
    /* bookkeeping of the last sweep */
    double vmax;
    long long n_yield;
    double *hist; int hist_cap, hist_len;
    /* frozen plasticity: 0 off; 1 the next sweep stores its centre Lambda;
     * 2 sweeps use the stored Lambda instead of the return mapping */
    int freeze;
    double *lamf;
    int late;                 /* the iteration's return uses pt_blend_late */
};

/* ---------------------------------------------------------------- sizes */
static long n_cells(const orc_state* s) { return (long)s->nx * s->ny * (s->ndim == 3 ? s->nz : 1); }
static long n_vx(const orc_state* s) { return (long)(s->nx + 1) * s->ny * (s->ndim == 3 ? s->nz : 1); }
static long n_vy(const orc_state* s) { return (long)s->nx * (s->ny + 1) * (s->ndim == 3 ? s->nz : 1); }
static long n_vz(const orc_state* s) { return s->ndim == 3 ? (long)s->nx * s->ny * (s->nz + 1) : 0; }
static long n_xy(const orc_state* s) { return (long)(s->nx + 1) * (s->ny + 1) * (s->ndim == 3 ? s->nz : 1); }
static long n_xz(const orc_state* s) { return s->ndim == 3 ? (long)(s->nx + 1) * s->ny * (s->nz + 1) : 0; }
static long n_yz(const orc_state* s) { return s->ndim == 3 ? (long)s->nx * (s->ny + 1) * (s->nz + 1) : 0; }

/* ------------------------------------------------------------- indexing */
/* 2D */
#define C2(i, j)  ((i) + nx * (j))
#define VX2(i, j) ((i) + (nx + 1) * (j))
#define VY2(i, j) ((i) + nx * (j))
#define XY2(i, j) ((i) + (nx + 1) * (j))
/* 3D */
#define C3(i, j, k)  ((i) + nx * ((j) + ny * (k)))
#define VX3(i, j, k) ((i) + (nx + 1) * ((j) + ny * (k)))
#define VY3(i, j, k) ((i) + nx * ((j) + (ny + 1) * (k)))
#define VZ3(i, j, k) ((i) + nx * ((j) + ny * (k)))
#define XY3(i, j, k) ((i) + (nx + 1) * ((j) + (ny + 1) * (k)))
#define XZ3(i, j, k) ((i) + (nx + 1) * ((j) + ny * (k)))
#define YZ3(i, j, k) ((i) + nx * ((j) + (ny + 1) * (k)))

static int imax(int a, int b) { return a > b ? a : b; }

static double* zalloc(long n) { return n > 0 ? (double*)calloc((size_t)n, sizeof(double)) : NULL; }

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Drucker-Prager constants (Plasticity section): 2D A = sin phi, B = cos phi;
 * 3D A = 6 sin phi / (sqrt3 (3 - sin phi)), B = 6 cos phi / (sqrt3 (3 - sin phi)). */
static void dp_constants(int ndim, double phi_deg, double* A, double* B)
{
    double ph = phi_deg * PI_D / 180.0;
    if (ndim == 2) {
        *A = sin(ph);
        *B = cos(ph);
    } else {
        double den = sqrt(3.0) * (3.0 - sin(ph));
        *A = 6.0 * sin(ph) / den;
        *B = 6.0 * cos(ph) / den;
    }
}

static void set_wall_velocities(orc_state* s)
{
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const double xw = 0.5 * s->prm.lx, yw = 0.5 * s->prm.ly, zw = 0.5 * s->prm.lz;
    const double ax = s->prm.erate[0], ay = s->prm.erate[1], az = s->prm.erate[2];
    if (s->ndim == 2) {
        for (int j = 0; j < ny; ++j) { s->vx[VX2(0, j)] = -ax * xw; s->vx[VX2(nx, j)] = ax * xw; }
        for (int i = 0; i < nx; ++i) { s->vy[VY2(i, 0)] = -ay * yw; s->vy[VY2(i, ny)] = ay * yw; }
    } else {
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j) { s->vx[VX3(0, j, k)] = -ax * xw; s->vx[VX3(nx, j, k)] = ax * xw; }
        for (int k = 0; k < nz; ++k)
            for (int i = 0; i < nx; ++i) { s->vy[VY3(i, 0, k)] = -ay * yw; s->vy[VY3(i, ny, k)] = ay * yw; }
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) { s->vz[VZ3(i, j, 0)] = -az * zw; s->vz[VZ3(i, j, nz)] = az * zw; }
    }
}

orc_state* orc_create(const orc_params* prm, const double* cohesion)
{
    if (!prm || (prm->ndim != 2 && prm->ndim != 3)) return NULL;
    if (prm->nx < 3 || prm->ny < 3 || (prm->ndim == 3 && prm->nz < 3)) return NULL;
    if (!(prm->bulk > 0) || !(prm->shear > 0) || !(prm->dt > 0) || !(prm->tol > 0)) return NULL;
    if (!(prm->psi_deg >= 0.0) || prm->psi_deg > prm->phi_deg) return NULL;
    if (!(prm->visc > 0)) return NULL;
    if (!(prm->eta_vp >= 0.0) || isinf(prm->eta_vp)) return NULL;
    if (!(prm->pt_blend >= 0.0 && prm->pt_blend <= 1.0)) return NULL;
    if (!(prm->pt_blend_late >= 0.0 && prm->pt_blend_late <= 1.0)) return NULL;
    orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
    s->prm = *prm;
    s->ndim = prm->ndim;
    s->nx = prm->nx; s->ny = prm->ny; s->nz = prm->ndim == 3 ? prm->nz : 1;
    s->dx = prm->lx / prm->nx;
    s->dy = prm->ly / prm->ny;
    s->dz = prm->ndim == 3 ? prm->lz / prm->nz : 1.0;
    s->inv_mus = isinf(prm->visc) ? 0.0 : 1.0 / prm->visc;
    dp_constants(s->ndim, prm->phi_deg, &s->A, &s->B);
    {   /* C of the plastic potential: the friction-angle expression of A with psi */
        double dummy;
        dp_constants(s->ndim, prm->psi_deg, &s->C, &dummy);
    }

    double re = prm->re > 0 ? prm->re : 3.0 * sqrt(10.0) * PI_D / 2.0;
    double cfl = prm->cfl > 0 ? prm->cfl : 0.9 / sqrt((double)s->ndim);
    double r = prm->r > 0 ? prm->r : 0.5;
    s->eta = 1.0 / (1.0 / (prm->shear * prm->dt) + s->inv_mus);
    s->h = fmin(s->dx, s->dy);
    s->L = fmax(prm->lx, prm->ly);
    if (s->ndim == 3) { s->h = fmin(s->h, s->dz); s->L = fmax(s->L, prm->lz); }
    s->gdtau = re * s->eta * cfl * s->h / (s->L * (r + 4.0 / 3.0));
    s->kdtau = r * s->gdtau;
    s->dtrho = cfl * s->h * s->L / (re * s->eta);
    if (s->prm.n_check <= 0) s->prm.n_check = s->ndim == 3 ? 10 : 100;

    long nc = n_cells(s);
    s->vx = zalloc(n_vx(s)); s->vy = zalloc(n_vy(s)); s->vz = zalloc(n_vz(s));
    s->vxn = zalloc(n_vx(s)); s->vyn = zalloc(n_vy(s)); s->vzn = zalloc(n_vz(s));
    s->vx0 = zalloc(n_vx(s)); s->vy0 = zalloc(n_vy(s)); s->vz0 = zalloc(n_vz(s));
    s->ux = zalloc(n_vx(s)); s->uy = zalloc(n_vy(s)); s->uz = zalloc(n_vz(s));
    s->p = zalloc(nc); s->txx = zalloc(nc); s->tyy = zalloc(nc); s->tzz = zalloc(nc);
    s->p_old = zalloc(nc); s->txx_old = zalloc(nc); s->tyy_old = zalloc(nc); s->tzz_old = zalloc(nc);
    s->pn = zalloc(nc); s->txxn = zalloc(nc); s->tyyn = zalloc(nc); s->tzzn = zalloc(nc);
    s->coh = zalloc(nc); s->dv = zalloc(nc);
    s->exx = zalloc(nc); s->eyy = zalloc(nc); s->ezz = zalloc(nc); s->eps_p = zalloc(nc);
    s->lam = zalloc(nc); s->tII = zalloc(nc); s->yld = zalloc(nc); s->lamdot = zalloc(nc);
    s->lamf = zalloc(nc);
    s->txy = zalloc(n_xy(s)); s->txy_old = zalloc(n_xy(s)); s->txyn = zalloc(n_xy(s));
    s->Txy = zalloc(n_xy(s)); s->exy = zalloc(n_xy(s)); s->Sxy = zalloc(n_xy(s));
    s->txz = zalloc(n_xz(s)); s->txz_old = zalloc(n_xz(s)); s->txzn = zalloc(n_xz(s));
    s->Txz = zalloc(n_xz(s)); s->exz = zalloc(n_xz(s)); s->Sxz = zalloc(n_xz(s));
    s->tyz = zalloc(n_yz(s)); s->tyz_old = zalloc(n_yz(s)); s->tyzn = zalloc(n_yz(s));
    s->Tyz = zalloc(n_yz(s)); s->eyz = zalloc(n_yz(s)); s->Syz = zalloc(n_yz(s));

    if (cohesion) memcpy(s->coh, cohesion, (size_t)nc * sizeof(double));

    /* initial state: p = tau = 0, v = background pure-shear field */
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const double ax = prm->erate[0], ay = prm->erate[1], az = prm->erate[2];
    if (s->ndim == 2) {
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) s->vx[VX2(i, j)] = ax * (-0.5 * prm->lx + i * s->dx);
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) s->vy[VY2(i, j)] = ay * (-0.5 * prm->ly + j * s->dy);
    } else {
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i <= nx; ++i) s->vx[VX3(i, j, k)] = ax * (-0.5 * prm->lx + i * s->dx);
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i < nx; ++i) s->vy[VY3(i, j, k)] = ay * (-0.5 * prm->ly + j * s->dy);
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) s->vz[VZ3(i, j, k)] = az * (-0.5 * prm->lz + k * s->dz);
    }
    return s;
}

void orc_free(orc_state* s)
{
    if (!s) return;
    double** all[] = {
        &s->vx, &s->vy, &s->vz, &s->vxn, &s->vyn, &s->vzn, &s->vx0, &s->vy0, &s->vz0,
        &s->ux, &s->uy, &s->uz, &s->p, &s->txx, &s->tyy, &s->tzz,
        &s->p_old, &s->txx_old, &s->tyy_old, &s->tzz_old, &s->pn, &s->txxn, &s->tyyn, &s->tzzn,
        &s->coh, &s->igdc, &s->dv, &s->exx, &s->eyy, &s->ezz, &s->eps_p, &s->lam, &s->tII, &s->yld, &s->lamdot, &s->lamf,
        &s->txy, &s->txy_old, &s->txyn, &s->Txy, &s->exy,
        &s->txz, &s->txz_old, &s->txzn, &s->Txz, &s->exz,
        &s->tyz, &s->tyz_old, &s->tyzn, &s->Tyz, &s->eyz,
        &s->Sxy, &s->Sxz, &s->Syz,
    };
    for (size_t q = 0; q < sizeof(all) / sizeof(all[0]); ++q) free(*all[q]);
    free(s);
}

static double* field_ptr(const orc_state* s, int f, long* n)
{
    switch (f) {
    case ORC_VX: *n = n_vx(s); return s->vx;
    case ORC_VY: *n = n_vy(s); return s->vy;
    case ORC_VZ: *n = n_vz(s); return s->vz;
    case ORC_P: *n = n_cells(s); return s->p;
    case ORC_TXX: *n = n_cells(s); return s->txx;
    case ORC_TYY: *n = n_cells(s); return s->tyy;
    case ORC_TZZ: *n = s->ndim == 3 ? n_cells(s) : 0; return s->tzz;
    case ORC_TXY: *n = n_xy(s); return s->txy;
    case ORC_TXZ: *n = n_xz(s); return s->txz;
    case ORC_TYZ: *n = n_yz(s); return s->tyz;
    case ORC_P_OLD: *n = n_cells(s); return s->p_old;
    case ORC_TXX_OLD: *n = n_cells(s); return s->txx_old;
    case ORC_TYY_OLD: *n = n_cells(s); return s->tyy_old;
    case ORC_TZZ_OLD: *n = s->ndim == 3 ? n_cells(s) : 0; return s->tzz_old;
    case ORC_TXY_OLD: *n = n_xy(s); return s->txy_old;
    case ORC_TXZ_OLD: *n = n_xz(s); return s->txz_old;
    case ORC_TYZ_OLD: *n = n_yz(s); return s->tyz_old;
    case ORC_UX: *n = n_vx(s); return s->ux;
    case ORC_UY: *n = n_vy(s); return s->uy;
    case ORC_UZ: *n = n_vz(s); return s->uz;
    case ORC_EXX: *n = n_cells(s); return s->exx;
    case ORC_EYY: *n = n_cells(s); return s->eyy;
    case ORC_EZZ: *n = s->ndim == 3 ? n_cells(s) : 0; return s->ezz;
    case ORC_EXY: *n = n_xy(s); return s->exy;
    case ORC_EXZ: *n = n_xz(s); return s->exz;
    case ORC_EYZ: *n = n_yz(s); return s->eyz;
    case ORC_EPS_P: *n = n_cells(s); return s->eps_p;
    case ORC_COHESION: *n = n_cells(s); return s->coh;
    case ORC_LAMBDA: *n = n_cells(s); return s->lamdot;
    case ORC_TAU_II: *n = n_cells(s); return s->tII;
    case ORC_YIELD: *n = n_cells(s); return s->yld;
    case ORC_LAMBDA_FROZEN: *n = n_cells(s); return s->lamf;
    default: *n = -1; return NULL;
    }
}

long orc_field_size(const orc_state* s, int field)
{
    long n; field_ptr(s, field, &n); return n;
}

int orc_get(const orc_state* s, int field, double* out)
{
    long n; double* p = field_ptr(s, field, &n);
    if (n < 0) return -1;
    if (n > 0) memcpy(out, p, (size_t)n * sizeof(double));
    return 0;
}

int orc_set(orc_state* s, int field, const double* in)
{
    long n; double* p = field_ptr(s, field, &n);
    if (n < 0) return -1;
    if (n > 0) memcpy(p, in, (size_t)n * sizeof(double));
    return 0;
}

void orc_scalars(const orc_state* s, double out[8])
{
    out[0] = s->gdtau; out[1] = s->kdtau; out[2] = s->dtrho; out[3] = s->eta;
    out[4] = s->A; out[5] = s->B; out[6] = s->h; out[7] = s->L;
}

void orc_history(orc_state* s, double* buf, int cap) { s->hist = buf; s->hist_cap = cap; s->hist_len = 0; }
int orc_history_len(const orc_state* s) { return s->hist_len; }

/* Plastic rate of a yielding centre (called only when the trial stress lies
 * outside the bound).
 * Dilatancy (psi > 0; Plasticity section, potential Q = sqrt(J2) - C p): the
 * plastic strain rate lambda_dot dQ/dsigma has the volumetric part
 * lambda_dot C, which enters the pressure equation like a source:
 *     p = p_tr + lambda_dot C k,
 * with p_tr the pressure update without it and k its compliance
 * (1 / (1/(K~dtau) + 1/(K dt)); K dt when the pseudo-time terms are removed).
 * Regularisation (eta_vp > 0; the visco-plastic strain rate of the
 * constitutive section, with the consistency viscosity of the literature the
 * introduction cites): the consistency condition becomes
 * tauII = max(0, A p + B c) + eta_vp lambda_dot, a viscous overstress.
 * With a deviator of compliance D, tauII D + lambda_dot = sqrt(J2) of the
 * trial, so lambda_dot solves
 *     D (max(0, A p + B c) + eta_vp lambda_dot) + lambda_dot = sqrt(J2),
 * p = p_tr + lambda_dot C k, whose left side increases with lambda_dot and is
 * linear on either side of the apex.  The root of the piece with a
 * non-negative bound,
 *     lambda_dot = (sqrt(J2) - D (A p_tr + B c)) / (1 + D A C k + D eta_vp),
 * is the solution when its bound is non-negative; otherwise the solution lies
 * on the apex piece, lambda_dot = sqrt(J2) / (1 + D eta_vp).  With C = 0 and
 * eta_vp = 0 this is the radial return lambda_dot = sqrt(J2) - D Y.
 * Returns Lambda = lambda_dot / tauII (+inf when tauII = 0); *p gets the
 * corrected pressure, *tII the returned tauII, *Y the bound. */
static double plastic_lambda(double sq, double D, double p_tr, double c, double A, double B, double C,
                             double k, double eta_vp, double* p, double* tII_ret, double* Y_out, double* lamdot)
{
    double ld = (sq - D * (A * p_tr + B * c)) / (1.0 + D * A * C * k + D * eta_vp);
    if (A * (p_tr + ld * C * k) + B * c < 0.0) ld = sq / (1.0 + D * eta_vp);
    *p = p_tr + ld * C * k;
    double Y = A * (*p) + B * c;
    if (Y < 0.0) Y = 0.0;
    double tII = Y + eta_vp * ld;
    *lamdot = ld;
    *tII_ret = tII;
    *Y_out = Y;
    return tII > 0.0 ? ld / tII : INFINITY;
}

/* Return mapping at a centre (Return mapping section; readings on the
 * staggered grid, the Lambda form): the deviatoric update of the iteration is
 * tau = T / (D + Lambda), T = tau_k/(G~dtau) + S, S = tau^/(G dt) + 2 e',
 * D = 1/(G~dtau) + Dp, Dp = 1/(G dt) + 1/mu_s, and a shear point takes the
 * mean Lambda of its four centres.
 *
 * The plastic multiplier is set by the physical trial S, in which the
 * pseudo-time terms are absent: with the shear components of S averaged from
 * the four (2D) or four-per-plane (3D) shear points, Lambda_phys is the
 * radial return of S against the bound, sqrt(J2(S)) = (Dp + Lambda) tauII,
 * tauII = max(0, A p + B c) (+ eta_vp lambda_dot).  At the fixed point of
 * the iteration tau = S / (Dp + Lambda), so the converged state is the
 * solution of the increment's equations with the pseudo-time terms removed,
 * whatever the pseudo-time steps are (the paper's Re and r only set the
 * convergence).
 *
 * The iteration uses Lambda = Lambda_phys + blend (Lambda_pt - Lambda_phys),
 * blend = pt_blend until the first check at or after 16 max(nx, ny, nz)
 * iterations of an increment and pt_blend_late afterwards,
 * Lambda_pt being the radial return of the pseudo-time trial: the centre's
 * normal T with the averaged shear trial scaled to the pseudo-time form it
 * has at the fixed point, f S_shear, f = (D + Lambda_phys)/(Dp + Lambda_phys),
 * against D.  At the fixed point Lambda_pt = Lambda_phys, so the blend only
 * changes the path (blend = 0: the physical return alone); the pressure takes
 * the same blend of the two dilatant corrections.
 *
 * nT2 = (1/2) sum of the squared normal components of T, nS2 the same of S,
 * sh2 = sum of the squared averaged shear components of S.  Returns Lambda
 * (0 elastic, +inf at the apex); *p the pressure; the diagnostics (*tII, *Y,
 * *lamdot) are those of the physical return. */
static double centre_return(const orc_state* s, double nT2, double nS2, double sh2, double Dp, double D,
                            double k, double p_tr, double c, double* p, double* tII, double* Y, double* lamdot)
{
    const double A = s->A, B = s->B, C = s->C, vp = s->prm.eta_vp;
    double Y0 = A * p_tr + B * c;
    if (Y0 < 0.0) Y0 = 0.0;                  /* apex: nothing can be carried */
    const double sqS = sqrt(nS2 + sh2);
    *p = p_tr;
    *Y = Y0;
    *lamdot = 0.0;
    if (!(sqS / Dp > Y0)) {                  /* elastic: yield only above the bound */
        *tII = sqS / Dp;
        return 0.0;
    }
    double lam = plastic_lambda(sqS, Dp, p_tr, c, A, B, C, k, vp, p, tII, Y, lamdot);
    const double blend = s->late ? s->prm.pt_blend_late : s->prm.pt_blend;
    if (blend == 0.0 || D == Dp || isinf(lam)) return lam;
    /* pseudo-time trial */
    const double f = (D + lam) / (Dp + lam);
    const double sqT = sqrt(nT2 + f * f * sh2);
    double lam_t = 0.0, p_t = p_tr;
    if (sqT / D > Y0) {
        double t1, t2, t3;
        lam_t = plastic_lambda(sqT, D, p_tr, c, A, B, C, k, vp, &p_t, &t1, &t2, &t3);
    }
    if (isinf(lam_t)) return lam;
    *p = *p + blend * (p_t - *p);
    return lam + blend * (lam_t - lam);
}

static double p_res_visc(const orc_state* s) { return isinf(s->prm.bulk) ? s->eta : s->prm.bulk * s->prm.dt; }

/* Compliance 1/(G dt) of the interior vertex (i, j): the uniform value, or the
 * mean over its four cells when G is given per cell. */
static double igd_vertex(const orc_state* s, int i, int j, double igd)
{
    if (!s->igdc) return igd;
    const int nx = s->nx;
    return 0.25 * (s->igdc[(i - 1) + (long)nx * (j - 1)] + s->igdc[i + (long)nx * (j - 1)]
                 + s->igdc[(i - 1) + (long)nx * j] + s->igdc[i + (long)nx * j]);
}

static double sweep2d(orc_state* s, int mode)
{
    const int physical = mode == 1;
    const int nx = s->nx, ny = s->ny;
    const double dx = s->dx, dy = s->dy;
    const double igt = physical ? 0.0 : 1.0 / s->gdtau;
    /* incompressible limit (K = +inf): the pressure has no local physical
     * law, so the physical evaluation keeps its pseudo-time term (a reading) */
    const double ikt = (physical && !isinf(s->prm.bulk)) ? 0.0 : 1.0 / s->kdtau;
    const double igd = 1.0 / (s->prm.shear * s->prm.dt);
    const double ikd = 1.0 / (s->prm.bulk * s->prm.dt);
    const double kk = 1.0 / (ikt + ikd);      /* pressure compliance of one update */

    /* 1. divergence and pressure at centres */
#pragma omp parallel for
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double div = (s->vx[VX2(i + 1, j)] - s->vx[VX2(i, j)]) / dx
                       + (s->vy[VY2(i, j + 1)] - s->vy[VY2(i, j)]) / dy;
            s->dv[C2(i, j)] = div;
            s->pn[C2(i, j)] = (s->p[C2(i, j)] * ikt + s->p_old[C2(i, j)] * ikd - div) / (ikt + ikd);
        }
    /* 2. shear trial at vertices (zero on the walls: free slip) */
#pragma omp parallel for
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            if (i == 0 || i == nx || j == 0 || j == ny) { s->Txy[XY2(i, j)] = 0.0; continue; }
            double exy = 0.5 * ((s->vx[VX2(i, j)] - s->vx[VX2(i, j - 1)]) / dy
                              + (s->vy[VY2(i, j)] - s->vy[VY2(i - 1, j)]) / dx);
            s->Sxy[XY2(i, j)] = s->txy_old[XY2(i, j)] * igd_vertex(s, i, j, igd) + 2.0 * exy;
            s->Txy[XY2(i, j)] = s->txy[XY2(i, j)] * igt + s->Sxy[XY2(i, j)];
        }
    /* 3. normal trial and return mapping at centres */
    long long ny_count = 0;
    double dpm = 0.0, dtm = 0.0;
#pragma omp parallel for reduction(+ : ny_count) reduction(max : dpm, dtm)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const long c = C2(i, j);
            double div = s->dv[c];
            double exx = (s->vx[VX2(i + 1, j)] - s->vx[VX2(i, j)]) / dx - div / 3.0;
            double eyy = (s->vy[VY2(i, j + 1)] - s->vy[VY2(i, j)]) / dy - div / 3.0;
            const double igdc = s->igdc ? s->igdc[c] : igd;
            const double Dp = igdc + s->inv_mus;     /* physical compliance 1/eta */
            const double D = igt + Dp;
            double Sxx = s->txx_old[c] * igdc + 2.0 * exx;
            double Syy = s->tyy_old[c] * igdc + 2.0 * eyy;
            double Txx = s->txx[c] * igt + Sxx;
            double Tyy = s->tyy[c] * igt + Syy;
            double Sb = 0.25 * (s->Sxy[XY2(i, j)] + s->Sxy[XY2(i + 1, j)]
                              + s->Sxy[XY2(i, j + 1)] + s->Sxy[XY2(i + 1, j + 1)]);
            double J2 = 0.5 * (Sxx * Sxx + Syy * Syy) + Sb * Sb;   /* J2 of the physical trial */
            double tret, Y, ld;
            const double ptr = s->pn[c];
            double lam = centre_return(s, 0.5 * (Txx * Txx + Tyy * Tyy), 0.5 * (Sxx * Sxx + Syy * Syy), Sb * Sb,
                                       Dp, D, kk, ptr, s->coh[c], &s->pn[c], &tret, &Y, &ld);
            s->lamdot[c] = ld;
            s->tII[c] = tret;
            s->yld[c] = Y;
            if (lam > 0.0) ny_count++;
            if (mode == 0 && s->freeze == 1) s->lamf[c] = lam;
            if (s->freeze == 2) {   /* held Lambda, also in the certificate */
                lam = s->lamf[c];
                /* held Lambda: lambda_dot = Lambda tauII = Lambda sqrt(J2) / (D + Lambda) */
                if (s->C > 0.0) s->pn[c] = ptr + lam * sqrt(J2) / (Dp + lam) * s->C * kk;
            }
            s->lam[c] = lam;
            s->txxn[c] = Txx / (D + lam);
            s->tyyn[c] = Tyy / (D + lam);
            dpm = fmax(dpm, fabs(s->pn[c] - s->p[c]));
            dtm = fmax(dtm, fmax(fabs(s->txxn[c] - s->txx[c]), fabs(s->tyyn[c] - s->tyy[c])));
        }
    s->n_yield = ny_count;
    /* 4. vertices: Lambda averaged from the four adjacent centres */
#pragma omp parallel for reduction(max : dtm)
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            if (i == 0 || i == nx || j == 0 || j == ny) { s->txyn[XY2(i, j)] = 0.0; continue; }
            double lv = 0.25 * (s->lam[C2(i - 1, j - 1)] + s->lam[C2(i, j - 1)]
                              + s->lam[C2(i - 1, j)] + s->lam[C2(i, j)]);
            s->txyn[XY2(i, j)] = s->Txy[XY2(i, j)] / (igt + igd_vertex(s, i, j, igd) + s->inv_mus + lv);
            dtm = fmax(dtm, fabs(s->txyn[XY2(i, j)] - s->txy[XY2(i, j)]));
        }
    /* 5. momentum residual and velocity update at interior faces */
    double rmax = 0.0, vmax = 0.0;
    long nbad = 0;
#pragma omp parallel for reduction(max : rmax, vmax) reduction(+ : nbad)
    for (int j = 0; j < ny; ++j)
        for (int i = 1; i < nx; ++i) {
            double sR = s->txxn[C2(i, j)] - s->pn[C2(i, j)];
            double sL = s->txxn[C2(i - 1, j)] - s->pn[C2(i - 1, j)];
            double R = (sR - sL) / dx + (s->txyn[XY2(i, j + 1)] - s->txyn[XY2(i, j)]) / dy;
            double vn = s->vx[VX2(i, j)] + s->dtrho * R;
            s->vxn[VX2(i, j)] = vn;
            rmax = fmax(rmax, fabs(R));
            if (!(fabs(R) <= DBL_MAX)) nbad++;
            vmax = fmax(vmax, fabs(vn));
        }
#pragma omp parallel for reduction(max : rmax, vmax) reduction(+ : nbad)
    for (int j = 1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double sT = s->tyyn[C2(i, j)] - s->pn[C2(i, j)];
            double sB = s->tyyn[C2(i, j - 1)] - s->pn[C2(i, j - 1)];
            double R = (sT - sB) / dy + (s->txyn[XY2(i + 1, j)] - s->txyn[XY2(i, j)]) / dx;
            double vn = s->vy[VY2(i, j)] + s->dtrho * R;
            s->vyn[VY2(i, j)] = vn;
            rmax = fmax(rmax, fabs(R));
            if (!(fabs(R) <= DBL_MAX)) nbad++;
            vmax = fmax(vmax, fabs(vn));
        }
    s->vmax = vmax;
    if (nbad) rmax = NAN;
    if (physical) return rmax;
    rmax = fmax(rmax, fmax(dpm * p_res_visc(s) / s->kdtau, dtm * s->eta / s->gdtau) / s->L);
    if (nbad) rmax = NAN;
    if (mode == 2) return rmax;
    /* commit (Jacobi: every update above read only old values) */
    for (int j = 0; j < ny; ++j) for (int i = 1; i < nx; ++i) s->vx[VX2(i, j)] = s->vxn[VX2(i, j)];
    for (int j = 1; j < ny; ++j) for (int i = 0; i < nx; ++i) s->vy[VY2(i, j)] = s->vyn[VY2(i, j)];
    memcpy(s->p, s->pn, (size_t)n_cells(s) * sizeof(double));
    memcpy(s->txx, s->txxn, (size_t)n_cells(s) * sizeof(double));
    memcpy(s->tyy, s->tyyn, (size_t)n_cells(s) * sizeof(double));
    memcpy(s->txy, s->txyn, (size_t)n_xy(s) * sizeof(double));
    return rmax;
}

/* ------------------------------------------------------------------ 3D */
/* Compliance 1/(G dt) of an interior 3D edge: the uniform value, or the mean
 * over the four cells around it when G is given per cell.  axis: the edge's
 * direction ('z': an xy edge at (i, j) of layer k; 'y': an xz edge; 'x': a yz
 * edge), the four cells in the order the edge's Lambda takes them. */
static double igd_edge(const orc_state* s, char axis, int i, int j, int k, double igd)
{
    if (!s->igdc) return igd;
    const long nx = s->nx, nxy = (long)s->nx * s->ny;
#define CELL(a, b, c) s->igdc[(a) + nx * (b) + nxy * (c)]
    if (axis == 'z') return 0.25 * (CELL(i - 1, j - 1, k) + CELL(i, j - 1, k) + CELL(i - 1, j, k) + CELL(i, j, k));
    if (axis == 'y') return 0.25 * (CELL(i - 1, j, k - 1) + CELL(i, j, k - 1) + CELL(i - 1, j, k) + CELL(i, j, k));
    return 0.25 * (CELL(i, j - 1, k - 1) + CELL(i, j, k - 1) + CELL(i, j - 1, k) + CELL(i, j, k));
#undef CELL
}

static double sweep3d(orc_state* s, int mode)
{
    const int physical = mode == 1;
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const double dx = s->dx, dy = s->dy, dz = s->dz;
    const double igt = physical ? 0.0 : 1.0 / s->gdtau;
    /* incompressible limit (K = +inf): the pressure has no local physical
     * law, so the physical evaluation keeps its pseudo-time term (a reading) */
    const double ikt = (physical && !isinf(s->prm.bulk)) ? 0.0 : 1.0 / s->kdtau;
    const double igd = 1.0 / (s->prm.shear * s->prm.dt);
    const double ikd = 1.0 / (s->prm.bulk * s->prm.dt);
    const double kk = 1.0 / (ikt + ikd);      /* pressure compliance of one update */

    /* 1. divergence and pressure */
#pragma omp parallel for
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double div = (s->vx[VX3(i + 1, j, k)] - s->vx[VX3(i, j, k)]) / dx
                           + (s->vy[VY3(i, j + 1, k)] - s->vy[VY3(i, j, k)]) / dy
                           + (s->vz[VZ3(i, j, k + 1)] - s->vz[VZ3(i, j, k)]) / dz;
                long c = C3(i, j, k);
                s->dv[c] = div;
                s->pn[c] = (s->p[c] * ikt + s->p_old[c] * ikd - div) / (ikt + ikd);
            }
    /* 2. shear trials at edges (zero on walls) */
#pragma omp parallel for
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                long e = XY3(i, j, k);
                if (i == 0 || i == nx || j == 0 || j == ny) { s->Txy[e] = 0.0; continue; }
                double exy = 0.5 * ((s->vx[VX3(i, j, k)] - s->vx[VX3(i, j - 1, k)]) / dy
                                  + (s->vy[VY3(i, j, k)] - s->vy[VY3(i - 1, j, k)]) / dx);
                s->Sxy[e] = s->txy_old[e] * igd_edge(s, 'z', i, j, k, igd) + 2.0 * exy;
                s->Txy[e] = s->txy[e] * igt + s->Sxy[e];
            }
#pragma omp parallel for
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                long e = XZ3(i, j, k);
                if (i == 0 || i == nx || k == 0 || k == nz) { s->Txz[e] = 0.0; continue; }
                double exz = 0.5 * ((s->vx[VX3(i, j, k)] - s->vx[VX3(i, j, k - 1)]) / dz
                                  + (s->vz[VZ3(i, j, k)] - s->vz[VZ3(i - 1, j, k)]) / dx);
                s->Sxz[e] = s->txz_old[e] * igd_edge(s, 'y', i, j, k, igd) + 2.0 * exz;
                s->Txz[e] = s->txz[e] * igt + s->Sxz[e];
            }
#pragma omp parallel for
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long e = YZ3(i, j, k);
                if (j == 0 || j == ny || k == 0 || k == nz) { s->Tyz[e] = 0.0; continue; }
                double eyz = 0.5 * ((s->vy[VY3(i, j, k)] - s->vy[VY3(i, j, k - 1)]) / dz
                                  + (s->vz[VZ3(i, j, k)] - s->vz[VZ3(i, j - 1, k)]) / dy);
                s->Syz[e] = s->tyz_old[e] * igd_edge(s, 'x', i, j, k, igd) + 2.0 * eyz;
                s->Tyz[e] = s->tyz[e] * igt + s->Syz[e];
            }
    /* 3. normal trials and return mapping at centres */
    long long ny_count = 0;
    double dpm = 0.0, dtm = 0.0;
#pragma omp parallel for reduction(+ : ny_count) reduction(max : dpm, dtm)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long c = C3(i, j, k);
                double div = s->dv[c];
                double exx = (s->vx[VX3(i + 1, j, k)] - s->vx[VX3(i, j, k)]) / dx - div / 3.0;
                double eyy = (s->vy[VY3(i, j + 1, k)] - s->vy[VY3(i, j, k)]) / dy - div / 3.0;
                double ezz = (s->vz[VZ3(i, j, k + 1)] - s->vz[VZ3(i, j, k)]) / dz - div / 3.0;
                const double igdc = s->igdc ? s->igdc[c] : igd;
                const double Dp = igdc + s->inv_mus;     /* physical compliance 1/eta */
                const double D = igt + Dp;
                double Sxx = s->txx_old[c] * igdc + 2.0 * exx;
                double Syy = s->tyy_old[c] * igdc + 2.0 * eyy;
                double Szz = s->tzz_old[c] * igdc + 2.0 * ezz;
                double Txx = s->txx[c] * igt + Sxx;
                double Tyy = s->tyy[c] * igt + Syy;
                double Tzz = s->tzz[c] * igt + Szz;
                double Sxyb = 0.25 * (s->Sxy[XY3(i, j, k)] + s->Sxy[XY3(i + 1, j, k)]
                                    + s->Sxy[XY3(i, j + 1, k)] + s->Sxy[XY3(i + 1, j + 1, k)]);
                double Sxzb = 0.25 * (s->Sxz[XZ3(i, j, k)] + s->Sxz[XZ3(i + 1, j, k)]
                                    + s->Sxz[XZ3(i, j, k + 1)] + s->Sxz[XZ3(i + 1, j, k + 1)]);
                double Syzb = 0.25 * (s->Syz[YZ3(i, j, k)] + s->Syz[YZ3(i, j + 1, k)]
                                    + s->Syz[YZ3(i, j, k + 1)] + s->Syz[YZ3(i, j + 1, k + 1)]);
                double J2 = 0.5 * (Sxx * Sxx + Syy * Syy + Szz * Szz)
                          + Sxyb * Sxyb + Sxzb * Sxzb + Syzb * Syzb;   /* J2 of the physical trial */
                double tret, Y, ld;
                const double ptr = s->pn[c];
                double lam = centre_return(s, 0.5 * (Txx * Txx + Tyy * Tyy + Tzz * Tzz),
                                           0.5 * (Sxx * Sxx + Syy * Syy + Szz * Szz),
                                           Sxyb * Sxyb + Sxzb * Sxzb + Syzb * Syzb, Dp, D, kk, ptr, s->coh[c],
                                           &s->pn[c], &tret, &Y, &ld);
                s->lamdot[c] = ld;
                s->tII[c] = tret;
                s->yld[c] = Y;
                if (lam > 0.0) ny_count++;
                if (mode == 0 && s->freeze == 1) s->lamf[c] = lam;
                if (s->freeze == 2) {   /* held Lambda, also in the certificate */
                    lam = s->lamf[c];
                    if (s->C > 0.0) s->pn[c] = ptr + lam * sqrt(J2) / (Dp + lam) * s->C * kk;
                }
                s->lam[c] = lam;
                s->txxn[c] = Txx / (D + lam);
                s->tyyn[c] = Tyy / (D + lam);
                s->tzzn[c] = Tzz / (D + lam);
                dpm = fmax(dpm, fabs(s->pn[c] - s->p[c]));
                dtm = fmax(dtm, fmax(fabs(s->txxn[c] - s->txx[c]),
                                     fmax(fabs(s->tyyn[c] - s->tyy[c]), fabs(s->tzzn[c] - s->tzz[c]))));
            }
    s->n_yield = ny_count;
    /* 4. edges: Lambda averaged from the four adjacent centres */
#pragma omp parallel for reduction(max : dtm)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                long e = XY3(i, j, k);
                if (i == 0 || i == nx || j == 0 || j == ny) { s->txyn[e] = 0.0; continue; }
                double lv = 0.25 * (s->lam[C3(i - 1, j - 1, k)] + s->lam[C3(i, j - 1, k)]
                                  + s->lam[C3(i - 1, j, k)] + s->lam[C3(i, j, k)]);
                s->txyn[e] = s->Txy[e] / (igt + igd_edge(s, 'z', i, j, k, igd) + s->inv_mus + lv);
                dtm = fmax(dtm, fabs(s->txyn[e] - s->txy[e]));
            }
#pragma omp parallel for reduction(max : dtm)
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                long e = XZ3(i, j, k);
                if (i == 0 || i == nx || k == 0 || k == nz) { s->txzn[e] = 0.0; continue; }
                double lv = 0.25 * (s->lam[C3(i - 1, j, k - 1)] + s->lam[C3(i, j, k - 1)]
                                  + s->lam[C3(i - 1, j, k)] + s->lam[C3(i, j, k)]);
                s->txzn[e] = s->Txz[e] / (igt + igd_edge(s, 'y', i, j, k, igd) + s->inv_mus + lv);
                dtm = fmax(dtm, fabs(s->txzn[e] - s->txz[e]));
            }
#pragma omp parallel for reduction(max : dtm)
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long e = YZ3(i, j, k);
                if (j == 0 || j == ny || k == 0 || k == nz) { s->tyzn[e] = 0.0; continue; }
                double lv = 0.25 * (s->lam[C3(i, j - 1, k - 1)] + s->lam[C3(i, j, k - 1)]
                                  + s->lam[C3(i, j - 1, k)] + s->lam[C3(i, j, k)]);
                s->tyzn[e] = s->Tyz[e] / (igt + igd_edge(s, 'x', i, j, k, igd) + s->inv_mus + lv);
                dtm = fmax(dtm, fabs(s->tyzn[e] - s->tyz[e]));
            }
    /* 5. momentum residual and velocity update */
    double rmax = 0.0, vmax = 0.0;
    long nbad = 0;
#pragma omp parallel for reduction(max : rmax, vmax) reduction(+ : nbad)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 1; i < nx; ++i) {
                double sR = s->txxn[C3(i, j, k)] - s->pn[C3(i, j, k)];
                double sL = s->txxn[C3(i - 1, j, k)] - s->pn[C3(i - 1, j, k)];
                double R = (sR - sL) / dx
                         + (s->txyn[XY3(i, j + 1, k)] - s->txyn[XY3(i, j, k)]) / dy
                         + (s->txzn[XZ3(i, j, k + 1)] - s->txzn[XZ3(i, j, k)]) / dz;
                double vn = s->vx[VX3(i, j, k)] + s->dtrho * R;
                s->vxn[VX3(i, j, k)] = vn;
                rmax = fmax(rmax, fabs(R));
            if (!(fabs(R) <= DBL_MAX)) nbad++;
                vmax = fmax(vmax, fabs(vn));
            }
#pragma omp parallel for reduction(max : rmax, vmax) reduction(+ : nbad)
    for (int k = 0; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double sT = s->tyyn[C3(i, j, k)] - s->pn[C3(i, j, k)];
                double sB = s->tyyn[C3(i, j - 1, k)] - s->pn[C3(i, j - 1, k)];
                double R = (s->txyn[XY3(i + 1, j, k)] - s->txyn[XY3(i, j, k)]) / dx
                         + (sT - sB) / dy
                         + (s->tyzn[YZ3(i, j, k + 1)] - s->tyzn[YZ3(i, j, k)]) / dz;
                double vn = s->vy[VY3(i, j, k)] + s->dtrho * R;
                s->vyn[VY3(i, j, k)] = vn;
                rmax = fmax(rmax, fabs(R));
            if (!(fabs(R) <= DBL_MAX)) nbad++;
                vmax = fmax(vmax, fabs(vn));
            }
#pragma omp parallel for reduction(max : rmax, vmax) reduction(+ : nbad)
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double sU = s->tzzn[C3(i, j, k)] - s->pn[C3(i, j, k)];
                double sD = s->tzzn[C3(i, j, k - 1)] - s->pn[C3(i, j, k - 1)];
                double R = (s->txzn[XZ3(i + 1, j, k)] - s->txzn[XZ3(i, j, k)]) / dx
                         + (s->tyzn[YZ3(i, j + 1, k)] - s->tyzn[YZ3(i, j, k)]) / dy
                         + (sU - sD) / dz;
                double vn = s->vz[VZ3(i, j, k)] + s->dtrho * R;
                s->vzn[VZ3(i, j, k)] = vn;
                rmax = fmax(rmax, fabs(R));
            if (!(fabs(R) <= DBL_MAX)) nbad++;
                vmax = fmax(vmax, fabs(vn));
            }
    s->vmax = vmax;
    if (nbad) rmax = NAN;
    if (physical) return rmax;
    rmax = fmax(rmax, fmax(dpm * p_res_visc(s) / s->kdtau, dtm * s->eta / s->gdtau) / s->L);
    if (nbad) rmax = NAN;
    if (mode == 2) return rmax;
    for (int k = 0; k < nz; ++k) for (int j = 0; j < ny; ++j) for (int i = 1; i < nx; ++i)
        s->vx[VX3(i, j, k)] = s->vxn[VX3(i, j, k)];
    for (int k = 0; k < nz; ++k) for (int j = 1; j < ny; ++j) for (int i = 0; i < nx; ++i)
        s->vy[VY3(i, j, k)] = s->vyn[VY3(i, j, k)];
    for (int k = 1; k < nz; ++k) for (int j = 0; j < ny; ++j) for (int i = 0; i < nx; ++i)
        s->vz[VZ3(i, j, k)] = s->vzn[VZ3(i, j, k)];
    long nc = n_cells(s);
    memcpy(s->p, s->pn, (size_t)nc * sizeof(double));
    memcpy(s->txx, s->txxn, (size_t)nc * sizeof(double));
    memcpy(s->tyy, s->tyyn, (size_t)nc * sizeof(double));
    memcpy(s->tzz, s->tzzn, (size_t)nc * sizeof(double));
    memcpy(s->txy, s->txyn, (size_t)n_xy(s) * sizeof(double));
    memcpy(s->txz, s->txzn, (size_t)n_xz(s) * sizeof(double));
    memcpy(s->tyz, s->tyzn, (size_t)n_yz(s) * sizeof(double));
    return rmax;
}

double orc_sweep(orc_state* s, int mode)
{
    return s->ndim == 2 ? sweep2d(s, mode) : sweep3d(s, mode);
}

/* ------------------------------------------------------------ increment */
static void copy_n(double* dst, const double* src, long n) { if (n > 0) memcpy(dst, src, (size_t)n * sizeof(double)); }

/* ------------------------------------------------- objective stress update */
/* Paper: Jaumann rate of stress (equations j1-j14) and the appendix on the
 * objective stress terms.  Over one increment, explicitly, with the current
 * velocities v:
 *     tau <- tau + dt (tau^R - v . grad tau),     p <- p - dt v . grad p,
 * tau^R_ij = w_ik tau_jk + w_jk tau_ik in the appendix's component form, with
 * w_ij = (dv_i/dx_j - dv_j/dx_i) / 2 (the reading of the paper's index
 * convention under which a rigid rotation leaves the rate zero).
 * Discretisation (a reading; the paper gives none): w at its natural shear
 * points (2D vertices, 3D xy/xz/yz edges) from the adjacent face
 * velocities, zero on wall points (where the free-slip shear stress is zero
 * too); centre terms are 4-point means of the shear products; shear-point
 * terms use 4-point means of the centre stresses and of the other shear
 * components; advection is first-order upwind with the velocity averaged to
 * the point, zero gradient where the upwind neighbour lies outside the
 * grid.  Wall shear points keep their (zero) stresses. */

/* value of a field stored with extents ex x ey (x fastest) */
static double fat(const double* f, int ex, int ey, int i, int j, int k) { return f[i + (long)ex * (j + (long)ey * k)]; }

/* first-order upwind derivative of f along axis d at (i, j, k) for the
 * advecting velocity u; 0 when the upwind neighbour does not exist */
static double upwind(const double* f, int ex, int ey, int ez, int i, int j, int k, int d, double u, double h)
{
    int n[3] = {ex, ey, ez}, q[3] = {i, j, k};
    q[d] += (u > 0.0) ? -1 : 1;
    if (q[d] < 0 || q[d] >= n[d]) return 0.0;
    double f0 = fat(f, ex, ey, i, j, k), f1 = fat(f, ex, ey, q[0], q[1], q[2]);
    return (u > 0.0) ? (f0 - f1) / h : (f1 - f0) / h;
}

static void objective2d(orc_state* s)
{
    const int nx = s->nx, ny = s->ny;
    const double dx = s->dx, dy = s->dy, dt = s->prm.dt;
    const long nc = n_cells(s), nv = n_xy(s);
    double* w = zalloc(nv);
    double *pn = zalloc(nc), *xx = zalloc(nc), *yy = zalloc(nc), *xy = zalloc(nv);
    for (int j = 1; j < ny; ++j)
        for (int i = 1; i < nx; ++i)
            w[XY2(i, j)] = 0.5 * ((s->vx[VX2(i, j)] - s->vx[VX2(i, j - 1)]) / dy
                                - (s->vy[VY2(i, j)] - s->vy[VY2(i - 1, j)]) / dx);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double ux = 0.5 * (s->vx[VX2(i, j)] + s->vx[VX2(i + 1, j)]);
            const double uy = 0.5 * (s->vy[VY2(i, j)] + s->vy[VY2(i, j + 1)]);
            double pxy = 0.0;   /* mean of tau_xy w_xy over the 4 vertices */
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) pxy += s->txy[XY2(i + a, j + b)] * w[XY2(i + a, j + b)];
            pxy *= 0.25;
            const double rxx = 2.0 * pxy, ryy = -2.0 * pxy;
#define ADV2(f) (ux * upwind(f, nx, ny, 1, i, j, 0, 0, ux, dx) + uy * upwind(f, nx, ny, 1, i, j, 0, 1, uy, dy))
            pn[C2(i, j)] = s->p[C2(i, j)] - dt * ADV2(s->p);
            xx[C2(i, j)] = s->txx[C2(i, j)] + dt * (rxx - ADV2(s->txx));
            yy[C2(i, j)] = s->tyy[C2(i, j)] + dt * (ryy - ADV2(s->tyy));
#undef ADV2
        }
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            if (i == 0 || i == nx || j == 0 || j == ny) { xy[XY2(i, j)] = s->txy[XY2(i, j)]; continue; }
            const double ux = 0.5 * (s->vx[VX2(i, j - 1)] + s->vx[VX2(i, j)]);
            const double uy = 0.5 * (s->vy[VY2(i - 1, j)] + s->vy[VY2(i, j)]);
            double d = 0.0;     /* mean of tau_yy - tau_xx over the 4 centres */
            for (int b = -1; b < 1; ++b)
                for (int a = -1; a < 1; ++a) d += s->tyy[C2(i + a, j + b)] - s->txx[C2(i + a, j + b)];
            d *= 0.25;
            const double rxy = w[XY2(i, j)] * d;
            const double adv = ux * upwind(s->txy, nx + 1, ny + 1, 1, i, j, 0, 0, ux, dx)
                             + uy * upwind(s->txy, nx + 1, ny + 1, 1, i, j, 0, 1, uy, dy);
            xy[XY2(i, j)] = s->txy[XY2(i, j)] + dt * (rxy - adv);
        }
    copy_n(s->p, pn, nc);
    copy_n(s->txx, xx, nc);
    copy_n(s->tyy, yy, nc);
    copy_n(s->txy, xy, nv);
    free(w); free(pn); free(xx); free(yy); free(xy);
}

static void objective3d(orc_state* s)
{
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const double dx = s->dx, dy = s->dy, dz = s->dz, dt = s->prm.dt;
    const long nc = n_cells(s), nxy = n_xy(s), nxz = n_xz(s), nyz = n_yz(s);
    const double *vx = s->vx, *vy = s->vy, *vz = s->vz;
    double *wxy = zalloc(nxy), *wxz = zalloc(nxz), *wyz = zalloc(nyz);
    double *pn = zalloc(nc), *xx = zalloc(nc), *yy = zalloc(nc), *zz = zalloc(nc);
    double *xy = zalloc(nxy), *xz = zalloc(nxz), *yz = zalloc(nyz);
    /* vorticity at the interior shear points */
    for (int k = 0; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 1; i < nx; ++i)
                wxy[XY3(i, j, k)] = 0.5 * ((vx[VX3(i, j, k)] - vx[VX3(i, j - 1, k)]) / dy
                                         - (vy[VY3(i, j, k)] - vy[VY3(i - 1, j, k)]) / dx);
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 1; i < nx; ++i)
                wxz[XZ3(i, j, k)] = 0.5 * ((vx[VX3(i, j, k)] - vx[VX3(i, j, k - 1)]) / dz
                                         - (vz[VZ3(i, j, k)] - vz[VZ3(i - 1, j, k)]) / dx);
    for (int k = 1; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                wyz[YZ3(i, j, k)] = 0.5 * ((vy[VY3(i, j, k)] - vy[VY3(i, j, k - 1)]) / dz
                                         - (vz[VZ3(i, j, k)] - vz[VZ3(i, j - 1, k)]) / dy);
    /* centres */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const double ux = 0.5 * (vx[VX3(i, j, k)] + vx[VX3(i + 1, j, k)]);
                const double uy = 0.5 * (vy[VY3(i, j, k)] + vy[VY3(i, j + 1, k)]);
                const double uz = 0.5 * (vz[VZ3(i, j, k)] + vz[VZ3(i, j, k + 1)]);
                double pxy = 0.0, pxz = 0.0, pyz = 0.0;   /* 4-point means of tau_ab w_ab */
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a) {
                        pxy += s->txy[XY3(i + a, j + b, k)] * wxy[XY3(i + a, j + b, k)];
                        pxz += s->txz[XZ3(i + a, j, k + b)] * wxz[XZ3(i + a, j, k + b)];
                        pyz += s->tyz[YZ3(i, j + a, k + b)] * wyz[YZ3(i, j + a, k + b)];
                    }
                pxy *= 0.25; pxz *= 0.25; pyz *= 0.25;
                const double rxx = 2.0 * (pxy + pxz);
                const double ryy = -2.0 * (pxy - pyz);
                const double rzz = -2.0 * (pxz + pyz);
#define ADV3(f) (ux * upwind(f, nx, ny, nz, i, j, k, 0, ux, dx) + uy * upwind(f, nx, ny, nz, i, j, k, 1, uy, dy) \
               + uz * upwind(f, nx, ny, nz, i, j, k, 2, uz, dz))
                const long c = C3(i, j, k);
                pn[c] = s->p[c] - dt * ADV3(s->p);
                xx[c] = s->txx[c] + dt * (rxx - ADV3(s->txx));
                yy[c] = s->tyy[c] + dt * (ryy - ADV3(s->tyy));
                zz[c] = s->tzz[c] + dt * (rzz - ADV3(s->tzz));
#undef ADV3
            }
    /* xy edges (x_i, y_j, z_k+1/2) */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                const long e = XY3(i, j, k);
                if (i == 0 || i == nx || j == 0 || j == ny) { xy[e] = s->txy[e]; continue; }
                const double ux = 0.5 * (vx[VX3(i, j - 1, k)] + vx[VX3(i, j, k)]);
                const double uy = 0.5 * (vy[VY3(i - 1, j, k)] + vy[VY3(i, j, k)]);
                double uz = 0.0, d = 0.0, tyz = 0.0, w_yz = 0.0, txz = 0.0, w_xz = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = -1; b < 1; ++b)
                        for (int a = -1; a < 1; ++a) uz += vz[VZ3(i + a, j + b, k + c)];
                uz *= 0.125;
                for (int b = -1; b < 1; ++b)
                    for (int a = -1; a < 1; ++a) d += s->tyy[C3(i + a, j + b, k)] - s->txx[C3(i + a, j + b, k)];
                for (int c = 0; c < 2; ++c)
                    for (int a = -1; a < 1; ++a) {        /* yz edges (x_i+a+1/2, y_j, z_k+c) */
                        tyz += s->tyz[YZ3(i + a, j, k + c)];
                        w_yz += wyz[YZ3(i + a, j, k + c)];
                    }
                for (int c = 0; c < 2; ++c)
                    for (int b = -1; b < 1; ++b) {        /* xz edges (x_i, y_j+b+1/2, z_k+c) */
                        txz += s->txz[XZ3(i, j + b, k + c)];
                        w_xz += wxz[XZ3(i, j + b, k + c)];
                    }
                d *= 0.25; tyz *= 0.25; w_yz *= 0.25; txz *= 0.25; w_xz *= 0.25;
                const double r = wxy[e] * d + tyz * w_xz + txz * w_yz;
                const double adv = ux * upwind(s->txy, nx + 1, ny + 1, nz, i, j, k, 0, ux, dx)
                                 + uy * upwind(s->txy, nx + 1, ny + 1, nz, i, j, k, 1, uy, dy)
                                 + uz * upwind(s->txy, nx + 1, ny + 1, nz, i, j, k, 2, uz, dz);
                xy[e] = s->txy[e] + dt * (r - adv);
            }
    /* xz edges (x_i, y_j+1/2, z_k) */
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                const long e = XZ3(i, j, k);
                if (i == 0 || i == nx || k == 0 || k == nz) { xz[e] = s->txz[e]; continue; }
                const double ux = 0.5 * (vx[VX3(i, j, k - 1)] + vx[VX3(i, j, k)]);
                const double uz = 0.5 * (vz[VZ3(i - 1, j, k)] + vz[VZ3(i, j, k)]);
                double uy = 0.0, d = 0.0, tyz = 0.0, w_yz = 0.0, txy = 0.0, w_xy = 0.0;
                for (int c = -1; c < 1; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = -1; a < 1; ++a) uy += vy[VY3(i + a, j + b, k + c)];
                uy *= 0.125;
                for (int c = -1; c < 1; ++c)
                    for (int a = -1; a < 1; ++a) d += s->tzz[C3(i + a, j, k + c)] - s->txx[C3(i + a, j, k + c)];
                for (int b = 0; b < 2; ++b)
                    for (int a = -1; a < 1; ++a) {        /* yz edges (x_i+a+1/2, y_j+b, z_k) */
                        tyz += s->tyz[YZ3(i + a, j + b, k)];
                        w_yz += wyz[YZ3(i + a, j + b, k)];
                    }
                for (int c = -1; c < 1; ++c)
                    for (int b = 0; b < 2; ++b) {         /* xy edges (x_i, y_j+b, z_k+c+1/2) */
                        txy += s->txy[XY3(i, j + b, k + c)];
                        w_xy += wxy[XY3(i, j + b, k + c)];
                    }
                d *= 0.25; tyz *= 0.25; w_yz *= 0.25; txy *= 0.25; w_xy *= 0.25;
                const double r = wxz[e] * d + tyz * w_xy - txy * w_yz;
                const double adv = ux * upwind(s->txz, nx + 1, ny, nz + 1, i, j, k, 0, ux, dx)
                                 + uy * upwind(s->txz, nx + 1, ny, nz + 1, i, j, k, 1, uy, dy)
                                 + uz * upwind(s->txz, nx + 1, ny, nz + 1, i, j, k, 2, uz, dz);
                xz[e] = s->txz[e] + dt * (r - adv);
            }
    /* yz edges (x_i+1/2, y_j, z_k) */
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const long e = YZ3(i, j, k);
                if (j == 0 || j == ny || k == 0 || k == nz) { yz[e] = s->tyz[e]; continue; }
                const double uy = 0.5 * (vy[VY3(i, j, k - 1)] + vy[VY3(i, j, k)]);
                const double uz = 0.5 * (vz[VZ3(i, j - 1, k)] + vz[VZ3(i, j, k)]);
                double ux = 0.0, d = 0.0, txy = 0.0, w_xy = 0.0, txz = 0.0, w_xz = 0.0;
                for (int c = -1; c < 1; ++c)
                    for (int b = -1; b < 1; ++b)
                        for (int a = 0; a < 2; ++a) ux += vx[VX3(i + a, j + b, k + c)];
                ux *= 0.125;
                for (int c = -1; c < 1; ++c)
                    for (int b = -1; b < 1; ++b) d += s->tzz[C3(i, j + b, k + c)] - s->tyy[C3(i, j + b, k + c)];
                for (int c = -1; c < 1; ++c)
                    for (int a = 0; a < 2; ++a) {         /* xy edges (x_i+a, y_j, z_k+c+1/2) */
                        txy += s->txy[XY3(i + a, j, k + c)];
                        w_xy += wxy[XY3(i + a, j, k + c)];
                    }
                for (int b = -1; b < 1; ++b)
                    for (int a = 0; a < 2; ++a) {         /* xz edges (x_i+a, y_j+b+1/2, z_k) */
                        txz += s->txz[XZ3(i + a, j + b, k)];
                        w_xz += wxz[XZ3(i + a, j + b, k)];
                    }
                d *= 0.25; txy *= 0.25; w_xy *= 0.25; txz *= 0.25; w_xz *= 0.25;
                const double r = wyz[e] * d - txy * w_xz - txz * w_xy;
                const double adv = ux * upwind(s->tyz, nx, ny + 1, nz + 1, i, j, k, 0, ux, dx)
                                 + uy * upwind(s->tyz, nx, ny + 1, nz + 1, i, j, k, 1, uy, dy)
                                 + uz * upwind(s->tyz, nx, ny + 1, nz + 1, i, j, k, 2, uz, dz);
                yz[e] = s->tyz[e] + dt * (r - adv);
            }
    copy_n(s->p, pn, nc);
    copy_n(s->txx, xx, nc);
    copy_n(s->tyy, yy, nc);
    copy_n(s->tzz, zz, nc);
    copy_n(s->txy, xy, nxy);
    copy_n(s->txz, xz, nxz);
    copy_n(s->tyz, yz, nyz);
    free(wxy); free(wxz); free(wyz); free(pn); free(xx); free(yy); free(zz); free(xy); free(xz); free(yz);
}

/* Per-cell shear modulus (the heterogeneous setups' G field).  The physical
 * compliance 1/(G dt) of a cell replaces the uniform one in its stress
 * update; a vertex (2D) or edge (3D) takes the mean compliance of its four
 * cells (the harmonic mean of G; a reading).  The pseudo-time steps stay
 * those of prm.shear, which must bound every G.  Returns 0, or -1 (a G that
 * is not in (0, prm.shear]). */
int orc_set_shear_modulus(orc_state* s, const double* G)
{
    const long nc = n_cells(s);
    for (long c = 0; c < nc; ++c)
        if (!(G[c] > 0.0) || !(G[c] <= s->prm.shear)) return -1;
    if (!s->igdc) s->igdc = (double*)malloc((size_t)nc * sizeof(double));
    for (long c = 0; c < nc; ++c) s->igdc[c] = 1.0 / (G[c] * s->prm.dt);
    return 0;
}

void orc_set_strain_rate(orc_state* s, const double erate[3])
{
    for (int d = 0; d < 3; ++d) s->prm.erate[d] = (s->ndim == 3 || d < 2) ? erate[d] : 0.0;
}

void orc_objective_update(orc_state* s)
{
    if (s->ndim == 2) objective2d(s);
    else objective3d(s);
}

/* Copy the stresses of the last evaluation (orc_sweep modes 1 and 2 leave
 * them in the new-value arrays) into the state. */
static void commit_evaluated_stresses(orc_state* s)
{
    long nc = n_cells(s);
    copy_n(s->p, s->pn, nc);
    copy_n(s->txx, s->txxn, nc);
    copy_n(s->tyy, s->tyyn, nc);
    copy_n(s->tzz, s->tzzn, s->ndim == 3 ? nc : 0);
    copy_n(s->txy, s->txyn, n_xy(s));
    copy_n(s->txz, s->txzn, n_xz(s));
    copy_n(s->tyz, s->tyzn, n_yz(s));
}

static void save_start(orc_state* s)
{
    long nc = n_cells(s);
    copy_n(s->p_old, s->p, nc);
    copy_n(s->txx_old, s->txx, nc);
    copy_n(s->tyy_old, s->tyy, nc);
    copy_n(s->tzz_old, s->tzz, s->ndim == 3 ? nc : 0);
    copy_n(s->txy_old, s->txy, n_xy(s));
    copy_n(s->txz_old, s->txz, n_xz(s));
    copy_n(s->tyz_old, s->tyz, n_yz(s));
    copy_n(s->vx0, s->vx, n_vx(s));
    copy_n(s->vy0, s->vy, n_vy(s));
    copy_n(s->vz0, s->vz, n_vz(s));
}

static void roll_back(orc_state* s)
{
    long nc = n_cells(s);
    copy_n(s->p, s->p_old, nc);
    copy_n(s->txx, s->txx_old, nc);
    copy_n(s->tyy, s->tyy_old, nc);
    copy_n(s->tzz, s->tzz_old, s->ndim == 3 ? nc : 0);
    copy_n(s->txy, s->txy_old, n_xy(s));
    copy_n(s->txz, s->txz_old, n_xz(s));
    copy_n(s->tyz, s->tyz_old, n_yz(s));
    copy_n(s->vx, s->vx0, n_vx(s));
    copy_n(s->vy, s->vy0, n_vy(s));
    copy_n(s->vz, s->vz0, n_vz(s));
}

/* Accumulated displacement, strain and plastic strain; per-increment
 * diagnostics (integrated sigma_xx over columns, yield statistics). */
static void epilogue(orc_state* s, orc_stats* st)
{
    /* centre diagnostics (Lambda, plastic rate, returned tauII, bound) of the
     * accepted state: its physical evaluation, which commits nothing */
    orc_sweep(s, 1);
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const double A = s->A, B = s->B;
    const double dt = s->prm.dt, dx = s->dx, dy = s->dy, dz = s->dz;
    for (long q = 0; q < n_vx(s); ++q) s->ux[q] += dt * s->vx[q];
    for (long q = 0; q < n_vy(s); ++q) s->uy[q] += dt * s->vy[q];
    for (long q = 0; q < n_vz(s); ++q) s->uz[q] += dt * s->vz[q];
    double vio = -INFINITY;
    if (s->ndim == 2) {
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long c = C2(i, j);
                s->exx[c] += dt * (s->vx[VX2(i + 1, j)] - s->vx[VX2(i, j)]) / dx;
                s->eyy[c] += dt * (s->vy[VY2(i, j + 1)] - s->vy[VY2(i, j)]) / dy;
                s->eps_p[c] += dt * 0.5 * s->lamdot[c];
                double tb = 0.25 * (s->txy[XY2(i, j)] + s->txy[XY2(i + 1, j)]
                                  + s->txy[XY2(i, j + 1)] + s->txy[XY2(i + 1, j + 1)]);
                double tII = sqrt(0.5 * (s->txx[c] * s->txx[c] + s->tyy[c] * s->tyy[c]) + tb * tb);
                vio = fmax(vio, tII - fmax(0.0, A * s->p[c] + B * s->coh[c]));
            }
        for (int j = 1; j < ny; ++j)
            for (int i = 1; i < nx; ++i)
                s->exy[XY2(i, j)] += dt * 0.5 * ((s->vx[VX2(i, j)] - s->vx[VX2(i, j - 1)]) / dy
                                               + (s->vy[VY2(i, j)] - s->vy[VY2(i - 1, j)]) / dx);
        double sc = 0, sl = 0, sr = 0;
        for (int j = 0; j < ny; ++j) {
            sc += (s->txx[C2(nx / 2, j)] - s->p[C2(nx / 2, j)]) * dy;
            sl += (s->txx[C2(0, j)] - s->p[C2(0, j)]) * dy;
            sr += (s->txx[C2(nx - 1, j)] - s->p[C2(nx - 1, j)]) * dy;
        }
        st->sxx_centre = sc; st->sxx_left = sl; st->sxx_right = sr;
    } else {
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    long c = C3(i, j, k);
                    s->exx[c] += dt * (s->vx[VX3(i + 1, j, k)] - s->vx[VX3(i, j, k)]) / dx;
                    s->eyy[c] += dt * (s->vy[VY3(i, j + 1, k)] - s->vy[VY3(i, j, k)]) / dy;
                    s->ezz[c] += dt * (s->vz[VZ3(i, j, k + 1)] - s->vz[VZ3(i, j, k)]) / dz;
                    s->eps_p[c] += dt * 0.5 * s->lamdot[c];
                    double bxy = 0.25 * (s->txy[XY3(i, j, k)] + s->txy[XY3(i + 1, j, k)]
                                       + s->txy[XY3(i, j + 1, k)] + s->txy[XY3(i + 1, j + 1, k)]);
                    double bxz = 0.25 * (s->txz[XZ3(i, j, k)] + s->txz[XZ3(i + 1, j, k)]
                                       + s->txz[XZ3(i, j, k + 1)] + s->txz[XZ3(i + 1, j, k + 1)]);
                    double byz = 0.25 * (s->tyz[YZ3(i, j, k)] + s->tyz[YZ3(i, j + 1, k)]
                                       + s->tyz[YZ3(i, j, k + 1)] + s->tyz[YZ3(i, j + 1, k + 1)]);
                    double tII = sqrt(0.5 * (s->txx[c] * s->txx[c] + s->tyy[c] * s->tyy[c]
                                             + s->tzz[c] * s->tzz[c])
                                      + bxy * bxy + bxz * bxz + byz * byz);
                    vio = fmax(vio, tII - fmax(0.0, A * s->p[c] + B * s->coh[c]));
                }
        for (int k = 0; k < nz; ++k)
            for (int j = 1; j < ny; ++j)
                for (int i = 1; i < nx; ++i)
                    s->exy[XY3(i, j, k)] += dt * 0.5 * ((s->vx[VX3(i, j, k)] - s->vx[VX3(i, j - 1, k)]) / dy
                                                      + (s->vy[VY3(i, j, k)] - s->vy[VY3(i - 1, j, k)]) / dx);
        for (int k = 1; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 1; i < nx; ++i)
                    s->exz[XZ3(i, j, k)] += dt * 0.5 * ((s->vx[VX3(i, j, k)] - s->vx[VX3(i, j, k - 1)]) / dz
                                                      + (s->vz[VZ3(i, j, k)] - s->vz[VZ3(i - 1, j, k)]) / dx);
        for (int k = 1; k < nz; ++k)
            for (int j = 1; j < ny; ++j)
                for (int i = 0; i < nx; ++i)
                    s->eyz[YZ3(i, j, k)] += dt * 0.5 * ((s->vy[VY3(i, j, k)] - s->vy[VY3(i, j, k - 1)]) / dz
                                                      + (s->vz[VZ3(i, j, k)] - s->vz[VZ3(i, j - 1, k)]) / dy);
        double sc = 0, sl = 0, sr = 0;
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j) {
                sc += (s->txx[C3(nx / 2, j, k)] - s->p[C3(nx / 2, j, k)]) * dy * dz;
                sl += (s->txx[C3(0, j, k)] - s->p[C3(0, j, k)]) * dy * dz;
                sr += (s->txx[C3(nx - 1, j, k)] - s->p[C3(nx - 1, j, k)]) * dy * dz;
            }
        st->sxx_centre = sc; st->sxx_left = sl; st->sxx_right = sr;
    }
    st->n_yield = s->n_yield;
    st->max_violation = vio;
}

int orc_load_step(orc_state* s, orc_stats* st)
{
    orc_stats dummy;
    if (!st) st = &dummy;
    memset(st, 0, sizeof(*st));
    s->hist_len = 0;
    /* objective stress update of the carried stresses with the velocities
     * of the previous increment; the result is this increment's start */
    if (s->prm.objective) orc_objective_update(s);
    save_start(s);
    set_wall_velocities(s);

    /* normalisation: physical residual of the plain guess, floored by the
     * stress increment of the background loading over the domain size */
    double emax = fmax(fabs(s->prm.erate[0]), fmax(fabs(s->prm.erate[1]), fabs(s->prm.erate[2])));
    double dsig = 2.0 * s->prm.shear * emax * s->prm.dt;
    st->r_ref = orc_sweep(s, 1);
    st->ref = fmax(st->r_ref, dsig / s->L);
    if (!(st->r_ref <= DBL_MAX)) {           /* NaN / Inf in the starting state */
        st->status = -5;
        roll_back(s);
        return -5;
    }
    /* the pseudo-time iteration starts from the physical stresses of the
     * guessed velocities (the evaluation above), not from the previous
     * increment's stresses: same fixed point, no pseudo-time relaxation of
     * stresses that the guess already determines */
    commit_evaluated_stresses(s);

    const int nchk = s->prm.n_check;
    int status = -4;
    double res = NAN;
    int it;
    s->freeze = 0;
    /* a starting state that already meets the tolerance is accepted as it
     * is (its residual is the certificate): pseudo-time sweeps would first
     * roughen it (its stresses are already the physical ones) */
    if (st->r_ref <= s->prm.tol * st->ref) {
        st->iters = 0;
        st->resid = st->cert = st->r_ref;
        st->eps_rel = 0.0;
        st->status = 0;
        epilogue(s, st);
        return 0;
    }
    for (it = 1; it <= s->prm.max_iter; ++it) {
        res = orc_sweep(s, 0);
        if (s->freeze == 1) s->freeze = 2;   /* that sweep stored its Lambda */
        if (it % nchk == 0) {
            if (s->hist && s->hist_len < s->hist_cap) s->hist[s->hist_len++] = res;
            if (s->prm.progress > 0 && it % s->prm.progress == 0) {
                fprintf(stderr, "oracle: iteration %d residual/ref %.3e\n", it, res / st->ref);
                fflush(stderr);
            }
            if (!(res == res) || isinf(res) || res > 1e8 * st->ref) { status = -5; break; }
            if (res <= s->prm.tol * st->ref) {
                /* acceptance: the momentum residual of the physical stresses
                 * of the current velocities (pseudo-time terms removed) must
                 * meet the tolerance too; that evaluation is the accepted
                 * state's certificate, and its stresses the accepted ones */
                double cert = orc_sweep(s, 1);
                if (s->prm.progress > 0 && it % s->prm.progress == 0) {
                    fprintf(stderr, "oracle: iteration %d certificate/ref %.3e\n", it, cert / st->ref);
                    fflush(stderr);
                }
                if (cert <= s->prm.tol * st->ref) {
                    st->cert = cert;
                    commit_evaluated_stresses(s);
                    status = 0;
                    break;
                }
            }
            /* the blend of the iteration's return changes once, at the
             * first check at or after 16 max(nx, ny, nz) iterations */
            if (!s->late && it >= 16 * imax(s->nx, imax(s->ny, s->nz))) s->late = 1;
            /* frozen plasticity: an increment still iterating after
             * freeze_iter iterations continues with the plastic multiplier
             * of the next sweep held fixed (a linear problem) */
            if (s->prm.freeze_iter > 0 && s->freeze == 0 && it >= s->prm.freeze_iter) {
                s->freeze = 1;
                st->frozen_at = it;
            }
        }
    }
    s->freeze = 0;
    s->late = 0;
    st->iters = it > s->prm.max_iter ? s->prm.max_iter : it;
    st->resid = res;
    st->eps_rel = s->vmax > 0 ? s->dtrho * res / s->vmax : 0.0;
    st->status = status;
    if (status != 0) { roll_back(s); return status; }
    epilogue(s, st);
    return 0;
}
