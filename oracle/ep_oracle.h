/*
 * CPU oracle for the per-increment elasto-plastic pseudo-transient solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, FP64 statement of what
 * the GPU library computes; only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header or constant with
 * the GPU library.
 *
 * Layout: every field is its own array with its natural staggered shape and
 * x fastest (no padding):
 *   2D cells (nx,ny); vx (nx+1,ny); vy (nx,ny+1); vertices txy (nx+1,ny+1)
 *   3D cells (nx,ny,nz); vx (nx+1,ny,nz); vy (nx,ny+1,nz); vz (nx,ny,nz+1);
 *      edges txy (nx+1,ny+1,nz), txz (nx+1,ny,nz+1), tyz (nx,ny+1,nz+1)
 */
#ifndef EP_ORACLE_H
#define EP_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
    int    ndim;             /* 2 or 3 */
    int    nx, ny, nz;       /* cells per direction (nz ignored in 2D) */
    double lx, ly, lz;       /* domain extents, domain centred at the origin */
    double bulk, shear;      /* K, G */
    double visc;             /* mu_s; +inf for the elasto-plastic limit */
    double phi_deg, psi_deg; /* friction and dilation angles, 0 <= psi <= phi */
    double dt;               /* physical time increment */
    double erate[3];         /* background strain rate, diagonal */
    double tol;              /* residual tolerance (normalised) */
    int    max_iter;         /* pseudo-time iteration cap per increment */
    int    n_check;          /* check the residual every n_check iterations */
    double re, r, cfl;       /* PT numerical Reynolds number, Ktilde/Gtilde, Courant number */
    int    freeze_iter;      /* 0: off; else freeze Lambda at the first check at or after
                                this iteration that has not converged */
    int    objective;        /* 1: objective (Jaumann) stress update at the start of every
                                increment (orc_objective_update); 0: off */
    double eta_vp;           /* consistency regularisation of the return: yielding points
                                carry tauII = A p + B c + eta_vp lambda_dot (0: perfect
                                plasticity) */
    double pt_blend;         /* weight in [0, 1] of the pseudo-time trial in the centre plastic
                                multiplier during the iteration (0: the physical trial alone);
                                the converged state does not depend on it */
    double pt_blend_late;    /* the weight after the first check at or after 16 max(nx, ny, nz)
                                iterations of an increment */
    int    progress;         /* 0: silent; else one line on stderr (iteration, normalised
                                residual) at every check whose iteration is a multiple of it */
} orc_params;

typedef struct orc_stats {
    int    status;           /* 0 converged, -4 not converged, -5 diverged */
    int    iters;            /* PT iterations performed */
    double r_ref;            /* residual of the physical stresses of the plain guess */
    double ref;              /* max(r_ref, dsigma_ref / L) */
    double resid;            /* residual of the iteration at the accepted check (absolute) */
    double cert;             /* momentum residual of the accepted state's physical stresses
                                (pseudo-time terms removed): the certificate, <= tol * ref */
    double eps_rel;          /* max|v^{k+1}-v^k| / max|v| at the final check */
    double sxx_centre;       /* integral of sigma_xx over the centre column */
    double sxx_left;         /* ... over the first column */
    double sxx_right;        /* ... over the last column */
    long long n_yield;       /* yielding cells in the physical evaluation of the accepted state */
    double max_violation;    /* max over cells of tauII(stored stresses) - max(0, A p + B c) */
    int    frozen_at;        /* iteration whose check froze Lambda (0: not frozen) */
} orc_stats;

enum {
    ORC_VX = 0, ORC_VY, ORC_VZ,
    ORC_P, ORC_TXX, ORC_TYY, ORC_TZZ, ORC_TXY, ORC_TXZ, ORC_TYZ,
    ORC_P_OLD, ORC_TXX_OLD, ORC_TYY_OLD, ORC_TZZ_OLD, ORC_TXY_OLD, ORC_TXZ_OLD, ORC_TYZ_OLD,
    ORC_UX, ORC_UY, ORC_UZ,
    ORC_EXX, ORC_EYY, ORC_EZZ, ORC_EXY, ORC_EXZ, ORC_EYZ,
    ORC_EPS_P, ORC_COHESION, ORC_LAMBDA, ORC_TAU_II, ORC_YIELD,
    ORC_LAMBDA_FROZEN,       /* centre Lambda held fixed by the last frozen increment */
    ORC_NFIELDS
};

typedef struct orc_state orc_state;

orc_state* orc_create(const orc_params* prm, const double* cohesion);
/* Objective stress update (paper: Jaumann rate of stress, equations j1-j14,
 * and the appendix on the objective stress terms), explicit over one
 * increment with the current velocities:
 *   tau <- tau + dt (tau^R - v.grad tau),  p <- p - dt v.grad p,
 * tau^R from the vorticity w_ij = (dv_i/dx_j - dv_j/dx_i)/2 (the reading of
 * the paper's index convention under which the rate is objective);
 * first-order upwind advection.  orc_load_step applies it to the carried
 * stresses before the increment when prm.objective is set. */
void orc_objective_update(orc_state* s);
/* Background strain rate of the next increments (walls take it at the next
 * orc_load_step). */
void orc_set_strain_rate(orc_state* s, const double erate[3]);
int  orc_set_shear_modulus(orc_state* s, const double* G);  /* per-cell G (see the source) */
void   orc_free(orc_state* s);
long   orc_field_size(const orc_state* s, int field);
int    orc_get(const orc_state* s, int field, double* out);
int    orc_set(orc_state* s, int field, const double* in);
/* One pseudo-transient iteration.  mode 0 updates the state; mode 1
 * evaluates the stresses of the current velocities with the pseudo-time terms
 * removed and returns their momentum residual; mode 2 evaluates one PT
 * iteration (filling the centre diagnostics) without committing it.  Modes 1
 * and 2 leave the state unchanged.  Returns the residual. */
double orc_sweep(orc_state* s, int mode);
int    orc_load_step(orc_state* s, orc_stats* st);
/* PT scalars: [G~dtau, K~dtau, dtau/rho~, eta_ve, A, B, h, L] */
void   orc_scalars(const orc_state* s, double out[8]);
/* Residual after each check of the most recent increment (cap entries). */
void   orc_history(orc_state* s, double* buf, int cap);
int    orc_history_len(const orc_state* s);
int    orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
