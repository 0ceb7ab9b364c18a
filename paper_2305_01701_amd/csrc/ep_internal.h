// Internal interface between the host runtime (ep_api.hip) and the kernels.
//
// Device layout: every field lives in its own array with one common padded
// shape, x fastest: element (i, j, k) is at i + sy*j + sz*k with
// sy = round_up(nx + 1, 32) and sz = sy * (ny + 1).  Cells use i < nx,
// x-faces i <= nx, vertices / edges the corresponding "+1" extents, so the
// neighbour offsets of every staggered field are the same +-1, +-sy, +-sz.
// Padding entries are never read.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ep {

// Index of the iteration fields in the field tables.
enum { F_VX = 0, F_VY, F_VZ, F_P, F_TXX, F_TYY, F_TXY, F_TXZ, F_TYZ, F_NIT };
// Index of the previous-increment stresses.
enum { O_P = 0, O_TXX, O_TYY, O_TXY, O_TXZ, O_TYZ, O_N };

// Reduction slots (uint64 bit patterns of non-negative doubles; max by
// integer atomicMax; NaN is mapped to +inf before reduction).
enum { RED_RESID = 0, RED_MOM, RED_VMAX, RED_NYIELD, RED_VIOL, RED_SMAX, RED_CONT, RED_N = 8 };

// Scalars of one PT sweep.  Kernel arguments by value.
template <typename R>
struct SweepArgs {
    const R* it[F_NIT];    // iteration k (read)
    R* nx_[F_NIT];         // iteration k+1 (written)
    const R* old[O_N];     // stresses at the start of the increment
    const R* coh;          // cohesion at cells
    R* lam;                // unfused path: centre Lambda of this sweep
    unsigned long long* red;
    int nx, ny, nz;
    int sy;
    long sz;
    R idx, idy, idz;       // inverse spacings
    R igt, ikt;            // 1/(G~ dtau), 1/(K~ dtau); 0 for a physical evaluation
    R igd, ikd;            // 1/(G dt), 1/(K dt)
    R D;                   // igt + igd + 1/mu_s
    R invD;                // 1 / D
    R Dp, invDp;           // physical compliance igd + 1/mu_s and its inverse (uniform G)
    R blend;               // weight of the pseudo-time trial in the iteration's centre Lambda
    R ikk;                 // 1 / (ikt + ikd)
    R dtrho;               // dtau / rho~
    R A, B;                // Drucker-Prager constants
    R Cik;                 // dilatancy: C of the plastic potential / (ikt + ikd), the pressure
                           // change per unit plastic rate (0 for psi = 0)
    R vp;                  // consistency regularisation viscosity eta_vp (0: perfect plasticity)
    const R* igdc;         // 2D: per-cell 1/(G dt) (nullptr: uniform G, igd)
    R imus;                // 1/mu_s
    R rK, rG;              // pseudo-rate -> residual factors: K dt/(K~dtau L), eta/(G~dtau L)
    R ebx, eby, ebz;       // background strain rate subtracted from the stored velocities
                           // (FP32 fields store v - erate * x; 0 when v is stored in full)
    int lam_mode;          // 2D tile sweep: LAM_* (frozen plasticity)
    long fs;               // 3D: element stride between consecutive fields of it, nx_ and old
                           // (field f of a group = group[0] + f * fs; 0 when not uniform)
};

// Centre Lambda of the 2D tile sweep: from the return mapping; from the
// return mapping and stored to lam (the sweep that freezes it); read from lam.
enum { LAM_COMPUTE = 0, LAM_STORE = 1, LAM_FROZEN = 2 };

// Sweep modes.
enum { MODE_UPDATE = 0,    // write iteration k+1
       MODE_CHECK = 1,     // write k+1 and reduce the residual
       MODE_PHYS = 2 };    // physical evaluation (pseudo-time terms removed): write the stresses
                           // of the current velocities to the k+1 buffer, reduce the momentum
                           // residual, leave the velocities

// ---- launchers (ep_sweep_unfused.hip, ep_sweep_fused.hip) -------------------
template <typename R> void launch_sweep_unfused_2d(const SweepArgs<R>& a, int mode, hipStream_t s);
template <typename R> void launch_sweep_unfused_3d(const SweepArgs<R>& a, int mode, hipStream_t s);
template <typename R> void launch_sweep_fused_3d(const SweepArgs<R>& a, int mode, hipStream_t s);
// Whether the automatic choice uses the fused sweep for this case.
bool fused_preferred(int ndim, bool fp32);

// ---- batched 2D sweep (ep_sweep_batch.hip) ---------------------------------
struct TileRef {
    int model;             // index into the model table
    short bx, by;          // tile coordinates in the model's grid
};
constexpr int BATCH_SHAPES = 6;
extern const int kBatchTiles[BATCH_SHAPES][3];   // (TX, TY, threads) of each tile shape
constexpr int SINGLE_SHAPE = 4;                   // 64 x 16: the shape of single 2D models
// One sweep of every tile in list[0 .. *count) with the tile shape `shape`;
// table[model] holds the model's arguments (reads of iteration k, writes of
// k+1).  `grid` workgroups walk the list (persistent grid).
template <typename R>
void launch_sweep_batch_2d(int shape, const SweepArgs<R>* table, const TileRef* list, const int* count, int mode,
                           int grid, hipStream_t s);
// Resident workgroups per CU of the batched kernel with this tile shape.
template <typename R> int batch_blocks_per_cu(int shape);

// ---- auxiliary kernels (ep_aux.hip) ----------------------------------------
struct AuxGrid {
    int ndim, nx, ny, nz, sy;
    long sz;
    long nelem;            // elements per padded array
};

void launch_fill(double* p, double v, long n, hipStream_t s);
void launch_copy(double* dst, const double* src, long n, hipStream_t s);
// compact array of extents ext (x fastest; FP32 when f32, else FP64; nullptr:
// none) plus a padded base field (nullptr: none) -> padded FP64 field
void launch_guess_in(double* dst, const void* src, bool f32, const double* base, const int ext[3], long sy, long sz,
                     hipStream_t s);
void launch_to_f32(float* dst, const double* src, long n, hipStream_t s);
void launch_to_f64(double* dst, const float* src, long n, hipStream_t s);
// Velocity component d (0 x, 1 y, 2 z) between the full FP64 field and the
// FP32 field that stores v - erate_d * x_d (x_d the face coordinate).
void launch_vel_to_f32(const AuxGrid& g, int d, float* dst, const double* src, double erate, double len,
                       double spacing, hipStream_t s);
void launch_vel_to_f64(const AuxGrid& g, int d, double* dst, const float* src, double erate, double len,
                       double spacing, hipStream_t s);
// dst64 = base64 + (double)(x32 - base32)   (increment form)
void launch_incr_to_f64(double* dst, const double* base64, const float* x32, const float* base32,
                        long n, hipStream_t s);
void launch_reset_red(unsigned long long* red, hipStream_t s);
// Reduction slots of n_models consecutive models (a fill kernel, so that it
// can be captured in a graph).
void launch_reset_red_n(unsigned long long* red, int n_models, hipStream_t s);
// Background velocities at the wall faces.
void launch_set_walls(const AuxGrid& g, double* vx, double* vy, double* vz, const double erate[3],
                      double lx, double ly, double lz, hipStream_t s);
// Accumulators: u += v dt at faces; strains += grad v dt; eps_p += dt lamdot / 2.
void launch_accumulate(const AuxGrid& g, double dt, double idx, double idy, double idz,
                       const double* const v[3], double* const u[3], double* const e[6],
                       double* epsp, const double* lamdot, hipStream_t s);
// Centre diagnostics of the accepted state (one PT evaluation without writes):
// lamdot = D (tauII_tr - Y) where yielding, tauII returned, Y; counts yielding
// cells and the max violation tauII(stored) - Y into red.
template <typename R>
void launch_diagnostics(const SweepArgs<R>& a, double* lamdot, double* tii, double* yld,
                        hipStream_t s);
// Objective (Jaumann) update of the stresses carried into an increment
// (paper: Jaumann rate of stress and the appendix on the objective stress
// terms), explicit over dt with the velocities in `in`: out = tau + dt (tau^R
// - v.grad tau), p - dt v.grad p.  `in` and `out` hold the fields F_* (only
// the stress entries of `out` are written); out must not alias in.
struct ObjectiveArgs {
    const double* in[F_NIT];
    double* out[F_NIT];
    double dx, dy, dz, dt;
};
void launch_objective(const AuxGrid& g, const ObjectiveArgs& a, hipStream_t s);
// Continuity residual max |(p - p^) ikd + div v| over cells into *red_slot
// (ikd = 1/(K dt); 0 in the incompressible limit).
void launch_continuity(const AuxGrid& g, const double* const v[3], const double* p, const double* p_old, double ikd,
                       double idx, double idy, double idz, unsigned long long* red_slot, hipStream_t s);
// Column integrals of sigma_xx at columns i = 0, nx/2, nx-1 (3 doubles).
void launch_column_integrals(const AuxGrid& g, const double* p, const double* txx, double dy,
                             double dz, double* out3, hipStream_t s);

}  // namespace ep
