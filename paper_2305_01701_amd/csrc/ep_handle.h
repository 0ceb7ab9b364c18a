// Host-side state of one solver handle and the pieces of the increment
// driver, shared by the single-model entry points and the batched driver.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <vector>

#include "ep.h"
#include "ep_internal.h"

namespace ep {

// Control state of the increment in progress.
struct StepCtl {
    ep_step_stats* st;
    std::chrono::steady_clock::time_point t0;
    double tol_abs;       // absolute residual tolerance
    double sw;            // FP32 -> FP64 hand-over threshold (absolute)
    int stall_checks;
    double best;          // best FP32 residual so far
    int since_best;
    bool use32;           // sweeps currently run in FP32
    bool running;
    bool cert_pending;    // the last check met the tolerance: the certificate decides
    int status;
    double resid, vmax;
};

}  // namespace ep

struct ep_handle {
    ep_params prm;
    hipStream_t st;
    ep::AuxGrid g;
    int ndim, nx, ny, nz, sy;
    long sz, nelem;
    double dx, dy, dz, eta, gdtau, kdtau, dtrho, A, B, C, L, h, inv_mus, dsig_ref;
    int n_check;
    bool fp32, fused32, fused64;
    double* it64[2][ep::F_NIT];
    int cur64;
    double* old64[ep::O_N];
    double *coh64, *lam64;
    double* igdc64;        // 2D: per-cell 1/(G dt) when has_g
    double* vstart64[3];
    double* u64[3];
    double* e64[6];
    double *epsp64, *lamdot64, *tii64, *yld64, *cols64;
    float* it32[2][ep::F_NIT];
    int cur32;
    float* old32[ep::O_N];
    float *coh32, *lam32;
    float* igdc32;
    bool has_g;
    unsigned long long* red;
    bool it32_valid, old32_valid, it64_valid;
    bool timing;
    hipEvent_t ev0, ev1;
    double t_ms[2];
    long t_n[2];
    std::vector<double> hist_r;
    std::vector<int> hist_p;
    // 2D: tables and tile list of the tile kernel (one model, tile shape 0)
    ep::SweepArgs<double>* tab64;
    ep::SweepArgs<float>* tab32;
    ep::TileRef* tiles;
    int* tcount;
    long ntiles;
    int grid2[2];
    ep::StepCtl ctl;
    double* vguess64[3];   // 3D: velocities of a supplied starting guess
    bool guess_ready;      // the next increment tries vguess64
    int freeze;            // 0 off, 1 the next sweep stores Lambda, 2 Lambda frozen
    bool lam_in32;         // the frozen Lambda is in lam32 (else lam64)
    bool late;             // the increment's return uses pt_blend_late
    bool in_batch;         // owned by an ep_batch (ep_destroy ignores it)
    char err[512];
};

namespace ep {

SweepArgs<double> args64(const ep_handle* h, bool physical, int from);
SweepArgs<float> args32(const ep_handle* h, int from);
void ensure_it32(ep_handle* h);
void ensure_it64(ep_handle* h);
int set_err(ep_handle* h, int code, const char* fmt, ...);
int validate(const ep_params* p);
// Workspace bytes of one model (with h: also assign its device pointers).
size_t carve(const ep_params* p, ep_handle* h, char* base);
// Create a handle in d_workspace (carve(p) bytes, 256-byte aligned) and set
// the initial state; p must be valid.
void handle_free(ep_handle* h);
// (Re-)write the device tables of the 2D tile kernel (after h->red moved).
int upload_tables(ep_handle* h);
// LAM_* mode of sweep b of the next batch of sweeps.
int sweep_lam_mode(const ep_handle* h, int b);
int handle_create(const ep_params* p, const double* cohesion, char* d_workspace, hipStream_t stream,
                  ep_handle** out);

// Increment driver in pieces.  The device work of each piece is queued on the
// handle's stream; the pieces that take reduction values expect the caller to
// have read them after a synchronisation.
//  step_begin:  prologue (increment-start stresses, wall velocities, saved
//               velocities) and the physical evaluation of the plain guess
//               into h->red.
//  step_start:  from that reduction: reference residual, divergence check of
//               the start state, physical start; returns EP_OK or a failure
//               code (state rolled back, stats filled).
//  step_check:  after nb sweeps in the current precision and their check
//               reduction: history, divergence, precision hand-over,
//               convergence; returns whether the increment continues.
//  step_finish: for a converged increment queue the epilogue kernels and
//               return EP_OK; otherwise roll back and return the status.
//  step_report: after step_finish(EP_OK) and a synchronisation, fill the
//               diagnostics from h->red and the column integrals.
void step_begin(ep_handle* h, ep_step_stats* st);
int step_start(ep_handle* h, const double red[RED_N]);
bool step_check(ep_handle* h, const double red[RED_N], int nb);
//  step_certify_launch / step_certify: after a check that set
//               ctl.cert_pending, the physical evaluation of the current
//               velocities; its FP64 momentum residual (read after a
//               synchronisation) accepts the increment with those stresses,
//               or the iteration continues.
void step_certify_launch(ep_handle* h);
bool step_certify(ep_handle* h, const double red[RED_N]);
// freeze and iteration-cap decisions after a check that did not converge
void check_limits(ep_handle* h);
int step_finish(ep_handle* h);
void step_report(ep_handle* h, const double red[RED_N], const double cols[4]);
// Reduction slots as doubles (raw uint64 patterns; RED_NYIELD is a count).
void decode_red(const unsigned long long raw[RED_N], double out[RED_N]);

}  // namespace ep
