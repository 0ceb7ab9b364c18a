// Host runtime of libep.so: parameter checks, workspace carving, the
// per-increment driver (prologue, PT loop with residual checks, precision
// switch, epilogue) and field I/O.  Everything that runs per point runs in
// the kernels of ep_sweep_*.hip and ep_aux.hip.
#include <hip/hip_runtime.h>

#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "ep.h"
#include "ep_handle.h"
#include "ep_internal.h"

using namespace ep;


namespace ep {

const double PI = 3.14159265358979323846;

int set_err(ep_handle* h, int code, const char* fmt, ...)
{
    if (h) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(h->err, sizeof(h->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIPCHK(h, x)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess)                                                               \
            return set_err((h), EP_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_));    \
    } while (0)

bool field_exists_it(int ndim, int f) { return ndim == 3 || (f != F_VZ && f != F_TXZ && f != F_TYZ); }
bool field_exists_old(int ndim, int f) { return ndim == 3 || (f != O_TXZ && f != O_TYZ); }
bool field_exists_e(int ndim, int f) { return ndim == 3 || f == 0 || f == 1 || f == 3; }

int validate(const ep_params* p)
{
    if (!p) return EP_EINVAL;
    if (p->ndim != 2 && p->ndim != 3) return EP_EINVAL;
    if (p->nx < 3 || p->ny < 3 || (p->ndim == 3 && p->nz < 3)) return EP_EINVAL;
    if (!(p->lx > 0) || !(p->ly > 0) || (p->ndim == 3 && !(p->lz > 0))) return EP_EINVAL;
    if (!(p->bulk > 0) || !(p->shear > 0) || !(p->visc > 0) || !(p->dt > 0) || !(p->tol > 0)) return EP_EINVAL;
    if (!(p->psi_deg >= 0.0) || p->psi_deg > p->phi_deg) return EP_EINVAL;
    if (p->max_iter <= 0 || p->n_check < 0) return EP_EINVAL;
    if (p->cfl < 0 || p->re < 0 || p->r < 0) return EP_EINVAL;
    if (p->cfl > 0 && p->cfl >= 1.0 / std::sqrt((double)p->ndim)) return EP_EINVAL;
    if (p->precision != EP_FP64 && p->precision != EP_FP32_FIELDS) return EP_EINVAL;
    if (p->sweep < EP_SWEEP_AUTO || p->sweep > EP_SWEEP_UNFUSED) return EP_EINVAL;
    if (p->freeze_iter < 0 || p->guess_accept < 0) return EP_EINVAL;
    if (p->objective != 0 && p->objective != 1) return EP_EINVAL;
    if (!(p->eta_vp >= 0.0) || std::isinf(p->eta_vp)) return EP_EINVAL;
    if (!(p->pt_blend >= 0.0 && p->pt_blend <= 1.0)) return EP_EINVAL;
    if (!(p->pt_blend_late >= 0.0 && p->pt_blend_late <= 1.0)) return EP_EINVAL;
    return EP_OK;
}

// Walk the workspace layout; with h != nullptr assign the pointers.
size_t carve(const ep_params* p, ep_handle* h, char* base)
{
    const int nx = p->nx, ny = p->ny, nz = p->ndim == 3 ? p->nz : 0;
    const long sy = ((nx + 1) + 31) / 32 * 32;
    const long sz = sy * (ny + 1);
    const long nelem = sz * (p->ndim == 3 ? nz + 1 : 1);
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) / 256 * 256;
        char* r = base ? base + off : nullptr;
        off += bytes;
        return r;
    };
    const size_t b64 = nelem * sizeof(double), b32 = nelem * sizeof(float);
    const bool fp32 = p->precision == EP_FP32_FIELDS;
    for (int b = 0; b < 2; ++b)
        for (int f = 0; f < F_NIT; ++f) {
            char* q = field_exists_it(p->ndim, f) ? take(b64) : nullptr;
            if (h) h->it64[b][f] = (double*)q;
        }
    for (int f = 0; f < O_N; ++f) {
        char* q = field_exists_old(p->ndim, f) ? take(b64) : nullptr;
        if (h) h->old64[f] = (double*)q;
    }
    char* q;
    q = take(b64); if (h) h->coh64 = (double*)q;
    q = take(b64); if (h) h->lam64 = (double*)q;
    q = take(b64); if (h) h->igdc64 = (double*)q;
    for (int d = 0; d < 3; ++d) {
        char* a = d < p->ndim ? take(b64) : nullptr;
        char* u = d < p->ndim ? take(b64) : nullptr;
        if (h) { h->vstart64[d] = (double*)a; h->u64[d] = (double*)u; }
    }
    for (int f = 0; f < 6; ++f) {
        q = field_exists_e(p->ndim, f) ? take(b64) : nullptr;
        if (h) h->e64[f] = (double*)q;
    }
    q = take(b64); if (h) h->epsp64 = (double*)q;
    q = take(b64); if (h) h->lamdot64 = (double*)q;
    q = take(b64); if (h) h->tii64 = (double*)q;
    q = take(b64); if (h) h->yld64 = (double*)q;
    q = take(4 * sizeof(double)); if (h) h->cols64 = (double*)q;
    q = take(RED_N * sizeof(unsigned long long)); if (h) h->red = (unsigned long long*)q;
    for (int b = 0; b < 2; ++b)
        for (int f = 0; f < F_NIT; ++f) {
            q = fp32 && field_exists_it(p->ndim, f) ? take(b32) : nullptr;
            if (h) h->it32[b][f] = (float*)q;
        }
    for (int f = 0; f < O_N; ++f) {
        q = fp32 && field_exists_old(p->ndim, f) ? take(b32) : nullptr;
        if (h) h->old32[f] = (float*)q;
    }
    q = fp32 ? take(b32) : nullptr; if (h) h->coh32 = (float*)q;
    q = fp32 ? take(b32) : nullptr; if (h) h->igdc32 = (float*)q;
    q = fp32 ? take(b32) : nullptr; if (h) h->lam32 = (float*)q;
    for (int d = 0; d < 3; ++d) {
        q = d < p->ndim ? take(b64) : nullptr;
        if (h) h->vguess64[d] = (double*)q;
    }
    if (p->ndim == 2) {
        const long nt = (long)((nx + kBatchTiles[SINGLE_SHAPE][0] - 1) / kBatchTiles[SINGLE_SHAPE][0]) *
                        ((ny + kBatchTiles[SINGLE_SHAPE][1] - 1) / kBatchTiles[SINGLE_SHAPE][1]);
        q = take(10 * sizeof(SweepArgs<double>)); if (h) h->tab64 = (SweepArgs<double>*)q;
        q = take(6 * sizeof(SweepArgs<float>)); if (h) h->tab32 = (SweepArgs<float>*)q;
        q = take(nt * sizeof(TileRef)); if (h) h->tiles = (TileRef*)q;
        q = take(sizeof(int)); if (h) h->tcount = (int*)q;
        if (h) h->ntiles = nt;
    }
    if (h) {
        h->sy = (int)sy;
        h->sz = sz;
        h->nelem = nelem;
    }
    return (off + 255) / 256 * 256;
}

void derive(ep_handle* h)
{
    const ep_params& p = h->prm;
    h->ndim = p.ndim;
    h->nx = p.nx;
    h->ny = p.ny;
    h->nz = p.ndim == 3 ? p.nz : 0;
    h->dx = p.lx / p.nx;
    h->dy = p.ly / p.ny;
    h->dz = p.ndim == 3 ? p.lz / p.nz : 1.0;
    h->inv_mus = std::isinf(p.visc) ? 0.0 : 1.0 / p.visc;
    const double ph = p.phi_deg * PI / 180.0, ps = p.psi_deg * PI / 180.0;
    if (p.ndim == 2) {
        h->A = std::sin(ph);
        h->B = std::cos(ph);
        h->C = std::sin(ps);
    } else {
        const double den = std::sqrt(3.0) * (3.0 - std::sin(ph));
        h->A = 6.0 * std::sin(ph) / den;
        h->B = 6.0 * std::cos(ph) / den;
        h->C = 6.0 * std::sin(ps) / (std::sqrt(3.0) * (3.0 - std::sin(ps)));
    }
    const double re = p.re > 0 ? p.re : 3.0 * std::sqrt(10.0) * PI / 2.0;
    const double cfl = p.cfl > 0 ? p.cfl : 0.9 / std::sqrt((double)p.ndim);
    const double r = p.r > 0 ? p.r : 0.5;
    h->eta = 1.0 / (1.0 / (p.shear * p.dt) + h->inv_mus);
    h->h = std::fmin(h->dx, h->dy);
    h->L = std::fmax(p.lx, p.ly);
    if (p.ndim == 3) {
        h->h = std::fmin(h->h, h->dz);
        h->L = std::fmax(h->L, p.lz);
    }
    // Vtilde dtau = cfl h; rho~ = Re eta / (V~ L); G~ = rho~ V~^2 / (r + 4/3); K~ = r G~
    h->gdtau = re * h->eta * cfl * h->h / (h->L * (r + 4.0 / 3.0));
    h->kdtau = r * h->gdtau;
    h->dtrho = cfl * h->h * h->L / (re * h->eta);
    const double emax = std::fmax(std::fabs(p.erate[0]), std::fmax(std::fabs(p.erate[1]), std::fabs(p.erate[2])));
    h->dsig_ref = 2.0 * p.shear * emax * p.dt;
    h->n_check = p.n_check > 0 ? p.n_check : (p.ndim == 3 ? 10 : 100);
    h->fp32 = p.precision == EP_FP32_FIELDS;
    h->g.ndim = p.ndim;
    h->g.nx = h->nx;
    h->g.ny = h->ny;
    h->g.nz = h->nz;
}

template <typename R>
SweepArgs<R> make_args(const ep_handle* h, R* const* from, R* const* to, R* const* old, const R* coh, R* lam,
                       bool physical)
{
    SweepArgs<R> a;
    for (int f = 0; f < F_NIT; ++f) {
        a.it[f] = from[f];
        a.nx_[f] = to[f];
    }
    for (int f = 0; f < O_N; ++f) a.old[f] = old[f];
    a.coh = coh;
    a.lam = lam;
    a.red = h->red;
    a.nx = h->nx;
    a.ny = h->ny;
    a.nz = h->nz;
    a.sy = h->sy;
    a.sz = h->sz;
    a.idx = (R)(1.0 / h->dx);
    a.idy = (R)(1.0 / h->dy);
    a.idz = (R)(1.0 / h->dz);
    const double igt = physical ? 0.0 : 1.0 / h->gdtau;
    // incompressible limit (K = +inf, 1/(K dt) = 0): the pressure has no local
    // physical law, so a physical evaluation keeps its pseudo-time term
    const bool incompressible = std::isinf(h->prm.bulk);
    const double ikt = (physical && !incompressible) ? 0.0 : 1.0 / h->kdtau;
    const double igd = 1.0 / (h->prm.shear * h->prm.dt);
    const double ikd = 1.0 / (h->prm.bulk * h->prm.dt);
    a.igt = (R)igt;
    a.ikt = (R)ikt;
    a.igd = (R)igd;
    a.ikd = (R)ikd;
    a.D = (R)(igt + igd + h->inv_mus);
    a.invD = (R)(1.0 / (igt + igd + h->inv_mus));
    a.Dp = (R)(igd + h->inv_mus);
    a.invDp = (R)(1.0 / (igd + h->inv_mus));
    a.blend = (R)(h->late ? h->prm.pt_blend_late : h->prm.pt_blend);
    a.ikk = (R)(1.0 / (ikt + ikd));
    a.dtrho = (R)h->dtrho;
    a.A = (R)h->A;
    a.B = (R)h->B;
    // dilatancy (psi > 0): pressure change per unit plastic rate in this update
    a.Cik = (R)(h->C / (ikt + ikd));
    a.vp = (R)h->prm.eta_vp;
    a.imus = (R)h->inv_mus;
    a.igdc = nullptr;
    if (h->has_g) {
        if constexpr (sizeof(R) == 4) a.igdc = h->igdc32;
        else a.igdc = h->igdc64;
    }
    // pressure residual factor: K dt, or the visco-elastic viscosity in the
    // incompressible limit (the pressure rate is then the divergence)
    a.rK = (R)((incompressible ? h->eta : h->prm.bulk * h->prm.dt) / (h->kdtau * h->L));
    a.rG = (R)(h->eta / (h->gdtau * h->L));
    // FP32 velocity fields store the deviation from the background field
    const bool bg = sizeof(R) == 4;
    a.ebx = (R)(bg ? h->prm.erate[0] : 0.0);
    a.eby = (R)(bg ? h->prm.erate[1] : 0.0);
    a.ebz = (R)(bg && h->ndim == 3 ? h->prm.erate[2] : 0.0);
    a.lam_mode = LAM_COMPUTE;
    // the workspace takes the fields of a group one after the other, equal
    // sizes, equal alignment: a uniform stride in 3D (checked here)
    a.fs = 0;
    if (h->ndim == 3) {
        const long fs = from[1] - from[0];
        bool ok = fs > 0;
        for (int f = 0; f < F_NIT; ++f) ok = ok && from[f] == from[0] + f * fs && to[f] == to[0] + f * fs;
        for (int f = 0; f < O_N; ++f) ok = ok && old[f] == old[0] + f * fs;
        if (ok) a.fs = fs;
    }
    return a;
}

double face_len(const ep_handle* h, int d) { return d == 0 ? h->prm.lx : d == 1 ? h->prm.ly : h->prm.lz; }
double face_sp(const ep_handle* h, int d) { return d == 0 ? h->dx : d == 1 ? h->dy : h->dz; }

SweepArgs<double> args64(const ep_handle* h, bool physical, int from)
{
    return make_args<double>(h, h->it64[from], h->it64[1 - from], h->old64, h->coh64, h->lam64, physical);
}
SweepArgs<float> args32(const ep_handle* h, int from)
{
    return make_args<float>(h, h->it32[from], h->it32[1 - from], h->old32, h->coh32, h->lam32, false);
}

// One PT sweep reading buffer `from` (physical: pseudo-time terms removed;
// lam_mode: LAM_*, 2D tile sweeps only).  2D fused sweeps run the batched
// tile kernel on this model's own one-entry table and tile list, so that a
// model gives bitwise the same iterates alone and inside a batch.
template <typename R>
void launch_sweep(const ep_handle* h, bool physical, int from, int mode, int lam_mode = LAM_COMPUTE)
{
    const bool fused = sizeof(R) == 4 ? h->fused32 : h->fused64;
    if (h->ndim == 2 && fused) {
        if (sizeof(R) == 4)
            launch_sweep_batch_2d<float>(SINGLE_SHAPE, h->tab32 + 2 * lam_mode + from, h->tiles, h->tcount, mode,
                                         h->grid2[1], h->st);
        else
            launch_sweep_batch_2d<double>(SINGLE_SHAPE,
                                          h->tab64 + (physical ? 6 + 2 * (lam_mode == LAM_FROZEN) : 2 * lam_mode) + from,
                                          h->tiles, h->tcount, mode, h->grid2[0], h->st);
        return;
    }
    SweepArgs<R> a;
    if constexpr (sizeof(R) == 4) a = args32(h, from);
    else a = args64(h, physical, from);
    a.lam_mode = lam_mode;
    if (h->ndim == 2) {
        launch_sweep_unfused_2d<R>(a, mode, h->st);
    } else {
        if (fused && a.fs > 0) launch_sweep_fused_3d<R>(a, mode, h->st);
        else launch_sweep_unfused_3d<R>(a, mode, h->st);
    }
}

// Device tables of the 2D tile kernel: FP64 [lam mode][from], then physical
// [from] and physical with the frozen Lambda [from]; FP32 [lam mode][from].
// The tile list (shape 0) is written once.
int upload_tables(ep_handle* h)
{
    if (h->ndim != 2) return EP_OK;
    SweepArgs<double> t64[10];
    SweepArgs<float> t32[6];
    for (int lm = 0; lm < 3; ++lm)
        for (int from = 0; from < 2; ++from) {
            t64[2 * lm + from] = args64(h, false, from);
            t64[2 * lm + from].lam_mode = lm;
            if (h->fp32) {
                t32[2 * lm + from] = args32(h, from);
                t32[2 * lm + from].lam_mode = lm;
            }
        }
    for (int from = 0; from < 2; ++from) {
        t64[6 + from] = args64(h, true, from);
        t64[8 + from] = args64(h, true, from);
        t64[8 + from].lam_mode = LAM_FROZEN;
    }
    HIPCHK(h, hipMemcpyAsync(h->tab64, t64, sizeof(t64), hipMemcpyHostToDevice, h->st));
    if (h->fp32) HIPCHK(h, hipMemcpyAsync(h->tab32, t32, sizeof(t32), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return EP_OK;
}

void decode_red(const unsigned long long raw[RED_N], double out[RED_N])
{
    for (int q = 0; q < RED_N; ++q) {
        double d;
        std::memcpy(&d, &raw[q], sizeof(d));
        out[q] = d;
    }
    out[RED_NYIELD] = (double)raw[RED_NYIELD];
}

int read_red(ep_handle* h, double out[RED_N])
{
    unsigned long long raw[RED_N];
    HIPCHK(h, hipMemcpyAsync(raw, h->red, sizeof(raw), hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    HIPCHK(h, hipGetLastError());
    decode_red(raw, out);
    return EP_OK;
}

void copy_it64(ep_handle* h, double* const* dst, double* const* src)
{
    for (int f = 0; f < F_NIT; ++f)
        if (dst[f]) launch_copy(dst[f], src[f], h->nelem, h->st);
}

// Make it64[cur64] current after FP32 sweeps (stresses in increment form).
void ensure_it64(ep_handle* h)
{
    if (h->it64_valid) return;
    if (h->freeze == 2 && h->lam_in32) {     // Lambda frozen by an FP32 sweep
        launch_to_f64(h->lam64, h->lam32, h->nelem, h->st);
        h->lam_in32 = false;
    }
    for (int f = 0; f < F_NIT; ++f) {
        if (!h->it64[h->cur64][f]) continue;
        int o = f == F_P ? O_P : f == F_TXX ? O_TXX : f == F_TYY ? O_TYY : f == F_TXY ? O_TXY
              : f == F_TXZ ? O_TXZ : f == F_TYZ ? O_TYZ : -1;
        if (o >= 0)
            launch_incr_to_f64(h->it64[h->cur64][f], h->old64[o], h->it32[h->cur32][f], h->old32[o], h->nelem, h->st);
        else                                    // velocity: add the background back
            launch_vel_to_f64(h->g, f - F_VX, h->it64[h->cur64][f], h->it32[h->cur32][f], h->prm.erate[f - F_VX],
                              face_len(h, f - F_VX), face_sp(h, f - F_VX), h->st);
    }
    h->it64_valid = true;
}

void ensure_it32(ep_handle* h)
{
    if (!h->fp32) return;
    if (!h->old32_valid) {
        for (int o = 0; o < O_N; ++o)
            if (h->old64[o]) launch_to_f32(h->old32[o], h->old64[o], h->nelem, h->st);
        launch_to_f32(h->coh32, h->coh64, h->nelem, h->st);
        if (h->has_g) launch_to_f32(h->igdc32, h->igdc64, h->nelem, h->st);
        h->old32_valid = true;
    }
    if (!h->it32_valid) {
        for (int f = 0; f < F_NIT; ++f) {
            if (!h->it64[h->cur64][f]) continue;
            if (f <= F_VZ)                      // velocity: store the deviation from the background
                launch_vel_to_f32(h->g, f, h->it32[h->cur32][f], h->it64[h->cur64][f], h->prm.erate[f],
                                  face_len(h, f), face_sp(h, f), h->st);
            else
                launch_to_f32(h->it32[h->cur32][f], h->it64[h->cur64][f], h->nelem, h->st);
        }
        h->it32_valid = true;
    }
}

// Lambda mode of sweep b of a batch: the first sweep after a freeze decision
// stores Lambda, every later sweep reads it.
int sweep_lam_mode(const ep_handle* h, int b)
{
    if (h->freeze == 0) return LAM_COMPUTE;
    return (h->freeze == 1 && b == 0) ? LAM_STORE : LAM_FROZEN;
}

// Run nb sweeps in one precision; the last one reduces the residual.
int run_batch(ep_handle* h, bool use32, int nb, bool check_last)
{
    if (h->timing) HIPCHK(h, hipEventRecord(h->ev0, h->st));
    launch_reset_red(h->red, h->st);
    for (int b = 0; b < nb; ++b) {
        int mode = (check_last && b == nb - 1) ? MODE_CHECK : MODE_UPDATE;
        const int lm = sweep_lam_mode(h, b);
        if (use32) {
            launch_sweep<float>(h, false, h->cur32, mode, lm);
            h->cur32 = 1 - h->cur32;
        } else {
            launch_sweep<double>(h, false, h->cur64, mode, lm);
            h->cur64 = 1 - h->cur64;
        }
    }
    if (h->freeze == 1 && nb > 0) {
        h->freeze = 2;
        h->lam_in32 = use32;
    }
    if (use32) h->it64_valid = false;
    else h->it32_valid = false;
    if (h->timing) HIPCHK(h, hipEventRecord(h->ev1, h->st));
    HIPCHK(h, hipGetLastError());
    return EP_OK;
}

void add_timing(ep_handle* h, bool use32, int nb)
{
    if (!h->timing) return;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) {
        h->t_ms[use32 ? 1 : 0] += ms;
        h->t_n[use32 ? 1 : 0] += nb;
    }
}

void roll_back(ep_handle* h)
{
    double** it = h->it64[h->cur64];
    for (int d = 0; d < h->ndim; ++d) launch_copy(it[F_VX + d], h->vstart64[d], h->nelem, h->st);
    const int map[O_N] = {F_P, F_TXX, F_TYY, F_TXY, F_TXZ, F_TYZ};
    for (int o = 0; o < O_N; ++o)
        if (h->old64[o]) launch_copy(it[map[o]], h->old64[o], h->nelem, h->st);
    h->it64_valid = true;
    h->it32_valid = false;
}

double seconds_since(const StepCtl& c)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - c.t0).count();
}

// Objective update of the FP64 state in place, through the increment-start
// arrays (which end up holding the updated stresses too).
void objective_update(ep_handle* h)
{
    ensure_it64(h);
    double** it = h->it64[h->cur64];
    const int map[O_N] = {F_P, F_TXX, F_TYY, F_TXY, F_TXZ, F_TYZ};
    ObjectiveArgs oa{};
    for (int f = 0; f < F_NIT; ++f) oa.in[f] = it[f];
    for (int o = 0; o < O_N; ++o) oa.out[map[o]] = h->old64[o];
    oa.dx = h->dx;
    oa.dy = h->dy;
    oa.dz = h->dz;
    oa.dt = h->prm.dt;
    launch_objective(h->g, oa, h->st);
    for (int o = 0; o < O_N; ++o)
        if (h->old64[o]) launch_copy(it[map[o]], h->old64[o], h->nelem, h->st);
    h->it32_valid = false;
    h->old32_valid = false;
}

void step_begin(ep_handle* h, ep_step_stats* st)
{
    StepCtl& c = h->ctl;
    c = StepCtl();
    c.st = st;
    c.t0 = std::chrono::steady_clock::now();
    c.running = false;
    c.status = EP_ENOTCONV;
    c.resid = NAN;
    c.vmax = 0;
    std::memset(st, 0, sizeof(*st));
    h->freeze = 0;
    h->lam_in32 = false;
    if (h->late) {
        h->late = false;
        if (!h->in_batch) upload_tables(h);
    }

    // increment start state and wall velocities
    ensure_it64(h);
    double** it = h->it64[h->cur64];
    const int map[O_N] = {F_P, F_TXX, F_TYY, F_TXY, F_TXZ, F_TYZ};
    if (h->prm.objective) {
        // objective update of the carried stresses with the previous
        // increment's velocities: the result is this increment's start
        objective_update(h);
    } else {
        for (int o = 0; o < O_N; ++o)
            if (h->old64[o]) launch_copy(h->old64[o], it[map[o]], h->nelem, h->st);
    }
    launch_set_walls(h->g, it[F_VX], it[F_VY], it[F_VZ], h->prm.erate, h->prm.lx, h->prm.ly, h->prm.lz, h->st);
    for (int d = 0; d < h->ndim; ++d) launch_copy(h->vstart64[d], it[F_VX + d], h->nelem, h->st);
    h->it32_valid = false;
    h->old32_valid = false;
    // normaliser: physical residual of the plain guess
    launch_reset_red(h->red, h->st);
    launch_sweep<double>(h, true, h->cur64, MODE_PHYS);
}

int step_start(ep_handle* h, const double red[RED_N])
{
    StepCtl& c = h->ctl;
    ep_step_stats* st = c.st;
    st->r_ref = red[RED_MOM];
    st->ref = std::fmax(st->r_ref, h->dsig_ref / h->L);
    if (!(st->r_ref <= 1e300)) {            // NaN / Inf in the starting state
        st->status = EP_EDIVERGED;
        c.status = EP_EDIVERGED;
        roll_back(h);
        st->seconds = seconds_since(c);
        return EP_EDIVERGED;
    }
    if (h->guess_ready) {
        // a supplied guess replaces the plain one when its physical stresses
        // balance better; the normaliser stays that of the plain guess
        h->guess_ready = false;
        double** it = h->it64[h->cur64];
        for (int d = 0; d < h->ndim; ++d) launch_copy(it[F_VX + d], h->vguess64[d], h->nelem, h->st);
        launch_set_walls(h->g, it[F_VX], it[F_VY], it[F_VZ], h->prm.erate, h->prm.lx, h->prm.ly, h->prm.lz, h->st);
        launch_reset_red(h->red, h->st);
        launch_sweep<double>(h, true, h->cur64, MODE_PHYS);
        double rg[RED_N];
        int rc = read_red(h, rg);
        if (rc) return rc;
        st->r_guess = rg[RED_MOM];
        const double accept = h->prm.guess_accept > 0 ? h->prm.guess_accept : 1.0;
        if (rg[RED_MOM] < accept * st->r_ref) {
            st->guess_used = 1;
        } else {
            for (int d = 0; d < h->ndim; ++d)
                launch_copy(h->it64[h->cur64][F_VX + d], h->vstart64[d], h->nelem, h->st);
            launch_reset_red(h->red, h->st);
            launch_sweep<double>(h, true, h->cur64, MODE_PHYS);
        }
    }
    // the physical stresses just written to the other buffer are the
    // pseudo-time starting point; the velocities carry over unchanged
    for (int d = 0; d < h->ndim; ++d)
        launch_copy(h->it64[1 - h->cur64][F_VX + d], h->it64[h->cur64][F_VX + d], h->nelem, h->st);
    h->cur64 = 1 - h->cur64;
    h->hist_r.clear();
    h->hist_p.clear();

    c.tol_abs = h->prm.tol * st->ref;
    // a starting state that already meets the tolerance is accepted as it is:
    // its stresses are the physical ones, its residual the certificate
    const double r_start = st->guess_used == 1 ? st->r_guess : st->r_ref;
    if (r_start <= c.tol_abs) {
        st->cert = r_start;
        c.resid = r_start;
        c.status = EP_OK;
        c.running = false;
        return EP_OK;
    }
    c.sw = (h->prm.fp32_switch > 0 ? h->prm.fp32_switch : 2.0 * h->prm.tol) * st->ref;
    c.use32 = h->fp32;
    if (c.use32) ensure_it32(h);
    const int nmax = std::max(h->nx, std::max(h->ny, h->nz));
    c.stall_checks = h->prm.fp32_stall > 0 ? h->prm.fp32_stall
                   : h->prm.fp32_stall < 0 ? INT_MAX : std::max(8, 16 * nmax / h->n_check);
    c.best = INFINITY;
    c.since_best = 0;
    c.running = true;
    return EP_OK;
}

bool step_check(ep_handle* h, const double red[RED_N], int nb)
{
    StepCtl& c = h->ctl;
    ep_step_stats* st = c.st;
    st->iters += nb;
    if (c.use32) st->iters_fp32 += nb;
    c.resid = red[RED_RESID];
    c.vmax = red[RED_VMAX];
    h->hist_r.push_back(c.resid / st->ref);
    h->hist_p.push_back(c.use32 ? EP_FP32_FIELDS : EP_FP64);
    if (!(c.resid <= 1e8 * st->ref)) {
        c.status = EP_EDIVERGED;
        c.running = false;
    } else if (c.use32) {
        // FP32 rounding of the stresses bounds what an FP32 sweep can
        // resolve: about 8 u32 max|sigma| / h in residual units (measured:
        // 2-3 times that on a converged 3D plastic increment, up to ~10
        // times on frozen 2D increments).  Above that multiple (3 in 3D, 10
        // in 2D) FP32 keeps iterating, also through plateaus where the
        // yielding zone reorganises; there, or within 2x of the tolerance,
        // or after a stall within 20x of the floor, or after a 4x longer
        // stall anywhere, FP64 sweeps take over.
        const double floor32 = 8.0 * 5.96e-8 * red[RED_SMAX] / h->h;
        const double at_floor = (h->ndim == 3 ? 3.0 : 10.0) * floor32;
        if (c.resid < 0.5 * c.best) {
            c.best = c.resid;
            c.since_best = 0;
        } else {
            ++c.since_best;
        }
        const bool near_floor = c.resid <= 20.0 * floor32;
        const bool stalled = c.since_best >= c.stall_checks;
        if (c.resid <= std::max(c.sw, at_floor) || (near_floor && stalled) ||
            c.since_best / 4 >= c.stall_checks) {
            ensure_it64(h);          // continue from the FP32 state in FP64
            c.use32 = false;
            st->fp32_exit = c.resid / st->ref;
        }
    } else if (c.resid <= c.tol_abs) {
        // acceptance needs the certificate (step_certify_launch, step_certify)
        c.cert_pending = true;
        return true;
    }
    check_limits(h);
    return c.running;
}

void check_limits(ep_handle* h)
{
    StepCtl& c = h->ctl;
    ep_step_stats* st = c.st;
    // the return's blend changes once, at the first check at or after
    // 16 max(nx, ny, nz) iterations
    if (c.running && !h->late && st->iters >= 16 * std::max(h->nx, std::max(h->ny, h->nz))) {
        h->late = true;
        if (!h->in_batch) upload_tables(h);
    }
    // frozen plasticity: still iterating at freeze_iter -> the next sweep
    // stores its centre Lambda and later sweeps hold it fixed
    if (c.running && h->prm.freeze_iter > 0 && h->freeze == 0 && st->iters >= h->prm.freeze_iter) {
        h->freeze = 1;
        st->frozen_at = st->iters;
    }
    if (c.running && st->iters >= h->prm.max_iter) {
        c.status = EP_ENOTCONV;
        c.running = false;
    }
}

void step_certify_launch(ep_handle* h)
{
    // physical stresses of the current velocities (the held Lambda when
    // frozen) into the other buffer, their momentum residual into h->red
    launch_reset_red(h->red, h->st);
    launch_sweep<double>(h, true, h->cur64, MODE_PHYS, h->freeze == 2 ? LAM_FROZEN : LAM_COMPUTE);
}

bool step_certify(ep_handle* h, const double red[RED_N])
{
    StepCtl& c = h->ctl;
    c.cert_pending = false;
    if (red[RED_MOM] <= c.tol_abs) {
        // accepted: the physical stresses with the current velocities
        for (int d = 0; d < h->ndim; ++d)
            launch_copy(h->it64[1 - h->cur64][F_VX + d], h->it64[h->cur64][F_VX + d], h->nelem, h->st);
        h->cur64 = 1 - h->cur64;
        h->it32_valid = false;
        c.st->cert = red[RED_MOM];
        c.status = EP_OK;
        c.running = false;
        return false;
    }
    check_limits(h);
    return c.running;
}

int step_finish(ep_handle* h)
{
    h->freeze = 0;                  // sweeps outside an increment compute Lambda
    if (h->late) {                  // ... with the first blend
        h->late = false;
        if (!h->in_batch) upload_tables(h);
    }
    StepCtl& c = h->ctl;
    ep_step_stats* st = c.st;
    st->resid = c.resid;
    st->eps_rel = c.vmax > 0 ? h->dtrho * c.resid / c.vmax : 0.0;
    st->status = c.status;
    if (c.status != EP_OK) {
        ensure_it64(h);
        roll_back(h);
        st->seconds = seconds_since(c);
        return c.status;
    }
    // diagnostics of the accepted state, FP64 accumulators
    launch_reset_red(h->red, h->st);
    launch_diagnostics<double>(args64(h, true, h->cur64), h->lamdot64, h->tii64, h->yld64, h->st);
    double** it = h->it64[h->cur64];
    const double* v[3] = {it[F_VX], it[F_VY], it[F_VZ]};
    launch_accumulate(h->g, h->prm.dt, 1.0 / h->dx, 1.0 / h->dy, 1.0 / h->dz, v, h->u64, h->e64, h->epsp64,
                      h->lamdot64, h->st);
    launch_column_integrals(h->g, it[F_P], it[F_TXX], h->dy, h->dz, h->cols64, h->st);
    return EP_OK;
}

void step_report(ep_handle* h, const double red[RED_N], const double cols[4])
{
    ep_step_stats* st = h->ctl.st;
    st->sxx_left = cols[0];
    st->sxx_centre = cols[1];
    st->sxx_right = cols[2];
    st->n_yield = (long long)red[RED_NYIELD];
    st->max_violation = red[RED_VIOL] - 1.0;
    st->seconds = seconds_since(h->ctl);
}

struct FieldRef {
    double* dev;     // padded device array (nullptr for derived fields)
    int ext[3];      // staggered extents
    bool writable;
};

FieldRef field_ref(ep_handle* h, int f)
{
    const int nx = h->nx, ny = h->ny, nz = h->ndim == 3 ? h->nz : 1;
    const bool d3 = h->ndim == 3;
    FieldRef r{nullptr, {0, 0, 0}, false};
    auto set = [&](double* d, int a, int b, int c, bool w) { r.dev = d; r.ext[0] = a; r.ext[1] = b; r.ext[2] = c; r.writable = w; };
    double** it = h->it64[h->cur64];
    switch (f) {
    case EP_F_VX: set(it[F_VX], nx + 1, ny, nz, true); break;
    case EP_F_VY: set(it[F_VY], nx, ny + 1, nz, true); break;
    case EP_F_VZ: if (d3) set(it[F_VZ], nx, ny, nz + 1, true); break;
    case EP_F_P: set(it[F_P], nx, ny, nz, true); break;
    case EP_F_TXX: set(it[F_TXX], nx, ny, nz, true); break;
    case EP_F_TYY: set(it[F_TYY], nx, ny, nz, true); break;
    case EP_F_TZZ: if (d3) set(nullptr, nx, ny, nz, false); break;
    case EP_F_TXY: set(it[F_TXY], nx + 1, ny + 1, nz, true); break;
    case EP_F_TXZ: if (d3) set(it[F_TXZ], nx + 1, ny, nz + 1, true); break;
    case EP_F_TYZ: if (d3) set(it[F_TYZ], nx, ny + 1, nz + 1, true); break;
    case EP_F_P_OLD: set(h->old64[O_P], nx, ny, nz, true); break;
    case EP_F_TXX_OLD: set(h->old64[O_TXX], nx, ny, nz, true); break;
    case EP_F_TYY_OLD: set(h->old64[O_TYY], nx, ny, nz, true); break;
    case EP_F_TZZ_OLD: if (d3) set(nullptr, nx, ny, nz, false); break;
    case EP_F_TXY_OLD: set(h->old64[O_TXY], nx + 1, ny + 1, nz, true); break;
    case EP_F_TXZ_OLD: if (d3) set(h->old64[O_TXZ], nx + 1, ny, nz + 1, true); break;
    case EP_F_TYZ_OLD: if (d3) set(h->old64[O_TYZ], nx, ny + 1, nz + 1, true); break;
    case EP_F_UX: set(h->u64[0], nx + 1, ny, nz, true); break;
    case EP_F_UY: set(h->u64[1], nx, ny + 1, nz, true); break;
    case EP_F_UZ: if (d3) set(h->u64[2], nx, ny, nz + 1, true); break;
    case EP_F_EXX: set(h->e64[0], nx, ny, nz, true); break;
    case EP_F_EYY: set(h->e64[1], nx, ny, nz, true); break;
    case EP_F_EZZ: if (d3) set(h->e64[2], nx, ny, nz, true); break;
    case EP_F_EXY: set(h->e64[3], nx + 1, ny + 1, nz, true); break;
    case EP_F_EXZ: if (d3) set(h->e64[4], nx + 1, ny, nz + 1, true); break;
    case EP_F_EYZ: if (d3) set(h->e64[5], nx, ny + 1, nz + 1, true); break;
    case EP_F_EPS_P: set(h->epsp64, nx, ny, nz, true); break;
    case EP_F_COHESION: set(h->coh64, nx, ny, nz, true); break;
    case EP_F_LAMBDA_DOT: set(h->lamdot64, nx, ny, nz, false); break;
    case EP_F_TAU_II: set(h->tii64, nx, ny, nz, false); break;
    case EP_F_YIELD: set(h->yld64, nx, ny, nz, false); break;
    case EP_F_LAMBDA_FROZEN: if (!d3) set(h->lam64, nx, ny, nz, false); break;
    default: break;
    }
    return r;
}

int get_padded(ep_handle* h, const double* dev, std::vector<double>& buf)
{
    buf.resize(h->nelem);
    HIPCHK(h, hipMemcpyAsync(buf.data(), dev, h->nelem * sizeof(double), hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return EP_OK;
}

void gather(const ep_handle* h, const std::vector<double>& pad, const int ext[3], double* out)
{
    long q = 0;
    for (int k = 0; k < ext[2]; ++k)
        for (int j = 0; j < ext[1]; ++j)
            for (int i = 0; i < ext[0]; ++i) out[q++] = pad[i + (long)h->sy * j + h->sz * k];
}

void scatter(const ep_handle* h, const double* in, const int ext[3], std::vector<double>& pad)
{
    long q = 0;
    for (int k = 0; k < ext[2]; ++k)
        for (int j = 0; j < ext[1]; ++j)
            for (int i = 0; i < ext[0]; ++i) pad[i + (long)h->sy * j + h->sz * k] = in[q++];
}

int upload(ep_handle* h, double* dev, const double* in, const int ext[3])
{
    std::vector<double> pad;
    int rc = get_padded(h, dev, pad);
    if (rc) return rc;
    scatter(h, in, ext, pad);
    HIPCHK(h, hipMemcpyAsync(dev, pad.data(), h->nelem * sizeof(double), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return EP_OK;
}

int handle_create(const ep_params* p, const double* cohesion, char* d_workspace, hipStream_t stream,
                  ep_handle** out)
{
    *out = nullptr;
    const size_t need = carve(p, nullptr, nullptr);
    ep_handle* h = new (std::nothrow) ep_handle();
    if (!h) return EP_ENOMEM;
    h->prm = *p;
    h->st = stream;
    derive(h);
    carve(p, h, (char*)d_workspace);
    h->g.sy = h->sy;
    h->g.sz = h->sz;
    h->g.nelem = h->nelem;
    // EP_SWEEP_AUTO takes, per precision, the faster implementation measured on
    // MI355X; FUSED / UNFUSED force one for both precisions
    h->fused32 = p->sweep == EP_SWEEP_FUSED || (p->sweep == EP_SWEEP_AUTO && fused_preferred(p->ndim, true));
    h->fused64 = p->sweep == EP_SWEEP_FUSED || (p->sweep == EP_SWEEP_AUTO && fused_preferred(p->ndim, false));
    h->cur64 = 0;
    h->cur32 = 0;
    auto fail = [&](int code) { delete h; return code; };
    if (hipMemsetAsync(d_workspace, 0, need, h->st) != hipSuccess) return fail(EP_EDEVICE);
    if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) return fail(EP_EDEVICE);
    // cohesion and the background velocity field
    std::vector<double> pad(h->nelem, 0.0);
    const int nz1 = h->ndim == 3 ? h->nz : 1;
    if (cohesion) {
        int ext[3] = {h->nx, h->ny, nz1};
        scatter(h, cohesion, ext, pad);
        if (hipMemcpyAsync(h->coh64, pad.data(), h->nelem * sizeof(double), hipMemcpyHostToDevice, h->st) != hipSuccess)
            return fail(EP_EDEVICE);
        if (hipStreamSynchronize(h->st) != hipSuccess) return fail(EP_EDEVICE);
    }
    for (int d = 0; d < h->ndim; ++d) {
        std::fill(pad.begin(), pad.end(), 0.0);
        const int ex[3] = {h->nx + (d == 0), h->ny + (d == 1), nz1 + (d == 2)};
        const double len = d == 0 ? p->lx : d == 1 ? p->ly : p->lz;
        const double sp = d == 0 ? h->dx : d == 1 ? h->dy : h->dz;
        for (int k = 0; k < ex[2]; ++k)
            for (int j = 0; j < ex[1]; ++j)
                for (int i = 0; i < ex[0]; ++i) {
                    const int n = d == 0 ? i : d == 1 ? j : k;
                    pad[i + (long)h->sy * j + h->sz * k] = p->erate[d] * (-0.5 * len + n * sp);
                }
        if (hipMemcpyAsync(h->it64[0][F_VX + d], pad.data(), h->nelem * sizeof(double), hipMemcpyHostToDevice, h->st) !=
            hipSuccess)
            return fail(EP_EDEVICE);
        if (hipStreamSynchronize(h->st) != hipSuccess) return fail(EP_EDEVICE);
    }
    h->it64_valid = true;
    h->it32_valid = false;
    h->old32_valid = false;
    if (h->ndim == 2) {
        // tile list of the whole model and the persistent grid sizes
        const int tx = kBatchTiles[SINGLE_SHAPE][0], ty = kBatchTiles[SINGLE_SHAPE][1];
        const int nbx = (h->nx + tx - 1) / tx;
        std::vector<TileRef> tl(h->ntiles);
        for (long t = 0; t < h->ntiles; ++t) tl[t] = TileRef{0, (short)(t % nbx), (short)(t / nbx)};
        const int cnt = (int)h->ntiles;
        if (hipMemcpyAsync(h->tiles, tl.data(), tl.size() * sizeof(TileRef), hipMemcpyHostToDevice, h->st) !=
                hipSuccess ||
            hipMemcpyAsync(h->tcount, &cnt, sizeof(int), hipMemcpyHostToDevice, h->st) != hipSuccess ||
            hipStreamSynchronize(h->st) != hipSuccess)
            return fail(EP_EDEVICE);
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess || ncu <= 0) ncu = 256;
        h->grid2[0] =
            (int)std::min<long>(h->ntiles, (long)ncu * std::min(8, batch_blocks_per_cu<double>(SINGLE_SHAPE)));
        h->grid2[1] =
            (int)std::min<long>(h->ntiles, (long)ncu * std::min(8, batch_blocks_per_cu<float>(SINGLE_SHAPE)));
        if (upload_tables(h) != EP_OK) return fail(EP_EDEVICE);
    }
    if (hipGetLastError() != hipSuccess) return fail(EP_EDEVICE);
    *out = h;
    return EP_OK;
}

void handle_free(ep_handle* h)
{
    (void)hipEventDestroy(h->ev0);
    (void)hipEventDestroy(h->ev1);
    delete h;
}

// ---- allocation-free residual: the static device scratch ------------------
// File-scope device array that ep_residual_noalloc stages its reduction
// counters, sweep-argument tables and 2D tile list in (each GPU the library
// runs on holds one copy until the process ends).  Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
constexpr size_t NOALLOC_SCRATCH_BYTES = 64 * 1024;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// Layout: reduction counters, then two FP64 argument tables (PT and physical
// evaluation), then the tile count and the tile list (2D models).
constexpr size_t NA_RED = 0;
constexpr size_t NA_TAB = 256;
constexpr size_t NA_CNT = NA_TAB + (2 * sizeof(SweepArgs<double>) + 255) / 256 * 256;
constexpr size_t NA_TILES = NA_CNT + 256;
constexpr long NOALLOC_MAX_TILES = (long)((NOALLOC_SCRATCH_BYTES - NA_TILES) / sizeof(TileRef));

// Device address of `scratch` on the current device, looked up once per device.
int noalloc_scratch(ep_handle* h, char** out)
{
    static char* addr[64] = {};
    int dev = 0;
    HIPCHK(h, hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_err(h, EP_EDEVICE, "device %d out of range", dev);
    if (!addr[dev]) {
        void* ptr = nullptr;
        HIPCHK(h, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        addr[dev] = (char*)ptr;
    }
    *out = addr[dev];
    return EP_OK;
}

}  // namespace ep

// =========================================================================
extern "C" {

int ep_abi_version(void) { return EP_ABI_VERSION; }

int ep_workspace_size(const ep_params* p, size_t* bytes)
{
    if (!bytes || validate(p) != EP_OK) return EP_EINVAL;
    *bytes = carve(p, nullptr, nullptr);
    return EP_OK;
}

int ep_init(const ep_params* p, const double* cohesion, const double* shear, void* d_workspace, size_t ws_bytes,
            void* stream, ep_handle** out)
{
    if (!out) return EP_EINVAL;
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    if (!d_workspace || ws_bytes < carve(p, nullptr, nullptr)) return EP_ENOMEM;
    if (((uintptr_t)d_workspace & 255) != 0) return EP_EINVAL;
    if (shear) {            // checked before any device work
        const long nc = (long)p->nx * p->ny * (p->ndim == 3 ? p->nz : 1);
        for (long c = 0; c < nc; ++c)
            if (!(shear[c] > 0.0) || !(shear[c] <= p->shear)) return EP_EINVAL;
    }
    rc = handle_create(p, cohesion, (char*)d_workspace, (hipStream_t)stream, out);
    if (rc || !shear) return rc;
    rc = ep_set_shear_modulus(*out, shear);
    if (rc) {
        handle_free(*out);
        *out = nullptr;
    }
    return rc;
}

void ep_destroy(ep_handle* h)
{
    if (!h || h->in_batch) return;     // models of a batch belong to the batch
    handle_free(h);
}

const char* ep_last_error(const ep_handle* h) { return h ? h->err : "no handle"; }

int ep_enable_timing(ep_handle* h, int on)
{
    if (!h) return EP_EINVAL;
    h->timing = on != 0;
    h->t_ms[0] = h->t_ms[1] = 0;
    h->t_n[0] = h->t_n[1] = 0;
    return EP_OK;
}

int ep_sweep_timing(const ep_handle* h, int precision, double* avg_ms, long* sweeps)
{
    if (!h || (precision != EP_FP64 && precision != EP_FP32_FIELDS)) return EP_EINVAL;
    const int q = precision == EP_FP32_FIELDS ? 1 : 0;
    if (avg_ms) *avg_ms = h->t_n[q] ? h->t_ms[q] / h->t_n[q] : 0.0;
    if (sweeps) *sweeps = h->t_n[q];
    return EP_OK;
}

int ep_sweep(ep_handle* h, int n, double* resid)
{
    if (!h || n <= 0) return EP_EINVAL;
    int rc;
    if (h->fp32) {
        ensure_it32(h);
        rc = run_batch(h, true, n, true);
    } else {
        rc = run_batch(h, false, n, true);
    }
    if (rc) return rc;
    double red[RED_N];
    if ((rc = read_red(h, red))) return rc;
    add_timing(h, h->fp32, n);
    if (resid) *resid = red[RED_RESID];
    return EP_OK;
}

int ep_residual(ep_handle* h, ep_residual_info* r)
{
    if (!h || !r) return EP_EINVAL;
    ensure_it64(h);
    double red[RED_N];
    int rc;
    // one PT evaluation into the scratch buffer (state untouched)
    launch_reset_red(h->red, h->st);
    launch_sweep<double>(h, false, h->cur64, MODE_CHECK);
    if ((rc = read_red(h, red))) return rc;
    r->resid = red[RED_RESID];
    r->momentum = red[RED_MOM];
    r->vmax = red[RED_VMAX];
    r->eps_rel = red[RED_VMAX] > 0 ? h->dtrho * red[RED_MOM] / red[RED_VMAX] : 0.0;
    launch_reset_red(h->red, h->st);
    launch_sweep<double>(h, true, h->cur64, MODE_PHYS);
    double** it = h->it64[h->cur64];
    const double* v[3] = {it[F_VX], it[F_VY], it[F_VZ]};
    const double ikd = std::isinf(h->prm.bulk) ? 0.0 : 1.0 / (h->prm.bulk * h->prm.dt);
    launch_continuity(h->g, v, it[F_P], h->old64[O_P], ikd, 1.0 / h->dx, 1.0 / h->dy, 1.0 / h->dz, h->red + RED_CONT,
                      h->st);
    if ((rc = read_red(h, red))) return rc;
    r->physical = red[RED_MOM];
    r->continuity = red[RED_CONT];
    return EP_OK;
}

int ep_residual_noalloc(ep_handle* h, ep_residual_info* r)
{
    if (!h || !r) return EP_EINVAL;
    char* base = nullptr;
    int rc;
    if ((rc = noalloc_scratch(h, &base))) return rc;
    const bool tiles2d = h->ndim == 2 && h->fused64;
    if (tiles2d && h->ntiles > NOALLOC_MAX_TILES)
        return set_err(h, EP_EINVAL, "ep_residual_noalloc: %ld tiles exceed the scratch capacity of %ld (%zu bytes)",
                       h->ntiles, NOALLOC_MAX_TILES, NOALLOC_SCRATCH_BYTES);
    ensure_it64(h);
    auto* red = (unsigned long long*)(base + NA_RED);
    auto* tab = (SweepArgs<double>*)(base + NA_TAB);
    auto* cnt = (int*)(base + NA_CNT);
    auto* tiles = (TileRef*)(base + NA_TILES);
    SweepArgs<double> a[2] = {args64(h, false, h->cur64), args64(h, true, h->cur64)};
    for (auto& x : a) x.red = red;
    if (tiles2d) {
        // stage the two argument tables and this model's tile list
        const int n = (int)h->ntiles;
        HIPCHK(h, hipMemcpyAsync(tab, a, sizeof(a), hipMemcpyHostToDevice, h->st));
        HIPCHK(h, hipMemcpyAsync(cnt, &n, sizeof(int), hipMemcpyHostToDevice, h->st));
        HIPCHK(h, hipMemcpyAsync(tiles, h->tiles, h->ntiles * sizeof(TileRef), hipMemcpyDeviceToDevice, h->st));
        HIPCHK(h, hipStreamSynchronize(h->st));          // the host tables leave scope
    }
    auto sweep = [&](int q, int mode) {
        if (tiles2d)
            launch_sweep_batch_2d<double>(SINGLE_SHAPE, tab + q, tiles, cnt, mode, h->grid2[0], h->st);
        else if (h->ndim == 2)
            launch_sweep_unfused_2d<double>(a[q], mode, h->st);
        else if (h->fused64 && a[q].fs > 0)
            launch_sweep_fused_3d<double>(a[q], mode, h->st);
        else
            launch_sweep_unfused_3d<double>(a[q], mode, h->st);
    };
    unsigned long long raw[RED_N];
    double v[RED_N];
    // one PT evaluation (written to the second iteration buffer; state untouched)
    launch_reset_red(red, h->st);
    sweep(0, MODE_CHECK);
    HIPCHK(h, hipMemcpyAsync(raw, red, sizeof(raw), hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    HIPCHK(h, hipGetLastError());
    decode_red(raw, v);
    r->resid = v[RED_RESID];
    r->momentum = v[RED_MOM];
    r->vmax = v[RED_VMAX];
    r->eps_rel = v[RED_VMAX] > 0 ? h->dtrho * v[RED_MOM] / v[RED_VMAX] : 0.0;
    // physical evaluation and the continuity residual
    launch_reset_red(red, h->st);
    sweep(1, MODE_PHYS);
    double** it = h->it64[h->cur64];
    const double* vv[3] = {it[F_VX], it[F_VY], it[F_VZ]};
    const double ikd = std::isinf(h->prm.bulk) ? 0.0 : 1.0 / (h->prm.bulk * h->prm.dt);
    launch_continuity(h->g, vv, it[F_P], h->old64[O_P], ikd, 1.0 / h->dx, 1.0 / h->dy, 1.0 / h->dz, red + RED_CONT,
                      h->st);
    HIPCHK(h, hipMemcpyAsync(raw, red, sizeof(raw), hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    HIPCHK(h, hipGetLastError());
    decode_red(raw, v);
    r->physical = v[RED_MOM];
    r->continuity = v[RED_CONT];
    return EP_OK;
}

int ep_set_shear_modulus(ep_handle* h, const double* shear)
{
    if (!h || !shear || h->in_batch) return EP_EINVAL;
    const int nz1 = h->ndim == 3 ? h->nz : 1;
    const long nc = (long)h->nx * h->ny * nz1;
    std::vector<double> igd(nc);
    for (long c = 0; c < nc; ++c) {
        if (!(shear[c] > 0.0) || !(shear[c] <= h->prm.shear))
            return set_err(h, EP_EINVAL, "shear modulus of cell %ld not in (0, shear]", c);
        igd[c] = 1.0 / (shear[c] * h->prm.dt);
    }
    std::vector<double> pad(h->nelem, 0.0);
    int ext[3] = {h->nx, h->ny, nz1};
    scatter(h, igd.data(), ext, pad);
    HIPCHK(h, hipMemcpyAsync(h->igdc64, pad.data(), h->nelem * sizeof(double), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    h->has_g = true;
    h->old32_valid = false;                         // the FP32 copy is re-derived before FP32 sweeps
    return upload_tables(h);
}

int ep_set_strain_rate(ep_handle* h, const double erate[3])
{
    if (!h || !erate || h->in_batch) return EP_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(erate[d])) return set_err(h, EP_EINVAL, "strain rate %d not finite", d);
    // FP32 velocities are stored relative to the background field of the
    // old rate: make the FP64 state current, then re-derive FP32 from it
    ensure_it64(h);
    for (int d = 0; d < 3; ++d) h->prm.erate[d] = h->ndim == 3 || d < 2 ? erate[d] : 0.0;
    const double emax = std::fmax(std::fabs(h->prm.erate[0]), std::fmax(std::fabs(h->prm.erate[1]),
                                                                       std::fabs(h->prm.erate[2])));
    h->dsig_ref = 2.0 * h->prm.shear * emax * h->prm.dt;
    h->it32_valid = false;
    if (h->ndim == 2) {
        int rc = upload_tables(h);                  // the tables carry the background rate
        if (rc) return rc;
    }
    HIPCHK(h, hipGetLastError());
    return EP_OK;
}

int ep_objective_update(ep_handle* h)
{
    if (!h) return EP_EINVAL;
    objective_update(h);
    HIPCHK(h, hipGetLastError());
    return EP_OK;
}

int ep_load_step(ep_handle* h, ep_step_stats* st)
{
    if (!h) return EP_EINVAL;
    ep_step_stats dummy;
    if (!st) st = &dummy;
    int rc;
    double red[RED_N];
    step_begin(h, st);
    if ((rc = read_red(h, red))) return rc;
    if ((rc = step_start(h, red))) return rc;
    const StepCtl& c = h->ctl;
    while (c.running) {
        const bool use32 = c.use32;
        const int nb = std::min(h->n_check, h->prm.max_iter - st->iters);
        if ((rc = run_batch(h, use32, nb, true))) return rc;
        if ((rc = read_red(h, red))) return rc;
        add_timing(h, use32, nb);
        step_check(h, red, nb);
        if (c.cert_pending) {
            step_certify_launch(h);
            if ((rc = read_red(h, red))) return rc;
            step_certify(h, red);
        }
    }
    if ((rc = step_finish(h))) {
        if (st->guess_used != 1) return rc;
        // failed from the supplied guess: the state is back at the increment
        // start; redo the increment from the plain guess
        const ep_step_stats first = *st;
        rc = ep_load_step(h, st);
        st->guess_used = -1;
        st->r_guess = first.r_guess;
        st->iters += first.iters;
        st->iters_fp32 += first.iters_fp32;
        st->seconds += first.seconds;
        return rc;
    }
    double cols[4];
    HIPCHK(h, hipMemcpyAsync(cols, h->cols64, sizeof(cols), hipMemcpyDeviceToHost, h->st));
    if ((rc = read_red(h, red))) return rc;
    step_report(h, red, cols);
    return EP_OK;
}

int ep_step_history(const ep_handle* h, double* resid, int* precision, int cap)
{
    if (!h || cap < 0) return EP_EINVAL;
    const int n = (int)h->hist_r.size();
    for (int q = 0; q < n && q < cap; ++q) {
        if (resid) resid[q] = h->hist_r[q];
        if (precision) precision[q] = h->hist_p[q];
    }
    return n;
}

long ep_field_shape(const ep_handle* h, int field, int shape[3])
{
    if (!h || field < 0 || field >= EP_F_COUNT) return EP_EINVAL;
    FieldRef r = field_ref(const_cast<ep_handle*>(h), field);
    if (shape) {
        shape[0] = r.ext[0];
        shape[1] = r.ext[1];
        shape[2] = r.ext[2];
    }
    return (long)r.ext[0] * r.ext[1] * r.ext[2];
}

int ep_set_guess(ep_handle* h, const double* vx, const double* vy, const double* vz)
{
    if (!h || !vx || !vy || (h->ndim == 3 && !vz)) return EP_EINVAL;
    const double* src[3] = {vx, vy, vz};
    const int nz1 = h->ndim == 3 ? h->nz : 1;
    int rc;
    for (int d = 0; d < h->ndim; ++d) {
        const int ext[3] = {h->nx + (d == 0), h->ny + (d == 1), nz1 + (d == 2)};
        if ((rc = upload(h, h->vguess64[d], src[d], ext))) return rc;
    }
    h->guess_ready = true;
    return EP_OK;
}

// a device array of the current device (rejects host and foreign memory
// before a kernel could dereference it)
static bool is_device_array(const void* p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == dev;
}

int ep_set_guess_device(ep_handle* h, int kind, int dtype, const void* vx, const void* vy, const void* vz)
{
    if (!h) return EP_EINVAL;
    if (kind != EP_GUESS_VELOCITY && kind != EP_GUESS_CHANGE && kind != EP_GUESS_ZERO)
        return set_err(h, EP_EINVAL, "ep_set_guess_device: bad kind %d", kind);
    if (dtype != EP_GUESS_F64 && dtype != EP_GUESS_F32)
        return set_err(h, EP_EINVAL, "ep_set_guess_device: bad dtype %d", dtype);
    const void* src[3] = {vx, vy, vz};
    if (kind != EP_GUESS_ZERO)
        for (int d = 0; d < h->ndim; ++d)
            if (!src[d] || !is_device_array(src[d]))
                return set_err(h, EP_EINVAL, "ep_set_guess_device: velocity array %d is not device memory", d);
    ensure_it64(h);
    const int nz1 = h->ndim == 3 ? h->nz : 1;
    double** it = h->it64[h->cur64];
    for (int d = 0; d < h->ndim; ++d) {
        const int ext[3] = {h->nx + (d == 0), h->ny + (d == 1), nz1 + (d == 2)};
        launch_guess_in(h->vguess64[d], kind == EP_GUESS_ZERO ? nullptr : src[d], dtype == EP_GUESS_F32,
                        kind == EP_GUESS_CHANGE ? it[F_VX + d] : nullptr, ext, h->sy, h->sz, h->st);
    }
    HIPCHK(h, hipGetLastError());
    h->guess_ready = true;
    return EP_OK;
}

int ep_fields(ep_handle* h, int field, int dir, double* host, size_t count)
{
    if (!h || !host || field < 0 || field >= EP_F_COUNT || (dir != EP_GET && dir != EP_SET)) return EP_EINVAL;
    ensure_it64(h);
    FieldRef r = field_ref(h, field);
    const size_t n = (size_t)r.ext[0] * r.ext[1] * r.ext[2];
    if (n == 0 || count != n) return set_err(h, EP_EINVAL, "field %d: count %zu, expected %zu", field, count, n);
    int rc;
    if (dir == EP_GET) {
        std::vector<double> pad;
        if (field == EP_F_TZZ || field == EP_F_TZZ_OLD) {
            std::vector<double> a, b;
            const double* px = field == EP_F_TZZ ? h->it64[h->cur64][F_TXX] : h->old64[O_TXX];
            const double* py = field == EP_F_TZZ ? h->it64[h->cur64][F_TYY] : h->old64[O_TYY];
            if ((rc = get_padded(h, px, a)) || (rc = get_padded(h, py, b))) return rc;
            for (long q = 0; q < h->nelem; ++q) a[q] = -(a[q] + b[q]);
            gather(h, a, r.ext, host);
            return EP_OK;
        }
        if ((rc = get_padded(h, r.dev, pad))) return rc;
        gather(h, pad, r.ext, host);
        return EP_OK;
    }
    if (!r.writable) return set_err(h, EP_EINVAL, "field %d is read-only", field);
    if ((rc = upload(h, r.dev, host, r.ext))) return rc;
    if (field <= EP_F_TYZ) h->it32_valid = false;
    else h->old32_valid = false;    // old stresses, cohesion (and harmlessly for accumulators)
    return EP_OK;
}

}  // extern "C"
