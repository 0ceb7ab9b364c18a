// Batched driver: many independent 2D models (a parameter sweep) solved
// increment by increment together.
//
// Every model is an ordinary solver handle carved from the batch workspace,
// so prologue, precision conversions, epilogue and field I/O are the
// single-model code.  What is shared is the PT iteration: a graph of n_check
// sweeps (a reduction reset, then per sweep one persistent launch per
// precision and tile shape in use, the last sweep with the residual check)
// is captured on first use and replayed; each launch walks a device tile list of the
// models still iterating in that precision.  After a replay the host reads
// every model's residual in one copy, applies the single-model convergence
// logic per model, and retires or re-files the models whose state changed by
// rewriting the lists (their length is read by the kernels, so the graph
// stays valid).  The tile shape of each model size is chosen by an
// autotuner that times the whole batched sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "ep.h"
#include "ep_handle.h"
#include "ep_internal.h"

using namespace ep;

struct ep_batch {
    int n;
    hipStream_t st;
    hipStream_t cs;                     // capture stream (graph recording only)
    bool fp32;
    int n_check;
    std::vector<ep_handle*> m;
    std::vector<long> cells;
    std::vector<int> shape;             // tile shape per model (sweeps in the batch precision)
    std::vector<int> shape64;           // FP32-field batches: tile shape of the FP64 finishing sweeps
    unsigned long long* red;            // n x RED_N
    double* cols;                       // n x 4
    SweepArgs<double>* tab64;           // 2 x n (parity of the ping-pong buffers)
    SweepArgs<float>* tab32;
    TileRef* list[2][BATCH_SHAPES];     // [precision: 0 FP64, 1 FP32][shape]
    int* cnt;                           // 2 x BATCH_SHAPES
    int grid[2][BATCH_SHAPES];
    std::vector<SweepArgs<double>> h_tab64;
    std::vector<SweepArgs<float>> h_tab32;
    std::vector<TileRef> h_list[2][BATCH_SHAPES];
    int h_cnt[2 * BATCH_SHAPES];
    std::vector<unsigned long long> h_red;
    std::vector<double> h_cols;
    double cs32, cs64;                  // cell-sweeps of the current replay set-up
    // captured replays keyed by the set of non-empty tile lists (a precision
    // whose lists are empty is not launched at all)
    std::map<unsigned, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    bool timing;
    hipEvent_t ev0, ev1;
    double t_ms, t_cs32, t_cs64;
    long t_replays;
    char err[512];
};

namespace {

int berr(ep_batch* b, int code, const char* fmt, ...)
{
    if (b) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(b->err, sizeof(b->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define BCHK(b, x)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess)                                                               \
            return berr((b), EP_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_));       \
    } while (0)

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int resolved_check(const ep_params& p) { return p.n_check > 0 ? p.n_check : (p.ndim == 3 ? 10 : 100); }

long tiles_of(const ep_params& p, int s)
{
    const int tx = kBatchTiles[s][0], ty = kBatchTiles[s][1];
    return (long)((p.nx + tx - 1) / tx) * ((p.ny + ty - 1) / ty);
}

int validate_batch(int n, const ep_params* p)
{
    if (n <= 0 || !p) return EP_EINVAL;
    const int nc = resolved_check(p[0]);
    for (int i = 0; i < n; ++i) {
        if (validate(&p[i]) != EP_OK) return EP_EINVAL;
        if (p[i].ndim != 2 || p[i].precision != p[0].precision) return EP_EINVAL;
        if (resolved_check(p[i]) != nc || nc % 2 != 0) return EP_EINVAL;
        if ((p[i].nx + 31) / 32 > 32767 || (p[i].ny + 3) / 4 > 32767) return EP_EINVAL;
    }
    return EP_OK;
}

// Layout of the batch workspace: the models, then the batch arrays.
struct BatchLayout {
    std::vector<size_t> model_off;
    size_t red, cols, tab64, tab32, lists[2][BATCH_SHAPES], cnt, total;
};

BatchLayout layout(int n, const ep_params* p)
{
    BatchLayout L;
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        L.model_off.push_back(off);
        off = align256(off + carve(&p[i], nullptr, nullptr));
    }
    auto take = [&](size_t bytes) { size_t r = off; off = align256(off + bytes); return r; };
    L.red = take((size_t)n * RED_N * sizeof(unsigned long long));
    L.cols = take((size_t)n * 4 * sizeof(double));
    L.tab64 = take((size_t)3 * n * sizeof(SweepArgs<double>));
    L.tab32 = take((size_t)3 * n * sizeof(SweepArgs<float>));
    const bool fp32 = p[0].precision == EP_FP32_FIELDS;
    for (int q = 0; q < 2; ++q)
        for (int s = 0; s < BATCH_SHAPES; ++s) {
            long c = 0;
            if (q == 0 || fp32)
                for (int i = 0; i < n; ++i) c += tiles_of(p[i], s);
            L.lists[q][s] = take((size_t)std::max(c, 1L) * sizeof(TileRef));
        }
    L.cnt = take(2 * BATCH_SHAPES * sizeof(int));
    L.total = off;
    return L;
}

// Model tables, 3 x n entries: [0] the first sweep of a replay (reads the
// current buffers; stores Lambda when a freeze was just decided), [1] and [2]
// the later sweeps reading the current / the other buffers.
void fill_tables(ep_batch* b)
{
    const int n = b->n;
    for (int i = 0; i < n; ++i) {
        ep_handle* h = b->m[i];
        const int lm_first = sweep_lam_mode(h, 0), lm_rest = sweep_lam_mode(h, 1);
        for (int slot = 0; slot < 3; ++slot) {
            const int par = slot == 2 ? 1 : 0;
            const int lm = slot == 0 ? lm_first : lm_rest;
            b->h_tab64[slot * n + i] = args64(h, false, h->cur64 ^ par);
            b->h_tab64[slot * n + i].lam_mode = lm;
            if (b->fp32) {
                b->h_tab32[slot * n + i] = args32(h, h->cur32 ^ par);
                b->h_tab32[slot * n + i].lam_mode = lm;
            }
        }
    }
}

// Tile lists of the running models (precision of each model's current
// sweeps), or of all models when all_models is set, in FP32 when all32 (the
// batch precision) else in FP64.
void fill_lists(ep_batch* b, bool all_models, bool all32 = true)
{
    for (int q = 0; q < 2; ++q)
        for (int s = 0; s < BATCH_SHAPES; ++s) b->h_list[q][s].clear();
    b->cs32 = b->cs64 = 0;
    for (int i = 0; i < b->n; ++i) {
        ep_handle* h = b->m[i];
        bool use32;
        if (all_models) {
            use32 = b->fp32 && all32;
        } else {
            if (!h->ctl.running) continue;
            use32 = h->ctl.use32;
        }
        const int s = (use32 || !b->fp32) ? b->shape[i] : b->shape64[i];
        const int tx = kBatchTiles[s][0], ty = kBatchTiles[s][1];
        const int nbx = (h->nx + tx - 1) / tx, nby = (h->ny + ty - 1) / ty;
        auto& L = b->h_list[use32 ? 1 : 0][s];
        for (int by = 0; by < nby; ++by)
            for (int bx = 0; bx < nbx; ++bx) L.push_back(TileRef{i, (short)bx, (short)by});
        (use32 ? b->cs32 : b->cs64) += (double)b->cells[i] * b->n_check;
    }
    for (int q = 0; q < 2; ++q)
        for (int s = 0; s < BATCH_SHAPES; ++s) b->h_cnt[q * BATCH_SHAPES + s] = (int)b->h_list[q][s].size();
}

int upload(ep_batch* b)
{
    const size_t n2 = 3 * (size_t)b->n;
    BCHK(b, hipMemcpyAsync(b->tab64, b->h_tab64.data(), n2 * sizeof(SweepArgs<double>), hipMemcpyHostToDevice, b->st));
    if (b->fp32)
        BCHK(b, hipMemcpyAsync(b->tab32, b->h_tab32.data(), n2 * sizeof(SweepArgs<float>), hipMemcpyHostToDevice,
                               b->st));
    for (int q = 0; q < 2; ++q)
        for (int s = 0; s < BATCH_SHAPES; ++s)
            if (!b->h_list[q][s].empty())
                BCHK(b, hipMemcpyAsync(b->list[q][s], b->h_list[q][s].data(), b->h_list[q][s].size() * sizeof(TileRef),
                                       hipMemcpyHostToDevice, b->st));
    BCHK(b, hipMemcpyAsync(b->cnt, b->h_cnt, sizeof(b->h_cnt), hipMemcpyHostToDevice, b->st));
    // the host vectors may change right after this call
    BCHK(b, hipStreamSynchronize(b->st));
    return EP_OK;
}

bool shape_used(const ep_batch* b, int s)
{
    for (int i = 0; i < b->n; ++i)
        if (b->shape[i] == s || b->shape64[i] == s) return true;
    return false;
}

// Bit q * BATCH_SHAPES + shape for every non-empty tile list (q: 0 FP64, 1 FP32).
unsigned list_mask(const ep_batch* b)
{
    unsigned m = 0;
    for (int q = 0; q < 2; ++q)
        for (int sh = 0; sh < BATCH_SHAPES; ++sh)
            if (b->h_cnt[q * BATCH_SHAPES + sh] > 0) m |= 1u << (q * BATCH_SHAPES + sh);
    return m;
}

// nsw sweeps of every tile in the lists selected by mask; the last one in
// CHECK mode when check is set.  With alternate, the sweeps advance the
// iteration (ping-pong); without, every sweep reads the current buffers and
// writes the other ones (timing runs that leave the state unchanged).
void enqueue_sweeps(ep_batch* b, int nsw, bool check, bool reset, bool alternate, unsigned mask, hipStream_t s)
{
    if (reset) launch_reset_red_n(b->red, b->n, s);
    for (int k = 0; k < nsw; ++k) {
        const int mode = (check && k == nsw - 1) ? MODE_CHECK : MODE_UPDATE;
        const int slot = !alternate ? 1 : k == 0 ? 0 : (k & 1) ? 2 : 1;
        for (int sh = 0; sh < BATCH_SHAPES; ++sh) {
            if (b->fp32 && (mask >> (BATCH_SHAPES + sh) & 1u))
                launch_sweep_batch_2d<float>(sh, b->tab32 + slot * b->n, b->list[1][sh], b->cnt + BATCH_SHAPES + sh,
                                             mode, b->grid[1][sh], s);
            if (mask >> sh & 1u)
                launch_sweep_batch_2d<double>(sh, b->tab64 + slot * b->n, b->list[0][sh], b->cnt + sh, mode,
                                              b->grid[0][sh], s);
        }
    }
}

void drop_graphs(ep_batch* b)
{
    for (auto& g : b->graphs) {
        (void)hipGraphExecDestroy(g.second.second);
        (void)hipGraphDestroy(g.second.first);
    }
    b->graphs.clear();
}

// The replay of n_check sweeps for the lists in mask (captured on first use).
int replay_for(ep_batch* b, unsigned mask, hipGraphExec_t* out)
{
    auto it = b->graphs.find(mask);
    if (it != b->graphs.end()) {
        *out = it->second.second;
        return EP_OK;
    }
    BCHK(b, hipStreamBeginCapture(b->cs, hipStreamCaptureModeRelaxed));
    enqueue_sweeps(b, b->n_check, true, true, true, mask, b->cs);
    hipGraph_t g = nullptr;
    BCHK(b, hipStreamEndCapture(b->cs, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return berr(b, EP_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    b->graphs[mask] = {g, ex};
    *out = ex;
    return EP_OK;
}

int read_all(ep_batch* b, bool cols)
{
    BCHK(b, hipMemcpyAsync(b->h_red.data(), b->red, b->h_red.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, b->st));
    if (cols)
        BCHK(b, hipMemcpyAsync(b->h_cols.data(), b->cols, b->h_cols.size() * sizeof(double), hipMemcpyDeviceToHost,
                               b->st));
    BCHK(b, hipStreamSynchronize(b->st));
    BCHK(b, hipGetLastError());
    return EP_OK;
}

void model_red(const ep_batch* b, int i, double out[RED_N]) { decode_red(&b->h_red[(size_t)i * RED_N], out); }

void destroy_batch(ep_batch* b)
{
    drop_graphs(b);
    for (ep_handle* h : b->m) handle_free(h);
    if (b->cs) (void)hipStreamDestroy(b->cs);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    delete b;
}

}  // namespace

// =========================================================================
extern "C" {

int ep_batch_workspace_size(int n, const ep_params* p, size_t* bytes)
{
    if (!bytes || validate_batch(n, p) != EP_OK) return EP_EINVAL;
    *bytes = layout(n, p).total;
    return EP_OK;
}

int ep_batch_init(int n, const ep_params* p, const double* const* cohesion, void* d_workspace, size_t ws_bytes,
                  void* stream, ep_batch** out)
{
    if (!out) return EP_EINVAL;
    *out = nullptr;
    if (validate_batch(n, p) != EP_OK) return EP_EINVAL;
    const BatchLayout L = layout(n, p);
    if (!d_workspace || ws_bytes < L.total) return EP_ENOMEM;
    if (((uintptr_t)d_workspace & 255) != 0) return EP_EINVAL;
    ep_batch* b = new (std::nothrow) ep_batch();
    if (!b) return EP_ENOMEM;
    char* base = (char*)d_workspace;
    b->n = n;
    b->st = (hipStream_t)stream;
    b->fp32 = p[0].precision == EP_FP32_FIELDS;
    b->n_check = resolved_check(p[0]);
    auto fail = [&](int code) { destroy_batch(b); return code; };
    if (hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess) return fail(EP_EDEVICE);
    if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) return fail(EP_EDEVICE);
    b->red = (unsigned long long*)(base + L.red);
    b->cols = (double*)(base + L.cols);
    b->tab64 = (SweepArgs<double>*)(base + L.tab64);
    b->tab32 = (SweepArgs<float>*)(base + L.tab32);
    for (int q = 0; q < 2; ++q)
        for (int s = 0; s < BATCH_SHAPES; ++s) b->list[q][s] = (TileRef*)(base + L.lists[q][s]);
    b->cnt = (int*)(base + L.cnt);
    if (hipMemsetAsync(base + L.red, 0, L.total - L.red, b->st) != hipSuccess) return fail(EP_EDEVICE);
    for (int i = 0; i < n; ++i) {
        ep_handle* h = nullptr;
        int rc = handle_create(&p[i], cohesion ? cohesion[i] : nullptr, base + L.model_off[i], b->st, &h);
        if (rc) return fail(rc);
        h->in_batch = true;
        h->red = b->red + (size_t)i * RED_N;
        h->cols64 = b->cols + (size_t)i * 4;
        if ((rc = upload_tables(h))) return fail(rc);
        b->m.push_back(h);
        b->cells.push_back((long)p[i].nx * p[i].ny);
        b->shape.push_back(0);
        b->shape64.push_back(0);
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess || ncu <= 0) ncu = 256;
    for (int s = 0; s < BATCH_SHAPES; ++s) {
        b->grid[0][s] = ncu * std::min(8, batch_blocks_per_cu<double>(s));
        b->grid[1][s] = ncu * std::min(8, batch_blocks_per_cu<float>(s));
    }
    b->h_tab64.resize(3 * (size_t)n);
    b->h_tab32.resize(3 * (size_t)n);
    b->h_red.assign((size_t)n * RED_N, 0ull);
    b->h_cols.assign((size_t)n * 4, 0.0);
    if (hipGetLastError() != hipSuccess) return fail(EP_EDEVICE);
    *out = b;
    return EP_OK;
}

void ep_batch_destroy(ep_batch* b)
{
    if (b) destroy_batch(b);
}

const char* ep_batch_last_error(const ep_batch* b) { return b ? b->err : "no batch"; }

ep_handle* ep_batch_model(ep_batch* b, int i)
{
    if (!b || i < 0 || i >= b->n) return nullptr;
    return b->m[i];
}

int ep_batch_tile_shape(const ep_batch* b, int i, int* tx, int* ty)
{
    if (!b || i < 0 || i >= b->n) return EP_EINVAL;
    if (tx) *tx = kBatchTiles[b->shape[i]][0];
    if (ty) *ty = kBatchTiles[b->shape[i]][1];
    return EP_OK;
}

int ep_batch_tune(ep_batch* b, int reps)
{
    if (!b || reps <= 0) return EP_EINVAL;
    // the timed sweeps read the current buffers and write the other ones, so
    // the state is unchanged
    for (ep_handle* h : b->m) {
        if (b->fp32) ensure_it32(h);
        else ensure_it64(h);
    }
    fill_tables(b);
    // models grouped by size: one tile shape per size class
    std::map<std::pair<int, int>, std::vector<int>> classes;
    for (int i = 0; i < b->n; ++i) classes[{b->m[i]->nx, b->m[i]->ny}].push_back(i);
    // coordinate descent over the size classes for one precision's shapes
    auto descend = [&](std::vector<int>& shape, bool all32) -> int {
        auto time_config = [&](double* ms) -> int {
            fill_lists(b, true, all32);
            int rc = upload(b);
            if (rc) return rc;
            const unsigned mask = list_mask(b);
            enqueue_sweeps(b, 1, false, false, false, mask, b->st);    // warm-up
            BCHK(b, hipEventRecord(b->ev0, b->st));
            enqueue_sweeps(b, reps, false, false, false, mask, b->st);
            BCHK(b, hipEventRecord(b->ev1, b->st));
            BCHK(b, hipEventSynchronize(b->ev1));
            BCHK(b, hipGetLastError());
            float t = 0.f;
            BCHK(b, hipEventElapsedTime(&t, b->ev0, b->ev1));
            *ms = t / reps;
            return EP_OK;
        };
        double best = 0;
        int rc = time_config(&best);
        if (rc) return rc;
        for (int pass = 0; pass < 2; ++pass) {
            for (auto& cl : classes) {
                const int keep = shape[cl.second[0]];
                int best_s = keep;
                for (int s = 0; s < BATCH_SHAPES; ++s) {
                    if (s == keep) continue;
                    for (int i : cl.second) shape[i] = s;
                    double t;
                    if ((rc = time_config(&t))) return rc;
                    if (t < best) {
                        best = t;
                        best_s = s;
                    }
                }
                for (int i : cl.second) shape[i] = best_s;
            }
        }
        return EP_OK;
    };
    int rc = descend(b->shape, true);
    if (rc) return rc;
    if (b->fp32) {
        // the FP64 finishing sweeps have their own best shapes (8-byte LDS
        // planes limit the workgroups per CU differently)
        for (ep_handle* h : b->m) ensure_it64(h);
        fill_tables(b);
        if ((rc = descend(b->shape64, false))) return rc;
    }
    drop_graphs(b);                     // recaptured for the new shapes when used
    return EP_OK;
}

int ep_batch_enable_timing(ep_batch* b, int on)
{
    if (!b) return EP_EINVAL;
    b->timing = on != 0;
    b->t_ms = b->t_cs32 = b->t_cs64 = 0;
    b->t_replays = 0;
    return EP_OK;
}

int ep_batch_timing(const ep_batch* b, double* ms, double* cell_sweeps32, double* cell_sweeps64, long* replays)
{
    if (!b) return EP_EINVAL;
    if (ms) *ms = b->t_ms;
    if (cell_sweeps32) *cell_sweeps32 = b->t_cs32;
    if (cell_sweeps64) *cell_sweeps64 = b->t_cs64;
    if (replays) *replays = b->t_replays;
    return EP_OK;
}

int ep_batch_load_step(ep_batch* b, ep_step_stats* st)
{
    if (!b || !st) return EP_EINVAL;
    int rc;
    // prologue of every model, then one read of all reference residuals
    for (int i = 0; i < b->n; ++i) step_begin(b->m[i], &st[i]);
    if ((rc = read_all(b, false))) return rc;
    for (int i = 0; i < b->n; ++i) {
        double red[RED_N];
        model_red(b, i, red);
        step_start(b->m[i], red);       // a failed start leaves the model not running
    }
    auto any_running = [&]() {
        for (ep_handle* h : b->m)
            if (h->ctl.running) return true;
        return false;
    };
    bool dirty = true;
    while (any_running()) {
        if (dirty) {
            fill_tables(b);
            fill_lists(b, false);
            if ((rc = upload(b))) return rc;
            dirty = false;
        }
        if (b->timing) BCHK(b, hipEventRecord(b->ev0, b->st));
        hipGraphExec_t ex = nullptr;
        if ((rc = replay_for(b, list_mask(b), &ex))) return rc;
        BCHK(b, hipGraphLaunch(ex, b->st));
        if (b->timing) BCHK(b, hipEventRecord(b->ev1, b->st));
        if ((rc = read_all(b, false))) return rc;
        if (b->timing) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, b->ev0, b->ev1) == hipSuccess) {
                b->t_ms += t;
                b->t_cs32 += b->cs32;
                b->t_cs64 += b->cs64;
                ++b->t_replays;
            }
        }
        for (int i = 0; i < b->n; ++i) {
            ep_handle* h = b->m[i];
            if (!h->ctl.running) continue;
            // an even number of sweeps leaves every model's current buffer in place
            const bool was32 = h->ctl.use32;
            if (was32) h->it64_valid = false;
            else h->it32_valid = false;
            if (h->freeze == 1) {           // the replay's first sweep stored Lambda
                h->freeze = 2;
                h->lam_in32 = was32;
                dirty = true;
            }
            double red[RED_N];
            model_red(b, i, red);
            const int freeze_before = h->freeze;
            const bool late_before = h->late;
            const bool cont = step_check(h, red, b->n_check);
            if (!cont || h->ctl.use32 != was32 || h->freeze != freeze_before || h->late != late_before) dirty = true;
        }
        // certificates of the models whose check met the tolerance (the
        // single-model evaluation on each model's own reduction slots)
        bool any_cert = false;
        for (ep_handle* h : b->m)
            if (h->ctl.running && h->ctl.cert_pending) {
                step_certify_launch(h);
                any_cert = true;
            }
        if (any_cert) {
            if ((rc = read_all(b, false))) return rc;
            for (int i = 0; i < b->n; ++i) {
                ep_handle* h = b->m[i];
                if (!h->ctl.running || !h->ctl.cert_pending) continue;
                double red[RED_N];
                model_red(b, i, red);
                const int freeze_before = h->freeze;
                const bool late_before = h->late;
                if (!step_certify(h, red) || h->freeze != freeze_before || h->late != late_before) dirty = true;
            }
        }
    }
    int worst = EP_OK;
    for (int i = 0; i < b->n; ++i) {
        const int s = step_finish(b->m[i]);
        if (s != EP_OK && worst == EP_OK) worst = s;
    }
    if ((rc = read_all(b, true))) return rc;
    for (int i = 0; i < b->n; ++i) {
        if (st[i].status != EP_OK) continue;
        double red[RED_N];
        model_red(b, i, red);
        step_report(b->m[i], red, &b->h_cols[(size_t)i * 4]);
    }
    return worst;
}

}  // extern "C"
