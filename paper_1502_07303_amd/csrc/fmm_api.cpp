// C ABI of libfmm (declared in include/fmm.h): argument validation, workspace
// carving and the enqueue sequence: workspace reset, tiled speeds, seeds ->
// restart driver -> finalize.
#include <math.h>
#include <string.h>

#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/fmm.h"
#include "fmm_adjoint.h"
#include "fmm_internal.h"

using namespace fmm;

// Workspace of fmm_solve_noalloc(): a fixed device array, one copy per GPU,
// reserved when the library's code object is loaded onto that GPU.  In host
// code `scratch` names a host-side stand-in, not device memory: kernels and
// copies get the device address that hipGetSymbolAddress() returns for the
// current device, looked up once per device and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[FMM_NOALLOC_MAX_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];

// Device address of the current device's scratch array (nullptr on failure).
void *scratch_for_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

namespace {

int resolve_edge(const fmm_opts *o)
{
    const int e = o ? o->tile_edge : 0;
    return e == 0 ? 8 : e;
}

bool opts_ok(const fmm_opts *o)
{
    if (!o) return true;
    if (isnan(o->band_width) || o->band_width < 0.0) return false;
    if (isnan(o->stride) || isnan(o->inner_stride) || isnan(o->stride_h)) return false;
    if (!(o->tile_edge == 0 || o->tile_edge == 4 || o->tile_edge == 8 || o->tile_edge == 16)) return false;
    if (o->max_restarts < 0) return false;
    if (o->flags & ~(uint32_t)(FMM_VALIDATE | FMM_TIMING | FMM_ONE_MARCH)) return false;
    for (int a = 0; a < 3; a++)
        if (!(o->axis_scale[a] == 0.0 || (o->axis_scale[a] > 0.0 && isfinite(o->axis_scale[a])))) return false;
    return true;
}

// Effective spacing factors: 0 means 1; the weighted solver only when one differs.
Spacing spacing_of(const double sc[3])
{
    Spacing sp;
    sp.aniso = 0;
    for (int a = 0; a < 3; a++) {
        sp.s[a] = sc[a] == 0.0 ? 1.0 : sc[a];
        if (sp.s[a] != 1.0) sp.aniso = 1;
    }
    return sp;
}

bool problem_ok(const fmm_problem &q)
{
    int32_t t[3];
    uint64_t nt;
    if (!tile_grid(q.n0, q.n1, q.n2, 4, t, &nt)) return false;
    if (!(q.h > 0.0) || !isfinite(q.h)) return false;
    if (!q.F || !q.T_out) return false;
    if (q.n_seeds < 0 || (q.n_seeds > 0 && (!q.seed_idx || !q.seed_val))) return false;
    return true;
}

std::vector<int64_t> dims_of(int64_t n, const fmm_problem *q)
{
    std::vector<int64_t> d((size_t)n * 3);
    for (int64_t i = 0; i < n; i++) {
        d[3 * i] = q[i].n0;
        d[3 * i + 1] = q[i].n1;
        d[3 * i + 2] = q[i].n2;
    }
    return d;
}

// Restart stride of one problem (Alg. 16's delta-s, world units).
double stride_of(const fmm_opts &o, double h)
{
    if (o.stride_h > 0.0) return o.stride_h * h;
    if (o.stride > 0.0) return o.stride;
    return 2.0 * h;
}

Params make_params(const Layout &L, void *ws, const fmm_opts &o)
{
    char *b = (char *)ws;
    Params P;
    memset(&P, 0, sizeof P);
    P.sp = spacing_of(o.axis_scale);
    P.n_inst = L.n_inst;
    P.ntiles = L.ntiles;
    P.mask_words = L.mask_words;
    P.width = o.band_width;
    P.inner = (o.inner_stride > 0.0) ? o.inner_stride : INFINITY;
    P.two_march = (o.flags & FMM_ONE_MARCH) ? 0 : 1;
    P.max_restarts = o.max_restarts > 0 ? (int64_t)o.max_restarts : 0;
    // the driver reads the 100 MHz constant clock
    P.time_limit_ticks = 100000000ull * (unsigned long long)(o.time_limit_s ? o.time_limit_s : 300u);
    P.ctrl = (Ctrl *)(b + L.off_ctrl);
    P.inst = (const Inst *)(b + L.off_inst);
    P.ictl = (InstCtl *)(b + L.off_ictl);
    P.tinst = (uint32_t *)(b + L.off_tinst);
    P.meta = (TileMeta *)(b + L.off_meta);
    P.dirty0 = (uint32_t *)(b + L.off_dirty0);
    P.dirty1 = (uint32_t *)(b + L.off_dirty1);
    P.epoch = (uint32_t *)(b + L.off_epoch);
    P.tflags = (uint32_t *)(b + L.off_flags);
    P.visit = (uint32_t *)(b + L.off_visit);
    P.text = (unsigned long long *)(b + L.off_text);
    P.Tt = (double *)(b + L.off_Tt);
    P.Ft = (void *)(b + L.off_Ft);
    P.Zf = (double *)(b + L.off_Zf);
    P.mask = (unsigned long long *)(b + L.off_mask);
    P.list0 = (uint32_t *)(b + L.off_list0);
    P.list1 = (uint32_t *)(b + L.off_list1);
    P.dlist = (uint32_t *)(b + L.off_dlist);
    return P;
}

// HIP events of timed solves, keyed by workspace address (host objects only).
struct StageEvents {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool valid = false;
};
std::mutex g_ev_mu;
std::unordered_map<const void *, StageEvents> g_events;

StageEvents *events_for(const void *ws, bool create)
{
    std::lock_guard<std::mutex> lk(g_ev_mu);
    auto it = g_events.find(ws);
    if (it != g_events.end()) return &it->second;
    if (!create) return nullptr;
    StageEvents e;
    for (auto &x : e.ev)
        if (hipEventCreate(&x) != hipSuccess) return nullptr;
    return &(g_events[ws] = e);
}

// Problem descriptor of q for tile edge E, its tiles numbered from `base`.
Inst make_inst(const fmm_problem &q, int E, uint32_t base, const fmm_opts &o)
{
    Inst I;
    memset(&I, 0, sizeof I);
    int32_t t[3];
    uint64_t nt = 0;
    tile_grid(q.n0, q.n1, q.n2, E, t, &nt);
    I.n0 = q.n0;
    I.n1 = q.n1;
    I.n2 = q.n2;
    I.t0 = t[0];
    I.t1 = t[1];
    I.t2 = t[2];
    I.base = base;
    I.ntiles = (uint32_t)nt;
    I.h = q.h;
    I.stride = stride_of(o, q.h);
    I.F = q.F;
    I.T = q.T_out;
    I.status = q.status_out;
    I.seed_idx = q.n_seeds > 0 ? q.seed_idx : nullptr;
    I.seed_val = q.n_seeds > 0 ? q.seed_val : nullptr;
    I.n_seeds = q.n_seeds;
    return I;
}

// Argument checks shared by every solve entry point.
int check_solve_args(int64_t n, const fmm_problem *q, fmm_dtype F_dtype, const fmm_opts *opts)
{
    if (n <= 0 || n > MAX_PROBLEMS || !q) return FMM_EINVAL;
    if (F_dtype != FMM_F32 && F_dtype != FMM_F64) return FMM_EINVAL;
    if (!opts_ok(opts)) return FMM_EINVAL;
    for (int64_t i = 0; i < n; i++)
        if (!problem_ok(q[i])) return FMM_EINVAL;
    return FMM_OK;
}

// The launch sequence of a solve: preparation (workspace reset, tiled
// speeds, seeds), the restart driver, finalize; with stage events if `ev`.
int enqueue_solve(const Params &P, const Inst *insts, int64_t n, int E, const fmm_opts &o, bool f64,
                  StageEvents *ev, hipStream_t s)
{
    if (ev && hipEventRecord(ev->ev[0], s) != hipSuccess) return FMM_EHIP;
    if (launch_prepare(P, insts, n, E, (o.flags & FMM_VALIDATE) != 0, f64, s) != hipSuccess) return FMM_EHIP;
    if (ev && hipEventRecord(ev->ev[1], s) != hipSuccess) return FMM_EHIP;
    uint32_t nwg = 0;
    if (launch_driver(P, E, f64, s, &nwg) != hipSuccess) return FMM_EHIP;
    if (ev && hipEventRecord(ev->ev[2], s) != hipSuccess) return FMM_EHIP;
    if (launch_finalize(P, insts, n, E, s) != hipSuccess) return FMM_EHIP;
    if (ev) {
        if (hipEventRecord(ev->ev[3], s) != hipSuccess) return FMM_EHIP;
        ev->valid = true;
    }
    return FMM_OK;
}

int run_batch(int64_t n, const fmm_problem *q, fmm_dtype F_dtype, const fmm_opts *opts, void *workspace,
              size_t workspace_bytes, void *stream)
{
    int rc = check_solve_args(n, q, F_dtype, opts);
    if (rc != FMM_OK) return rc;
    if (!workspace || ((uintptr_t)workspace & 255u) != 0) return FMM_EINVAL;
    fmm_opts o;
    if (opts)
        o = *opts;
    else
        fmm_default_opts(&o);
    const int E = resolve_edge(&o);
    Layout L;
    std::vector<uint32_t> bases((size_t)n);
    const std::vector<int64_t> dims = dims_of(n, q);
    if (!make_layout(n, dims.data(), E, F_dtype == FMM_F64 ? 8 : 4, &L, bases.data())) return FMM_EINVAL;
    if (workspace_bytes < L.total) return FMM_ENOMEM;
    Params P = make_params(L, workspace, o);
    std::vector<Inst> insts((size_t)n);
    for (int64_t i = 0; i < n; i++) insts[(size_t)i] = make_inst(q[i], E, bases[(size_t)i], o);
    hipStream_t s = (hipStream_t)stream;
    StageEvents *ev = nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return FMM_EHIP;
    // stage timing is a property of eager solves; a captured sequence has none
    if (cs == hipStreamCaptureStatusActive) o.flags &= ~(uint32_t)FMM_TIMING;
    if (o.flags & FMM_TIMING) {
        ev = events_for(workspace, true);
        if (!ev) return FMM_EHIP;
        ev->valid = false;
    } else if ((ev = events_for(workspace, false)) != nullptr) {
        ev->valid = false;
        ev = nullptr;
    }
    return enqueue_solve(P, insts.data(), n, E, o, F_dtype == FMM_F64, ev, s);
}

// Statistics of problems [0, n) of the last solve in `workspace`.
int read_stats(const void *workspace, int64_t n, fmm_stats *out, void *stream)
{
    if (!workspace || !out || n <= 0 || n > MAX_PROBLEMS) return FMM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Ctrl c;
    if (hipMemcpyAsync(&c, workspace, sizeof c, hipMemcpyDeviceToHost, s) != hipSuccess) return FMM_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return FMM_EHIP;
    // a workspace no solve has initialised holds no statistics
    if (c.magic != CTRL_MAGIC || c.n_inst == 0 || c.n_inst > MAX_PROBLEMS || (int64_t)c.n_inst < n)
        return FMM_EINVAL;
    // the per-problem records follow the control block and the problem table
    const size_t off_ictl = align_up(align_up(sizeof(Ctrl), 256) + sizeof(Inst) * (size_t)c.n_inst, 256);
    std::vector<InstCtl> ic((size_t)n);
    if (hipMemcpyAsync(ic.data(), (const char *)workspace + off_ictl, sizeof(InstCtl) * (size_t)n,
                       hipMemcpyDeviceToHost, s) != hipSuccess)
        return FMM_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return FMM_EHIP;
    double t[3] = {-1.0, -1.0, -1.0};
    if (StageEvents *ev = events_for(workspace, false)) {
        float x[3];
        if (ev->valid && hipEventElapsedTime(&x[0], ev->ev[0], ev->ev[1]) == hipSuccess &&
            hipEventElapsedTime(&x[1], ev->ev[1], ev->ev[2]) == hipSuccess &&
            hipEventElapsedTime(&x[2], ev->ev[2], ev->ev[3]) == hipSuccess) {
            t[0] = x[0];
            t[1] = x[1];
            t[2] = x[2];
        }
    }
    for (int64_t i = 0; i < n; i++) {
        fmm_stats &o = out[i];
        memset(&o, 0, sizeof o);
        o.n_accepted = (int64_t)ic[(size_t)i].n_accepted;
        o.n_restarts = (int64_t)ic[(size_t)i].restarts;
        double m;
        memcpy(&m, &ic[(size_t)i].max_abs_bits, sizeof m);
        o.max_abs_T = m;
        o.n_reopened = (int64_t)c.n_reopen;
        o.n_tile_marches = (int64_t)c.n_march;
        o.n_solves = (int64_t)c.n_solve;
        o.n_rounds = (int64_t)c.n_round;
        o.device_error = c.error | c.error_run;
        o.tile_edge = c.tile_edge;
        o.n_workgroups = (int64_t)c.nwg;
        o.ms_prepare = t[0];
        o.ms_driver = t[1];
        o.ms_finalize = t[2];
    }
    const uint32_t err = c.error | c.error_run;
    if (err & ERR_NOCONV) return FMM_ENOCONV;
    if (err) return FMM_EDEVICE;
    return FMM_OK;
}

}  // namespace

extern "C" {

void fmm_default_opts(fmm_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->band_width = INFINITY;
    o->stride = 0.0;
    o->inner_stride = 0.0;
    o->tile_edge = 8;
    o->max_restarts = 0;
    o->flags = 0;
    o->stride_h = 0.0;
}

size_t fmm_workspace_bytes(int64_t n0, int64_t n1, int64_t n2, int64_t n_seeds, fmm_dtype F_dtype,
                           const fmm_opts *opts)
{
    if (n_seeds < 0 || !opts_ok(opts)) return 0;
    if (F_dtype != FMM_F32 && F_dtype != FMM_F64) return 0;
    Layout L;
    const int64_t d[3] = {n0, n1, n2};
    if (!make_layout(1, d, resolve_edge(opts), F_dtype == FMM_F64 ? 8 : 4, &L, nullptr)) return 0;
    return L.total;
}

int fmm_solve(int64_t n0, int64_t n1, int64_t n2, double h, const void *F, fmm_dtype F_dtype,
              const int64_t *seed_idx, const double *seed_val, int64_t n_seeds, const fmm_opts *opts,
              double *T_out, uint8_t *status_out, void *workspace, size_t workspace_bytes, void *stream)
{
    fmm_problem q;
    q.n0 = n0;
    q.n1 = n1;
    q.n2 = n2;
    q.h = h;
    q.F = F;
    q.seed_idx = seed_idx;
    q.seed_val = seed_val;
    q.n_seeds = n_seeds;
    q.T_out = T_out;
    q.status_out = status_out;
    return run_batch(1, &q, F_dtype, opts, workspace, workspace_bytes, stream);
}

int fmm_solve_noalloc(int64_t n0, int64_t n1, int64_t n2, double h, const void *F, fmm_dtype F_dtype,
                      const int64_t *seed_idx, const double *seed_val, int64_t n_seeds, const fmm_opts *opts,
                      double *T_out, uint8_t *status_out, uint32_t *error_out, void *stream)
{
    fmm_problem q;
    q.n0 = n0;
    q.n1 = n1;
    q.n2 = n2;
    q.h = h;
    q.F = F;
    q.seed_idx = seed_idx;
    q.seed_val = seed_val;
    q.n_seeds = n_seeds;
    q.T_out = T_out;
    q.status_out = status_out;
    int rc = check_solve_args(1, &q, F_dtype, opts);
    if (rc != FMM_OK) return rc;
    fmm_opts o;
    if (opts)
        o = *opts;
    else
        fmm_default_opts(&o);
    o.flags &= ~(uint32_t)FMM_TIMING;  // no stage events: creating them allocates
    const int E = resolve_edge(&o);
    Layout L;
    uint32_t base = 0;
    const int64_t dims[3] = {n0, n1, n2};
    if (!make_layout(1, dims, E, F_dtype == FMM_F64 ? 8 : 4, &L, &base)) return FMM_EINVAL;
    if (L.total > (size_t)FMM_NOALLOC_MAX_BYTES) return FMM_ENOMEM;
    void *ws = scratch_for_current_device();
    if (!ws) return FMM_EHIP;
    const Params P = make_params(L, ws, o);
    const Inst I = make_inst(q, E, base, o);
    hipStream_t s = (hipStream_t)stream;
    rc = enqueue_solve(P, &I, 1, E, o, F_dtype == FMM_F64, nullptr, s);
    if (rc != FMM_OK) return rc;
    if (error_out && launch_report_error(P, error_out, s) != hipSuccess) return FMM_EHIP;
    return FMM_OK;
}

int fmm_get_stats(const void *workspace, fmm_stats *out, void *stream)
{
    return read_stats(workspace, 1, out, stream);
}

size_t fmm_batch_workspace_bytes(int64_t n_problems, const fmm_problem *problems, fmm_dtype F_dtype,
                                 const fmm_opts *opts)
{
    if (n_problems <= 0 || n_problems > MAX_PROBLEMS || !problems || !opts_ok(opts)) return 0;
    if (F_dtype != FMM_F32 && F_dtype != FMM_F64) return 0;
    Layout L;
    const std::vector<int64_t> dims = dims_of(n_problems, problems);
    if (!make_layout(n_problems, dims.data(), resolve_edge(opts), F_dtype == FMM_F64 ? 8 : 4, &L, nullptr))
        return 0;
    return L.total;
}

int fmm_solve_batch(int64_t n_problems, const fmm_problem *problems, fmm_dtype F_dtype, const fmm_opts *opts,
                    void *workspace, size_t workspace_bytes, void *stream)
{
    return run_batch(n_problems, problems, F_dtype, opts, workspace, workspace_bytes, stream);
}

int fmm_get_batch_stats(const void *workspace, int64_t n_problems, fmm_stats *out, void *stream)
{
    return read_stats(workspace, n_problems, out, stream);
}

int fmm_tune_batch(int64_t n_problems, const fmm_problem *problems, fmm_dtype F_dtype, const fmm_opts *opts,
                   const int32_t *edges, int32_t n_edges, const double *strides_h, int32_t n_strides, int32_t reps,
                   void *workspace, size_t workspace_bytes, void *stream, fmm_opts *best, float *ms_out)
{
    if (!edges || n_edges <= 0 || !strides_h || n_strides <= 0 || reps <= 0 || !best) return FMM_EINVAL;
    if (!opts_ok(opts)) return FMM_EINVAL;
    fmm_opts base;
    if (opts)
        base = *opts;
    else
        fmm_default_opts(&base);
    base.flags &= ~(uint32_t)FMM_TIMING;
    for (int32_t a = 0; a < n_edges; a++) {
        if (!(edges[a] == 4 || edges[a] == 8 || edges[a] == 16)) return FMM_EINVAL;
        fmm_opts o = base;
        o.tile_edge = edges[a];
        const size_t need = fmm_batch_workspace_bytes(n_problems, problems, F_dtype, &o);
        if (need == 0) return FMM_EINVAL;
        if (need > workspace_bytes) return FMM_ENOMEM;
    }
    for (int32_t b = 0; b < n_strides; b++)
        if (!(strides_h[b] > 0.0)) return FMM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return FMM_EHIP;
    }
    std::vector<fmm_stats> st((size_t)n_problems);
    float best_ms = -1.0f;
    int rc = FMM_OK;
    for (int32_t a = 0; a < n_edges && rc == FMM_OK; a++) {
        for (int32_t b = 0; b < n_strides && rc == FMM_OK; b++) {
            fmm_opts o = base;
            o.tile_edge = edges[a];
            o.stride_h = strides_h[b];
            float ms = -1.0f;
            bool ok = true;
            for (int32_t k = 0; k <= reps && ok; k++) {
                if (k > 0 && hipEventRecord(e0, s) != hipSuccess) rc = FMM_EHIP;
                int r = run_batch(n_problems, problems, F_dtype, &o, workspace, workspace_bytes, stream);
                if (r != FMM_OK) {
                    rc = r;
                    break;
                }
                if (k > 0 && hipEventRecord(e1, s) != hipSuccess) rc = FMM_EHIP;
                r = read_stats(workspace, n_problems, st.data(), stream);  // synchronises
                if (r == FMM_EHIP) rc = r;
                if (r != FMM_OK) ok = false;
                float x = 0.0f;
                if (k > 0 && ok && rc == FMM_OK) {
                    if (hipEventElapsedTime(&x, e0, e1) != hipSuccess) rc = FMM_EHIP;
                    if (ms < 0.0f || x < ms) ms = x;
                }
            }
            if (!ok) ms = -1.0f;
            if (ms_out) ms_out[a * n_strides + b] = ms;
            if (ms >= 0.0f && (best_ms < 0.0f || ms < best_ms)) {
                best_ms = ms;
                *best = o;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != FMM_OK) return rc;
    if (best_ms < 0.0f) return FMM_EDEVICE;
    return FMM_OK;
}

static bool adj_problem_ok(const fmm_adjoint_problem &q)
{
    int32_t t[3];
    uint64_t nt;
    if (!tile_grid(q.n0, q.n1, q.n2, 4, t, &nt)) return false;
    if (!(q.h > 0.0) || !isfinite(q.h)) return false;
    for (int a = 0; a < 3; a++)
        if (!(q.axis_scale[a] == 0.0 || (q.axis_scale[a] > 0.0 && isfinite(q.axis_scale[a])))) return false;
    return q.F && q.T && q.status && q.dL_dT && q.dL_dF;
}

static uint64_t adj_total(int64_t n, const fmm_adjoint_problem *q, std::vector<AdjInst> *insts)
{
    uint64_t total = 0;
    for (int64_t i = 0; i < n; i++) {
        if (insts) {
            AdjInst &I = (*insts)[(size_t)i];
            memset(&I, 0, sizeof I);
            I.n0 = q[i].n0;
            I.n1 = q[i].n1;
            I.n2 = q[i].n2;
            I.base = (int64_t)total;
            I.h = q[i].h;
            I.F = q[i].F;
            I.T = q[i].T;
            I.status = q[i].status;
            I.dL_dT = q[i].dL_dT;
            I.dL_dF = q[i].dL_dF;
            I.sp = spacing_of(q[i].axis_scale);
        }
        total += (uint64_t)(q[i].n0 * q[i].n1 * q[i].n2);
    }
    return total;
}

size_t fmm_adjoint_workspace_bytes(int64_t n_problems, const fmm_adjoint_problem *problems)
{
    if (n_problems <= 0 || n_problems > MAX_PROBLEMS || !problems) return 0;
    for (int64_t i = 0; i < n_problems; i++) {
        int32_t t[3];
        uint64_t nt;
        if (!tile_grid(problems[i].n0, problems[i].n1, problems[i].n2, 4, t, &nt)) return 0;
    }
    return adj_layout(n_problems, adj_total(n_problems, problems, nullptr)).total;
}

int fmm_adjoint_batch(int64_t n_problems, const fmm_adjoint_problem *problems, fmm_dtype F_dtype,
                      void *workspace, size_t workspace_bytes, void *stream)
{
    if (n_problems <= 0 || n_problems > MAX_PROBLEMS || !problems || !workspace) return FMM_EINVAL;
    if (F_dtype != FMM_F32 && F_dtype != FMM_F64) return FMM_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return FMM_EINVAL;
    for (int64_t i = 0; i < n_problems; i++)
        if (!adj_problem_ok(problems[i])) return FMM_EINVAL;
    // problems that share an output array must have the same grid
    std::unordered_map<const void *, int64_t> out_owner;
    for (int64_t i = 0; i < n_problems; i++) {
        auto it = out_owner.emplace(problems[i].dL_dF, i).first;
        const fmm_adjoint_problem &a = problems[it->second], &b = problems[i];
        if (a.n0 != b.n0 || a.n1 != b.n1 || a.n2 != b.n2) return FMM_EINVAL;
    }
    std::vector<AdjInst> insts((size_t)n_problems);
    const uint64_t total = adj_total(n_problems, problems, &insts);
    if (total >= (1ull << 40)) return FMM_EINVAL;
    const AdjLayout L = adj_layout(n_problems, total);
    if (workspace_bytes < L.total) return FMM_ENOMEM;
    char *b = (char *)workspace;
    AdjParams P;
    P.ctrl = (AdjCtrl *)(b + L.off_ctrl);
    P.inst = (const AdjInst *)(b + L.off_inst);
    P.acc = (double *)(b + L.off_acc);
    P.cnt = (uint32_t *)(b + L.off_cnt);
    P.code = (uint8_t *)(b + L.off_code);
    P.list0 = (uint64_t *)(b + L.off_list0);
    P.list1 = (uint64_t *)(b + L.off_list1);
    if (launch_adjoint(P, insts.data(), n_problems, F_dtype == FMM_F64, (hipStream_t)stream) != hipSuccess)
        return FMM_EHIP;
    return FMM_OK;
}

int fmm_adjoint(int64_t n0, int64_t n1, int64_t n2, double h, const void *F, fmm_dtype F_dtype, const double *T,
                const uint8_t *status, const double *dL_dT, double *dL_dF, void *workspace, size_t workspace_bytes,
                void *stream)
{
    fmm_adjoint_problem q;
    q.n0 = n0;
    q.n1 = n1;
    q.n2 = n2;
    q.h = h;
    q.F = F;
    q.T = T;
    q.status = status;
    q.dL_dT = dL_dT;
    q.dL_dF = dL_dF;
    q.axis_scale[0] = q.axis_scale[1] = q.axis_scale[2] = 0.0;
    return fmm_adjoint_batch(1, &q, F_dtype, workspace, workspace_bytes, stream);
}

int fmm_get_adjoint_stats(const void *workspace, fmm_adjoint_stats *out, void *stream)
{
    if (!workspace || !out) return FMM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    AdjCtrl c;
    if (hipMemcpyAsync(&c, workspace, sizeof c, hipMemcpyDeviceToHost, s) != hipSuccess) return FMM_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return FMM_EHIP;
    memset(out, 0, sizeof *out);
    if (c.magic != ADJ_MAGIC) return FMM_EINVAL;
    out->n_points = (int64_t)c.n_points;
    out->n_levels = (int64_t)c.levels;
    out->device_error = c.error;
    return c.error ? FMM_EDEVICE : FMM_OK;
}

int fmm_eval_godunov(const double *a, const double *r, double *out, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!a || !r || !out))) return FMM_EINVAL;
    return launch_eval_godunov(a, r, out, n, (hipStream_t)stream) == hipSuccess ? FMM_OK : FMM_EHIP;
}

const char *fmm_strerror(int status)
{
    switch (status) {
    case FMM_OK: return "ok";
    case FMM_EINVAL: return "invalid argument";
    case FMM_ENOMEM: return "workspace too small";
    case FMM_EHIP: return "HIP runtime error";
    case FMM_ENOCONV: return "restart limit reached";
    case FMM_EDEVICE: return "device-detected input error or abort";
    default: return "unknown status";
    }
}

}  // extern "C"
