// C ABI of libfmm (declared in include/fmm.h): argument validation, workspace
// carving and the enqueue sequence: workspace reset, tiled speeds, seeds ->
// restart driver -> finalize.
#include <math.h>
#include <string.h>

#include <mutex>
#include <unordered_map>

#include "../../include/fmm.h"
#include "fmm_internal.h"

using namespace fmm;

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
    if (isnan(o->stride) || isnan(o->inner_stride)) return false;
    if (!(o->tile_edge == 0 || o->tile_edge == 4 || o->tile_edge == 8 || o->tile_edge == 16)) return false;
    if (o->max_restarts < 0) return false;
    if (o->flags & ~(uint32_t)(FMM_VALIDATE | FMM_TIMING | FMM_ONE_MARCH)) return false;
    return true;
}

Params make_params(int64_t n0, int64_t n1, int64_t n2, double h, const void *F, double *T, const Layout &L,
                   void *ws, double width, double stride, double inner, int64_t max_restarts,
                   uint32_t time_limit_s)
{
    char *b = (char *)ws;
    Params P;
    memset(&P, 0, sizeof P);
    P.n0 = n0;
    P.n1 = n1;
    P.n2 = n2;
    P.t0 = L.t0;
    P.t1 = L.t1;
    P.t2 = L.t2;
    P.ntiles = L.ntiles;
    P.mask_words = L.mask_words;
    P.h = h;
    P.width = width;
    P.stride = stride;
    P.inner = inner;
    P.two_march = 1;
    P.max_restarts = max_restarts;
    // the driver reads the 100 MHz constant clock
    P.time_limit_ticks = 100000000ull * (unsigned long long)(time_limit_s ? time_limit_s : 300u);
    P.T = T;
    P.F = F;
    P.ctrl = (Ctrl *)(b + L.off_ctrl);
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
}

size_t fmm_workspace_bytes(int64_t n0, int64_t n1, int64_t n2, int64_t n_seeds, fmm_dtype F_dtype,
                           const fmm_opts *opts)
{
    if (n_seeds < 0 || !opts_ok(opts)) return 0;
    if (F_dtype != FMM_F32 && F_dtype != FMM_F64) return 0;
    Layout L;
    if (!make_layout(n0, n1, n2, resolve_edge(opts), F_dtype == FMM_F64 ? 8 : 4, &L)) return 0;
    return L.total;
}

int fmm_solve(int64_t n0, int64_t n1, int64_t n2, double h, const void *F, fmm_dtype F_dtype,
              const int64_t *seed_idx, const double *seed_val, int64_t n_seeds, const fmm_opts *opts,
              double *T_out, uint8_t *status_out, void *workspace, size_t workspace_bytes, void *stream)
{
    if (n0 <= 0 || n1 <= 0 || n2 <= 0) return FMM_EINVAL;
    if (n0 > (1ll << 40) / n1 / n2) return FMM_EINVAL;
    if (!(h > 0.0) || !isfinite(h)) return FMM_EINVAL;
    if (!F || !T_out || !workspace) return FMM_EINVAL;
    if (F_dtype != FMM_F32 && F_dtype != FMM_F64) return FMM_EINVAL;
    if (n_seeds < 0 || (n_seeds > 0 && (!seed_idx || !seed_val))) return FMM_EINVAL;
    if (!opts_ok(opts)) return FMM_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return FMM_EINVAL;
    fmm_opts o;
    if (opts)
        o = *opts;
    else
        fmm_default_opts(&o);
    const int E = resolve_edge(&o);
    Layout L;
    if (!make_layout(n0, n1, n2, E, F_dtype == FMM_F64 ? 8 : 4, &L)) return FMM_EINVAL;
    if (workspace_bytes < L.total) return FMM_ENOMEM;
    const double stride = (o.stride > 0.0) ? o.stride : 2.0 * h;
    const int64_t maxr = o.max_restarts > 0 ? (int64_t)o.max_restarts : 0;
    const double inner = (o.inner_stride > 0.0) ? o.inner_stride : INFINITY;
    Params P = make_params(n0, n1, n2, h, F, T_out, L, workspace, o.band_width, stride, inner, maxr, o.time_limit_s);
    P.two_march = (o.flags & FMM_ONE_MARCH) ? 0 : 1;
    hipStream_t s = (hipStream_t)stream;
    const bool f64 = F_dtype == FMM_F64;
    StageEvents *ev = nullptr;
    if (o.flags & FMM_TIMING) {
        ev = events_for(workspace, true);
        if (!ev) return FMM_EHIP;
        ev->valid = false;
    } else if ((ev = events_for(workspace, false)) != nullptr) {
        ev->valid = false;
        ev = nullptr;
    }
    if (ev && hipEventRecord(ev->ev[0], s) != hipSuccess) return FMM_EHIP;
    if (launch_prepare(P, seed_idx, seed_val, n_seeds, E, (o.flags & FMM_VALIDATE) != 0, f64, s) != hipSuccess)
        return FMM_EHIP;
    if (ev && hipEventRecord(ev->ev[1], s) != hipSuccess) return FMM_EHIP;
    uint32_t nwg = 0;
    if (launch_driver(P, E, f64, s, &nwg) != hipSuccess) return FMM_EHIP;
    if (ev && hipEventRecord(ev->ev[2], s) != hipSuccess) return FMM_EHIP;
    if (launch_finalize(P, E, status_out, s) != hipSuccess) return FMM_EHIP;
    if (ev) {
        if (hipEventRecord(ev->ev[3], s) != hipSuccess) return FMM_EHIP;
        ev->valid = true;
    }
    return FMM_OK;
}

int fmm_get_stats(const void *workspace, fmm_stats *out, void *stream)
{
    if (!workspace || !out) return FMM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Ctrl c;
    if (hipMemcpyAsync(&c, workspace, sizeof c, hipMemcpyDeviceToHost, s) != hipSuccess) return FMM_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return FMM_EHIP;
    memset(out, 0, sizeof *out);
    out->n_accepted = (int64_t)c.n_accepted;
    out->n_restarts = (int64_t)c.restarts;
    out->n_reopened = (int64_t)c.n_reopen;
    out->n_tile_marches = (int64_t)c.n_march;
    out->n_solves = (int64_t)c.n_solve;
    out->n_rounds = (int64_t)c.n_round;
    double m;
    memcpy(&m, &c.max_abs_bits, sizeof m);
    out->max_abs_T = m;
    out->device_error = c.error | c.error_run;
    out->tile_edge = c.tile_edge;
    out->n_workgroups = (int64_t)c.nwg;
    out->ms_prepare = out->ms_driver = out->ms_finalize = -1.0;
    if (StageEvents *ev = events_for(workspace, false)) {
        float t[3];
        if (ev->valid && hipEventElapsedTime(&t[0], ev->ev[0], ev->ev[1]) == hipSuccess &&
            hipEventElapsedTime(&t[1], ev->ev[1], ev->ev[2]) == hipSuccess &&
            hipEventElapsedTime(&t[2], ev->ev[2], ev->ev[3]) == hipSuccess) {
            out->ms_prepare = t[0];
            out->ms_driver = t[1];
            out->ms_finalize = t[2];
        }
    }
    if (out->device_error & ERR_NOCONV) return FMM_ENOCONV;
    if (out->device_error) return FMM_EDEVICE;
    return FMM_OK;
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
