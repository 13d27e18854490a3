// Internal definitions shared by the kernels and the host side of libfmm.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fmm {

// Per-restart bookkeeping.  Restart r reads slot[r % 3] (band minimum per side,
// live-tile list length, tiles left dirty by the previous restart) and
// accumulates into slot[(r + 1) % 3]; slot[(r + 2) % 3] is cleared at its start.
struct alignas(128) Slot {
    unsigned long long gmin[2];  // bit patterns of non-negative doubles
    uint32_t live_len;           // entries of the live-tile list for this restart
    uint32_t pending;            // tiles dirtied after the last march of the previous restart
    uint32_t d_len;              // tiles dirtied during march-1 of this restart
    uint32_t pad[25];
};

constexpr int WORK_SEGS = 8;  // item-list segments, one per XCD

struct Ctrl {
    alignas(128) uint32_t bar;  // grid barrier arrivals (monotonic)
    alignas(128) uint32_t abort;
    uint32_t error;      // input errors found before the driver starts
    uint32_t error_run;  // errors raised while the restart driver runs
    uint32_t restarts;
    uint32_t nwg;
    uint32_t tile_edge;
    alignas(128) Slot slot[3];
    alignas(128) unsigned long long n_march;
    unsigned long long n_solve;
    unsigned long long n_round;
    unsigned long long n_reopen;
    unsigned long long n_accepted;
    unsigned long long max_abs_bits;
    // cycle counters of builds with FMM_PROFILE defined (zero otherwise)
    alignas(128) unsigned long long prof[16];
    // work counters of the phase loop: per phase (mod 3) one counter per
    // segment of the item list, 128 B apart so that each has its own line
    alignas(128) uint32_t work[3][WORK_SEGS][32];
};

// Per-tile record: smallest |T| per side among the tile's pending band values
// (see the march) and the band bound of the tile's last march.
struct TileMeta {
    double tmin[2];
    double lastb[2];
};

enum : uint32_t { TF_SEED = 1u, TF_INIT = 2u };

enum : uint32_t {
    ERR_SEED_RANGE = 1u,
    ERR_SEED_DUP = 2u,
    ERR_SEED_VALUE = 4u,
    ERR_SPEED = 8u,
    ERR_NOCONV = 16u,
    ERR_BARRIER = 32u,
    ERR_ROUNDS = 64u,
    ERR_LAUNCH = 128u,
    ERR_TIMEOUT = 256u,
};

// Carving of the caller's workspace.  Besides the per-tile bookkeeping it
// holds the tiled working copies of T and F (each tile's E^3 values
// contiguous, axis 2 fastest inside the tile) and, per tile, the two faces
// normal to axis 2 (the only halo faces that are strided in the tiled layout).
struct Layout {
    int E;
    int32_t t0, t1, t2;
    uint32_t ntiles;
    uint32_t mask_words;  // 64-bit seed-mask words per tile
    size_t off_ctrl, off_meta, off_dirty0, off_dirty1, off_epoch, off_flags, off_visit, off_text, off_mask,
        off_list0, off_list1, off_dlist, off_Tt, off_Ft, off_Zf, total;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline bool make_layout(int64_t n0, int64_t n1, int64_t n2, int E, size_t fsize, Layout *L)
{
    if (n0 <= 0 || n1 <= 0 || n2 <= 0) return false;
    if (!(E == 4 || E == 8 || E == 16)) return false;
    int64_t t0 = (n0 + E - 1) / E, t1 = (n1 + E - 1) / E, t2 = (n2 + E - 1) / E;
    int64_t nt = t0 * t1 * t2;
    if (nt >= (int64_t)0xFFFFFFF0u || t0 > INT32_MAX || t1 > INT32_MAX || t2 > INT32_MAX) return false;
    L->E = E;
    L->t0 = (int32_t)t0;
    L->t1 = (int32_t)t1;
    L->t2 = (int32_t)t2;
    L->ntiles = (uint32_t)nt;
    L->mask_words = (uint32_t)((E * E * E + 63) / 64);
    size_t o = 0;
    L->off_ctrl = o;
    o = align_up(o + sizeof(Ctrl), 256);
    L->off_meta = o;
    o = align_up(o + sizeof(TileMeta) * nt, 256);
    L->off_dirty0 = o;
    o = align_up(o + 4 * nt, 256);
    L->off_dirty1 = o;
    o = align_up(o + 4 * nt, 256);
    L->off_epoch = o;
    o = align_up(o + 4 * nt, 256);
    L->off_flags = o;
    o = align_up(o + 4 * nt, 256);
    L->off_visit = o;
    o = align_up(o + 4 * nt, 256);
    L->off_text = o;
    o = align_up(o + 48 * nt, 256);
    L->off_mask = o;
    o = align_up(o + 8 * (size_t)L->mask_words * nt, 256);
    L->off_list0 = o;
    o = align_up(o + 4 * nt, 256);
    L->off_list1 = o;
    o = align_up(o + 4 * nt, 256);
    L->off_dlist = o;
    o = align_up(o + 4 * nt, 256);
    const size_t V = (size_t)E * E * E;
    L->off_Tt = o;
    o = align_up(o + 8 * V * nt, 256);
    L->off_Ft = o;
    o = align_up(o + fsize * V * nt, 256);
    L->off_Zf = o;
    o = align_up(o + 8 * 2 * (size_t)E * E * nt, 256);
    L->total = o;
    return true;
}

struct Params {
    int64_t n0, n1, n2;
    int32_t t0, t1, t2;
    uint32_t ntiles;
    uint32_t mask_words;
    double h, width, stride, inner;
    int64_t max_restarts;
    int32_t two_march;  // second march of Alg. 16 after the exchange (1) or not (0)
    unsigned long long time_limit_ticks;  // restart-driver wall-clock limit (100 MHz ticks)
    double *T;        // output, row-major (written by the finalize kernel)
    const void *F;    // input speeds, row-major
    double *Tt;       // tiled working T
    void *Ft;         // tiled speeds (type of F)
    double *Zf;       // per tile: its i2 = 0 and i2 = E-1 faces
    Ctrl *ctrl;
    TileMeta *meta;
    uint32_t *dirty0, *dirty1, *epoch, *tflags;
    uint32_t *visit;  // 0: never written; else 1 + the phase that first wrote the tile
    // per tile, phase slot (phase % 3) and side: smallest band value a
    // neighbour passed on in that phase, [(t * 3 + slot) * 2 + side]
    unsigned long long *text;
    unsigned long long *mask;
    uint32_t *list0, *list1, *dlist;
};

// Host-side launchers (defined in fmm_kernels.hip).
hipError_t launch_prepare(const Params &P, const int64_t *seed_idx, const double *seed_val, int64_t n_seeds,
                          int E, bool validate, bool f64, hipStream_t s);
hipError_t launch_driver(const Params &P, int E, bool f64, hipStream_t s, uint32_t *nwg_out);
hipError_t launch_finalize(const Params &P, int E, uint8_t *status, hipStream_t s);
hipError_t launch_eval_godunov(const double *a, const double *r, double *out, int64_t n, hipStream_t s);

}  // namespace fmm
