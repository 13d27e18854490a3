// Internal definitions shared by the kernels and the host side of libfmm.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fmm_device.h"

namespace fmm {

// Per-restart bookkeeping of the shared tile lists.  Restart r reads
// slot[r % 3] (live-tile list length) and appends into slot[(r + 1) % 3];
// slot[(r + 2) % 3] is cleared at its start.
struct alignas(128) Slot {
    uint32_t live_len;  // entries of the live-tile list for this restart
    uint32_t d_len;     // tiles dirtied during march-1 of this restart
    uint32_t pad[30];
};

// One problem of a batch: its grid, its place in the tile numbering and its
// caller buffers.  A single solve is a batch of one.
struct Inst {
    int64_t n0, n1, n2;
    int32_t t0, t1, t2;  // tiles per axis
    uint32_t base;       // global index of the problem's first tile
    uint32_t ntiles;
    uint32_t pad;
    double h, stride;
    const void *F;  // row-major speeds
    double *T;      // row-major output
    uint8_t *status;
    const int64_t *seed_idx;
    const double *seed_val;
    int64_t n_seeds;
};

// Per-problem restart state (Alg. 16 runs once per problem: its own minimum,
// bound, dirty count and exit test).  Restart r reads slot[r % 3] and
// accumulates into slot[(r + 1) % 3].
struct alignas(64) InstSlot {
    unsigned long long gmin[2];  // bit patterns of non-negative doubles
    uint32_t pending;            // tiles dirtied after the last march of the previous restart
    uint32_t pad[11];
};
struct alignas(128) InstCtl {
    InstSlot slot[3];
    uint32_t restarts;  // restart at which the exit test passed (0: still running)
    uint32_t pad;
    unsigned long long n_accepted;
    unsigned long long max_abs_bits;
};

constexpr int WORK_SEGS = 8;  // item-list segments, one per XCD
constexpr uint32_t CTRL_MAGIC = 0x464d4d31u;

struct Ctrl {
    alignas(128) uint32_t bar;  // grid barrier arrivals (monotonic)
    alignas(128) uint32_t abort;
    uint32_t error;      // input errors found before the driver starts
    uint32_t error_run;  // errors raised while the restart driver runs
    uint32_t restarts;   // restarts of the whole batch
    uint32_t nwg;
    uint32_t tile_edge;
    uint32_t n_inst;  // problems of the last solve
    uint32_t magic;   // CTRL_MAGIC once a solve has initialised the workspace
    alignas(128) Slot slot[3];
    alignas(128) unsigned long long n_march;
    unsigned long long n_solve;
    unsigned long long n_round;
    unsigned long long n_reopen;
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
// The tiles of the problems of a batch are numbered consecutively, problem by
// problem; every per-tile array is indexed by that global number.
struct Layout {
    int E;
    uint32_t n_inst;
    uint32_t ntiles;      // over all problems
    uint32_t mask_words;  // 64-bit seed-mask words per tile
    size_t off_ctrl, off_inst, off_ictl, off_tinst, off_meta, off_dirty0, off_dirty1, off_epoch, off_flags,
        off_visit, off_text, off_mask, off_list0, off_list1, off_dlist, off_Tt, off_Ft, off_Zf, total;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr int64_t MAX_PROBLEMS = 1 << 20;

// Tiles per axis of an n0 x n1 x n2 grid; false for an invalid grid.
inline bool tile_grid(int64_t n0, int64_t n1, int64_t n2, int E, int32_t t[3], uint64_t *nt)
{
    if (n0 <= 0 || n1 <= 0 || n2 <= 0) return false;
    if (n0 > (1ll << 40) / n1 / n2) return false;
    const int64_t a = (n0 + E - 1) / E, b = (n1 + E - 1) / E, c = (n2 + E - 1) / E;
    if (a > INT32_MAX || b > INT32_MAX || c > INT32_MAX) return false;
    t[0] = (int32_t)a;
    t[1] = (int32_t)b;
    t[2] = (int32_t)c;
    *nt = (uint64_t)a * (uint64_t)b * (uint64_t)c;
    return true;
}

// dims: 3 extents per problem.  bases (nullable): first global tile of each
// problem.
inline bool make_layout(int64_t n_inst, const int64_t *dims, int E, size_t fsize, Layout *L, uint32_t *bases)
{
    if (n_inst <= 0 || n_inst > MAX_PROBLEMS || !dims) return false;
    if (!(E == 4 || E == 8 || E == 16)) return false;
    uint64_t nt = 0;
    for (int64_t i = 0; i < n_inst; i++) {
        int32_t t[3];
        uint64_t n = 0;
        if (!tile_grid(dims[3 * i], dims[3 * i + 1], dims[3 * i + 2], E, t, &n)) return false;
        if (bases) bases[i] = (uint32_t)nt;
        nt += n;
        if (nt >= 0xFFFFFFF0ull) return false;
    }
    L->E = E;
    L->n_inst = (uint32_t)n_inst;
    L->ntiles = (uint32_t)nt;
    L->mask_words = (uint32_t)((E * E * E + 63) / 64);
    size_t o = 0;
    L->off_ctrl = o;
    o = align_up(o + sizeof(Ctrl), 256);
    L->off_inst = o;
    o = align_up(o + sizeof(Inst) * (size_t)n_inst, 256);
    L->off_ictl = o;
    o = align_up(o + sizeof(InstCtl) * (size_t)n_inst, 256);
    L->off_tinst = o;
    o = align_up(o + 4 * nt, 256);
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
    Spacing sp;  // per-axis spacing factors of the batch
    uint32_t n_inst;
    uint32_t ntiles;  // over all problems
    uint32_t mask_words;
    double width, inner;
    int64_t max_restarts;
    int32_t two_march;  // second march of Alg. 16 after the exchange (1) or not (0)
    unsigned long long time_limit_ticks;  // restart-driver wall-clock limit (100 MHz ticks)
    const Inst *inst;     // problem descriptors
    InstCtl *ictl;        // per-problem restart state and statistics
    uint32_t *tinst;      // problem of each tile
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

// Host-side launchers (defined in fmm_kernels.hip).  `insts` is a host array
// of the n problem descriptors (the same values the workspace holds).
hipError_t launch_prepare(const Params &P, const Inst *insts, int64_t n, int E, bool validate, bool f64,
                          hipStream_t s);
hipError_t launch_driver(const Params &P, int E, bool f64, hipStream_t s, uint32_t *nwg_out);
hipError_t launch_finalize(const Params &P, const Inst *insts, int64_t n, int E, hipStream_t s);
hipError_t launch_eval_godunov(const double *a, const double *r, double *out, int64_t n, hipStream_t s);
hipError_t launch_report_error(const Params &P, uint32_t *out, hipStream_t s);

}  // namespace fmm
