// Internal definitions of the adjoint kernels (fmm_adjoint.hip) shared with
// the host side of libfmm.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fmm_device.h"

namespace fmm {

// One problem of an adjoint batch (device copy).  Arrays are the caller's,
// row-major (n0, n1, n2).
struct AdjInst {
    int64_t n0, n1, n2;
    int64_t base;  // global index of the problem's first point in the workspace arrays
    double h;
    const void *F;
    const double *T;
    const uint8_t *status;
    const double *dL_dT;
    double *dL_dF;
    Spacing sp;  // per-axis spacing factors (weights 1 / s^2)
};

enum : uint32_t { ADJ_ERR_BARRIER = 32u };
constexpr uint32_t ADJ_MAGIC = 0x41444a31u;

struct AdjCtrl {
    alignas(128) uint32_t bar;  // grid barrier arrivals (monotonic)
    alignas(128) uint32_t abort;
    uint32_t error;
    uint32_t n_inst;
    uint32_t nwg;
    uint32_t levels;                  // frontier levels processed
    uint32_t magic;                   // ADJ_MAGIC once a run has initialised the workspace
    alignas(128) unsigned long long len[3];  // frontier lengths, by level mod 3
    alignas(128) unsigned long long n_points;  // points of the linear system
};

struct AdjParams {
    AdjCtrl *ctrl;
    const AdjInst *inst;
    double *acc;      // per point: S_p lambda_p being accumulated; once processed, its dL/dF term
    uint32_t *cnt;    // per point: dependents not yet processed
    uint8_t *code;    // per point: upwind set, 2 bits per axis
    uint64_t *list0, *list1;  // frontiers
};

constexpr int ADJ_PACK = 16;
struct AdjPack {
    AdjInst v[ADJ_PACK];
    uint32_t first, n;
};

// Output gather: out[p] (accumulate ? += : =) sum over the m problems whose
// points start at base[k] of their gradient terms.
constexpr int ADJ_GATHER = 64;
struct AdjGather {
    double *out;
    int64_t n;
    int64_t base[ADJ_GATHER];
    uint32_t m, accumulate;
};

// Workspace carving for `total` points over n problems.
struct AdjLayout {
    size_t off_ctrl, off_inst, off_acc, off_cnt, off_code, off_list0, off_list1, total;
};

inline size_t adj_align(size_t x) { return (x + 255) / 256 * 256; }

inline AdjLayout adj_layout(int64_t n, uint64_t total)
{
    AdjLayout L;
    size_t o = 0;
    L.off_ctrl = o;
    o = adj_align(o + sizeof(AdjCtrl));
    L.off_inst = o;
    o = adj_align(o + sizeof(AdjInst) * (size_t)n);
    L.off_acc = o;
    o = adj_align(o + 8 * total);
    L.off_cnt = o;
    o = adj_align(o + 4 * total);
    L.off_code = o;
    o = adj_align(o + total);
    L.off_list0 = o;
    o = adj_align(o + 8 * total);
    L.off_list1 = o;
    o = adj_align(o + 8 * total);
    L.total = o;
    return L;
}

hipError_t launch_adjoint(const AdjParams &P, const AdjInst *insts, int64_t n, bool f64, hipStream_t s);

}  // namespace fmm
