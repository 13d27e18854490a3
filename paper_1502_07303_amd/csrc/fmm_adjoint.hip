// Adjoint of the discrete Eikonal solve: dL/dF from dL/dT on the GPU.
//
// The paper solves the first-order Godunov system (Sec. 2.1, Eqs. 2-3) and
// does not differentiate it; this is an extension built on that
// discretisation.  At the forward solution every accepted non-seed point p
// with F_p > 0 satisfies, with u = |T| and U_p its upwind set (for each of the
// k axes whose values the local solver's root used, the neighbour on that
// axis with the smaller value),
//     sum_{q in U_p} w_q (u_p - u_q)^2 = (h / F_p)^2,
// (w_q = 1 / s^2 for a grid spacing h s along q's axis, 1 on a uniform grid)
// and its linearisation is
//     S_p du_p - sum_{q in U_p} w_q (u_p - u_q) du_q = -(h^2 / F_p^3) dF_p,
//     S_p = sum_{q in U_p} w_q (u_p - u_q).
// Seeds and points outside the accepted set are fixed.  The transposed system
// is solved exactly, in reverse dependency order: with lt_q = S_q lambda_q,
//     lt_q = dL/du_q + sum_{p : q in U_p} (w_q (u_p - u_q) / S_p) lt_p,
//     dL/dF_p = -(h^2 / (F_p^3 S_p)) lt_p,
// where dL/du = sign(T) dL/dT.  Since u_q < u_p for q in U_p, the dependency
// graph is acyclic: a point is final once all the points that used it are.
//
// GPU mapping: one setup pass per problem recomputes U_p from the final T
// (the same local solver as the forward march, so the same root and the same
// k) into 2 bits per axis, and counts each point's dependents.  A persistent
// cooperative kernel then processes frontiers level by level: a frontier
// point pushes its contributions to its upwind points with FP64 atomics and
// decrements their counters; the point whose counter reaches zero joins the
// next frontier.  All problems of a batch share the frontiers.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fmm_device.h"
#include "fmm_adjoint.h"

namespace fmm {

constexpr uint64_t ADJ_LOCAL_MASK = (1ull << 40) - 1;  // item = problem << 40 | local point

// Upwind set of point p of problem I from the final values (the forward
// march's Alg. 11 filter and root): 2 bits per axis, 1 = the minus neighbour,
// 2 = the plus neighbour, 0 = not used.  Returns 0 when p is not an accepted
// non-seed point with F > 0 (or has no upwind value).
template <typename FT>
__device__ __forceinline__ uint32_t upwind_code(const AdjInst &I, int64_t p, int64_t i0, int64_t i1, int64_t i2)
{
    const uint8_t st = I.status[p];
    if ((st & 3u) != 2u) return 0;
    const double f = (double)((const FT *)I.F)[p];
    if (!(f > 0.0)) return 0;
    const double up = fabs(I.T[p]);
    const uint8_t side = st & 0x80u;
    const int64_t n[3] = {I.n0, I.n1, I.n2};
    const int64_t c[3] = {i0, i1, i2};
    const int64_t str[3] = {I.n1 * I.n2, I.n2, 1};
    double a[3];
    uint32_t pick[3];
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        a[ax] = FMM_INF;
        pick[ax] = 0;
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const bool in = s == 0 ? c[ax] > 0 : c[ax] + 1 < n[ax];
            if (!in) continue;
            const int64_t q = s == 0 ? p - str[ax] : p + str[ax];
            const uint8_t sq = I.status[q];
            if ((sq & 3u) < 2u || (sq & 0x80u) != side) continue;
            const double v = fabs(I.T[q]);
            if (v < up && v < a[ax]) {
                a[ax] = v;
                pick[ax] = (uint32_t)(s + 1);
            }
        }
    }
    int k = 0;
    (void)local_solve(I.sp, a[0], a[1], a[2], I.h / f, &k);
    // the k smallest per-axis values, ties in axis order
    uint32_t code = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        int rank = 0;
#pragma unroll
        for (int b = 0; b < 3; b++)
            if (b != ax && (a[b] < a[ax] || (a[b] == a[ax] && b < ax))) rank++;
        if (rank < k) code |= pick[ax] << (2 * ax);
    }
    return code;
}

// Counter offset of points outside the linear system (see k_adj_setup).
constexpr uint32_t ADJ_FIXED_COUNT = 1u << 30;

// Reset: accumulators, counters and codes of every problem.
__global__ void k_adj_zero(AdjParams P, AdjInst I)
{
    const int64_t N = I.n0 * I.n1 * I.n2;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = I.base + p;
        P.acc[g] = 0.0;
        P.cnt[g] = 0u;
        P.code[g] = 0u;
    }
}

template <typename FT> __global__ void k_adj_setup(AdjParams P, AdjInst I)
{
    const int64_t N = I.n0 * I.n1 * I.n2;
    const int64_t n12 = I.n1 * I.n2;
    unsigned long long mine = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i0 = p / n12, rem = p - i0 * n12, i1 = rem / I.n2, i2 = rem - i1 * I.n2;
        const uint32_t code = upwind_code<FT>(I, p, i0, i1, i2);
        if (!code) {
            // a fixed point (seed or outside the accepted set): its counter
            // starts far above the at most six decrements it can receive, so
            // it never reaches zero and never joins a frontier
            atomicAdd(&P.cnt[I.base + p], ADJ_FIXED_COUNT);
            continue;
        }
        mine++;
        const int64_t g = I.base + p;
        P.code[g] = (uint8_t)code;
        const double sgn = I.T[p] < 0.0 ? -1.0 : 1.0;
        P.acc[g] = sgn * I.dL_dT[p];
        const int64_t str[3] = {n12, I.n2, 1};
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            const uint32_t c = (code >> (2 * ax)) & 3u;
            if (c) atomicAdd(&P.cnt[I.base + (c == 1 ? p - str[ax] : p + str[ax])], 1u);
        }
    }
    mine = wave_sum(mine);
    if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&P.ctrl->n_points, mine);
}

// Wave-aggregated append of up to one item per lane.
__device__ __forceinline__ void push_item(bool want, uint64_t item, unsigned long long *len, uint64_t *list)
{
    const unsigned long long m = __ballot(want);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    unsigned long long base = 0;
    const int leader = __ffsll((long long)m) - 1;
    if (lane == leader) base = atomicAdd(len, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    if (want) list[base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull))] = item;
}

// First frontier: points in the system that no other point used.
__global__ void k_adj_front0(AdjParams P, AdjInst I, uint32_t j)
{
    const int64_t N = I.n0 * I.n1 * I.n2;
    const int64_t n_iter = (N + (int64_t)blockDim.x - 1) / blockDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_iter;
         p += (int64_t)gridDim.x * blockDim.x) {
        bool want = false;
        if (p < N) {
            const int64_t g = I.base + p;
            want = P.code[g] != 0 && P.cnt[g] == 0;
        }
        push_item(want, ((uint64_t)j << 40) | (uint64_t)p, &P.ctrl->len[0], P.list0);
    }
}

#ifndef FMM_ADJ_WG_PER_CU
#define FMM_ADJ_WG_PER_CU 1
#endif
#ifndef FMM_ADJ_BLOCK
#define FMM_ADJ_BLOCK 256
#endif
constexpr int ADJ_BLOCK = FMM_ADJ_BLOCK;

// Process one frontier point: its gradient term, its contributions to its
// upwind points, and the upwind points whose last dependent it was join the
// next frontier (read only after the barrier that ends this level, so every
// contribution to them is complete).  New frontier entries are staged in LDS
// and appended with one atomic per workgroup.
template <typename FT>
__device__ __forceinline__ void adj_point(const AdjParams &P, uint64_t it, bool active, uint64_t *s_items,
                                          uint32_t *s_n)
{
    if (!active) return;
    const uint32_t j = (uint32_t)(it >> 40);
    const int64_t p = (int64_t)(it & ADJ_LOCAL_MASK);
    const AdjInst &I = P.inst[j];
    const int64_t g = I.base + p;
    const double lt = __hip_atomic_load(&P.acc[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t code = P.code[g];
    const double up = fabs(I.T[p]);
    const double f = (double)((const FT *)I.F)[p];
    const int64_t str[3] = {I.n1 * I.n2, I.n2, 1};
    int64_t q[3];
    double d[3];
    double S = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        // weighted difference w_a (u_p - u_q), w_a = 1 / s_a^2 (1 on a uniform grid)
        const uint32_t cc = (code >> (2 * ax)) & 3u;
        const double w = I.sp.aniso ? 1.0 / (I.sp.s[ax] * I.sp.s[ax]) : 1.0;
        q[ax] = cc == 0 ? -1 : (cc == 1 ? p - str[ax] : p + str[ax]);
        d[ax] = cc == 0 ? 0.0 : w * (up - fabs(I.T[q[ax]]));
        S += d[ax];
    }
    // this point's gradient term; its accumulator is not needed any more
    P.acc[g] = -(I.h * I.h) / (f * f * f * S) * lt;
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        if (q[ax] < 0) continue;
        const int64_t gq = I.base + q[ax];
        atomicAdd(&P.acc[gq], (d[ax] / S) * lt);
        // the last dependent of an upwind point in the system (fixed points
        // never count down to zero)
        const uint32_t old = atomicSub(&P.cnt[gq], 1u);
        if (old == 1u) s_items[atomicAdd(s_n, 1u)] = ((uint64_t)j << 40) | (uint64_t)q[ax];
    }
}

template <typename FT> __global__ void __launch_bounds__(ADJ_BLOCK) k_adj_sweep(AdjParams P)
{
    __shared__ uint32_t s_ok, s_n;
    __shared__ unsigned long long s_base;
    __shared__ uint64_t s_items[3 * ADJ_BLOCK];
    AdjCtrl *c = P.ctrl;
    const uint32_t nwg = gridDim.x;
    uint32_t gen = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) c->nwg = nwg;
    const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
    uint32_t level = 0;
    for (;;) {
        const unsigned long long n = ld_acq64(&c->len[level % 3]);
        if (n == 0) break;
        // the counter of the level after next is free: its last reader was
        // the previous level; the barrier below publishes the reset
        if (blockIdx.x == 0 && threadIdx.x == 0) c->len[(level + 2) % 3] = 0;
        const uint64_t *cur = (level & 1) ? P.list1 : P.list0;
        uint64_t *nxt = (level & 1) ? P.list0 : P.list1;
        unsigned long long *nlen = &c->len[(level + 1) % 3];
        // the pass count is uniform within a workgroup (barriers inside)
        for (unsigned long long k0 = (unsigned long long)blockIdx.x * blockDim.x; k0 < n; k0 += nth) {
            if (threadIdx.x == 0) s_n = 0;
            __syncthreads();
            const unsigned long long k = k0 + threadIdx.x;
            adj_point<FT>(P, k < n ? cur[k] : 0, k < n, s_items, &s_n);
            __syncthreads();
            const uint32_t m = s_n;
            if (threadIdx.x == 0 && m) s_base = atomicAdd(nlen, (unsigned long long)m);
            __syncthreads();
            for (uint32_t t = threadIdx.x; t < m; t += blockDim.x) nxt[s_base + t] = s_items[t];
            __syncthreads();
        }
        level++;
        if (!grid_sync(&c->bar, &c->abort, &c->error, ADJ_ERR_BARRIER, gen, nwg, &s_ok)) break;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) c->levels = level;
}

// dL/dF of one output array: the sum of the gradient terms of the problems
// that share it (a point outside a problem's system contributes 0).
__global__ void k_adj_gather(AdjParams P, AdjGather G)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < G.n; p += (int64_t)gridDim.x * blockDim.x) {
        double s = G.accumulate ? G.out[p] : 0.0;
        for (uint32_t k = 0; k < G.m; k++) {
            const int64_t g = G.base[k] + p;
            if (P.code[g]) s += P.acc[g];
        }
        G.out[p] = s;
    }
}

__global__ void k_adj_init(AdjParams P, uint32_t n_inst)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        AdjCtrl *c = P.ctrl;
        c->bar = 0;
        c->abort = 0;
        c->error = 0;
        c->n_inst = n_inst;
        c->nwg = 0;
        c->levels = 0;
        c->len[0] = c->len[1] = c->len[2] = 0;
        c->n_points = 0;
        c->magic = ADJ_MAGIC;
    }
}

__global__ void k_adj_set_inst(AdjInst *dst, AdjPack pk)
{
    const uint32_t k = threadIdx.x;
    if (k < pk.n) dst[pk.first + k] = pk.v[k];
}

// ---------------------------------------------------------------------------
// Host-side launcher.

static int adj_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 1;
    }
    return cus;
}

template <typename FT> static hipError_t launch_adjoint_t(const AdjParams &P, const AdjInst *insts, int64_t n,
                                                       hipStream_t s)
{
    const int cus = adj_cus();
    hipError_t e;
    hipLaunchKernelGGL(k_adj_init, dim3(1), dim3(64), 0, s, P, (uint32_t)n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int64_t first = 0; first < n; first += ADJ_PACK) {
        AdjPack pk;
        memset(&pk, 0, sizeof pk);
        pk.first = (uint32_t)first;
        pk.n = (uint32_t)std::min<int64_t>(ADJ_PACK, n - first);
        for (uint32_t k = 0; k < pk.n; k++) pk.v[k] = insts[first + k];
        hipLaunchKernelGGL(k_adj_set_inst, dim3(1), dim3(64), 0, s, (AdjInst *)P.inst, pk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    auto blocks_for = [&](const AdjInst &I) {
        const int64_t N = I.n0 * I.n1 * I.n2;
        return (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + 255) / 256, (int64_t)cus * 16));
    };
    for (int64_t j = 0; j < n; j++) {
        hipLaunchKernelGGL(k_adj_zero, dim3(blocks_for(insts[j])), dim3(256), 0, s, P, insts[j]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int64_t j = 0; j < n; j++) {
        hipLaunchKernelGGL(k_adj_setup<FT>, dim3(blocks_for(insts[j])), dim3(256), 0, s, P, insts[j]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int64_t j = 0; j < n; j++) {
        hipLaunchKernelGGL(k_adj_front0, dim3(blocks_for(insts[j])), dim3(256), 0, s, P, insts[j], (uint32_t)j);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    static int occ = -1;
    auto kern = k_adj_sweep<FT>;
    if (occ < 0) {
        int nb = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, ADJ_BLOCK, 0)) != hipSuccess) return e;
        occ = nb;
    }
    if (occ <= 0) return hipErrorInvalidConfiguration;
    const unsigned grid = (unsigned)(std::min(occ, FMM_ADJ_WG_PER_CU) * cus);
    AdjParams Pc = P;
    void *args[] = {&Pc};
    if ((e = launch_coresident((const void *)kern, dim3(grid), dim3(ADJ_BLOCK), args, s)) != hipSuccess) return e;
    // gather each output array over the problems that share it
    std::vector<bool> done((size_t)n, false);
    for (int64_t j = 0; j < n; j++) {
        if (done[(size_t)j]) continue;
        AdjGather G;
        memset(&G, 0, sizeof G);
        G.out = insts[j].dL_dF;
        G.n = insts[j].n0 * insts[j].n1 * insts[j].n2;
        for (int64_t k = j; k < n; k++) {
            if (done[(size_t)k] || insts[k].dL_dF != G.out) continue;
            done[(size_t)k] = true;
            G.base[G.m++] = insts[k].base;
            if (G.m == ADJ_GATHER) {
                hipLaunchKernelGGL(k_adj_gather, dim3(blocks_for(insts[j])), dim3(256), 0, s, P, G);
                if ((e = hipGetLastError()) != hipSuccess) return e;
                G.accumulate = 1;
                G.m = 0;
            }
        }
        if (G.m) {
            hipLaunchKernelGGL(k_adj_gather, dim3(blocks_for(insts[j])), dim3(256), 0, s, P, G);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_adjoint(const AdjParams &P, const AdjInst *insts, int64_t n, bool f64, hipStream_t s)
{
    return f64 ? launch_adjoint_t<double>(P, insts, n, s) : launch_adjoint_t<float>(P, insts, n, s);
}

}  // namespace fmm
