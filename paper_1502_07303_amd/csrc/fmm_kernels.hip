// HIP kernels of the restarted narrow-band fast marching method for gfx950.
//
// Mapping of the paper's parallel algorithm (Sec. 4) onto one GPU:
//   subdomain Xi_p with its ghost layer (Sec. 4.1)  -> a cubic grid tile of edge E
//                                                     held in LDS with a one-point
//                                                     halo, marched by one wavefront
//   Initialize_Interface/Heap_Parallel (Alg. 8, 9) -> k_prepare + the first phase
//                                                     of k_driver
//   restart loop (Alg. 16)                          -> k_driver: persistent kernel,
//                                                     device-wide barriers, no host
//                                                     round trip
//   AllReduce of the heap-top minima and of the
//   count of new overlap points (Alg. 16)           -> per-workgroup reduction and
//                                                     one atomic per workgroup
//   March_Narrow_Band_Parallel (Alg. 12, 10, 11)    -> tile_march(): label-correcting
//                                                     relaxation of the tile's band
//                                                     up to the restart bound
//   Collect/Exchange/Integrate (Alg. 13-15)         -> owner writes its interior to
//                                                     HBM and flags the neighbour
//                                                     tiles whose halo changed by a
//                                                     value that can improve them;
//                                                     they re-read the halo in the
//                                                     second march of the restart
// Every floating-point expression of the local solver is written out in the
// order used by the specification of fmm_eval_godunov(); the file is compiled
// with -ffp-contract=off so no multiply-add is fused.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "fmm_device.h"
#include "fmm_internal.h"
#include "fmm_tile.h"

namespace fmm {

__global__ void k_eval_godunov(const double *__restrict__ a, const double *__restrict__ r,
                               double *__restrict__ out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = godunov(a[3 * i], a[3 * i + 1], a[3 * i + 2], r[i]);
}

// ---------------------------------------------------------------------------
// Tile geometry, thread groups and per-tile LDS.

// A tile is marched by a group of G threads: one wavefront (G = 64) for the
// 4^3 and 8^3 tiles, several per workgroup; the whole workgroup of G / 64
// wavefronts for a 16^3 tile, so that a front crossing the tile is handed
// from cell to cell in LDS instead of across tile faces through HBM.
template <int G> struct Grp {
    static constexpr int NWV = G / 64;  // wavefronts in the group
    __device__ static __forceinline__ int rank() { return G == 64 ? (int)(threadIdx.x & 63) : (int)threadIdx.x; }
    // The rank made opaque to the optimiser (its range stays known): the
    // offsets derived from it are then formed where they are used instead of
    // being hoisted out of the phase loop and kept, and spilled, for the
    // whole kernel.
    __device__ static __forceinline__ int rank_here()
    {
        int r = rank();
        asm volatile("" : "+v"(r));
        return r & (G - 1);
    }
    __device__ static __forceinline__ int wave()
    {
        return G == 64 ? 0 : (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    }
    __device__ static __forceinline__ void sync()
    {
        if constexpr (G == 64)
            wave_sync();
        else
            __syncthreads();
    }
};

// Wavefronts per workgroup of the 8^3-tile driver (one workgroup per CU; LDS
// bounds it at 12 for FP32 speeds and 10 for FP64).
#ifndef FMM_E8_WAVES_F32
#define FMM_E8_WAVES_F32 12
#endif
#ifndef FMM_E8_WAVES_F64
#define FMM_E8_WAVES_F64 10
#endif

constexpr int STAGE = 64;  // staged list appends per group before a flush
constexpr int MAX_ROUNDS = 1 << 16;

// Cell flags.  FL_SRC caches "is a source at the current level" (a seed, or a
// finite value within the level of its side): set when the tile is loaded,
// when a value drops to the level and when the level rises.  Values only
// decrease and the level only rises during a march, so it is never cleared.
enum : uint8_t { FL_SEED = 1, FL_UPD = 2, FL_CHG = 4, FL_SRC = 8 };
enum { MODE_INIT = 0, MODE_M1 = 1, MODE_M2 = 2 };

// LDS of one tile march.  Candidate flags are bytes for a one-wavefront group
// (compacted eight at a time) and bits for a workgroup (a 16^3 tile's bytes
// would not leave room for two tiles per CU).
template <int E, typename FT, int G> struct TileLds {
    static constexpr bool BITS = G > 64;
    static constexpr int NWV = G / 64;
    double T[Geo<E>::DV];                                // domain values (interior + face halos)
    FT F[Geo<E>::V];                                     // interior speeds (FP32), or h / F (FP64)
    uint16_t list[Geo<E>::V];                            // candidate list (interior indices)
    alignas(8) uint8_t cf[BITS ? 8 : Geo<E>::CFB];       // byte flags (+ per-lane spares)
    uint32_t cfw[BITS ? Geo<E>::V / 32 : 1];             // bit flags
    uint8_t fl[Geo<E>::DV];                              // FL_* per domain cell
    uint32_t stL[STAGE];                                 // staged live-list appends
    uint32_t stD[STAGE];                                 // staged dirty-list appends
    unsigned long long bm[12];                           // per face and side: smallest changed band value
    // group scratch (G > 64): per-wavefront candidate counts and partial
    // reductions, and broadcast words
    uint32_t gcnt[NWV], gu[NWV];
    double gd0[NWV], gd1[NWV];
    uint32_t bc[8];
};

constexpr uint32_t NO_INST = 0xFFFFFFFFu;

template <int NW> struct WgShared {
    uint32_t cntL[NW], cntD[NW], pend[NW], inst[NW];
    double gmin0[NW], gmin1[NW];
    uint32_t baseL, baseD;
    uint32_t ok;
};

#ifdef FMM_PROFILE
#define PROF_CLOCK(x) const unsigned long long x = clock64()
#define PROF_ADD(i, v) (ws.prof[i] += (v))
#else
#define PROF_CLOCK(x)
#define PROF_ADD(i, v)
#endif

struct WaveState {
#ifdef FMM_PROFILE
    unsigned long long prof[16];
#endif
    uint32_t nL, nD;      // staged entries (group-uniform; kept by the group's first wavefront)
    uint32_t acc;         // problem the three accumulators below belong to (NO_INST: none)
    uint32_t pending;     // tiles newly dirtied for the next restart (first wavefront of the group)
    double gmin0, gmin1;  // running min of band minima
    unsigned long long n_march, n_round;  // group-uniform counters (first wavefront of the group)
    // per-lane counters for the statistics only, 32-bit (cheaper to count in
    // the relaxation loop).  They are widened when summed at the end; a lane
    // would wrap only after 4.3e9 local solves, some 2e4 times what one lane
    // makes on a 1024^3 grid.
    uint32_t n_solve, n_reopen;
};

// ---------------------------------------------------------------------------
// Group reductions and broadcasts.  For G > 64 every value that steers
// control flow must be the same in all wavefronts of the group, so values
// read from memory that other workgroups may be changing are read by one
// thread and broadcast through LDS.

template <int E, typename FT, int G>
__device__ __forceinline__ bool grp_any(TileLds<E, FT, G> &L, bool b)
{
    const bool w = __ballot(b) != 0ull;
    if constexpr (G == 64) {
        return w;
    } else {
        if ((threadIdx.x & 63) == 0) L.gu[Grp<G>::wave()] = w ? 1u : 0u;
        __syncthreads();
        uint32_t r = 0;
#pragma unroll
        for (int k = 0; k < G / 64; k++) r |= L.gu[k];
        __syncthreads();
        return r != 0;
    }
}

template <int E, typename FT, int G>
__device__ __forceinline__ uint32_t grp_or(TileLds<E, FT, G> &L, uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    if constexpr (G == 64) {
        return v;
    } else {
        if ((threadIdx.x & 63) == 0) L.gu[Grp<G>::wave()] = v;
        __syncthreads();
        uint32_t r = 0;
#pragma unroll
        for (int k = 0; k < G / 64; k++) r |= L.gu[k];
        __syncthreads();
        return r;
    }
}

template <int E, typename FT, int G>
__device__ __forceinline__ void grp_min2(TileLds<E, FT, G> &L, double &a, double &b)
{
    a = wave_min(a);
    b = wave_min(b);
    if constexpr (G > 64) {
        if ((threadIdx.x & 63) == 0) {
            L.gd0[Grp<G>::wave()] = a;
            L.gd1[Grp<G>::wave()] = b;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < G / 64; k++) {
            a = fmin(a, L.gd0[k]);
            b = fmin(b, L.gd1[k]);
        }
        __syncthreads();
    }
}

// Broadcast a value held by rank 0 of the group to all of it.
template <int E, typename FT, int G>
__device__ __forceinline__ uint32_t grp_bcast(TileLds<E, FT, G> &L, uint32_t v)
{
    if constexpr (G == 64) {
        return bcast0(v);
    } else {
        if (threadIdx.x == 0) L.bc[0] = v;
        __syncthreads();
        const uint32_t r = L.bc[0];
        __syncthreads();
        return r;
    }
}

// ---------------------------------------------------------------------------
// Device-wide barrier for the persistent driver.  All workgroups of the
// cooperative launch are co-resident.  A bounded wait turns any failure into
// an abort that every workgroup observes, so the kernel always terminates.

__device__ bool grid_barrier(Ctrl *c, uint32_t &gen, uint32_t nwg, uint32_t *s_ok)
{
    return grid_sync(&c->bar, &c->abort, &c->error_run, ERR_BARRIER, gen, nwg, s_ok);
}

// ---------------------------------------------------------------------------
// Wave-level list staging (called by one wavefront: the group's first).

__device__ __forceinline__ void stage_push(uint32_t *st, uint32_t &n, uint32_t v, uint32_t *counter, uint32_t *list)
{
    const int lane = threadIdx.x & 63;
    if (lane == 0) st[n] = v;
    n++;
    if (n == STAGE) {
        wave_sync();
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(counter, (uint32_t)STAGE);
        base = bcast0(base);
        list[base + lane] = st[lane];
        n = 0;
        wave_sync();
    }
}

// Set candidate flag q if `on`.  Byte flags take one store from every lane:
// a lane that does not mark writes its own spare dword (distinct banks), so
// no lane mask has to be set up around the store; bit flags an LDS atomic OR.
template <int E, typename FT, int G>
__device__ __forceinline__ void mark_cand(TileLds<E, FT, G> &L, bool on, int q)
{
    if constexpr (TileLds<E, FT, G>::BITS) {
        if (on) atomicOr(&L.cfw[q >> 5], 1u << (q & 31));
    } else {
        L.cf[on ? q : Geo<E>::spare((int)__lane_id())] = 1;
    }
}

// Compact the candidate flags into the list (ascending interior index within
// each wavefront's part), clearing them; returns the count (group-uniform).
// One wavefront: byte flags, one list.  A workgroup: bit flags; wavefront w
// owns interior cells [w 64 C, (w + 1) 64 C) (C = V / G cells per thread) and
// writes its candidates to the same range of the list, its count to gcnt[w].
template <int E, typename FT, int G> __device__ __forceinline__ int compact(TileLds<E, FT, G> &L)
{
    constexpr int K = Geo<E>::K;
    const int lane = Grp<G>::rank_here() & 63;
    uint16_t *out = L.list;
    uint32_t cnt = 0;
    if constexpr (G > 64) {
        constexpr int C = Geo<E>::V / G;
        static_assert(C >= 1 && C <= 32 && 32 % C == 0, "cells per thread must divide a word");
        const int r = Grp<G>::rank_here(), wv = Grp<G>::wave();
        const int word = (r * C) >> 5, sh = (r * C) & 31;
        const uint32_t wbits = L.cfw[word];
        uint32_t bits = C == 32 ? wbits : (wbits >> sh) & ((1u << (C & 31)) - 1u);
        cnt = (uint32_t)__popc(bits);
        uint32_t pre = 0, total = 0;
        const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
        for (int b = 0; (1 << b) <= C; b++) {
            const unsigned long long m = __ballot((cnt >> b) & 1u);
            pre += (uint32_t)__popcll(m & lt) << b;
            total += (uint32_t)__popcll(m) << b;
        }
        uint16_t *seg = out + wv * 64 * C;
        while (bits) {
            const int b = __builtin_ctz(bits);
            seg[pre++] = (uint16_t)(r * C + b);
            bits &= bits - 1u;
        }
        // every lane sharing the word read it above (same wavefront)
        if (sh == 0 && wbits) L.cfw[word] = 0u;
        if (lane == 0) L.gcnt[wv] = total;
        __syncthreads();
        int n = 0;
#pragma unroll
        for (int k = 0; k < G / 64; k++) n += (int)L.gcnt[k];
        return n;
    } else if constexpr (K % 8 == 0) {
        // flags are 0/1 bytes: a 64-bit word holds 8 of them
        unsigned long long *w = (unsigned long long *)&L.cf[lane * K];
        unsigned long long x[K / 8];
#pragma unroll
        for (int j = 0; j < K / 8; j++) {
            x[j] = w[j];
            cnt += (uint32_t)__popcll(x[j]);
        }
        uint32_t pre = 0, total = 0;
        const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
        for (int b = 0; (1 << b) <= K; b++) {
            const unsigned long long m = __ballot((cnt >> b) & 1u);
            pre += (uint32_t)__popcll(m & lt) << b;
            total += (uint32_t)__popcll(m) << b;
        }
#pragma unroll
        for (int j = 0; j < K / 8; j++) {
            // the eight 0/1 bytes as an 8-bit mask: byte k holds bit 8k, and
            // shifting by 7k moves it to bit k (the other bits land at 9 and up)
            const uint32_t lo = (uint32_t)x[j], hi = (uint32_t)(x[j] >> 32);
            uint32_t y = ((lo | (lo >> 7) | (lo >> 14) | (lo >> 21)) & 0xFu) |
                         (((hi | (hi >> 7) | (hi >> 14) | (hi >> 21)) & 0xFu) << 4);
            while (y) {
                const int bit = __builtin_ctz(y);
                out[pre++] = (uint16_t)(lane * K + j * 8 + bit);
                y &= y - 1u;
            }
            if (x[j]) w[j] = 0ull;
        }
        wave_sync();
        return (int)total;
    } else {
        if (lane * K < Geo<E>::V) {
#pragma unroll
            for (int j = 0; j < K; j++) cnt += L.cf[lane * K + j] != 0;
        }
        uint32_t pre = 0, total = 0;
        const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
        for (int b = 0; (1 << b) <= K; b++) {
            const unsigned long long m = __ballot((cnt >> b) & 1u);
            pre += (uint32_t)__popcll(m & lt) << b;
            total += (uint32_t)__popcll(m) << b;
        }
        if (cnt) {
#pragma unroll
            for (int j = 0; j < K; j++) {
                const int p = lane * K + j;
                if (L.cf[p]) {
                    out[pre++] = (uint16_t)p;
                    L.cf[p] = 0;
                }
            }
        }
        wave_sync();
        return (int)total;
    }
}

// The k-th candidate of the last compaction.
template <int E, typename FT, int G> __device__ __forceinline__ int cand_at(const TileLds<E, FT, G> &L, int k)
{
    if constexpr (G == 64) {
        return L.list[k];
    } else {
        constexpr int C = Geo<E>::V / G;
        int w = 0;
#pragma unroll
        for (int q = 0; q < G / 64 - 1; q++) {
            if (k < (int)L.gcnt[w]) break;
            k -= (int)L.gcnt[w];
            w++;
        }
        return L.list[w * 64 * C + k];
    }
}

// Mark the updatable interior neighbours of interior point p (domain cell d)
// that lie downwind of the value magnitude a: only they can use p as an
// upwind point (the |T_lmn| > |T_ijk| guard of Alg. 10).
template <int E, typename FT, int G>
__device__ __forceinline__ void mark_nbrs(TileLds<E, FT, G> &L, int p, int d, double a)
{
    using Gm = Geo<E>;
    // all twelve reads first (one LDS round trip); a halo neighbour never
    // carries FL_UPD, so its out-of-interior index is never marked
    const int od[6] = {-Gm::OX, Gm::OX, -Gm::OY, Gm::OY, -Gm::OZ, Gm::OZ};
    const int op[6] = {-E * E, E * E, -E, E, -1, 1};
    uint8_t f[6];
    double v[6];
#pragma unroll
    for (int k = 0; k < 6; k++) {
        f[k] = L.fl[d + od[k]];
        v[k] = L.T[d + od[k]];
    }
#pragma unroll
    for (int k = 0; k < 6; k++) mark_cand(L, (f[k] & FL_UPD) && fabs(v[k]) > a, p + op[k]);
}

// A domain cell is a source of the relaxation when it is a seed, or when its
// value is finite and within the band bound of its side (the KNOWN-class
// points of Alg. 11 for this restart).
__device__ __forceinline__ bool is_source(double v, uint8_t fl, const double bnd[2])
{
    double a = fabs(v);
    if (!(a < FMM_INF)) return false;
    if (fl & FL_SEED) return true;
    return a <= (v < 0.0 ? bnd[0] : bnd[1]);
}

// r = h / F of interior point p (+inf for seeds and impassable cells).
template <int E, typename FT, int G>
__device__ __forceinline__ double cell_r(const TileLds<E, FT, G> &L, int p, double h)
{
    if constexpr (sizeof(FT) == 8) {
        return L.F[p];
    } else {
        // fixed cells (seeds, impassable cells) hold speed 0
        const float f = L.F[p];
        return f > 0.0f ? solver_div(h, (double)f) : FMM_INF;
    }
}

// Evaluate Solve_Quadratic_Parallel at interior point p: returns true and the
// new signed value if it improves on the current one.  Also hands back what
// the update step needs without another LDS round trip: the old value and the
// magnitudes of the six neighbours (order -x,+x,-y,+y,-z,+z).
// TWO = false is the path for a tile whose values are all on the positive
// side (no negative value in the tile or its halo, so none can appear): one
// minimum per axis and one solve.  That path
// takes the per-axis minimum over all neighbours, sources or not, upwind or
// not.  A neighbour value a >= vp only adds roots above a (strict causality),
// which cannot beat vp.  A band value below vp is an upper bound of its final
// value, and the local solver is monotone in its inputs, so the result is
// still an upper bound of the final value at p; when that neighbour later
// becomes a source with a smaller value it marks p again, so the fixed point
// (the discrete system of Eq. 2-3) is the same.
template <int E, typename FT, int G, bool AN, bool TWO>
__device__ __forceinline__ bool eval_point(const TileLds<E, FT, G> &L, const Spacing &sp, int p, double h,
                                           const double bnd[2], double &out,
                                           double &vp, double na[6])
{
    using Gm = Geo<E>;
    const int d = Gm::domp(p);
    vp = L.T[d];
    if constexpr (!TWO) {
        // the neighbours are read first and the speed right after them, so
        // that all reads share one LDS round trip
        double m[3];
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            const int off = ax == 0 ? Gm::OX : ax == 1 ? Gm::OY : Gm::OZ;
            na[2 * ax] = L.T[d - off];
            na[2 * ax + 1] = L.T[d + off];
        }
        const double r = cell_r(L, p, h);
#pragma unroll
        for (int ax = 0; ax < 3; ax++) m[ax] = fmin(na[2 * ax], na[2 * ax + 1]);
        // no finite neighbour: the solver returns +inf, which never beats vp
        int kk;
        const double u = AN ? godunov_w_sel(m[0], m[1], m[2], sp.s[0], sp.s[1], sp.s[2], r, &kk)
                            : godunov_sel(m[0], m[1], m[2], r, &kk);
        out = u;
        return u < vp;
    }
    const double ap = fabs(vp);
    double am[3], ap3[3];  // per-axis minima for side - and side +
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        const int off = ax == 0 ? Gm::OX : ax == 1 ? Gm::OY : Gm::OZ;
        double mneg = FMM_INF, mpos = FMM_INF;
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const int dn = s ? d + off : d - off;
            const double v = L.T[dn];
            const uint8_t fl = L.fl[dn];
            const double a = fabs(v);
            na[2 * ax + s] = a;
            if (a < ap && (fl & FL_SRC)) {
                if (v < 0.0)
                    mneg = fmin(mneg, a);
                else
                    mpos = fmin(mpos, a);
            }
        }
        am[ax] = mneg;
        ap3[ax] = mpos;
    }
    const double r = cell_r(L, p, h);
    double best = ap;
    bool neg = vp < 0.0;
    bool improved = false;
    // one local solve per side that has an upwind point (kept as a loop so
    // the solver is emitted once)
#pragma unroll 1
    for (int side = 0; side < 2; side++) {
        const double x = side == 0 ? am[0] : ap3[0];
        const double y = side == 0 ? am[1] : ap3[1];
        const double z = side == 0 ? am[2] : ap3[2];
        if (!(fmin(x, fmin(y, z)) < FMM_INF)) continue;
        int kk;
        const double u = AN ? godunov_w_sel(x, y, z, sp.s[0], sp.s[1], sp.s[2], r, &kk) : godunov_sel(x, y, z, r, &kk);
        const bool take = u < best || (side == 0 && u == best && !neg && best < FMM_INF);
        if (take) {
            best = u;
            neg = side == 0;
            improved = true;
        }
    }
    out = neg ? -best : best;
    return improved;
}

// Relaxation at level th until no candidate improves; returns the number of
// rounds.  Candidates are taken G at a time.  In a one-wavefront group all
// evaluations of a chunk read before any of its writes and later chunks see
// earlier ones.  In a workgroup the threads write as they finish: a read
// racing with a write returns the old or the new value, both upper bounds of
// the neighbour's final value, and a write that can lower a neighbour marks
// it for the next round, so the fixed point is the same either way.
// Neighbours are marked from the magnitudes the evaluation read; values only
// decrease, so a neighbour lowered meanwhile is at worst marked needlessly,
// never missed.
template <int E, typename FT, int G, bool AN, bool TWO>
__device__ __forceinline__ int relax(const Params &P, TileLds<E, FT, G> &L, double h, const double th[2],
                                     WaveState &ws)
{
    using Gm = Geo<E>;
    const int r = Grp<G>::rank_here();
    int n = compact(L);
    int rounds = 0;
    while (n > 0) {
        if (++rounds > MAX_ROUNDS) {
            if (r == 0) atomicOr(&P.ctrl->error_run, ERR_ROUNDS);
            break;
        }
        for (int base = 0; base < n; base += G) {
            const int k = base + r;
            double nv = 0.0, vp = 0.0, na[6];
            bool ch = false;
            int p = 0;
            if (k < n) {
                p = cand_at(L, k);
                ch = eval_point<E, FT, G, AN, TWO>(L, P.sp, p, h, th, nv, vp, na);
                ws.n_solve++;
            }
            if constexpr (G == 64) wave_sync();
            if (ch) {
                const int d = Gm::domp(p);
                const uint8_t fo = L.fl[d];
                // reopened: the old value was already a source.  The level
                // never drops below the bound of the tile's previous march, so
                // this covers every value that march released.
                ws.n_reopen += (fo >> 3) & 1u;  // FL_SRC
                L.T[d] = nv;
                // one-sided tiles: nv is positive and finite (it beat vp)
                const bool src = TWO ? is_source(nv, 0, th) : nv <= th[1];
                L.fl[d] = fo | (src ? (uint8_t)(FL_CHG | FL_SRC) : (uint8_t)FL_CHG);
                const double a = TWO ? fabs(nv) : nv;
                if (src) {
                    // mark the downwind interior neighbours.  Seeds and
                    // impassable cells may be marked too: their LDS speed is
                    // 0, so their solve gives +inf and changes nothing.
                    const int i0 = p >> (2 * Gm::LOG), i1 = (p >> Gm::LOG) & (E - 1), i2 = p & (E - 1);
                    mark_cand(L, i0 > 0 && na[0] > a, p - E * E);
                    mark_cand(L, i0 < E - 1 && na[1] > a, p + E * E);
                    mark_cand(L, i1 > 0 && na[2] > a, p - E);
                    mark_cand(L, i1 < E - 1 && na[3] > a, p + E);
                    mark_cand(L, i2 > 0 && na[4] > a, p - 1);
                    mark_cand(L, i2 < E - 1 && na[5] > a, p + 1);
                }
            }
            if constexpr (G == 64) wave_sync();
        }
        if constexpr (G > 64) __syncthreads();
        n = compact(L);
    }
    return rounds;
}

// Smallest pending band value per side above level th: interior band values,
// and halo values next to an interior cell that is not yet a source (they
// become sources of this tile later).  Group-uniform result.  The reads of
// up to eight cells per thread are issued before any of them is used, so a
// pass waits for one LDS round trip instead of one per cell.
template <int E, typename FT, int G>
__device__ __forceinline__ void band_min(TileLds<E, FT, G> &L, const double th[2], double &m0, double &m1)
{
    using Gm = Geo<E>;
    constexpr int V = Gm::V, FACE = Gm::FACE;
    constexpr int NI = V / G, NF = (6 * FACE + G - 1) / G;
    constexpr int BI = NI < 8 ? NI : 8, BF = NF < 8 ? NF : 8;
    static_assert(V % G == 0, "interior cells per thread");
    const int r = Grp<G>::rank_here();
    double a0 = FMM_INF, a1 = FMM_INF;
    for (int j0 = 0; j0 < NI; j0 += BI) {
        double v[BI];
        uint8_t f[BI];
#pragma unroll
        for (int j = 0; j < BI; j++) {
            const int d = Gm::domp(r + G * (j0 + j));
            f[j] = L.fl[d];
            v[j] = L.T[d];
        }
#pragma unroll
        for (int j = 0; j < BI; j++) {
            if (!(f[j] & FL_UPD)) continue;
            const double a = fabs(v[j]);
            if (a < FMM_INF) {
                if (v[j] < 0.0) {
                    if (a > th[0]) a0 = fmin(a0, a);
                } else if (a > th[1]) {
                    a1 = fmin(a1, a);
                }
            }
        }
    }
    for (int j0 = 0; j0 < NF; j0 += BF) {
        double v[BF];
        uint8_t fh[BF], fi[BF];
#pragma unroll
        for (int j = 0; j < BF; j++) {
            const int q = r + G * (j0 + j);
            v[j] = FMM_INF;  // a thread past the last face cell takes nothing
            fh[j] = fi[j] = 0;
            if (q < 6 * FACE) {
                const int f = q / FACE, uv = q - f * FACE, u = uv / E, w = uv - u * E;
                int c0, c1, c2;
                face_cell<E>(f, u, w, c0, c1, c2);
                const int d = Gm::dom(c0, c1, c2);
                face_inner<E>(f, c0, c1, c2);
                v[j] = L.T[d];
                fh[j] = L.fl[d];
                fi[j] = L.fl[Gm::dom(c0, c1, c2)];
            }
        }
#pragma unroll
        for (int j = 0; j < BF; j++) {
            const double a = fabs(v[j]);
            if (!(a < FMM_INF) || (fh[j] & FL_SEED)) continue;
            if (a <= (v[j] < 0.0 ? th[0] : th[1])) continue;
            if (!(fi[j] & FL_UPD) || (fi[j] & FL_SRC)) continue;
            if (v[j] < 0.0)
                a0 = fmin(a0, a);
            else
                a1 = fmin(a1, a);
        }
    }
    grp_min2(L, a0, a1);
    m0 = a0;
    m1 = a1;
}

// Mark the candidates next to cells whose value lies in (lo, hi] of their
// side: they become sources when the level rises from lo to hi.  The first
// reads of a pass are issued together, as in band_min.
template <int E, typename FT, int G>
__device__ __forceinline__ void mark_new_sources(TileLds<E, FT, G> &L, const double lo[2], const double hi[2])
{
    using Gm = Geo<E>;
    constexpr int V = Gm::V, FACE = Gm::FACE;
    constexpr int NI = V / G, NF = (6 * FACE + G - 1) / G;
    constexpr int BI = NI < 8 ? NI : 8, BF = NF < 8 ? NF : 8;
    const int r = Grp<G>::rank_here();
    for (int j0 = 0; j0 < NI; j0 += BI) {
        double v[BI];
        uint8_t f[BI];
#pragma unroll
        for (int j = 0; j < BI; j++) {
            const int d = Gm::domp(r + G * (j0 + j));
            f[j] = L.fl[d];
            v[j] = L.T[d];
        }
#pragma unroll
        for (int j = 0; j < BI; j++) {
            const int p = r + G * (j0 + j);
            const int d = Gm::domp(p);
            if (!(f[j] & FL_UPD)) continue;
            const double a = fabs(v[j]);
            const int s = v[j] < 0.0 ? 0 : 1;
            if (a < FMM_INF && a > lo[s] && a <= hi[s]) {
                L.fl[d] = f[j] | FL_SRC;
                mark_nbrs(L, p, d, a);
            }
        }
    }
    for (int j0 = 0; j0 < NF; j0 += BF) {
        double v[BF];
        uint8_t fh[BF];
#pragma unroll
        for (int j = 0; j < BF; j++) {
            const int q = r + G * (j0 + j);
            v[j] = FMM_INF;  // a thread past the last face cell takes nothing
            fh[j] = 0;
            if (q < 6 * FACE) {
                const int f = q / FACE, uv = q - f * FACE, u = uv / E, w = uv - u * E;
                int c0, c1, c2;
                face_cell<E>(f, u, w, c0, c1, c2);
                const int d = Gm::dom(c0, c1, c2);
                v[j] = L.T[d];
                fh[j] = L.fl[d];
            }
        }
#pragma unroll
        for (int j = 0; j < BF; j++) {
            const double a = fabs(v[j]);
            const int s = v[j] < 0.0 ? 0 : 1;
            if (!(a < FMM_INF && a > lo[s] && a <= hi[s]) || (fh[j] & FL_SEED)) continue;
            const int q = r + G * (j0 + j);
            const int f = q / FACE, uv = q - f * FACE, u = uv / E, w = uv - u * E;
            int c0, c1, c2;
            face_cell<E>(f, u, w, c0, c1, c2);
            L.fl[Gm::dom(c0, c1, c2)] = fh[j] | FL_SRC;
            face_inner<E>(f, c0, c1, c2);
            const int di = Gm::dom(c0, c1, c2);
            if ((L.fl[di] & FL_UPD) && fabs(L.T[di]) > a) mark_cand(L, true, (c0 * E + c1) * E + c2);
        }
    }
    Grp<G>::sync();
}

// What a tile march needs to know about the problem the tile belongs to.
struct TileGeo {
    uint32_t base;       // first tile of the problem
    int32_t t0, t1, t2;  // tiles per axis of the problem
    double h;
};

// ---------------------------------------------------------------------------
// One activation of a tile by its group: load tile + halo into LDS, relax
// its band up to the restart bound (Alg. 12 via Alg. 10/11), write back the
// changed points, pass changed boundary values on to the neighbours (Alg.
// 13-15), and record the tile's pending band minimum (the heap top of Alg. 16).
//
// Data of a neighbour tile is used only if that tile was first written in an
// earlier phase (visit stamp); otherwise its cells count as +inf, which is a
// valid upper bound, and the writer's flag makes this tile read them again.

template <int E, typename FT, int G, bool AN>
__device__ __forceinline__ void tile_march(const Params &P, TileLds<E, FT, G> &L, const TileGeo &G0, uint32_t t,
                                           int mode,
                                           uint32_t dbits,
                                           const double bnd[2], const double lastb[2], uint32_t epoch, uint32_t phase,
                                           bool second, WaveState &ws, uint32_t *listNext, uint32_t *cntNext,
                                           uint32_t *dlist, uint32_t *cntD, uint32_t *dprod)
{
    using Gm = Geo<E>;
    constexpr int V = Gm::V, FACE = Gm::FACE;
    // The lane offsets are formed per march (a reload of a spilled address
    // among the tile's loads would make them wait for one another).
    const int rk = Grp<G>::rank_here();
    const int lane = G == 64 ? rk : (int)(threadIdx.x & 63);
    const bool lead = Grp<G>::wave() == 0;  // the group's first wavefront
    const FT *__restrict__ Ft = (const FT *)P.Ft;
    double *__restrict__ Tt = P.Tt;

    // tile coordinates inside its problem; neighbours are t +- stride.  The
    // divisions run on the vector unit; the results are uniform and are
    // moved back to scalar registers, so that neighbour tiles and their base
    // addresses stay scalar.
    const uint32_t tl = t - G0.base;
    const int32_t tz = (int32_t)__builtin_amdgcn_readfirstlane(tl % (uint32_t)G0.t2);
    const int32_t ty = (int32_t)__builtin_amdgcn_readfirstlane((tl / (uint32_t)G0.t2) % (uint32_t)G0.t1);
    const int32_t tx = (int32_t)__builtin_amdgcn_readfirstlane(tl / ((uint32_t)G0.t2 * (uint32_t)G0.t1));
    const uint32_t tsx = (uint32_t)G0.t1 * (uint32_t)G0.t2, tsy = (uint32_t)G0.t2;
    const unsigned long long *mask = P.mask + (size_t)t * P.mask_words;
    const size_t tbase = (size_t)t * V;

    PROF_CLOCK(t_begin);
    // ---- load the tile and its six face halos in one round trip: every
    // address is inside the workspace, so all loads are issued first and the
    // visit/seed selections are applied afterwards.  Axis-0 faces are
    // contiguous E^2 runs of the neighbour tile, axis-1 faces E runs of E,
    // axis-2 faces come from the neighbour's face buffer; +inf outside the
    // grid or for a tile not yet written in an earlier phase.
    constexpr int NI = (V + G - 1) / G, NF = (6 * FACE + G - 1) / G;
    constexpr int CI = NI < 8 ? NI : 8;
    static_assert(NF <= 8, "face-halo cells per thread");
    // the level the march starts at (the sources it loads)
    const double th0[2] = {mode == MODE_INIT ? -1.0 : lastb[0], mode == MODE_INIT ? -1.0 : lastb[1]};
    bool anyneg = false;  // a negative value in the tile or its halo
    double vi[CI];
    FT fi[CI];
    auto load_interior = [&](int j0) {
#pragma unroll
        for (int j = 0; j < CI; j++) {
            const int p = rk + G * (j0 + j);
            if (p < V) {
                vi[j] = Tt[tbase + p];
                fi[j] = Ft[tbase + p];
            }
        }
    };
    auto store_interior = [&](int j0, bool hasSeed, bool fresh) {
#pragma unroll
        for (int j = 0; j < CI; j++) {
            const int p = rk + G * (j0 + j);
            if (p < V) {
                const int d = Gm::domp(p);
                const bool seed = hasSeed && ((mask[p >> 6] >> (p & 63)) & 1ull);
                const double tv = fresh ? FMM_INF : vi[j];
                uint8_t f8 = seed ? FL_SEED : ((double)fi[j] > 0.0 ? FL_UPD : 0);
                if (is_source(tv, f8, th0)) f8 |= FL_SRC;
                anyneg |= tv < 0.0;
                L.T[d] = tv;
                // seeds and impassable cells (F <= 0 or NaN) keep speed 0 in
                // LDS (r = h/0 = +inf), so the relaxation never changes them.
                // An FP64 slot holds r = h / F itself, computed once per cell
                // with the same expression as for FP32 speeds.
                const bool fixed = seed || !((double)fi[j] > 0.0);
                // An infinite FP32 speed (r = 0) is kept as the largest finite
                // one: the march's division wants a finite divisor, and
                // h / FLT_MAX is below the rounding of any value it is added to
                // unless that value is itself below about 1e-26.
                if constexpr (sizeof(FT) == 8)
                    L.F[p] = fixed ? FMM_INF : G0.h / (double)fi[j];
                else
                    L.F[p] = fixed ? (FT)0 : fminf(fi[j], 3.402823466e38f);
                L.fl[d] = f8;
                if constexpr (!TileLds<E, FT, G>::BITS) L.cf[p] = 0;
            }
        }
    };
    // the first interior chunk and every face-halo read are issued before
    // any of them is used.  The halo reads take no branch: a face on the
    // grid boundary reads the tile's own cells (a valid address) and its
    // stamp counts as "never written", so the cells come out +inf.  With one
    // face per group pass (E^2 = G) the face of pass j is j itself, so the
    // neighbour tile and its base addresses are known per pass.
    load_interior(0);
    double vh[NF];
    uint32_t vis_h[NF], tf_h[NF];
#pragma unroll
    for (int j = 0; j < NF; j++) {
        const int q = rk + G * j;
        vis_h[j] = 0;
        tf_h[j] = 0;
        if (q < 6 * FACE) {
            const int f = FACE == G ? j : q / FACE, uv = q - f * FACE, u = uv / E, w = uv - u * E;
            const int ax = f >> 1;
            const bool plus = f & 1;
            int c0, c1, c2;
            face_cell<E>(f, u, w, c0, c1, c2);
            const int32_t tca = ax == 0 ? tx : ax == 1 ? ty : tz;
            const int32_t tna = ax == 0 ? G0.t0 : ax == 1 ? G0.t1 : G0.t2;
            const bool inside = plus ? tca + 1 < tna : tca > 0;
            const uint32_t ts = ax == 0 ? tsx : ax == 1 ? tsy : 1u;
            const uint32_t tnb = inside ? (plus ? t + ts : t - ts) : t;
            const int n0c = ax == 0 ? (plus ? 0 : E - 1) : c0;
            const int n1c = ax == 1 ? (plus ? 0 : E - 1) : c1;
            const int n2c = ax == 2 ? (plus ? 0 : E - 1) : c2;
            const uint32_t vs = P.visit[tnb];
            const uint32_t tf = P.tflags[tnb];
            vh[j] = ax == 2 ? P.Zf[((size_t)tnb * 2 + (plus ? 0 : 1)) * FACE + n0c * E + n1c]
                            : Tt[(size_t)tnb * V + (n0c * E + n1c) * E + n2c];
            vis_h[j] = inside ? vs : 0u;
            tf_h[j] = inside ? tf : 0u;
        }
    }
    // the tile's own flags and stamp are requested after its cells (their
    // use must not hold back the cell reads)
    const bool hasSeed = (P.tflags[t] & TF_SEED) != 0;
    const bool fresh = P.visit[t] == 0;  // never written: every cell is +inf
    store_interior(0, hasSeed, fresh);
    for (int j0 = CI; j0 < NI; j0 += CI) {
        load_interior(j0);
        store_interior(j0, hasSeed, fresh);
    }
#pragma unroll
    for (int j = 0; j < NF; j++) {
        const int q = rk + G * j;
        if (q < 6 * FACE) {
            const int f = FACE == G ? j : q / FACE, uv = q - f * FACE, u = uv / E, w = uv - u * E;
            const int ax = f >> 1;
            const bool plus = f & 1;
            int c0, c1, c2;
            face_cell<E>(f, u, w, c0, c1, c2);
            double v = FMM_INF;
            uint8_t fl = 0;
            if (vis_h[j] != 0 && vis_h[j] <= phase) v = vh[j];
            if (tf_h[j] & TF_SEED) {
                // rare: the neighbour holds seeds; fetch its seed bit
                const uint32_t ts = ax == 0 ? tsx : ax == 1 ? tsy : 1u;
                const uint32_t tnb = plus ? t + ts : t - ts;
                const int n0c = ax == 0 ? (plus ? 0 : E - 1) : c0;
                const int n1c = ax == 1 ? (plus ? 0 : E - 1) : c1;
                const int n2c = ax == 2 ? (plus ? 0 : E - 1) : c2;
                const int pn = (n0c * E + n1c) * E + n2c;
                if ((P.mask[(size_t)tnb * P.mask_words + (pn >> 6)] >> (pn & 63)) & 1ull) fl = FL_SEED;
            }
            const int d = Gm::dom(c0, c1, c2);
            if (is_source(v, fl, th0)) fl |= FL_SRC;
            anyneg |= v < 0.0;
            L.T[d] = v;
            L.fl[d] = fl;
        }
    }
    if constexpr (TileLds<E, FT, G>::BITS)
        for (int q = rk; q < V / 32; q += G) L.cfw[q] = 0u;
    if (rk < 12) L.bm[rk] = bits_of(FMM_INF);
    const bool two = grp_any(L, anyneg);  // both sides present: the general relaxation
    Grp<G>::sync();

    // ---- ordered relaxation.  Sources at level th are the seeds and the
    // cells with |T| <= th of their side (the KNOWN-class points of Alg. 11).
    // The level starts at the bound of the tile's previous march and climbs to
    // this restart's bound in steps th = (smallest pending band value) + inner,
    // so values become sources in increasing order, as the heap of Alg. 12
    // would release them, up to the step width.
    PROF_CLOCK(t_loaded);
    PROF_ADD(2, t_loaded - t_begin);
    const bool init = mode == MODE_INIT;
    double th[2] = {init ? -1.0 : lastb[0], init ? -1.0 : lastb[1]};
    if (init) {
        // Alg. 9: the neighbours of every seed (in the tile or its halo).
        for (int p = rk; p < V; p += G) {
            const int d = Gm::domp(p);
            if (L.fl[d] & FL_SEED) mark_nbrs(L, p, d, fabs(L.T[d]));
        }
        for (int q = rk; q < 6 * FACE; q += G) {
            const int f = q / FACE, uv = q - f * FACE, u = uv / E, w = uv - u * E;
            int c0, c1, c2;
            face_cell<E>(f, u, w, c0, c1, c2);
            const int d = Gm::dom(c0, c1, c2);
            face_inner<E>(f, c0, c1, c2);
            const int di = Gm::dom(c0, c1, c2);
            if ((L.fl[d] & FL_SEED) && (L.fl[di] & FL_UPD) && fabs(L.T[di]) > fabs(L.T[d]))
                mark_cand(L, true, (c0 * E + c1) * E + c2);
        }
    } else if (dbits) {
        // interior cells next to a halo source on a face whose values changed
        // (Alg. 15's KNOWN_OLD values update their neighbours, Alg. 10).  Halo
        // values above the starting level are not sources yet: the level loop
        // marks their neighbours when it reaches them (mark_new_sources), and
        // a band value never marks anything, so a cell gets a tentative value
        // only from an accepted neighbour, as in the sequential march.
        // the reads of a thread's face cells are issued together
        constexpr int NQ = (6 * FACE + G - 1) / G, BQ = NQ < 8 ? NQ : 8;
        for (int j0 = 0; j0 < NQ; j0 += BQ) {
            uint8_t fh[BQ], fi[BQ];
            double vh[BQ], vi[BQ];
#pragma unroll
            for (int j = 0; j < BQ; j++) {
                const int q = rk + G * (j0 + j);
                fh[j] = fi[j] = 0;
                vh[j] = vi[j] = FMM_INF;
                if (q >= 6 * FACE) continue;
                const int f = q / FACE, uv = q - f * FACE, u = uv / E, w = uv - u * E;
                if (!((dbits >> f) & 1u)) continue;
                int c0, c1, c2;
                face_cell<E>(f, u, w, c0, c1, c2);
                const int dh = Gm::dom(c0, c1, c2);
                face_inner<E>(f, c0, c1, c2);
                const int di = Gm::dom(c0, c1, c2);
                fh[j] = L.fl[dh];
                vh[j] = L.T[dh];
                fi[j] = L.fl[di];
                vi[j] = L.T[di];
            }
#pragma unroll
            for (int j = 0; j < BQ; j++) {
                if (!(fh[j] & FL_SRC) || !(fi[j] & FL_UPD) || !(fabs(vi[j]) > fabs(vh[j]))) continue;
                const int q = rk + G * (j0 + j);
                const int f = q / FACE, uv = q - f * FACE, u = uv / E, w = uv - u * E;
                int c0, c1, c2;
                face_cell<E>(f, u, w, c0, c1, c2);
                face_inner<E>(f, c0, c1, c2);
                mark_cand(L, true, (c0 * E + c1) * E + c2);
            }
        }
    }
    Grp<G>::sync();
    int rounds = 0;
    double tm0, tm1;
    PROF_CLOCK(t_marked);
    PROF_ADD(3, t_marked - t_loaded);
    for (;;) {
        PROF_CLOCK(t_r0);
        rounds += two ? relax<E, FT, G, AN, true>(P, L, G0.h, th, ws) : relax<E, FT, G, AN, false>(P, L, G0.h, th, ws);
        PROF_CLOCK(t_r1);
        PROF_ADD(4, t_r1 - t_r0);
        PROF_ADD(8, 1);
        band_min(L, th, tm0, tm1);
        const bool more0 = tm0 < FMM_INF && tm0 <= bnd[0];
        const bool more1 = tm1 < FMM_INF && tm1 <= bnd[1];
        if (!(more0 || more1)) break;
        const double nt[2] = {more0 ? fmin(tm0 + P.inner, bnd[0]) : th[0],
                              more1 ? fmin(tm1 + P.inner, bnd[1]) : th[1]};
        mark_new_sources(L, th, nt);
        th[0] = nt[0];
        th[1] = nt[1];
        PROF_CLOCK(t_r2);
        PROF_ADD(5, t_r2 - t_r1);
    }
    PROF_CLOCK(t_levels);
    if (lead) {
        ws.n_round += (unsigned long long)rounds;
        ws.n_march++;
    }
    PROF_ADD(10 + mode, 1);

    // ---- write back (every cell on the first write of the tile, else the
    // changed ones) and classify the changed boundary cells per face: a new
    // source value is sent at once (the neighbour re-marches, KNOWN_OLD of Alg.
    // 15), a band value only joins the neighbour's pending minimum (BAND_OLD).
    uint32_t fsrc = 0, fany = 0;
#ifdef FMM_PROFILE
    bool any_chg = false;
#endif
    // the flags and values of a thread's cells are read together (one LDS
    // round trip); the changed-cell flags are kept as a bit mask
    constexpr int NW = V / G;
    static_assert(NW <= 32, "cells per thread");
    double vw[NW];
    uint32_t chgm = 0;
#pragma unroll
    for (int j = 0; j < NW; j++) {
        const int d = Gm::domp(rk + G * j);
        const uint8_t fj = L.fl[d];
        vw[j] = L.T[d];
        chgm |= (uint32_t)((fj >> 2) & 1u) << j;  // FL_CHG
    }
#pragma unroll
    for (int j = 0; j < NW; j++) {
        const int p = rk + G * j;
        const int d = Gm::domp(p);
        const bool chg = (chgm >> j) & 1u;
#ifdef FMM_PROFILE
        any_chg |= chg;
#endif
        if (!(chg || fresh)) continue;
        const int i0 = p >> (2 * Gm::LOG), i1 = (p >> Gm::LOG) & (E - 1), i2 = p & (E - 1);
        const double v = vw[j];
        Tt[tbase + p] = v;
        if (i2 == 0) P.Zf[((size_t)t * 2 + 0) * FACE + i0 * E + i1] = v;
        if (i2 == E - 1) P.Zf[((size_t)t * 2 + 1) * FACE + i0 * E + i1] = v;
        if (!chg) continue;
        // faces this boundary cell lies on whose neighbouring cell it can
        // improve: the halo holds that cell's value as loaded, an upper bound
        // of its current value (values only decrease), and a root from v
        // exceeds |v|; so |v| >= the halo magnitude means nothing to send
        const double av = fabs(v);
        const uint32_t fm = (i0 == 0 && av < fabs(L.T[d - Gm::OX]) ? 1u : 0u) |
                            (i0 == E - 1 && av < fabs(L.T[d + Gm::OX]) ? 2u : 0u) |
                            (i1 == 0 && av < fabs(L.T[d - Gm::OY]) ? 4u : 0u) |
                            (i1 == E - 1 && av < fabs(L.T[d + Gm::OY]) ? 8u : 0u) |
                            (i2 == 0 && av < fabs(L.T[d - Gm::OZ]) ? 16u : 0u) |
                            (i2 == E - 1 && av < fabs(L.T[d + Gm::OZ]) ? 32u : 0u);
        if (!fm) continue;
        fany |= fm;
        if (is_source(v, 0, bnd)) {
            fsrc |= fm;
        } else {
            const int sd = v < 0.0 ? 0 : 1;
            const unsigned long long b = bits_of(fabs(v));
            for (int f = 0; f < 6; f++)
                if ((fm >> f) & 1u) atomicMin(&L.bm[f * 2 + sd], b);
        }
    }
#ifdef FMM_PROFILE
    PROF_ADD(15, (__ballot(any_chg) == 0ull && mode == MODE_M2) ? 1 : 0);
#endif
    uint32_t srcFaces = 0, anyFaces = 0;
    if constexpr (G == 64) {
#pragma unroll
        for (int f = 0; f < 6; f++) {
            if (__ballot((fsrc >> f) & 1u)) srcFaces |= 1u << f;
            if (__ballot((fany >> f) & 1u)) anyFaces |= 1u << f;
        }
        wave_sync();
    } else {
        // also orders every write of the band minima bm before they are read
        const uint32_t m = grp_or(L, fsrc | (fany << 8));
        srcFaces = m & 0x3Fu;
        anyFaces = (m >> 8) & 0x3Fu;
    }
    if (fresh && rk == 0) __hip_atomic_store(&P.visit[t], phase + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    if (rk == 0) {
        TileMeta m;
        m.tmin[0] = tm0;
        m.tmin[1] = tm1;
        m.lastb[0] = bnd[0];
        m.lastb[1] = bnd[1];
        P.meta[t] = m;
    }
    ws.gmin0 = fmin(ws.gmin0, tm0);
    ws.gmin1 = fmin(ws.gmin1, tm1);

    // ---- pass changed boundary values to the neighbours (Alg. 13-15).  Lane
    // f < 6 of the group's first wavefront handles face f and lane 6 the tile
    // itself, so the atomics of all faces are in flight together.
    if (lead) {
        uint32_t u = 0;
        bool have = false, src = false;
        if (lane < 6 && ((anyFaces >> lane) & 1u)) {
            const int f = lane, ax = f >> 1;
            const bool plus = f & 1;
            const int32_t tca = ax == 0 ? tx : ax == 1 ? ty : tz;
            const int32_t tna = ax == 0 ? G0.t0 : ax == 1 ? G0.t1 : G0.t2;
            if (plus ? tca + 1 < tna : tca > 0) {
                const uint32_t ts = ax == 0 ? tsx : ax == 1 ? tsy : 1u;
                u = plus ? t + ts : t - ts;
                have = true;
                src = (srcFaces >> f) & 1u;
            }
        }
        const bool self = lane == 6 && (tm0 < FMM_INF || tm1 < FMM_INF);
        if (self) u = t;
        // a face with only band values: they join the neighbour's pending
        // minimum, and the neighbour joins the next live list
        const bool band = have && !src;
        if (band) {
            const unsigned long long b0 = L.bm[lane * 2], b1 = L.bm[lane * 2 + 1];
            unsigned long long *ux = P.text + ((size_t)u * 3 + phase % 3u) * 2;
            if (b0 != bits_of(FMM_INF)) atomicMin(&ux[0], b0);
            if (b1 != bits_of(FMM_INF)) atomicMin(&ux[1], b1);
        }
        // a new source value crossed the face: the neighbour re-marches.  The
        // dirty word and the live-list tag are requested together.
        uint32_t old = 1;
        if (have && src) old = atomicOr(&dprod[u], 1u << (lane ^ 1));
        bool append = false;
        if (self || band) append = atomicExch(&P.epoch[u], epoch) != epoch;
        bool toD = false;
        if (have && src && old == 0) {
            if (second)
                toD = true;
            else
                append = atomicExch(&P.epoch[u], epoch) != epoch;
        }
        const bool live = self || band || (have && src && old == 0 && !second);
        // wave-uniform follow-up
        const unsigned long long mD = __ballot(toD), mL = __ballot(append);
        const unsigned long long mP = __ballot(have && src && live);
        ws.pending += (uint32_t)__popcll(mP);
        for (int f = 0; f < 6; f++) {
            if (!((anyFaces >> f) & 1u) || ((srcFaces >> f) & 1u)) continue;
            ws.gmin0 = fmin(ws.gmin0, bitsd(L.bm[f * 2]));
            ws.gmin1 = fmin(ws.gmin1, bitsd(L.bm[f * 2 + 1]));
        }
        for (int k = 0; k < 7; k++) {
            const uint32_t uk = __shfl(u, k);
            if ((mD >> k) & 1ull) stage_push(L.stD, ws.nD, uk, cntD, dlist);
            if ((mL >> k) & 1ull) stage_push(L.stL, ws.nL, uk, cntNext, listNext);
        }
        PROF_ADD(13, __popcll(__ballot(have && src)));
        PROF_ADD(14, __popcll(__ballot(have && !src)));
    }
    Grp<G>::sync();
    PROF_CLOCK(t_end);
    PROF_ADD(6, t_end - t_levels);
}

// ---------------------------------------------------------------------------
// Persistent restart driver (Alg. 16).

// Alg. 16's exit test for one problem: no band value within the width on
// either side (an empty band reports +inf) and no tile left dirty.
__device__ __forceinline__ bool inst_done(double g0, double g1, uint32_t pend, double width)
{
    const bool done0 = !(g0 < FMM_INF && g0 <= width);
    const bool done1 = !(g1 < FMM_INF && g1 <= width);
    return done0 && done1 && pend == 0;
}

// The problem a wavefront is working on in the current restart: geometry,
// band bound per side (Alg. 16: min(minval + stride, width)) and whether the
// problem has already passed its exit test.
struct InstView {
    uint32_t j;
    TileGeo g;
    double bnd[2];
    bool done;
};

__device__ __forceinline__ void load_inst(const Params &P, uint32_t j, uint32_t r, int mode, InstView &v)
{
    const Inst &I = P.inst[j];
    v.j = j;
    v.g.base = I.base;
    v.g.t0 = I.t0;
    v.g.t1 = I.t1;
    v.g.t2 = I.t2;
    v.g.h = I.h;
    if (mode == MODE_INIT) {
        // heap initialisation: only seeds are sources
        v.bnd[0] = v.bnd[1] = -1.0;
        v.done = false;
        return;
    }
    InstSlot &S = P.ictl[j].slot[r % 3];
    const double g0 = bitsd(ld_acq64(&S.gmin[0])), g1 = bitsd(ld_acq64(&S.gmin[1]));
    v.done = inst_done(g0, g1, ld_acq(&S.pending), P.width);
    v.bnd[0] = fmin(g0 + I.stride, P.width);
    v.bnd[1] = fmin(g1 + I.stride, P.width);
}

// Hand a wavefront's band minima and dirty count to its problem's next slot.
__device__ __forceinline__ void flush_acc(const Params &P, WaveState &ws, uint32_t r)
{
    if (ws.acc != NO_INST && (threadIdx.x & 63) == 0) {
        InstSlot &S = P.ictl[ws.acc].slot[(r + 1) % 3];
        if (ws.gmin0 < FMM_INF) atomicMin(&S.gmin[0], bits_of(ws.gmin0));
        if (ws.gmin1 < FMM_INF) atomicMin(&S.gmin[1], bits_of(ws.gmin1));
        if (ws.pending) atomicAdd(&S.pending, ws.pending);
    }
    ws.acc = NO_INST;
    ws.pending = 0;
    ws.gmin0 = ws.gmin1 = FMM_INF;
}

template <int E, int NW, typename FT, bool AN, int G>
__device__ __forceinline__ void run_phase(const Params &P, TileLds<E, FT, G> &L, WgShared<NW> &S, int mode, uint32_t r,
                                          uint32_t phase, const uint32_t *items, uint32_t nitems, WaveState &ws)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int rk = Grp<G>::rank();
    const bool lead = Grp<G>::wave() == 0;
    Ctrl *c = P.ctrl;
    Slot &cur = c->slot[r % 3];
    Slot &nxt = c->slot[(r + 1) % 3];
    uint32_t *listNext = ((r + 1) & 1) ? P.list1 : P.list0;
    const uint32_t epoch = r + 1;
    // flags raised in phase p are read in phase p + 1: dirty[p % 2] is written,
    // dirty[(p + 1) % 2] (raised in the previous phase) is consumed
    uint32_t *dcons = (phase & 1u) ? P.dirty0 : P.dirty1;
    uint32_t *dprod = (phase & 1u) ? P.dirty1 : P.dirty0;
    // with a second march, tiles flagged by march-1 are handled in it;
    // otherwise they carry over to the next restart
    const bool second = mode == MODE_M1 && P.two_march;
    PROF_CLOCK(t_phase0);
    // The counters of the next phase are cleared now; their last use ended
    // two barriers ago and the barrier that ends this phase publishes them.
    if (blockIdx.x == 0 && threadIdx.x < WORK_SEGS) c->work[(phase + 1) % 3][threadIdx.x][0] = 0;

    // Dynamic distribution: the item list is cut into WORK_SEGS segments, one
    // per XCD (workgroups are dispatched to XCDs round robin), each with its
    // own counter.  A group claims items of its own segment one at a time
    // and then helps with the others; the claim for the next item is issued
    // before the current one is marched so its latency overlaps the loads.
    // In a workgroup group everything that steers the loop (claims, the abort
    // flag, a tile's due test) is read by rank 0 and broadcast.
    uint32_t(*cnt)[32] = c->work[phase % 3];
    uint32_t seg = blockIdx.x % WORK_SEGS, left = WORK_SEGS;
    uint32_t claim = 0;
    InstView iv;
    iv.j = NO_INST;
    if (rk == 0) claim = atomicAdd(&cnt[seg][0], 1u);
    for (;;) {
        const uint32_t k = grp_bcast(L, claim);
        const uint32_t lo = (uint32_t)(((uint64_t)nitems * seg) / WORK_SEGS);
        const uint32_t hi = (uint32_t)(((uint64_t)nitems * (seg + 1)) / WORK_SEGS);
        if (k >= hi - lo) {
            if (--left == 0) break;
            seg = (seg + 1) % WORK_SEGS;
            if (rk == 0) claim = atomicAdd(&cnt[seg][0], 1u);
            continue;
        }
        if (rk == 0) claim = atomicAdd(&cnt[seg][0], 1u);
        // the item and the abort flag are requested together (one round trip)
        const uint32_t i = lo + k;
        const uint32_t item = items[i];
        if constexpr (G == 64) {
            if (ld_acq(&c->abort)) break;
        } else {
            if (grp_bcast(L, rk == 0 ? ld_acq(&c->abort) : 0u)) break;
        }
        const uint32_t t = __builtin_amdgcn_readfirstlane(item);
        const uint32_t j = P.n_inst == 1 ? 0u : __builtin_amdgcn_readfirstlane(P.tinst[t]);
        if (j != iv.j) load_inst(P, j, r, mode, iv);
        // a problem that passed its exit test takes no further part
        if (iv.done) continue;
        if (j != ws.acc) {
            flush_acc(P, ws, r);
            ws.acc = j;
        }
        uint32_t dbits = 0;
        double lastb[2] = {-FMM_INF, -FMM_INF};
        if (mode != MODE_INIT) {
            // the word was last raised before the barrier that began this
            // phase, and no other group handles tile t in this phase.  It is
            // read with the tile's record (one round trip) and cleared below.
            dbits = dcons[t];
            const TileMeta m = P.meta[t];
            lastb[0] = m.lastb[0];
            lastb[1] = m.lastb[1];
            // pending minimum: the tile's own, and band values its neighbours
            // have passed on since (Alg. 15, BAND_OLD), one slot per phase
            unsigned long long *tx = P.text + (size_t)t * 6;
            unsigned long long xb[6];
#pragma unroll
            for (int q = 0; q < 6; q++) xb[q] = ld_acq64(&tx[q]);
            double p0 = fmin(m.tmin[0], fmin(bitsd(xb[0]), fmin(bitsd(xb[2]), bitsd(xb[4]))));
            double p1 = fmin(m.tmin[1], fmin(bitsd(xb[1]), fmin(bitsd(xb[3]), bitsd(xb[5]))));
            if constexpr (G == 64) {
                dbits = bcast0(dbits);
            } else {
                // neighbours may be writing the current phase's slots: rank 0's
                // reading decides for the whole group
                if (rk == 0) {
                    L.bc[1] = dbits;
                    L.bc[2] = (uint32_t)bits_of(p0);
                    L.bc[3] = (uint32_t)(bits_of(p0) >> 32);
                    L.bc[4] = (uint32_t)bits_of(p1);
                    L.bc[5] = (uint32_t)(bits_of(p1) >> 32);
                }
                __syncthreads();
                dbits = L.bc[1];
                p0 = bitsd((unsigned long long)L.bc[2] | ((unsigned long long)L.bc[3] << 32));
                p1 = bitsd((unsigned long long)L.bc[4] | ((unsigned long long)L.bc[5] << 32));
                __syncthreads();
            }
            if (rk == 0 && dbits) dcons[t] = 0u;
            const bool due =
                dbits != 0 || (p0 < FMM_INF && p0 <= iv.bnd[0]) || (p1 < FMM_INF && p1 <= iv.bnd[1]);
            if (!due) {
                // carried over unchanged to the next restart
                ws.gmin0 = fmin(ws.gmin0, p0);
                ws.gmin1 = fmin(ws.gmin1, p1);
                if (lead && (p0 < FMM_INF || p1 < FMM_INF)) {
                    uint32_t oe = 0;
                    if (lane == 0) oe = atomicExch(&P.epoch[t], epoch);
                    oe = bcast0(oe);
                    if (oe != epoch) stage_push(L.stL, ws.nL, t, &nxt.live_len, listNext);
                }
                PROF_ADD(7, 1);
                continue;
            }
            // the march reads the whole halo, so the values passed on in earlier
            // phases (whose data the barrier made visible) are consumed; the
            // current phase's slot stays for a later march
            if (rk == 0) {
#pragma unroll
                for (int q = 0; q < 6; q++)
                    if ((uint32_t)(q >> 1) != phase % 3u && xb[q] != bits_of(FMM_INF))
                        __hip_atomic_store(&tx[q], bits_of(FMM_INF), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            Grp<G>::sync();
        }
        tile_march<E, FT, G, AN>(P, L, iv.g, t, mode, dbits, iv.bnd, lastb, epoch, phase, second, ws, listNext,
                                 &nxt.live_len, P.dlist, &cur.d_len, dprod);
    }

    PROF_CLOCK(t_phase1);
    PROF_ADD(0, t_phase1 - t_phase0);
    // ---- workgroup epilogue: one atomic per list and per problem's
    // reduction per workgroup
    if (lane == 0) {
        S.cntL[wid] = ws.nL;
        S.cntD[wid] = ws.nD;
        S.pend[wid] = ws.pending;
        S.inst[wid] = ws.acc;
        S.gmin0[wid] = ws.gmin0;
        S.gmin1[wid] = ws.gmin1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tl = 0, td = 0;
        for (int w = 0; w < NW; w++) {
            tl += S.cntL[w];
            td += S.cntD[w];
        }
        S.baseL = tl ? atomicAdd(&nxt.live_len, tl) : 0u;
        S.baseD = td ? atomicAdd(&cur.d_len, td) : 0u;
        // wavefronts holding the same problem are combined
        for (int w = 0; w < NW; w++) {
            const uint32_t j = S.inst[w];
            if (j == NO_INST) continue;
            uint32_t tp = 0;
            double g0 = FMM_INF, g1 = FMM_INF;
            for (int u = w; u < NW; u++) {
                if (S.inst[u] != j) continue;
                tp += S.pend[u];
                g0 = fmin(g0, S.gmin0[u]);
                g1 = fmin(g1, S.gmin1[u]);
                if (u > w) S.inst[u] = NO_INST;
            }
            InstSlot &Z = P.ictl[j].slot[(r + 1) % 3];
            if (tp) atomicAdd(&Z.pending, tp);
            if (g0 < FMM_INF) atomicMin(&Z.gmin[0], bits_of(g0));
            if (g1 < FMM_INF) atomicMin(&Z.gmin[1], bits_of(g1));
        }
    }
    __syncthreads();
    uint32_t offL = S.baseL, offD = S.baseD;
    for (int w = 0; w < wid; w++) {
        offL += S.cntL[w];
        offD += S.cntD[w];
    }
    for (uint32_t q = lane; q < ws.nL; q += 64) listNext[offL + q] = L.stL[q];
    for (uint32_t q = lane; q < ws.nD; q += 64) P.dlist[offD + q] = L.stD[q];
    ws.nL = ws.nD = 0;
    ws.acc = NO_INST;
    ws.pending = 0;
    ws.gmin0 = ws.gmin1 = FMM_INF;
}

// NW wavefronts per workgroup in groups of G threads; WPE is the occupancy
// the register budget is fitted to (wavefronts per SIMD).
template <int E, int NW, typename FT, bool AN, int G, int WPE>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE))) k_driver(Params P)
{
    static_assert(G == 64 || G == NW * 64, "a group is one wavefront or the whole workgroup");
    __shared__ TileLds<E, FT, G> s_tile[NW * 64 / G];
    __shared__ WgShared<NW> s_g;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    TileLds<E, FT, G> &L = s_tile[G == 64 ? wid : 0];
    Ctrl *c = P.ctrl;
    const uint32_t nwg = gridDim.x;
    uint32_t gen = 0;
    WaveState ws;
    ws.nL = ws.nD = 0;
    ws.acc = NO_INST;
    ws.pending = 0;
    ws.gmin0 = ws.gmin1 = FMM_INF;
    ws.n_march = ws.n_round = ws.n_solve = ws.n_reopen = 0;
#ifdef FMM_PROFILE
    for (int k = 0; k < 16; k++) ws.prof[k] = 0;
#endif

    const unsigned long long t_start = wall_clock64();
    if (blockIdx.x == 0 && threadIdx.x == 0) c->nwg = nwg;
    // Phase sequence: heap initialisation (Alg. 9: only seeds are sources),
    // then per restart r = 1, 2, ...: march-1 over the live tiles, march-2
    // over the tiles whose halo changed (Alg. 16).  Every problem of a batch
    // has its own bound and exit test; the phases are shared, and the batch
    // ends when every problem has passed.  One call site keeps the march
    // inlined once.
    int mode = MODE_INIT;
    uint32_t r = 0;
    uint32_t phase = 1;  // phases are numbered from 1; tile visit stamps refer to them
    const uint32_t *items = P.list0;
    uint32_t nitems = ld_acq(&c->slot[0].live_len);
    bool run = ld_acq(&c->error) == 0;
    while (run) {
        PROF_CLOCK(t_p0);
        run_phase<E, NW, FT, AN, G>(P, L, s_g, mode, r, phase, items, nitems, ws);
        PROF_CLOCK(t_p1);
        const bool passed = grid_barrier(c, gen, nwg, &s_g.ok);
        PROF_CLOCK(t_p2);
        PROF_ADD(1, t_p2 - t_p0);
        PROF_ADD(9, t_p2 - t_p1);
        if (!passed) break;
        phase++;
        if (mode == MODE_M1 && P.two_march) {
            mode = MODE_M2;
            items = P.dlist;
            nitems = ld_acq(&c->slot[r % 3].d_len);
            continue;
        }
        r++;
        const uint32_t len = ld_acq(&c->slot[r % 3].live_len);
        // Alg. 16 exit tests, one per problem, on the minima gathered in the
        // restart that just ended.  Workgroup 0 also records when each problem
        // finished and clears the slots of the restart after next.
        int active = 0;
        for (uint32_t k = threadIdx.x; k < P.n_inst; k += blockDim.x) {
            InstCtl &ic = P.ictl[k];
            InstSlot &S = ic.slot[r % 3];
            const double g0 = bitsd(ld_acq64(&S.gmin[0])), g1 = bitsd(ld_acq64(&S.gmin[1]));
            const bool done = inst_done(g0, g1, ld_acq(&S.pending), P.width);
            active |= done ? 0 : 1;
            if (blockIdx.x == 0) {
                if (done && ic.restarts == 0) ic.restarts = r;
                InstSlot &Z = ic.slot[(r + 2) % 3];
                Z.gmin[0] = Z.gmin[1] = bits_of(FMM_INF);
                Z.pending = 0;
            }
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            Slot &Z = c->slot[(r + 2) % 3];
            Z.live_len = Z.d_len = 0;
        }
        if (!__syncthreads_or(active)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) c->restarts = r;
            break;
        }
        if (P.max_restarts > 0 && (int64_t)r > P.max_restarts) {
            if (blockIdx.x == 0) {
                for (uint32_t k = threadIdx.x; k < P.n_inst; k += blockDim.x)
                    if (P.ictl[k].restarts == 0) P.ictl[k].restarts = r;
                if (threadIdx.x == 0) {
                    atomicOr(&c->error_run, ERR_NOCONV);
                    c->restarts = r;
                }
            }
            break;
        }
        // Safety net: workgroup 0 aborts a solve that exceeds the time limit
        // (one clock read, shared through LDS); the others leave at their
        // next barrier.
        if (blockIdx.x == 0) {
            if (threadIdx.x == 0) s_g.ok = (wall_clock64() - t_start > P.time_limit_ticks) ? 1u : 0u;
            __syncthreads();
            const bool late = s_g.ok != 0;
            __syncthreads();
            if (late) {
                if (threadIdx.x == 0) {
                    atomicOr(&c->error_run, ERR_TIMEOUT);
                    atomicExch(&c->abort, 1u);
                    c->restarts = r;
                }
                break;
            }
        }
        mode = MODE_M1;
        items = (r & 1) ? P.list1 : P.list0;
        nitems = len;
    }
    // ---- statistics
    const unsigned long long ns = wave_sum((unsigned long long)ws.n_solve),
                             nr = wave_sum((unsigned long long)ws.n_reopen);
#ifdef FMM_PROFILE
    if (lane == 0)
        for (int k = 0; k < 16; k++) atomicAdd(&c->prof[k], ws.prof[k]);
#endif
    if (lane == 0) {
        atomicAdd(&c->n_march, ws.n_march);
        atomicAdd(&c->n_round, ws.n_round);
        atomicAdd(&c->n_solve, ns);
        atomicAdd(&c->n_reopen, nr);
    }
    (void)wid;
}

// ---------------------------------------------------------------------------
// Preparation (Alg. 8): problem table, workspace reset, tiled copy of F,
// seeds and the initial tile list.  Tiles never written hold +inf implicitly
// (visit = 0), so T is not filled.  Per-problem kernels take the problem's
// descriptor by value.

constexpr int INST_PACK = 16;
struct InstPack {
    Inst v[INST_PACK];
    uint32_t first, n;
};

// Copy up to INST_PACK problem descriptors into the workspace table (kernel
// arguments rather than a host copy, so the whole solve is a sequence of
// kernel launches).
__global__ void k_set_inst(Inst *dst, InstPack pk)
{
    const uint32_t k = threadIdx.x;
    if (k < pk.n) dst[pk.first + k] = pk.v[k];
}

__global__ void k_init_ws(Params P, int E)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) {
        Ctrl *c = P.ctrl;
        c->bar = 0;
        c->abort = 0;
        c->error = 0;
        c->error_run = 0;
        c->restarts = 0;
        c->nwg = 0;
        c->tile_edge = (uint32_t)E;
        c->n_inst = P.n_inst;
        c->magic = CTRL_MAGIC;
        for (int k = 0; k < 3; k++) c->slot[k].live_len = c->slot[k].d_len = 0;
        c->n_march = c->n_solve = c->n_round = c->n_reopen = 0;
        for (int k = 0; k < 16; k++) c->prof[k] = 0;
        for (int k = 0; k < 3; k++)
            for (int g = 0; g < WORK_SEGS; g++) c->work[k][g][0] = 0;
    }
    for (int64_t i = i0; i < (int64_t)P.n_inst; i += stride) {
        InstCtl &ic = P.ictl[i];
        for (int k = 0; k < 3; k++) {
            ic.slot[k].gmin[0] = ic.slot[k].gmin[1] = bits_of(FMM_INF);
            ic.slot[k].pending = 0;
        }
        ic.restarts = 0;
        ic.n_accepted = 0;
        ic.max_abs_bits = 0;
    }
    for (int64_t i = i0; i < (int64_t)P.ntiles; i += stride) {
        TileMeta m;
        m.tmin[0] = m.tmin[1] = FMM_INF;
        m.lastb[0] = m.lastb[1] = -FMM_INF;
        P.meta[i] = m;
        P.dirty0[i] = 0;
        P.dirty1[i] = 0;
        P.epoch[i] = 0;
        P.tflags[i] = 0;
        P.visit[i] = 0;
#pragma unroll
        for (int k = 0; k < 6; k++) P.text[i * 6 + k] = bits_of(FMM_INF);
    }
    const int64_t nm = (int64_t)P.ntiles * P.mask_words;
    for (int64_t i = i0; i < nm; i += stride) P.mask[i] = 0ull;
}

// Tiled copy of one problem's speeds (0 outside its grid) and the problem
// index of each of its tiles.
template <int E, typename FT> __global__ void __launch_bounds__(STAGE_THREADS) k_tile_speed(Params P, Inst I, uint32_t j)
{
    using S = Stage<E, FT>;
    constexpr int V = S::V, CH = S::CH, W = S::W, R = S::R, TS = S::TS;
    constexpr int NL = R * W / STAGE_THREADS, NS = CH * V / STAGE_THREADS;  // values per thread and side
    __shared__ FT buf[CH * TS];
    const FT *F = (const FT *)I.F;
    FT *Ft = (FT *)P.Ft;
    const int64_t nch = (I.t2 + CH - 1) / CH;
    const int64_t units = (int64_t)I.t0 * I.t1 * nch;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t cc = u % nch, ab = u / nch, b = ab % I.t1, a = ab / I.t1;
        const int64_t c0 = cc * CH;
        const int nt = (int)(I.t2 - c0 < CH ? I.t2 - c0 : CH);
        // eight loads of the thread are in flight before the first is used
        for (int q0 = 0; q0 < NL; q0 += STAGE_BATCH) {
            FT v[STAGE_BATCH];
#pragma unroll
            for (int q = 0; q < STAGE_BATCH; q++) {
                const int idx = (int)threadIdx.x + (q0 + q) * STAGE_THREADS;
                const int r = idx / W, c = idx - r * W;
                const int64_t i0 = a * E + r / E, i1 = b * E + r % E, i2 = c0 * E + c;
                v[q] = (FT)0;
                if (q0 + q < NL && c / E < nt && i0 < I.n0 && i1 < I.n1 && i2 < I.n2)
                    v[q] = F[(i0 * I.n1 + i1) * I.n2 + i2];
            }
#pragma unroll
            for (int q = 0; q < STAGE_BATCH; q++) {
                const int idx = (int)threadIdx.x + (q0 + q) * STAGE_THREADS;
                const int r = idx / W, c = idx - r * W;
                if (q0 + q < NL) buf[(c / E) * TS + r * E + c % E] = v[q];
            }
        }
        __syncthreads();
        const size_t t0 = (size_t)I.base + (size_t)((a * I.t1 + b) * I.t2 + c0);
#pragma unroll 8
        for (int q = 0; q < NS; q++) {
            const int idx = (int)threadIdx.x + q * STAGE_THREADS;
            const int k = idx / V;
            if (k < nt) Ft[t0 * V + idx] = buf[k * TS + (idx - k * V)];
        }
        if ((int)threadIdx.x < nt) P.tinst[t0 + threadIdx.x] = j;
        __syncthreads();
    }
}

__device__ __forceinline__ void add_init_tile(const Params &P, uint32_t t)
{
    const uint32_t old = atomicOr(&P.tflags[t], (uint32_t)TF_INIT);
    if (!(old & TF_INIT)) {
        const uint32_t pos = atomicAdd(&P.ctrl->slot[0].live_len, 1u);
        P.list0[pos] = t;
    }
}

// Locate a seed of problem I: global tile index and interior index, or false
// if out of range.
__device__ __forceinline__ bool seed_cell(const Inst &I, int64_t g, int E, uint32_t &t, int &p, int l[3],
                                          int64_t c[3])
{
    const int64_t N = I.n0 * I.n1 * I.n2;
    if (g < 0 || g >= N) return false;
    const int64_t i0 = g / (I.n1 * I.n2), rem = g - i0 * (I.n1 * I.n2);
    const int64_t i1 = rem / I.n2, i2 = rem - i1 * I.n2;
    c[0] = i0 / E;
    c[1] = i1 / E;
    c[2] = i2 / E;
    l[0] = (int)(i0 - c[0] * E);
    l[1] = (int)(i1 - c[1] * E);
    l[2] = (int)(i2 - c[2] * E);
    t = I.base + (uint32_t)((c[0] * I.t1 + c[1]) * I.t2 + c[2]);
    p = (l[0] * E + l[1]) * E + l[2];
    return true;
}

// Seeds, pass 1: validate, set the seed bits, and list the seed tiles and
// the neighbours across any tile face a seed lies on.
__global__ void k_seed_mark(Params P, Inst I, int E)
{
    const int64_t *__restrict__ idx = I.seed_idx;
    const double *__restrict__ val = I.seed_val;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < I.n_seeds;
         k += (int64_t)gridDim.x * blockDim.x) {
        uint32_t t;
        int p, l[3];
        int64_t c[3];
        if (!seed_cell(I, idx[k], E, t, p, l, c)) {
            atomicOr(&P.ctrl->error, ERR_SEED_RANGE);
            continue;
        }
        if (!(fabs(val[k]) < FMM_INF)) {
            atomicOr(&P.ctrl->error, ERR_SEED_VALUE);
            continue;
        }
        const unsigned long long bit = 1ull << (p & 63);
        const unsigned long long old = atomicOr(&P.mask[(size_t)t * P.mask_words + (p >> 6)], bit);
        if (old & bit) {
            atomicOr(&P.ctrl->error, ERR_SEED_DUP);
            continue;
        }
        atomicOr(&P.tflags[t], (uint32_t)TF_SEED);
        add_init_tile(P, t);
        const uint32_t ts[3] = {(uint32_t)I.t1 * (uint32_t)I.t2, (uint32_t)I.t2, 1u};
        const int32_t tn[3] = {I.t0, I.t1, I.t2};
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            if (l[ax] == 0 && c[ax] > 0) add_init_tile(P, t - ts[ax]);
            if (l[ax] == E - 1 && c[ax] + 1 < tn[ax]) add_init_tile(P, t + ts[ax]);
        }
    }
}

// Seeds, pass 2 (all problems at once): every seed tile starts as +inf
// (tiled T and face buffer).
template <int E> __global__ void k_seed_fill(Params P)
{
    constexpr int V = E * E * E, FACE = E * E;
    const uint32_t n = P.ctrl->slot[0].live_len;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint32_t t = P.list0[i];
        if (!(P.tflags[t] & TF_SEED)) continue;
        for (int p = threadIdx.x; p < V; p += blockDim.x) P.Tt[(size_t)t * V + p] = FMM_INF;
        for (int p = threadIdx.x; p < 2 * FACE; p += blockDim.x) P.Zf[(size_t)t * 2 * FACE + p] = FMM_INF;
        if (threadIdx.x == 0) P.visit[t] = 1u;
    }
}

// Seeds, pass 3: the values (KNOWN_FIX points of Alg. 8).
__global__ void k_seed_scatter(Params P, Inst I, int E)
{
    if (P.ctrl->error) return;
    const int V = E * E * E, FACE = E * E;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < I.n_seeds;
         k += (int64_t)gridDim.x * blockDim.x) {
        uint32_t t;
        int p, l[3];
        int64_t c[3];
        if (!seed_cell(I, I.seed_idx[k], E, t, p, l, c)) continue;
        const double v = I.seed_val[k];
        P.Tt[(size_t)t * V + p] = v;
        if (l[2] == 0) P.Zf[((size_t)t * 2 + 0) * FACE + l[0] * E + l[1]] = v;
        if (l[2] == E - 1) P.Zf[((size_t)t * 2 + 1) * FACE + l[0] * E + l[1]] = v;
    }
}

template <typename FT> __global__ void k_validate(Params P, Inst I)
{
    const int64_t N = I.n0 * I.n1 * I.n2;
    const FT *F = (const FT *)I.F;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        bad |= !(fabs((double)F[i]) < FMM_INF);
    if (bad) atomicOr(&P.ctrl->error, ERR_SPEED);
}

// ---------------------------------------------------------------------------
// Finalize one problem: row-major T (accepted points and seeds keep their
// values, all others +inf), status bytes and statistics.  Work units as for
// the speeds: a unit reads its CH tiles as one contiguous run (tiles never
// written are skipped: they hold +inf) and writes E * E row pieces.  Every
// value is read and written once, so both sides go through non-temporal
// accesses.

template <int E> __global__ void __launch_bounds__(STAGE_THREADS) k_finalize(Params P, Inst I, uint32_t j)
{
    using S = Stage<E, double>;
    constexpr int V = S::V, CH = S::CH, W = S::W, R = S::R, TS = S::TS;
    constexpr int NL = CH * V / STAGE_THREADS, NS = R * W / STAGE_THREADS;  // values per thread and side
    __shared__ double buf[CH * TS];
    __shared__ uint32_t s_vis[CH], s_tf[CH];
    const int64_t nch = (I.t2 + CH - 1) / CH;
    const int64_t units = (int64_t)I.t0 * I.t1 * nch;
    unsigned long long acc = 0;
    double mx = 0.0;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t cc = u % nch, ab = u / nch, b = ab % I.t1, a = ab / I.t1;
        const int64_t c0 = cc * CH;
        const int nt = (int)(I.t2 - c0 < CH ? I.t2 - c0 : CH);
        const size_t t0 = (size_t)I.base + (size_t)((a * I.t1 + b) * I.t2 + c0);
        if ((int)threadIdx.x < nt) {
            s_vis[threadIdx.x] = P.visit[t0 + threadIdx.x];
            s_tf[threadIdx.x] = P.tflags[t0 + threadIdx.x];
        }
        __syncthreads();
        for (int q0 = 0; q0 < NL; q0 += STAGE_BATCH) {
            double v[STAGE_BATCH];
#pragma unroll
            for (int q = 0; q < STAGE_BATCH; q++) {
                const int idx = (int)threadIdx.x + (q0 + q) * STAGE_THREADS;
                const int k = idx / V;
                v[q] = FMM_INF;
                if (q0 + q < NL && k < nt && s_vis[k]) v[q] = __builtin_nontemporal_load(&P.Tt[t0 * V + idx]);
            }
#pragma unroll
            for (int q = 0; q < STAGE_BATCH; q++) {
                const int idx = (int)threadIdx.x + (q0 + q) * STAGE_THREADS;
                const int k = idx / V;
                if (q0 + q < NL) buf[k * TS + (idx - k * V)] = v[q];
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < NS; q++) {
            const int idx = (int)threadIdx.x + q * STAGE_THREADS;
            const int r = idx / W, c = idx - r * W, k = c / E;
            const int64_t i0 = a * E + r / E, i1 = b * E + r % E, i2 = c0 * E + c;
            if (k >= nt || i0 >= I.n0 || i1 >= I.n1 || i2 >= I.n2) continue;
            const int p = r * E + c % E;
            const double x = buf[k * TS + p];
            bool seed = false;
            if (s_tf[k] & TF_SEED) seed = (P.mask[(t0 + k) * P.mask_words + (p >> 6)] >> (p & 63)) & 1ull;
            const double ax = fabs(x);
            const uint8_t neg = x < 0.0 ? 0x80 : 0;
            uint8_t st;
            double out = FMM_INF;
            if (seed) {
                st = 3 | neg;
                out = x;
                mx = fmax(mx, ax);
            } else if (ax < FMM_INF && ax <= P.width) {
                st = 2 | neg;
                out = x;
                acc++;
                mx = fmax(mx, ax);
            } else if (ax < FMM_INF) {
                st = 1 | neg;
            } else {
                st = 0;
            }
            const int64_t g = (i0 * I.n1 + i1) * I.n2 + i2;
            // streamed out once: non-temporal stores (0.7 ms less per 1024^3
            // solve than plain ones)
            __builtin_nontemporal_store(out, &I.T[g]);
            if (I.status) __builtin_nontemporal_store(st, &I.status[g]);
        }
        __syncthreads();
    }
    __shared__ unsigned long long s_acc[STAGE_THREADS / 64];
    __shared__ double s_mx[STAGE_THREADS / 64];
    acc = wave_sum(acc);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        s_acc[wid] = acc;
        s_mx[wid] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sa = 0;
        double m = 0.0;
        for (int w = 0; w < STAGE_THREADS / 64; w++) {
            sa += s_acc[w];
            m = fmax(m, s_mx[w]);
        }
        if (sa) atomicAdd(&P.ictl[j].n_accepted, sa);
        atomicMax(&P.ictl[j].max_abs_bits, bits_of(m));
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers.

static int num_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 1;
    }
    return cus;
}

template <int E> static hipError_t launch_prepare_t(const Params &P, const Inst *insts, int64_t n, bool validate,
                                                   bool f64, hipStream_t s)
{
    const int cus = num_cus();
    hipError_t e;
    for (int64_t first = 0; first < n; first += INST_PACK) {
        InstPack pk;
        memset(&pk, 0, sizeof pk);
        pk.first = (uint32_t)first;
        pk.n = (uint32_t)std::min<int64_t>(INST_PACK, n - first);
        for (uint32_t k = 0; k < pk.n; k++) pk.v[k] = insts[first + k];
        hipLaunchKernelGGL(k_set_inst, dim3(1), dim3(64), 0, s, (Inst *)P.inst, pk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int64_t init_items = std::max<int64_t>((int64_t)P.ntiles, (int64_t)P.n_inst);
    const unsigned ib = (unsigned)std::max<int64_t>(1, std::min<int64_t>((init_items + 255) / 256, (int64_t)cus * 4));
    hipLaunchKernelGGL(k_init_ws, dim3(ib), dim3(256), 0, s, P, E);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int64_t j = 0; j < n; j++) {
        const Inst &I = insts[j];
        const int ch = f64 ? Stage<E, double>::CH : Stage<E, float>::CH;
        const int64_t units = (int64_t)I.t0 * I.t1 * ((I.t2 + ch - 1) / ch);
        const unsigned tb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(units, (int64_t)cus * 8));
        if (f64)
            hipLaunchKernelGGL((k_tile_speed<E, double>), dim3(tb), dim3(STAGE_THREADS), 0, s, P, I, (uint32_t)j);
        else
            hipLaunchKernelGGL((k_tile_speed<E, float>), dim3(tb), dim3(STAGE_THREADS), 0, s, P, I, (uint32_t)j);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    bool any_seeds = false;
    for (int64_t j = 0; j < n; j++) {
        const Inst &I = insts[j];
        if (I.n_seeds <= 0) continue;
        any_seeds = true;
        const unsigned blocks = (unsigned)std::min<int64_t>((I.n_seeds + 255) / 256, (int64_t)cus * 16);
        hipLaunchKernelGGL(k_seed_mark, dim3(blocks), dim3(256), 0, s, P, I, E);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (any_seeds) {
        hipLaunchKernelGGL(k_seed_fill<E>, dim3(cus * 8), dim3(256), 0, s, P);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int64_t j = 0; j < n; j++) {
            const Inst &I = insts[j];
            if (I.n_seeds <= 0) continue;
            const unsigned blocks = (unsigned)std::min<int64_t>((I.n_seeds + 255) / 256, (int64_t)cus * 16);
            hipLaunchKernelGGL(k_seed_scatter, dim3(blocks), dim3(256), 0, s, P, I, E);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (validate) {
        for (int64_t j = 0; j < n; j++) {
            if (f64)
                hipLaunchKernelGGL(k_validate<double>, dim3(cus * 8), dim3(256), 0, s, P, insts[j]);
            else
                hipLaunchKernelGGL(k_validate<float>, dim3(cus * 8), dim3(256), 0, s, P, insts[j]);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_prepare(const Params &P, const Inst *insts, int64_t n, int E, bool validate, bool f64,
                          hipStream_t s)
{
    switch (E) {
    case 4: return launch_prepare_t<4>(P, insts, n, validate, f64, s);
    case 8: return launch_prepare_t<8>(P, insts, n, validate, f64, s);
    case 16: return launch_prepare_t<16>(P, insts, n, validate, f64, s);
    default: return hipErrorInvalidValue;
    }
}

template <int E, int NW, typename FT, bool AN, int G, int WPE>
static hipError_t launch_driver_t(const Params &P, hipStream_t s, uint32_t *nwg_out)
{
    static int occ = -1;
    auto kern = k_driver<E, NW, FT, AN, G, WPE>;
    if (occ < 0) {
        int nb = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, NW * 64, 0);
        if (e != hipSuccess) return e;
        occ = nb;
    }
    if (occ <= 0) return hipErrorInvalidConfiguration;
    const unsigned grid = (unsigned)(occ * num_cus());
    Params Pc = P;
    void *args[] = {&Pc};
    if (nwg_out) *nwg_out = grid;
    // one full occupancy wave, launched cooperatively (also under stream
    // capture); should the workgroups still not be resident together, the
    // barrier's bounded wait aborts the solve
    return launch_coresident((const void *)kern, dim3(grid), dim3(NW * 64), args, s);
}

// The weighted local solver (per-axis spacing) is a separate instantiation,
// so the uniform-grid march carries none of its code.
template <bool AN> static hipError_t launch_driver_a(const Params &P, int E, bool f64, hipStream_t s, uint32_t *nwg_out)
{
    // 4^3 and 8^3 tiles: one wavefront per tile, one workgroup per CU (three
    // wavefronts per SIMD).  16^3 tiles: one workgroup per tile, four
    // wavefronts and two tiles per CU with FP32 speeds (the LDS of two fits),
    // eight wavefronts and one tile per CU with FP64 speeds.
    switch (E) {
    case 4:
        return f64 ? launch_driver_t<4, 12, double, AN, 64, 3>(P, s, nwg_out)
                   : launch_driver_t<4, 12, float, AN, 64, 3>(P, s, nwg_out);
    case 8:
        return f64 ? launch_driver_t<8, FMM_E8_WAVES_F64, double, AN, 64, 3>(P, s, nwg_out)
                   : launch_driver_t<8, FMM_E8_WAVES_F32, float, AN, 64, 3>(P, s, nwg_out);
    case 16:
        return f64 ? launch_driver_t<16, 8, double, AN, 512, 2>(P, s, nwg_out)
                   : launch_driver_t<16, 4, float, AN, 256, 2>(P, s, nwg_out);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_driver(const Params &P, int E, bool f64, hipStream_t s, uint32_t *nwg_out)
{
    return P.sp.aniso ? launch_driver_a<true>(P, E, f64, s, nwg_out) : launch_driver_a<false>(P, E, f64, s, nwg_out);
}

template <int E> static hipError_t launch_finalize_t(const Params &P, const Inst *insts, int64_t n, hipStream_t s)
{
    const int cus = num_cus();
    for (int64_t j = 0; j < n; j++) {
        const Inst &I = insts[j];
        const int64_t units = (int64_t)I.t0 * I.t1 * ((I.t2 + Stage<E, double>::CH - 1) / Stage<E, double>::CH);
        const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(units, (int64_t)cus * 8));
        hipLaunchKernelGGL(k_finalize<E>, dim3(blocks), dim3(STAGE_THREADS), 0, s, P, I, (uint32_t)j);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_finalize(const Params &P, const Inst *insts, int64_t n, int E, hipStream_t s)
{
    switch (E) {
    case 4: return launch_finalize_t<4>(P, insts, n, s);
    case 8: return launch_finalize_t<8>(P, insts, n, s);
    case 16: return launch_finalize_t<16>(P, insts, n, s);
    default: return hipErrorInvalidValue;
    }
}

// The device error bits of the last solve (input errors found before the
// driver and errors raised while it ran) copied to a caller's word.
__global__ void k_report_error(const Ctrl *c, uint32_t *out)
{
    if (threadIdx.x == 0) *out = c->error | c->error_run;
}

hipError_t launch_report_error(const Params &P, uint32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_report_error, dim3(1), dim3(64), 0, s, (const Ctrl *)P.ctrl, out);
    return hipGetLastError();
}

hipError_t launch_eval_godunov(const double *a, const double *r, double *out, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)num_cus() * 32);
    hipLaunchKernelGGL(k_eval_godunov, dim3((unsigned)blocks), dim3(256), 0, s, a, r, out, n);
    return hipGetLastError();
}

}  // namespace fmm
