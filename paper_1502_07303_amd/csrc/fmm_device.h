// Device helpers shared by the forward solver and the adjoint kernels, and
// the launch of their persistent kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

namespace fmm {

#define FMM_INF __builtin_huge_val()

// ---------------------------------------------------------------------------
// Correctly rounded square root and division by 3 for the local solver, in
// fewer instructions than the general library sequences.
//
// solver_sqrt: the hardware reciprocal square root estimate y ~ 1/sqrt(x),
// one coupled Newton step on s ~ sqrt(x) and h ~ 1/(2 sqrt(x)) (Goldschmidt's
// iteration), then two residual corrections s += (x - s^2) h; the last one
// rounds correctly.  The general routine additionally rescales tiny inputs
// and patches 0 and +inf.  Here inputs below 2^-767 (0 included) take the
// library routine on a branch that the solver's discriminants practically
// never reach; +inf (only when r = +inf, where the solver returns +inf from
// its first root) gives NaN, which the root comparisons reject.
__device__ __forceinline__ double solver_sqrt(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y, h = y * 0.5;
    const double e = __builtin_fma(-h, s, 0.5);
    s = __builtin_fma(s, e, s);
    h = __builtin_fma(h, e, h);
    double d = __builtin_fma(-s, s, x);
    s = __builtin_fma(d, h, s);
    d = __builtin_fma(-s, s, x);
    s = __builtin_fma(d, h, s);
    if (__builtin_expect(x < 0x1p-767, 0)) {
        asm volatile("");  // keeps the rare path a branch (not computed and selected)
        s = sqrt(x);
    }
    return s;
}

// x / 3, correctly rounded: q = x * RN(1/3) is within one ulp, and one
// remainder step q + (x - 3 q) RN(1/3) rounds correctly (Markstein's
// theorem; x / 3 is never a tie).
__device__ __forceinline__ double div3(double x)
{
    const double third = 1.0 / 3.0;
    const double q = x * third;
    return __builtin_fma(__builtin_fma(-q, 3.0, x), third, q);
}

// h / f for the march's r = h / F: a reciprocal estimate refined by two
// Newton steps, the quotient, and one remainder correction.  For operands of
// moderate exponents this is the correctly rounded quotient (the general
// routine additionally rescales extreme exponents and patches special
// values).  f must be positive and finite (the tile load keeps an infinite
// FP32 speed as the largest finite one).
__device__ __forceinline__ double solver_div(double h, double f)
{
    double y = __builtin_amdgcn_rcp(f);
    y = __builtin_fma(y, __builtin_fma(-f, y, 1.0), y);
    y = __builtin_fma(y, __builtin_fma(-f, y, 1.0), y);
    const double q = h * y;
    return __builtin_fma(__builtin_fma(-f, q, h), y, q);
}

// ---------------------------------------------------------------------------
// Local solver (Alg. 11 with Eqs. 4-7).  a = per-axis upwind values (+inf when
// an axis has no upwind neighbour), r = h / F.  With a1 <= a2 <= a3:
//   u1 = a1 + r
//   u2 = ((a1 + a2) + sqrt(2 r^2 - (a2 - a1)^2)) * 0.5          causal iff u2 > a2
//   u3 = (((a1 + a2) + a3) + sqrt(3 r^2 - (((a2-a1)^2 + (a3-a1)^2) + (a3-a2)^2))) / 3
//                                                                causal iff u3 > a3
// and G is the smallest causal root (discriminants must be >= 0).  This is the
// paper's quadratic with the identity (sum a)^2 - k sum a^2 = -sum_{i<j}(a_i-a_j)^2
// applied, so nothing of size T^2/h^2 cancels.  *k receives how many of the
// sorted values the returned root uses (0 when there is no upwind value).
__device__ __forceinline__ double godunov_sel(double x, double y, double z, double r, int *k)
{
    double lo = fmin(x, y), hi = fmax(x, y);
    double a3 = fmax(hi, z), m = fmin(hi, z);
    double a1 = fmin(lo, m), a2 = fmax(lo, m);
    // no upwind value: a1 = +inf makes the first root +inf (r >= 0), with
    // no branch ahead of the one on a2
    *k = a1 < FMM_INF ? 1 : 0;
    double r2 = r * r;
    double best = a1 + r;
    if (a2 < FMM_INF) {
        double d12 = a2 - a1;
        double D2 = 2.0 * r2 - d12 * d12;
        if (D2 >= 0.0) {
            double u2 = ((a1 + a2) + solver_sqrt(D2)) * 0.5;
            if (u2 > a2 && u2 < best) {
                best = u2;
                *k = 2;
            }
        }
        if (a3 < FMM_INF) {
            double d13 = a3 - a1, d23 = a3 - a2;
            double D3 = 3.0 * r2 - ((d12 * d12 + d13 * d13) + d23 * d23);
            if (D3 >= 0.0) {
                double u3 = div3(((a1 + a2) + a3) + solver_sqrt(D3));
                if (u3 > a3 && u3 < best) {
                    best = u3;
                    *k = 3;
                }
            }
        }
    }
    return best;
}

__device__ __forceinline__ double godunov(double x, double y, double z, double r)
{
    int k;
    return godunov_sel(x, y, z, r, &k);
}

// The local solver with per-axis spacing h s_i (weights w_i = 1 / s_i^2):
// sum_i w_i max(u - a_i, 0)^2 = r^2, r = h / F.  For the k smallest values,
// sorted together with their scales (ties keep axis order),
//   u1 = a1 + r s1
//   u2 = ((w1 a1 + w2 a2) + sqrt((w1+w2) r^2 - (w1 w2)(a2-a1)^2)) / (w1+w2)
//   u3 = (((w1 a1 + w2 a2) + w3 a3) + sqrt(((w1+w2)+w3) r^2
//          - (((w1 w2)(a2-a1)^2 + (w1 w3)(a3-a1)^2) + (w2 w3)(a3-a2)^2))) / ((w1+w2)+w3)
// with the same causality rule and minimum.  With unit scales every
// operation is the one of godunov_sel().
__device__ __forceinline__ double godunov_w_sel(double x, double y, double z, double sx, double sy, double sz,
                                                double r, int *k)
{
    double a1 = x, a2 = y, a3 = z, s1 = sx, s2 = sy, s3 = sz, t;
    if (a1 > a2) { t = a1; a1 = a2; a2 = t; t = s1; s1 = s2; s2 = t; }
    if (a2 > a3) {
        t = a2; a2 = a3; a3 = t; t = s2; s2 = s3; s3 = t;
        if (a1 > a2) { t = a1; a1 = a2; a2 = t; t = s1; s1 = s2; s2 = t; }
    }
    const double w1 = 1.0 / (s1 * s1), w2 = 1.0 / (s2 * s2), w3 = 1.0 / (s3 * s3);
    *k = 0;
    if (!(a1 < FMM_INF)) return FMM_INF;
    double r2 = r * r;
    double best = a1 + r * s1;
    *k = 1;
    if (a2 < FMM_INF) {
        double d12 = a2 - a1;
        double D2 = (w1 + w2) * r2 - (w1 * w2) * (d12 * d12);
        if (D2 >= 0.0) {
            double u2 = ((w1 * a1 + w2 * a2) + sqrt(D2)) / (w1 + w2);
            if (u2 > a2 && u2 < best) {
                best = u2;
                *k = 2;
            }
        }
        if (a3 < FMM_INF) {
            double d13 = a3 - a1, d23 = a3 - a2;
            double D3 = ((w1 + w2) + w3) * r2 -
                        (((w1 * w2) * (d12 * d12) + (w1 * w3) * (d13 * d13)) + (w2 * w3) * (d23 * d23));
            if (D3 >= 0.0) {
                double u3 = (((w1 * a1 + w2 * a2) + w3 * a3) + sqrt(D3)) / ((w1 + w2) + w3);
                if (u3 > a3 && u3 < best) {
                    best = u3;
                    *k = 3;
                }
            }
        }
    }
    return best;
}

// Per-axis grid spacing factors of a solve (spacing h * s[a] along axis a).
struct Spacing {
    double s[3];
    int aniso;  // 0: all factors are 1 (the isotropic solver is used)
};

__device__ __forceinline__ double local_solve(const Spacing &sp, double x, double y, double z, double r, int *k)
{
    if (sp.aniso) return godunov_w_sel(x, y, z, sp.s[0], sp.s[1], sp.s[2], r, k);
    return godunov_sel(x, y, z, r, k);
}

// ---------------------------------------------------------------------------
// Small helpers.

__device__ __forceinline__ unsigned long long bits_of(double x) { return (unsigned long long)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T> __device__ __forceinline__ T bcast0(T v) { return __shfl(v, 0); }

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ uint32_t ld_acq(uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_acq64(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-wide barrier of a persistent launch whose workgroups are all
// resident: a monotonic arrival counter (`bar`), agent-scope release and
// acquire fences, and a bounded wait.  A timeout (20 s) or an abort raised
// elsewhere sets `abort` (and `timeout_bit` in *err), so every workgroup
// leaves and the kernel always terminates.  Returns false on abort.
// The workgroup barrier first orders every wavefront's writes before thread
// 0's agent-scope release, which publishes them (release is cumulative), and
// thread 0's acquire, which invalidates the CU's and the XCD's caches, comes
// before the barrier that lets the other wavefronts read: one cache
// write-back and one invalidation per workgroup instead of one per wavefront.
__device__ __forceinline__ bool grid_sync(uint32_t *bar, uint32_t *abort, uint32_t *err, uint32_t timeout_bit,
                                          uint32_t &gen, uint32_t nwg, uint32_t *s_ok)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        gen++;
        uint32_t target = gen * nwg;
        uint32_t ok = 1;
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long t0 = wall_clock64();
        while (ld_acq(bar) < target) {
            if (ld_acq(abort)) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            if (wall_clock64() - t0 > 2000000000ull) {  // 20 s at the 100 MHz constant clock
                atomicOr(err, timeout_bit);
                atomicExch(abort, 1u);
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// ---------------------------------------------------------------------------
// Host side, shared by the forward driver and the adjoint sweep.

// Launch a persistent kernel whose workgroups must all be resident at once
// (its device-wide barriers wait for every workgroup): a cooperative launch.
// Stream capture records the launch as an ordinary kernel node, so the
// cooperative attribute is set on the node the launch just added (the
// stream's only capture dependency), and a replay of the graph keeps the
// guarantee.
inline hipError_t launch_coresident(const void *kern, dim3 grid, dim3 block, void **args, hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return e;
    if ((e = hipLaunchCooperativeKernel(kern, grid, block, args, 0, s)) != hipSuccess) return e;
    if (cs != hipStreamCaptureStatusActive) return hipSuccess;
    const hipGraphNode_t *deps = nullptr;
    size_t nd = 0;
    hipGraph_t g = nullptr;
    unsigned long long id = 0;
    if ((e = hipStreamGetCaptureInfo_v2(s, &cs, &id, &g, &deps, &nd)) != hipSuccess) return e;
    if (nd != 1 || !deps) return hipErrorStreamCaptureUnsupported;
    hipGraphNodeType ty = hipGraphNodeTypeEmpty;
    if ((e = hipGraphNodeGetType(deps[0], &ty)) != hipSuccess) return e;
    if (ty != hipGraphNodeTypeKernel) return hipErrorStreamCaptureUnsupported;
    hipLaunchAttributeValue v;
    memset(&v, 0, sizeof v);
    v.cooperative = 1;
    return hipGraphKernelNodeSetAttribute(deps[0], hipLaunchAttributeCooperative, &v);
}

}  // namespace fmm
