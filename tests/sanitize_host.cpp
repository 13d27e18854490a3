// Drives the host side of libfmm (argument validation, workspace sizing and
// carving, option handling of every entry point) for a build whose host code
// carries AddressSanitizer and UndefinedBehaviorSanitizer.  Every call here
// returns before any device work: invalid arguments, too-small workspaces,
// sizes only.  Exits non-zero on a wrong return code.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "fmm.h"

static int fails = 0;
#define EXPECT(c)                                                    \
    do {                                                             \
        if (!(c)) {                                                  \
            fprintf(stderr, "line %d: expected %s\n", __LINE__, #c); \
            fails++;                                                 \
        }                                                            \
    } while (0)

int main()
{
    void *fake = (void *)0x100000;  // never dereferenced: every call fails validation first
    fmm_opts o;
    fmm_default_opts(&o);
    for (int e : {0, 4, 8, 16}) {
        o.tile_edge = e;
        for (int dt : {FMM_F32, FMM_F64}) {
            for (long n : {1L, 7L, 33L, 100L, 1024L}) {
                const size_t b = fmm_workspace_bytes(n, n + 1, n + 2, 3, (fmm_dtype)dt, &o);
                EXPECT(b > 0 && b % 256 == 0);
                // one byte short: FMM_ENOMEM before anything is enqueued
                EXPECT(fmm_solve(n, n + 1, n + 2, 0.1, fake, (fmm_dtype)dt, (const int64_t *)fake,
                                 (const double *)fake, 3, &o, (double *)fake, nullptr, fake, b - 1,
                                 nullptr) == FMM_ENOMEM);
            }
        }
    }
    fmm_default_opts(&o);
    // invalid arguments and options
    EXPECT(fmm_workspace_bytes(0, 4, 4, 1, FMM_F64, nullptr) == 0);
    EXPECT(fmm_workspace_bytes(4, 4, 4, -1, FMM_F64, nullptr) == 0);
    EXPECT(fmm_workspace_bytes(1L << 20, 1L << 20, 1L << 20, 1, FMM_F64, nullptr) == 0);
    fmm_opts bad = o;
    bad.band_width = NAN;
    EXPECT(fmm_workspace_bytes(8, 8, 8, 1, FMM_F64, &bad) == 0);
    bad = o;
    bad.tile_edge = 12;
    EXPECT(fmm_solve(8, 8, 8, 0.1, fake, FMM_F64, nullptr, nullptr, 0, &bad, (double *)fake, nullptr, fake,
                     1 << 30, nullptr) == FMM_EINVAL);
    bad = o;
    bad.axis_scale[1] = -1.0;
    EXPECT(fmm_solve(8, 8, 8, 0.1, fake, FMM_F64, nullptr, nullptr, 0, &bad, (double *)fake, nullptr, fake,
                     1 << 30, nullptr) == FMM_EINVAL);
    EXPECT(fmm_solve(8, 8, 8, 0.0, fake, FMM_F64, nullptr, nullptr, 0, &o, (double *)fake, nullptr, fake, 1 << 30,
                     nullptr) == FMM_EINVAL);
    EXPECT(fmm_solve(8, 8, 8, 0.1, nullptr, FMM_F64, nullptr, nullptr, 0, &o, (double *)fake, nullptr, fake,
                     1 << 30, nullptr) == FMM_EINVAL);
    EXPECT(fmm_solve(8, 8, 8, 0.1, fake, FMM_F64, nullptr, nullptr, 0, &o, (double *)fake, nullptr,
                     (char *)fake + 16, 1 << 30, nullptr) == FMM_EINVAL);
    EXPECT(fmm_solve_noalloc(200, 200, 200, 0.1, fake, FMM_F32, nullptr, nullptr, 0, &o, (double *)fake, nullptr,
                             nullptr, nullptr) == FMM_ENOMEM);
    EXPECT(fmm_solve_noalloc(8, 8, 8, 0.1, fake, (fmm_dtype)5, nullptr, nullptr, 0, &o, (double *)fake, nullptr,
                             nullptr, nullptr) == FMM_EINVAL);
    // batches: sizing adds up, invalid problems are rejected
    std::vector<fmm_problem> P(37);
    for (size_t i = 0; i < P.size(); i++) {
        memset(&P[i], 0, sizeof P[i]);
        P[i].n0 = 5 + (long)i;
        P[i].n1 = 9 + 2 * (long)i;
        P[i].n2 = 3 + 3 * (long)i;
        P[i].h = 0.01;
        P[i].F = fake;
        P[i].T_out = (double *)fake;
        P[i].n_seeds = (long)(i % 3);
        P[i].seed_idx = (const int64_t *)fake;
        P[i].seed_val = (const double *)fake;
    }
    const size_t bb = fmm_batch_workspace_bytes((long)P.size(), P.data(), FMM_F32, &o);
    EXPECT(bb > 0);
    EXPECT(fmm_solve_batch((long)P.size(), P.data(), FMM_F32, &o, fake, bb - 256, nullptr) == FMM_ENOMEM);
    P[20].h = -1.0;
    EXPECT(fmm_solve_batch((long)P.size(), P.data(), FMM_F32, &o, fake, bb, nullptr) == FMM_EINVAL);
    int32_t edges[2] = {8, 5};
    double strides[1] = {2.0};
    fmm_opts best;
    EXPECT(fmm_tune_batch(1, P.data(), FMM_F32, &o, edges, 2, strides, 1, 1, fake, bb, nullptr, &best, nullptr) ==
           FMM_EINVAL);
    // adjoint sizing and validation
    std::vector<fmm_adjoint_problem> A(5);
    for (size_t i = 0; i < A.size(); i++) {
        memset(&A[i], 0, sizeof A[i]);
        A[i].n0 = A[i].n1 = A[i].n2 = 6 + (long)i;
        A[i].h = 0.1;
        A[i].F = fake;
        A[i].T = (const double *)fake;
        A[i].status = (const uint8_t *)fake;
        A[i].dL_dT = (const double *)fake;
        A[i].dL_dF = (double *)fake + i * 1000;
    }
    const size_t ab = fmm_adjoint_workspace_bytes((long)A.size(), A.data());
    EXPECT(ab > 0);
    EXPECT(fmm_adjoint_batch((long)A.size(), A.data(), FMM_F64, fake, ab - 1, nullptr) == FMM_ENOMEM);
    A[3].dL_dF = A[0].dL_dF;  // a shared output needs equal grids
    EXPECT(fmm_adjoint_batch((long)A.size(), A.data(), FMM_F64, fake, ab, nullptr) == FMM_EINVAL);
    for (int c = -6; c <= 1; c++) EXPECT(fmm_strerror(c) != nullptr);
    EXPECT(fmm_eval_godunov(nullptr, nullptr, nullptr, 3, nullptr) == FMM_EINVAL);
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
