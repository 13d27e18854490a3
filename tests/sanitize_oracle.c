/* Drives the CPU oracle through its paths (one- and two-sided marches, bands,
 * barriers, FP32 and FP64 speeds, per-axis spacing, acceptance-order logs,
 * rejected inputs, fast sweeping, the local solvers) for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer.  Exits non-zero on a
 * wrong return code; the sanitizers abort on any memory or UB error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n_accepted, n_popped, n_solves, n_reopened;
    double max_abs_T;
} oracle_stats;

int oracle_solve(int64_t n0, int64_t n1, int64_t n2, double h, const void *F, int F_is_f64, const int64_t *seed_idx,
                 const double *seed_val, int64_t n_seeds, double width, double *T, uint8_t *status, int64_t *order,
                 int64_t order_cap, oracle_stats *st_out, const double *axis_scale);
int64_t oracle_sweep(int64_t n0, int64_t n1, int64_t n2, double h, const double *F, const int64_t *seed_idx,
                     const double *seed_val, int64_t n_seeds, double *T, int64_t max_cycles);
double oracle_godunov(double x, double y, double z, double r);
double oracle_godunov_k(double x, double y, double z, double r, int *k);
double oracle_godunov_w(double x, double y, double z, double sx, double sy, double sz, double r, int *k);
void oracle_godunov_batch(const double *a, const double *r, double *out, int64_t n);

static uint64_t rng = 88172645463325252ull;
static double urand(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 9007199254740992.0;
}

static int fails = 0;
#define EXPECT(c)                                                   \
    do {                                                            \
        if (!(c)) {                                                 \
            fprintf(stderr, "line %d: expected %s\n", __LINE__, #c); \
            fails++;                                                \
        }                                                           \
    } while (0)

int main(void)
{
    const int64_t shapes[][3] = {{1, 1, 1}, {5, 1, 7}, {9, 10, 11}, {17, 13, 19}, {24, 3, 30}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; s++) {
        const int64_t n0 = shapes[s][0], n1 = shapes[s][1], n2 = shapes[s][2], N = n0 * n1 * n2;
        double *F = malloc(sizeof(double) * N), *T = malloc(sizeof(double) * N), *T2 = malloc(sizeof(double) * N);
        float *F32 = malloc(sizeof(float) * N);
        uint8_t *st = malloc(N);
        int64_t *order = malloc(sizeof(int64_t) * N);
        for (int64_t i = 0; i < N; i++) {
            F[i] = urand() < 0.07 ? 0.0 : 0.5 + 1.5 * urand();
            F32[i] = (float)F[i];
        }
        int64_t idx[3] = {0, N / 2, N - 1};
        double val[3] = {0.0, -0.05, 0.02};
        const int ns = N >= 3 ? 3 : 1;
        double scale[3] = {0.7, 1.0, 1.9};
        oracle_stats os;
        for (int variant = 0; variant < 6; variant++) {
            const double width = variant == 1 ? 0.1 : INFINITY;
            const void *Fp = variant == 2 ? (const void *)F32 : (const void *)F;
            const double *sc = variant == 3 ? scale : NULL;
            int64_t *ord = variant == 4 ? order : NULL;
            const int nseeds = variant == 5 ? 0 : ns;
            int rc = oracle_solve(n0, n1, n2, 0.1, Fp, variant != 2, idx, val, nseeds, width, T, st, ord,
                                  ord ? N : 0, &os, sc);
            EXPECT(rc == 0);
        }
        /* one-sided fast sweeping on the same grid */
        double zero = 0.0;
        int64_t one = N / 2;
        for (int64_t i = 0; i < N; i++) F[i] = F[i] > 0.0 ? F[i] : 1.0;
        EXPECT(oracle_sweep(n0, n1, n2, 0.1, F, &one, &zero, 1, T2, 1000) >= 0);
        /* rejected inputs: duplicate, out-of-range and non-finite seeds, bad sizes */
        int64_t dup[2] = {one, one};
        double dv[2] = {0.0, 0.0};
        EXPECT(oracle_solve(n0, n1, n2, 0.1, F, 1, dup, dv, 2, INFINITY, T, st, NULL, 0, &os, NULL) != 0 || N < 2);
        int64_t bad = N;
        EXPECT(oracle_solve(n0, n1, n2, 0.1, F, 1, &bad, &zero, 1, INFINITY, T, st, NULL, 0, &os, NULL) != 0);
        double nanv = NAN;
        EXPECT(oracle_solve(n0, n1, n2, 0.1, F, 1, &one, &nanv, 1, INFINITY, T, st, NULL, 0, &os, NULL) != 0);
        EXPECT(oracle_solve(0, n1, n2, 0.1, F, 1, &one, &zero, 1, INFINITY, T, st, NULL, 0, &os, NULL) != 0);
        EXPECT(oracle_solve(n0, n1, n2, -1.0, F, 1, &one, &zero, 1, INFINITY, T, st, NULL, 0, &os, NULL) != 0);
        free(F);
        free(T);
        free(T2);
        free(F32);
        free(st);
        free(order);
    }
    /* local solvers, including absent axes and ties */
    double a[3 * 64], r[64], out[64];
    for (int i = 0; i < 64; i++) {
        r[i] = 1e-3 + urand();
        for (int k = 0; k < 3; k++) a[3 * i + k] = urand() < 0.2 ? INFINITY : urand() * 5.0;
        int kk = 0;
        (void)oracle_godunov_k(a[3 * i], a[3 * i + 1], a[3 * i + 2], r[i], &kk);
        (void)oracle_godunov_w(a[3 * i], a[3 * i + 1], a[3 * i + 2], 0.5, 1.0, 2.0, r[i], &kk);
    }
    oracle_godunov_batch(a, r, out, 64);
    EXPECT(oracle_godunov(INFINITY, INFINITY, INFINITY, 1.0) == INFINITY);
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
