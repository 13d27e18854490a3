/*
 * fmm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU reference for the narrow-band fast marching
 * method of Yang & Stern, "A highly scalable massively parallel fast marching
 * method for the Eikonal equation" (J. Comp. Phys.; arXiv 1502.07303).
 *
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline load this library.  The product library never links, includes or
 * calls anything from this directory, and this file shares no code with it.
 *
 * What is computed (Sec. 2.1, Eqs. 1-3): on a uniform grid with spacing h the
 * first-order Godunov upwind discretisation of |grad T| F = 1 with T fixed at
 * the seed points.  The solve follows the paper's own "sequentialised"
 * reference (Sec. 5.2, accuracy study): Initialize_Interface_Parallel (Alg. 8),
 * Initialize_Heap_Parallel (Alg. 9), then a single March_Narrow_Band_Parallel
 * (Alg. 12) with the band bound equal to the band width, using
 * Update_Neighbors_Parallel (Alg. 10) and Solve_Quadratic_Parallel (Alg. 11).
 * On one subdomain the augmented tags reduce to FAR / BAND / KNOWN (Sec. 4.2).
 *
 * Readings of the paper that this file fixes (each is also listed in the
 * design notes of the repository):
 *  - grid: the n0 x n1 x n2 node array is the whole computational domain Xi;
 *    stencils are truncated at the array ends and no boundary condition is
 *    imposed (Sec. 4.1).
 *  - local solver: Alg. 11 (3-D, 2-D with the largest upwind value dropped,
 *    1-D; minimum of the causal roots), evaluated with the cancellation-free
 *    form documented at oracle_godunov() below.  Alg. 4 is not used (it lacks
 *    the 2-D/1-D fallback and the paper's own sequential runs used Alg. 11).
 *  - causality test is strict (u > a_k); a neighbour is upwind only if it is
 *    KNOWN-class, on the same side, and |T| strictly below the current |T|.
 *  - acceptance: a point is accepted iff |T| <= band width (Alg. 12 pops while
 *    |T| <= bound); width = +inf is the full-domain march.
 *  - side of a seed: negative iff its value < 0 (+0 and -0 are positive).
 *  - F <= 0 (or NaN) marks an impassable point: never solved, stays FAR
 *    (case 6 barriers, Eq. 16).
 *  - heap ties are broken by the linear index, so the march is deterministic.
 *  - two-sided problems are assumed to have the two sides separated by their
 *    seeds (Sec. 3); a point takes the side whose front reaches it with the
 *    smaller magnitude, exact ties going to the negative side.
 *
 * The two-sided heap of Sec. 3 is one array with negative indices; here each
 * side simply owns its own array-backed indexed binary heap (the textbook
 * indexed priority queue the paper cites), which is the same data structure
 * split in two.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)
#define ORACLE_ESEED (-5)

/* Augmented status tags (Sec. 4.2).  The OLD variants never occur in a
 * single-subdomain run but are kept so the tag tests read like Alg. 10-12. */
enum { FAR = 0, BAND_NEW = 1, BAND_OLD = 2, KNOWN_FIX = 3, KNOWN_NEW = 4, KNOWN_OLD = 5 };

/* Output status byte: bits 0-1 FAR=0 / BAND=1 / ACCEPTED=2 / SEED=3, bit 7 =
 * negative side. */
#define ST_FAR 0u
#define ST_BAND 1u
#define ST_ACCEPTED 2u
#define ST_SEED 3u
#define ST_NEG 0x80u

typedef struct {
    int64_t n_accepted; /* accepted non-seed points */
    int64_t n_popped;   /* heap pops (Locate_Min/Remove_Min pairs) */
    int64_t n_solves;   /* Solve_Quadratic_Parallel calls */
    int64_t n_reopened; /* KNOWN points re-tagged BAND_NEW by Alg. 10 */
    double max_abs_T;   /* max |T| over accepted points and seeds */
} oracle_stats;

static inline int is_known(uint8_t g) { return g == KNOWN_FIX || g == KNOWN_NEW || g == KNOWN_OLD; }
static inline int side_of(double v) { return v < 0.0 ? -1 : 1; }

/* ------------------------------------------------------------------------ */
/* Local solver: Eqs. 2-7 with the subset rule of Alg. 11.
 *
 * Inputs are the per-axis upwind values a (any order, +inf for an axis with
 * no upwind neighbour) and r = h / F.  With a1 <= a2 <= a3 the candidates are
 *   k=1: u1 = a1 + r
 *   k=2: D2 = 2 r^2 - (a2-a1)^2,                       u2 = ((a1+a2) + sqrt(D2)) * 0.5
 *   k=3: D3 = 3 r^2 - (((a2-a1)^2 + (a3-a1)^2) + (a3-a2)^2),
 *                                                        u3 = (((a1+a2)+a3) + sqrt(D3)) / 3
 * and candidate k is causal iff its discriminant is >= 0 and u_k > a_k.  The
 * result is the smallest causal candidate.  This is the paper's quadratic
 * a u^2 + b u + c = 0 of Alg. 11 divided through by 1/h^2, rewritten with the
 * identity (sum a)^2 - k sum a^2 = -sum_{i<j} (a_i - a_j)^2 so that no
 * O(T^2/h^2) terms cancel.  Every operation is written out in the order shown
 * (this file is compiled with -ffp-contract=off). */
/* The same local solve, also reporting in *k how many of the sorted upwind
 * values the returned root uses (1, 2 or 3; 0 when there is none).  Those k
 * smallest per-axis values are the point's upwind set in the linearisation
 * of the discrete equation (used by the adjoint reference). */
double oracle_godunov_k(double x, double y, double z, double r, int *k)
{
    double a1 = x, a2 = y, a3 = z, t;
    if (a1 > a2) { t = a1; a1 = a2; a2 = t; }
    if (a2 > a3) { t = a2; a2 = a3; a3 = t; }
    if (a1 > a2) { t = a1; a1 = a2; a2 = t; }
    *k = 0;
    if (!(a1 < INFINITY)) return INFINITY;
    double r2 = r * r;
    double best = a1 + r;
    *k = 1;
    if (a2 < INFINITY) {
        double d12 = a2 - a1;
        double D2 = 2.0 * r2 - d12 * d12;
        if (D2 >= 0.0) {
            double u2 = ((a1 + a2) + sqrt(D2)) * 0.5;
            if (u2 > a2 && u2 < best) { best = u2; *k = 2; }
        }
        if (a3 < INFINITY) {
            double d13 = a3 - a1, d23 = a3 - a2;
            double D3 = 3.0 * r2 - ((d12 * d12 + d13 * d13) + d23 * d23);
            if (D3 >= 0.0) {
                double u3 = (((a1 + a2) + a3) + sqrt(D3)) / 3.0;
                if (u3 > a3 && u3 < best) { best = u3; *k = 3; }
            }
        }
    }
    return best;
}

double oracle_godunov(double x, double y, double z, double r)
{
    int k;
    return oracle_godunov_k(x, y, z, r, &k);
}

/* Local solver on a grid with per-axis spacing h_i = h s_i (the paper's
 * Delta x, Delta y, Delta z, Sec. 2.1): with weights w_i = 1 / s_i^2 and
 * r = h / F the upwind equation is sum_i w_i max(u - a_i, 0)^2 = r^2.  For the
 * k smallest values (sorted together with their weights) its roots are
 *   k=1: u1 = a1 + r s1
 *   k=2: D2 = (w1+w2) r^2 - (w1 w2) (a2-a1)^2,
 *        u2 = ((w1 a1 + w2 a2) + sqrt(D2)) / (w1+w2)
 *   k=3: D3 = ((w1+w2)+w3) r^2 - (((w1 w2)(a2-a1)^2 + (w1 w3)(a3-a1)^2) + (w2 w3)(a3-a2)^2),
 *        u3 = (((w1 a1 + w2 a2) + w3 a3) + sqrt(D3)) / ((w1+w2)+w3)
 * (the identity (sum w a)^2 - (sum w)(sum w a^2) = -sum_{i<j} w_i w_j (a_i-a_j)^2
 * again removes the cancellation), with the same causality rule and minimum.
 * With all s_i = 1 every operation reduces to the one of oracle_godunov(), so
 * the two agree bit for bit. */
double oracle_godunov_w(double x, double y, double z, double sx, double sy, double sz, double r, int *k)
{
    double a[3] = {x, y, z}, sc[3] = {sx, sy, sz};
    /* sort the values, carrying each axis' scale along (stable) */
    for (int i = 1; i < 3; i++)
        for (int j = i; j > 0 && a[j - 1] > a[j]; j--) {
            double t = a[j]; a[j] = a[j - 1]; a[j - 1] = t;
            t = sc[j]; sc[j] = sc[j - 1]; sc[j - 1] = t;
        }
    double a1 = a[0], a2 = a[1], a3 = a[2];
    double w1 = 1.0 / (sc[0] * sc[0]), w2 = 1.0 / (sc[1] * sc[1]), w3 = 1.0 / (sc[2] * sc[2]);
    *k = 0;
    if (!(a1 < INFINITY)) return INFINITY;
    double r2 = r * r;
    double best = a1 + r * sc[0];
    *k = 1;
    if (a2 < INFINITY) {
        double d12 = a2 - a1;
        double D2 = (w1 + w2) * r2 - (w1 * w2) * (d12 * d12);
        if (D2 >= 0.0) {
            double u2 = ((w1 * a1 + w2 * a2) + sqrt(D2)) / (w1 + w2);
            if (u2 > a2 && u2 < best) { best = u2; *k = 2; }
        }
        if (a3 < INFINITY) {
            double d13 = a3 - a1, d23 = a3 - a2;
            double D3 = ((w1 + w2) + w3) * r2 -
                        (((w1 * w2) * (d12 * d12) + (w1 * w3) * (d13 * d13)) + (w2 * w3) * (d23 * d23));
            if (D3 >= 0.0) {
                double u3 = (((w1 * a1 + w2 * a2) + w3 * a3) + sqrt(D3)) / ((w1 + w2) + w3);
                if (u3 > a3 && u3 < best) { best = u3; *k = 3; }
            }
        }
    }
    return best;
}

/* Batch form for tests: out[i] = G(a[3i], a[3i+1], a[3i+2], r[i]). */
void oracle_godunov_batch(const double *a, const double *r, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; i++) out[i] = oracle_godunov(a[3 * i], a[3 * i + 1], a[3 * i + 2], r[i]);
}

/* ------------------------------------------------------------------------ */
/* Indexed binary min-heap keyed by (|T|, linear index). */
typedef struct {
    int64_t *a; /* point indices, 0-based heap */
    int64_t n, cap;
} heap_t;

typedef struct {
    int64_t n0, n1, n2, N;
    double h;
    const double *scale; /* per-axis spacing factors, NULL: isotropic */
    const void *F;
    int F_is_f64;
    double *T;
    uint8_t *G;
    int32_t *pos;  /* position in its side's heap, -1 if absent */
    heap_t H[2];   /* H[0] side -1, H[1] side +1 */
    oracle_stats *st;
} solver_t;

static inline int hidx(int s) { return s < 0 ? 0 : 1; }

static inline int key_less(const solver_t *S, int64_t p, int64_t q)
{
    double ap = fabs(S->T[p]), aq = fabs(S->T[q]);
    if (ap < aq) return 1;
    if (ap > aq) return 0;
    return p < q;
}

static void heap_swap(solver_t *S, heap_t *H, int64_t i, int64_t j)
{
    int64_t t = H->a[i];
    H->a[i] = H->a[j];
    H->a[j] = t;
    S->pos[H->a[i]] = (int32_t)i;
    S->pos[H->a[j]] = (int32_t)j;
}

static void up_heap(solver_t *S, heap_t *H, int64_t i)
{
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!key_less(S, H->a[i], H->a[p])) break;
        heap_swap(S, H, i, p);
        i = p;
    }
}

static void down_heap(solver_t *S, heap_t *H, int64_t i)
{
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < H->n && key_less(S, H->a[l], H->a[m])) m = l;
        if (r < H->n && key_less(S, H->a[r], H->a[m])) m = r;
        if (m == i) break;
        heap_swap(S, H, i, m);
        i = m;
    }
}

static int insert_heap(solver_t *S, heap_t *H, int64_t p)
{
    if (H->n == H->cap) {
        int64_t nc = H->cap ? 2 * H->cap : 1024;
        int64_t *na = (int64_t *)realloc(H->a, (size_t)nc * sizeof(int64_t));
        if (!na) return ORACLE_ENOMEM;
        H->a = na;
        H->cap = nc;
    }
    H->a[H->n] = p;
    S->pos[p] = (int32_t)H->n;
    H->n++;
    up_heap(S, H, H->n - 1);
    return ORACLE_OK;
}

/* Remove an arbitrary element (used by Remove_Min and by a side change). */
static void remove_at(solver_t *S, heap_t *H, int64_t i)
{
    int64_t p = H->a[i];
    H->n--;
    S->pos[p] = -1;
    if (i != H->n) {
        int64_t moved = H->a[H->n];
        H->a[i] = moved;
        S->pos[moved] = (int32_t)i;
        up_heap(S, H, i);
        down_heap(S, H, S->pos[moved]);
    }
}

/* ------------------------------------------------------------------------ */
static inline double speed_at(const solver_t *S, int64_t p)
{
    return S->F_is_f64 ? ((const double *)S->F)[p] : (double)((const float *)S->F)[p];
}

/* Solve_Quadratic_Parallel (Alg. 11) at linear index p for side s. */
static double solve_quadratic(solver_t *S, int64_t p, int s)
{
    S->st->n_solves++;
    double F = speed_at(S, p);
    if (!(F > 0.0)) return INFINITY; /* impassable */
    int64_t i0 = p / (S->n1 * S->n2), rem = p % (S->n1 * S->n2);
    int64_t i1 = rem / S->n2, i2 = rem % S->n2;
    double cur = fabs(S->T[p]);
    const int64_t coord[3] = {i0, i1, i2};
    const int64_t ext[3] = {S->n0, S->n1, S->n2};
    const int64_t stride[3] = {S->n1 * S->n2, S->n2, 1};
    double a[3];
    for (int ax = 0; ax < 3; ax++) {
        /* Check this direction: the smaller of the two KNOWN-class, same-side,
         * strictly-upwind neighbours (the "+1" neighbour wins only if it is
         * strictly smaller). */
        int d = 0;
        double best = INFINITY;
        if (coord[ax] - 1 >= 0) {
            int64_t q = p - stride[ax];
            if (is_known(S->G[q]) && side_of(S->T[q]) == s && fabs(S->T[q]) < cur) {
                d = -1;
                best = fabs(S->T[q]);
            }
        }
        if (coord[ax] + 1 < ext[ax]) {
            int64_t q = p + stride[ax];
            if (is_known(S->G[q]) && side_of(S->T[q]) == s && fabs(S->T[q]) < cur) {
                if (d == 0 || fabs(S->T[q]) < best) {
                    d = 1;
                    best = fabs(S->T[q]);
                }
            }
        }
        a[ax] = d != 0 ? best : INFINITY;
    }
    double r = S->h / F;
    if (S->scale) {
        int k;
        return oracle_godunov_w(a[0], a[1], a[2], S->scale[0], S->scale[1], S->scale[2], r, &k);
    }
    return oracle_godunov(a[0], a[1], a[2], r);
}

/* Update_Neighbors_Parallel (Alg. 10) around the point p of side s. */
static int update_neighbors(solver_t *S, int64_t p, int s)
{
    int64_t i0 = p / (S->n1 * S->n2), rem = p % (S->n1 * S->n2);
    int64_t i1 = rem / S->n2, i2 = rem % S->n2;
    const int64_t coord[3] = {i0, i1, i2};
    const int64_t ext[3] = {S->n0, S->n1, S->n2};
    const int64_t stride[3] = {S->n1 * S->n2, S->n2, 1};
    double ap = fabs(S->T[p]);
    for (int ax = 0; ax < 3; ax++) {
        for (int dir = -1; dir <= 1; dir += 2) {
            int64_t c = coord[ax] + dir;
            if (c < 0 || c >= ext[ax]) continue; /* (l,m,n) not in Xi */
            int64_t q = p + dir * stride[ax];
            if (S->G[q] == KNOWN_FIX) continue;
            double oldv = S->T[q];
            double aq = fabs(oldv);
            if (!(aq > ap)) continue;
            double u = solve_quadratic(S, q, s);
            int oside = side_of(oldv);
            int take = (u < aq) || (u == aq && s < 0 && oside > 0 && oldv < INFINITY);
            if (!take) continue;
            if (is_known(S->G[q])) S->st->n_reopened++;
            if (S->pos[q] >= 0 && oside != s) remove_at(S, &S->H[hidx(oside)], S->pos[q]);
            S->T[q] = s < 0 ? -u : u;
            S->G[q] = BAND_NEW;
            heap_t *H = &S->H[hidx(s)];
            if (S->pos[q] < 0) {
                int rc = insert_heap(S, H, q);
                if (rc) return rc;
            } else {
                up_heap(S, H, S->pos[q]);
            }
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
int oracle_solve(int64_t n0, int64_t n1, int64_t n2, double h, const void *F, int F_is_f64,
                 const int64_t *seed_idx, const double *seed_val, int64_t n_seeds, double width,
                 double *T, uint8_t *status, int64_t *order, int64_t order_cap, oracle_stats *st_out,
                 const double *axis_scale)
{
    if (n0 <= 0 || n1 <= 0 || n2 <= 0 || !(h > 0.0) || !isfinite(h) || !F || !T || n_seeds < 0 ||
        (n_seeds > 0 && (!seed_idx || !seed_val)) || isnan(width) || width < 0.0)
        return ORACLE_EINVAL;
    if (axis_scale)
        for (int ax = 0; ax < 3; ax++)
            if (!(axis_scale[ax] > 0.0) || !isfinite(axis_scale[ax])) return ORACLE_EINVAL;
    oracle_stats st_local;
    memset(&st_local, 0, sizeof st_local);
    solver_t S;
    memset(&S, 0, sizeof S);
    S.n0 = n0;
    S.n1 = n1;
    S.n2 = n2;
    S.N = n0 * n1 * n2;
    S.h = h;
    S.scale = axis_scale;
    S.F = F;
    S.F_is_f64 = F_is_f64;
    S.T = T;
    S.st = &st_local;
    S.G = (uint8_t *)malloc((size_t)S.N);
    S.pos = (int32_t *)malloc((size_t)S.N * sizeof(int32_t));
    int rc = ORACLE_OK;
    if (!S.G || !S.pos) {
        rc = ORACLE_ENOMEM;
        goto done;
    }

    /* Initialize_Interface_Parallel (Alg. 8). */
    for (int64_t p = 0; p < S.N; p++) {
        T[p] = INFINITY;
        S.G[p] = FAR;
        S.pos[p] = -1;
    }
    for (int64_t k = 0; k < n_seeds; k++) {
        int64_t p = seed_idx[k];
        if (p < 0 || p >= S.N || !isfinite(seed_val[k]) || S.G[p] == KNOWN_FIX) {
            rc = ORACLE_ESEED;
            goto done;
        }
        T[p] = seed_val[k];
        S.G[p] = KNOWN_FIX;
    }

    /* Initialize_Heap_Parallel (Alg. 9): every KNOWN_FIX point updates its
     * neighbours, in grid order. */
    for (int64_t p = 0; p < S.N; p++) {
        if (S.G[p] != KNOWN_FIX) continue;
        rc = update_neighbors(&S, p, side_of(T[p]));
        if (rc) goto done;
    }

    /* March_Narrow_Band_Parallel (Alg. 12) once, bound = width. */
    int64_t n_order = 0;
    for (int s = -1; s <= 1; s += 2) {
        heap_t *H = &S.H[hidx(s)];
        for (;;) {
            if (H->n == 0) break;
            int64_t p = H->a[0]; /* Locate_Min(s) */
            if (fabs(T[p]) > width) break;
            if (S.G[p] != KNOWN_OLD) S.G[p] = KNOWN_NEW;
            remove_at(&S, H, 0); /* Remove_Min(s) */
            st_local.n_popped++;
            if (order && n_order < order_cap) order[n_order] = p;
            n_order++;
            rc = update_neighbors(&S, p, s);
            if (rc) goto done;
        }
    }

    /* Output: accepted points and seeds keep their values, everything else is
     * +inf; the status byte records the tag and side. */
    for (int64_t p = 0; p < S.N; p++) {
        uint8_t g = S.G[p];
        double v = T[p];
        uint8_t neg = (v < 0.0) ? ST_NEG : 0u;
        uint8_t out;
        if (g == KNOWN_FIX) {
            out = ST_SEED | neg;
            if (fabs(v) > st_local.max_abs_T) st_local.max_abs_T = fabs(v);
        } else if (g == KNOWN_NEW || g == KNOWN_OLD) {
            out = ST_ACCEPTED | neg;
            st_local.n_accepted++;
            if (fabs(v) > st_local.max_abs_T) st_local.max_abs_T = fabs(v);
        } else if (g == BAND_NEW || g == BAND_OLD) {
            out = ST_BAND | neg;
            T[p] = INFINITY;
        } else {
            out = ST_FAR;
            T[p] = INFINITY;
        }
        if (status) status[p] = out;
    }

done:
    free(S.G);
    free(S.pos);
    free(S.H[0].a);
    free(S.H[1].a);
    if (st_out) *st_out = st_local;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Fast sweeping (Zhao 2005, cited in Sec. 1) -- an independent check of the
 * marcher, not part of the method.  Gauss-Seidel sweeps of the Godunov update
 * over the eight axis orderings, T_p <- min(T_p, G(neighbour minima)), until
 * a whole cycle of eight sweeps leaves every value bitwise unchanged.
 * One-sided (all seed values >= 0).  Returns the number of cycles, or < 0. */
int64_t oracle_sweep(int64_t n0, int64_t n1, int64_t n2, double h, const double *F,
                     const int64_t *seed_idx, const double *seed_val, int64_t n_seeds, double *T,
                     int64_t max_cycles)
{
    if (n0 <= 0 || n1 <= 0 || n2 <= 0 || !(h > 0.0) || !F || !T || n_seeds < 0) return ORACLE_EINVAL;
    int64_t N = n0 * n1 * n2;
    uint8_t *fixed = (uint8_t *)calloc((size_t)N, 1);
    if (!fixed) return ORACLE_ENOMEM;
    for (int64_t p = 0; p < N; p++) T[p] = INFINITY;
    for (int64_t k = 0; k < n_seeds; k++) {
        int64_t p = seed_idx[k];
        if (p < 0 || p >= N || fixed[p] || !(seed_val[k] >= 0.0)) {
            free(fixed);
            return ORACLE_ESEED;
        }
        T[p] = seed_val[k];
        fixed[p] = 1;
    }
    int64_t cycles = 0;
    for (;;) {
        int changed = 0;
        for (int o = 0; o < 8; o++) {
            int64_t s0 = (o & 1) ? -1 : 1, s1 = (o & 2) ? -1 : 1, s2 = (o & 4) ? -1 : 1;
            for (int64_t c0 = 0; c0 < n0; c0++) {
                int64_t i0 = s0 > 0 ? c0 : n0 - 1 - c0;
                for (int64_t c1 = 0; c1 < n1; c1++) {
                    int64_t i1 = s1 > 0 ? c1 : n1 - 1 - c1;
                    for (int64_t c2 = 0; c2 < n2; c2++) {
                        int64_t i2 = s2 > 0 ? c2 : n2 - 1 - c2;
                        int64_t p = (i0 * n1 + i1) * n2 + i2;
                        if (fixed[p] || !(F[p] > 0.0)) continue;
                        double ax = INFINITY, ay = INFINITY, az = INFINITY;
                        if (i0 > 0 && T[p - n1 * n2] < ax) ax = T[p - n1 * n2];
                        if (i0 + 1 < n0 && T[p + n1 * n2] < ax) ax = T[p + n1 * n2];
                        if (i1 > 0 && T[p - n2] < ay) ay = T[p - n2];
                        if (i1 + 1 < n1 && T[p + n2] < ay) ay = T[p + n2];
                        if (i2 > 0 && T[p - 1] < az) az = T[p - 1];
                        if (i2 + 1 < n2 && T[p + 1] < az) az = T[p + 1];
                        double u = oracle_godunov(ax, ay, az, h / F[p]);
                        if (u < T[p]) {
                            T[p] = u;
                            changed = 1;
                        }
                    }
                }
            }
        }
        cycles++;
        if (!changed || cycles >= max_cycles) break;
    }
    free(fixed);
    return cycles;
}
