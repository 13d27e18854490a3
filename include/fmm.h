/*
 * fmm.h -- C ABI of the MI355X restarted narrow-band fast marching solver.
 *
 * Solves the Eikonal equation |grad T| F = 1 (Sec. 2.1, Eq. 1) on a uniform
 * n0 x n1 x n2 node grid with spacing h, using the first-order Godunov upwind
 * scheme (Eqs. 2-3) and the restarted narrow band method of Yang & Stern
 * (Sec. 4, Alg. 8-16): tiles of the grid play the paper's subdomains, a
 * device-wide minimum sets the band bound of each restart (Alg. 16), tiles
 * march their own narrow band (Alg. 12 with Alg. 10/11) and exchange updated
 * overlap values through HBM (Alg. 13-15).  All arithmetic is FP64.
 *
 * Layout: every grid array is C-contiguous (n0, n1, n2), axis 2 fastest; the
 * linear index of point (i0, i1, i2) is (i0 * n1 + i1) * n2 + i2.
 *
 * Pointers: unless stated otherwise all array arguments are DEVICE pointers
 * (memory of the current HIP device).  The caller owns every buffer; the
 * library allocates no device memory.  `stream` is a hipStream_t passed as
 * void* (NULL = the default stream); calls are asynchronous and ordered on it.
 *
 * Threading: calls on different streams with different workspaces are
 * independent.  Two calls that share a workspace must be ordered by the caller.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes.  Host-detectable argument errors are reported synchronously;
 * errors found on the device are recorded in the workspace and reported by
 * fmm_get_stats(). */
typedef enum {
    FMM_OK = 0,
    FMM_EINVAL = -1,  /* bad argument (dims, h, pointer, dtype, option)            */
    FMM_ENOMEM = -2,  /* workspace smaller than fmm_workspace_bytes()            */
    FMM_EHIP = -3,    /* a HIP runtime call or kernel launch failed              */
    FMM_ENOCONV = -4, /* restart limit reached before the band was complete      */
    FMM_EDEVICE = -5  /* device-detected input error (seeds, speed) or abort     */
} fmm_status;

/* Storage type of the speed array F (the arithmetic is FP64 either way).
 * The last enumerator only widens the type's range to every int, so that an
 * invalid value a caller passes is a defined value the library can reject
 * (FMM_EINVAL) rather than undefined behaviour in C++. */
typedef enum { FMM_F32 = 0, FMM_F64 = 1, FMM_DTYPE_RANGE_ = 0x7fffffff } fmm_dtype;

/* Option flags. */
#define FMM_VALIDATE 1u /* check on the device that every F value is finite */
#define FMM_TIMING 2u   /* record HIP events around each stage; fmm_get_stats reports them */
/* Run one march per restart instead of Alg. 16's two: tiles whose halo
 * received new values are marched in the next restart rather than in a
 * second march after the exchange.  Same result; different cost balance. */
#define FMM_ONE_MARCH 4u

/* Device error bits (fmm_stats.device_error). */
#define FMM_DERR_SEED_RANGE 1u  /* a seed index outside [0, n0*n1*n2)       */
#define FMM_DERR_SEED_DUP 2u    /* the same index given twice               */
#define FMM_DERR_SEED_VALUE 4u  /* a non-finite seed value                  */
#define FMM_DERR_SPEED 8u       /* non-finite F (only with FMM_VALIDATE)    */
#define FMM_DERR_NOCONV 16u     /* max_restarts exceeded                    */
#define FMM_DERR_BARRIER 32u    /* device-wide barrier timed out (abort)    */
#define FMM_DERR_ROUNDS 64u     /* a tile relaxation exceeded its round cap */
#define FMM_DERR_LAUNCH 128u    /* the restart driver could not be launched */
#define FMM_DERR_TIMEOUT 256u   /* the restart driver exceeded opts.time_limit_s */

typedef struct {
    /* Accept a point iff |T| <= band_width (Alg. 12 pops while |T| <= bound;
     * the paper's width_band).  INFINITY marches the whole domain. */
    double band_width;
    /* Restart stride delta-s in world units (Alg. 16: bound = min(minval +
     * stride, band_width)).  INFINITY lets every tile march to an empty
     * band in each restart; a value <= 0 selects 2h, the paper's
     * recommended stride (Sec. 5.5). */
    double stride;
    /* Step of the ordered relaxation inside a tile march, in world units: a
     * cell becomes a source of its tile once its value is within `inner` of
     * the tile's smallest pending band value (an implementation parameter,
     * not one of the paper's).  INFINITY relaxes the whole band of the
     * restart at once; a value <= 0 selects INFINITY (fastest measured). */
    double inner_stride;
    /* Edge of the cubic grid tiles that play the subdomains: 4, 8 or 16;
     * 0 selects 8. */
    int32_t tile_edge;
    /* Upper bound on restarts (0 = no practical limit); exceeding it stops
     * the solve with FMM_ENOCONV. */
    int32_t max_restarts;
    uint32_t flags; /* FMM_VALIDATE */
    /* Wall-clock limit of the restart driver in seconds (0 selects 300); a
     * solve that exceeds it stops with FMM_DERR_TIMEOUT. */
    uint32_t time_limit_s;
    /* Restart stride in units of each problem's own h; a value > 0 takes
     * precedence over `stride` (useful for a batch whose problems have
     * different spacings). */
    double stride_h;
    /* Per-axis grid spacing factors: the spacing along axis a is
     * h * axis_scale[a] (the paper's Delta x, Delta y, Delta z, Sec. 2.1).
     * 0 means 1; all 1 is the uniform grid.  The local solver then solves
     * sum_a max(u - a_a, 0)^2 / axis_scale[a]^2 = (h / F)^2. */
    double axis_scale[3];
} fmm_opts;

typedef struct {
    int64_t n_accepted;     /* accepted non-seed points (|T| <= band_width)       */
    int64_t n_restarts;     /* entries of the restart loop incl. the exiting one  */
    int64_t n_reopened;     /* values lowered after they had been accepted        */
    int64_t n_tile_marches; /* tile activations (Alg. 12 calls on a subdomain)    */
    int64_t n_solves;       /* local solver evaluations                           */
    int64_t n_rounds;       /* relaxation rounds summed over tile activations     */
    double max_abs_T;       /* max |T| over accepted points and seeds             */
    uint32_t device_error;  /* FMM_DERR_* bits                                     */
    uint32_t tile_edge;     /* tile edge actually used                             */
    int64_t n_workgroups;   /* persistent workgroups of the restart driver        */
    /* With FMM_TIMING: milliseconds of the preparation kernels (workspace
     * reset, T = +inf, seeds), of the restart driver and of the finalize
     * kernel, from HIP events on the solve's stream; -1 otherwise. */
    double ms_prepare, ms_driver, ms_finalize;
} fmm_stats;

/* Fill *opts with the defaults: band_width = INFINITY, stride = 2h (<= 0),
 * tile_edge = 8, max_restarts = 0, flags = 0, time_limit_s = 0 (300 s),
 * stride_h = 0 (unused), axis_scale = {0, 0, 0} (uniform grid). */
void fmm_default_opts(fmm_opts *opts);

/* Bytes of device workspace fmm_solve() needs for this problem (0 if the
 * arguments are invalid).  `opts` may be NULL for the defaults.  The
 * workspace holds tiled working copies of T and F, so it is about
 * (8 + sizeof(F)) bytes per grid point plus the per-tile bookkeeping. */
size_t fmm_workspace_bytes(int64_t n0, int64_t n1, int64_t n2, int64_t n_seeds, fmm_dtype F_dtype,
                           const fmm_opts *opts);

/* Solve.  Inputs (device):
 *   F         n0*n1*n2 speeds of type F_dtype; F <= 0 (or NaN) marks an
 *             impassable point that is never solved (cf. case 6, Eq. 16).
 *   seed_idx  n_seeds distinct linear indices of the points adjacent to the
 *             interface (Alg. 1/8: the KNOWN_FIX points), may be NULL if
 *             n_seeds == 0.
 *   seed_val  their values; the sign selects the side (value < 0 is the
 *             negative side; +0 and -0 are positive).  Both sides march in
 *             one pass (Sec. 3); the two sides must be separated by the seeds.
 * Outputs (device), written once by the last kernel of the solve:
 *   T_out       n0*n1*n2 FP64; accepted points and seeds hold their signed
 *               values (seeds verbatim), all other points +INFINITY.
 *   status_out  n0*n1*n2 bytes or NULL: bits 0-1 FAR=0, BAND=1, ACCEPTED=2,
 *               SEED=3; bit 7 set on the negative side.
 * Workspace: device memory of at least fmm_workspace_bytes() bytes, 256-byte
 * aligned; after the call it holds the statistics read by fmm_get_stats().
 * Returns FMM_OK once all work is enqueued; device-side errors surface in
 * fmm_get_stats(). */
int fmm_solve(int64_t n0, int64_t n1, int64_t n2, double h, const void *F, fmm_dtype F_dtype,
              const int64_t *seed_idx, const double *seed_val, int64_t n_seeds, const fmm_opts *opts,
              double *T_out, uint8_t *status_out, void *workspace, size_t workspace_bytes, void *stream);

/* Synchronise `stream`, copy the statistics of the last solve that used
 * `workspace` into *out (host), and return FMM_OK, or FMM_ENOCONV /
 * FMM_EDEVICE when the device recorded an error (FMM_EINVAL for a workspace
 * no solve has used).  The stage timings of
 * FMM_TIMING belong to the last timed solve on this workspace; the events
 * are host-side objects the library keeps per workspace address. */
int fmm_get_stats(const void *workspace, fmm_stats *out, void *stream);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * fmm_solve_noalloc() is fmm_solve() without the workspace arguments.  Its
 * workspace is a fixed device array of FMM_NOALLOC_MAX_BYTES bytes inside the
 * library: every GPU the library's code is loaded onto holds one copy until
 * the process ends.  The call allocates nothing (no hipMalloc, no host
 * containers, no events); the caller passes inputs and outputs as for
 * fmm_solve().
 *   - A problem whose fmm_workspace_bytes() exceeds FMM_NOALLOC_MAX_BYTES is
 *     rejected with FMM_ENOMEM before anything is enqueued: with 8^3 tiles
 *     the largest cubes that fit are 160^3 (FP32 speeds, about 14.4 bytes
 *     per point) and 152^3 (FP64 speeds, about 18.4 bytes per point).
 *   - error_out (device pointer, may be NULL) receives, in stream order after
 *     the solve, the FMM_DERR_* bits of this solve (0 when it succeeded).
 *     fmm_get_stats() does not apply to this entry point.
 *   - FMM_TIMING is ignored.
 *   - All calls on one GPU share that GPU's array and it keeps the last
 *     call's contents (each solve resets what it reads).  Calls that overlap
 *     in time on one GPU (different streams, different host threads) race
 *     and give undefined results: the caller must order them, e.g. on one
 *     stream.
 * Returns the host-detectable codes of fmm_solve() (FMM_EINVAL, FMM_ENOMEM,
 * FMM_EHIP) or FMM_OK once the work is enqueued.
 * ------------------------------------------------------------------------ */
#define FMM_NOALLOC_MAX_BYTES (64u << 20)
int fmm_solve_noalloc(int64_t n0, int64_t n1, int64_t n2, double h, const void *F, fmm_dtype F_dtype,
                      const int64_t *seed_idx, const double *seed_val, int64_t n_seeds, const fmm_opts *opts,
                      double *T_out, uint8_t *status_out, uint32_t *error_out, void *stream);

/* The local solver on the device (Alg. 11, Eqs. 2-7): out[i] = G(a[3i],
 * a[3i+1], a[3i+2], r[i]) for i < n, where a holds per-axis upwind values
 * (+INFINITY for an axis without one) and r = h / F.  All device pointers. */
int fmm_eval_godunov(const double *a, const double *r, double *out, int64_t n, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many independent problems in one persistent launch.
 *
 * The problems may differ in grid size, spacing, speeds and seeds; they share
 * the speed storage type and the options.  Their tiles are numbered
 * consecutively and march from one shared work list, while every problem
 * runs its own restart loop (Alg. 16): its own band minimum, bound and exit
 * test, so a finished problem drops out and a slow one does not hold back
 * the others' bounds.  The launch sequence contains kernels only (no host
 * copies or memsets), so it can be captured into a HIP graph and replayed;
 * a replay reads the problems' current F and seed arrays from the same
 * addresses.
 * ------------------------------------------------------------------------ */

/* One problem of a batch.  The struct itself lives in host memory; the
 * pointers it holds are device pointers with the meaning and layout of the
 * fmm_solve() arguments of the same names. */
typedef struct {
    int64_t n0, n1, n2;
    double h;
    const void *F;
    const int64_t *seed_idx;
    const double *seed_val;
    int64_t n_seeds;
    double *T_out;
    uint8_t *status_out; /* may be NULL */
} fmm_problem;

/* Bytes of device workspace for the batch (0 if invalid).  Only the sizes in
 * `problems` are read.  At most 2^20 problems and 2^32 - 16 tiles in all. */
size_t fmm_batch_workspace_bytes(int64_t n_problems, const fmm_problem *problems, fmm_dtype F_dtype,
                                 const fmm_opts *opts);

/* Solve every problem of the batch (asynchronous on `stream`).  Each
 * problem's outputs follow the fmm_solve() conventions and are identical to
 * what fmm_solve() returns for that problem alone with the same options (up
 * to rounding-order differences that the per-point solver cannot see: the
 * accepted set and every value agree with a single solve to the tolerance
 * the parity tests state).  Returns FMM_EINVAL for an invalid problem or
 * option, FMM_ENOMEM for a small workspace. */
int fmm_solve_batch(int64_t n_problems, const fmm_problem *problems, fmm_dtype F_dtype, const fmm_opts *opts,
                    void *workspace, size_t workspace_bytes, void *stream);

/* Synchronise `stream` and copy per-problem statistics of the last batch
 * solved in `workspace` into out[0 .. n_problems) (host).  n_accepted,
 * n_restarts (restarts of that problem's own loop) and max_abs_T are per
 * problem; the counters of tile work, device_error, tile_edge,
 * n_workgroups and the stage timings are those of the whole batch.  Return
 * codes as fmm_get_stats(). */
int fmm_get_batch_stats(const void *workspace, int64_t n_problems, fmm_stats *out, void *stream);

/* Autotuner: solve the batch once untimed and `reps` times timed (HIP
 * events on `stream`, minimum taken) for every pair of tile edge in
 * edges[0 .. n_edges) and stride (in units of each problem's h) in
 * strides_h[0 .. n_strides), then return in *best a copy of *opts (NULL:
 * defaults) with the fastest tile_edge and stride_h.  ms_out (host, may be
 * NULL) receives n_edges * n_strides times, edge-major, -1 for a pair whose
 * solve failed.  The workspace must hold the largest candidate
 * (fmm_batch_workspace_bytes() for each edge).  Synchronises `stream`; the
 * problems' outputs hold the last candidate's solution afterwards. */
int fmm_tune_batch(int64_t n_problems, const fmm_problem *problems, fmm_dtype F_dtype, const fmm_opts *opts,
                   const int32_t *edges, int32_t n_edges, const double *strides_h, int32_t n_strides, int32_t reps,
                   void *workspace, size_t workspace_bytes, void *stream, fmm_opts *best, float *ms_out);

/* ------------------------------------------------------------------------
 * Adjoint: the gradient of a loss L(T) with respect to the speeds.
 *
 * The paper solves the first-order Godunov system (Eqs. 2-3) and does not
 * differentiate it; this is an extension built on that discretisation.  At
 * the solution every accepted non-seed point p with F_p > 0 satisfies
 * sum_{q in U_p} (|T_p| - |T_q|)^2 = (h / F_p)^2, where U_p holds, for each
 * of the k axes whose values the local solver's root used (Alg. 11), the
 * neighbour on that axis with the smaller |T| (the lower index on a tie).
 * Seeds and points outside the accepted set are fixed.  The adjoint solves the
 * transpose of the linearised system A d|T| = B dF exactly, in reverse
 * dependency order (descending |T|), where row p of A has S_p on the diagonal
 * (S_p = sum_{q in U_p} (|T_p| - |T_q|)) and -(|T_p| - |T_q|) at q in U_p, and
 * B_p = -h^2 / F_p^3.  It returns dL/dF = B A^-T (sign(T) dL/dT), which is 0
 * at seeds, at points outside the accepted set and where F <= 0.  U_p is recomputed from the forward
 * solution, so nothing besides T and the status bytes needs to be kept.
 * Where the solution map has a kink (two neighbours of an axis with equal
 * values, or a change of k exactly at the solution) this is one of the
 * one-sided derivatives.
 * ------------------------------------------------------------------------ */

/* One adjoint problem: the forward problem's grid, spacing and speeds, its
 * solution (T_out and status_out of fmm_solve or fmm_solve_batch), the
 * gradient of the loss with respect to T (entries outside the accepted set
 * are ignored) and the output.  All pointers are device pointers, row-major
 * (n0, n1, n2).  Several problems of the same grid may pass the same dL_dF
 * pointer: their gradients are summed (e.g. many sources over one speed
 * model); distinct dL_dF arrays must not overlap. */
typedef struct {
    int64_t n0, n1, n2;
    double h;
    const void *F;
    const double *T;
    const uint8_t *status;
    const double *dL_dT;
    double *dL_dF;
    double axis_scale[3]; /* the forward solve's fmm_opts.axis_scale (0 means 1) */
} fmm_adjoint_problem;

typedef struct {
    int64_t n_points;      /* equations in the linear system (accepted non-seed points with F > 0) */
    int64_t n_levels;      /* dependency levels processed (frontiers of the reverse sweep)          */
    uint32_t device_error; /* FMM_DERR_BARRIER on a barrier timeout, else 0                          */
    uint32_t pad;
} fmm_adjoint_stats;

/* Device workspace for an adjoint batch (0 if invalid): about 29 bytes per
 * grid point of all problems. */
size_t fmm_adjoint_workspace_bytes(int64_t n_problems, const fmm_adjoint_problem *problems);

/* dL/dF of every problem of the batch (asynchronous on `stream`; each dL_dF
 * is overwritten, or summed over the problems that share it).  Returns
 * FMM_EINVAL for an invalid problem, FMM_ENOMEM for a small workspace. */
int fmm_adjoint_batch(int64_t n_problems, const fmm_adjoint_problem *problems, fmm_dtype F_dtype,
                      void *workspace, size_t workspace_bytes, void *stream);

/* Single-problem form of fmm_adjoint_batch() on a uniform grid (use the
 * batch form for per-axis spacing). */
int fmm_adjoint(int64_t n0, int64_t n1, int64_t n2, double h, const void *F, fmm_dtype F_dtype, const double *T,
                const uint8_t *status, const double *dL_dT, double *dL_dF, void *workspace, size_t workspace_bytes,
                void *stream);

/* Synchronise `stream` and read the statistics of the last adjoint run in
 * `workspace`; returns FMM_EDEVICE if the device recorded an error. */
int fmm_get_adjoint_stats(const void *workspace, fmm_adjoint_stats *out, void *stream);

/* Human-readable text for a return code. */
const char *fmm_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* FMM_H */
