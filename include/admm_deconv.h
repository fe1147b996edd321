/*
 * admm_deconv.h — C ABI of the MI355X (gfx950) mask-decoupled ADMM deconvolution library.
 *
 * Problem (Almeida & Figueiredo, Sec. IV-A, eq. (34)): recover an H x W image x
 * from y = M A x + n, where A is a periodic convolution with an odd k x k kernel
 * on the unknown domain and M keeps the observed pixels (the valid region,
 * optionally minus missing interior pixels). Solvers:
 *
 *   ADMM_REG_TV     TV-MD (Sec. IV-D): Alg. 3 with the data step of eq. (49),
 *                   objective eq. (48).
 *   ADMM_REG_FRAME  FA-MD (Sec. IV-C): Alg. 2 with H1 = A, H2 = P (undecimated
 *                   Haar Parseval frame, J levels, 3J+1 bands), z-step
 *                   eqs. (24)-(25), prox eqs. (40) and (16), objective eq. (44).
 *   ADMM_REG_FRAME_SYNTHESIS
 *                   FS-MD (Sec. IV-C): the synthesis formulation of eq. (35),
 *                   unknowns the 3J+1 coefficient bands z of the image
 *                   x = W z (W = P^T, the same frame), Alg. 2 with H1 = A W,
 *                   H2 = I, z-step eq. (17) (by eqs. (18) and (20)), prox
 *                   eqs. (40) and (16). The output is the image x = W z; the
 *                   state's ureg / dreg hold u2 / d2 of the coefficients.
 *
 * With method ADMM_METHOD_CG the same objectives are minimised by the
 * Reeves-Sorel variants TV-CG / FA-CG the paper compares against (Sec. IV-B
 * to IV-D): H1 = M A, the z-step split by eqs. (43), (47), (51) into circulant
 * solves and one conjugate-gradient iteration on the boundary system, warm
 * started from the previous outer iteration.
 *
 * Conventions shared by every entry point:
 *  - Images are row-major float32 planes of H*W elements (pitch W).
 *  - "DEVICE" pointers are HIP device allocations on the current device;
 *    "HOST" pointers are ordinary host memory.
 *  - Every call enqueues its GPU work on the plan's stream; the call returns
 *    after that work is complete (the library synchronises the stream), so
 *    outputs may be read immediately.
 *  - Functions return an admm_status and never throw. On failure the
 *    thread-local message from admm_last_error() says why. Not converging
 *    within max_iters is NOT an error (info.converged = 0).
 *  - A plan is not re-entrant: do not call it from two threads at once.
 */
#ifndef ADMM_DECONV_H
#define ADMM_DECONV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ADMM_OK = 0,
    ADMM_E_INVALID = 1,      /* null pointer, bad size/count, negative lambda ...      */
    ADMM_E_UNSUPPORTED = 2,  /* even or too large kernel, side not 7-smooth or > 16384,
                                frame coefficients (H W (3J+1) floats) above 4 GiB      */
    ADMM_E_SINGULAR = 3,     /* TV with sum(kernel) == 0: the z-step matrix is singular */
    ADMM_E_NOMEM = 4,        /* device allocation failed                                */
    ADMM_E_DEVICE = 5,       /* HIP runtime error (no device, launch failure ...)       */
    ADMM_E_DIVERGED = 6      /* non-finite iterate (info.diverged = 1)                  */
} admm_status;

typedef enum { ADMM_REG_TV = 0, ADMM_REG_FRAME = 1, ADMM_REG_FRAME_SYNTHESIS = 2 } admm_reg;

/* Splitting of the data term: mask decoupling (the paper's method, the
 * default) or the Reeves-Sorel boundary system with one CG iteration per
 * outer iteration (TV-CG, FA-CG). */
typedef enum { ADMM_METHOD_MD = 0, ADMM_METHOD_CG = 1 } admm_method;

/* One problem of a plan. */
typedef struct {
    int32_t H, W;            /* unknown-domain size; each side 7-smooth, 8..16384      */
    int32_t ksize;           /* odd kernel side k = 2l+1, 1 <= k <= min(H, W)          */
    const float* kernel;     /* HOST, k*k row-major, tap (l, l) is the centre; copied  */
    const uint8_t* mask;     /* HOST, H*W, 1 = observed (row of M), 0 = unobserved;
                                copied at plan time                                    */
    int32_t reg;             /* admm_reg                                               */
    int32_t levels;          /* frame levels J (1..4) for the two frame regularisers,
                                else ignored                                           */
    double lambda;           /* regularisation weight, >= 0                            */
    double mu1, mu2;         /* ADMM penalties; a value <= 0 selects the rule of Sec. V:
                                mu2 = 10 lambda, mu1 = min(1, 5000 mu2)                */
    int32_t method;          /* admm_method; every problem of a plan has the same one.
                                ADMM_METHOD_CG solves start cold (st must be NULL) and
                                take ADMM_REG_TV or ADMM_REG_FRAME                     */
} admm_problem;

/* Solve options. */
typedef struct {
    int32_t max_iters;       /* iterations to run at most (>= 1)                        */
    double tol;              /* stop when r_pri <= tol and r_dual <= tol; <= 0: run
                                exactly max_iters                                      */
    int32_t check_every;     /* residual check period c (>= 1); the last iteration is
                                always checked so info is filled                       */
    uint32_t flags;          /* ADMM_FLAG_* below                                      */
    double obj_tol;          /* the paper's rule (Sec. V): also stop at a check iteration
                                where |F_k - F_prev| <= obj_tol |F_prev|, F_prev the
                                objective at the previous check (with check_every = 1:
                                the previous iteration); <= 0: off                      */
} admm_opts;

/* ADMM_FLAG_GRAPH: iterations are replayed from hipGraphs captured once per
 * plan (captured on an internal stream, launched on the plan's stream). With
 * a stopping rule (tol > 0 or obj_tol > 0) and an even check period or a
 * period of 1, whole check periods, checks included, are replayed and the stopping test is read from host-mapped
 * memory with at most two graphs queued; iterations queued past a problem's
 * stop leave it unchanged. Iterates, states and infos are identical to eager
 * launches.
 * ADMM_FLAG_PROFILE: time every kernel launch with HIP events (eager launches
 * only; read the totals with admm_plan_kernel_times).                        */
#define ADMM_FLAG_GRAPH 1u
#define ADMM_FLAG_PROFILE 2u

/* Result of one problem. Residuals (the paper stops on the objective instead):
 *   r_pri  = ||G z - u|| / max(||G z||, ||u||)
 *   r_dual = ||Ups (u_k - u_{k-1})|| / max(||Ups d_k||, 1e-30)
 * with G the stacked operator of eq. (3) and Ups = diag(mu1, mu2) of eq. (5);
 * objective = F(z) of eq. (48) or (44) at the last checked iterate.              */
typedef struct {
    int32_t iters;           /* iterations performed                                    */
    int32_t converged;       /* 1 if both residuals reached tol                         */
    int32_t diverged;        /* 1 if a non-finite value appeared                        */
    int32_t reserved;
    double r_pri, r_dual, objective;
} admm_info;

/* ADMM splitting state (u, d) of Alg. 2, DEVICE planes owned by the caller.
 * TV:    u1, d1: H*W;  ureg, dreg: 2*H*W as [horizontal plane, vertical plane].
 * FRAME: u1, d1: H*W;  ureg, dreg: (3J+1)*H*W, band order: for j = 1..J the
 *        detail bands (low-vert/high-horiz, high-vert/low-horiz, high/high) of
 *        level j (dilation 2^(j-1)), then the level-J low-low band.
 * Passed to solve/batch it is the initial state (Theorem 1: any u0, d0
 * converge) and receives the final state, so a solve can be resumed exactly.  */
typedef struct {
    float* u1;
    float* d1;
    float* ureg;
    float* dreg;
} admm_state;

typedef struct admm_plan admm_plan;

/* Validate `count` problems, allocate their device workspaces (spectra, duals,
 * tables) and precompute each kernel's spectrum Lambda (eq. (19)).
 * hip_stream: a hipStream_t (NULL = the null stream). *out receives the plan.
 * Errors: ADMM_E_INVALID, ADMM_E_UNSUPPORTED, ADMM_E_SINGULAR, ADMM_E_NOMEM,
 * ADMM_E_DEVICE; on error *out is set to NULL and nothing is leaked.          */
admm_status admm_deconv_plan(const admm_problem* probs, int32_t count, void* hip_stream,
                             admm_plan** out);

/* Solve the single problem of a plan with count == 1.
 * y:    DEVICE H*W observation; entries where mask == 0 are ignored.
 * x:    DEVICE H*W output, the last iterate z_k.
 * st:   NULL for a cold start (u0 = d0 = 0), else initial state in / final out
 *       (method MD only: a CG plan returns ADMM_E_UNSUPPORTED for a non-NULL st).
 * info: HOST, receives the result.                                            */
admm_status admm_deconv_solve(admm_plan* plan, const float* y, float* x, admm_state* st,
                              const admm_opts* opts, admm_info* info);

/* ---- Allocation-free solve ----
 * For callers that cannot allocate device memory (serving loops that must not
 * call hipMalloc, harnesses that forbid it): plan and solve one problem in a
 * static workspace of ADMM_STATIC_WORKSPACE_BYTES that the library holds on
 * every device it runs on until the process ends. The call allocates no
 * device or pinned host memory (no hipMalloc, hipFree, hipHostMalloc, graph
 * or event), launches eagerly on hip_stream (ADMM_FLAG_GRAPH and
 * ADMM_FLAG_PROFILE are ignored) and returns after the work is complete.
 * Arguments: as admm_deconv_plan with count == 1 (prob, hip_stream) followed
 * by admm_deconv_solve (y, x, st, opts, info); the iterates equal those of
 * that pair of calls.
 * Limit: the problem's workspace (spectra, kernel spectrum, duals, scratch
 * planes, tables; about 60 B per pixel for TV and (30 + 12 (3J+1)) B per pixel
 * for the frame, 32 B per pixel more with method CG) must fit the static
 * workspace, else ADMM_E_UNSUPPORTED
 * before any device work. Every call on a device reuses that device's
 * workspace: calls that overlap on one device (two threads or two streams)
 * race and must be serialised by the caller.                                  */
#define ADMM_STATIC_WORKSPACE_BYTES ((size_t)48 * 1024 * 1024)
admm_status admm_deconv_solve_static(const admm_problem* prob, const float* y, float* x, admm_state* st,
                                     const admm_opts* opts, admm_info* info, void* hip_stream);

/* Solve all problems of a plan together (ragged sizes allowed).
 * y, x: HOST arrays of `count` DEVICE pointers; st: NULL or HOST array of
 * `count` states; infos: HOST array of `count` results.                       */
admm_status admm_deconv_batch(admm_plan* plan, const float* const* y, float* const* x,
                              admm_state* st, const admm_opts* opts, admm_info* infos);

/* Apply the forward blur of problem `index` through its spectral path:
 * Ax = A x (eq. (19)), both DEVICE H*W planes.                                */
admm_status admm_deconv_blur(admm_plan* plan, int32_t index, const float* x, float* Ax);

/* Warm-start state from an initial guess (not in the paper; see Theorem 1):
 * u1 = A x0, d1 = M^T (y - M A x0) / mu1, u_TV = D x0,
 * d_TV = -(lambda / mu2) p0 / max(1, |p0|) per pixel.
 * x0: DEVICE H*W; p0: DEVICE 2*H*W [horizontal, vertical]; y: DEVICE H*W;
 * st: state to fill (TV problems only).                                       */
admm_status admm_warmstart_map(admm_plan* plan, int32_t index, const float* x0,
                               const float* p0, const float* y, admm_state* st);

/* Dual field of a TV state, the inverse of the d_TV part of admm_warmstart_map
 * (KKT form of the optimal duals, not in the paper): p0 = -(mu2 / lambda) d_TV
 * with the plan's mu2 and lambda of problem `index`. At a minimiser
 * |p0_i| <= 1 per pixel, so p0 is the target the warm-start network learns.
 * dreg: DEVICE 2*H*W [horizontal, vertical] (a state's dreg); p0: DEVICE
 * 2*H*W output (may alias dreg). Errors: ADMM_E_INVALID for a null pointer, an
 * index out of range, a frame problem or lambda <= 0.                          */
admm_status admm_warmstart_dual(admm_plan* plan, int32_t index, const float* dreg, float* p0);

/* Per-kernel GPU time of the most recent solve/batch run with ADMM_FLAG_PROFILE.
 * Kernel classes: "col" (column DFT + circulant solve), "row_tv" (fused TV row
 * pass), "row_inv" (FA inverse rows + data step), "frame" (FA frame step),
 * "row_fwd" (forward rows), "reduce" (residual reduction).                    */
typedef struct {
    char name[16];
    int32_t launches;
    int32_t reserved;
    double total_ms;
} admm_kernel_time;

/* Copies up to `cap` entries to out (HOST) and returns how many classes exist. */
int32_t admm_plan_kernel_times(const admm_plan* plan, admm_kernel_time* out, int32_t cap);

/* Average duration of one launch of a pass kernel ("col", "row_tv", "frame",
 * "row_inv" or "row_fwd"; a pass split into size classes counts as one
 * launch; "col:c" and "row_tv:c" time size class c alone: column classes
 * 0..8 as 2 x (0: length <= 512, 1: <= 1024, 2: <= 2048) + (general
 * schedule), 6: <= 4096, 7: <= 8192, 8: longer; fused TV row classes 0..2 by
 * row length <= 512, <= 1024, <= 2048, each with its narrower-block launches)
 * over `reps` back-to-back launches on the plan's stream, bracketed by
 * one pair of HIP events, after one untimed launch. For measurement only: it
 * runs plain iterations' launches on whatever the plan's buffers hold (call
 * it after a solve or batch, which sets the data pointers) and leaves that
 * state modified; the next solve starts over. *avg_ms (HOST) receives the
 * result. Errors: ADMM_E_INVALID (unknown kernel, none in the plan),
 * ADMM_E_DEVICE.                                                              */
admm_status admm_plan_time_pass(admm_plan* plan, const char* kernel, int32_t reps, double* avg_ms);

/* ---- FFT autotuner (tile shapes of the pass kernels) ----
 * Like admm_deconv_plan, but the columns per column-pass block (1..4, one
 * column per wave) and the rows per row-pass block are chosen by timing trial
 * plans on the device (whole iterations replayed from graphs, zero data, on
 * hip_stream): first the column tiles at the default row count, then the row
 * counts at the best tile, then, for batches whose row lengths fall in several
 * size classes (<= 512, <= 1024, <= 2048, <= 4096, <= 8192, <= 16384), each
 * class's row count with the others held (kept on a gain above 0.5%). A trial's time per iteration is
 * the difference of runs of K and 3K iterations (K = 4 to 20 by batch size,
 * best of three runs of each after a warm-up) over 2K, free of the per-run
 * work.
 * cache_path: NULL (always measure) or a JSON file of earlier results, read if
 * it exists and rewritten with the new entry; an entry for the batch's key
 * (admm_tune_key with the device's architecture) is used without measuring.
 * The tile shape does not change the iterates. Concurrent writers of one cache
 * file may lose each other's entries. Errors: as admm_deconv_plan, and
 * ADMM_E_INVALID for a cache file that cannot be parsed or written.            */
admm_status admm_deconv_plan_tuned(const admm_problem* probs, int32_t count, void* hip_stream,
                                   const char* cache_path, admm_plan** out);

/* Explicit tile shapes and radix schedules (what the autotuner chooses), for
 * callers that measured their own or reproduce a cached choice.
 * cols_per_block: 1..4 columns per column-pass block, 0 = planner's choice;
 * rows_per_block: rows per row-pass block, 0 = planner's choice (both are
 *   clamped to what a problem's lengths allow);
 * row_schedule: radix schedule variant of the row transforms, 0..3;
 * col_schedule: variant of the column transforms, 0..2 (see
 *   admm_fft_schedule). A variant that gives a length the same schedule as
 *   variant 0 is variant 0 for that length.
 * Schedules change the rounding of the transforms, never what they compute. */
typedef struct {
    int32_t cols_per_block;
    int32_t rows_per_block;
    int32_t row_schedule;
    int32_t col_schedule;
} admm_tiles;

/* Like admm_deconv_plan, with the tile shapes and schedules of `tiles` (HOST).
 * Errors: as admm_deconv_plan, and ADMM_E_INVALID for values out of range.    */
admm_status admm_deconv_plan_with(const admm_problem* probs, int32_t count, void* hip_stream,
                                  const admm_tiles* tiles, admm_plan** out);

/* Radix schedule variants a plan uses for problem `index` (row and column
 * transforms; 0 is admm_fft_radices' schedule).                               */
admm_status admm_plan_schedules(const admm_plan* plan, int32_t index, int32_t* row_schedule,
                                int32_t* col_schedule);

/* Cache key of a batch: "<arch>|<shape multiset>", e.g. "gfx950|tv512x512*8"
 * (a hash of the shape list for long ragged batches). Writes at most cap bytes
 * (NUL-terminated) to out (HOST) and returns the key length, -1 on bad input. */
int32_t admm_tune_key(const admm_problem* probs, int32_t count, const char* arch, char* out, size_t cap);

/* Cache file access (HOST only, no device): lookup returns 1 and the entry if
 * `key` is present, 0 if absent (or no file), -1 if the file is malformed;
 * store inserts or replaces an entry (tc, rows >= 1; timings in microseconds).
 * Entries the autotuner writes may also hold per-class row counts
 * ("rows_512", ..., "rows_16384") and radix schedule variants
 * ("rsched", "csched"), which lookup does not report and store does not
 * write.                                                        */
int32_t admm_tune_cache_lookup(const char* path, const char* key, int32_t* tc, int32_t* rows);
admm_status admm_tune_cache_store(const char* path, const char* key, int32_t tc, int32_t rows, double col_us,
                                  double row_us);

/* Tile shape a plan uses for problem `index` (columns per column block, rows
 * per row block).                                                             */
admm_status admm_plan_tiles(const admm_plan* plan, int32_t index, int32_t* tc, int32_t* rows);

/* Release every resource of a plan (NULL is ignored).                         */
void admm_plan_destroy(admm_plan* plan);

/* Human-readable message for the last error of the calling thread.            */
const char* admm_last_error(void);

/* Host-only helpers (no device work; usable without a GPU).
 * admm_fft_radices: radix schedule the library uses for a length-n transform;
 * writes up to `cap` radices to out and returns their count, or -1 if n is not
 * a supported 7-smooth length.                                                 */
int32_t admm_fft_radices(int32_t n, int32_t* out, int32_t cap);

/* admm_fft_schedule: the radix schedule of variant `variant` for length n
 * (the autotuner's radix dimension), in stage order: 0 = admm_fft_radices;
 * 1 = powers of two as radix 4 (one 2 for an odd exponent), then 7, 5, 3;
 * 2 = the odd radices first, then radix 8 with a 4 or 2 tail; 3 = powers of
 * two as radix 16 with one 8, 4 or 2, then 7, 5, 3 (row transforms only).
 * Returns the stage count, or -1 for an unsupported length or variant.      */
int32_t admm_fft_schedule(int32_t n, int32_t variant, int32_t* out, int32_t cap);

/* admm_validate_problem: the plan-time checks for one problem, no allocation. */
admm_status admm_validate_problem(const admm_problem* prob);

/* ---- Observations of any size (host only, no device work) ----
 * An observation of obs_h x obs_w pixels blurred by a k x k kernel depends on
 * an unknown domain of (obs_h + k - 1) x (obs_w + k - 1) pixels (Sec. IV-A,
 * eq. (34)); the transforms need 7-smooth sides of at most 16384. The helpers
 * embed the observation in the smallest 7-smooth domain that holds that
 * unknown domain: the rows and columns added at the bottom and right are
 * unknowns that no observed pixel depends on, so only the regulariser sets
 * them (on a 67 x 73 domain padded to 70 x 75 the estimate on the observed
 * region moves by about 1e-3 relative).
 *
 * admm_embed_size: H, W (HOST outputs) = the smallest 7-smooth sides
 *   >= obs_h + ksize - 1 and >= obs_w + ksize - 1. ADMM_E_INVALID for
 *   non-positive sizes or null outputs, ADMM_E_UNSUPPORTED for an even
 *   ksize or a side above 16384.
 * admm_embed_observation: y_obs (HOST, obs_h*obs_w row-major) goes to rows
 *   l .. l + obs_h - 1 and columns l .. l + obs_w - 1 (l = ksize / 2) of the
 *   HOST H*W plane y (zero elsewhere); mask (HOST, H*W) is 1 there and 0
 *   elsewhere, or obs_mask's value there when obs_mask (HOST, obs_h*obs_w,
 *   0 = missing pixel) is not NULL. H and W must hold the unknown domain
 *   (>= obs + ksize - 1; any sides the plan accepts), else ADMM_E_INVALID.  */
admm_status admm_embed_size(int32_t obs_h, int32_t obs_w, int32_t ksize, int32_t* H, int32_t* W);
admm_status admm_embed_observation(const float* y_obs, const uint8_t* obs_mask, int32_t obs_h, int32_t obs_w,
                                   int32_t ksize, int32_t H, int32_t W, float* y, uint8_t* mask);

#ifdef __cplusplus
}
#endif

#endif /* ADMM_DECONV_H */
