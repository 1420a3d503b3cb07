/*
 * stencil.h - C ABI of the MI355X (gfx950) explicit stencil library.
 *
 * The library sweeps box and star stencils (d = 2 or 3, radius r, runtime
 * weights) over dense grids on the GPU, fusing T time steps per pass.  Two
 * kernel families compute the same operator:
 *   VALU : T sequential steps per pass, intermediates kept on chip
 *          (temporal fusion on general-purpose units);
 *   MFMA : the T-step composite kernel applied once per pass as banded
 *          (Toeplitz) matrix products on the matrix cores (kernel fusion),
 *          paying the sparsity factor S and the fusion redundancy alpha.
 * A host-side roofline model (paper, Sec. "Performance Formulation" and the
 * four-scenario analysis) predicts which family wins.
 *
 * Step operator (paper, Introduction; Sec. "Original Stencil Problem"):
 *     u'[x] = sum_{o in O} w[o] * ext(u)[x + o]
 *   O_box  = [-r, r]^d,                      K = (2r+1)^d
 *   O_star = {0} u {+-k e_i, 1 <= k <= r},   K = 2dr + 1
 *   ext(u) = u inside the grid; outside: the constant halo value h
 *            (Dirichlet, default 0) or the periodic image.
 * A run of N steps returns step^N(in), whatever T, path or batching.
 *
 * Conventions shared by every entry point
 *   - dims[] are slowest-first; grids are dense, contiguous, row-major, no
 *     halo stored.  Element type is given by the plan's dtype.
 *   - Weight vectors are float64 in canonical order:
 *       box : row-major over (o_0..o_{d-1}) in [-r,r]^d, o_{d-1} fastest
 *       star: centre, then axis 0 offsets -r..-1,+1..+r, then axis 1, ...
 *   - Device pointers are HIP device addresses; `stream` is a hipStream_t
 *     passed as void* (NULL = the default stream).
 *   - Every function that can fail returns an int status (STENCIL_OK = 0);
 *     stencil_last_error() gives a thread-local message for the last failure.
 *     Argument validation happens before any HIP call.
 */
#ifndef STENCIL_MI355_H
#define STENCIL_MI355_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- enumerations -------------------------------------------------------- */
enum stencil_shape { STENCIL_STAR = 0, STENCIL_BOX = 1 };

/* Storage type of the grids.  STENCIL_F32_BF16X3 stores float32 and runs the
 * MFMA path on bf16 hi/lo splits of data and weights (three products, lo*lo
 * dropped) with float32 accumulation. */
enum stencil_dtype {
    STENCIL_F64 = 0,
    STENCIL_F32 = 1,
    STENCIL_BF16 = 2,
    STENCIL_F16 = 3,
    STENCIL_F32_BF16X3 = 4
};

enum stencil_boundary { STENCIL_DIRICHLET = 0, STENCIL_PERIODIC = 1 };

/* STENCIL_PATH_MFMA_SPARSE: the MFMA path on 2:4 structured-sparse matrix
 * instructions (v_smfmac_f32_16x16x64, paper, Sec. "Further Acceleration with
 * Sparse Hardware"): bf16/f16 storage, d = 2, composite radius r*T <= 7; one
 * instruction covers two kernel columns of the band layout.  Never chosen by
 * STENCIL_PATH_AUTO; the autotuner may pick it. */
/* STENCIL_PATH_MFMA_SEQ: the matrix cores with sequential-step fusion: T
 * single-step band products per pass with the intermediate fields in LDS
 * (alpha = 1, halo recomputed per step; Sec. "Handling Stencils with Small
 * Radius" contrasts the two fusions); d = 2, r <= 3, T <= 4, every dtype but
 * the compensated one; exact on Dirichlet grids without a band fix-up.
 * Never chosen by STENCIL_PATH_AUTO. */
enum stencil_path {
    STENCIL_PATH_AUTO = 0,
    STENCIL_PATH_VALU = 1,
    STENCIL_PATH_MFMA = 2,
    STENCIL_PATH_MFMA_SPARSE = 3,
    STENCIL_PATH_MFMA_SEQ = 4
};

enum stencil_status {
    STENCIL_OK = 0,
    STENCIL_ERR_INVALID_ARG = 1, /* bad shape/d/r/T/dims/weights/steps/pointer */
    STENCIL_ERR_UNSUPPORTED = 2, /* dtype x path x (d, r, T) combination not built */
    STENCIL_ERR_ALIAS = 3,       /* in and out overlap */
    STENCIL_ERR_OOM = 4,         /* device or host allocation failed */
    STENCIL_ERR_HIP = 5          /* a HIP runtime call failed (message holds it) */
};

/* Options of stencil_plan_set (value is a double). */
enum stencil_option {
    STENCIL_OPT_PATH = 1,       /* stencil_path; AUTO = model prediction      */
    STENCIL_OPT_HALO_VALUE = 2, /* Dirichlet halo value h (default 0)         */
    STENCIL_OPT_TILE_ROWS = 3,  /* VALU: rows streamed per workgroup (0=auto) */
    STENCIL_OPT_T = 4           /* fusion depth T (>= 1)                      */
};

typedef struct stencil_plan_s *stencil_plan_t;

/* ---- plan ---------------------------------------------------------------- */

/* Read-only description of a plan. */
typedef struct {
    int shape, d, r, T, dtype, boundary;
    int path;          /* resolved path: STENCIL_PATH_VALU, _MFMA, _MFMA_SPARSE or _MFMA_SEQ */
    int64_t dims[3];
    int K;             /* points of the single-step pattern                   */
    int K_T;           /* non-zero points of the T-step composite kernel      */
    double alpha;      /* fusion redundancy K_T / (T K) (MFMA path)           */
    double S;          /* sparsity factor of the MFMA operand layout          */
    double gamma;      /* products per useful MAC (3 for bf16x3, else 1)      */
    double halo;       /* Dirichlet halo value                                */
    int64_t workspace_bytes; /* device memory the plan may own (upper bound) */
    double predicted_gst_valu;  /* model, GStencil/s                          */
    double predicted_gst_mfma;
    int predicted_winner;       /* -1 VALU, 0 tie, +1 MFMA                    */
    int scenario;               /* 1..4 as in the paper's four scenarios      */
    int tile_rows;              /* VALU rows (planes) streamed per workgroup,
                                   0 = chosen per launch                     */
    int T_fused;                /* steps one launch fuses in a full pass: T,
                                   or 1 where no kernel fuses T steps of this
                                   pattern and a pass runs as T one-step
                                   launches (same result, T times the
                                   traffic)                                   */
} stencil_plan_info_t;

/*
 * Create a plan for `shape`, dimensionality d (2 or 3), radius r >= 1, K
 * float64 weights (canonical order, copied: the caller may free them on
 * return), dims[d] (each >= 1; periodic needs every dim >= 2*r*T + 1 on the
 * MFMA path), fusion depth T >= 1, storage dtype and boundary.
 * The plan owns a scratch grid for ping-pong passes and the MFMA operand
 * blocks (upper bound in workspace_bytes).  Device memory is allocated on the
 * device current at the first run: the operand blocks then, the scratch grid
 * only when a run needs two or more passes (a run of steps <= T needs none).
 * Path AUTO resolves to the model's predicted winner among the paths built
 * for this combination.
 * Errors: INVALID_ARG (d not in {2,3}, r < 1, T < 1, NULL or non-finite
 * weights, dims < 1), UNSUPPORTED (no kernel for the combination; also a
 * Dirichlet MFMA plan with T > 1 whose boundary band, which kernel fusion
 * does not compute exactly, has no fused VALU kernel of the same T to redo
 * it, e.g. Box-3D1R T = 7), OOM, HIP.  On error *plan is NULL.
 */
int stencil_plan(stencil_plan_t *plan, int shape, int d, int r, const double *weights,
                 const int64_t *dims, int T, int dtype, int boundary);

/* Change an option (see enum stencil_option) before the next run.  Changing
 * PATH or T rebuilds the MFMA operand blocks.  Errors: INVALID_ARG,
 * UNSUPPORTED, OOM, HIP. */
int stencil_plan_set(stencil_plan_t plan, int option, double value);

/* Fill *out.  Errors: INVALID_ARG (NULL). */
int stencil_plan_info(stencil_plan_t plan, stencil_plan_info_t *out);

/*
 * out = step^steps(in) on `stream`.  `in` and `out` are device pointers to
 * dense grids of the plan's dims and dtype.  `in` is never written; `out` is
 * fully overwritten.  steps = 0 copies in to out.  The work is asynchronous;
 * kernel faults surface at stream synchronisation.  One run per plan may be
 * in flight (the plan's scratch grid is shared).
 * Passes: floor(steps / T) passes of T steps plus one pass of steps mod T.
 * Errors: INVALID_ARG (NULL pointers, steps < 0), ALIAS (in/out overlap),
 * HIP (launch failure).
 */
int stencil_run(stencil_plan_t plan, const void *in, void *out, int64_t steps, void *stream);

/*
 * Run n independent jobs (plans[i], ins[i] -> outs[i], steps[i] steps) as
 * batched launches on one stream: each round issues one pass of every job
 * that still has steps left, grouped by kernel variant, each group in a
 * single persistent launch whose workgroups pull tiles of all its jobs from
 * one work list.  Results equal stencil_run of each job alone, bit for bit.
 * Plans may not repeat within one call.  Errors as stencil_run; on an
 * argument error no job is started.
 */
int stencil_run_batch(int n, const stencil_plan_t *plans, const void *const *ins,
                      void *const *outs, const int64_t *steps, void *stream);

/*
 * Autotuner: choose the plan's path, fusion depth T and VALU rows per
 * workgroup.  Every runnable (path, T <= min(4, steps)) is ranked by the
 * roofline model (stencil_model_predict); the best `max_candidates` are timed
 * on `in` -> `out` (probe runs of up to two passes, HIP events on `stream`,
 * the call blocks until they finish) and the fastest is applied to the plan.
 * Results are cached per (shape, d, r, dtype, boundary, dims) for the process:
 * a later call for the same problem applies the cached choice without timing.
 * `out` is overwritten with an unspecified result; `in` is read only.
 * *best_gst (optional) receives the measured GStencil/s of the choice.
 * Errors: INVALID_ARG, ALIAS, UNSUPPORTED (nothing runnable), HIP.
 */
int stencil_plan_autotune(stencil_plan_t plan, const void *in, void *out, int64_t steps,
                          int max_candidates, void *stream, double *best_gst);

/* Size of the static device array stencil_run_noalloc uses (64 MiB). */
#define STENCIL_NOALLOC_SCRATCH_BYTES (64ll << 20)

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as stencil_run, with the same kernels, but the intermediate grid of
 * a run of two or more passes lives in a static device array of
 * STENCIL_NOALLOC_SCRATCH_BYTES held by each GPU the library runs on until the
 * process ends, and the call allocates nothing.  The caller passes `in` and
 * `out` as for stencil_run.  Every call on one GPU shares that GPU's array,
 * so calls that overlap on one GPU (other streams, other threads) race; the
 * array needs no clearing between calls.
 * Errors: INVALID_ARG (NULL pointers, steps < 0, or a run of two or more
 * passes over a grid larger than STENCIL_NOALLOC_SCRATCH_BYTES), ALIAS,
 * UNSUPPORTED (an MFMA plan whose operand fragments are not yet on the
 * current device: run it once with stencil_run there first, which uploads
 * them), HIP.
 */
int stencil_run_noalloc(stencil_plan_t plan, const void *in, void *out, int64_t steps, void *stream);

/* Release a plan and its device memory.  Call only after the stream that ran
 * it has drained.  NULL is ignored. */
void stencil_plan_destroy(stencil_plan_t plan);

/* Thread-local message of the last failure of this thread ("" if none). */
const char *stencil_last_error(void);

/* ---- host-only helpers (no GPU needed) ----------------------------------- */

/*
 * T-step composite kernel of kernel fusion (paper, Sec. "Handling Stencils
 * with Small Radius"): the T-fold full convolution of the weight pattern with
 * itself, radius R = r*T, written dense as (2R+1)^d float64 values indexed
 * by offset + R (row-major, last axis fastest) into out (caller-allocated).
 * Returns the number of non-zero displacements (K_T) in *k_t if non-NULL.
 * Errors: INVALID_ARG.
 */
int stencil_compose(int shape, int d, int r, const double *weights, int T, double *out,
                    int *k_t);

/* Hardware ceilings of the roofline model (flop/s, bytes/s). */
typedef struct {
    double BB;           /* memory bandwidth                                   */
    double PP_valu;      /* peak of the instructions the VALU path issues      */
    double PP_mfma;      /* dense matrix-core peak for the MFMA path's type    */
    double PP_mfma_sparse; /* 2:4 structured-sparse matrix-core peak           */
} stencil_hw_t;

/* MI355X datasheet ceilings for dtype's arithmetic (VALU without packed
 * FP32; MFMA dense; HBM3E 8 TB/s).  Errors: INVALID_ARG. */
int stencil_hw_default(int dtype, stencil_hw_t *out);

typedef struct {
    int shape, d, r, T;
    int dtype;       /* selects D (bytes per stored element) and gamma        */
    double S;        /* sparsity factor; <= 0 means: this library's layout    */
    double alpha;    /* redundancy factor; <= 0 means: K_T / (T K)            */
    int sparse;      /* 1: use PP_mfma_sparse for the matrix side, and (with S
                        <= 0) the S of this library's 2:4 sparse layout
                        where one exists (d = 2, 16-bit, r*T <= 7)           */
} stencil_model_in_t;

typedef struct {
    int K, K_T;
    double D, alpha, S, gamma;
    double C_valu;       /* flops per point per pass, VALU: 2 K T             */
    double C_mfma;       /* executed flops per point per pass: gamma alpha/S 2KT */
    double M;            /* bytes per point per pass: 2 D                     */
    double I_valu, I_mfma;
    double ridge_valu, ridge_mfma;
    double P_valu;       /* attainable useful flop/s, VALU                    */
    double P_mfma_raw;   /* attainable executed flop/s, MFMA                  */
    double P_mfma;       /* attainable useful flop/s, MFMA (raw * S/(gamma alpha)) */
    double gst_valu, gst_mfma; /* GStencil/s = point-steps / s / 1e9         */
    double ratio;        /* gst_mfma / gst_valu                               */
    int scenario;        /* 1 MB->MB, 2 MB->CB, 3 CB->MB, 4 CB->CB            */
    int sweet_spot;      /* alpha*gamma < S PP_mfma / PP_valu                 */
    int winner;          /* -1 VALU, 0 tie (ratio in [0.87, 1.15]), +1 MFMA    */
    /* Halo terms of this library's tilings (the paper's model omits halos and
     * attributes measured excess work to their recomputation):              */
    double halo_valu;    /* executed / useful VALU FMAs in the tile plane: the
                            ring each fused tile recomputes (r*T points per
                            side in 2D; r*(T-1) in 3D, whose input halo is
                            staged; 1 for one-step 3D passes)                 */
    double C_mfma_seq;   /* executed flops per point per pass of sequential-step
                            MFMA fusion (alpha = 1): T single-step band
                            products over step regions widened by the halo and
                            rounded up to 16 x 16 tiles (d = 2; 0 otherwise)  */
    double gst_mfma_seq; /* its GStencil/s on the roofline (0 when d = 3)     */
} stencil_model_out_t;

/*
 * Roofline prediction for both paths (paper, Sec. "Performance Formulation":
 * roofline, CUDA-core temporal fusion, Tensor-Core kernel fusion with S and
 * alpha; Sec. "Performance Comparative Analysis": speed-up ratio, four
 * scenarios, sweet spot; sparse units keep I and raise the peak).
 * hw NULL = stencil_hw_default(in->dtype).  Errors: INVALID_ARG.
 */
int stencil_model_predict(const stencil_model_in_t *in, const stencil_hw_t *hw,
                          stencil_model_out_t *out);

/*
 * Measured ceilings for the model (the call blocks; HIP events on `stream`):
 *   kind 0: HBM copy bandwidth, bytes/s, over `buf` (device, `bytes` >= 8 KiB,
 *           a multiple of 32: first half copied to the second half)
 *   kind 1: FP64 vector FMA, kind 2: FP32 scalar vector FMA (flop/s)
 *   kind 3: MFMA f64 16x16x4, kind 4: MFMA f32 16x16x4,
 *   kind 5: MFMA bf16 16x16x32 (flop/s);
 *   kind 6: FP32 FMA with a scalar-register multiplier, kind 7: FP32 FMA with
 *           vector-register operands only (flop/s); `buf` unused for kinds 1-7.
 * Errors: INVALID_ARG, OOM, HIP.
 */
int stencil_microbench(int kind, void *buf, int64_t bytes, void *stream, double *result);

/* Sparsity factor S of this library's MFMA operand layout for the T-step
 * composite of (shape, d, r) in dtype: useful MACs / executed MACs.
 * Returns a value in (0, 1], or a negative value on invalid arguments. */
double stencil_mfma_sparsity(int shape, int d, int r, int T, int dtype);

/* Whether this library has a kernel that fuses T steps of (shape, d, r) in
 * one pass of `path` (STENCIL_PATH_VALU or STENCIL_PATH_MFMA) for `dtype`.
 * Plans may ask for any T; a depth without a fused kernel runs as T passes
 * of one step (same result, T times the traffic), so callers that choose T
 * themselves (the server, autotuners) use this to keep to fused depths.
 * Host-only, thread-safe.  Returns 1 or 0; 0 also for invalid arguments. */
int stencil_kernel_available(int path, int dtype, int shape, int d, int r, int T);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL_MI355_H */
