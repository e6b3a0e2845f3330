/*
 * fe.h -- C ABI of the MI355X (gfx950) Fields-of-Experts Poisson denoiser.
 *
 * The library runs the inference scheme of Feng, Qiao & Chen, "Poisson Noise
 * Reduction with Higher-order Natural Image Prior Model", eq. 3.7:
 *
 *   v      = f_A(y) = 2 sqrt(y + 3/8)                         (eq. 2.3)
 *   u^0    = u^{-1} = v
 *   u~     = u^n - tau * grad F(u^n) + gamma * (u^n - u^{n-1}) (eq. 2.8)
 *            grad F(u) = sum_i alpha_i K_i^T rho'(K_i u),
 *            rho'(z) = 2z / (1 + z^2)                          (eq. 3.2, 2.6)
 *   u^{n+1} = prox_{tau G}(u~)                                 (eq. 2.9)
 *            quadratic G = lambda/2 |u - v|^2:
 *              (u~ + tau lambda v) / (1 + tau lambda)          (eq. 3.5)
 *            I-divergence G = lambda <u - v log u, 1>:
 *              (u~ - tau lambda + sqrt((u~ - tau lambda)^2
 *                                      + 4 tau lambda v)) / 2  (eq. 3.3, 3.6)
 *   x_hat  = I_C(u^N)                                          (eq. 2.4)
 *
 * K_i is correlation with the m x m taps k_i[a][b] at offset (a - r, b - r),
 * r = (m - 1) / 2, of the half-sample symmetric extension of the image
 * (u(-1-i) = u(i)); K_i^T is its exact transpose (ghost contributions are
 * folded back onto the pixels they mirror).  I_C is applied for
 * u >= sqrt(3/2), where it is exactly zero, and x_hat = 0 below.
 *
 * Conventions for every entry point:
 *   - every call returns fe_status; FE_OK == 0;
 *   - arguments are validated on the host before anything is enqueued; on
 *     error nothing is enqueued and fe_last_error() (thread-local) holds a
 *     message;
 *   - image buffers are row-major float32 on the device, owned by the
 *     caller; the library never frees caller memory, and the denoising
 *     calls (fe_denoise, fe_begin / fe_advance / fe_end, fe_denoise_binned,
 *     fe_energy_grad) never allocate: scratch comes from the caller's
 *     workspace.  fe_create, fe_autotune, fe_advance_graph_create and
 *     fe_server_create allocate what they document;
 *   - work is enqueued asynchronously on the caller's HIP stream
 *     (hipStream_t passed as void*, NULL = the null stream); a device fault
 *     is reported as FE_ERR_DEVICE by a later call or by the caller's own
 *     synchronisation;
 *   - debug mode: with the environment variable FE_VALIDATE=1, fe_denoise,
 *     fe_begin, fe_denoise_binned and fe_energy_grad first run a device pass
 *     over the counts and return FE_ERR_INVALID if any is negative, NaN or
 *     infinite (the pass allocates a few flags and synchronises the stream;
 *     it is skipped while the stream is being captured into a graph);
 *   - an fe_ctx may be used from several threads and streams at once, each
 *     with its own workspace; its filter bank is immutable after fe_create,
 *     its tuning table (fe_autotune, fe_tuning_load) is internally locked.
 */
#ifndef FE_H
#define FE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fe_ctx fe_ctx;

typedef int32_t fe_status;
#define FE_OK 0
#define FE_ERR_INVALID 1     /* bad argument (shape, NULL, range, workspace) */
#define FE_ERR_UNSUPPORTED 2 /* valid but not built (filter size, count)     */
#define FE_ERR_NOMEM 3       /* device allocation in fe_create failed        */
#define FE_ERR_DEVICE 4      /* HIP runtime reported an error                */

/* Data term selection (eq. 3.7). */
#define FE_DATA_AUTO 0      /* by job.peak: peak >= 5 quadratic, else I-div */
#define FE_DATA_QUADRATIC 1 /* eq. 3.4 / 3.5                                */
#define FE_DATA_IDIV 2      /* eq. 3.6 / 3.3                                */

/* Arithmetic of the filter-bank contractions (K_i u and K_i^T psi).  The
 * influence, the inertial step, the prox and I_C are FP32 in every mode. */
#define FE_PREC_FP32 0
#define FE_PREC_BF16 1 /* bf16 operands, fp32 accumulation */
#define FE_PREC_FP16 2 /* fp16 operands, fp32 accumulation; u = f_A(y) must
                          stay below the fp16 maximum 65504, y < ~1.07e9 */

/* The learned prior of eq. 2.5: N_f filters of m x m taps with weights. */
typedef struct {
    int32_t m;            /* odd filter side: 3, 5 or 7                      */
    int32_t n_filters;    /* N_f, 1..64                                      */
    const float *filters; /* HOST [n_filters][m][m] correlation taps, copied */
    const float *weights; /* HOST [n_filters] alpha_i >= 0, copied           */
} fe_prior;

/* One denoising job (one noisy image). */
typedef struct {
    int32_t height, width;  /* each >= r = (m - 1) / 2; H * W < 2^31       */
    const float *counts;    /* DEVICE H*W, y >= 0, integer valued          */
    float *out;             /* DEVICE H*W, x_hat = I_C(u_hat); may be NULL */
    float *out_anscombe;    /* DEVICE H*W, u_hat (Anscombe domain) or NULL */
    float lambda;           /* data-term weight, > 0                        */
    int32_t iterations;     /* >= 0; 0 gives x_hat = I_C(f_A(y))            */
    int32_t data_term;      /* FE_DATA_*                                    */
    float peak;             /* noise level, used only with FE_DATA_AUTO     */
    float tau;              /* iPiano step, > 0                             */
    float gamma;            /* iPiano inertia, 0 <= gamma < 1               */
    int32_t precision;      /* FE_PREC_*                                    */
} fe_job;

/* Create a context on HIP device `device`: uploads the filter bank in the
 * layouts the kernels use.  *out receives the context (NULL on error). */
fe_status fe_create(const fe_prior *prior, int device, fe_ctx **out);

/* Workspace bytes fe_denoise needs for this batch of jobs (the state
 * u^n, u^{n-1} of every job, plus the job table of the step launches). */
fe_status fe_workspace_size(const fe_ctx *ctx, const fe_job *jobs, int32_t n,
                            size_t *bytes);

/* Denoise n jobs (eq. 3.7) on `hip_stream`.  The workspace (DEVICE, at
 * least fe_workspace_size bytes, 256-byte aligned) must not be used by
 * another call until the stream has passed this one.  Every job's result
 * is written to its out / out_anscombe buffers.  Asynchronous. */
fe_status fe_denoise(const fe_ctx *ctx, const fe_job *jobs, int32_t n,
                     void *workspace, size_t ws_bytes, void *hip_stream);

/* ---- stepping interface ------------------------------------------------
 * fe_denoise is fe_begin + fe_advance + fe_end on states it carves from its
 * workspace.  Callers that keep jobs resident between calls (a serving loop
 * advancing many requests a few iterations at a time, or a checkpoint) use
 * the three calls directly.  A job's state is two caller-owned DEVICE
 * planes of H*W floats, contiguous ([2][H][W]); after `done` iterations
 * plane (done % 2) holds u^done and the other plane u^{done-1}.  The pair
 * (state, done) is the job's complete resume point. */

/* Bytes of one job's state (2 * H * W * sizeof(float)). */
fe_status fe_state_bytes(const fe_ctx *ctx, int32_t height, int32_t width,
                         size_t *bytes);

/* u^0 = u^{-1} = f_A(y) (eq. 2.3) into states[i] for every job.  Async. */
fe_status fe_begin(const fe_ctx *ctx, const fe_job *jobs, float *const *states,
                   int32_t n, void *hip_stream);

/* Workspace bytes fe_advance needs for a batch of n jobs (its job table). */
fe_status fe_advance_workspace_size(const fe_ctx *ctx, int32_t n, size_t *bytes);

/* Apply count[i] >= 0 further iPiano iterations (eq. 2.8) to job i whose
 * state holds done[i] >= 0 iterations; all jobs of the batch share the
 * step launches.  job.iterations is ignored here.  The workspace (DEVICE,
 * 256-byte aligned, fe_advance_workspace_size bytes) must not be reused
 * until the stream has passed this call.  Async. */
fe_status fe_advance(const fe_ctx *ctx, const fe_job *jobs, float *const *states,
                     const int32_t *done, const int32_t *count, int32_t n,
                     void *workspace, size_t ws_bytes, void *hip_stream);

/* ---- allocation-free stepping --------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * fe_advance with the job table of its launches in a static device array
 * owned by the library (256 KiB on every device the library runs on, held
 * until the process ends) instead of a caller workspace.  Same arguments,
 * checks and results as fe_advance (bitwise); the caller still owns the
 * jobs' counts and states.  Allocates no device memory.
 * At most FE_NOALLOC_MAX_JOBS jobs per call, else FE_ERR_INVALID.  The
 * array is shared by every call on a device and keeps the last call's
 * table: calls on one stream are ordered, but calls that overlap on one
 * device (other streams, threads or contexts) race on it, and the caller
 * must serialise them.  Async. */
#define FE_NOALLOC_MAX_JOBS 2048
fe_status fe_advance_noalloc(const fe_ctx *ctx, const fe_job *jobs, float *const *states,
                             const int32_t *done, const int32_t *count, int32_t n,
                             void *hip_stream);

/* x_hat = I_C(u^done) (eq. 2.4) into job.out, and u^done into
 * job.out_anscombe, for every job (either output may be NULL).  Async. */
fe_status fe_end(const fe_ctx *ctx, const fe_job *jobs, float *const *states,
                 const int32_t *done, int32_t n, void *hip_stream);

/* ---- tile-shape autotuning ----------------------------------------------
 * The step's tile width is fixed by its q-row width; its height, and for
 * FP32 the waves per workgroup (8: every operand in registers; 12: adjoint
 * tables in LDS), are picked per batch by a cost model and a default unless
 * this table holds a measured choice for the batch's signature (precision
 * and multiset of image sizes).  fe_autotune times up to six candidate
 * heights per wave count and precision group on scratch copies of the
 * jobs' states (allocated for the call and freed; the jobs' own buffers are
 * only read), trial_iterations (even) each, and records the fastest.
 * Synchronises the stream.  The table is internally locked; it can be saved
 * to and loaded from a text file (one "waves height key" line per entry,
 * '#' comments; a wave count the precision is not built for, or a height
 * outside 8..(the variant's LDS limit, at most 128), is rejected with
 * FE_ERR_INVALID).  The tile shape never changes results: every output
 * pixel is computed by the same arithmetic whichever tile holds it. */
fe_status fe_autotune(const fe_ctx *ctx, const fe_job *jobs, int32_t n,
                      int32_t trial_iterations, void *hip_stream);
fe_status fe_tuning_save(const fe_ctx *ctx, const char *path);
fe_status fe_tuning_load(const fe_ctx *ctx, const char *path);

/* ---- captured step sequence ---------------------------------------------
 * Captures one fe_advance (the job table upload and every step launch) into
 * a HIP graph.  Each fe_graph_launch applies count[i] iterations to job i
 * again; counts must be even so that a replay finds u^n in the plane it was
 * captured with.  States, counts buffers and the workspace are referenced,
 * not copied: keep them alive and unmodified while the graph is used.  No
 * memset nodes are captured. */
typedef struct fe_graph fe_graph;
fe_status fe_advance_graph_create(const fe_ctx *ctx, const fe_job *jobs,
                                  float *const *states, const int32_t *done,
                                  const int32_t *count, int32_t n,
                                  void *workspace, size_t ws_bytes, fe_graph **out);
fe_status fe_graph_launch(const fe_graph *graph, void *hip_stream);
void fe_graph_destroy(fe_graph *graph);

/* ---- binning variant (Section 4: 3 x 3 ones kernel, bilinear upscaling;
 * the data term follows the binned image's peak, eq. 3.7) ----------------
 * Each job's counts are summed over non-overlapping 3 x 3 blocks (the image
 * extended half-sample symmetrically to a multiple of 3), giving a
 * ceil(H/3) x ceil(W/3) image with nine times the peak; that image is
 * denoised with the job's parameters (with FE_DATA_AUTO the data term is
 * chosen for peak * 9; lambda applies to the binned problem); the result / 9
 * is placed at the bin centres (3i + 1, 3j + 1) and upsampled bilinearly
 * (constant beyond the outermost centres) into job.out (H x W).  If
 * job.out_anscombe is not NULL its first ceil(H/3) * ceil(W/3) values receive
 * the binned u_hat.  Requires ceil(H/3), ceil(W/3) >= r and H, W >= 2. */
fe_status fe_binned_workspace_size(const fe_ctx *ctx, const fe_job *jobs, int32_t n,
                                   size_t *bytes);
fe_status fe_denoise_binned(const fe_ctx *ctx, const fe_job *jobs, int32_t n,
                            void *workspace, size_t ws_bytes, void *hip_stream);

/* ---- continuous-batching server -----------------------------------------
 * A worker thread admits submitted jobs in arrival order as device memory
 * (a budget allocated once at create) frees up, keeps each admitted job's
 * state resident, and runs ticks: every tick advances the resident jobs by
 * up to iters_per_tick iterations each in shared launches (fe_advance),
 * starts newly admitted jobs (fe_begin) and finishes completed ones
 * (fe_end).  With tick_pixel_iters > 0 a tick offers its iterations to the
 * resident jobs oldest first and stops once it holds that many
 * pixel-iterations (the oldest job always advances), which bounds a tick's
 * duration and lets the oldest jobs finish first; with 0 every resident job
 * advances every tick.  Results are bitwise those of fe_denoise on the job
 * alone.  The client owns each job's counts and output buffers until its
 * completion is polled. */
typedef struct fe_server fe_server;

typedef struct {
    size_t hbm_budget_bytes;  /* device memory for resident job states        */
    int32_t iters_per_tick;   /* iterations per resident job per tick, >= 1   */
    int32_t max_active;       /* most jobs resident at once, >= 1             */
    int32_t ticks_in_flight;  /* ticks enqueued ahead of the device, 1..64    */
    int64_t tick_pixel_iters; /* work per tick (0: no limit), >= 0            */
} fe_server_config;

typedef struct {
    uint64_t tag;       /* the client's tag from fe_server_submit            */
    int32_t status;     /* FE_OK                                             */
    int32_t iterations;
    double t_submit;    /* seconds since server creation (host clock)        */
    double t_admit;     /* when its state became resident                    */
    double t_done;      /* when the tick that finished it completed (device  */
                        /* event, on the same time base)                     */
} fe_completion;

/* Create a server on the context's device; hip_stream NULL: its own stream.
 * Allocates the budget and the tick workspaces once. */
fe_status fe_server_create(const fe_ctx *ctx, const fe_server_config *cfg,
                           void *hip_stream, fe_server **out);
/* Queue one job (thread-safe, returns at once).  FE_ERR_INVALID if the job
 * is malformed or its state can never fit the budget. */
fe_status fe_server_submit(fe_server *srv, const fe_job *job, uint64_t tag);
/* Move up to max completions to out (*n of them), waiting up to wait_ms
 * for the first one. */
fe_status fe_server_poll(fe_server *srv, fe_completion *out, int32_t max,
                         int32_t *n, int32_t wait_ms);
/* Jobs queued and resident now, and the server clock (seconds). */
fe_status fe_server_load(fe_server *srv, int32_t *pending, int32_t *active,
                         double *now);
/* Finish every submitted job, then release the server (NULL allowed). */
void fe_server_destroy(fe_server *srv);
/* Message for the last non-OK status of a server call on this thread. */
const char *fe_server_last_error(void);

/* Workspace bytes fe_energy_grad needs for an H x W image (H * W < 2^31):
 * the launch's job table and two partial sums per workgroup tile. */
fe_status fe_energy_grad_workspace_size(const fe_ctx *ctx, int32_t height,
                                        int32_t width, size_t *bytes);

/* Energy E(u) = E_FoE(u) + D(u, v) (eq. 2.5 with eq. 3.4 or 3.6) and its
 * gradient grad E(u) = sum_i alpha_i K_i^T rho'(K_i u) + grad D (eq. 3.2),
 * at an Anscombe-domain image u (DEVICE H*W) for counts y (DEVICE H*W,
 * v = f_A(y)).  data_term is FE_DATA_QUADRATIC or FE_DATA_IDIV.  One fused
 * launch over the image's tiles, as the denoising step: the filter
 * responses stay on chip.  precision (FE_PREC_*) selects the contractions'
 * operands as in the denoising step: BF16 / FP16 round u and k_i in K_i u,
 * and z_i / (1 + z_i^2) and 2 alpha_i k_i in the adjoint, products
 * accumulated in FP32; the influence, rho(z) = log(1 + z^2) and the data
 * term stay FP32.  If `energy` (HOST) is not NULL the call synchronises the
 * stream and stores E there; with the I-divergence term E is +inf when any
 * u <= 0.  If `grad` (DEVICE H*W) is not NULL it receives grad E.  Energy
 * sums: FP32 per workgroup over the pixels its tile owns, then FP64 over
 * the workgroups in a fixed order on the device, so the result is
 * deterministic.  The workspace (DEVICE, 256-byte aligned) must not be
 * reused until the stream has passed the call.  This is
 * fe_energy_grad_batch on one image. */
fe_status fe_energy_grad(const fe_ctx *ctx, int32_t height, int32_t width,
                         const float *counts, const float *u, float lambda,
                         int32_t data_term, int32_t precision, double *energy,
                         float *grad, void *workspace, size_t ws_bytes,
                         void *hip_stream);

/* One image of fe_energy_grad_batch (the arguments of fe_energy_grad). */
typedef struct {
    int32_t height, width;  /* each >= r; H * W < 2^31                       */
    const float *counts;    /* DEVICE H*W, y >= 0                            */
    const float *u;         /* DEVICE H*W, Anscombe-domain image             */
    float *grad;            /* DEVICE H*W, receives grad E(u); may be NULL   */
    float lambda;           /* data-term weight, > 0                         */
    int32_t data_term;      /* FE_DATA_QUADRATIC or FE_DATA_IDIV             */
} fe_grad_job;

/* Workspace bytes fe_energy_grad_batch needs for these images. */
fe_status fe_energy_grad_batch_workspace_size(const fe_ctx *ctx, const fe_grad_job *jobs,
                                              int32_t n, size_t *bytes);

/* fe_energy_grad over n images in one launch (every tile of every image
 * shares it, as the denoising step's batches do): energies (HOST [n] or
 * NULL; if not NULL the call synchronises the stream) receives E of each
 * image, each job's grad (if not NULL) its gradient; contractions in
 * `precision` for every image.  Each image's gradient is bitwise that of
 * fe_energy_grad on it alone; its energy agrees to the rounding of the
 * FP32 per-tile sums (the tile height is chosen for the whole batch). */
fe_status fe_energy_grad_batch(const fe_ctx *ctx, const fe_grad_job *jobs, int32_t n,
                               int32_t precision, double *energies, void *workspace,
                               size_t ws_bytes, void *hip_stream);

/* Release the context (NULL is allowed). */
void fe_destroy(fe_ctx *ctx);

/* Message for the last non-OK status on the calling thread. */
const char *fe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FE_H */
