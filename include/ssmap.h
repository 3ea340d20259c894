/*
 * ssmap.h -- C ABI of libssmap: spatially-regularised, nonnegative
 * spatial-spectral partial-volume mapping with the LADMM iteration of
 * Liu, Mandal, Liao, Setsompop, Haldar (arXiv 2401.12890), run on one
 * AMD Instinct MI355X (gfx950).
 *
 * Problem (Eq. spat with the regulariser of Eq. l2, Sec. II-C):
 *     minimise_{f >= 0}  1/2 || m - (I_N (x) K) f ||^2 + lambda R(f),
 *     R(f) = sum_n sum_{m in Delta(n)} 1/2 || f_n - f_m ||^2 = 1/2 || D f ||^2,
 * with K the P x Q dictionary (linear mixture model, Sec. II-A), m_n the P
 * measurements of voxel n and f_n its Q spectral values.
 *
 * Method: Algorithm 2 of the paper (Sec. III-E) -- the single splitting
 * f = z of Eq. (Optprob_const), the low-rank f-step of Eq. (DictVecSVD)
 * and the linearised z-step of Eq. (z2) -- for a fixed number of
 * iterations from z = d = 0.
 *
 * Conventions used at this boundary:
 *   - Box grid (nx, ny, nz), nz = 1 for 2-D; voxel n = x + nx*(y + ny*z).
 *   - Delta(n): face neighbours (4 in 2-D, 6 in 3-D), free boundary (edge
 *     voxels have fewer neighbours). Every adjacent pair appears twice in
 *     the double sum of Eq. (l2), so D^T D = 2 L (L the grid Laplacian) and
 *     ||D^T D|| = 2 * sum_axes (2 + 2 cos(pi / n_axis)).
 *   - The returned map is z^K, the nonnegative iterate after K iterations.
 *   - Dictionaries, data and maps are dense, row-major, float64 on the host.
 *
 * Ownership: the caller owns every buffer it passes; ssmap_create copies K
 * and ssmap_solve copies M. A context owns all device memory it allocates
 * and frees it in ssmap_destroy. A context is not thread-safe; distinct
 * contexts may be used from distinct threads.
 *
 * Errors: functions return an ssmap_status (negative on failure) and never
 * throw across the ABI. After SSMAP_EINVAL, SSMAP_ENOMEM or SSMAP_ENONFINITE
 * the context stays usable. After SSMAP_EDEVICE it is poisoned: every later
 * call on it returns SSMAP_EDEVICE until ssmap_destroy. ssmap_last_error
 * gives a message for the last failure on a context.
 */
#ifndef SSMAP_H
#define SSMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssmap_ctx ssmap_ctx;

typedef enum {
    SSMAP_OK = 0,
    SSMAP_EINVAL = -1,      /* invalid argument (sizes, NULL, beta <= 0, ...) */
    SSMAP_ENOMEM = -2,      /* device memory (or SSMAP_HBM_BUDGET) exceeded    */
    SSMAP_EDEVICE = -3,     /* HIP runtime error; the context is poisoned       */
    SSMAP_ENONFINITE = -4,  /* NaN/Inf in the input or in a monitored iterate    */
    SSMAP_ENODEV = -5       /* no usable gfx950 device                           */
} ssmap_status;

/* Arithmetic of the iteration. The setup (SVD, rank, xi_p, coefficients)
 * and the monitoring reductions are float64 in every case. */
typedef enum {
    SSMAP_FP64 = 0,         /* float64 state and contractions                    */
    SSMAP_FP32 = 1,         /* float32 state and contractions                    */
    SSMAP_BF16X3 = 2        /* float32 state; contractions as three bf16 products
                               (hi*hi + hi*lo + lo*hi) with float32 accumulation */
} ssmap_precision;

/* Kernel family for the iteration (both compute the same iterates). */
typedef enum {
    SSMAP_KERNEL_AUTO = 0,  /* fused MFMA kernel when the rank allows (r <= 32), split
                               over chunks for small grids (see SPLIT); else the GEMM
                               path for float32 / bf16x3 without primal residual or
                               warm start; else unfused                           */
    SSMAP_KERNEL_UNFUSED = 1,
    SSMAP_KERNEL_FUSED = 2,
    SSMAP_KERNEL_SPLIT = 4, /* small grids, float64 / float32, r <= 32: the fused step
                               split over 16-node chunks, one workgroup per (brick,
                               chunk), the rank vectors carried as per-chunk partial
                               products summed in chunk order; no SSMAP_KEEP_AUX or
                               SSMAP_MONITOR_PRIMAL. AUTO takes it for grids of at
                               most 32 bricks and 2..32 chunks                    */
    SSMAP_KERNEL_GEMM = 3   /* any rank, float32 / bf16x3: the two contractions as
                               GEMMs over all voxels (hipBLASLt, else MFMA-tiled
                               GEMMs of this library; compute bound at high rank),
                               the stencil / z-update and the r-vector recursion as
                               elementwise passes; monitoring and SSMAP_KEEP_AUX
                               allowed (aux output needs the hipBLASLt products),
                               no SSMAP_MONITOR_PRIMAL or SSMAP_WARM_START         */
} ssmap_kernel;

enum {
    SSMAP_KEEP_AUX = 1,     /* keep f^K and d^K of the solve for ssmap_get_aux    */
    SSMAP_MONITOR_PRIMAL = 4, /* with check_every > 0: also the primal residual
                               ||z^k - f^k|| at every check (and DFCS of f^k when a
                               reference is set); f^k needs d^{k-1}, so the two
                               iterations before each check are bracketed by two
                               extra passes each (fused and unfused kernels only) */
    SSMAP_WARM_START = 8    /* start from the z^0 and d^0 set by ssmap_set_initial
                               instead of z = d = 0 (Algorithm 2's initialisation);
                               fused and unfused kernels only (AUTO picks them) */
};

/* LADMM parameters (Algorithm 2 inputs, Sec. III-E; selection rules, Sec. III-F). */
typedef struct {
    double beta;            /* penalty parameter, > 0                                    */
    double xi_p;            /* <= 0: 0.75 * lambda * ||D^T D|| + 1e-10 (Eq. sigma_cond)   */
    int rank;               /* 0: smallest r with ||K - K_r||_F < 5e-5 ||K||_F (Sec.
                               III-F); -1: min(P, Q), the unapproximated K; > 0: that r */
    int precision;          /* ssmap_precision                                           */
    int check_every;        /* 0: no monitoring; k > 0: objective, residuals and DFCS
                               (float64 reductions) every k iterations and after the
                               last one, into the stats history. Without stop_tol (and
                               with at most SSMAP_MAX_HIST checks) the checks are read
                               once, after the last iteration: a non-finite iterate
                               then returns SSMAP_ENONFINITE after the run, naming the
                               first check that saw it; with stop_tol each check is
                               read when it is taken and ends the solve there        */
    int flags;              /* SSMAP_KEEP_AUX | SSMAP_MONITOR_PRIMAL | SSMAP_WARM_START
                               (| SSMAP_AUTOTUNE for batches)                            */
    int kernel;             /* ssmap_kernel                                              */
    int reserved;
    double stop_tol;        /* 0: run all iters. > 0 (needs check_every > 0, no
                               SSMAP_KEEP_AUX): residual stopping rule, stop after
                               iteration k when k is a multiple of check_every and
                               ||z^k - z^{k-1}|| <= stop_tol ||z^k|| (the paper prints
                               no rule; stats.iters reports the count run)           */
} ssmap_steps;

#define SSMAP_MAX_HIST 512

/* Observability of the last solve on a context. */
typedef struct {
    int rank;               /* r used                                             */
    int rank_padded;        /* r rounded up for the contraction tiles              */
    int precision;
    int kernel;             /* ssmap_kernel actually used (1 to 4)                 */
    int iters;              /* iterations run                                      */
    int n_hist;             /* entries in the history arrays                       */
    double xi_p;            /* xi_p used                                           */
    double tau;             /* 1 / (xi_p + beta)                                   */
    double dtd_norm;        /* ||D^T D||                                           */
    double sigma_max;       /* largest singular value of K                         */
    double setup_ms;        /* ssmap_create: SVD and uploads                        */
    double project_ms;      /* data projection h = Sigma_r U_r^T m                  */
    double iterate_ms;      /* the iteration loop, monitoring included             */
    double output_ms;       /* z^K to the voxel-major output                        */
    double device_bytes;    /* device memory held by the context                   */
    double gemm_ms;         /* GEMM path: time in the two products (events; with the
                               fused kernels, their epilogues included)             */
    double gemm_flops;      /* GEMM path: flops of the two products as issued      */
    int hist_iter[SSMAP_MAX_HIST];
    double hist_objective[SSMAP_MAX_HIST];  /* 1/2||m - K_r z||^2 + lambda R(z)    */
    double hist_dual[SSMAP_MAX_HIST];       /* beta ||z^k - z^{k-1}||               */
    double hist_znorm[SSMAP_MAX_HIST];      /* ||z^k||                              */
    double hist_primal[SSMAP_MAX_HIST];     /* ||z^k - f^k|| (SSMAP_MONITOR_PRIMAL), else -1 */
    double hist_dfcs[SSMAP_MAX_HIST];       /* ||z^k - f*|| / ||f*|| (Eq. DFCS) with a
                                               reference set, else -1                */
    double hist_dfcs_f[SSMAP_MAX_HIST];     /* ||f^k - f*|| / ||f*|| (reference and
                                               SSMAP_MONITOR_PRIMAL), else -1        */
    int gemm_library;       /* GEMM path: 1 when the two products ran as library GEMMs
                               (hipBLASLt) with the elementwise steps as separate
                               passes, 0 for the library's own fused MFMA kernels   */
} ssmap_stats;

/* Factor the dictionary and prepare a context for a fixed grid.
 *   K     : P*Q float64, row-major (K[p*Q + q]); finite, not all zero.
 *   P, Q  : >= 1.
 *   grid  : {nx, ny, nz}, each >= 1 (nz = 1 for 2-D).
 *   out   : receives the context (NULL on failure).
 * Computes the thin SVD of K in float64 (Algorithm 2, SVD step) and
 * uploads the factors to the current HIP device. */
ssmap_status ssmap_create(const double *K, int P, int Q, const int64_t grid[3],
                          ssmap_ctx **out);

/* Run `iters` LADMM iterations (Algorithm 2) on host data.
 *   M      : N*P float64, voxel-major (M[n*P + p]); N = nx*ny*nz.
 *   lambda : regularisation weight, >= 0.
 *   steps  : LADMM parameters (see ssmap_steps).
 *   iters  : >= 0; 0 returns zeros (z^0 = 0).
 *   F_out  : N*Q float64, voxel-major; receives z^iters.
 * Blocks until the result is on the host. */
ssmap_status ssmap_solve(ssmap_ctx *ctx, const double *M, double lambda,
                         const ssmap_steps *steps, int iters, double *F_out);

/* Same as ssmap_solve on device buffers, ordered on `hip_stream` (a
 * hipStream_t; NULL = the default stream).
 *   dM : device, N*P voxel-major, float64 for SSMAP_FP64, else float32.
 *   dF : device, N*Q voxel-major, same element type as dM; receives z^iters.
 * The buffers are borrowed for the duration of the call, which returns
 * after the work has completed on the stream. */
ssmap_status ssmap_solve_device(ssmap_ctx *ctx, const void *dM, double lambda,
                                const ssmap_steps *steps, int iters, void *dF,
                                void *hip_stream);

/* Allocation-free variant of ssmap_solve_device, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). Same arguments, result and ordering on
 * `hip_stream` as ssmap_solve_device; it calls no hipMalloc, hipFree or other
 * allocating routine. Every device buffer of the solve (state, r-vectors,
 * constants, launch tables, monitoring sums) is carved from one static device
 * array of SSMAP_NOALLOC_MAX_BYTES that each GPU the library runs on holds
 * until the process ends; the solve initialises everything it reads there.
 * Limits: EINVAL when the solve needs more than SSMAP_NOALLOC_MAX_BYTES (about
 * (2 Qp + 3 RP) N words of state, Qp = Q rounded up to 16, RP = the rank
 * rounded up to 16, plus the dictionary's constants), with SSMAP_KEEP_AUX or
 * with SSMAP_KERNEL_GEMM; AUTO chooses as for ssmap_solve_device, with the
 * unfused kernels where that would be the GEMM path. All calls on one GPU share its array, which
 * keeps the last call's contents: calls that overlap on one GPU (other streams,
 * other threads or contexts) race and must be serialised by the caller. */
#define SSMAP_NOALLOC_MAX_BYTES (64ull << 20)
ssmap_status ssmap_solve_device_noalloc(ssmap_ctx *ctx, const void *dM, double lambda,
                                        const ssmap_steps *steps, int iters, void *dF,
                                        void *hip_stream);

/* f^iters and d^iters of the last solve run with SSMAP_KEEP_AUX (zeros after a
 * solve of zero iterations).
 *   f_out, d_out : N*Q float64 voxel-major host buffers; either may be NULL. */
ssmap_status ssmap_get_aux(ssmap_ctx *ctx, double *f_out, double *d_out);

/* Masked voxel set (Sec. II-C, maskless footnote): estimate only the voxels
 * inside the object, with no smoothness across its boundary. mask: N bytes
 * (voxel order as M's rows), nonzero = inside; copied. From then on every
 * solve on ctx keeps outside voxels at 0 (their rows of F are 0 and their rows
 * of M are not read), the regulariser of Eq. (l2) runs over face-neighbour
 * pairs with both voxels inside, and ||D^T D|| of that graph (float64
 * Lanczos) enters the xi_p rule. Bricks with no inside voxel are not
 * launched. mask = NULL restores the whole box. */
ssmap_status ssmap_set_mask(ssmap_ctx *ctx, const uint8_t *mask);

/* Reference map for the distance from the converged solution (Eq. DFCS,
 * Sec. IV: ||f^k - f*|| / ||f*||, f* the converged map of the unapproximated
 * K). f_star: N*Q float64 voxel-major (as F_out), finite, not all zero;
 * copied to the device. Every monitored solve on ctx then reports DFCS of z^k
 * (and of f^k with SSMAP_MONITOR_PRIMAL). f_star = NULL removes it. */
ssmap_status ssmap_set_reference(ssmap_ctx *ctx, const double *f_star);

/* Initial iterate for solves with SSMAP_WARM_START (Algorithm 2 starts from
 * z = d = 0; a warm start starts from a given z^0 and scaled dual d^0 instead,
 * e.g. the z^K and d^K of an earlier solve on the same data, lambda, beta and
 * rank (checkpoint and resume; d^K from ssmap_get_aux), or a minimiser z* with
 * d* = K_r^T (m - K_r z*), which the iteration leaves in place). z0, d0: N*Q
 * float64 voxel-major host buffers (as F_out), finite; either may be NULL for
 * zeros; copied to the device (N*Q*8 bytes each). From them the solve forms its
 * reduced state on the device in float64 (y^0 = V_r^T z^0, w^0 = a.h -
 * b.(y^0 - V_r^T d^0 / beta), Eq. DictVecSVD) and rounds it to the state
 * precision; outside a mask both are taken as 0. Both NULL removes the
 * initial iterate. EINVAL: a warm-started solve with none set, or with the
 * chunk-split or GEMM kernel, a batch, or the allocation-free entry point. */
ssmap_status ssmap_set_initial(ssmap_ctx *ctx, const double *z0, const double *d0);

/* Penalty selection heuristic (Sec. III-F): solve the centre patch of the
 * grid (3 voxels per axis longer than 1, fewer on shorter axes; the box
 * without any mask) for `iters` iterations at each of the n_betas candidate
 * penalties betas[i] > 0, with lambda and the other fields of steps as given
 * (beta, check_every, flags and stop_tol are overridden), and return through
 * *beta_out the candidate whose iterate has the lowest objective of
 * Eq. (spat) on the patch (float64, the first on ties). J_out (n_betas
 * entries, may be NULL) receives the objectives. M: the full N*P float64
 * data on the host. */
ssmap_status ssmap_tune_beta(ssmap_ctx *ctx, const double *M, double lambda,
                             const ssmap_steps *steps, int iters, const double *betas,
                             int n_betas, double *J_out, double *beta_out);

/* Statistics of the last solve (see ssmap_stats). */
ssmap_status ssmap_get_stats(const ssmap_ctx *ctx, ssmap_stats *out);

/* Singular values of K (descending), min(P, Q) of them, into sigma_out
 * (capacity `cap`); returns the count through *n_out. */
ssmap_status ssmap_get_singular_values(const ssmap_ctx *ctx, double *sigma_out,
                                       int cap, int *n_out);

/* Message for the last failure on ctx (or of the last failed ssmap_create
 * when ctx is NULL). Valid until the next call on the same context. */
const char *ssmap_last_error(const ssmap_ctx *ctx);

/* Release the context and its device memory. NULL is a no-op. */
void ssmap_destroy(ssmap_ctx *ctx);

/* Library version string. */
const char *ssmap_version(void);

/* ------------------------------------------------------------------------
 * Batches: many independent problems (each with its own dictionary, grid and
 * data, e.g. the slices of a study or the B1-binned dictionaries of the
 * paper's MRF experiment, Sec. IV-D) solved together. Problems of one class
 * (precision, padded rank, planar or volumetric grid) share each fused
 * launch: one launch walks the bricks of all of them, so many small problems
 * fill the GPU. Each problem's iterates are exactly those of ssmap_solve on
 * it alone with kernel SSMAP_KERNEL_FUSED (same kernels, same arithmetic order).
 * ---------------------------------------------------------------------- */
typedef struct ssmap_batch ssmap_batch;

enum {
    SSMAP_AUTOTUNE = 2      /* steps.flags: choose each class's brick shape by timing */
};

#define SSMAP_MAX_CLASSES 16

typedef struct {
    int njobs;
    int nclasses;           /* shared-launch classes of the last solve               */
    int solo_jobs;          /* jobs without a fused kernel (run one launch each)      */
    int iters;
    double voxels;          /* sum of N over the jobs                                */
    double project_ms;      /* projections of all jobs                               */
    double iterate_ms;      /* the iteration loop                                    */
    double output_ms;
    double autotune_ms;     /* shape search (0 when not requested)                   */
    int class_precision[SSMAP_MAX_CLASSES];
    int class_rank_padded[SSMAP_MAX_CLASSES];
    int class_jobs[SSMAP_MAX_CLASSES];
    int class_bricks[SSMAP_MAX_CLASSES];
    int class_brick_y[SSMAP_MAX_CLASSES];    /* chosen brick: 16 x brick_y x brick_z  */
    int class_brick_z[SSMAP_MAX_CLASSES];
} ssmap_batch_stats;

/* Factor `njobs` dictionaries (as ssmap_create, one context per job).
 *   K[j] : P[j]*Q[j] float64 row-major;  grids : njobs*3 int64 {nx, ny, nz}.
 * All arrays are caller-owned and copied. */
ssmap_status ssmap_batch_create(int njobs, const double *const *K, const int *P, const int *Q,
                                const int64_t *grids, ssmap_batch **out);

/* Masked voxel set of job `job` (0 <= job < njobs), exactly as ssmap_set_mask
 * for a single problem (Sec. II-C, maskless footnote): outside voxels stay 0,
 * the regulariser runs over inside face pairs, the xi_p rule takes the masked
 * graph's ||D^T D||, the job's bricks with no inside voxel leave the shared
 * launches, and its rows of M outside are not read. mask = NULL restores the
 * whole box. EINVAL for a job index out of range. */
ssmap_status ssmap_batch_set_mask(ssmap_batch *b, int job, const uint8_t *mask);

/* Solve every job for `iters` iterations on device buffers, ordered on
 * `hip_stream`. dM[j] / dF[j] as in ssmap_solve_device for job j; lambda and
 * steps are per job (njobs entries). steps[j].check_every may be set per job
 * (its history then goes to ssmap_batch_get_job_stats); stop_tol must be 0 and
 * SSMAP_KEEP_AUX, SSMAP_MONITOR_PRIMAL and SSMAP_WARM_START unset (use the
 * single-problem entry points for those). Each job's map equals, bit for bit,
 * its single solve with SSMAP_KERNEL_FUSED (and its mask).
 * SSMAP_AUTOTUNE in any job's flags turns the shape search on; the shapes it
 * chooses are kept in `b` and used by its later solves of the same classes
 * (same precision, rank bucket and member jobs) until it is destroyed. */
ssmap_status ssmap_batch_solve_device(ssmap_batch *b, const void *const *dM, const double *lambda,
                                      const ssmap_steps *steps, int iters, void *const *dF,
                                      void *hip_stream);

/* Host-buffer variant (float64 M[j], F_out[j]); blocks until done. */
ssmap_status ssmap_batch_solve(ssmap_batch *b, const double *const *M, const double *lambda,
                               const ssmap_steps *steps, int iters, double *const *F_out);

ssmap_status ssmap_batch_get_stats(const ssmap_batch *b, ssmap_batch_stats *out);

/* Statistics of job `job` in the last batch solve, as ssmap_get_stats for a
 * single problem: rank, xi_p, precision, and with check_every > 0 the job's
 * monitoring history (objective, dual residual, ||z||, DFCS against a reference
 * is not available in batches). EINVAL for a job index out of range. */
ssmap_status ssmap_batch_get_job_stats(const ssmap_batch *b, int job, ssmap_stats *out);

/* Message for the last failure on b (or of the last failed ssmap_batch_create when b is NULL). */
const char *ssmap_batch_last_error(const ssmap_batch *b);

/* Release the batch, its contexts and device memory. NULL is a no-op. */
void ssmap_batch_destroy(ssmap_batch *b);

/* ------------------------------------------------------------------------
 * Serving: independent mapping jobs arriving over time (the per-job problem
 * of Eq. (spat) solved by Algorithm 2 for a fixed iteration count). A job's
 * state (z ping-pong and its r-vectors) stays in device memory from
 * admission to retirement. Admission is first in, first out under a device-
 * memory budget reserved at creation; a job that does not fit waits, and so
 * do the jobs behind it. Running jobs of one class (precision, padded rank,
 * u K-step bucket, brick shape, and size band: below 64 MB, below 1 GB or
 * above of state moved per iteration) advance together, one iteration per shared
 * fused launch; a job joins its class at an iteration boundary and leaves
 * after its last iteration while the others keep running (continuous
 * batching). Jobs of the large band iterate one at a time, in arrival order
 * (two of them sharing the GPU would each take about twice as long); small and
 * middle jobs run beside them. Classes are spread over up to four HIP streams
 * and progress independently of one another. A served job's result is exactly that of
 * ssmap_solve_device with kernel SSMAP_KERNEL_FUSED on the same input (same
 * kernels, same arithmetic order). A server is not thread-safe.
 * ---------------------------------------------------------------------- */
typedef struct ssmap_server ssmap_server;

typedef struct {
    double hbm_budget;      /* bytes of device memory for job state, reserved at create (>= 256) */
    int streams;            /* HIP streams the classes are spread over, 1..4 (0 -> 4)           */
    int reserved[3];
} ssmap_server_opts;

enum { SSMAP_JOB_QUEUED = 0, SSMAP_JOB_RUNNING = 1, SSMAP_JOB_DONE = 2 };

typedef struct {
    int state;              /* SSMAP_JOB_*                                                        */
    int status;             /* SSMAP_OK, or SSMAP_ENONFINITE when M held a NaN or Inf (F undefined) */
    int rank, rank_padded, precision, iters;
    double xi_p;
    double state_bytes;     /* device bytes the job holds while running                          */
    double submit_ms;       /* host clock at submit, ms since ssmap_server_create                 */
    double admit_ms;        /* host clock when the job's first kernels were enqueued              */
    double done_ms;         /* device clock (event) when F was complete; valid once SSMAP_JOB_DONE */
} ssmap_job_info;

typedef struct {
    int64_t submitted, admitted, completed;
    int64_t launches;       /* shared fused launches enqueued                                     */
    int classes, streams;
    double budget_bytes, in_use_bytes, peak_bytes;
    double voxel_iterations;   /* sum of N * iters over completed jobs                           */
} ssmap_server_stats;

/* Reserve the budget and create the streams on the current device. */
ssmap_status ssmap_server_create(const ssmap_server_opts *opts, ssmap_server **out);

/* Factor a dictionary once (K: P*Q float64 row-major, copied; thin SVD on the
 * host) for every job that names it; returns its id through *dict_id. */
ssmap_status ssmap_server_add_dictionary(ssmap_server *sv, const double *K, int P, int Q,
                                         int *dict_id);

/* Queue a job on dictionary dict_id and grid {nx, ny, nz}. dM (N*P,
 * voxel-major) and dF (N*Q, voxel-major; receives z^iters) are device buffers
 * in the precision's I/O type (float64 for SSMAP_FP64, else float32), borrowed
 * until the job is done. lambda, steps and iters as in ssmap_solve, with
 * steps->flags = 0, no stop_tol and kernel AUTO or FUSED; steps->check_every
 * > 0 monitors the job (at most 32 checks, iters / check_every rounded up;
 * read with ssmap_server_get_job_stats; the job holds r N + N doubles more);
 * EINVAL when no fused kernel covers the precision, rank and size; ENOMEM
 * when the job alone needs more than the budget. Returns the job id. */
ssmap_status ssmap_server_submit(ssmap_server *sv, int dict_id, const int64_t grid[3],
                                 const void *dM, double lambda, const ssmap_steps *steps,
                                 int iters, void *dF, int64_t *job_id);

/* ssmap_server_submit for a job on a masked voxel set (the maskless footnote of
 * Sec. II-C, as ssmap_set_mask for a single solve): mask holds N bytes (host,
 * copied; nonzero = inside). Outside voxels are not unknowns (their rows of dM
 * are not read, their z is 0), the regulariser runs over the graph the mask
 * induces, and xi_p <= 0 takes ||D^T D|| of that graph (computed at submit,
 * Lanczos on the host). The job holds N bytes more; bricks without an inside
 * voxel are left out of the shared launches. NULL mask: ssmap_server_submit. */
ssmap_status ssmap_server_submit_masked(ssmap_server *sv, int dict_id, const int64_t grid[3],
                                        const uint8_t *mask, const void *dM, double lambda,
                                        const ssmap_steps *steps, int iters, void *dF,
                                        int64_t *job_id);

/* Admit the queued jobs that fit, then enqueue about horizon_ms of iterations
 * for every class. Asynchronous: the host blocks only to keep at most two such
 * chunks per class in flight. *n_pending (may be NULL) = jobs not yet done. */
ssmap_status ssmap_server_pump(ssmap_server *sv, double horizon_ms, int *n_pending);

/* State, status and timings of one job. */
ssmap_status ssmap_server_poll(ssmap_server *sv, int64_t job_id, ssmap_job_info *out);

/* Monitoring record of a finished job submitted with steps->check_every > 0
 * (objective of Eq. spat, dual residual and ||z|| after every check_every-th
 * iteration and the last, float64 reductions, as ssmap_get_stats gives for a
 * single solve; hist_primal and the DFCS entries are -1). rank, xi_p, tau and
 * iters describe the job; n_hist is 0 for an unmonitored job. EINVAL while the
 * job is not done. A check that saw a non-finite iterate makes the job's status
 * SSMAP_ENONFINITE. */
ssmap_status ssmap_server_get_job_stats(ssmap_server *sv, int64_t job_id, ssmap_stats *out);

/* Pump until every submitted job is done and the device work has finished. */
ssmap_status ssmap_server_drain(ssmap_server *sv);

ssmap_status ssmap_server_get_stats(const ssmap_server *sv, ssmap_server_stats *out);

/* Message for the last failure on sv (or of the last failed ssmap_server_create when sv is NULL). */
const char *ssmap_server_last_error(const ssmap_server *sv);

/* Wait for the device work, then release the server and its memory. NULL is a no-op. */
void ssmap_server_destroy(ssmap_server *sv);

#ifdef __cplusplus
}
#endif

#endif /* SSMAP_H */
