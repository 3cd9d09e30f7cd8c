/*
 * smsm.h - C ABI of the MI355X SMS-MUSSELS solver.
 *
 * The library reconstructs simultaneous-multislice (SMS), multi-shot
 * diffusion k-space by minimising
 *
 *     || A(x) - y ||^2  +  lambda * sum_l || H_l(x_l) ||_*          (Eq. 10)
 *
 * (Mani et al., "SMS MUSSELS", Theory section, Eq. 10) with iteratively
 * reweighted least squares: for k = 0 .. n_irls-1 the weights
 * W_l = (H_l^H H_l + eps_l I)^(-1/2) are formed from the current iterate and
 * n_cg conjugate-gradient steps are taken on
 *
 *     N(x) = A^H A x + (lambda/2) sum_l H_l^H(H_l(x_l) W_l) = A^H y.
 *
 * Operators (all conventions fixed here, the paper leaves them open):
 *  - DFT F: centred and unitary, DC at index n/2 in both domains.
 *  - A (Fig. 1): (A x)_{i,c} = M_i . sum_l theta_l . F(S_{l,c} . F^-1(x_{l,i}))
 *    with theta_l[j2] = exp(-2 pi i s_l (j2 - n2/2)) (blipped CAIPI, Eq. 1
 *    and its multi-shot form Eq. 3) and M_i the ky lines of shot i (Eq. 2).
 *  - H_l (Eq. 8-9): rows = valid r x r patch anchors (n2-r+1)(n1-r+1),
 *    columns = (shot, b2, b1); entry x_{l,i}[p2+b2][p1+b1].
 *  - eps_l(k) = max(eps_frac * eps_decay^-k, eps_floor_frac) * sigma_l with
 *    sigma_l the largest eigenvalue of H_l^H H_l at x0 = A^H y; a slice with
 *    sigma_l = 0 is not regularised.
 *
 * Layouts: row-major, kx (n1) fastest.  Complex numbers are interleaved
 * (re, im) pairs: "c64" = 2 x float, "c128" = 2 x double.
 *   x    [L][Ns][n2][n1]   slice-unfolded k-space of every shot
 *   y    [Ns][Nc][n2][n1]  measured k-space, zero-filled; entries of ky
 *                          lines a shot does not acquire are ignored
 *   S    [L][Nc][n2][n1]   coil sensitivities per slice (image domain)
 *   G, W [L][K][K]         K = Ns r^2, row/column index (i*r + b2)*r + b1
 *
 * Pointers named *_dev are device pointers of the device that was current
 * when the plan was created; host pointers are read during the call only.
 * Memory: the plan holds only what smsm_plan_create derives (the coil maps,
 * transform and phase tables, the status word).  Every buffer a solve or an
 * operator chain writes (the CG vectors, the Gram, weight and band tables,
 * partial sums) lives in a caller-owned workspace of smsm_workspace_bytes()
 * bytes bound with smsm_set_workspace; no entry point that runs kernels
 * allocates device memory.
 * Every entry point that takes a stream enqueues its work on that stream
 * (NULL = the default stream) and returns without waiting; kernel faults
 * show at the caller's next synchronisation.  A plan is not re-entrant: use
 * it from one stream at a time.  No entry point aborts or throws; invalid
 * arguments are reported synchronously through the return status.
 */
#ifndef SMSM_H
#define SMSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smsm_plan smsm_plan;   /* opaque */
typedef struct smsm_batch smsm_batch; /* opaque: solves of several plans captured as one graph */

typedef enum {
    SMSM_OK = 0,
    SMSM_E_INVALID = -1,      /* bad pointer, size or parameter */
    SMSM_E_UNSUPPORTED = -2,  /* valid but not implemented (e.g. a sampling pattern) */
    SMSM_E_NOMEM = -3,        /* device allocation failed in plan creation */
    SMSM_E_DEVICE = -4,       /* a HIP runtime call failed */
    SMSM_E_NUMERIC = -5,      /* NaN/Inf met in the CG recurrences (smsm_plan_status) */
    SMSM_E_NOT_CONVERGED = -6,/* the weights iteration hit ns_max_iter (smsm_plan_status) */
    SMSM_E_SCRATCH = -7       /* workspace above SMSM_NOALLOC_SCRATCH_BYTES (smsm_solve_noalloc) */
} smsm_status;

typedef struct {
    int32_t n1;        /* kx / readout size, 16..256: a power of two, or 3 or 7 times one, a multiple of 16 (e.g. 192, 224) */
    int32_t n2;        /* ky / phase-encode size, the same set */
    int32_t n_slices;  /* L, simultaneously excited slices, 1..4 */
    int32_t n_shots;   /* Ns, interleaved shots, power of two 1..8, n2/Ns >= 8 */
    int32_t n_coils;   /* Nc, receive channels, >= 1 */
    int32_t filt;      /* r, Hankel filter support, 2 <= r, Ns r^2 <= 256, 2r-1 <= min(n1,n2)/2 */
} smsm_geometry;

typedef struct {
    double  lambda;          /* lambda of Eq. 10, >= 0 */
    int32_t n_irls;          /* IRLS iterations, >= 1 */
    int32_t n_cg;            /* CG iterations per IRLS iteration, >= 0 */
    double  eps_frac;        /* eps schedule start (fraction of sigma_l), > 0 */
    double  eps_decay;       /* eta >= 1 */
    double  eps_floor_frac;  /* >= 0 */
    int32_t ns_max_iter;     /* cap on Newton-Schulz iterations for W (0 = 16) */
    uint32_t flags;          /* SMSM_FLAG_* */
} smsm_params;

/* x written by smsm_solve is complex128 instead of complex64. */
#define SMSM_FLAG_X_C128 0x1u
/* Mixed-precision form: the regulariser's tables that every CG iteration
 * reads (the image-domain Hankel kernel of the column pass, the band
 * kernel's transformed row tables and corner tables) are stored complex64
 * and widened to FP64 on load; everything else stays FP64.  Takes effect
 * when the weights are next built (each IRLS step, smsm_set_weights); the
 * error against the FP64 oracle is reported per instance by the tests. */
#define SMSM_FLAG_REG_F32 0x2u
/* Mixed-precision Gram: G_l = H_l^H H_l is formed as a GEMM over the patch
 * anchors on the BF16 matrix cores (every entry of H split into three BF16
 * parts per real component, the six leading part products of each real
 * product, FP32 sums over chunks of 2048 anchors, FP64 across chunks)
 * instead of from image-domain correlations in FP64; everything else stays
 * FP64.  The error against the FP64 oracle is reported per instance by the
 * tests and the benchmark.  Takes effect in smsm_solve and smsm_gram.  The
 * plan must be created with it (its workspace then holds the chunk partials,
 * L * ceil(P/2048) * KB(KB+1)/2 * 64 KiB, P = (n1-r+1)(n2-r+1) anchors, KB =
 * ceil(K/64));
 * smsm_plan_set_params returns SMSM_E_UNSUPPORTED when it would turn the
 * flag on for a plan created without it. */
#define SMSM_FLAG_GRAM_BF16 0x4u

/*
 * Create a plan for one geometry.  coil_maps_dev: c64 [L][Nc][n2][n1] on
 * the current device, copied (re-laid out) into the plan on `stream`, which
 * the call synchronises before returning.  shot_mask: host uint8 [Ns][n2],
 * 1 where shot i acquires ky line j2; this build supports the interleaved
 * pattern of Eq. 2 only (j2 % Ns == i) and returns SMSM_E_UNSUPPORTED for
 * any other.  Geometries whose column pass does not fit one workgroup's
 * shared memory (at most 5120 = L Ns n2 image points per column, fewer
 * with large filters) also return SMSM_E_UNSUPPORTED.  caipi_shift: host
 * [L] shift of each slice as a fraction of the FOV (NULL = l/L).  The plan's
 * own device memory (coil maps widened to
 * complex128, transform and phase tables: smsm_plan_device_bytes) is
 * allocated here and released by smsm_plan_destroy; the plan has no
 * workspace until smsm_set_workspace binds one.  On failure *out is NULL.
 */
smsm_status smsm_plan_create(const smsm_geometry* geom, const smsm_params* params,
                             const void* coil_maps_dev, const uint8_t* shot_mask,
                             const double* caipi_shift, void* stream, smsm_plan** out);

/* Release the plan and its device memory (synchronises the device first). NULL is a no-op. */
smsm_status smsm_plan_destroy(smsm_plan* plan);

/* Bytes of device memory the plan holds (not counting the workspace). */
size_t smsm_plan_device_bytes(const smsm_plan* plan);

/* Bytes of device workspace a plan needs: about 7 c128 vectors of
 * [L][Ns][n2][n1], the folded data, the image-domain Hankel kernel and the
 * band, Gram and weight tables (about 240 MB for 256 x 256, 3 slices, 4
 * shots, 32 coils, 7 x 7 filter).  0 for a null plan. */
size_t smsm_workspace_bytes(const smsm_plan* plan);

/* Bind caller-owned device memory (e.g. a torch tensor) as the plan's
 * workspace: ws_dev on the plan's device, 256-byte aligned, bytes >=
 * smsm_workspace_bytes(plan); NULL unbinds.  The library neither frees nor
 * clears it; its contents between calls are the library's (weights loaded by
 * smsm_set_weights live there and are forgotten when another workspace is
 * bound).  The caller keeps it allocated while the plan may use it, and while
 * a batch built on the plan exists.  Entry points that run kernels return
 * SMSM_E_INVALID while no workspace is bound.  Errors: SMSM_E_INVALID for a
 * null plan, a short or misaligned buffer. */
smsm_status smsm_set_workspace(smsm_plan* plan, void* ws_dev, size_t bytes);

/* Replace the solver parameters of an existing plan (same geometry). */
smsm_status smsm_plan_set_params(smsm_plan* plan, const smsm_params* params);

/*
 * The IRLS solve.  y_dev: c64 [Ns][Nc][n2][n1]; x_dev: c64 (or c128 with
 * SMSM_FLAG_X_C128) [L][Ns][n2][n1]; y and x must not overlap.  All work is
 * asynchronous on `stream` and runs in the bound workspace (SMSM_E_INVALID
 * without one); no device memory is allocated.
 */
smsm_status smsm_solve(smsm_plan* plan, const void* y_dev, void* x_dev, void* stream);

/* Size of the static device scratch of smsm_solve_noalloc: 64 MiB. */
#define SMSM_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * The IRLS solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * exactly smsm_solve (same kernels, same order, same result bit for bit),
 * run in a static device array of SMSM_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends, instead of the
 * bound workspace (which may be absent and is left untouched).  No device
 * memory is allocated or freed.  Every call on one device shares that
 * device's array and leaves its contents behind: calls that overlap on one
 * device (any plans, any streams) race and must be serialised by the caller.
 * Errors: SMSM_E_INVALID for null arguments; SMSM_E_SCRATCH when
 * smsm_workspace_bytes(plan) exceeds the array (enough for 64 x 64 and most
 * 128 x 128 geometries, not for 256 x 256 with 32 coils); SMSM_E_DEVICE if
 * the array's address cannot be taken; else as smsm_solve.
 */
smsm_status smsm_solve_noalloc(smsm_plan* plan, const void* y_dev, void* x_dev, void* stream);

/*
 * Numeric status since the last call: SMSM_E_NUMERIC if a CG step met a
 * non-finite or non-positive curvature (NaN or Inf in y, for instance),
 * else SMSM_E_NOT_CONVERGED if a weights iteration of a solve or of
 * smsm_weights left a slice above the tolerance after ns_max_iter steps
 * (its W is then the last iterate), else SMSM_OK.  Synchronises the device
 * and clears both flags.
 */
smsm_status smsm_plan_status(smsm_plan* plan);

/* Static description of a status code. */
const char* smsm_status_string(smsm_status s);

/* ---- batches: many slice groups as one submission ---------------------- */

/* Captures the solves x_devs[k] = solve(plans[k], y_devs[k]), k < n, into one
 * hipGraph: the plans are dealt round-robin to min(n_streams, distinct plans)
 * concurrent streams (default priority) joined at the end, so independent
 * slice groups (any mix of the geometries the plans were created for) overlap
 * on the GPU.
 * Each solve computes exactly what smsm_solve computes (same kernels, same
 * order within its plan: results are bitwise equal).  A plan may appear
 * several times (e.g. the diffusion directions of one slice group): its solves
 * share its scratch memory, so they all run in entry order on the stream of
 * its first entry, while distinct plans are dealt round-robin to the streams.
 * Ownership: the plans stay alive, with the workspaces bound at capture, and
 * unused by other calls while the batch exists; y_devs/x_devs (layouts as for smsm_solve; every x distinct) are
 * baked into the graph, so the caller keeps them allocated and refills y_devs
 * before each launch.  Per-launch kernel timing must be off on every plan.
 * Errors: SMSM_E_INVALID (null plan or buffer, a plan without a workspace, n < 1,
 * n_streams outside [1, 64], plans on different devices, timing on),
 * SMSM_E_NOMEM, SMSM_E_DEVICE (stream, capture or instantiation failure), or
 * the first error a captured solve returned.
 * The entries are captured in consecutive segments of at most 30 entries
 * holding at most 5 of any one plan, one graph per segment, launched in order (a
 * plan's solves form one dependency chain, which a segment keeps short; a
 * single graph holding 30 solves of a plan, about 67,000 kernels deep, ended
 * the process in its launch on this runtime).
 * n_streams = 0 autotunes the launch shape: a graph is captured for each
 * stream count in {1, 2, 3, 4, 6, 8} up to the number of distinct plans, each
 * is launched once untimed and twice timed (hipEvents on an internal stream),
 * and the fastest is kept (smsm_batch_streams tells which).  Autotuning runs
 * the batch 3 times per candidate, writing x_devs, and synchronises with
 * those launches. */
smsm_status smsm_batch_create(smsm_plan* const* plans, int n, const void* const* y_devs,
                              void* const* x_devs, int n_streams, smsm_batch** out);

/* Number of concurrent streams of a batch (the autotuner's choice when it was
 * created with n_streams = 0); 0 for a null batch. */
int smsm_batch_streams(const smsm_batch* batch);

/* Runs every solve of the batch once, ordered after prior work on `stream`;
 * later work on `stream` waits for all of them.  Asynchronous. */
smsm_status smsm_batch_launch(smsm_batch* batch, void* stream);

/* Waits for the device, then frees the graph, its streams and events
 * (not the plans or buffers).  A null batch is a no-op. */
smsm_status smsm_batch_destroy(smsm_batch* batch);

/* Launch shapes by measurement: for the plan's geometry, each candidate
 * number of rows per workgroup of the row transforms (2 .. 32 where the
 * kernel can take it) and of image columns per wave of the hybrid vector pass
 * (1, 2, 4 where they tile the image) is timed with hipEvents over `reps`
 * launches of its kernels (smsm_launch_kernel, after one untimed launch) on
 * the plan's buffers, whatever they hold, and the fastest is kept; the
 * numeric flags the timed launches raise are cleared.  The row shape leaves
 * every result bit for bit the same; the vector pass's shape sets the order
 * of the |r|^2 partial sums, so solves change at rounding level.
 * shape[0] = rows per workgroup, shape[1] = columns per wave (may be NULL).
 * Capture a batch after tuning its plans (a batch keeps the shapes it was
 * captured with).  Synchronous.  Errors: SMSM_E_INVALID for a null plan, reps
 * outside [1, 1000] or no workspace; SMSM_E_DEVICE. */
smsm_status smsm_plan_autotune(smsm_plan* plan, int reps, int* shape, void* stream);

/* ---- operator entry points (one kernel chain each, asynchronous) ------- */

/* y = A x (Fig. 1).  x_dev c128 [L][Ns][n2][n1] -> y_dev c128 [Ns][Nc][n2][n1]
 * (lines a shot does not acquire are written as zero). */
smsm_status smsm_apply_A(smsm_plan* plan, const void* x_dev, void* y_dev, void* stream);

/* x = A^H y.  y_dev c64 [Ns][Nc][n2][n1] (as smsm_solve takes it) -> x_dev c128. */
smsm_status smsm_apply_AH(smsm_plan* plan, const void* y_dev, void* x_dev, void* stream);

/* out = A^H A x, c128 -> c128. */
smsm_status smsm_apply_AHA(smsm_plan* plan, const void* x_dev, void* out_dev, void* stream);

/* G_l = H_l(x_l)^H H_l(x_l) for every slice: x c128 -> G c128 [L][K][K] (Eq. 8-9). */
smsm_status smsm_gram(smsm_plan* plan, const void* x_dev, void* g_dev, void* stream);

/* W_l = (G_l + eps_l I)^(-1/2): G c128 [L][K][K] -> W c128 [L][K][K], by a
 * scaled coupled Newton-Schulz iteration run until ||I - Z Y||_F < 1e-10 or
 * for ns_max_iter steps (condition numbers up to about 1e8 converge within
 * the default cap; a slice still above the tolerance at the cap sets the
 * SMSM_E_NOT_CONVERGED flag of smsm_plan_status).  eps: host [L]; eps_l <= 0
 * gives W_l = 0 (unregularised slice).  Synchronises `stream`. */
smsm_status smsm_weights(smsm_plan* plan, const void* g_dev, const double* eps,
                         void* w_dev, void* stream);

/* Largest eigenvalue of each G_l: G c128 [L][K][K] -> lmax_dev double [L]. */
smsm_status smsm_lambda_max(smsm_plan* plan, const void* g_dev, void* lmax_dev, void* stream);

/* Load weights W c128 [L][K][K] into the plan (used by smsm_apply_reg and
 * smsm_apply_normal until the next solve). */
smsm_status smsm_set_weights(smsm_plan* plan, const void* w_dev, void* stream);

/* out = (lambda/2) sum_l H_l^H(H_l(x_l) W_l) with the loaded weights, c128 -> c128. */
smsm_status smsm_apply_reg(smsm_plan* plan, const void* x_dev, void* out_dev, void* stream);

/* out = N(x) = A^H A x + (lambda/2) sum_l H_l^H(H_l(x_l) W_l), c128 -> c128. */
smsm_status smsm_apply_normal(smsm_plan* plan, const void* x_dev, void* out_dev, void* stream);

/* Root-sum-of-squares image of each slice,
 *     img[l][y][x] = sqrt(sum_i |F^-1(x_{l,i})[y][x]|^2),
 * with F^-1 the centred unitary inverse 2-D DFT of the forward model (Fig. 1):
 * the per-shot images of the reconstructed k-space combined over shots (the
 * paper compares against single-band images without saying how shots are
 * combined; root-sum-of-squares is the reading used).  x_dev c128
 * [L][Ns][n2][n1] (k-space, as smsm_solve writes it with SMSM_FLAG_X_C128) ->
 * img_dev double [L][n2][n1] (image, y-major, x contiguous), caller-owned
 * device memory.  Uses the plan's scratch vectors; asynchronous on `stream`.
 * Errors: SMSM_E_INVALID for null arguments, SMSM_E_DEVICE if a launch fails. */
smsm_status smsm_images_sos(smsm_plan* plan, const void* x_dev, void* img_dev, void* stream);

/* ---- diagnostics ------------------------------------------------------- */

/* Kernels that smsm_launch_kernel can re-run.  CG runs on the hybrid layout
 * (image x, k-space ky; the kx transform is unitary): one CG iteration is
 * COL_NORMAL, BAND_EXTRACT, BAND_CORR and CG_UPDATE (BAND_EXTRACT and
 * BAND_CORR only when lambda > 0 adds the band). */
typedef enum {
    SMSM_KERNEL_COL_NORMAL = 0,  /* x += alpha p and p = r + beta p (the previous step's length and
                                    direction), then per column: SENSE coil loop, image-domain
                                    Hankel term, Re <p, q> partials */
    SMSM_KERNEL_ROWS_INV = 1,    /* kx inverse DFT, natural -> hybrid (Gram and operator entry points) */
    SMSM_KERNEL_ROWS_FWD = 2,    /* kx forward DFT, hybrid -> natural (Gram and the solve's output) */
    SMSM_KERNEL_BAND_CORR = 3,   /* Hankel band correction (rows hybrid, columns and corners natural) */
    SMSM_KERNEL_CG_UPDATE = 4,   /* step length from the Re <p, q> partials, band injection,
                                    r update, |r|^2 partials */
    SMSM_KERNEL_BAND_EXTRACT = 5 /* natural kx columns of p within 2(r-1) of the kx edges */
} smsm_kernel_id;

/*
 * Launch one kernel of the CG iteration `reps` times back to back on the
 * plan's internal buffers (whatever the last solve left there), for timing
 * and profiling.  The plan's vectors are overwritten; call smsm_solve again
 * before reading results.  Asynchronous on `stream`.
 */
smsm_status smsm_launch_kernel(smsm_plan* plan, int kernel_id, int reps, void* stream);

/* Algorithmic cost of one launch of a kernel of smsm_launch_kernel for this
 * plan's geometry: FP64 flops and compulsory HBM bytes (reads + writes). */
smsm_status smsm_kernel_cost(const smsm_plan* plan, int kernel_id, double* flops, double* bytes);

/* Per-launch timing of one kernel inside whatever the plan runs next (a
 * solve, operator chains, smsm_launch_kernel): one launch in every `stride`
 * of `kernel_id` (the first, then every stride-th), up to `capacity` of them,
 * is dispatched with a start/stop event pair (the timestamps of the dispatch
 * itself; nothing is added to the stream, but a timed dispatch starts a few
 * microseconds later, so a stride well above 1 keeps the timed work close to
 * the untimed one).  capacity 0 turns timing off and releases the events.
 * Only SMSM_KERNEL_COL_NORMAL on the fast column pass is supported
 * (otherwise SMSM_E_UNSUPPORTED); the events are created here, never on a
 * solve path.  Errors: SMSM_E_INVALID for a null plan, capacity outside
 * [0, 2^20] or stride < 1, SMSM_E_DEVICE if an event cannot be created. */
smsm_status smsm_kernel_timer_start(smsm_plan* plan, int kernel_id, int capacity, int stride);

/* Waits for the last timed launch, then returns the summed durations (ms) of
 * the launches timed since smsm_kernel_timer_start or the previous read and
 * their count, and starts a new count (the capacity is not renewed: launches
 * past it are not timed).  Errors: SMSM_E_INVALID for null arguments,
 * SMSM_E_DEVICE if an event query fails. */
smsm_status smsm_kernel_timer_read(smsm_plan* plan, double* total_ms, int* launches);

/* ---- learned unrolled solver ------------------------------------------
 *
 * An extension beyond the paper: a learned prior stands in for the Hankel
 * IRLS step.  From x_0 = A^H y, each of n_unroll iterations applies
 *     z = x + s C(x / s),   x <- (A^H A + mu I)^-1 (A^H y + mu z)
 * with C a real CNN over the 2 Ns channels (real and imaginary part of each
 * shot's k-space) of every slice: five 3x3 layers 2Ns -> width -> width ->
 * width -> width -> 2Ns, zero padding, ReLU after the first four, weights
 * shared across iterations; s = sqrt(mean |A^H y|^2).  The network runs in
 * FP32; each data-consistency solve is n_cg CG steps in FP64 warm-started at
 * z.  Training minimises ||x_K - x*||^2 / ||x*||^2 against a reference x*
 * (the plain solver's output) with Adam; its backward pass takes each
 * data-consistency solve as the exact inverse (n_cg CG steps from zero).
 *
 * Parameters (host layout, float32): per layer, weights [co][ci][3][3] then
 * bias [co], layers in order.  The object holds the parameters, gradients,
 * Adam moments and buffers for the plan's geometry, and uses the plan's
 * workspace: the plan must outlive the object and have a workspace bound
 * when the object solves (SMSM_E_INVALID otherwise), and calls on one plan
 * (solver or learned) must not overlap.
 * Requires 2 Ns to be a multiple of 4 (SMSM_E_UNSUPPORTED otherwise).
 * Vectors: y_dev c64 [Ns][Nc][n2][n1]; x_dev, xt_dev c128 [L][Ns][n2][n1]. */
typedef struct smsm_learned smsm_learned;

/* width: hidden channels (multiple of 8, 8..256); n_unroll, n_cg >= 1;
 * mu > 0; params_host: smsm_learned_param_count() floats of initial
 * parameters.  Synchronous. */
smsm_status smsm_learned_create(smsm_plan* plan, int width, int n_unroll, int n_cg, double mu,
                                const float* params_host, smsm_learned** out);
/* Frees the object (not the plan).  Null is a no-op. */
smsm_status smsm_learned_destroy(smsm_learned* net);
/* Number of float parameters; 0 for null. */
long smsm_learned_param_count(const smsm_learned* net);
/* Copies the parameters to / from host memory (synchronous; setting them
 * also resets the Adam state). */
smsm_status smsm_learned_get_params(smsm_learned* net, float* params_host);
smsm_status smsm_learned_set_params(smsm_learned* net, const float* params_host);

/* Weight format of the network's convolutions.  on = 0 (default): FP32
 * weights and accumulation on the vector ALU.  on = 1: BF16 weights (rounded
 * to nearest even from the FP32 parameters, refreshed after every change) on
 * the BF16 matrix cores, FP32 activations entering each product in three
 * BF16 parts (products exact to FP32), FP32 accumulation.  on = 2: the BF16
 * network on the matrix cores: BF16 weights, every convolution input (the
 * network input and the hidden activations, stored as BF16 values) and the
 * gradient entering each backward-data convolution rounded to BF16, FP32
 * accumulation and biases; weight gradients from the FP32 output gradients
 * and the stored activations.  Gradients are taken with respect to the BF16
 * weights and applied to the FP32 parameters.  Errors: SMSM_E_INVALID for a
 * null object or on outside 0..2.  Synchronous. */
smsm_status smsm_learned_set_bf16(smsm_learned* net, int on);

/* The network alone: out = C(in), in_dev and out_dev float [L][2Ns][n2][n1]. */
smsm_status smsm_learned_cnn_forward(smsm_learned* net, const void* in_dev, void* out_dev, void* stream);
/* Gradients of sum(gout * C(in)): gin_dev (same layout) and all parameter
 * gradients into grads_host (param_count floats).  Synchronous. */
smsm_status smsm_learned_cnn_backward(smsm_learned* net, const void* in_dev, const void* gout_dev, void* gin_dev,
                                      float* grads_host, void* stream);

/* x = the unrolled solver's output for measurement y.  Asynchronous. */
smsm_status smsm_learned_solve(smsm_learned* net, const void* y_dev, void* x_dev, void* stream);
/* Loss against xt and the gradients of every parameter (into grads_host
 * when it is not null); the parameters do not change.  Synchronous. */
smsm_status smsm_learned_gradients(smsm_learned* net, const void* y_dev, const void* xt_dev, double* loss,
                                   float* grads_host, void* stream);
/* One Adam step (b1 0.9, b2 0.999, eps 1e-8) on the gradients of y, xt with
 * learning rate lr > 0; *loss is the loss before the step.  Synchronous. */
smsm_status smsm_learned_train_step(smsm_learned* net, const void* y_dev, const void* xt_dev, double lr,
                                    double* loss, void* stream);
/* *res = ||A x - y|| (the data-consistency residual by which a caller falls
 * back to the plain solver).  Synchronous. */
smsm_status smsm_learned_residual(smsm_learned* net, const void* x_dev, const void* y_dev, double* res,
                                  void* stream);

/* The learned solve with the plain IRLS solve as its fallback: x = the
 * learned solve of y and r_l = ||A x - y||.  The reference residual r_p is
 * res_ref when res_ref > 0 (e.g. the plain solver's residual on an earlier
 * input of the slice group), else that of the plain solve of y, run here with
 * the plan's parameters.  When r_l > ratio * r_p, x is replaced by the plain
 * solve (run here if it has not been) and *fell_back = 1, else 0.
 * res_out[0] = r_l, res_out[1] = r_p.  x_dev c128 [L][Ns][n2][n1].  The plain
 * solve uses the plan's workspace and one of the object's vectors.  Errors:
 * SMSM_E_INVALID for null arguments or ratio <= 0; else as the solves.
 * Synchronous. */
smsm_status smsm_learned_solve_fallback(smsm_learned* net, const void* y_dev, void* x_dev, double ratio,
                                        double res_ref, double* res_out, int* fell_back, void* stream);

/* ---- augmented-Lagrangian solve -----------------------------------------
 *
 * The paper's own solver of Eq. 10 (Theory, the paragraph after Eq. 10;
 * Methods, "Reconstruction"; its steps are left to a cited paper, so they are
 * taken from the method): split Z_l = H_l(x_l) with scaled duals U_l and
 * repeat n_outer times
 *     x   <- n_cg CG steps, warm-started, on
 *            (A^H A + (beta/2) c) x = A^H y + (beta/2) sum_l H_l^H(Z_l - U_l)
 *     Z_l <- singular-value soft thresholding of M_l = H_l(x_l) + U_l at
 *            tau = lambda / beta,   U_l <- M_l - Z_l
 * from x0 = A^H y, Z_l = H_l(x0), U_l = 0 (c = H_l^H H_l, the number of valid
 * patches holding a sample).  The thresholding is M_l f(M_l^H M_l) with
 * f(s^2) = max(1 - tau/s, 0), formed from the K x K Gram on the FP64 matrix
 * cores (a scaled Newton-Schulz sign iteration for the projector on the
 * singular values above tau, then the coupled iteration of the weights);
 * singular values within about 1e-14 ||M^H M - tau^2 I||_F / tau^2 of tau
 * relative may be placed on either side, where f is that close to zero.
 * A Newton-Schulz step that does not converge sets the SMSM_E_NOT_CONVERGED
 * flag of smsm_plan_status. */
typedef struct smsm_al smsm_al;

typedef struct {
    double  lambda;   /* lambda of Eq. 10, > 0 (the plan's own lambda is not used) */
    double  beta;     /* penalty weight of the split, > 0 */
    int32_t n_outer;  /* outer iterations, >= 1 */
    int32_t n_cg;     /* CG steps of each x-step, >= 0 */
    int32_t n_sign;   /* steps of the sign iteration (0: as many as the 1e-14 resolution needs, about 43) */
    uint32_t flags;   /* SMSM_FLAG_X_C128: x written complex128 */
} smsm_al_params;

/* Create the solver's state on a plan (same device): the duals in two
 * buffers of [L][K][stride] complex128 (stride = smsm_al_dual_stride >= the
 * (n1-r+1)(n2-r+1) patch anchors; about 1.2 GB for 256 x 256, 3 slices, 4
 * shots, 7 x 7), six vectors of [L][Ns][n2][n1] complex128, Gram partials and
 * K x K matrices, allocated here (smsm_al_device_bytes) and released by
 * smsm_al_destroy.  The plan must outlive it.  Errors: SMSM_E_INVALID for
 * null arguments or parameters out of range, SMSM_E_NOMEM, SMSM_E_DEVICE. */
smsm_status smsm_al_create(smsm_plan* plan, const smsm_al_params* params, smsm_al** out);

/* Release the state (synchronises the device first).  NULL is a no-op. */
smsm_status smsm_al_destroy(smsm_al* al);

/* Device bytes the state holds. */
size_t smsm_al_device_bytes(const smsm_al* al);

/* The solve: y_dev c64 [Ns][Nc][n2][n1] -> x_dev c64 (c128 with
 * SMSM_FLAG_X_C128) [L][Ns][n2][n1].  Runs the operator chains in the plan's
 * workspace (SMSM_E_INVALID without one); allocates nothing; asynchronous on
 * `stream`.  The state and the plan must not be used concurrently. */
smsm_status smsm_al_solve(smsm_al* al, const void* y_dev, void* x_dev, void* stream);

/* Copy the scaled duals U_l of the last solve into u_dev: c128
 * [L][K][stride], entry [l][k][p] = U_l[p][k] for patch anchor
 * p = p2 (n1-r+1) + p1 < (n1-r+1)(n2-r+1) and column k = (i r + b2) r + b1
 * (zero for p beyond the anchors).  At a solution, Y_l = (beta/lambda) U_l
 * certifies optimality for Eq. 10: A^H(A x - y) + (lambda/2) sum_l H_l^H(Y_l) = 0,
 * ||Y_l||_2 <= 1 and Re<Y_l, H_l(x_l)> = ||H_l(x_l)||_*.  Asynchronous. */
smsm_status smsm_al_dual(smsm_al* al, void* u_dev, void* stream);

/* Row stride (entries) of the dual layout; 0 for a null state. */
long smsm_al_dual_stride(const smsm_al* al);

#ifdef __cplusplus
}
#endif
#endif /* SMSM_H */
