/*
 * bf.h -- C ABI of the MI355X (gfx950) Fourier-kernel bilateral filter.
 *
 * Method: Ghosh & Chaudhury, "On Fast Bilateral Filtering using Fourier
 * Kernels".  The range kernel phi is fitted on {0..T} by the cosine series
 * phi_K(t) = d_0 + sum_{k=1..K} d_k cos(k w t), w = pi / T (eq. (6)), with the
 * progressive least-squares scheme of Algorithm 2 (Sec. 3); the filter then
 * evaluates eq. (9) -- the bilateral filter of eq. (1) with phi replaced by
 * phi_K -- through the shiftable decomposition of Algorithm 1 (Sec. 2): each
 * harmonic k modulates the image into cos(k w f), sin(k w f), f cos(k w f) and
 * f sin(k w f), smooths the four planes with the spatial kernel, demodulates
 * at the output pixel with the conjugate phase and accumulates numerator and
 * denominator, which are divided at the end.
 *
 * Conventions used by every entry point:
 *   - All functions are extern "C"; no C++ exception crosses the ABI.
 *   - Return value: BF_OK (0), a positive warning, or a negative error code.
 *     On an error nothing has been enqueued and no output was written;
 *     bf_last_error() returns a text for the calling thread.
 *   - Images are row-major float32 gray levels with a row pitch counted in
 *     elements (pitch >= width).  Pixel values are expected in [0, T]; the
 *     accuracy guarantee of eq. (12) assumes that range.
 *   - Device pointers (src, dst, workspace) are owned by the caller.  The
 *     library never allocates, frees or synchronises caller memory or the
 *     caller's stream; work is enqueued on `hip_stream` (a hipStream_t, NULL
 *     for the null stream) and runs asynchronously.  Host arrays passed in
 *     (phi_table, d) are read before the call returns.
 *   - Borders use half-sample symmetric extension (f(-1) = f(0),
 *     f(-2) = f(1), ...), which requires W < min(height, width).
 *   - The spatial kernel is the Gaussian of eq. (2), exp(-(x^2+y^2)/(2 s^2)),
 *     or a box (w = 1), on the window [-W, W]^2 (Sec. 1); it is scaled to unit
 *     sum, which does not change eq. (1) or eq. (9).
 */
#ifndef BF_H
#define BF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define BF_OK 0
#define BF_FIT_NOT_CONVERGED 1  /* warning: the fit stopped at K_max with E > eps; outputs are valid */
#define BF_E_INVALID (-1)       /* an argument violates the contract stated below */
#define BF_E_DEVICE (-2)        /* a HIP runtime call failed (text in bf_last_error) */
#define BF_E_WORKSPACE (-4)     /* workspace NULL or smaller than bf_workspace_bytes() */
#define BF_E_UNSUPPORTED (-5)   /* valid for the method but beyond this library's limits */

/* ---- limits of this implementation ------------------------------------- */
#define BF_MAX_T 1024           /* half-period T (phase table of 2T entries per workgroup) */
#define BF_MAX_K 255            /* harmonics usable by the filter (the fit accepts K_max <= T) */
#define BF_MAX_W 64             /* window half-width */

/* ---- enums -------------------------------------------------------------- */
typedef enum {
  BF_RANGE_GAUSSIAN = 0,     /* eq. (3): phi(t) = exp(-t^2 / (2 sigma_r^2)) */
  BF_RANGE_EXPONENTIAL = 1,  /* phi(t) = exp(-|t| / sigma_r) */
  BF_RANGE_TABLE = 2         /* phi given by its samples phi(0..T) (symmetric kernel) */
} bf_range_kind;

typedef enum {
  BF_SPATIAL_GAUSSIAN = 0,   /* eq. (2) on [-W, W]^2 */
  BF_SPATIAL_BOX = 1         /* w = 1 on [-W, W]^2 */
} bf_spatial_kind;

typedef enum {
  BF_PLANES_FP32 = 0,        /* planes, smoothing and accumulation in float32 */
  BF_PLANES_FP16 = 1,        /* planes and smoothing operands in float16 (RNE), float32 accumulation */
  BF_PLANES_BF16 = 2         /* modulated planes and row-pass weights in bfloat16 (RNE); the
                                row-smoothed planes and column-pass weights in float16 (RNE);
                                float32 accumulation */
} bf_planes;

/* flags of bf_job.flags */
#define BF_FLAG_INTEGER_INPUT 1 /* caller guarantees every pixel is an integer in [0, f_max]
                                   (f_max = T unless set): enables the exact table-only phase
                                   path.  With the flag set, a pixel outside that contract makes
                                   the outputs whose windows contain it unspecified. */
#define BF_FLAG_OFFSETS16 2     /* schedule only (no result bit changes): with 16-bit planes on
                                   integer images, stage 16-bit gray-level table offsets instead
                                   of 32-bit table addresses (the latter are used when the gray
                                   levels fit 256 table entries and the tile fits LDS).  In a
                                   batched call or plan it applies to the whole kernel class of
                                   the job. */

/*
 * bf_fit_coeffs -- Algorithm 2 (Sec. 3), on the host, in float64.
 *
 * Samples b = phi(0..T) (eq. (3), the exponential, or phi_table), then adds
 * the columns cos(n w t), n = 0, 1, 2, ... one at a time, growing a thin QR
 * factorisation by modified Gram-Schmidt and solving R d = Q^T b by
 * back-substitution, until E = ||b - A d||_2 <= eps (eq. (7)/(8)) or the
 * highest harmonic reaches K_max.  eps == 0 therefore gives exactly K_max
 * harmonics.  (The column added when the fit has N columns is harmonic
 * N - 1; the printed counts of Tables 3 and 4 are column counts K + 1.)
 *
 *   kind, sigma_r   range kernel; sigma_r > 0 unless kind == BF_RANGE_TABLE
 *   phi_table       host array of T+1 samples phi(0..T); required iff TABLE
 *   T               half-period, 1 <= T <= BF_MAX_T
 *   eps             tolerance on ||b - A d||_2, eps >= 0
 *   K_max           cap on the highest harmonic, 0 <= K_max <= T
 *   d               host output, room for K_max + 1 doubles: d_0..d_K
 *   K               host output: highest harmonic used
 *   err_l2, err_max optional host outputs (may be NULL): ||b - A d||_2 and
 *                   max_t |phi(t) - phi_K(t)| on {0..T} (eq. (10))
 * Returns BF_OK, BF_FIT_NOT_CONVERGED (K == K_max and E > eps; d is the
 * K_max fit), or BF_E_INVALID.  Host-only: needs no GPU.
 */
int bf_fit_coeffs(bf_range_kind kind, double sigma_r, const double* phi_table, int T,
                  double eps, int K_max, double* d, int* K, double* err_l2, double* err_max);

/*
 * One filtering job (one image).  Fields:
 *   src, dst        device pointers; dst must not overlap src
 *   height, width   image size in pixels, >= 1
 *   src_pitch, dst_pitch   row pitch in elements, >= width
 *   spatial         BF_SPATIAL_GAUSSIAN or BF_SPATIAL_BOX
 *   sigma_s         Gaussian spatial scale (> 0); ignored for the box
 *   W               window half-width, 0 <= W <= BF_MAX_W and W < min(height, width);
 *                   W < 0 with the Gaussian selects W = ceil(3 sigma_s) (Sec. 1)
 *   range, sigma_r, phi_table, T, eps, K_max   as for bf_fit_coeffs
 *   d, K            optional host coefficients d_0..d_K of phi_K; when d != NULL
 *                   the fit is skipped and range/sigma_r/phi_table/eps/K_max are
 *                   not used (T still sets w = pi / T)
 *   flags           BF_FLAG_* bits
 *   f_max           largest pixel value, 0 <= f_max <= BF_MAX_T; 0 means T.  Pixels
 *                   lie in [0, f_max] while T only has to bound the differences
 *                   |f(i - j) - f(i)| inside each window (the local dynamic range of
 *                   Sec. 3, see bf_dynamic_range), so T may be smaller than f_max.
 *                   With BF_FLAG_INTEGER_INPUT the gray-level tables cover 0..f_max.
 */
typedef struct bf_job {
  const float* src;
  float* dst;
  int height, width;
  int src_pitch, dst_pitch;
  bf_spatial_kind spatial;
  double sigma_s;
  int W;
  bf_range_kind range;
  double sigma_r;
  const double* phi_table;
  int T;
  double eps;
  int K_max;
  const double* d;
  int K;
  int flags;
  int f_max;
} bf_job;

/*
 * bf_workspace_bytes -- device workspace that bf_filter_batched needs for
 * these jobs and plane precision: the job table (one descriptor per image:
 * pointers, sizes, W, K, T, the unit-sum spatial profile of eq. (2) and
 * d_0..d_K) followed by the work items (one per output tile).  Runs the fits
 * of jobs without d.  Returns (size_t)-1 when an argument is invalid
 * (bf_last_error() says which).
 */
size_t bf_workspace_bytes(const bf_job* jobs, int n_jobs, bf_planes prec);

/*
 * bf_filter -- eq. (9) for one image via Algorithm 1 (Sec. 2), on the GPU.
 * Fits the range kernel first unless job->d is given (Algorithm 2), then runs
 * one fused kernel over the image's output tiles: modulation by cos/sin of
 * k w f (eq. (4)-(6), k = 0..K), separable smoothing of the planes with the
 * spatial kernel (row then column pass), demodulation with d_k, accumulation
 * of numerator and denominator of eq. (9) and the final division.
 *   prec        plane format (BF_PLANES_*); accumulation is float32
 *   workspace, ws_bytes   not used by the single-image path (its descriptor
 *               travels as a kernel argument); may be NULL / 0
 *   hip_stream  hipStream_t to enqueue on (NULL: the null stream)
 * Asynchronous: returns after the enqueue; dst is written when the stream
 * reaches the kernel.  Returns BF_OK, BF_FIT_NOT_CONVERGED (filter ran with
 * K = K_max), BF_E_INVALID, BF_E_UNSUPPORTED or BF_E_DEVICE.  dst is not
 * touched on a negative status.
 */
int bf_filter(const bf_job* job, bf_planes prec, void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * bf_filter_batched -- eq. (9) for n_jobs independent images of any sizes,
 * each with its own spatial window, range kernel and K.  Every job is
 * resolved on the host first (fits included); the images are cut into output
 * tiles, the tiles grouped by kernel (window class, kernel family; each group
 * with its own tile height), and each group runs as ONE launch of a
 * persistent kernel whose workgroups take tiles round-robin from a list
 * ordered by decreasing cost 4K+1.  No job's dst may overlap another job's
 * src or dst (jobs may share a src).  The job table and tile list are copied into
 * `workspace` (device memory of at least bf_workspace_bytes() bytes,
 * 16-byte aligned, owned by the caller) on `hip_stream`, asynchronously, from
 * library-owned pinned memory; the caller must not reuse the workspace for
 * anything else until the stream has passed the launches.
 * Inside a stream capture the table copy becomes a copy node of the
 * caller's graph; its pinned staging buffer is then reserved for that graph
 * and never reused.
 * Returns the first error found (nothing is enqueued then), else
 * BF_FIT_NOT_CONVERGED if any job's fit stopped at K_max, else BF_OK.
 */
int bf_filter_batched(const bf_job* jobs, int n_jobs, bf_planes prec,
                      void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * bf_filter_batched_noalloc -- bf_filter_batched for callers that cannot
 * allocate memory (code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same jobs, kernels and results, but
 * the job table and tile list go into a fixed device array of the library
 * (BF_NOALLOC_SCRATCH_BYTES on each GPU, held until the process ends)
 * instead of a caller workspace.  Nothing is allocated: no device, pinned or
 * managed memory, no staging buffer.  The table is copied from ordinary host
 * memory with hipMemcpyAsync on `hip_stream`, then the class launches follow
 * on the same stream.  The caller still owns src and dst.
 *   Limit: the table (bf_workspace_bytes() of the same jobs) must fit
 *   BF_NOALLOC_SCRATCH_BYTES, else BF_E_UNSUPPORTED and nothing is enqueued.
 *   Every call on one GPU uses that GPU's single array: calls that overlap in
 *   time on one GPU (several host threads, or several streams whose work
 *   overlaps) race on it and must not be made; calls in one stream order are
 *   safe.  The array keeps the last call's table, which the next call
 *   overwrites whole before its kernels read it.
 * Returns as bf_filter_batched.
 */
#define BF_NOALLOC_SCRATCH_BYTES (4u << 20)
int bf_filter_batched_noalloc(const bf_job* jobs, int n_jobs, bf_planes prec, void* hip_stream);

/*
 * Plans: bf_filter_batched split into its host part (done once) and its
 * device part (repeated), for callers that filter the same buffers again and
 * again (video frames written into the same src buffers, serving loops).
 *
 * bf_plan_create  resolves and fits every job and builds the tile list, as
 *                 bf_filter_batched does; no GPU call.  *plan receives an
 *                 opaque handle (NULL on error).  Returns BF_OK,
 *                 BF_FIT_NOT_CONVERGED, BF_E_INVALID or BF_E_UNSUPPORTED.
 *                 The plan keeps the jobs' src/dst pointers: they must stay
 *                 valid while the plan is launched.
 * bf_plan_workspace_bytes  workspace the plan needs ((size_t)-1 for NULL).
 * bf_plan_upload  copies the job table into `workspace` on `hip_stream`
 *                 (asynchronous, as in bf_filter_batched) and binds the plan
 *                 to that workspace and to the stream's device.
 * bf_plan_launch  enqueues the plan's launches on `hip_stream` (same device
 *                 as the upload).  use_graph == 0: one launch per group,
 *                 in order.  use_graph != 0: the first call captures the
 *                 launches into a HIP graph (groups as independent kernel
 *                 nodes, which may run concurrently) on streams of the
 *                 library, later calls replay it with hipGraphLaunch; the
 *                 graph holds kernel nodes only.  No allocation and no copy
 *                 after the first graph launch.  Calls on one plan must not
 *                 overlap in time from several host threads.
 * bf_plan_destroy waits for the last graph replay of the plan to finish,
 *                 then frees the plan (NULL is ignored).
 */
typedef struct bf_plan bf_plan;
int bf_plan_create(const bf_job* jobs, int n_jobs, bf_planes prec, bf_plan** plan);
size_t bf_plan_workspace_bytes(const bf_plan* plan);
int bf_plan_upload(bf_plan* plan, void* workspace, size_t ws_bytes, void* hip_stream);
int bf_plan_launch(bf_plan* plan, void* hip_stream, int use_graph);
void bf_plan_destroy(bf_plan* plan);

/*
 * bf_plan_tune    autotuner: for every kernel class of an uploaded plan,
 *                 times `reps` launches of each tile height the class's
 *                 jobs support (32 and 64 rows; 96 and 128 where the tile
 *                 fits: 16-bit planes up to W = 48, fp32 planes on integer
 *                 images; 144 for 16-bit planes up to W = 48) with
 *                 both grid modes (a persistent grid sized by occupancy, or
 *                 one workgroup per tile), keeps the fastest, re-uploads the
 *                 table and remembers the choice for later plans of this
 *                 process whose classes match (plane format, window class,
 *                 kernel family, round(log2(pixels))).  Synchronises
 *                 `hip_stream` (it reads events); writes the jobs' dst
 *                 buffers.  The output of a plan does not depend on these
 *                 choices (same per-tile arithmetic).  1 <= reps <= 1000.
 * bf_plan_describe  writes a JSON description of the plan's classes (window
 *                 class, family, tile rows and columns, grid mode, items,
 *                 jobs, tuned) into buf (truncated to len - 1 characters,
 *                 NUL-terminated); returns the full length, or BF_E_INVALID.
 */
int bf_plan_tune(bf_plan* plan, void* hip_stream, int reps);
int bf_plan_describe(const bf_plan* plan, char* buf, size_t len);

/*
 * The tuner's remembered choices, shared by the process, can be kept across
 * processes in a small text file ("bf-tune 1", then one line per entry:
 * planes, window class, family, round(log2(pixels)), tile rows, grid mode).
 * bf_tune_save   writes every entry; BF_OK or BF_E_INVALID (path).
 * bf_tune_load   merges a file's entries (a file's entry replaces the same
 *                key); returns the number of entries read (>= 0), or
 *                BF_E_INVALID for an unreadable or malformed file (nothing
 *                merged then).
 * bf_tune_clear  forgets every entry.
 * Plans created afterwards start from the remembered geometry.  Host-only.
 */
int bf_tune_save(const char* path);
int bf_tune_load(const char* path);
void bf_tune_clear(void);

/*
 * bf_dynamic_range -- the dynamic range T of Sec. 3 measured on the image:
 * the largest |f(i - j) - f(i)| over all pixels i and offsets j in
 * [-W, W]^2, i.e. the smallest T with which eq. (1) evaluates the range
 * kernel only on [-T, T]; rounded up to an integer (0 for a constant image).
 * The borders need no folding: under the half-sample symmetric extension a
 * folded neighbour is a pixel no farther away than its offset, so it adds no
 * new pair.  A smaller T needs fewer harmonics for the same tolerance
 * (Algorithm 2 with w = pi / T); pass it as bf_job.T with f_max set to the
 * largest pixel value.
 *   src, height, width, src_pitch   device float32 image, pitch in elements
 *   W           window half-width, 0 <= W <= BF_MAX_W
 *   T_out       device int that receives the result
 *   workspace   device memory of bf_dynamic_range_workspace_bytes(height,
 *               width) bytes (4 B per pixel plus one float per 64x64 tile),
 *               16-byte aligned
 *   hip_stream  stream to enqueue on (three launches; asynchronous)
 * Returns BF_OK, BF_E_INVALID, BF_E_WORKSPACE or BF_E_DEVICE.
 */
size_t bf_dynamic_range_workspace_bytes(int height, int width);
int bf_dynamic_range(const float* src, int height, int width, int src_pitch, int W, int* T_out,
                     void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * bf_filter_recursive -- eq. (9) for one image with every spatial
 * convolution of Algorithm 1 done by Deriche's recursive Gaussian, the
 * constant-time smoothing Sec. 2 cites (after eq. (5)): exp(-x^2 / 2 sigma_s^2)
 * fitted by two damped cosine/sine pairs, run as a causal plus an
 * anti-causal fourth-order recursion along rows, then along columns, over a
 * half-sample symmetric extension of about 16 sigma_s + 8 samples (where the
 * kernel's tail is below 1e-12 of its peak), with unit
 * sum.  Its run time does not grow with sigma_s beyond that extension; its
 * result differs from bf_filter's truncated Gaussian of eq. (2) by the
 * difference of the two spatial kernels (a variant, not the same filter).
 *   job         as for bf_filter, except: spatial must be BF_SPATIAL_GAUSSIAN,
 *               0 < sigma_s <= 256, W is not used, height x max(src_pitch,
 *               width) below 2^28 elements (BF_E_UNSUPPORTED otherwise);
 *               with BF_FLAG_INTEGER_INPUT the row pass takes cos and sin of
 *               k w f from a float32 table of pi m / T, m = k f mod 2T, and
 *               the column pass from a float64 one (same contract as for
 *               bf_filter: pixels are gray levels 0..f_max, others are
 *               clamped into that range), otherwise phases are computed per
 *               pixel in float64
 *   workspace   device memory of at least bf_recursive_workspace_bytes(job)
 *               bytes (16 (K + 1) + 16 ceil((K + 1) / 4) per pixel: the
 *               float32 row-smoothed planes of every harmonic and the float64
 *               shares of numerator and denominator of every group of four
 *               harmonics), 256-byte aligned, owned by the
 *               caller, not overlapping src or dst; in use until the stream
 *               has passed the launches
 *   hip_stream  stream to enqueue on: three launches, asynchronous
 * Returns BF_OK, BF_FIT_NOT_CONVERGED, BF_E_INVALID, BF_E_UNSUPPORTED,
 * BF_E_WORKSPACE or BF_E_DEVICE; nothing is enqueued on a negative status.
 * bf_recursive_workspace_bytes runs the fit of a job without d and returns
 * (size_t)-1 for an invalid job (bf_last_error() says which).
 */
size_t bf_recursive_workspace_bytes(const bf_job* job);
int bf_filter_recursive(const bf_job* job, void* workspace, size_t ws_bytes, void* hip_stream);

/* Thread-local text describing the last non-OK status of this thread. */
const char* bf_last_error(void);

/*
 * Environment variables (schedule only: none of them changes a result bit;
 * both are read when a plan or batched call is created, never per launch).
 *   BF_TILE_ROWS=32|64|96|128|144  preferred output-tile height of new plans and
 *                  batched calls (a class takes the tallest height not above
 *                  it that all its jobs support); read at plan creation.
 *   BF_BATCH_GRID=items|<n>    workgroups per class launch: one per tile, or
 *                  a fixed n; unset = a persistent grid sized by occupancy;
 *                  read at plan creation.
 * While either is set, remembered tuner choices are not
 * applied at plan creation; bf_plan_tune still times and sets the geometry.
 */

#ifdef __cplusplus
}
#endif

#endif /* BF_H */
