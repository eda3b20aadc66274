/*
 * ddh.h -- C ABI of the Dynamic DH-MBIR per-frame EM step on AMD MI355X (gfx950).
 *
 * Method: arXiv 2305.03284, "Dynamic DH-MBIR for Phase-Error Estimation from
 * Streaming Digital-Holography Data".  Model (Forward Model section, Eq. (1)):
 *   y = A_phi g + w,  A_phi = D_a D(exp(j phi)) F Gamma,  g ~ CN(0, diag r),
 * F the unitary 2D DFT, Gamma taken as identity.  One frame of the streaming
 * loop (Dynamic DH-MBIR section, Fig. 1) is
 *   y <- Normalize(y)                          (Eq. (4))
 *   phi <- RemoveTipTilt(phi)                  (least-squares plane removal)
 *   r <- (1-lambda) r + lambda alpha |A_phi^H y|^2    (Eq. (3))
 *   n_k times: (r, phi) <- EM(r, phi; y)       (DH-MBIR section)
 * and WriteData(n, r, phi) is ddh_get_phase / ddh_get_reflectance.
 *
 * Conventions for every entry point:
 *   - Arrays are N x N, row-major, C-contiguous.  Complex data is interleaved
 *     float pairs (re, im) ("complex64").  Device pointers point into HIP
 *     device memory on the current device; host pointers into host memory.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on it unless stated otherwise.
 *   - Return value: DDH_OK (0) or a negative DDH_E* code; ddh_error_string()
 *     names it.  Argument checks happen before any device work, so an
 *     invalid call enqueues nothing and leaves all state unchanged.
 *   - The library owns every device buffer it allocates (stream state,
 *     workspace, graphs); the caller owns y and all output buffers.
 *   - A stream handle is not thread-safe: use it from one host thread at a
 *     time.  Different handles are independent.
 */
#ifndef DDH_H
#define DDH_H

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define DDH_OK       0
#define DDH_EINVAL  (-1)   /* null pointer, unsupported N, parameter out of range */
#define DDH_ENOMEM  (-2)   /* device allocation refused                            */
#define DDH_EDEVICE (-3)   /* a HIP runtime call failed                            */
#define DDH_EDATA   (-4)   /* frame rejected: ||y - mean(y)|| = 0 or non-finite    */
#define DDH_ESTATE  (-5)   /* handle destroyed, or batch/stream mismatch           */

typedef struct ddh_stream_s* ddh_stream_t;
typedef struct ddh_batch_s* ddh_batch_t;

/* Algorithm parameters (one set per stream).
 *   N               grid size; one of 64, 128, 256, 512 (paper: N = 256).
 *   pupil_diameter  circular aperture a (diagonal of D_a) of this diameter in
 *                   pixels, centred at ((N-1)/2, (N-1)/2): pixel (i, j) is in
 *                   the pupil iff (2i-N+1)^2 + (2j-N+1)^2 <= diameter^2.
 *                   0 < diameter <= N*sqrt(2).  Used when ddh_init_stream
 *                   gets no aperture array.
 *   lambda, alpha   weights of Eq. (3), each in [0, 1] (paper: 0.45, 0.025).
 *   n_k             EM iterations per frame, >= 1 (Fig. 1; paper: 1).
 *   sigma_w2        noise variance of the normalised data, > 0.
 *   qg_p, qg_q, qg_T, qg_sigma
 *                   QGGMRF prior on r: rho(d) = |d|^p/(p s^p) / (1 + |d/(T s)|^(p-q)),
 *                   1 <= q <= p <= 2, T > 0, s = qg_sigma > 0.
 *   beta_phi        Gaussian-MRF weight on phi, >= 0:
 *                   beta * sum over 8-neighbour pupil pairs of b_ij (phi_i - phi_j)^2,
 *                   b_ij = 1/6 (edge) or 1/12 (diagonal).
 *   r_floor         positivity floor on r, > 0.
 */
typedef struct {
    int   N;
    float pupil_diameter;
    float lambda;
    float alpha;
    int   n_k;
    float sigma_w2;
    float qg_p;
    float qg_q;
    float qg_T;
    float qg_sigma;
    float beta_phi;
    float r_floor;
} ddh_params;

/* Fill *p with defaults for grid size N: diameter N, lambda 0.45, alpha 0.025,
 * n_k 1, sigma_w2 0.1, QGGMRF (2, 1.2, 0.1, 0.2), beta_phi 0.5, r_floor 1e-8. */
int ddh_default_params(int N, ddh_params* p);

/* Create a stream: r <- 0, phi <- 0, n <- 0 (Fig. 1: the loop starts from the
 * zero state).
 *   aperture  the camera aperture a, the diagonal of D_a in the operator
 *             A_phi = D_a D(exp(j phi)) F Gamma (Forward Model section): N*N
 *             floats, row-major, in host or device memory, each 0 or 1
 *             (binary: a pixel is measured or not); read during the call
 *             only.  RemoveTipTilt, Normalize's consumers, the phase update
 *             (which runs on aperture pixels only, with prior neighbours in
 *             the aperture) and the diagnostics all use it.  NULL: the circle
 *             of p->pupil_diameter described above (p->pupil_diameter is
 *             ignored when an array is given).
 * Allocates the per-stream device state and workspace (about 45 bytes per
 * pixel; ddh_stream_bytes) on the current device and zeroes r and phi on
 * hip_stream.  The first stream of a given N and pupil diameter on a device
 * also creates that circle's aperture table (1 byte per pixel), which the
 * library keeps, like its twiddle table, until the process ends; a stream
 * given an array keeps its own table.
 * Errors: DDH_EINVAL (p or out NULL, parameter out of range, an aperture
 * value other than 0 or 1, an aperture with no pixel, or one whose pixels
 * all lie on one line so that the plane of RemoveTipTilt is not determined;
 * these checks happen before any device work), DDH_ENOMEM, DDH_EDEVICE.  On
 * error *out is left unchanged. */
int ddh_init_stream(const ddh_params* p, const float* aperture, void* hip_stream, ddh_stream_t* out);

/* Release a stream and its device memory.  Synchronises the device first.
 * Destroying NULL is DDH_EINVAL.  The handle must not be used afterwards. */
int ddh_destroy_stream(ddh_stream_t s);

/* One frame of the DDH-MBIR loop (Fig. 1 body): Normalize (Eq. (4)),
 * RemoveTipTilt, the r initialisation of Eq. (3), then n_k EM iterations.
 * y: device pointer, N*N complex64, read-only, must stay valid until the
 * stream reaches this step (no pointer is kept afterwards).  If the frame is
 * rejected on the device (||y - mean|| zero or non-finite) the state is left
 * unchanged and the next ddh_status() returns DDH_EDATA.  Increments n.
 * The launches are eager; a stream created while the environment variable
 * DDH_SINGLE_GRAPH is "1" replays them as a HIP graph instead (same results,
 * measured slower for one stream). */
int ddh_step(ddh_stream_t s, const void* y, void* hip_stream);

/* One EM iteration EM(r, phi; y) of the plain DH-MBIR loop (DH-MBIR
 * section): Normalize y, then E-step, r M-step, phi M-step, with no
 * RemoveTipTilt and no Eq. (3) initialisation.  Same y contract as ddh_step. */
int ddh_em(ddh_stream_t s, const void* y, void* hip_stream);

/* Conventional single-shot DH-MBIR (DH-MBIR section): `iters` EM iterations
 * on the one frame y, with a bootstrap reset of r every `reset_every`
 * iterations (the paper's bootstrap resets every 200).  Iteration it
 * (0-based) with it % reset_every == 0 is a reset: the frame prologue
 * (Normalize, RemoveTipTilt), the Eq. (3) initialisation r = (1 - lambda) r
 * + lambda alpha |b|^2 with the stream's lambda (a stream made with lambda = 1
 * replaces r by the back-projection estimate, as the bootstrap does), then one
 * EM iteration; every other iteration is ddh_em.  The stream's n_k is not
 * used.  Continues from the stream's state (set r = phi = 0 with
 * ddh_set_state for the paper's cold start); the frame count grows by one.
 * Eager launches on hip_stream; same y contract as ddh_step.  DDH_EINVAL for
 * iters < 0 or reset_every < 1. */
int ddh_mbir(ddh_stream_t s, const void* y, int iters, int reset_every, void* hip_stream);

/* WriteData (Fig. 1): copy the current phase phi (radians, unwrapped, zero
 * off the pupil) or reflectance r (Normalize units) into out, a device
 * pointer to N*N floats, on hip_stream.  Synchronise before reading. */
int ddh_get_phase(ddh_stream_t s, float* out, void* hip_stream);
int ddh_get_reflectance(ddh_stream_t s, float* out, void* hip_stream);

/* Overwrite the state (r, phi, n) from device pointers to N*N floats, for
 * checkpoint/resume.  r must be >= r_floor; phi values off the pupil are
 * ignored (stored as zero, as the state always holds them). */
int ddh_set_state(ddh_stream_t s, const float* r, const float* phi, long long n, void* hip_stream);

/* Frames submitted so far (n of Fig. 1). */
int ddh_frame_count(ddh_stream_t s, long long* n);

/* Synchronise hip_stream and report whether the last frame submitted on s
 * was rejected (DDH_EDATA) or accepted (DDH_OK), or whether a bounded wait
 * between workgroups gave up on s since the last call (DDH_EDEVICE; reported
 * once): a wait of the work-list step (DDH_BATCH_WORKLIST), or a wait of the
 * first row pass for the statistics of the frame's other rows.  The frame's
 * result is then unspecified. */
int ddh_status(ddh_stream_t s, void* hip_stream);

/* Grid size and parameters of a stream. */
int ddh_get_params(ddh_stream_t s, ddh_params* out);

/* ------------------------------------------------------------ diagnostics */

/* FP64 value of the cost that EM does not increase, at the current (r, phi)
 * for frame y (device pointer, N*N complex64):
 *   U = sum_i |b_i|^2/(r_i + s2) + log(r_i + s2) + sum_pairs b_ij rho(r_i - r_j)
 *       + beta sum_pupil_pairs b_ij (phi_i - phi_j)^2,  b = A_phi^H Normalize(y)
 * (joint MAP cost Eq. (2) of the back-projected model).  Per-pixel terms and
 * the reduction are FP64.  Synchronises hip_stream; result in *U (host). */
int ddh_cost(ddh_stream_t s, const void* y, double* U, void* hip_stream);

/* FP64 peak Strehl ratio (Algorithm Parameters and Metrics section)
 *   S = max|F^H(a exp(j psi))|^2 / max|F^H a|^2,
 * psi = phi - phi_true with piston, tip and tilt removed over the pupil.
 * phi_true: device pointer, N*N floats.  Synchronises; result in *S (host). */
int ddh_strehl(ddh_stream_t s, const float* phi_true, double* S, void* hip_stream);

/* ---------------------------------------------------------------- batches */

/* Group `count` streams (any mix of N) so that one call advances all of them
 * by one frame.  Streams keep their own state and numerics: a stream gives
 * the same result alone and in any batch.  flags: DDH_BATCH_GRAPH captures the
 * per-frame launch sequence in a HIP graph on first use.  The streams are
 * split into lanes whose launch chains run on internal HIP streams forked
 * from and joined back into the caller's stream (a graph then has parallel
 * branches): by default (lane count 0) one lane per distinct N, so that the
 * launches of different sizes overlap (a uniform batch has one lane);
 * DDH_BATCH_LANES(n) (n = 1..8) instead splits the streams into n lanes
 * balanced by pixel count (on the 64 x N=256 and mixed-size workloads two or
 * more such lanes measured slower than one).  All n_k must be equal.  The
 * batch does not own the streams; destroy the batch before its streams. */
#define DDH_BATCH_GRAPH 1
#define DDH_BATCH_LANES(n) (((n) & 0xff) << 8)
/* DDH_BATCH_WORKLIST: each EM iteration of a frame runs as one persistent
 * work-list launch per N group -- the Normalize/RemoveTipTilt statistics,
 * the first row DFT pass, the fused column pass and the second row pass of
 * all the group's streams, as (stream, stage, tile) items that workgroups
 * claim in dependency order from one queue per XCD, so that the stages of
 * different streams overlap -- followed by the M-step launch (two launches
 * per iteration instead of four).  Results are bit-identical to the default
 * launches.  Every wait of an item on the previous stage of its stream is
 * bounded; a wait that gives up lets the launch finish, and ddh_status then
 * reports DDH_EDEVICE for that stream and clears its work-list control
 * words; its state is then unspecified: restore it with ddh_set_state (which
 * also clears those words) before its next frame.  DDH_BATCH_TEST_GIVEUP (with
 * DDH_BATCH_WORKLIST; for tests of that failure path only) makes every such
 * wait give up at once.  Within a queue the stages of one stream are spread
 * by `lag` streams' worth of items (environment variable DDH_WORKLIST_LAG at
 * batch creation, 1..64, default 2), so that an item rarely waits. */
#define DDH_BATCH_WORKLIST 2
#define DDH_BATCH_TEST_GIVEUP 4
int ddh_batch_create(const ddh_stream_t* streams, int count, int flags, ddh_batch_t* out);
int ddh_batch_destroy(ddh_batch_t b);

/* One DDH frame on every stream of the batch.  y: host array of `count`
 * device pointers (the i-th frame is for the i-th stream passed to
 * ddh_batch_create); the host array may be reused once the call returns. */
int ddh_batch_step(ddh_batch_t b, const void* const* y, void* hip_stream);

/* Per-kernel timing of the eager (non-graph) batch step: when enabled, each
 * ddh_batch_step launches its kernels one after another on the caller's
 * stream, each with a pair of HIP events that the launch itself records at
 * the kernel's start and end (the kernel's execution, as a profiler's kernel
 * trace sees it, without the dispatch before it).
 * ddh_batch_stage_times synchronises and writes, for each kernel kind k < *n
 * (on input *n is the capacity of the arrays), the summed milliseconds ms[k]
 * and launch count calls[k] since timing was enabled, and its name to
 * names[k] (static strings).  Kinds: 0 stats, 1 finalize, 2 row-ifft,
 * 3 col-fused, 4 row-fft, 5 m-step, 6 begin (frame start), 7 frame_worklist
 * (the persistent launch of a DDH_BATCH_WORKLIST batch), 8 stats_row_ifft
 * (the first row pass of a frame with the Normalize/RemoveTipTilt statistics
 * formed in the same launch; an eager step's first EM iteration starts with
 * it, later iterations with row-ifft).  The frame start is passed to that
 * kernel, so kinds 0, 1 and 6 stay at zero launches in a timed eager step
 * of a one-lane batch.  A batch with several lanes created without
 * DDH_BATCH_GRAPH (and a server call with several N groups) forms the
 * statistics with a launch of their own (kind 0) before row-ifft instead,
 * since its lanes' launches run at the same time and share the device with
 * the fused pass's waiting blocks (measured faster that way for eager
 * launches, slower for graph replay); the environment variable
 * DDH_FUSED_STATS (0 or 1, read once per process) overrides that choice.
 * Both forms give bit-identical results.  The fused pass takes 32 rows per
 * block for groups of 8 or more streams at N >= 256 and the row passes'
 * row_lines otherwise (DDH_FUSED_LINES = 4, 8, 16 or 32, read once per
 * process, overrides); results do not depend on it. */
int ddh_batch_set_timing(ddh_batch_t b, int enable);
int ddh_batch_stage_times(ddh_batch_t b, double* ms, long long* calls, const char** names, int* n);

/* --------------------------------------------------------------- serving */

/* Continuous batching: a server advances, in one call, whichever distinct
 * streams have a frame ready, in any mix of N and n_k, the set changing from
 * call to call (streams are admitted and retired between calls).  Per-stream
 * numerics are those of ddh_step: a stream gives the same result alone and in
 * any mix.  The server owns a device list of max_streams descriptor pointers
 * (8 bytes each) on the current device; it does not own the streams.  Calls
 * on one server must all use the HIP stream of its first call (DDH_ESTATE
 * otherwise), so that they run in order: a stream may then appear again in
 * the next call while this one is still on the GPU. */
typedef struct ddh_server_s* ddh_server_t;
int ddh_server_create(int max_streams, ddh_server_t* out);

/* Device bytes that ddh_init_stream allocates for a stream of grid size N
 * (state, work buffers and descriptor; the twiddle tables are shared per
 * device).  For admission by memory budget. */
int ddh_stream_bytes(int N, unsigned long long* bytes);
int ddh_server_destroy(ddh_server_t s);

/* One DDH frame on each of `count` (0..max_streams) distinct streams.  The
 * frames of each N run on an internal HIP stream of the server, forked from
 * and joined back into hip_stream, so that different sizes overlap.
 * streams: host array of handles; y: host array of device pointers to their
 * frames (N*N complex64 each).  Both host arrays may be reused once the call
 * returns.  DDH_EINVAL for a repeated stream or a null frame. */
int ddh_server_step(ddh_server_t s, const ddh_stream_t* streams, const void* const* y, int count,
                    void* hip_stream);

/* One DDH frame on each of `count` distinct streams (any mix of N and n_k),
 * without a batch or server handle: the one-shot form of ReadData /
 * WriteData of Fig. 1 for many streams.  streams: host array of handles; y:
 * host array of device pointers to their frames (N*N complex64 each); both
 * may be reused once the call returns; each frame must stay valid until
 * hip_stream reaches the step.  Per-stream numerics are those of ddh_step:
 * each stream's result is bit-identical to stepping it alone.  The frames of
 * each N run on an internal HIP stream forked from and joined back into
 * hip_stream, so that different sizes overlap.  The first call on a given
 * (device, hip_stream) pair allocates a device list of descriptor pointers
 * (8 bytes per stream, at least 64) and four internal HIP streams, kept until
 * the process ends; a later call on that pair with more streams than the
 * list holds synchronises hip_stream and replaces it.  Calls on one HIP
 * stream must come from one host thread at a time.  All streams must be on
 * one device (DDH_ESTATE otherwise).  DDH_EINVAL for a NULL array with
 * count > 0, a repeated stream, a NULL frame or count > 2^20. */
int ddh_step_batch(const ddh_stream_t* streams, const void* const* y, int count, void* hip_stream);

/* ddh_step_batch for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * frame on the same streams with the same per-stream results, bit for bit,
 * but the call allocates nothing -- no device memory, no HIP streams, no
 * host heap.  The device list of descriptor pointers that the frame's first
 * launches fill and its later launches read is a fixed array of 4096 entries
 * (32 KiB) that the library holds on every device it runs on until the
 * process ends (its address is taken when the first stream is created on a
 * device).  All groups of (n_k, N) run one after another on hip_stream
 * (no internal HIP streams).  Every call on one device shares that array and
 * leaves its contents behind: calls that overlap on one GPU (on different HIP
 * streams, or from different host threads) race and must be serialised by
 * the caller; calls queued on one HIP stream are ordered and safe.  Errors:
 * DDH_EINVAL for count < 0 or count > 4096 (checked first), a NULL array with
 * count > 0, a repeated stream or a NULL frame; DDH_ESTATE for a destroyed
 * handle or streams on more than one device. */
int ddh_step_batch_noalloc(const ddh_stream_t* streams, const void* const* y, int count, void* hip_stream);

/* -------------------------------------------------------- differentiation */

/* Gradient of K unrolled DDH frames.  Starting from r = 0 and phi = phi0, the
 * frames y[0..K-1] (host array of K device pointers, N*N complex64 each) are
 * processed as by ddh_step with n_k = 1; the loss is the piston-removed RMS
 * difference over the pupil between the last phase and phi_true (device,
 * N*N floats).  The adjoint of every step is hand-written: the colour passes
 * are reversed pass by pass, each reflectance update through the implicit
 * derivative of its cubic root, the phase data term through its arctangent
 * and sinc, the E-step, Eq. (3), both DFTs and the tip/tilt removal.  Writes
 * d loss / d phi0 to d_phi0 (device, N*N floats) and the loss and its
 * derivatives with respect to sigma_w = sqrt(sigma_w2), the QGGMRF scale
 * qg_sigma (prior weight 1/qg_sigma^2 and threshold qg_T qg_sigma) and
 * beta_phi to *out (host).  Only every ckpt-th state is kept during the
 * forward; the backward recomputes each segment of ckpt frames from it.
 * Points where the map is not differentiable take the derivative of the
 * branch the forward took (floors, the root choice, the phase wrap); the
 * QGGMRF weight's unbounded derivative at zero difference is taken as zero.
 * Parameters as for ddh_init_stream, with n_k = 1 and qg_p = 2 (DDH_EINVAL
 * otherwise).  Its workspace is allocated on the first call on a device,
 * grown when a call needs more and kept until the process ends; calls on
 * one device take turns on it (each returns synchronised with hip_stream).  DDH_EDATA
 * if a frame cannot be normalised or the loss is zero. */
typedef struct {
  double loss;
  double d_sigma_w, d_sigma_r, d_beta;
} ddh_grad_out;
int ddh_unrolled_grad(const ddh_params* p, int K, const void* const* y, const float* phi0, const float* phi_true,
                      int ckpt, float* d_phi0, ddh_grad_out* out, void* hip_stream);

/* The same for `count` independent streams of one N in one pass: each kernel
 * covers every stream (the stream is the grid's second dimension), and the
 * FP64 reductions are combined on the device, so the call synchronises
 * hip_stream once.  p: host array of count parameter sets (same N; n_k = 1,
 * qg_p = 2); y: host array of count*K device frame pointers, stream-major
 * (y[b*K + k] is frame k of stream b); phi0, phi_true, d_phi0: host arrays of
 * count device pointers (N*N floats each); out: host array of count results.
 * Each stream's results are bit-identical to ddh_unrolled_grad on that stream
 * alone.  Workspace about (8 ceil(K/ckpt) + 92 ckpt + 84) bytes per pixel per
 * stream.  DDH_EINVAL for mixed N or a null pointer; DDH_EDATA if a frame of
 * any stream cannot be normalised or a loss is zero (the other streams'
 * results are still written); DDH_EINVAL also if count*N*N exceeds 2^31 - 1. */
int ddh_unrolled_grad_batch(const ddh_params* p, int count, int K, const void* const* y, const float* const* phi0,
                            const float* const* phi_true, int ckpt, float* const* d_phi0, ddh_grad_out* out,
                            void* hip_stream);

/* ---------------------------------------------------------- FFT (a3, a6) */

/* Batched unitary 2D DFT of `count` N x N complex64 images (device pointers,
 * in and out may alias only if equal).  inverse = 0: kernel exp(-2 pi i k.n/N),
 * inverse = 1: exp(+2 pi i k.n/N); both scaled by 1/N (Forward Model: F is a
 * normalised DFT).  `work` is a device buffer of count*N*N complex64. */
int ddh_fft2(int N, int count, const void* in, void* out, void* work, int inverse, void* hip_stream);

/* ------------------------------------------------------------------ tiles */

/* Launch tiling for grid size N: cfg[0] lines per workgroup of the row
 * passes (4, 8, 16, 32), cfg[1] columns per workgroup of the column pass
 * (4, 8, 16, 32), cfg[2] x cfg[3] output tile of the M-step (16x16, 16x32,
 * 16x64, 32x32, 32x64, 64x64, 32x128; each side at most N), or 0 x 0 for
 * four whole-image colour-pass launches instead of one halo-tiled kernel.  Tiling never changes results: every pixel is computed
 * by the same arithmetic whichever workgroup computes it.  The setting is
 * process-wide; it applies to batches created afterwards and to single-stream
 * calls made afterwards (a single-stream graph keeps the tiling it was captured
 * with).  DDH_EINVAL for an unsupported combination. */
int ddh_set_tiles(int N, const int* cfg);
int ddh_get_tiles(int N, int* cfg);

/* Autotune the tiling for grid size N on the current device: time every
 * candidate of each kernel on `count` temporary streams (synthetic frames
 * generated on the device), keep the fastest per kernel, and install it as with
 * ddh_set_tiles.  Candidates are given to the timing batches only, on the
 * tuner's own HIP stream: the process-wide tiling changes once, at the end, and
 * other work on the device is not synchronised with while the tuner runs.
 * Writes the choice to cfg (4 ints) and the winners' average kernel times in
 * microseconds to us (4 doubles: both row passes together, column pass, 0,
 * M-step), either may be NULL.  Returns when the tuning work has finished;
 * on error the tiling in force before the call is kept. */
int ddh_autotune(int N, int count, int* cfg, double* us);

/* Autotune the tilings of a mix of sizes together: `count` temporary streams
 * with sizes Ns[0..count-1] (host array, each one of 64..512) form a batch with
 * the default lanes (one per N); the whole batched step is timed with HIP
 * events while each distinct size's row, column and M-step tilings are varied
 * in turn (sizes ascending), and a candidate replaces the current tiling only
 * if the step gets more than 1 % faster.  Candidates are given to the timing
 * batches only, on the tuner's own HIP stream; the result is installed, as
 * with ddh_set_tiles, once at the end, so other batches and single-stream
 * calls never run a candidate and are not synchronised with while the tuner
 * runs.  cfgs (may be NULL) receives 4 ints per distinct size, sizes
 * ascending; step_us (may be NULL) the final step time in microseconds.
 * Errors: DDH_EINVAL (Ns NULL, count outside 1..4096, an unsupported size),
 * DDH_ENOMEM, DDH_EDEVICE; on error nothing is installed. */
int ddh_autotune_mix(const int* Ns, int count, int* cfgs, double* step_us);

/* ------------------------------------------------------------------- misc */
const char* ddh_error_string(int code);
/* Last HIP error message seen by the library (static storage). */
const char* ddh_last_error_message(void);
/* Library version string. */
const char* ddh_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DDH_H */
