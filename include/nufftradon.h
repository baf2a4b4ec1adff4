/*
 * nufftradon — NUFFT-based Radon projector, its adjoint and a qGGMRF MBIR
 * step for AMD Instinct MI355X (gfx950).  Plain C ABI.
 *
 * The operators follow arXiv 2304.12934 (tomoCAM):
 *   - the Radon transform of a slice (Sec. 2.1, eq. "radon_transform") is
 *     computed through the central-slice theorem (eq. "fourier_radon"):
 *     the 2D spectrum of the slice sampled on polar lines is a type-2
 *     non-uniform FFT (Sec. 2.2, eqs. "nufft"-"nufft3" in reverse order),
 *     followed by a 1D inverse transform along every line;
 *   - the adjoint (Sec. 3, eq. "transpose") is the same chain transposed:
 *     a 1D transform per line, a type-1 non-uniform FFT (spreading onto the
 *     oversampled grid, eq. "nufft2") and an inverse 2D FFT with division by
 *     the kernel transform (eq. "nufft3");
 *   - the prior is the qGGMRF of Sec. 3 (eqs. "reg2", "reg3") over the 26
 *     neighbours of every voxel; the MBIR step is one accelerated-gradient
 *     iteration on the objective of eq. "objfn" with the gradient of
 *     eq. "gradient".
 *
 * Discrete geometry.  A slice is f[iy][ix] (float32, row-major) with pixel
 * centres x = ix - N/2, y = iy - N/2.  Angle theta_a (float64, radians)
 * has normal (cos theta, sin theta).  The sinogram is s[a][m] (float32)
 * with bins t_m = m - N_t/2.  The operator is
 *     s[a][m] = Re (1/N_t) sum_l Fhat_a(k_l) exp(+2 pi i k_l t_m),
 *     Fhat_a(k) = sum_{x,y} f(x,y) exp(-2 pi i k (x cos theta_a + y sin theta_a)),
 * with k_l = (l - N_t/2)/N_t; radon_adj is its exact transpose for real
 * inner products.  The non-uniform FFT approximates Fhat with a
 * Kaiser-Bessel kernel of width W on a grid oversampled by sigma = 2.
 * A slice whose rotation axis projects to bin N_t/2 + c (nr_slice.center)
 * has t_m replaced by t_m - c: the Fourier shift of Sec. 4.1, applied as a
 * phase exp(-2 pi i k c) on each radial line.
 *
 * Stacks.  A plan describes n_slices slices, each with its own size N,
 * detector count N_t and angle set, addressed by element offsets into flat
 * caller buffers: the volume at d_vol + vol_off (N*N floats), the sinogram
 * at d_sino + sino_off (n_angles*N_t floats), its angles at
 * angles_host + angle_off.  Offsets may alias between slices only for
 * angles.
 *
 * Ownership.  The caller allocates every device buffer, including the
 * workspace; the library never allocates or frees device memory.  A plan
 * owns host tables and, once it has run with more than one stream (tuning
 * key "streams"), that many HIP streams of default priority and their
 * events, created on first use on the current device and released by
 * nr_plan_destroy.  All device calls are asynchronous on the given stream
 * and return after enqueueing: work the plan forks onto its own streams
 * waits for what was enqueued on the given stream before the call, and the
 * given stream waits for all of it before anything enqueued after the call.
 * A plan is used by one stream at a time (its scratch is shared).
 *
 * Errors.  Every call returns an nr_status and never aborts.  Arguments are
 * validated before anything is enqueued.  nr_last_error() gives a
 * thread-local message for the last failure.  Asynchronous device faults
 * surface as NR_HIP_ERROR on a later call.
 */
#ifndef NUFFTRADON_H
#define NUFFTRADON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nr_status;
enum {
  NR_OK = 0,
  NR_INVALID_ARG = 1,        /* null pointer, bad size, bad parameter      */
  NR_UNSUPPORTED_SIZE = 2,   /* FFT length outside the compiled set, or too
                                many angles (see nr_slice)                  */
  NR_WORKSPACE_TOO_SMALL = 3,
  NR_HIP_ERROR = 4,          /* a HIP runtime call failed                   */
  NR_NONFINITE = 5,          /* NaN/Inf detected by a device reduction      */
  NR_INTERNAL = 6
};

/* Opaque stream handle: a hipStream_t (NULL = the default stream). */
typedef void* nr_stream;

typedef struct nr_plan nr_plan;

/* One slice of a stack.  n: slice width N (even, >= 8); n_det: detector
 * bins N_t (even, >= 8); n_angles >= 1, below 2^24 and below
 * 2^31 / 2^ceil(log2(N_t/2 + 1)) (the plan's 32-bit point codes; else
 * NR_UNSUPPORTED_SIZE).  Offsets are element offsets.
 * center: offset c of the rotation axis from the detector centre, in bins
 * (the axis projects to bin N_t/2 + c); finite, |c| <= N_t/2; 0 for a
 * centred axis. */
typedef struct {
  int32_t n, n_det, n_angles;
  int64_t vol_off, sino_off, angle_off;
  double center;
} nr_slice;

/* Filter of radon_fbp.  filter: NR_FBP_RAMP (|k|) or NR_FBP_BUTTERWORTH
 * (|k| / (1 + (|k|/cutoff)^(2 order))); cutoff in cycles per pixel (> 0;
 * the Nyquist frequency is 0.5), order 1..16 (both ignored for the ramp). */
enum { NR_FBP_RAMP = 0, NR_FBP_BUTTERWORTH = 1 };
typedef struct {
  int32_t filter, order;
  double cutoff;
} nr_fbp;

/* Non-uniform FFT parameters.  sigma: oversampling (only 2.0 is built);
 * width: kernel width W in grid cells (6, 7 or 8); beta <= 0 selects the
 * Kaiser-Bessel shape beta = pi*sqrt((W/sigma)^2 (sigma - 1/2)^2 - 0.8). */
typedef struct {
  double sigma;
  int32_t width;
  double beta;
} nr_nufft;

const char* nr_status_str(nr_status s);
const char* nr_last_error(void);
const char* nr_version(void);

/* Create a plan for a slice stack (host only, no device work).  Copies the
 * slice array and every referenced angle.  Sorts the polar points of each
 * distinct geometry into spreading tiles once.  *out is set on success. */
nr_status nr_plan_create(const nr_slice* slices, int32_t n_slices, const double* angles_host,
                         const nr_nufft* params, nr_plan** out);

/* Bytes of device workspace the plan needs (tables + per-slice scratch). */
nr_status nr_plan_workspace_bytes(const nr_plan* plan, size_t* bytes);

/* Bind caller-owned device workspace (256-byte aligned, at least
 * nr_plan_workspace_bytes) and upload the plan tables on `stream`.  The
 * workspace must stay valid until the plan is destroyed or re-bound. */
nr_status nr_plan_bind(nr_plan* plan, void* d_workspace, size_t bytes, nr_stream stream);

nr_status nr_plan_destroy(nr_plan* plan);

/* Set an execution parameter of a plan; none changes results beyond float32
 * rounding of the spreading sums.  Keys:
 *   "tile_w", "tile_h"  spreading tile (64x32 default; 32x32, 64x64, 128x32)
 *   "chunk"             most points per spreading or interpolation work item,
 *                       64..1024
 *                       (1024 default)
 *   "interp_mode"       0 = interpolation from LDS-staged grid tiles (every
 *                       point once, by the tile of its first tap) followed by
 *                       the radial transforms (default); 1 = one pass per
 *                       angle pair gathering straight from the grid (same
 *                       sums in the same order)
 *   "batch"             most slices per batch (0: no limit): each stage kernel
 *                       runs once per batch (and FFT length) over all its
 *                       slices; the workspace holds the scratch of the
 *                       largest batch
 *   "batch_mb"          scratch budget of one batch in MiB (160 default:
 *                       one 2560^2 slice, whose grids then stay in the 256 MB
 *                       last-level cache between stages; a slice larger than
 *                       the budget runs alone)
 *   "streams"           1..8 (2 default): batches run round-robin on this many
 *                       streams the plan owns (forked from and joined back to
 *                       the caller's stream on every call), each with its own
 *                       scratch, so that the stages of different batches
 *                       overlap on the device
 *   "spread_mode"       0 = LDS-tiled spreading (default), 1 = one thread per
 *                       point with global float atomics (a slow cross-check)
 *   "persistent"        1 = a forward + adjoint pass (radon_normal, and the
 *                       fwd-then-adj graph) runs each batch as ONE persistent
 *                       kernel: resident workgroups take the batch's units
 *                       from per-XCD work queues (each slice's units on one
 *                       XCD, stage-major) and wait, bounded, on per-slice
 *                       stage counters; needs kernel width 7, the 64x32 tile,
 *                       interp_mode 0 and FFT lengths 128..4096 (powers of
 *                       two), else the layout fails with UNSUPPORTED_SIZE;
 *                       0 (default) = one launch per stage.  Other calls and
 *                       profiled runs use the per-stage launches.
 * Changing any key but spread_mode unbinds the plan: query
 * nr_plan_workspace_bytes and call nr_plan_bind again. */
nr_status nr_plan_tune(nr_plan* plan, const char* key, int64_t value);

/* Stage timing for measurement.  While enabled, every stage launch of
 * radon_fwd / radon_adj / radon_normal / mbir_step runs on the caller's
 * stream, one at a time (the plan's own streams are not used), bracketed by
 * two HIP events.  nr_plan_profile_read waits for the last recorded event
 * and returns, per stage, the summed milliseconds and the launch count, then
 * forgets the records.  Stages: 0 forward rows, 1 forward columns, 2
 * interpolation + radial transform, 3 adjoint radial transform, 4 spreading,
 * 5 adjoint columns, 6 adjoint rows, 7 residual, 8 prior, 9 MBIR update,
 * 10 clearing the grid tiles that several spreading items share. */
nr_status nr_plan_profile(nr_plan* plan, int32_t enable);
nr_status nr_plan_profile_read(nr_plan* plan, double* ms, int64_t* launches, int32_t n_stages);

/* s = R f for every slice of the plan (Sec. 2, eq. "fourier_radon" via the
 * type-2 NUFFT).  d_vol: float32 slices at vol_off; d_sino: float32
 * sinograms at sino_off, overwritten.  Device pointers. */
nr_status radon_fwd(nr_plan* plan, const float* d_vol, float* d_sino, nr_stream stream);

/* g = R^T y for every slice (Sec. 3, eq. "transpose", the exact transpose
 * of radon_fwd).  d_sino: float32 input; d_vol: float32 output,
 * overwritten.  Device pointers. */
nr_status radon_adj(nr_plan* plan, const float* d_sino, float* d_vol, nr_stream stream);

/* Filtered back-projection for every slice (Sec. 2.1, eq. "inverse_radon"
 * discretised with dtheta = pi/N_theta and dk = 1/N_t):
 *     g(x) = (pi/N_theta) Re sum_a (1/N_t) sum_l w(k_l) Yhat_a(k_l) exp(2 pi i k_l <x, n_a>),
 *     Yhat_a(k) = sum_m y[a][m] exp(-2 pi i k (t_m - c)),
 * w from *filter.  radon_adj with the radial weight w(k) pi/N_theta applied
 * on each line; same buffers and layouts as radon_adj. */
nr_status radon_fbp(nr_plan* plan, const nr_fbp* filter, const float* d_sino, float* d_vol, nr_stream stream);

/* Host-resident stacks streamed through the GPU (Sec. 4.1: the partition
 * along the rotation axis, sub-partitions copied asynchronously).  The plan
 * describes one chunk; h_in and h_out hold n_chunks chunks back to back in
 * host memory, each laid out as the plan's flat buffers (a chunk's volume
 * has the extent of the plan's volume layout, its sinogram that of the
 * sinogram layout).  what: NR_STREAM_FWD (volume -> sinogram), NR_STREAM_ADJ
 * (sinogram -> volume) or NR_STREAM_FBP (sinogram -> volume, with *filter;
 * filter is ignored otherwise and may be NULL).
 * d_in[0..1] and d_out[0..1]: two caller-owned device buffers of one chunk
 * each, in the input and output layouts of `what`; chunk i uses d_in[i%2]
 * and d_out[i%2], so the copy of chunk i+1 to the device and of chunk i-1
 * back to the host overlap the computation of chunk i.  The copies run on
 * two streams the plan owns (default priority), the computation on
 * `stream`, which on return waits for the last copy back; h_out is complete
 * once `stream` has drained.  Host memory should be pinned (hipHostMalloc)
 * for the copies to be asynchronous; pageable memory gives the same result
 * with the copies serialised.  n_chunks = 0 enqueues nothing.  The four
 * device buffers must be distinct; results equal those of the
 * device-resident calls chunk by chunk. */
enum { NR_STREAM_FWD = 1, NR_STREAM_ADJ = 2, NR_STREAM_FBP = 3 };
nr_status radon_stream(nr_plan* plan, int32_t what, const nr_fbp* filter, const float* h_in, float* h_out,
                       int64_t n_chunks, float* const* d_in, float* const* d_out, nr_stream stream);

/* The gradient of the data term (Sec. 3, eq. "gradient"): d_sino = R f - b
 * (R f when d_b is NULL) and d_vol_out = R^T d_sino, for every slice.  Same
 * values as radon_fwd, the subtraction and radon_adj in sequence; each batch
 * of slices runs its forward, residual and adjoint back to back on one of
 * the plan's streams, with no wait for the other batches in between.
 * d_vol, d_b, d_sino, d_vol_out: float32 device buffers in the plan's layout
 * (d_sino and d_vol_out overwritten; d_vol_out must not alias d_vol). */
nr_status radon_normal(nr_plan* plan, const float* d_vol, const float* d_b, float* d_sino, float* d_vol_out,
                       nr_stream stream);

/* Data term of the objective (Sec. 3, eq. "objfn" with G = 1/2 ||R f - b||^2):
 * d_r = R f - b (sinogram layout, overwritten) and, when d_value is not NULL,
 * *d_value = 1/2 sum r^2 as one float64 on the device.  Its gradient is
 * radon_adj(d_r) (eq. "gradient"). */
nr_status radon_residual(nr_plan* plan, const float* d_vol, const float* d_b, float* d_r, double* d_value,
                         nr_stream stream);

/* qGGMRF prior (Sec. 3, eqs. "reg2"/"reg3") on a [nz][n][n] float32 volume:
 *   H(f) = lambda sum_m sum_{n in N26(m)} w_mn rho((f_m - f_n)/sigma),
 *   rho(u) = u^2/(c + |u|^(2-p)),
 * with w_face/w_edge/w_corner the weights of the 6/12/8 neighbours (voxels
 * outside the volume are dropped).  Adds scale * dH/df into d_grad_accum
 * (in place) and, when d_value is not NULL, writes H(f) as one float64. */
typedef struct {
  float p, sigma, c, lambda;
  float w_face, w_edge, w_corner;
} nr_prior;

nr_status qggmrf_grad(const float* d_vol, int32_t nz, int32_t n, const nr_prior* prior,
                      float scale, float* d_grad_accum, double* d_value, nr_stream stream);

/* Fills *out with the prior's parameters and neighbour weights (Sec. 3,
 * eq. "reg3": w_mn over the 26 neighbours, summing to one).  weights:
 * NR_WEIGHTS_INV_DISTANCE (w proportional to 1/||m - n||, the paper's
 * "inversely proportional to the distance") or NR_WEIGHTS_GAUSSIAN (w
 * proportional to exp(-||m - n||^2/2)).  Host only. */
enum { NR_WEIGHTS_INV_DISTANCE = 0, NR_WEIGHTS_GAUSSIAN = 1 };
nr_status nr_prior_init(nr_prior* out, float p, float sigma, float c, float lambda, int32_t weights);

/* *out = a Lipschitz constant of grad H (Sec. 3, the prior's part of the
 * step size): rho'' is largest at 0, rho''(0) = 2/c, so by Gershgorin
 * L_H = 8 lambda (6 w_face + 12 w_edge + 8 w_corner) / (c sigma^2).  Host only. */
nr_status nr_prior_lipschitz(const nr_prior* prior, double* out);

/* The largest eigenvalue of R^T R over every slice of the plan, by `iters`
 * power iterations (v <- R^T R v / ||R^T R v||, norms in float64 on the
 * device) from a seeded uniform start vector (splitmix64 of seed and the
 * element index), times `safety` (>= 1): the data term's part of the step
 * size (Sec. 3).  d_v, d_w: float32 scratch of the plan's volume layout
 * (max vol_off + N*N, distinct); d_sino: float32 scratch of its sinogram
 * layout; d_work: one float64.  Device pointers.  Synchronises `stream` and
 * writes the result to *h_out (host). */
nr_status nr_power_lipschitz(nr_plan* plan, int32_t iters, uint64_t seed, double safety, float* d_v, float* d_w,
                             float* d_sino, double* d_work, double* h_out, nr_stream stream);

/* One accelerated-gradient iteration (Sec. 3, last paragraph: an accelerated
 * gradient method with restart that keeps the objective from rising;
 * objective eq. "objfn" with G = 1/2 ||R f - b||^2):
 *   g = R^T (R y - b) + grad H(y);  x' = y - inv_L * g (max(x',0) if nonneg)
 *   restart (t = 1) if restart and <g, x' - x> > 0
 *   monotone: reject x' (keep x, t = 1, y = x) if Phi(x') > Phi(x), where
 *             Phi = 1/2 ||R f - b||^2 + H(f); the first step is accepted
 *   t' = (1 + sqrt(1 + 4 t^2))/2;  y' = x' + ((t - 1)/t') (x' - x)
 *   x_prev <- x;  x <- x' (when accepted)
 * inv_L: step 1/L with L >= the Lipschitz constant of grad Phi (nr_mbir_params);
 * restart, nonneg, monotone: 0 or 1.  A monotone step evaluates Phi(x') with
 * one more forward projection and prior pass.
 * All slices of the plan must share one N and the volume is the plan's
 * slices stacked in order (prior couples consecutive slices): slice z must
 * sit at vol_off = z*N*N.  d_b: data, same layout as radon_fwd's output.
 * d_x, d_x_prev, d_y, d_grad: float32 volumes (d_grad holds g on return;
 * d_x_prev holds the previous x, or x itself after a rejected step).
 * d_state: NR_MBIR_STATE_DOUBLES float64 on the device, set by
 * mbir_state_init before the first step: {t, last <g, x'-x>, nonfinite
 * flag, restart count, beta, Phi(x), Phi(x) known, data term of x', prior
 * of x', last x' accepted, rejected steps, 5 reserved}.  d_scratch: float32
 * scratch of the plan's sinogram size (max sino_off + n_angles*N_t).
 * Everything stays on the device: no host synchronisation; read d_state
 * when needed (flag != 0 means a NaN/Inf appeared). */
typedef struct {
  float inv_L;
  int32_t restart;
  int32_t nonneg;
  int32_t monotone;
} nr_mbir;

#define NR_MBIR_STATE_DOUBLES 16

nr_status mbir_step(nr_plan* plan, const nr_prior* prior, const nr_mbir* params,
                    const float* d_b, float* d_x, float* d_x_prev, float* d_y, float* d_grad,
                    float* d_scratch, double* d_state, nr_stream stream);

/* mbir_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same step, with the residual sinogram R y - b kept in a scratch array
 * the library reserves on each device it runs on, NR_NOALLOC_SCRATCH_BYTES
 * long, held until the process ends, instead of a caller's d_scratch.  The
 * caller still passes every input, output and state buffer, and the plan
 * must be bound.  Plans whose sinogram layout exceeds the array (max
 * sino_off + n_angles*N_t floats above NR_NOALLOC_SCRATCH_BYTES/4) are refused
 * with NR_INVALID_ARG before anything is enqueued.  The function itself
 * allocates no device memory (the plan's own streams are created by its first
 * multi-stream call of any entry point, as for mbir_step).  All calls on one
 * device share the array: calls that overlap in time on one device (other
 * streams, other threads) race and must be ordered by the caller; each call
 * writes every scratch value it reads. */
#define NR_NOALLOC_SCRATCH_BYTES (64u << 20)
nr_status mbir_step_noalloc(nr_plan* plan, const nr_prior* prior, const nr_mbir* params, const float* d_b,
                            float* d_x, float* d_x_prev, float* d_y, float* d_grad, double* d_state,
                            nr_stream stream);

/* One step of mbir_step's iteration over a volume that lives in host memory
 * (Sec. 4.1, the partition along the rotation axis streamed through the GPU):
 * the plan describes one chunk of nz uniform slices (shared N, angles and
 * bins, vol_off = z*N*N, sino_off = z*n_angles*n_det) and the volume is
 * n_chunks such chunks, Z = n_chunks*nz slices, stacked in order.
 * h_x = x_k and h_x_prev = x_{k-1} ([Z][N][N] float32, host), h_b the data
 * (n_chunks copies of the plan's sinogram layout back to back, host);
 * h_x_next (host, not aliasing the inputs) receives x_{k+1}.  The
 * extrapolated point y_k = x_k + beta (x_k - x_{k-1}) is formed on the device
 * per chunk (beta from d_state, set by the previous call's restart test;
 * mbir_state_init gives beta = 0, so the first call takes y_0 = x_0 with any
 * h_x_prev), with one halo slice each side for the prior; the gradient, x_{k+1}
 * = y_k - g/L (clamped when nonneg) and the restart dot product follow chunk
 * by chunk, and after the last chunk the restart test, t and beta as in
 * mbir_step.  The iterates equal mbir_step's over the whole volume up to
 * float32 rounding.  Chunk c + 1 is copied in on a plan-owned stream while
 * chunk c is computed on `stream` and chunk c - 1 copied out on another;
 * pinned host buffers let the copies overlap.  d_work: device work area of
 * mbir_stream_work_bytes bytes (two input sets of 2(nz + 2) slices and one
 * chunk of data, the extended y and prior gradient, the gradient, the
 * residual and two output chunks).  Non-monotone steps only (monotone = 1 is
 * NR_INVALID_ARG).  Asynchronous on `stream`: h_x_next is complete once
 * `stream` has reached this point. */
nr_status mbir_stream_work_bytes(const nr_plan* plan, size_t* bytes);
nr_status mbir_stream_iterate(nr_plan* plan, const nr_prior* prior, const nr_mbir* params, int64_t n_chunks,
                              const float* h_b, const float* h_x, const float* h_x_prev, float* h_x_next,
                              void* d_work, size_t work_bytes, double* d_state, nr_stream stream);

/* Resets an MBIR state (NR_MBIR_STATE_DOUBLES float64 on the device): t = 1,
 * every other entry 0.  Asynchronous on `stream`. */
nr_status mbir_state_init(double* d_state, nr_stream stream);

/* The step parameters of mbir_step: inv_L = 1/(lipschitz_data + L_H(prior))
 * with lipschitz_data the largest eigenvalue of R^T R (nr_power_lipschitz)
 * and L_H from nr_prior_lipschitz (prior may be NULL: no prior); restart,
 * nonneg and monotone copied (0 or 1).  Host only. */
nr_status nr_mbir_params(double lipschitz_data, const nr_prior* prior, int32_t restart, int32_t nonneg,
                         int32_t monotone, nr_mbir* out);

/* The update half of mbir_step for a gradient computed elsewhere (e.g. by
 * autograd through radon_fwd / radon_adj / qggmrf_grad): given g = grad
 * Phi(y) in d_grad, performs the restart test, the momentum update and
 * x_prev <- x, x <- x', y <- y' over `count` float32 elements, with d_state
 * as for mbir_step.  Device pointers; no host synchronisation.  The
 * monotone step needs the objective and is refused here (NR_INVALID_ARG). */
nr_status mbir_update(const nr_mbir* params, float* d_x, float* d_x_prev, float* d_y, const float* d_grad,
                      int64_t count, double* d_state, nr_stream stream);

/* Graphs: a whole forward/adjoint pass or a run of MBIR steps captured once
 * (on a private stream) into a HIP graph and replayed with one launch.  The
 * buffers are bound at capture; the plan must outlive the graph and stay
 * bound: nr_graph_launch refuses (NR_INVALID_ARG) a graph whose plan has
 * been re-tuned or re-bound since the capture.  what: 1 = radon_fwd(d_vol_in -> d_sino), 2 = radon_adj(d_sino ->
 * d_vol_out), 3 = both in that order. */
typedef struct nr_graph nr_graph;
nr_status nr_graph_capture_radon(nr_plan* plan, int32_t what, const float* d_vol_in, float* d_sino,
                                 float* d_vol_out, nr_graph** out);
nr_status nr_graph_capture_mbir(nr_plan* plan, const nr_prior* prior, const nr_mbir* params, const float* d_b,
                                float* d_x, float* d_x_prev, float* d_y, float* d_grad, float* d_scratch,
                                double* d_state, int32_t iters, nr_graph** out);
nr_status nr_graph_launch(nr_graph* graph, nr_stream stream);
nr_status nr_graph_destroy(nr_graph* graph);

/* Autotuner (Sec. 4: the execution schedule of the C++ core; batching and
 * the spreading tile are this library's own parameters).  Times forward +
 * adjoint passes (radon_normal, three repetitions after a warm-up, HIP
 * events on `stream`) of the plan's stack under candidate settings of the
 * tuning keys "batch_mb" {1, 160, 640, 1400, 2048}, "streams" {1, 2, 3, 6},
 * the spreading tile "tile_w" x "tile_h" {64x32, 32x32, 64x64, 128x32} and
 * "chunk" {256, 512, 1024}, one key at a time from the plan's current
 * setting (coordinate search), and keeps the fastest.  Every candidate
 * computes the same operator (the spreading sums differ in float32 order).
 * d_scratch (256-byte aligned, `bytes` long, device) holds the passes'
 * buffers and each candidate's workspace; candidates that do not fit are
 * skipped (nr_autotune_scratch_bytes gives a size that fits them all).
 * cache_json (may be NULL): a JSON file of tunings keyed by geometry and
 * device; a hit applies the cached setting without timing, a miss is
 * written back.  On return the plan holds the chosen setting and is
 * unbound: query nr_plan_workspace_bytes and call nr_plan_bind.
 * Synchronises `stream`. */
nr_status nr_autotune(nr_plan* plan, void* d_scratch, size_t bytes, const char* cache_json, nr_stream stream);
nr_status nr_autotune_scratch_bytes(nr_plan* plan, size_t* bytes);

/* Current value of a tuning key of nr_plan_tune, or "autotune_us" (best pass
 * time of the last nr_autotune in microseconds, -1 if none or cached) and
 * "autotune_trials" (candidates it timed). */
nr_status nr_plan_get_tune(const nr_plan* plan, const char* key, int64_t* value);

/* Host-only helpers (no device needed), used to test the plan's tables.
 * nr_kb_eval: for the plan-independent kernel with (width, beta), evaluates
 * phi(u) (normalised to phi(0)=1) at u[i] with the float64 series, phihat
 * (its continuous Fourier transform, same normalisation) at xi[i], and the
 * piecewise-polynomial device approximation of phi at u[i]. */
nr_status nr_kb_eval(int32_t width, double beta, int32_t count, const double* u, const double* xi,
                     double* phi, double* phihat, double* phi_poly);

/* Synchronises `stream` and reports NR_INTERNAL if a persistent launch of
 * the plan gave up waiting for a stage (a bounded wait ran out; the pass's
 * results are then invalid), resetting the flag; NR_OK otherwise. */
nr_status nr_plan_check(nr_plan* plan, nr_stream stream);

/* Describe how a plan splits work: fills up to 8 counts for slice `index`:
 * info[0] = oversampled grid G, info[1] = spreading tiles, info[2] = tile
 * point entries, info[3] = spreading work items, info[4] = polynomial degree,
 * info[5] = scratch slots (slices per batch), info[6] = batches,
 * info[7] = kernel launches of one forward + adjoint pass. */
nr_status nr_plan_info(const nr_plan* plan, int32_t index, int64_t* info, int32_t count);

#ifdef __cplusplus
}
#endif

#endif /* NUFFTRADON_H */
