/*
 * fwr.h -- C ABI of libfwr: Gerchberg slope extension and Fourier wave-front
 * reconstruction on AMD Instinct MI355X (gfx950).
 *
 * Method: Bond et al., "Iterative wave-front reconstruction in the Fourier
 * domain".  The library computes, per frame of Shack-Hartmann slopes:
 *   - the padded measurement: in-pupil slopes placed centred on an N x N grid,
 *     zeros elsewhere (Sec. 4.1: zero iterations = zero padding);
 *   - n_iter iterations of the modified Gerchberg loop (Sec. 3.3,
 *     Algorithm 1 steps 1-4): transform, least-squares phase reconstruction
 *     followed by re-derivation of the slopes (Eq. 2 and Eq. 3 with
 *     gamma = 0), inverse transform, re-imposition of the measured slopes
 *     inside the pupil;
 *   - optionally the periodicity condition of Eq. 5 (Algorithm 1 step 5);
 *   - the final Fourier reconstruction of Eq. 2 with the Wiener filter of
 *     Eq. 3 (gamma = 1 gives the MMSE filter; gamma = 0 least squares).
 * Two slope models (fwr_model): the Fried geometry, where a subaperture
 * measures the mean of the two phase differences across its four corner nodes
 * (the discrete model of Eq. 1), and the lenslet-averaging model of Eq. 4,
 * where it measures the difference of the phase averaged over its opposite
 * edges (transfer function with the sinc factor of Eq. 4).
 *
 * Conventions (all calls):
 *   - Row index = y, column index = x, row-major, float32, no padding.
 *   - Lenslet array n x n; grid N x N with N > n, N - n even; the array sits
 *     at offset o = (N - n) / 2 in both axes.
 *   - Slopes in:  float[B][2][n][n]  (plane 0 = x slopes, plane 1 = y), radians
 *     of phase difference across one subaperture.  Values on subapertures the
 *     mask marks invalid are ignored.
 *   - Phase out:  float[B][n+1][n+1]  on the Fried nodes of the lenslet array
 *     (grid nodes [o, o+n] x [o, o+n]); radians; the mean over the full N x N
 *     grid is zero.
 *   - Extended slopes out: float[B][2][N][N].
 *   - Every pointer argument of fwr_extend / fwr_reconstruct is a DEVICE
 *     pointer on the device the plan was created on.  The caller owns every
 *     input and output buffer and keeps it alive until the plan's stream has
 *     passed the enqueued work.
 *   - Calls are asynchronous: they validate, enqueue on the plan's stream and
 *     return.  Errors are reported only through the status code; nothing is
 *     thrown across this boundary.  A kernel fault surfaces as FWR_E_DEVICE
 *     from a later call or from the caller's own stream synchronisation.
 *   - One plan may be used from one host thread at a time.
 *   - Non-finite input is isolated per frame.  Under the Fried model frames
 *     are transformed in pairs (frame 2i in the real part and 2i+1 in the
 *     imaginary part of one complex field); a NaN or infinity among a frame's
 *     in-pupil measured slopes, or anywhere in its start values, enters that
 *     field as zero and the frame is flagged: its phases, extended slopes and
 *     residual are written as NaN (the residual then selects it for the
 *     fallback).  Other pairs are untouched; the partner is bit for bit what
 *     it is when the offending measured slopes are zero, and equal to rounding
 *     when the offending values are start values.  Under the
 *     lenslet-averaging model frames are not paired: such a frame's phases are
 *     NaN and no other frame is touched.  Slopes outside the pupil are never
 *     read.
 */
#ifndef FWR_H
#define FWR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FWR_OK = 0,
  FWR_E_INVAL = -1,        /* bad argument (NULL pointer, size out of range, ...) */
  FWR_E_UNSUPPORTED = -2,  /* valid request the library does not implement (e.g. grid size) */
  FWR_E_NOMEM = -3,        /* device allocation failed */
  FWR_E_DEVICE = -4,       /* HIP runtime error (launch failure, fault, no device) */
  FWR_E_STATE = -5         /* plan handle not valid */
} fwr_status;

typedef enum {
  FWR_MODEL_FRIED = 0,     /* Fried-geometry Shack-Hartmann slopes */
  FWR_MODEL_SINC = 1       /* lenslet-averaging model of Eq. 4: a subaperture measures the
                              difference of the phase averaged over its opposite edges;
                              transfer function exp(i pi (k'+l')/N) 2i sin(pi k'/N) sinc(l'/N)
                              (x; y transposed), signed frequencies, zero on the Nyquist row
                              and column; the d - d_px correction via fwr_params.d_px.
                              Grids N = 8, 16, 24, 32, 40, 48, 64, 80, 128 on chip, with
                              start values, the residual, per-iteration Eq. 5 and the Hudgin
                              extension as for the Fried model; N = 256 as passes through a
                              plan-owned workspace (Eq. 5 after the loop or every iteration;
                              no start values, residual or Hudgin extension); no device
                              generator (which samples Fried slopes). */
} fwr_model;

typedef struct fwr_plan_s *fwr_plan_t;   /* opaque; owns every device table */

typedef struct {
  int32_t n_sub;            /* n: lenslets per side, >= 1 */
  int32_t n_grid;           /* N: padded grid side; N > n, N - n even */
  const uint8_t *mask;      /* HOST pointer, n*n bytes, row = y; nonzero = valid
                               subaperture (the pupil P of Algorithm 1 step 4).
                               Copied at plan time. */
  int32_t n_iter;           /* Gerchberg iterations, 0 <= n_iter <= 10000 */
  int32_t periodic;         /* 1: apply Eq. 5 once after the loop (Algorithm 1 step 5) */
  int32_t periodic_each_iter; /* 1: apply Eq. 5 after every iteration's step 4 as well */
  int32_t model;            /* fwr_model */
  double gamma;             /* Eq. 3 gamma for the FINAL reconstruction (the loop always
                               uses gamma = 0, Sec. 3.3): 0 = LSQ, 1 = MMSE */
  double noise_var;         /* sigma^2 of the slope noise [rad^2] (W_eta, white) */
  double r0, L0;            /* von Karman W_phi: Fried parameter and outer scale [m] */
  double d;                 /* lenslet pitch [m] (grid spacing of the phase) */
  const double *alpha_map;  /* optional HOST N*N map (row = frequency l along y, column =
                               frequency k along x, unshifted DFT order) that replaces
                               gamma * W_eta / W_phi; NULL = use gamma, noise_var, r0, L0, d.
                               Finite, >= 0 and even, map[(N-l)%N][(N-k)%N] = map[l][k], as
                               the ratio of two spectra of real processes is (FWR_E_INVAL
                               otherwise); copied at plan time */
  int32_t max_batch;        /* largest B accepted by the calls, >= 1 */
  void *stream;             /* hipStream_t for every call; NULL = the null stream */
  double d_px;              /* FWR_MODEL_SINC: length of one detector pixel [m], 0 <= d_px < d
                               (the remark after Eq. 4: the edge-average difference is taken
                               over d - d_px; the two edge averages lie (d - d_px) apart, each
                               over the full edge, giving sin(pi k' (1 - d_px/d) / N) in place
                               of sin(pi k' / N)).  0 = no correction; must be 0 for the Fried
                               model (FWR_E_UNSUPPORTED), FWR_E_INVAL outside the range. */
} fwr_params;

/* Create a plan: validates the parameters, builds the filter, twiddle and
 * geometry tables in double precision on the host, rounds them to float and
 * uploads them.  Grid sizes: N = 4 * t with t in {2,3,4,5,6,8,10,12,16,20,32}
 * (N = 8 ... 128) run on-chip (one LDS tile per frame pair); N = 256 runs as
 * grid-wide passes through a plan-owned device workspace (start values and the
 * residual are on-chip only).  Other N
 * give FWR_E_UNSUPPORTED.  On success *out holds the plan; on failure *out is
 * set to NULL. */
fwr_status fwr_plan(const fwr_params *params, fwr_plan_t *out);

/* Algorithm 1 (steps 1-4 n_iter times, then step 5 if periodic) for B frames.
 * d_slopes: float[B][2][n][n]; d_ext: float[B][2][N][N].  Inside the pupil the
 * output equals the input bit for bit.  B = 0 is a no-op; B > max_batch or a
 * NULL pointer with B > 0 gives FWR_E_INVAL. */
fwr_status fwr_extend(fwr_plan_t plan, const float *d_slopes, float *d_ext, int32_t B);

/* Extension as fwr_extend, then the final reconstruction of Eq. 2 with the
 * Eq. 3 filter; writes the (n+1) x (n+1) node window of each frame.
 * d_slopes: float[B][2][n][n]; d_phase: float[B][n+1][n+1].  Same errors as
 * fwr_extend. */
fwr_status fwr_reconstruct(fwr_plan_t plan, const float *d_slopes, float *d_phase, int32_t B);

/* Release the plan and its device tables.  Work already enqueued must have
 * completed (the call synchronises the plan's stream first).  NULL is
 * FWR_E_STATE. */
fwr_status fwr_destroy(fwr_plan_t plan);

/* Change the stream later calls enqueue on. */
fwr_status fwr_set_stream(fwr_plan_t plan, void *stream);

/* Launch shape of the on-chip kernel (grids up to 128 x 128): frames per
 * workgroup, 2 (one frame pair) or 4, 8, 16 where the kernel is built for it and the
 * workgroup's LDS fits (FWR_E_UNSUPPORTED otherwise; FWR_E_INVAL for odd or < 2).
 * Plans of FWR_MODEL_SINC take 1 or 2 frames per workgroup (one frame per complex field).
 * Results do not depend on it.  Plans start from the choice autotuned earlier in the
 * process for the same device, N, n, n_iter and Eq. 5 mode, else from a rule that
 * balances the waves of a workgroup over the four SIMDs of a CU. */
fwr_status fwr_plan_set_group(fwr_plan_t plan, int32_t frames_per_group);

/* Radix schedule of the on-chip kernel's in-lane DFTs (length T = N/4): 0 = radix
 * 4 first, prime-factor (no twiddles) where the two factors are coprime (the
 * default); 1 = Cooley-Tukey with twiddles at every level, radix 5 (else 3, else 2)
 * first.  Both compute the exact DFT and round differently (each within the
 * parity tolerance).  Schedule 1 exists for the windowed kernel of 2x-padded plans
 * (n = N/2, N >= 24, no per-iteration Eq. 5; FWR_E_UNSUPPORTED otherwise,
 * FWR_E_INVAL for values other than 0, 1, 2); their calls with start values or
 * the extended-slope output take schedule 0.  On Fried plans of the multi-pass
 * path (N = 256) the schedules are launch shapes of the loop: 0 = one launch per
 * pass, the column pass with 16 threads per 256-point line (radix-16 DFTs in
 * registers, 256-thread workgroups); 1 = the same with 64 threads per line (one
 * wave per line, quads of lanes doing the 16-point sub-transforms, 1024-thread
 * workgroups: four times the waves for the same lines); 2 = the loop's column
 * passes and fused row steps in one persistent launch (288-thread workgroups that
 * take column tiles and row blocks from a counter and wait, through per-pair
 * counts in the plan's workspace, for the previous step of their own frame pair
 * only; the same arithmetic as 0, bit for bit).  Schedule 2 applies to calls with
 * at least two iterations and no per-iteration Eq. 5 (and fewer than 2^30 work
 * items, about 40 per frame pair and iteration), and not to items of a grouped
 * call with other items, whose concurrent work needs the CUs its waiting
 * workgroups would hold (those run as 0); a wait
 * that exceeds about a second gives up and writes the call's frames as NaN.
 * Schedule 2 is FWR_E_UNSUPPORTED on other plans.  Plans start from the schedule
 * autotuned earlier in the process for the same shape, else 0. */
fwr_status fwr_plan_set_schedule(fwr_plan_t plan, int32_t schedule);
fwr_status fwr_plan_get_schedule(fwr_plan_t plan, int32_t *schedule);

/* Watchdog of the persistent loop (schedule 2 of Fried multi-pass plans): the
 * number of polls (about 1 us each) a workgroup waits for the previous step of
 * its frame pair before the call gives up; a call that gives up writes every frame
 * of its output as NaN, and the next call starts afresh.  Default 2^20 (about a
 * second: a wait that long means the device is shared with work that holds it).
 * polls in [1, 2^24] (FWR_E_INVAL otherwise); FWR_E_UNSUPPORTED on other plans. */
fwr_status fwr_plan_set_wait_limit(fwr_plan_t plan, int32_t polls);

/* Autotuner: times every frames-per-workgroup choice of the plan on B frames (B <=
 * max_batch; device scratch is allocated and freed here), with each radix schedule
 * the plan allows (on the Fried multi-pass path: its three launch shapes), on the
 * plan's stream, synchronously; keeps the fastest pair in the plan and for later
 * plans of the same shape, and returns the frames per workgroup in
 * *frames_per_group (may be NULL; the schedule: fwr_plan_get_schedule).  Not for
 * use under graph capture. */
fwr_status fwr_plan_autotune(fwr_plan_t plan, int32_t B, int32_t *frames_per_group);

/* Launch shape of the reconstruction kernel, for reporting: threads per
 * workgroup, frames per workgroup, LDS bytes per workgroup (static + dynamic).
 * Multi-pass plans report the column pass's workgroup (the persistent loop's
 * with schedule 2) and 0 LDS bytes. */
fwr_status fwr_plan_launch_info(fwr_plan_t plan, int32_t *threads, int32_t *frames_per_group,
                                int32_t *lds_bytes);

/* ------------------------------------------------------------------------
 * Start values and residual (used by the learned initial extension).
 *
 * Algorithm 1 starts from the measurement padded with zeros (Sec. 4.1).  These
 * variants start from `d_start` (float[B][2][N][N], slopes on the padded grid)
 * outside the pupil instead; inside the pupil the measurement is used as
 * always.  `d_resid` (float[B], may be NULL) receives the in-pupil misfit of
 * the last iteration, ||P (G phi - s0)|| / ||P s0|| (0 when n_iter = 0 or the
 * pupil is empty).  On-chip grids (N <= 128) of both slope models; FWR_E_UNSUPPORTED
 * for the multi-pass grid (N = 256).
 * With n_iter = 0 the start is the extension: fwr_reconstruct_start then applies
 * Eq. 2/3 to (measurement inside, start outside); it needs periodic = 0 and no
 * residual, and fwr_extend_start needs n_iter >= 1 (FWR_E_INVAL otherwise).
 */
fwr_status fwr_extend_start(fwr_plan_t plan, const float *d_slopes, const float *d_start, float *d_ext,
                            float *d_resid, int32_t B);
fwr_status fwr_reconstruct_start(fwr_plan_t plan, const float *d_slopes, const float *d_start, float *d_phase,
                                 float *d_resid, int32_t B);

/* ------------------------------------------------------------------------
 * Comparison extension.
 *
 * fwr_hudgin_extend: the "Hudgin extension" the paper compares against (Sec. 3.2):
 * x slopes repeated up and down each column and y slopes left and right along each
 * row from the edge of the pupil, then Eq. 5.  Every cell outside the pupil takes the
 * slope of the nearest in-pupil cell of its column (x) or row (y), the upper / left one
 * on a tie (this also fills the central obstruction); a line without in-pupil cells is
 * zero.  d_slopes: float[B][2][n][n]; d_ext: float[B][2][N][N].  On-chip plans of either
 * slope model (FWR_E_UNSUPPORTED for N = 256).  The phase of this extension is
 * fwr_reconstruct_start on a plan with n_iter = 0 and periodic = 0 with d_ext as the start.
 */
fwr_status fwr_hudgin_extend(fwr_plan_t plan, const float *d_slopes, float *d_ext, int32_t B);

/* ------------------------------------------------------------------------
 * Forward slope model (the sensor of a simulation loop).
 *
 * fwr_fried_slopes: the plan's Fried slope model (Sec. 2, the geometry the reconstruction
 * inverts) applied to node phases: s_x(i, j) = (phi(i, j+1) - phi(i, j) + phi(i+1, j+1)
 * - phi(i+1, j)) / 2 and s_y(i, j) = (phi(i+1, j) - phi(i, j) + phi(i+1, j+1) -
 * phi(i, j+1)) / 2, plus d_noise when it is not NULL, zero on the subapertures the
 * plan's mask marks invalid.  d_phase: float[B][n+1][n+1] (row = y); d_noise:
 * float[B][2][n][n] or NULL; d_slopes: float[B][2][n][n], written.  Plans of the Fried
 * model on any grid (FWR_E_UNSUPPORTED for FWR_MODEL_SINC: that model needs the
 * continuous phase, not node values).  B = 0 is a no-op; B > max_batch or a NULL
 * phase / slope pointer is FWR_E_INVAL.  Asynchronous on the plan's stream.
 */
fwr_status fwr_fried_slopes(fwr_plan_t plan, const float *d_phase, const float *d_noise, float *d_slopes,
                            int32_t B);

/* ------------------------------------------------------------------------
 * Mixed batches and synthetic frames.
 *
 * fwr_reconstruct_group: several plans (grid sizes, iteration counts) with their
 * batches in one call.  The items run concurrently: one on `stream`
 * (hipStream_t; the first multi-pass item, else the first item), the others
 * on library-owned streams that fork from and join back into `stream`
 * (captured as parallel branches when `stream` is being captured into a HIP
 * graph).  Each item is as
 * fwr_reconstruct (d_start / d_resid optional, as fwr_reconstruct_start).  A
 * plan may appear in one item only (its workspace serves one batch at a time);
 * one call at a time per process.  Every item is checked before anything is
 * enqueued (the first failing item's status; nothing runs).  The first call
 * creates max(8, n_work - 1) streams and events on the current device, later
 * calls with more items add streams; a call made while `stream` is being captured
 * that would need new streams gives FWR_E_UNSUPPORTED, so make one call with
 * at least as many items before capturing.  After a failed launch the other
 * branches still join `stream` (FWR_E_DEVICE).
 */
typedef struct {
  fwr_plan_t plan;
  const float *d_slopes;    /* [B][2][n][n] */
  float *d_phase;           /* [B][n+1][n+1] */
  const float *d_start;     /* optional [B][2][N][N] start slopes, NULL = zeros */
  float *d_resid;           /* optional [B] residual */
  int32_t B;
} fwr_work;
fwr_status fwr_reconstruct_group(const fwr_work *work, int32_t n_work, void *stream);

/* fwr_generate: synthetic frames on the device for the plan's geometry, a
 * stand-in for measured data: a periodic von Karman phase screen on the padded
 * N x N grid (pitch = the plan's d, Fried parameter r0 and outer scale L0 [m],
 * phase in radians at the r0 wavelength), its Fried slopes on the lenslet
 * window (grid cells [o, o+n)), white Gaussian noise of `noise_sigma` [rad],
 * zeros on invalid subapertures.  Frame i of the batch is frame
 * first_frame + i (+ *d_counter when d_counter != NULL) of the sequence keyed
 * by `seed` (Philox4x32-10 counters, so a frame does not depend on its batch);
 * first_frame must be even.  When d_counter (DEVICE uint64) is given it is
 * advanced by the batch size rounded up to even afterwards (frames come in pairs), so a graph
 * replay draws fresh frames.
 * d_slopes: float[B][2][n][n]; d_phase (optional): float[B][n+1][n+1] true node phase.
 * Random numbers, for frame pair p (frames 2p, 2p+1) and key (seed low, seed high word):
 *   spectral sample (l, k), l, k in [0, N): Philox counter (p low, p high, l N + k, 0),
 *     words 0, 1 -> Box-Muller -> (g0, g1); screen pair = sum of (g0 + i g1) a(l, k)
 *     e^{+2 pi i (l m + k n) / N}, a = sqrt(Phi_vK(kappa)) / (N d), a(0, 0) = 0; the real
 *     part is frame 2p, the imaginary part frame 2p+1;
 *   noise of subaperture idx = i n + j: counter (p low, p high, idx, 1), words 0, 1 -> x, y
 *     noise of frame 2p, words 2, 3 -> x, y noise of frame 2p+1;
 *   Box-Muller on words (a, b): u1 = ((a >> 8) + 1) / 2^24, u2 = (b >> 8) / 2^24,
 *     (r cos 2 pi u2, r sin 2 pi u2), r = sqrt(-2 ln u1).
 * Uses the plan's stream (and, for N = 256, its workspace). */
fwr_status fwr_generate(fwr_plan_t plan, uint64_t seed, uint64_t first_frame, uint64_t *d_counter, float r0,
                        float L0, float noise_sigma, float *d_slopes, float *d_phase, int32_t B);

/* ------------------------------------------------------------------------
 * Learned initial extension (not part of the paper's method).
 *
 * A seven-layer 3x3 CNN (channels 3-32-32-32-32-32-32-2, ReLU after all but
 * the last layer, zero "same" padding) maps (padded x slopes, padded y slopes,
 * pupil indicator) on the N x N grid to x and y slopes on the whole grid; its
 * values outside the pupil start Algorithm 1 (fwr_*_start).  BF16 weights and
 * activations, FP32 accumulation (MFMA), FP32 master weights and Adam state.
 * Inputs are scaled by `input_scale` before the network and outputs divided by
 * it.  Parameters use the layout: for each layer, weights [out][in][3][3] then
 * biases [out], float32, 47714 values in total.
 */
typedef struct fwr_cnn_s *fwr_cnn_t;

/* mask: HOST n*n valid-subaperture bytes (as for fwr_plan); N >= 16 and N*N a
 * multiple of 64 (FWR_E_UNSUPPORTED otherwise).  training = 0 keeps two activation buffers (inference);
 * training = 1 keeps every layer's activations and gradient buffers.  Weights
 * start at zero: call fwr_cnn_set_params. */
fwr_status fwr_cnn_create(int32_t n_sub, int32_t n_grid, const uint8_t *mask, int32_t max_batch, float input_scale,
                          int32_t training, void *stream, fwr_cnn_t *out);
/* HOST parameter arrays of `count` = 47714 floats. set resets the Adam state. */
fwr_status fwr_cnn_set_params(fwr_cnn_t cnn, const float *h_params, int32_t count);
fwr_status fwr_cnn_get_params(fwr_cnn_t cnn, float *h_params, int32_t count);
/* d_slopes: float[B][2][n][n]; d_pred: float[B][2][N][N] predicted slopes.
 * Enqueues kernels only (may be captured in a HIP graph). */
fwr_status fwr_cnn_forward(fwr_cnn_t cnn, const float *d_slopes, float *d_pred, int32_t B);
/* After fwr_cnn_forward on the same batch (training mode): loss = mean over the
 * out-of-pupil cells of both channels of (scaled prediction - scaled target)^2,
 * gradients of every parameter into the plan's gradient buffer; *h_loss (may be
 * NULL) receives the loss (the call then waits for the stream).  Clears its
 * gradient buffers with memsets: not for graph capture. */
fwr_status fwr_cnn_backward(fwr_cnn_t cnn, const float *d_pred, const float *d_target, int32_t B, float *h_loss);
/* The loss of fwr_cnn_backward for any prediction-shaped map: d_pred, d_target
 * float[B][2][N][N] in slope units; writes d_grad, float[B][2][N][N], the gradient
 * of the loss with respect to d_pred (2 s^2 (pred - target) / count outside the
 * pupil, 0 inside, s = input_scale, count = 2 B times the out-of-pupil cells).
 * Used to train the network through Algorithm 1: the loop is linear in its start
 * and its out-of-pupil map is symmetric, so the gradient of a loss on the
 * extension after k iterations is the same k-iteration loop run on that loss's
 * gradient with zero measurements (fwr_extend_start).  *h_loss as for
 * fwr_cnn_backward. */
fwr_status fwr_cnn_loss_grad(fwr_cnn_t cnn, const float *d_pred, const float *d_target, float *d_grad, int32_t B,
                             float *h_loss);
/* After fwr_cnn_forward on the same batch (training mode): gradients of every
 * parameter from d_grad, float[B][2][N][N], the gradient of the caller's loss with
 * respect to the network's prediction (slope units), into the gradient buffer
 * read by fwr_cnn_get_grads and used by fwr_cnn_adam_step.  Clears the buffer
 * with a memset: not for graph capture. */
fwr_status fwr_cnn_backward_grad(fwr_cnn_t cnn, const float *d_grad, int32_t B);
fwr_status fwr_cnn_get_grads(fwr_cnn_t cnn, float *h_grads, int32_t count);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr. */
fwr_status fwr_cnn_adam_step(fwr_cnn_t cnn, float lr);
/* Rebind the network to another stream (hipStream_t), e.g. a stream being captured. */
fwr_status fwr_cnn_set_stream(fwr_cnn_t cnn, void *stream);
fwr_status fwr_cnn_destroy(fwr_cnn_t cnn);

/* Learned start with the plain loop as fallback, in one call: the network's
 * prediction (written to d_start, float[B][2][N][N]) starts Algorithm 1 with
 * `plan` (its n_iter >= 1; phase to d_phase, float[B][n+1][n+1]; in-pupil
 * residual of the last iteration to d_resid, float[B], as fwr_reconstruct_start);
 * the frames whose residual exceeds `threshold` are then recomputed from the
 * zero-padded start with `fallback` (same n and N, its own n_iter and Eq. 5
 * setting) and their phase replaced.  *h_count (may be NULL) receives the
 * number of recomputed frames.  plan, fallback and cnn must enqueue on the same
 * stream and hold B frames (FWR_E_INVAL otherwise; on-chip grids only).  The
 * call waits for the stream once, to size the fallback batch, so it cannot be
 * captured in a graph.  The first call allocates gather buffers for
 * fallback->max_batch frames in the fallback plan (freed by fwr_destroy); calls
 * that share a fallback plan must not overlap. */
fwr_status fwr_reconstruct_learned(fwr_plan_t plan, fwr_plan_t fallback, fwr_cnn_t cnn, const float *d_slopes,
                                   float *d_start, float *d_phase, float *d_resid, float threshold, int32_t B,
                                   int32_t *h_count);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): fwr_reconstruct_learned
 * without any allocation and without waiting for the stream.  Same arguments,
 * checks and results (bit for bit) as fwr_reconstruct_learned, except:
 *   - the number of recomputed frames goes to d_count (DEVICE int32, may be
 *     NULL) instead of a host variable; nothing is read back;
 *   - the frame list and the gathered slopes and phases of the fallback live in
 *     one fixed library workspace per GPU of FWR_NOALLOC_SCRATCH_BYTES (16 MiB,
 *     held until the process ends), not in buffers of the fallback plan.  The
 *     fallback runs in chunks that fit it (at most 2 * floor(S / (8 (2 n^2 +
 *     (n+1)^2))) frames per chunk, S the workspace after the frame list), each
 *     launch sized for a full chunk, the frames past the device-side count
 *     exiting at once;
 *   - B <= FWR_NOALLOC_MAX_FRAMES (FWR_E_INVAL beyond); the fallback plan must
 *     use the Fried model (FWR_E_UNSUPPORTED otherwise).
 * Every call on a GPU shares that GPU's workspace, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads) race and
 * must be ordered by the caller.  The workspace's address is looked up once per
 * device on the first call there (no allocation). */
#define FWR_NOALLOC_SCRATCH_BYTES (16u << 20)
#define FWR_NOALLOC_MAX_FRAMES 65536
fwr_status fwr_reconstruct_learned_noalloc(fwr_plan_t plan, fwr_plan_t fallback, fwr_cnn_t cnn,
                                           const float *d_slopes, float *d_start, float *d_phase,
                                           float *d_resid, float threshold, int32_t B, int32_t *d_count);

/* Static description of a status code (never NULL). */
const char *fwr_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* FWR_H */
