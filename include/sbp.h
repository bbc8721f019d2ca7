/*
 * sbp.h -- C-ABI of the sliding-ball (point-cloud) photoacoustic reconstruction
 * hot path on AMD Instinct MI355X (gfx950).
 *
 * The method is SlingBAG Pro (Li et al., arXiv 2601.00551): a 3-D photoacoustic
 * source is a cloud of balls (centre x, y, z, peak pressure p0, size a); a
 * differentiable forward model ("Simulate", section 4.2 and 4.3) predicts every
 * transducer's time series; the squared L2 residual is minimised by gradient
 * steps on the ball parameters (section 4.1, Algorithm 1), after a
 * zero-gradient filter has pruned the initial cloud (section 4.2) and while
 * the sampling rate is raised level by level (section 4.3).
 *
 * Conventions shared by every call
 *   Units: mm, us; c in mm/us.
 *   Memory: every data pointer is DEVICE memory owned by the caller.  The
 *     library never frees or keeps a pointer past the call.  Outputs are
 *     preallocated by the caller at the sizes stated.  The context owns only
 *     its internal scratch memory.
 *   Balls are structure-of-arrays.  Frames (independent reconstructions that
 *     share one transducer array) are stored back to back: frame f owns balls
 *     [ball_off[f], ball_off[f+1]).  ball_off is a DEVICE array of F+1 int64
 *     with ball_off[0] = 0; B_cap is a host-side upper bound on ball_off[F]
 *     (it sizes launches; the kernels read the true counts on the device, so a
 *     call can be captured in a HIP graph while counts change between replays).
 *   Signals are [F][D][T] row-major, T = the level's sample count T_k.
 *   Streams: `stream` is a hipStream_t (NULL = the null stream).  Every call is
 *     asynchronous on it; host-visible results (loss, counts) are ready only
 *     after the caller synchronises, unless a call says otherwise.
 *   Errors: every call returns SBP_OK (0) or a negative code and then sets a
 *     thread-local message readable with sbp_last_error().  Arguments are
 *     validated on the host BEFORE anything is enqueued, in the order: pointers
 *     and sizes, model fields, then the context; so a failed call enqueues
 *     nothing.
 *   Non-finite ball parameters (invalid input): a ball whose stored x, y, z,
 *     p0 or a (a~ under softplus) is NaN or infinite makes every sample of its
 *     frame NaN in sbp_simulate_signals (and its _f64 twin); its gradients are
 *     NaN in sbp_adjoint_gradients; sbp_filter_zero_grad gives it g = NaN and
 *     drops it.  Other frames and balls are computed as if it were absent
 *     (their fixed-point quantum included).  A non-finite cotangent value
 *     reaches the gradients of the balls whose pulse covers it.
 *   A context is used by one host thread and one stream at a time
 *     (its scratch memory is shared by the calls made through it); a captured
 *     graph owns its own workspace and may run on another stream.
 */
#ifndef SBP_H
#define SBP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ codes ----- */
#define SBP_OK 0
#define SBP_E_ARG (-1)      /* null pointer, negative or inconsistent size, F < 1 */
#define SBP_E_DOMAIN (-2)   /* c <= 0, dt <= 0, f < 1, T < 1, unknown enum, K outside (0, 12] */
#define SBP_E_HIP (-3)      /* a HIP runtime error; message in sbp_last_error() */
#define SBP_E_NOMEM (-4)    /* the context could not grow its scratch memory */
#define SBP_E_CAPACITY (-5) /* an output would exceed the caller's capacity */

#define SBP_PROFILE_UNIFORM 0 /* fhat(s) = 1 for |s| < a: the textbook N-shaped pulse */
#define SBP_PROFILE_GAUSS 1   /* fhat(s) = exp(-s^2 / (2 a^2)) for |s| < K a (section 4.1) */
#define SBP_DIR_OMNI 0        /* every transducer hears every direction equally */
#define SBP_DIR_COS 1         /* trace scaled by max(0, n_hat . e_hat) */
#define SBP_SAMPLING_BIN 0    /* sample n = mean pressure over [t0 + n dt_k, t0 + (n+1) dt_k) */
#define SBP_SAMPLING_POINT 1  /* sample n = pressure at t0 + n dt_k (GAUSS only) */

/* Gradient / update masks over the five ball parameters. */
#define SBP_X 1u
#define SBP_Y 2u
#define SBP_Z 4u
#define SBP_P0 8u
#define SBP_A 16u
#define SBP_XYZ 7u
#define SBP_ALL 31u
#define SBP_COARSE (SBP_P0 | SBP_A) /* coarse stage: positions fixed (section 4.1) */

#define SBP_MAX_FRAMES 64 /* F may not exceed this */
#define SBP_MAX_TAPS 4095 /* longest transducer response, in taps */

/* ------------------------------------------------------------ types ----- */

/* Forward model of one temporal level k (section 4.3: dt_k = f_k dt, T_k = T/f_k).
 * Sample n of a transducer is the mean pressure over the time bin
 * [t0 + n f dt, t0 + (n+1) f dt) (sampling = SBP_SAMPLING_BIN), or the
 * pressure at t0 + n f dt (SBP_SAMPLING_POINT, GAUSS profile only; its
 * pyramid is sbp_decimate).  a_softplus = 1 means the `a` arrays hold the
 * unconstrained a~ and the size is a = softplus(a~) = log(1 + e^a~) (the
 * positivity-constrained refinement of section 4.3); gradients are then with
 * respect to a~.
 * Transducer response (optional; response = NULL leaves it out, and the other
 * three response fields are then ignored): the modelled record is the
 * simulated record convolved in time with the element's impulse response,
 *   y[f][d][n] = sum_{j < L} h[row(d)][j] * s[f][d][n + zero - j]
 * (s the record described under sbp_simulate_signals, zero outside [0, T)),
 * with tap j at lag (j - zero) dt_k, row(d) = d when response_rows = D and 0
 * when response_rows = 1.  The taps must be those of this level's interval
 * dt_k (sbp_response_taps).  sbp_simulate_signals then returns y,
 * sbp_adjoint_gradients and sbp_filter_zero_grad take their cotangent and
 * reference with respect to y (they correlate it with the taps first), and
 * sbp_step fits y to y_ref.  The three calls and the step need F D T more
 * elements of scratch for the intermediate record. */
typedef struct sbp_model {
    double c;          /* speed of sound, mm/us, > 0 */
    double dt;         /* base sample interval, us, > 0 */
    double t0;         /* time of the first bin edge, us */
    double gauss_K;    /* GAUSS truncation in units of a, 0 < K <= 12 (5 is the default;
                          the tail beyond 12 a is below e^-72 of the peak) */
    int32_t T;         /* samples at this level, >= 1 */
    int32_t f;         /* downsampling factor of this level, >= 1 */
    int32_t profile;   /* SBP_PROFILE_* */
    int32_t directivity; /* SBP_DIR_* */
    int32_t a_softplus;  /* 0 or 1 */
    int32_t sampling;    /* SBP_SAMPLING_*; other values: SBP_E_DOMAIN */
    const float *response; /* NULL, or device taps [response_rows][response_taps] */
    int32_t response_taps; /* L, 1..SBP_MAX_TAPS */
    int32_t response_zero; /* the tap at zero lag, 0 <= zero < L */
    int32_t response_rows; /* 1 (one response for every transducer) or D */
    int32_t reserved;      /* 0 */
} sbp_model;

/* Transducer array: D positions q and unit normals n (SoA, device, float). */
typedef struct sbp_array {
    const float *qx, *qy, *qz;
    const float *nx, *ny, *nz;
    int32_t D;
    int32_t reserved;
} sbp_array;

/* Ball parameters or their gradients (SoA, device, float). */
typedef struct sbp_balls {
    float *x, *y, *z, *p0, *a;
} sbp_balls;

/* FP64 twins, used only by the double-precision entry points. */
typedef struct sbp_array_f64 {
    const double *qx, *qy, *qz;
    const double *nx, *ny, *nz;
    int32_t D;
    int32_t reserved;
} sbp_array_f64;

typedef struct sbp_balls_f64 {
    double *x, *y, *z, *p0, *a;
} sbp_balls_f64;

/* Adam hyper-parameters (PyTorch semantics: bias-corrected moments, eps added
 * after the square root).  lr is per parameter (x, y, z, p0, a). */
typedef struct sbp_adam_params {
    float lr[5];
    float beta1, beta2, eps;
    int32_t step;      /* 1-based step count of this update */
    uint32_t mask;     /* parameters to update (SBP_* bits) */
} sbp_adam_params;

/* Everything one reconstruction iteration touches (all device memory except
 * the two sizes).  grad is a gradient workspace of capacity B_cap; m and v are
 * the Adam moments. */
typedef struct sbp_state {
    sbp_balls balls;
    sbp_balls grad;
    sbp_balls m;
    sbp_balls v;
    int64_t *ball_off; /* F+1, device */
    int32_t F;
    int32_t reserved;
    int64_t B_cap;
} sbp_state;

/* Plain growth rule (section 4.1: split / destroy / duplicate by thresholds on
 * pressure and size; the paper does not give the thresholds).  Per frame:
 * destroy balls with p0 < destroy_frac * max p0 or a < a_min; split balls with
 * a > a_split into two children at -/+ a/2 along the axis of the largest
 * |position gradient| (size a / 2^(1/3), same p0); duplicate the
 * floor(dup_frac * n) non-split survivors of largest |grad r| (ties: lower
 * index) with a clone offset by -dup_offset * a * grad r / |grad r| (a ball
 * with zero position gradient gets a clone on itself).  Output per frame:
 * survivors in input order with split balls replaced in place by their two
 * children, then the clones in input order.  New balls get zero moments.  The
 * thresholds are float32 fields and the rule is defined on those values: the
 * destroy threshold is destroy_frac * max p0 rounded to float32, and
 * floor(dup_frac * n) is taken exactly from the float32 dup_frac (0.7 is
 * 0.699999988, so ten candidates give six clones). */
typedef struct sbp_growth_rule {
    float destroy_frac;
    float a_min;
    float a_split;
    float dup_frac;
    float dup_offset;
    int32_t reserved;
} sbp_growth_rule;

/* Launch shape of the forward and adjoint kernels (chosen by the autotuner).
 * sbp_ctx_set_tuning rejects values outside the ranges below.  When a level's
 * rows do not fit the LDS, the row count is lowered for that call. */
typedef struct sbp_tuning {
    int32_t fwd_dets;     /* transducer rows accumulated in LDS per workgroup, 1..16 */
    int32_t fwd_block;    /* threads per workgroup: 64, 128, 256 or 512 */
    int32_t fwd_bpt;      /* balls per thread per work item, 1..16 */
    int32_t fwd_grid;     /* persistent workgroups, 0 = as many as fit on the device */
    int32_t adj_dets;     /* transducer rows staged in LDS per pass, 1..16 */
    int32_t adj_block;    /* threads per workgroup: 64, 128, 256 or 512 */
    int32_t adj_bpt;      /* balls per thread, 1..3 */
    int32_t adj_grid;     /* persistent workgroups, 0 = as many as fit on the device */
    int32_t fwd_tile;     /* samples per LDS time tile, 0 = as many as fit, else >= 64 */
    int32_t adj_tile;     /* edges per LDS time tile, 0 = as many as fit, else >= 64 */
} sbp_tuning;

typedef struct sbp_ctx sbp_ctx;
typedef struct sbp_graph sbp_graph;

/* ---------------------------------------------------- context & errors -- */

/* Message of the last failed call on this thread ("" if none).  The pointer
 * stays valid until the next call on this thread. */
const char *sbp_last_error(void);

/* Create a context on HIP device `device` (it becomes current on this thread).
 * Errors: SBP_E_ARG (out NULL, device < 0), SBP_E_HIP (no such device). */
int sbp_ctx_create(sbp_ctx **out, int device);

/* Free the context and its scratch memory; NULL is accepted. */
int sbp_ctx_destroy(sbp_ctx *ctx);

/* Number of compute units of the context's device (host value). */
int sbp_ctx_num_cus(const sbp_ctx *ctx, int32_t *out);

/* Set / read the forward and adjoint launch shapes of this context. */
int sbp_ctx_set_tuning(sbp_ctx *ctx, const sbp_tuning *t);
int sbp_ctx_get_tuning(const sbp_ctx *ctx, sbp_tuning *t);

/* ------------------------------------------------------------ the path -- */

/* Downsample_f of section 4.3: y_out[r][n] = (1/f) sum_{j<f} y[r][n f + j] for
 * n < T/f (integer division; a tail shorter than f is dropped), for R = F*D
 * rows of length T.  y_out holds R * (T/f) floats.
 * Errors: SBP_E_ARG (NULL, R < 1), SBP_E_DOMAIN (f < 1, T/f < 1). */
int sbp_downsample(sbp_ctx *ctx, const float *y, int64_t R, int32_t T, int32_t f,
                   float *y_out, void *stream);

/* Decimation, the pyramid that pairs with SBP_SAMPLING_POINT (a point-sampled
 * record at dt, decimated by f, is the point-sampled record at f dt):
 * y_out[r][n] = y[r][n f] for n < T/f, R rows of length T; y_out holds
 * R * (T/f) floats.
 * Errors: SBP_E_ARG (NULL, R < 1), SBP_E_DOMAIN (f < 1, T/f < 1). */
int sbp_decimate(sbp_ctx *ctx, const float *y, int64_t R, int32_t T, int32_t f,
                 float *y_out, void *stream);

/* Simulate of section 4.2 / 4.3: y[f][d][n] = sum over the balls i of frame f of
 *   p0_i * D_id / (2 rho_id c dt_k) * (psi(u_n) - psi(u_{n+1})),
 *   u_m = rho_id - c (t0 + m dt_k),
 * the bin mean of the closed-form pressure pulse of ball i at transducer d
 * (psi is the antiderivative of u * fhat(u), zero outside the support;
 * rho_id = |r_i - q_d|; D_id is the directivity).  Pairs with
 * rho_id <= support half-width and balls with a <= 0 contribute nothing.
 * Under model->sampling = SBP_SAMPLING_POINT (GAUSS) sample n is instead the
 * pressure p0_i D_id u_n fhat(u_n) / (2 rho_id) itself, |u_n| < K a; the
 * adjoint and the filter follow the same model.
 * y is [F][D][model->T]; it is overwritten unless accumulate = 1.  Every
 * value a ball adds is rounded to the nearest multiple of a per-call
 * power-of-two quantum q and the multiples are summed exactly, so the result
 * is bitwise reproducible however the work is split.  The values are bin
 * values (UNIFORM), point samples, or, for GAUSS bin means, the pulse's
 * antiderivative at the bin edges (a sample is then the difference of its two
 * edges' sums).  q is the power of two with bound / 2^30 < q <= bound / 2^29,
 * bound = max over the call's finite balls of |p0| a / (2 K c dt_k) (GAUSS;
 * |p0| a / (4 c dt_k) UNIFORM, |p0| / (2 K) point samples), the largest value
 * any one ball can add.  The rounding error is absolute and unbiased: at most
 * half a quantum per ball reaching a sample (one quantum for GAUSS bin means,
 * two roundings), so a ball whose values are 10^k times smaller than the
 * bound keeps about 29 - 3.3 k significant bits.
 * The context's scratch holds 8 bytes per output sample (plus one per
 * transducer row) and 24 bytes per ball of B_cap during the call, and 4 more
 * per output sample with a transducer response (the record before it).
 * Errors: SBP_E_ARG, SBP_E_DOMAIN, SBP_E_HIP, SBP_E_NOMEM. */
int sbp_simulate_signals(sbp_ctx *ctx, const sbp_array *arr, const sbp_balls *balls,
                         const int64_t *ball_off, int32_t F, int64_t B_cap,
                         const sbp_model *model, float *y, int32_t accumulate, void *stream);

/* sbp_simulate_signals for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same result bit for bit, but the call's
 * workspace is a fixed device array of 128 MiB per GPU, held from the first
 * sbp_ctx_create on that GPU until the process ends, instead of the
 * context's scratch; the call makes no allocation of any kind.  Limit: the
 * workspace the call needs, 8 (T + 1) F D + 24 B_cap bytes, plus 4 T F D with
 * a transducer response (each part rounded up to 256 bytes), plus 512, must
 * fit in 128 MiB, else SBP_E_CAPACITY before
 * anything is enqueued.  Every call on one GPU, through any context, shares
 * that GPU's array: the call clears what it needs zeroed, but calls that
 * overlap on one GPU (other streams, other threads) race and must not be
 * issued.  Errors: as sbp_simulate_signals, plus SBP_E_CAPACITY. */
int sbp_simulate_signals_noalloc(sbp_ctx *ctx, const sbp_array *arr, const sbp_balls *balls,
                                 const int64_t *ball_off, int32_t F, int64_t B_cap,
                                 const sbp_model *model, float *y, int32_t accumulate,
                                 void *stream);

/* Data-fidelity loss of section 4.2 / 4.3: with e = y_sim - y_ref,
 * loss[f] = sum over frame f of e^2 (a sum, no 1/N), computed in FP64, and
 * (if v_out is not NULL) v_out = 2 e = dL/dy_sim.  v_out may alias y_sim.
 * n_per_frame = D * T.  loss is a DEVICE array of F doubles.
 * Errors: SBP_E_ARG. */
int sbp_residual_loss(sbp_ctx *ctx, const float *y_sim, const float *y_ref, int64_t n_per_frame,
                      int32_t F, float *v_out, double *loss, void *stream);

/* Backpropagation of section 4.2 / Algorithm 1 as a vector-Jacobian product:
 * grad.theta[i] = sum_{d,n} v[f][d][n] * d y[f][d][n] / d theta_i for every
 * parameter theta in `mask` (SBP_* bits).  v = dL/dy; for the L2 loss the
 * caller passes v = 2 (y_sim - y_ref) (the factor 2 is not applied here).
 * Gradient arrays outside `mask` may be NULL and are not touched; those in
 * the mask are overwritten for balls [0, ball_off[F]).  Small clouds are split
 * over transducer slices whose partial sums (in the context's scratch) are
 * added in a fixed order: results are reproducible run to run.
 * Errors: SBP_E_ARG (mask 0 or a needed pointer NULL), SBP_E_DOMAIN, SBP_E_HIP,
 * SBP_E_NOMEM. */
int sbp_adjoint_gradients(sbp_ctx *ctx, const sbp_array *arr, const sbp_balls *balls,
                          const int64_t *ball_off, int32_t F, int64_t B_cap,
                          const sbp_model *model, const float *v, uint32_t mask,
                          sbp_balls *grad, void *stream);

/* Zero-gradient filtering of section 4.2 and Algorithm 1.  With every p0 set
 * to 0 the simulated signal vanishes, so g_i = dL/dp0_i = -2 <y_ref, h_i>
 * with h_i ball i's unit-p0 signal; ball i is kept if g_i < 0 (strict = 1,
 * Algorithm 1) or g_i <= 0 (strict = 0, the inequalities of section 4.2).
 * Kept balls are copied, in their original order, to `out` with their stored
 * p0 (the restore step); off_out (device, F+1) receives the new frame
 * offsets.  g_out (nullable, [B_cap]) receives g.  mom_in/mom_out (both
 * nullable; if one is given the other must be) compact the Adam moments the
 * same way.  `out` must not overlap `in`.  Capacity of `out`: B_cap.
 * g is formed with the balls visited in a spatial order (a counting sort by
 * Morton cell, built per call in the context's scratch, about 8 bytes per
 * ball of B_cap); each g_i equals the storage-order value bit for bit.
 * Errors: SBP_E_ARG, SBP_E_DOMAIN, SBP_E_HIP, SBP_E_NOMEM. */
int sbp_filter_zero_grad(sbp_ctx *ctx, const sbp_array *arr, const sbp_balls *in,
                         const int64_t *off_in, int32_t F, int64_t B_cap, const sbp_model *model,
                         const float *y_ref, int32_t strict, sbp_balls *out, int64_t *off_out,
                         float *g_out, const sbp_balls *m_in, const sbp_balls *v_in,
                         sbp_balls *m_out, sbp_balls *v_out, void *stream);

/* One Adam update (PyTorch semantics) of the parameters in p->mask for balls
 * [0, ball_off[F]):  m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 * theta -= lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps).
 * If step_dev is not NULL the step count t is read from that device int32
 * (so a captured graph can advance it) instead of p->step.
 * Errors: SBP_E_ARG, SBP_E_DOMAIN (betas outside [0,1), step < 1). */
int sbp_adam_update(sbp_ctx *ctx, sbp_state *state, const sbp_adam_params *p,
                    const int32_t *step_dev, void *stream);

/* One reconstruction iteration of Algorithm 1 at level `model`:
 * simulate (y_work) -> residual and loss (y_work becomes 2 e) -> adjoint for
 * p->mask -> Adam on p->mask.  loss (device, F doubles) receives the loss of
 * the balls as they were before the update.  y_ref and y_work are [F][D][T].
 * Errors: as the calls above. */
int sbp_step(sbp_ctx *ctx, const sbp_array *arr, sbp_state *state, const sbp_model *model,
             const float *y_ref, float *y_work, const sbp_adam_params *p, double *loss,
             void *stream);

/* Capture `iters` consecutive sbp_step iterations into one HIP graph.
 * Iteration i of a launch uses the step count *step_dev + i (device int32),
 * and the launch ends by adding iters to *step_dev, so successive launches
 * continue the Adam schedule.  loss receives iters * F doubles (iteration-major).  The ball
 * counts in state->ball_off may change between launches (up to B_cap).  The
 * graph keeps the pointers it was created with.
 * Errors: as sbp_step, plus SBP_E_HIP on capture failure. */
int sbp_step_graph_create(sbp_ctx *ctx, const sbp_array *arr, sbp_state *state,
                          const sbp_model *model, const float *y_ref, float *y_work,
                          const sbp_adam_params *p, int32_t *step_dev, double *loss,
                          int32_t iters, sbp_graph **out, void *stream);
int sbp_graph_launch(sbp_graph *g, void *stream);
int sbp_graph_destroy(sbp_graph *g);

/* Switch the size parameterisation of the positivity-constrained refinement
 * (section 4.3): to_softplus = 1 replaces every a in state->balls.a (balls
 * [0, ball_off[F])) by a~ = log(e^a - 1), so that a = softplus(a~) (a <= 0
 * becomes a~ = -88); to_softplus = 0 replaces a~ by softplus(a~).  Calls that
 * follow must set model->a_softplus to match.  state->m.a and state->v.a, if
 * not NULL, are reset to zero (the optimised variable changes).
 * Errors: SBP_E_ARG. */
int sbp_softplus_reparam(sbp_ctx *ctx, sbp_state *state, int32_t to_softplus, void *stream);

/* Plain growth rule (see sbp_growth_rule) applied to `in` (uses in->grad for
 * the split axis and the duplication ranking) and written to `out`
 * (balls, zeroed-or-copied moments, ball_off); out->B_cap is its capacity.
 * This call synchronises `stream` to return the new total in *count (host).
 * Errors: SBP_E_ARG, SBP_E_CAPACITY (out->B_cap too small; out is then
 * unspecified), SBP_E_HIP. */
int sbp_grow(sbp_ctx *ctx, const sbp_state *in, const sbp_growth_rule *rule, sbp_state *out,
             int64_t *count, void *stream);

/* ------------------------------------------- transducer response ----- */
/* The elements of the in vivo array of section 2.2 have a mean centre
 * frequency of 2.02 MHz and a bandwidth of 54 %; the forward model of
 * sections 4.2 and 4.3 leaves the element's response out.  These calls model
 * it as a Gaussian-envelope cosine,
 *   h(t) = A exp(-t^2 / (2 s_t^2)) cos(2 pi fc t),
 * whose amplitude spectrum is a Gaussian centred on fc with full width bw fc
 * at half its peak (-6 dB): s_f = bw fc / (2 sqrt(2 ln 2)),
 * s_t = 1 / (2 pi s_f), A = 2 / (s_t sqrt(2 pi)) (unit gain at fc).  fc in
 * MHz, bw a fraction, t in us. */

/* Tap count and zero-lag tap that cover +-n_sigma envelope widths s_t of the
 * widest response (the one of least fc * bw) at interval dt_k:
 * zero = ceil(n_sigma s_t / dt_k), L = 2 zero + 1.  Host-only; no context.
 * Errors: SBP_E_ARG (NULL outputs), SBP_E_DOMAIN (fc, bw, dt_k or n_sigma
 * not positive and finite), SBP_E_CAPACITY (L > SBP_MAX_TAPS). */
int sbp_response_length(double fc, double bw, double dt_k, double n_sigma, int32_t *L,
                        int32_t *zero);

/* Taps h[r][j] = dt_k h_r((j - zero) dt_k) of rows responses (device arrays
 * fc[rows], bw[rows]), computed in FP64 and rounded to float once; the factor
 * dt_k turns the convolution integral into the sum over taps.  h is
 * [rows][L], device.  A row whose fc or bw is not positive and finite gets
 * NaN taps.
 * Errors: SBP_E_ARG (NULL, rows < 1), SBP_E_DOMAIN (dt_k not positive and
 * finite, L outside [1, SBP_MAX_TAPS], zero outside [0, L)). */
int sbp_response_taps(sbp_ctx *ctx, const float *fc, const float *bw, int32_t rows, double dt_k,
                      int32_t L, int32_t zero, float *h, void *stream);

/* Apply the response to R = F D records of T samples (row r is transducer
 * r mod D):
 *   adjoint = 0:  out[r][n] (+)= sum_j h[row][j] y[r][n + zero - j]
 *   adjoint = 1:  out[r][n] (+)= sum_j h[row][j] y[r][n - zero + j]
 * (the correlation, the adjoint of the convolution), zeros outside [0, T),
 * row = 0 when rows_h = 1 and r mod D when rows_h = D.  The sum runs in the
 * records' precision with the taps in a fixed order, so results are
 * reproducible.  out is overwritten unless accumulate = 1; it must not
 * overlap y.
 * Errors: SBP_E_ARG (NULL, R < 1, D < 1, R not a multiple of D when
 * rows_h = D, rows_h not 1 or D, out overlapping y, flags not 0 or 1),
 * SBP_E_DOMAIN (T < 1, L outside [1, SBP_MAX_TAPS], zero outside [0, L)). */
int sbp_response_apply(sbp_ctx *ctx, const float *h, int32_t rows_h, int32_t L, int32_t zero,
                       const float *y, int64_t R, int32_t D, int32_t T, int32_t adjoint,
                       int32_t accumulate, float *out, void *stream);

/* Double-precision twins of sbp_simulate_signals and sbp_adjoint_gradients
 * (same contract, FP64 buffers), used to check gradients by finite
 * differences. */
int sbp_simulate_signals_f64(sbp_ctx *ctx, const sbp_array_f64 *arr, const sbp_balls_f64 *balls,
                             const int64_t *ball_off, int32_t F, int64_t B_cap,
                             const sbp_model *model, double *y, int32_t accumulate, void *stream);
int sbp_adjoint_gradients_f64(sbp_ctx *ctx, const sbp_array_f64 *arr, const sbp_balls_f64 *balls,
                              const int64_t *ball_off, int32_t F, int64_t B_cap,
                              const sbp_model *model, const double *v, uint32_t mask,
                              sbp_balls_f64 *grad, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SBP_H */
