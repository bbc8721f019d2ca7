/*
 * sbp_mlp.h -- the learned growth-proposal network of the reconstruction
 * (an addition to SlingBAG Pro's plain split / destroy / duplicate rule of
 * section 4.1): a multilayer perceptron 31 -> 256 -> 256 -> 256 -> 2 with ReLU,
 * BF16 operands on the MI355X matrix cores (v_mfma_f32_16x16x32_bf16) and FP32
 * accumulation.  Output 0 is the logit of "grow a ball at this candidate
 * site", output 1 its initial p0.  The plain rule remains the fallback; the
 * data-fidelity loss decides whether the network is used.
 *
 * Conventions are those of sbp.h (device pointers owned by the caller,
 * host-side validation before anything is enqueued, asynchronous on `stream`).
 *
 * Parameters are one flat FP32 vector (row-major [in][out] weights, then the
 * bias), in this order and at these offsets:
 *   W1 [32][256] at 0 (input row 31 is a zero-padding feature), b1 [256] at 8192,
 *   W2 [256][256] at 8448, b2 at 73984, W3 [256][256] at 74240, b3 at 139776,
 *   W4 [256][2] at 140032, b4 [2] at 140544; total SBP_MLP_NPARAM = 140546.
 * The kernels read BF16 working copies (transposed and padded for the matrix
 * cores) kept in a caller-owned buffer of SBP_MLP_NWORK bf16 values, refreshed
 * from the FP32 vector by sbp_mlp_sync (and by sbp_mlp_adam).
 * Row counts M are padded to Mp = multiple of 64 in the training buffers.
 */
#ifndef SBP_MLP_H
#define SBP_MLP_H

#include <stdint.h>

#include "sbp.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SBP_MLP_IN 31
#define SBP_MLP_HID 256
#define SBP_MLP_OUT 2
#define SBP_MLP_NPARAM 140546
#define SBP_MLP_NWORK 278528

/* Refresh the BF16 working copies `work` from the FP32 parameters. */
int sbp_mlp_sync(sbp_ctx *ctx, const float *params, uint16_t *work, void *stream);

/* out[m][0..1] for the rows X[m][0..30] (FP32, row-major), m < M.  X and the
 * weights are rounded to BF16, hidden activations are rounded to BF16 after
 * bias and ReLU, accumulation and the output are FP32.  If acts is not NULL
 * (training) it receives the transposed BF16 input and activations:
 * [32][Mp] input, then [256][Mp] for each hidden layer (zeros in padded rows).
 * Errors: SBP_E_ARG. */
int sbp_mlp_forward(sbp_ctx *ctx, const float *params, const uint16_t *work, const float *X,
                    int64_t M, float *out, uint16_t *acts, void *stream);

/* Training loss over M rows, averaged:
 *   pos_weight * y * softplus(-z) + (1 - y) * softplus(z) + y * (p - p_target)^2,
 * z = out[m][0], p = out[m][1], y = label_grow[m] in {0, 1}.  loss (device,
 * one double) receives the mean; dout [Mp][2] FP32 and dout_t [16][Mp] BF16
 * (rows 2..15 zero) receive d loss / d out. */
int sbp_mlp_loss(sbp_ctx *ctx, const float *out, const float *label_grow, const float *label_p0,
                 int64_t M, float pos_weight, double *loss, float *dout, uint16_t *dout_t,
                 void *stream);

/* Backpropagation through the network: grad (FP32, SBP_MLP_NPARAM, overwritten)
 * = d loss / d params, from the activations of sbp_mlp_forward and the output
 * gradient of sbp_mlp_loss.  dacts is a workspace of 3 * 256 * Mp BF16.  The
 * weight gradients are summed per slice of rows into the context's scratch
 * (up to 256 x 257 x 256 floats, grown on demand) and the slices added in a
 * fixed order, so the result does not depend on scheduling.
 * Errors: SBP_E_ARG (NULL, M < 1), SBP_E_NOMEM (scratch), SBP_E_HIP. */
int sbp_mlp_backward(sbp_ctx *ctx, const uint16_t *work, const uint16_t *acts, const float *dout,
                     const uint16_t *dout_t, int64_t M, uint16_t *dacts, float *grad,
                     void *stream);

/* One Adam step on the flat parameter vector (lr = p->lr[0], PyTorch
 * semantics, p->mask ignored), then refresh `work`. */
int sbp_mlp_adam(sbp_ctx *ctx, float *params, const float *grad, float *m, float *v,
                 const sbp_adam_params *p, uint16_t *work, void *stream);

/* ------------------------------------------------- candidate sites & features */

/* A regular grid of cells: cell (i, j, k) covers
 * [origin + (i, j, k) * h, origin + (i+1, j+1, k+1) * h), 0 <= i < nx etc. */
typedef struct sbp_grid {
    float ox, oy, oz, h;
    int32_t nx, ny, nz, reserved;
} sbp_grid;

/* mass[(i * ny + j) * nz + k] = sum of p0 of the balls of frame 0 (balls
 * [ball_off[0], ball_off[1])) whose centre lies in cell (i, j, k); mass has
 * nx*ny*nz floats and is overwritten (FP32 atomics: the order of the sum is
 * unspecified).  Errors: SBP_E_ARG, SBP_E_DOMAIN (h <= 0, empty grid). */
int sbp_grid_mass(sbp_ctx *ctx, const sbp_balls *balls, const int64_t *ball_off, int64_t B_cap,
                  const sbp_grid *grid, float *mass, void *stream);

/* Candidate growth sites: centres of the cells with mass < occ whose 26
 * neighbours include a cell with mass >= occ, in cell order (i slowest, k
 * fastest).  sites (SoA, capacity cap) receives x, y, z = the cell centre and
 * the probe ball p0 = 1, a = a_probe, ready for sbp_adjoint_gradients;
 * *count (host) the number found (the call synchronises `stream`).
 * Errors: SBP_E_ARG, SBP_E_DOMAIN (h <= 0, empty grid, a_probe <= 0),
 * SBP_E_CAPACITY (more than cap sites; *count still holds the number). */
int sbp_candidates(sbp_ctx *ctx, const sbp_grid *grid, const float *mass, float occ, float a_probe,
                   const sbp_balls *sites, int64_t cap, int64_t *count, void *stream);

/* Feature rows X[m][0..30] (FP32, row-major) of the M candidate sites:
 *   0      -dL/dp0 of the unit probe ball at the site, over max_m |dL/dp0|
 *   1      |dL/dr| of the probe, over its maximum over the sites
 *   2..27  masses of the 26 neighbour cells (di, dj, dk in -1..1, di slowest,
 *          the centre skipped; 0 outside the grid), over the largest cell mass
 *   28..30 the site's x, y, z over `half`
 * (a zero maximum gives zero features).  g holds the probe gradients (p0, x,
 * y, z) from sbp_adjoint_gradients on `sites`.  Errors: SBP_E_ARG,
 * SBP_E_DOMAIN (half <= 0, h <= 0). */
int sbp_features(sbp_ctx *ctx, const sbp_grid *grid, const float *mass, const sbp_balls *sites,
                 int64_t M, const sbp_balls *g, float half, float *X, void *stream);

/* Append the candidates whose logit out[m][0] > 0 to frame 0 of `state`
 * (balls at sites x, y, z with p0 = max(out[m][1], 0) * p0_scale and size
 * a_init, zero gradient and moments), in site order after the existing balls;
 * ball_off[1] grows accordingly.  The new total is returned in *count (host;
 * the call synchronises `stream`).  The same out gives the same sites, so a
 * caller can remove the appended balls (ball_off[1] back to its old value)
 * and append them again with another p0_scale.
 * Errors: SBP_E_ARG (state->F != 1, NULL arrays), SBP_E_DOMAIN (a_init <= 0,
 * p0_scale < 0), SBP_E_CAPACITY (state unchanged). */
int sbp_append_proposals(sbp_ctx *ctx, sbp_state *state, const sbp_balls *sites, const float *out,
                         int64_t M, float a_init, float p0_scale, int64_t *count, void *stream);

/* The proposals of every frame of a multi-frame state, merged into a new
 * state.  The candidate sites of all frames are back to back: frame f owns
 * sites [site_off[f], site_off[f+1]) (site_off: device, F+1 int64, ascending,
 * site_off[F] = M_total), with network outputs out[m][0..1].  Site m of frame
 * f is accepted when out[m][0] > 0 and p0_scale[f] > 0 (p0_scale: device, F
 * floats; 0 leaves frame f as it is).  out_state receives, frame by frame, the
 * balls of `in` in order with their gradients and moments (zeros where `in`
 * has no such array; arrays of out_state that are NULL are skipped), then the
 * frame's accepted sites in site order with x, y, z = the site, p0 =
 * max(out[m][1], 0) * p0_scale[f], a = a_init and zero gradients and moments;
 * out_state->ball_off gets the new offsets and *count (host) the new total
 * (the call synchronises `stream`).  `in` and out_state must not share
 * arrays.  An `in` with no balls (B_cap = 0, offsets all zero) gives the
 * proposals alone.
 * Errors: SBP_E_ARG (NULL, M_total < 0, F outside [1, SBP_MAX_FRAMES] or
 * different in the two states), SBP_E_DOMAIN (a_init <= 0), SBP_E_CAPACITY
 * (more than out_state->B_cap balls; out_state unchanged). */
int sbp_merge_proposals(sbp_ctx *ctx, const sbp_state *in, const sbp_balls *sites,
                        const int64_t *site_off, const float *out, int64_t M_total,
                        const float *p0_scale, float a_init, sbp_state *out_state, int64_t *count,
                        void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SBP_MLP_H */
