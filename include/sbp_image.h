/*
 * sbp_image.h -- the last step of Algorithm 1 of SlingBAG Pro (arXiv
 * 2601.00551): the reconstructed point cloud is turned into a voxel grid
 * ("point cloud to voxel shader"), and the image-quality figures the paper
 * reports against a ground truth (MSE, PSNR, SSIM; Table 1) are computed on
 * the GPU.
 *
 * Conventions are those of sbp.h: device pointers owned by the caller,
 * host-side validation before anything is enqueued, asynchronous on `stream`.
 */
#ifndef SBP_IMAGE_H
#define SBP_IMAGE_H

#include <stdint.h>

#include "sbp.h"
#include "sbp_mlp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Voxelisation.  vox[(i * ny + j) * nz + k] (nx*ny*nz floats, overwritten) is
 * the initial pressure of the cloud at the voxel centre
 * c = origin + (i + 1/2, j + 1/2, k + 1/2) h, i.e. the sum over the balls of
 * frame 0 (balls [ball_off[0], ball_off[1])) of p0 * fhat(|c - r| / a) with the
 * ball profile of section 4.1: GAUSS fhat = exp(-d^2 / (2 a^2)) for d < K a,
 * UNIFORM fhat = 1 for d < a (profile, gauss_K and a_softplus come from
 * `model`; balls with a <= 0 add nothing).  FP32 atomic sums: the order of the
 * additions is unspecified.
 * Errors: SBP_E_ARG, SBP_E_DOMAIN (bad grid or model). */
int sbp_voxelize(sbp_ctx *ctx, const sbp_balls *balls, const int64_t *ball_off, int64_t B_cap,
                 const sbp_model *model, const sbp_grid *grid, float *vox, void *stream);

/* Image quality of `img` against the reference `ref` (both nx*ny*nz floats,
 * same layout as sbp_voxelize), after dividing both by `scale` (> 0; the
 * paper's figures are on volumes normalised to the ground truth's maximum):
 *   out[0] = MSE  = mean (img - ref)^2
 *   out[1] = PSNR = 10 log10(1 / MSE) (dB, data range 1)
 *   out[2] = SSIM = mean over the voxels whose whole window lies inside the
 *            volume of ((2 mx my + C1)(2 sxy + C2)) / ((mx^2 + my^2 + C1)(sx + sy + C2)),
 *            with m, s the Gaussian-weighted (sigma 1.5 voxels, 11 taps per
 *            axis, normalised) local means, variances and covariance,
 *            C1 = 0.01^2, C2 = 0.03^2 (Wang et al. 2004, in 3-D).
 * out is a DEVICE array of 3 doubles.  The volume must be at least 11 voxels
 * along each axis.  work holds 10 * nx*ny*nz floats (the separable blur's
 * intermediate fields).
 * Errors: SBP_E_ARG, SBP_E_DOMAIN (scale <= 0, volume too small). */
int sbp_image_metrics(sbp_ctx *ctx, const float *img, const float *ref, int32_t nx, int32_t ny,
                      int32_t nz, float scale, float *work, double *out, void *stream);

/* ------------------------------------------ initialisation inside the array */

/* Envelope test for the random initial cloud of Algorithm 1 (a closed
 * polygonal envelope mesh built from the array, points drawn inside it by ray
 * casting).  tri (device, F triangles x 9 floats: v0, v1, v2) is a closed,
 * consistently triangulated mesh.  For each point i < N (px, py, pz):
 *   inside[i] = 1 if the ray from the point along the fixed direction
 *     (1, 0.7071, 0.3183) crosses the mesh an odd number of times (Moller-
 *     Trumbore, FP32, hits at t > 0) and the point is at least `margin` from
 *     every triangle; else 0.
 *   dist[i] (if dist is not NULL) = the distance to the nearest triangle.
 * Errors: SBP_E_ARG, SBP_E_DOMAIN (F < 4, margin < 0). */
int sbp_mesh_inside(sbp_ctx *ctx, const float *tri, int32_t F, const float *px, const float *py,
                    const float *pz, int64_t N, float margin, uint8_t *inside, float *dist,
                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SBP_IMAGE_H */
