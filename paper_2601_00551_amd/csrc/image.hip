// Point cloud to voxel grid, and image-quality figures on the GPU (declared in
// include/sbp_image.h).
#include <cmath>

#include "../../include/sbp_image.h"
#include "sbp_internal.hpp"

namespace sbp {

constexpr int kIb = 256;
constexpr int kTaps = 11;   // SSIM window: Gaussian, sigma 1.5, radius 5
constexpr int kRad = 5;

struct Taps {
    float w[kTaps];
};

// One thread per ball: adds p0 * fhat(d / a) to every voxel centre within the
// ball's support.
__global__ void k_voxelize(BallsP<float> b, const int64_t *__restrict__ off, int profile, float K,
                           int a_softplus, float ox, float oy, float oz, float h, int nx, int ny,
                           int nz, float *__restrict__ vox) {
    const int64_t lo = off[0], hi = off[1];
    for (int64_t t = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < hi;
         t += (int64_t)gridDim.x * blockDim.x) {
        float a = b.a[t];
        if (a_softplus) a = softplus_dev(a);
        if (!(a > 0.0f)) continue;
        const float p0 = b.p0[t];
        const float x = b.x[t], y = b.y[t], z = b.z[t];
        const float w = profile == GAUSS ? K * a : a;
        const float w2 = w * w;
        const float q = -0.5f / (a * a);
        // voxel centres (i + 1/2) h within [x - w, x + w]
        const int i0 = max(0, (int)ceilf((x - w - ox) / h - 0.5f));
        const int i1 = min(nx - 1, (int)floorf((x + w - ox) / h - 0.5f));
        const int j0 = max(0, (int)ceilf((y - w - oy) / h - 0.5f));
        const int j1 = min(ny - 1, (int)floorf((y + w - oy) / h - 0.5f));
        const int k0 = max(0, (int)ceilf((z - w - oz) / h - 0.5f));
        const int k1 = min(nz - 1, (int)floorf((z + w - oz) / h - 0.5f));
        for (int i = i0; i <= i1; ++i) {
            const float dx = ox + (i + 0.5f) * h - x;
            for (int j = j0; j <= j1; ++j) {
                const float dy = oy + (j + 0.5f) * h - y;
                const float dxy = dx * dx + dy * dy;
                if (dxy >= w2) continue;
                float *row = vox + ((int64_t)i * ny + j) * nz;
                for (int k = k0; k <= k1; ++k) {
                    const float dz = oz + (k + 0.5f) * h - z;
                    const float d2 = dxy + dz * dz;
                    if (d2 < w2) atomicAdd(row + k, profile == GAUSS ? p0 * expf(q * d2) : p0);
                }
            }
        }
    }
}

// MSE partial sums (FP64 per block).
__global__ void k_sqdiff(const float *__restrict__ img, const float *__restrict__ ref, int64_t n,
                         float inv, double *__restrict__ partial) {
    __shared__ double s_red[kIb / 64];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)(img[i] * inv) - (double)(ref[i] * inv);
        acc += d * d;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kIb / 64; ++w) s += s_red[w];
        partial[blockIdx.x] = s;
    }
}

// Blur along z ('valid'), forming the five fields x, y, x^2, y^2, xy on the fly.
// out: 5 fields of nx * ny * mz (mz = nz - 10).
__global__ void k_blur_z(const float *__restrict__ img, const float *__restrict__ ref, float inv,
                         int nx, int ny, int nz, Taps tp, float *__restrict__ out) {
    const int mz = nz - 2 * kRad;
    const int64_t n = (int64_t)nx * ny * mz;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(o % mz);
        const int64_t ij = o / mz;
        const int64_t base = ij * nz + k;
        float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < kTaps; ++t) {
            const float x = img[base + t] * inv, y = ref[base + t] * inv, w = tp.w[t];
            s[0] = fmaf(w, x, s[0]);
            s[1] = fmaf(w, y, s[1]);
            s[2] = fmaf(w, x * x, s[2]);
            s[3] = fmaf(w, y * y, s[3]);
            s[4] = fmaf(w, x * y, s[4]);
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) out[f * n + o] = s[f];
    }
}

// Blur along y ('valid'): in 5 x nx*ny*mz -> out 5 x nx*my*mz.
__global__ void k_blur_y(const float *__restrict__ in, int nx, int ny, int mz, Taps tp,
                         float *__restrict__ out) {
    const int my = ny - 2 * kRad;
    const int64_t nin = (int64_t)nx * ny * mz, n = (int64_t)nx * my * mz;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(o % mz);
        const int j = (int)((o / mz) % my);
        const int i = (int)(o / ((int64_t)mz * my));
        const int64_t base = ((int64_t)i * ny + j) * mz + k;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < kTaps; ++t) s = fmaf(tp.w[t], in[f * nin + base + (int64_t)t * mz], s);
            out[f * n + o] = s;
        }
    }
}

// Blur along x ('valid') and the SSIM map, summed per block (FP64).
__global__ void k_blur_x_ssim(const float *__restrict__ in, int nx, int my, int mz, Taps tp,
                              double *__restrict__ partial) {
    __shared__ double s_red[kIb / 64];
    const int mx = nx - 2 * kRad;
    const int64_t nin = (int64_t)nx * my * mz, n = (int64_t)mx * my * mz;
    const int64_t plane = (int64_t)my * mz;
    const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
    double acc = 0.0;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int64_t jk = o % plane;
        const int i = (int)(o / plane);
        const int64_t base = (int64_t)i * plane + jk;
        float s[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            float v = 0.f;
#pragma unroll
            for (int t = 0; t < kTaps; ++t) v = fmaf(tp.w[t], in[f * nin + base + (int64_t)t * plane], v);
            s[f] = v;
        }
        const float mx_ = s[0], my_ = s[1];
        const float vx = s[2] - mx_ * mx_, vy = s[3] - my_ * my_, cxy = s[4] - mx_ * my_;
        const float num = (2.f * mx_ * my_ + C1) * (2.f * cxy + C2);
        const float den = (mx_ * mx_ + my_ * my_ + C1) * (vx + vy + C2);
        acc += (double)(num / den);
    }
    for (int o2 = 32; o2 > 0; o2 >>= 1) acc += __shfl_down(acc, o2, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kIb / 64; ++w) t += s_red[w];
        partial[blockIdx.x] = t;
    }
}

__global__ void k_metrics_final(const double *__restrict__ p_mse, int nb_mse, int64_t n,
                                const double *__restrict__ p_ssim, int nb_ssim, int64_t nvalid,
                                double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < nb_mse; ++i) a += p_mse[i];
        for (int i = 0; i < nb_ssim; ++i) b += p_ssim[i];
        const double mse = a / (double)n;
        out[0] = mse;
        out[1] = 10.0 * log10(1.0 / mse);
        out[2] = b / (double)nvalid;
    }
}

static int nblocks(int64_t n, int cap) {
    int64_t b = (n + kIb - 1) / kIb;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace sbp

using namespace sbp;

extern "C" {

int sbp_voxelize(sbp_ctx *ctx, const sbp_balls *balls, const int64_t *ball_off, int64_t B_cap,
                 const sbp_model *model, const sbp_grid *grid, float *vox, void *stream) {
    if (!balls || !ball_off || !model || !grid || !vox) return fail(SBP_E_ARG, "a required pointer is NULL");
    if (B_cap < 0) return fail(SBP_E_ARG, "B_cap must be >= 0");
    if (B_cap > 0 && (!balls->x || !balls->y || !balls->z || !balls->p0 || !balls->a))
        return fail(SBP_E_ARG, "balls has a NULL array");
    if (!(grid->h > 0.0f) || grid->nx < 1 || grid->ny < 1 || grid->nz < 1)
        return fail(SBP_E_DOMAIN, "grid needs h > 0 and at least one cell");
    if (model->profile != SBP_PROFILE_GAUSS && model->profile != SBP_PROFILE_UNIFORM)
        return fail(SBP_E_DOMAIN, "unknown profile");
    if (model->profile == SBP_PROFILE_GAUSS && !(model->gauss_K > 0.0)) return fail(SBP_E_DOMAIN, "gauss_K must be > 0");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nv = (int64_t)grid->nx * grid->ny * grid->nz;
    int rc = launch_fill<float>(vox, nv, 0.0f, st);
    if (rc) return rc;
    if (B_cap == 0) return SBP_OK;
    hipLaunchKernelGGL(k_voxelize, dim3(nblocks(B_cap, 8192)), dim3(kIb), 0, st,
                       BallsP<float>{balls->x, balls->y, balls->z, balls->p0, balls->a}, ball_off,
                       model->profile, (float)model->gauss_K, model->a_softplus, grid->ox, grid->oy,
                       grid->oz, grid->h, grid->nx, grid->ny, grid->nz, vox);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

int sbp_image_metrics(sbp_ctx *ctx, const float *img, const float *ref, int32_t nx, int32_t ny,
                      int32_t nz, float scale, float *work, double *out, void *stream) {
    if (!img || !ref || !work || !out) return fail(SBP_E_ARG, "a required pointer is NULL");
    if (!(scale > 0.0f)) return fail(SBP_E_DOMAIN, "scale must be > 0");
    if (nx < kTaps || ny < kTaps || nz < kTaps) return fail(SBP_E_DOMAIN, "volume must be >= 11 voxels per axis");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    hipStream_t st = (hipStream_t)stream;
    Taps tp;
    double wsum = 0.0, wd[kTaps];
    for (int t = 0; t < kTaps; ++t) {
        const double d = t - kRad;
        wd[t] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        wsum += wd[t];
    }
    for (int t = 0; t < kTaps; ++t) tp.w[t] = (float)(wd[t] / wsum);
    const int64_t n = (int64_t)nx * ny * nz;
    const int mx = nx - 2 * kRad, my = ny - 2 * kRad, mz = nz - 2 * kRad;
    const int64_t nvalid = (int64_t)mx * my * mz;
    const int nb_mse = nblocks(n, 1024), nb_ssim = nblocks(nvalid, 1024);
    int rc = ensure_scratch(&ctx->c, (size_t)(nb_mse + nb_ssim) * sizeof(double));
    if (rc) return rc;
    double *p_mse = (double *)ctx->c.scratch, *p_ssim = p_mse + nb_mse;
    const float inv = 1.0f / scale;
    float *A = work, *B = work + 5 * n;
    hipLaunchKernelGGL(k_sqdiff, dim3(nb_mse), dim3(kIb), 0, st, img, ref, n, inv, p_mse);
    hipLaunchKernelGGL(k_blur_z, dim3(nblocks((int64_t)nx * ny * mz, 8192)), dim3(kIb), 0, st, img, ref, inv,
                       nx, ny, nz, tp, A);
    hipLaunchKernelGGL(k_blur_y, dim3(nblocks((int64_t)nx * my * mz, 8192)), dim3(kIb), 0, st, (const float *)A,
                       nx, ny, mz, tp, B);
    hipLaunchKernelGGL(k_blur_x_ssim, dim3(nb_ssim), dim3(kIb), 0, st, (const float *)B, nx, my, mz, tp, p_ssim);
    hipLaunchKernelGGL(k_metrics_final, dim3(1), dim3(64), 0, st, (const double *)p_mse, nb_mse, n,
                       (const double *)p_ssim, nb_ssim, nvalid, out);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

}  // extern "C"

namespace sbp {

constexpr int kTriTile = 256;

// Distance from p to triangle (a, b, c): the closest point by the region
// tests of the triangle's Voronoi regions (vertex, edge, face).
__device__ inline float tri_dist2(float3 p, float3 a, float3 b, float3 c) {
    auto sub = [](float3 u, float3 v) { return make_float3(u.x - v.x, u.y - v.y, u.z - v.z); };
    auto dot = [](float3 u, float3 v) { return u.x * v.x + u.y * v.y + u.z * v.z; };
    auto d2 = [&](float3 u) { return dot(u, u); };
    const float3 ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
    const float d1 = dot(ab, ap), d2_ = dot(ac, ap);
    if (d1 <= 0.f && d2_ <= 0.f) return d2(ap);
    const float3 bp = sub(p, b);
    const float d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0.f && d4 <= d3) return d2(bp);
    const float vc = d1 * d4 - d3 * d2_;
    if (vc <= 0.f && d1 >= 0.f && d3 <= 0.f) {
        const float v = d1 / (d1 - d3);
        return d2(make_float3(ap.x - v * ab.x, ap.y - v * ab.y, ap.z - v * ab.z));
    }
    const float3 cp = sub(p, c);
    const float d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0.f && d5 <= d6) return d2(cp);
    const float vb = d5 * d2_ - d1 * d6;
    if (vb <= 0.f && d2_ >= 0.f && d6 <= 0.f) {
        const float w = d2_ / (d2_ - d6);
        return d2(make_float3(ap.x - w * ac.x, ap.y - w * ac.y, ap.z - w * ac.z));
    }
    const float va = d3 * d6 - d5 * d4;
    if (va <= 0.f && (d4 - d3) >= 0.f && (d5 - d6) >= 0.f) {
        const float w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        const float3 bc = sub(c, b);
        return d2(make_float3(bp.x - w * bc.x, bp.y - w * bc.y, bp.z - w * bc.z));
    }
    const float den = 1.f / (va + vb + vc);
    const float v = vb * den, w = vc * den;
    return d2(make_float3(ap.x - ab.x * v - ac.x * w, ap.y - ab.y * v - ac.y * w, ap.z - ab.z * v - ac.z * w));
}

// One thread per point; the block stages the triangles through LDS.
__global__ void k_mesh_inside(const float *__restrict__ tri, int F, const float *__restrict__ px,
                              const float *__restrict__ py, const float *__restrict__ pz, int64_t N,
                              float margin, int want_dist, uint8_t *__restrict__ inside,
                              float *__restrict__ dist) {
    __shared__ float s_tri[kTriTile * 9];
    const float dx = 1.0f, dy = 0.7071f, dz = 0.3183f;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < N; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const bool act = i < N;
        const float3 p = act ? make_float3(px[i], py[i], pz[i]) : make_float3(0.f, 0.f, 0.f);
        int hits = 0;
        float best = 3.0e38f;
        for (int t0 = 0; t0 < F; t0 += kTriTile) {
            const int nt = min(kTriTile, F - t0);
            __syncthreads();
            for (int q = threadIdx.x; q < nt * 9; q += blockDim.x) s_tri[q] = tri[(int64_t)t0 * 9 + q];
            __syncthreads();
            if (!act) continue;
            for (int t = 0; t < nt; ++t) {
                const float *v = s_tri + t * 9;
                const float3 a = make_float3(v[0], v[1], v[2]), b = make_float3(v[3], v[4], v[5]),
                             c = make_float3(v[6], v[7], v[8]);
                // Moller-Trumbore
                const float e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
                const float e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
                const float hx = dy * e2z - dz * e2y, hy = dz * e2x - dx * e2z, hz = dx * e2y - dy * e2x;
                const float det = e1x * hx + e1y * hy + e1z * hz;
                if (det != 0.0f) {
                    const float f = 1.0f / det;
                    const float sx = p.x - a.x, sy = p.y - a.y, sz = p.z - a.z;
                    const float u = f * (sx * hx + sy * hy + sz * hz);
                    if (u >= 0.0f && u <= 1.0f) {
                        const float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
                        const float w = f * (dx * qx + dy * qy + dz * qz);
                        if (w >= 0.0f && u + w <= 1.0f) {
                            const float tt = f * (e2x * qx + e2y * qy + e2z * qz);
                            if (tt > 0.0f) ++hits;
                        }
                    }
                }
                if (margin > 0.0f || want_dist) best = fminf(best, tri_dist2(p, a, b, c));
            }
        }
        if (act) {
            const float d = sqrtf(best);
            inside[i] = (uint8_t)((hits & 1) && (!(margin > 0.0f) || d >= margin));
            if (dist) dist[i] = d;
        }
    }
}

}  // namespace sbp

extern "C" int sbp_mesh_inside(sbp_ctx *ctx, const float *tri, int32_t F, const float *px, const float *py,
                               const float *pz, int64_t N, float margin, uint8_t *inside, float *dist,
                               void *stream) {
    using namespace sbp;
    if (!tri || (N > 0 && (!px || !py || !pz || !inside))) return fail(SBP_E_ARG, "a required pointer is NULL");
    if (N < 0) return fail(SBP_E_ARG, "N must be >= 0");
    if (F < 4) return fail(SBP_E_DOMAIN, "a closed mesh has at least 4 triangles");
    if (!(margin >= 0.0f)) return fail(SBP_E_DOMAIN, "margin must be >= 0");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    if (N == 0) return SBP_OK;
    hipLaunchKernelGGL(k_mesh_inside, dim3(nblocks(N, 4096)), dim3(kIb), 0, (hipStream_t)stream, tri, F, px, py,
                       pz, N, margin, dist ? 1 : 0, inside, dist);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}
