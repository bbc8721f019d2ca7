// Candidate sites and features of the growth-proposal network, and the
// insertion of accepted proposals (declared in include/sbp_mlp.h).
#include "../../include/sbp_mlp.h"
#include "sbp_internal.hpp"

namespace sbp {

constexpr int kPb = 256;

struct GridD {
    float ox, oy, oz, h;
    int nx, ny, nz;
};

static GridD gd(const sbp_grid *g) { return GridD{g->ox, g->oy, g->oz, g->h, g->nx, g->ny, g->nz}; }

__device__ inline bool cell_of(const GridD &g, float x, float y, float z, int &i, int &j, int &k) {
    i = (int)floorf((x - g.ox) / g.h);
    j = (int)floorf((y - g.oy) / g.h);
    k = (int)floorf((z - g.oz) / g.h);
    return i >= 0 && j >= 0 && k >= 0 && i < g.nx && j < g.ny && k < g.nz;
}

__device__ inline float mass_at(const GridD &g, const float *m, int i, int j, int k) {
    if (i < 0 || j < 0 || k < 0 || i >= g.nx || j >= g.ny || k >= g.nz) return 0.0f;
    return m[((int64_t)i * g.ny + j) * g.nz + k];
}

__global__ void k_grid_mass(BallsP<float> b, const int64_t *__restrict__ off, GridD g, float *mass) {
    const int64_t n = off[1];
    for (int64_t t = off[0] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        if (cell_of(g, b.x[t], b.y[t], b.z[t], i, j, k))
            atomicAdd(mass + ((int64_t)i * g.ny + j) * g.nz + k, b.p0[t]);
    }
}

__device__ inline bool is_candidate(const GridD &g, const float *m, int64_t c, float occ) {
    const int k = (int)(c % g.nz);
    const int j = (int)((c / g.nz) % g.ny);
    const int i = (int)(c / ((int64_t)g.ny * g.nz));
    if (m[c] >= occ) return false;
    for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj)
            for (int dk = -1; dk <= 1; ++dk)
                if ((di | dj | dk) && mass_at(g, m, i + di, j + dj, k + dk) >= occ) return true;
    return false;
}

// Generic stable compaction helpers over flags given by a functor.
template <typename Pred>
__global__ void k_flag_count(int64_t n, Pred pred, int *cnt) {
    const int64_t t = (int64_t)blockIdx.x * kPb + threadIdx.x;
    const int c = __syncthreads_count(t < n && pred(t));
    if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

__global__ void k_flag_scan(const int *__restrict__ cnt, int nblk, int64_t *__restrict__ pre) {
    __shared__ int64_t s_wave[16];
    __shared__ int64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int base = 0; base < nblk; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const int64_t x = i < nblk ? cnt[i] : 0;
        int64_t s = x;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t u = __shfl_up(s, o, 64);
            if (lane >= o) s += u;
        }
        if (lane == 63) s_wave[wid] = s;
        __syncthreads();
        int64_t wp = 0;
        for (int w = 0; w < wid; ++w) wp += s_wave[w];
        const int64_t carry = s_carry;
        if (i < nblk) pre[i] = carry + wp + s - x;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) s_carry = carry + wp + s;
        __syncthreads();
    }
    if (threadIdx.x == 0) pre[nblk] = s_carry;
}

// Rank of this thread's element among the flagged ones of the whole range
// (meaningful where f holds); every thread of the block must call it.
__device__ inline int64_t flag_rank(bool f, const int64_t *pre, int *s_wave) {
    const unsigned long long bal = __ballot(f);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int below = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[wid] = __popcll(bal);
    __syncthreads();
    int wp = 0;
    for (int w = 0; w < wid; ++w) wp += s_wave[w];
    return pre[blockIdx.x] + wp + below;
}

struct CandPred {
    GridD g;
    const float *m;
    float occ;
    __device__ bool operator()(int64_t c) const { return is_candidate(g, m, c, occ); }
};

__global__ void k_cand_scatter(int64_t n, CandPred p, const int64_t *__restrict__ pre,
                               float a_probe, BallsP<float> out) {
    __shared__ int s_wave[kPb / 64];
    const int64_t c = (int64_t)blockIdx.x * kPb + threadIdx.x;
    const bool f = c < n && p(c);
    const int64_t r = flag_rank(f, pre, s_wave);
    if (f) {
        const int k = (int)(c % p.g.nz);
        const int j = (int)((c / p.g.nz) % p.g.ny);
        const int i = (int)(c / ((int64_t)p.g.ny * p.g.nz));
        out.x[r] = p.g.ox + (i + 0.5f) * p.g.h;
        out.y[r] = p.g.oy + (j + 0.5f) * p.g.h;
        out.z[r] = p.g.oz + (k + 0.5f) * p.g.h;
        out.p0[r] = 1.0f;
        out.a[r] = a_probe;
    }
}

// maxima of |g_p0|, |g_r| and the cell mass, as float bits (non-negative)
__global__ void k_feature_scales(GridD g, const float *__restrict__ mass, int64_t ncell,
                                 const float *__restrict__ gp, const float *__restrict__ gx,
                                 const float *__restrict__ gy, const float *__restrict__ gz, int64_t M,
                                 unsigned *scales) {
    float a = 0.0f, b = 0.0f, c = 0.0f;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < M;
         t += (int64_t)gridDim.x * blockDim.x) {
        a = fmaxf(a, fabsf(gp[t]));
        b = fmaxf(b, sqrtf(gx[t] * gx[t] + gy[t] * gy[t] + gz[t] * gz[t]));
    }
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
         t += (int64_t)gridDim.x * blockDim.x)
        c = fmaxf(c, fabsf(mass[t]));
    for (int o = 32; o > 0; o >>= 1) {
        a = fmaxf(a, __shfl_down(a, o, 64));
        b = fmaxf(b, __shfl_down(b, o, 64));
        c = fmaxf(c, __shfl_down(c, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(scales + 0, __float_as_uint(a));
        atomicMax(scales + 1, __float_as_uint(b));
        atomicMax(scales + 2, __float_as_uint(c));
    }
}

__global__ void k_features(GridD g, const float *__restrict__ mass, BallsP<float> site, int64_t M,
                           const float *__restrict__ gp, const float *__restrict__ gx,
                           const float *__restrict__ gy, const float *__restrict__ gz, float half,
                           const unsigned *__restrict__ scales, float *__restrict__ X) {
    const float sa = __uint_as_float(scales[0]), sb = __uint_as_float(scales[1]),
                sc = __uint_as_float(scales[2]);
    const float ia = sa > 0.0f ? 1.0f / sa : 0.0f, ib = sb > 0.0f ? 1.0f / sb : 0.0f,
                ic = sc > 0.0f ? 1.0f / sc : 0.0f;
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M;
         m += (int64_t)gridDim.x * blockDim.x) {
        float *row = X + m * SBP_MLP_IN;
        const float x = site.x[m], y = site.y[m], z = site.z[m];
        row[0] = -gp[m] * ia;
        row[1] = sqrtf(gx[m] * gx[m] + gy[m] * gy[m] + gz[m] * gz[m]) * ib;
        int i, j, k;
        const bool in = cell_of(g, x, y, z, i, j, k);
        int q = 2;
        for (int di = -1; di <= 1; ++di)
            for (int dj = -1; dj <= 1; ++dj)
                for (int dk = -1; dk <= 1; ++dk) {
                    if (!(di | dj | dk)) continue;
                    row[q++] = in ? mass_at(g, mass, i + di, j + dj, k + dk) * ic : 0.0f;
                }
        row[28] = x / half;
        row[29] = y / half;
        row[30] = z / half;
    }
}

struct AcceptPred {
    const float *out;
    __device__ bool operator()(int64_t m) const { return out[2 * m] > 0.0f; }
};

__global__ void k_append(int64_t M, AcceptPred p, const int64_t *__restrict__ pre,
                         BallsP<float> site, float a_init, float p0_scale, sbp_state s) {
    __shared__ int s_wave[kPb / 64];
    const int64_t m = (int64_t)blockIdx.x * kPb + threadIdx.x;
    const bool f = m < M && p(m);
    const int64_t r = flag_rank(f, pre, s_wave);
    if (f) {
        const int64_t o = s.ball_off[1] + r;
        s.balls.x[o] = site.x[m];
        s.balls.y[o] = site.y[m];
        s.balls.z[o] = site.z[m];
        s.balls.p0[o] = fmaxf(p.out[2 * m + 1], 0.0f) * p0_scale;
        s.balls.a[o] = a_init;
        if (s.grad.x) s.grad.x[o] = 0.0f;
        if (s.grad.y) s.grad.y[o] = 0.0f;
        if (s.grad.z) s.grad.z[o] = 0.0f;
        if (s.grad.p0) s.grad.p0[o] = 0.0f;
        if (s.grad.a) s.grad.a[o] = 0.0f;
        if (s.m.x) s.m.x[o] = 0.0f;
        if (s.m.y) s.m.y[o] = 0.0f;
        if (s.m.z) s.m.z[o] = 0.0f;
        if (s.m.p0) s.m.p0[o] = 0.0f;
        if (s.m.a) s.m.a[o] = 0.0f;
        if (s.v.x) s.v.x[o] = 0.0f;
        if (s.v.y) s.v.y[o] = 0.0f;
        if (s.v.z) s.v.z[o] = 0.0f;
        if (s.v.p0) s.v.p0[o] = 0.0f;
        if (s.v.a) s.v.a[o] = 0.0f;
    }
}

__global__ void k_bump_count(int64_t *off, const int64_t *__restrict__ pre, int nblk) {
    if (threadIdx.x == 0 && blockIdx.x == 0) off[1] += pre[nblk];
}

// ------------------------------------------------ merge into a new state --
struct MergePred {
    const float *out;
    const int64_t *site_off;
    const float *scale;
    int F;
    __device__ bool operator()(int64_t m) const {
        return out[2 * m] > 0.0f && scale[frame_of(site_off, F, m)] > 0.0f;
    }
};

// Rank of the flagged sites below index t: the block's prefix plus the flags
// of its earlier elements (t may equal n: the total).
__device__ inline int64_t rank_below(const MergePred &p, int64_t n, const int64_t *pre, int64_t t) {
    const int64_t blk = t / kPb;
    int64_t r = pre[blk];
    for (int64_t u = blk * kPb; u < t && u < n; ++u) r += p(u) ? 1 : 0;
    return r;
}

// One workgroup: per frame the rank of its first site (racc[f]) and the new
// offsets off_out[f] = sum over g < f of (balls of g + accepted sites of g).
__global__ void k_merge_offsets(MergePred p, int64_t n, const int64_t *__restrict__ pre,
                                const int64_t *__restrict__ off_in, int64_t *__restrict__ racc,
                                int64_t *__restrict__ off_out) {
    const int F = p.F;
    for (int f = threadIdx.x; f <= F; f += blockDim.x) racc[f] = rank_below(p, n, pre, p.site_off[f]);
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t o = 0;
        off_out[0] = 0;
        for (int f = 0; f < F; ++f) {
            o += (off_in[f + 1] - off_in[f]) + (racc[f + 1] - racc[f]);
            off_out[f + 1] = o;
        }
    }
}

__device__ inline void copy_or_zero(float *dst, const float *src, int64_t o, int64_t i) {
    if (dst) dst[o] = src ? src[i] : 0.0f;
}

// The existing balls, frame by frame, to their new places (with gradients and
// moments where both sides have them).
__global__ void k_merge_balls(sbp_state in, const int64_t *__restrict__ off_out, sbp_state out) {
    __shared__ int64_t s_in[SBP_MAX_FRAMES + 1], s_out[SBP_MAX_FRAMES + 1];
    const int F = in.F;
    for (int f = threadIdx.x; f <= F; f += blockDim.x) {
        s_in[f] = in.ball_off[f];
        s_out[f] = off_out[f];
    }
    __syncthreads();
    for (int64_t i = s_in[0] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s_in[F];
         i += (int64_t)gridDim.x * blockDim.x) {
        const int f = frame_of(s_in, F, i);
        const int64_t o = s_out[f] + (i - s_in[f]);
        out.balls.x[o] = in.balls.x[i];
        out.balls.y[o] = in.balls.y[i];
        out.balls.z[o] = in.balls.z[i];
        out.balls.p0[o] = in.balls.p0[i];
        out.balls.a[o] = in.balls.a[i];
        copy_or_zero(out.grad.x, in.grad.x, o, i);
        copy_or_zero(out.grad.y, in.grad.y, o, i);
        copy_or_zero(out.grad.z, in.grad.z, o, i);
        copy_or_zero(out.grad.p0, in.grad.p0, o, i);
        copy_or_zero(out.grad.a, in.grad.a, o, i);
        copy_or_zero(out.m.x, in.m.x, o, i);
        copy_or_zero(out.m.y, in.m.y, o, i);
        copy_or_zero(out.m.z, in.m.z, o, i);
        copy_or_zero(out.m.p0, in.m.p0, o, i);
        copy_or_zero(out.m.a, in.m.a, o, i);
        copy_or_zero(out.v.x, in.v.x, o, i);
        copy_or_zero(out.v.y, in.v.y, o, i);
        copy_or_zero(out.v.z, in.v.z, o, i);
        copy_or_zero(out.v.p0, in.v.p0, o, i);
        copy_or_zero(out.v.a, in.v.a, o, i);
    }
}

// The accepted sites after their frame's balls, in site order.
__global__ void k_merge_sites(int64_t n, MergePred p, const int64_t *__restrict__ pre,
                              const int64_t *__restrict__ racc, const int64_t *__restrict__ off_in,
                              const int64_t *__restrict__ off_out, BallsP<float> site, float a_init,
                              sbp_state out) {
    __shared__ int s_wave[kPb / 64];
    const int64_t m = (int64_t)blockIdx.x * kPb + threadIdx.x;
    const bool fl = m < n && p(m);
    const int64_t r = flag_rank(fl, pre, s_wave);
    if (!fl) return;
    const int f = frame_of(p.site_off, p.F, m);
    const int64_t o = off_out[f] + (off_in[f + 1] - off_in[f]) + (r - racc[f]);
    out.balls.x[o] = site.x[m];
    out.balls.y[o] = site.y[m];
    out.balls.z[o] = site.z[m];
    out.balls.p0[o] = fmaxf(p.out[2 * m + 1], 0.0f) * p.scale[f];
    out.balls.a[o] = a_init;
    float *zero[15] = {out.grad.x, out.grad.y, out.grad.z, out.grad.p0, out.grad.a,
                       out.m.x,    out.m.y,    out.m.z,    out.m.p0,    out.m.a,
                       out.v.x,    out.v.y,    out.v.z,    out.v.p0,    out.v.a};
#pragma unroll
    for (int k = 0; k < 15; ++k)
        if (zero[k]) zero[k][o] = 0.0f;
}

}  // namespace sbp

using namespace sbp;

extern "C" {

int sbp_grid_mass(sbp_ctx *ctx, const sbp_balls *balls, const int64_t *ball_off, int64_t B_cap,
                  const sbp_grid *grid, float *mass, void *stream) {
    if (!balls || !ball_off || !grid || !mass) return fail(SBP_E_ARG, "a required pointer is NULL");
    if (B_cap < 0) return fail(SBP_E_ARG, "B_cap must be >= 0");
    if (B_cap > 0 && (!balls->x || !balls->y || !balls->z || !balls->p0)) return fail(SBP_E_ARG, "balls has a NULL array");
    if (!(grid->h > 0.0f) || grid->nx < 1 || grid->ny < 1 || grid->nz < 1)
        return fail(SBP_E_DOMAIN, "grid needs h > 0 and at least one cell");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    hipStream_t st = (hipStream_t)stream;
    const int64_t ncell = (int64_t)grid->nx * grid->ny * grid->nz;
    int rc = launch_fill<float>(mass, ncell, 0.0f, st);
    if (rc) return rc;
    if (B_cap == 0) return SBP_OK;
    int64_t nb = (B_cap + kPb - 1) / kPb;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_grid_mass, dim3((unsigned)nb), dim3(kPb), 0, st,
                       BallsP<float>{balls->x, balls->y, balls->z, balls->p0, balls->a}, ball_off, gd(grid), mass);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

static bool soa_ok(const sbp_balls *b, bool need_pa) {
    return b && b->x && b->y && b->z && (!need_pa || (b->p0 && b->a));
}

static bool grid_ok(const sbp_grid *g) {
    return g->h > 0.0f && g->nx >= 1 && g->ny >= 1 && g->nz >= 1;
}

int sbp_candidates(sbp_ctx *ctx, const sbp_grid *grid, const float *mass, float occ, float a_probe,
                   const sbp_balls *sites, int64_t cap, int64_t *count, void *stream) {
    if (!grid || !mass || !count || !sites) return fail(SBP_E_ARG, "a required pointer is NULL");
    if (cap < 0) return fail(SBP_E_ARG, "cap must be >= 0");
    if (cap > 0 && !soa_ok(sites, true)) return fail(SBP_E_ARG, "sites has a NULL array");
    if (!grid_ok(grid)) return fail(SBP_E_DOMAIN, "grid needs h > 0 and at least one cell");
    if (!(a_probe > 0.0f)) return fail(SBP_E_DOMAIN, "a_probe must be > 0");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
    const int64_t nblk64 = (n + kPb - 1) / kPb;
    if (nblk64 > INT32_MAX / 2) return fail(SBP_E_ARG, "grid too large");
    const int nblk = (int)nblk64;
    const size_t off_pre = ((size_t)(nblk + 1) * sizeof(int) + 255) & ~(size_t)255;
    int rc = ensure_scratch(&ctx->c, off_pre + (size_t)(nblk + 2) * sizeof(int64_t));
    if (rc) return rc;
    int *cnt = (int *)ctx->c.scratch;
    int64_t *pre = (int64_t *)((char *)ctx->c.scratch + off_pre);
    CandPred p{gd(grid), mass, occ};
    hipLaunchKernelGGL(k_flag_count<CandPred>, dim3(nblk), dim3(kPb), 0, st, n, p, cnt);
    hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, st, cnt, nblk, pre);
    SBP_HIP(hipGetLastError());
    int64_t total = 0;
    SBP_HIP(hipMemcpyAsync(&total, pre + nblk, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SBP_HIP(hipStreamSynchronize(st));
    *count = total;
    if (total > cap) return fail(SBP_E_CAPACITY, "%lld candidates, capacity %lld", (long long)total, (long long)cap);
    if (total > 0) {
        hipLaunchKernelGGL(k_cand_scatter, dim3(nblk), dim3(kPb), 0, st, n, p, pre, a_probe,
                           BallsP<float>{sites->x, sites->y, sites->z, sites->p0, sites->a});
        SBP_HIP(hipGetLastError());
    }
    return SBP_OK;
}

int sbp_features(sbp_ctx *ctx, const sbp_grid *grid, const float *mass, const sbp_balls *sites, int64_t M,
                 const sbp_balls *g, float half, float *X, void *stream) {
    if (M < 0) return fail(SBP_E_ARG, "M must be >= 0");
    if (!grid || !mass || !sites || !g || (M > 0 && !X)) return fail(SBP_E_ARG, "a required pointer is NULL");
    if (M > 0 && (!soa_ok(sites, false) || !soa_ok(g, false) || !g->p0))
        return fail(SBP_E_ARG, "sites or g has a NULL array");
    if (!(half > 0.0f) || !grid_ok(grid)) return fail(SBP_E_DOMAIN, "half and h must be > 0, grid non-empty");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    if (M == 0) return SBP_OK;
    hipStream_t st = (hipStream_t)stream;
    unsigned *scales = ctx->c.misc + kMiscScales;
    int rc = launch_fill<int32_t>((int32_t *)scales, 3, 0, st);
    if (rc) return rc;
    const int64_t ncell = (int64_t)grid->nx * grid->ny * grid->nz;
    hipLaunchKernelGGL(k_feature_scales, dim3(512), dim3(kPb), 0, st, gd(grid), mass, ncell, g->p0, g->x,
                       g->y, g->z, M, scales);
    int64_t nb = (M + kPb - 1) / kPb;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_features, dim3((unsigned)nb), dim3(kPb), 0, st, gd(grid), mass,
                       BallsP<float>{sites->x, sites->y, sites->z, nullptr, nullptr}, M, g->p0, g->x, g->y,
                       g->z, half, scales, X);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

int sbp_merge_proposals(sbp_ctx *ctx, const sbp_state *in, const sbp_balls *sites,
                        const int64_t *site_off, const float *out, int64_t M_total,
                        const float *p0_scale, float a_init, sbp_state *out_state, int64_t *count,
                        void *stream) {
    if (!in || !out_state || !count || !sites || !site_off || !p0_scale || (M_total > 0 && !out))
        return fail(SBP_E_ARG, "a required pointer is NULL");
    if (M_total < 0) return fail(SBP_E_ARG, "M_total must be >= 0");
    if (in->F < 1 || in->F > SBP_MAX_FRAMES || out_state->F != in->F)
        return fail(SBP_E_ARG, "F must be in [1, %d] and equal in both states", SBP_MAX_FRAMES);
    if (!in->ball_off || !out_state->ball_off) return fail(SBP_E_ARG, "ball_off is NULL");
    if (in->B_cap < 0 || out_state->B_cap < 0) return fail(SBP_E_ARG, "B_cap must be >= 0");
    if (in->B_cap > 0 && !soa_ok(&in->balls, true)) return fail(SBP_E_ARG, "in.balls has a NULL array");
    if (out_state->B_cap > 0 && !soa_ok(&out_state->balls, true))
        return fail(SBP_E_ARG, "out_state.balls has a NULL array");
    if (M_total > 0 && !soa_ok(sites, false)) return fail(SBP_E_ARG, "sites has a NULL array");
    if (!(a_init > 0.0f)) return fail(SBP_E_DOMAIN, "a_init must be > 0");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    hipStream_t st = (hipStream_t)stream;
    const int F = in->F;
    const int64_t nblk64 = (M_total + kPb - 1) / kPb;
    if (nblk64 > INT32_MAX / 2) return fail(SBP_E_ARG, "too many sites");
    const int nblk = (int)nblk64;
    // scratch: [block counts][block prefix][rank of each frame's first site][new offsets]
    const size_t off_pre = ((size_t)(nblk + 1) * sizeof(int) + 255) & ~(size_t)255;
    const size_t off_racc = off_pre + (((size_t)(nblk + 2) * sizeof(int64_t) + 255) & ~(size_t)255);
    const size_t off_new = off_racc + 1024;
    int rc = ensure_scratch(&ctx->c, off_new + 1024);
    if (rc) return rc;
    char *sc = (char *)ctx->c.scratch;
    int *cnt = (int *)sc;
    int64_t *pre = (int64_t *)(sc + off_pre);
    int64_t *racc = (int64_t *)(sc + off_racc);
    int64_t *noff = (int64_t *)(sc + off_new);
    MergePred p{out, site_off, p0_scale, F};
    if (nblk > 0) hipLaunchKernelGGL(k_flag_count<MergePred>, dim3(nblk), dim3(kPb), 0, st, M_total, p, cnt);
    hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, st, cnt, nblk, pre);
    hipLaunchKernelGGL(k_merge_offsets, dim3(1), dim3(64), 0, st, p, M_total, pre, in->ball_off, racc, noff);
    SBP_HIP(hipGetLastError());
    int64_t total = 0;
    SBP_HIP(hipMemcpyAsync(&total, noff + F, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SBP_HIP(hipStreamSynchronize(st));
    *count = total;
    if (total > out_state->B_cap)
        return fail(SBP_E_CAPACITY, "%lld balls after merging, capacity %lld", (long long)total,
                    (long long)out_state->B_cap);
    SBP_HIP(hipMemcpyAsync(out_state->ball_off, noff, (size_t)(F + 1) * sizeof(int64_t),
                           hipMemcpyDeviceToDevice, st));
    if (in->B_cap > 0) {
        int64_t nb = (in->B_cap + kPb - 1) / kPb;
        if (nb > 4096) nb = 4096;
        hipLaunchKernelGGL(k_merge_balls, dim3((unsigned)nb), dim3(kPb), 0, st, *in, noff, *out_state);
    }
    if (nblk > 0)
        hipLaunchKernelGGL(k_merge_sites, dim3(nblk), dim3(kPb), 0, st, M_total, p, pre, racc,
                           in->ball_off, noff,
                           BallsP<float>{sites->x, sites->y, sites->z, nullptr, nullptr}, a_init,
                           *out_state);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

int sbp_append_proposals(sbp_ctx *ctx, sbp_state *state, const sbp_balls *sites, const float *out,
                         int64_t M, float a_init, float p0_scale, int64_t *count, void *stream) {
    if (!state || !count || !sites || (M > 0 && !out)) return fail(SBP_E_ARG, "a required pointer is NULL");
    if (M < 0) return fail(SBP_E_ARG, "M must be >= 0");
    if (M > 0 && !soa_ok(sites, false)) return fail(SBP_E_ARG, "sites has a NULL array");
    if (state->F != 1 || !state->ball_off) return fail(SBP_E_ARG, "state must hold one frame");
    if (!soa_ok(&state->balls, true)) return fail(SBP_E_ARG, "state.balls has a NULL array");
    if (!(a_init > 0.0f)) return fail(SBP_E_DOMAIN, "a_init must be > 0");
    if (!(p0_scale >= 0.0f)) return fail(SBP_E_DOMAIN, "p0_scale must be >= 0");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    hipStream_t st = (hipStream_t)stream;
    const int nblk = (int)((M + kPb - 1) / kPb);
    const size_t off_pre = ((size_t)(nblk + 1) * sizeof(int) + 255) & ~(size_t)255;
    int rc = ensure_scratch(&ctx->c, off_pre + (size_t)(nblk + 2) * sizeof(int64_t));
    if (rc) return rc;
    int *cnt = (int *)ctx->c.scratch;
    int64_t *pre = (int64_t *)((char *)ctx->c.scratch + off_pre);
    AcceptPred p{out};
    if (nblk > 0) hipLaunchKernelGGL(k_flag_count<AcceptPred>, dim3(nblk), dim3(kPb), 0, st, M, p, cnt);
    hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, st, cnt, nblk, pre);
    SBP_HIP(hipGetLastError());
    int64_t host[2] = {0, 0};
    SBP_HIP(hipMemcpyAsync(&host[0], pre + nblk, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SBP_HIP(hipMemcpyAsync(&host[1], state->ball_off + 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SBP_HIP(hipStreamSynchronize(st));
    if (host[0] + host[1] > state->B_cap) {
        *count = host[1];
        return fail(SBP_E_CAPACITY, "%lld balls after appending, capacity %lld",
                    (long long)(host[0] + host[1]), (long long)state->B_cap);
    }
    *count = host[0] + host[1];
    if (host[0] > 0) {
        hipLaunchKernelGGL(k_append, dim3(nblk), dim3(kPb), 0, st, M, p, pre,
                           BallsP<float>{sites->x, sites->y, sites->z, nullptr, nullptr}, a_init, p0_scale,
                           *state);
        hipLaunchKernelGGL(k_bump_count, dim3(1), dim3(64), 0, st, state->ball_off, pre, nblk);
        SBP_HIP(hipGetLastError());
    }
    return SBP_OK;
}

}  // extern "C"
