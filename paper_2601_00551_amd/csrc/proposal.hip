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
