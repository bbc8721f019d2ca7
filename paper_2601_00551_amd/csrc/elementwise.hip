// Bandwidth-bound steps of the iteration on gfx950: fill, Downsample_f
// (section 4.3), residual + loss (section 4.2 / 4.3), Adam, and the stable
// stream compaction behind zero-gradient filtering (section 4.2).
#include "sbp_internal.hpp"

namespace sbp {

constexpr int kEw = 256;  // threads per workgroup of the elementwise kernels

template <typename R>
__global__ void k_fill(R *__restrict__ p, int64_t n, R value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

static int ew_grid(int64_t n) {
    int64_t g = (n + kEw - 1) / kEw;
    if (g > 65536) g = 65536;
    return g < 1 ? 1 : (int)g;
}

template <typename R>
int launch_fill(R *p, int64_t n, R value, hipStream_t st) {
    if (n <= 0) return SBP_OK;
    hipLaunchKernelGGL(k_fill<R>, dim3(ew_grid(n)), dim3(kEw), 0, st, p, n, value);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}
template int launch_fill<float>(float *, int64_t, float, hipStream_t);
template int launch_fill<double>(double *, int64_t, double, hipStream_t);
template int launch_fill<int32_t>(int32_t *, int64_t, int32_t, hipStream_t);
template int launch_fill<int64_t>(int64_t *, int64_t, int64_t, hipStream_t);
template int launch_fill<uint64_t>(uint64_t *, int64_t, uint64_t, hipStream_t);

// ------------------------------------------------------------ downsample --

__global__ void k_downsample(const float *__restrict__ y, int64_t R_, int T, int f, int Tk,
                             float *__restrict__ out) {
    const int64_t n_out = R_ * (int64_t)Tk;
    const float inv = 1.0f / (float)f;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n_out;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = o / Tk;
        const int n = (int)(o - r * Tk);
        const float *src = y + r * (int64_t)T + (int64_t)n * f;
        float s = 0.0f;
        for (int j = 0; j < f; ++j) s += src[j];
        out[o] = (f & (f - 1)) == 0 ? s * inv : s / (float)f;
    }
}

int launch_downsample(const float *y, int64_t R_, int T, int f, float *out, hipStream_t st) {
    const int Tk = T / f;
    hipLaunchKernelGGL(k_downsample, dim3(ew_grid(R_ * (int64_t)Tk)), dim3(kEw), 0, st, y, R_, T,
                       f, Tk, out);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

// Decimation, the pyramid of point-sampled records: out[r][n] = y[r][n f].
__global__ void k_decimate(const float *__restrict__ y, int64_t R_, int T, int f, int Tk,
                           float *__restrict__ out) {
    const int64_t n_out = R_ * (int64_t)Tk;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n_out;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = o / Tk;
        const int n = (int)(o - r * Tk);
        out[o] = y[r * (int64_t)T + (int64_t)n * f];
    }
}

int launch_decimate(const float *y, int64_t R_, int T, int f, float *out, hipStream_t st) {
    const int Tk = T / f;
    hipLaunchKernelGGL(k_decimate, dim3(ew_grid(R_ * (int64_t)Tk)), dim3(kEw), 0, st, y, R_, T, f, Tk,
                       out);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

// ------------------------------------------------------- residual + loss --


__global__ void k_residual(const float *__restrict__ ys, const float *__restrict__ yr, int64_t n,
                           float *v, double *__restrict__ partial) {
    __shared__ double s_part[kEw / 64];
    const int f = blockIdx.y;
    const float *a = ys + (int64_t)f * n;
    const float *b = yr + (int64_t)f * n;
    float *vo = v ? v + (int64_t)f * n : nullptr;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float e = a[i] - b[i];
        if (vo) vo[i] = 2.0f * e;
        acc += (double)e * (double)e;
    }
    const double t = block_sum(acc, s_part);
    if (threadIdx.x == 0) partial[(int64_t)f * gridDim.x + blockIdx.x] = t;
}

__global__ void k_loss_final(const double *__restrict__ partial, int nblk, double *__restrict__ loss) {
    __shared__ double s_part[kEw / 64];
    const int f = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partial[(int64_t)f * nblk + i];
    const double t = block_sum(acc, s_part);
    if (threadIdx.x == 0) loss[f] = t;
}

size_t residual_ws_bytes(int F) { return (size_t)F * kLossBlocks * sizeof(double); }

int launch_residual_loss(double *partial, const float *ys, const float *yr, int64_t n, int F,
                         float *v, double *loss, hipStream_t st) {
    hipLaunchKernelGGL(k_residual, dim3(kLossBlocks, F), dim3(kEw), 0, st, ys, yr, n, v, partial);
    SBP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_loss_final, dim3(F), dim3(kEw), 0, st, partial, kLossBlocks, loss);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

// ------------------------------------------------------------------- Adam --

struct AdamArgs {
    float *param[5];
    float *grad[5];
    float *m[5];
    float *v[5];
    float lr[5];
    float beta1, beta2, eps;
    int32_t step;
    uint32_t mask;
    // fused work of a reconstruction step (AdamFuse)
    const float *part;
    int nsl;
    int64_t pstride;
    int a_softplus;
    const double *loss_partial;
    double *loss;
    unsigned *misc_clear;
    int step_add;
    int n_adam;   // workgroups of the update; the F after them reduce the loss
    // with the cotangent formed in the adjoint (AdamFuse): the row sums, and
    // frames without balls handled here; the edge sums zeroed
    const double *row_loss;
    int D, T;
    const float *y_ref;
    float *y_work;
    unsigned long long *gacc;
    int64_t n_gacc;
};

// PyTorch's single-tensor Adam in FP32: m.lerp_(g, 1-b1); v = v*b2 + (1-b2) g g;
// denom = sqrt(v) / sqrt(bc2) + eps; param += (-lr/bc1) * m / denom, where the
// bias corrections are formed in FP64 and rounded once.  blockIdx.y is the
// parameter.  Inside a step the same kernel first adds the adjoint's
// transducer slices into the gradient (same order and chain factor as
// k_adj_reduce, so the same bits), and its last F workgroups of parameter 0
// reduce the loss partial sums (as k_loss_final).
__global__ void k_adam(AdamArgs a, const int64_t *__restrict__ ball_off, int F,
                       const int32_t *__restrict__ step_dev) {
    __shared__ double s_part[kEw / 64];
    const int k = (int)blockIdx.y;
    if ((int)blockIdx.x >= a.n_adam) {
        if (k != 0) return;
        const int f = (int)blockIdx.x - a.n_adam;
        double acc = 0.0;
        if (a.row_loss) {
            if (ball_off[f + 1] > ball_off[f]) {
                for (int i = threadIdx.x; i < a.D; i += blockDim.x)
                    acc += a.row_loss[(int64_t)f * a.D + i];
            } else {
                // no balls, so no adjoint items: y = 0 and v = -2 y_ref here
                const int64_t n = (int64_t)a.D * a.T;
                const float *rr = a.y_ref + (int64_t)f * n;
                float *yw = a.y_work + (int64_t)f * n;
                for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
                    const float e = 0.0f - rr[i];
                    yw[i] = 2.0f * e;
                    acc += (double)e * (double)e;
                }
            }
        } else {
            for (int i = threadIdx.x; i < kLossBlocks; i += blockDim.x)
                acc += a.loss_partial[(int64_t)f * kLossBlocks + i];
        }
        const double t = block_sum(acc, s_part);
        if (threadIdx.x == 0) a.loss[f] = t;
        return;
    }
    if (a.gacc) {   // the forward's edge sums, zero again for the next forward
        const int64_t stride = (int64_t)a.n_adam * 5 * blockDim.x;
        for (int64_t i = ((int64_t)k * a.n_adam + blockIdx.x) * blockDim.x + threadIdx.x;
             i < a.n_gacc; i += stride)
            a.gacc[i] = 0ull;
    }
    if (a.misc_clear && blockIdx.x == 0 && k == 0)
        for (int i = threadIdx.x; i < kMiscFlags + SBP_MAX_FRAMES; i += blockDim.x) a.misc_clear[i] = 0u;
    if (!(a.mask & (1u << k))) return;
    // the bias corrections once per workgroup (FP64 pow is costly per lane)
    __shared__ float s_bc[2];
    if (threadIdx.x == 0) {
        const int step = step_dev ? *step_dev + a.step_add : a.step;
        const double bc1 = 1.0 - step_power((double)a.beta1, step);
        const double bc2 = 1.0 - step_power((double)a.beta2, step);
        s_bc[0] = (float)sqrt(bc2);
        s_bc[1] = (float)(-(double)a.lr[k] / bc1);
    }
    __syncthreads();
    const int64_t count = ball_off[F];
    const float bc2_sqrt = s_bc[0];
    const float step_size = s_bc[1];
    const float w1 = 1.0f - a.beta1;
    const float w2 = 1.0f - a.beta2;
    float *param = a.param[k], *grad = a.grad[k], *mk = a.m[k], *vk = a.v[k];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)a.n_adam * blockDim.x) {
        float g;
        if (a.part) {
            g = slice_sum(a.part + (int64_t)k * a.pstride + i, a.nsl, 5 * a.pstride);
            if (k == 4 && a.a_softplus) g *= sigmoid_dev(param[i]);
            grad[i] = g;
        } else {
            g = grad[i];
        }
        float m = mk[i];
        float v = vk[i];
        m = m + w1 * (g - m);
        v = v * a.beta2 + w2 * g * g;
        const float denom = sqrtf(v) / bc2_sqrt + a.eps;
        param[i] = param[i] + step_size * (m / denom);
        mk[i] = m;
        vk[i] = v;
    }
}

int launch_adam(const sbp_state *s, const sbp_adam_params *p, const int32_t *step_dev,
                int a_softplus, hipStream_t st, const AdamFuse *fuse) {
    (void)a_softplus;
    AdamArgs a;
    float *P[5] = {s->balls.x, s->balls.y, s->balls.z, s->balls.p0, s->balls.a};
    float *Gr[5] = {s->grad.x, s->grad.y, s->grad.z, s->grad.p0, s->grad.a};
    float *M[5] = {s->m.x, s->m.y, s->m.z, s->m.p0, s->m.a};
    float *V[5] = {s->v.x, s->v.y, s->v.z, s->v.p0, s->v.a};
    for (int k = 0; k < 5; ++k) {
        a.param[k] = P[k];
        a.grad[k] = Gr[k];
        a.m[k] = M[k];
        a.v[k] = V[k];
        a.lr[k] = p->lr[k];
    }
    a.beta1 = p->beta1;
    a.beta2 = p->beta2;
    a.eps = p->eps;
    a.step = p->step;
    a.mask = p->mask;
    a.part = fuse ? fuse->adj.part : nullptr;
    a.nsl = fuse ? fuse->adj.nsl : 0;
    a.pstride = fuse ? fuse->adj.pstride : 0;
    a.a_softplus = fuse ? fuse->a_softplus : 0;
    a.loss_partial = fuse ? fuse->loss_partial : nullptr;
    a.loss = fuse ? fuse->loss : nullptr;
    a.misc_clear = fuse ? fuse->misc_clear : nullptr;
    a.step_add = fuse ? fuse->step_add : 0;
    a.row_loss = fuse ? fuse->row_loss : nullptr;
    a.D = fuse ? fuse->D : 0;
    a.T = fuse ? fuse->T : 0;
    a.y_ref = fuse ? fuse->y_ref : nullptr;
    a.y_work = fuse ? fuse->y_work : nullptr;
    a.gacc = fuse ? fuse->gacc : nullptr;
    a.n_gacc = fuse ? fuse->n_gacc : 0;
    a.n_adam = ew_grid(s->B_cap) < 2048 ? ew_grid(s->B_cap) : 2048;   // per parameter row
    const int nloss = (a.loss_partial || a.row_loss) ? s->F : 0;
    if (s->B_cap == 0 && nloss == 0 && !a.misc_clear && !a.gacc) return SBP_OK;
    hipLaunchKernelGGL(k_adam, dim3(a.n_adam + nloss, 5), dim3(kEw), 0, st, a, s->ball_off, s->F,
                       step_dev);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

// a <-> a~ for balls [0, count): to_softplus = 1 stores a~ = log(expm1(a))
// (a <= 0 becomes a~ = -88, i.e. a ~ 1e-38), to_softplus = 0 stores
// a = softplus(a~).  The size's Adam moments restart at zero when given.
__global__ void k_reparam(float *a, float *m, float *v, const int64_t *__restrict__ ball_off, int F,
                          int to_softplus) {
    const int64_t count = ball_off[F];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float x = a[i];
        float r;
        if (to_softplus) {
            const double xd = (double)x;
            r = x > 0.0f ? (float)(xd > 30.0 ? xd : log(expm1(xd))) : -88.0f;
        } else {
            r = softplus_dev(x);
        }
        a[i] = r;
        if (m) m[i] = 0.0f;
        if (v) v[i] = 0.0f;
    }
}

int launch_reparam(float *a, float *m, float *v, const int64_t *ball_off, int F, int64_t B_cap,
                   int to_softplus, hipStream_t st) {
    if (B_cap == 0) return SBP_OK;
    hipLaunchKernelGGL(k_reparam, dim3(ew_grid(B_cap)), dim3(kEw), 0, st, a, m, v, ball_off, F,
                       to_softplus);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

__global__ void k_incr(int32_t *p, int32_t by) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p += by;
}

int launch_incr(int32_t *p, hipStream_t st) { return launch_incr_by(p, 1, st); }

int launch_incr_by(int32_t *p, int32_t by, hipStream_t st) {
    hipLaunchKernelGGL(k_incr, dim3(1), dim3(64), 0, st, p, by);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

// ------------------------------------------------------------- compaction --
// Stable compaction of the balls whose filter gradient passes the keep test.
// Blocks of kEw consecutive indices: count, exclusive scan of the counts in one
// workgroup, then a scatter where each wave ranks its lanes with a ballot.

__device__ inline bool keep_of(const float *g, int64_t i, int64_t count, int strict) {
    if (i >= count) return false;
    const float v = g[i];
    return strict ? (v < 0.0f) : (v <= 0.0f);
}

__global__ void k_count_keep(const float *__restrict__ g, int strict,
                             const int64_t *__restrict__ off_in, int F, int *__restrict__ cnt) {
    const int64_t count = off_in[F];
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    const int c = __syncthreads_count(keep_of(g, i, count, strict));
    if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

__global__ void k_scan_counts(const int *__restrict__ cnt, int nblk, int64_t *__restrict__ pre) {
    __shared__ int64_t s_carry;
    __shared__ int64_t s_wave[1024 / 64];
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int base = 0; base < nblk; base += blockDim.x) {
        const int i = base + threadIdx.x;
        int64_t x = i < nblk ? cnt[i] : 0;
        // inclusive wave scan
        int64_t s = x;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t t = __shfl_up(s, o, 64);
            if (lane >= o) s += t;
        }
        if (lane == 63) s_wave[wid] = s;
        __syncthreads();
        int64_t wpre = 0;
        for (int w = 0; w < wid; ++w) wpre += s_wave[w];
        const int64_t carry = s_carry;
        if (i < nblk) pre[i] = carry + wpre + s - x;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) s_carry = carry + wpre + s;
        __syncthreads();
    }
    if (threadIdx.x == 0) pre[nblk] = s_carry;
}

struct CompactArgs {
    const float *src[15];
    float *dst[15];
    int narr;
};

__global__ void k_scatter_keep(const float *__restrict__ g, int strict,
                               const int64_t *__restrict__ off_in, int F,
                               const int64_t *__restrict__ pre, CompactArgs ca) {
    __shared__ int s_wave[kEw / 64];
    const int64_t count = off_in[F];
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    const bool k = keep_of(g, i, count, strict);
    const unsigned long long bal = __ballot(k);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int below = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[wid] = __popcll(bal);
    __syncthreads();
    int wpre = 0;
    for (int w = 0; w < wid; ++w) wpre += s_wave[w];
    if (k) {
        const int64_t dst = pre[blockIdx.x] + wpre + below;
        for (int a = 0; a < ca.narr; ++a) ca.dst[a][dst] = ca.src[a][i];
    }
}

__global__ void k_frame_offsets(const float *__restrict__ g, int strict,
                                const int64_t *__restrict__ off_in, int F, int nblk,
                                const int64_t *__restrict__ pre, int64_t *__restrict__ off_out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f > F) return;
    const int64_t count = off_in[F];
    const int64_t p = off_in[f];
    const int64_t blk = p / kEw;
    if (blk >= nblk) {
        off_out[f] = pre[nblk];
        return;
    }
    int64_t c = pre[blk];
    for (int64_t i = blk * kEw; i < p; ++i) c += keep_of(g, i, count, strict) ? 1 : 0;
    off_out[f] = c;
}

size_t compact_ws_bytes(int64_t B_cap) {
    const int64_t nblk = (B_cap + kEw - 1) / kEw;
    return (size_t)(nblk + 1) * sizeof(int) + 256 + (size_t)(nblk + 2) * sizeof(int64_t);
}

int launch_compact(void *ws, const float *g, int strict, const BallsP<float> &in,
                   const int64_t *off_in, int F, int64_t B_cap, const BallsP<float> &out,
                   int64_t *off_out, const BallsP<float> *m_in, const BallsP<float> *v_in,
                   const BallsP<float> *m_out, const BallsP<float> *v_out, hipStream_t st) {
    const int64_t nblk64 = (B_cap + kEw - 1) / kEw;
    if (nblk64 > (int64_t)1 << 30) return fail(SBP_E_ARG, "B_cap too large");
    const int nblk = (int)nblk64;
    int *cnt = (int *)ws;
    const size_t off_pre = ((size_t)(nblk + 1) * sizeof(int) + 255) & ~(size_t)255;
    int64_t *pre = (int64_t *)((char *)ws + off_pre);
    if (nblk > 0) {
        hipLaunchKernelGGL(k_count_keep, dim3(nblk), dim3(kEw), 0, st, g, strict, off_in, F, cnt);
        SBP_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, cnt, nblk, pre);
    SBP_HIP(hipGetLastError());
    CompactArgs ca;
    int n = 0;
    const BallsP<float> *srcs[3] = {&in, m_in, v_in};
    const BallsP<float> *dsts[3] = {&out, m_out, v_out};
    for (int s = 0; s < 3; ++s) {
        if (!srcs[s] || !dsts[s]) continue;
        const BallsP<float> &a = *srcs[s];
        const BallsP<float> &b = *dsts[s];
        const float *sa[5] = {a.x, a.y, a.z, a.p0, a.a};
        float *da[5] = {b.x, b.y, b.z, b.p0, b.a};
        for (int k = 0; k < 5; ++k) {
            ca.src[n] = sa[k];
            ca.dst[n] = da[k];
            ++n;
        }
    }
    ca.narr = n;
    if (nblk > 0) {
        hipLaunchKernelGGL(k_scatter_keep, dim3(nblk), dim3(kEw), 0, st, g, strict, off_in, F, pre,
                           ca);
        SBP_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_frame_offsets, dim3(1), dim3(SBP_MAX_FRAMES + 64), 0, st, g, strict,
                       off_in, F, nblk, pre, off_out);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

// ---------------------------------------------------------------------------
// Spatial visiting order of a cloud.  The gather-form kernels give each lane
// its own balls and sum every ball's terms in a fixed order, so the order in
// which balls are assigned to lanes changes no result; it does change speed:
// when a wave's balls are neighbours their times of flight are close, the
// staged-row reads of one instruction fall on nearby LDS addresses (fewer
// bank conflicts) and the directivity and window tests agree across the wave.
// order[off[0] + k], k = 0 .. count-1, lists the balls of every frame sorted
// by (frame, Morton code of a 2^bits-per-axis cell grid over the cloud's
// bounding box); within a cell the order is whatever the atomics produce.
constexpr int kOrdBoxBlocks = 256;
constexpr int kOrdMaxKeys = 1 << 17;

__global__ void k_ord_box(const BallsP<float> b, const int64_t *__restrict__ off, int F,
                          float *__restrict__ part) {
    __shared__ float s[6][kEw];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t i0 = off[0], i1 = off[F];
    for (int64_t i = i0 + (int64_t)blockIdx.x * kEw + threadIdx.x; i < i1;
         i += (int64_t)gridDim.x * kEw) {
        const float v[3] = {b.x[i], b.y[i], b.z[i]};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], v[k]);
            hi[k] = fmaxf(hi[k], v[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s[k][threadIdx.x] = lo[k];
        s[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int w = kEw / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                s[k][threadIdx.x] = fminf(s[k][threadIdx.x], s[k][threadIdx.x + w]);
                s[3 + k][threadIdx.x] = fmaxf(s[3 + k][threadIdx.x], s[3 + k][threadIdx.x + w]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__device__ inline int ord_spread(int v, int bits) {
    int r = 0;
    for (int k = 0; k < bits; ++k) r |= ((v >> k) & 1) << (3 * k);
    return r;
}

// Key of every ball (frame * 8^bits + Morton cell) and the per-key counts.
__global__ void k_ord_key(const BallsP<float> b, const int64_t *__restrict__ off, int F, int bits,
                          const float *__restrict__ part, int *__restrict__ key,
                          int *__restrict__ cnt) {
    __shared__ float s_box[6];
    __shared__ int64_t s_off[SBP_MAX_FRAMES + 1];
    if (threadIdx.x < 6) {
        const bool mx = threadIdx.x >= 3;
        float r = mx ? -INFINITY : INFINITY;
        for (int j = 0; j < kOrdBoxBlocks; ++j) {
            const float v = part[j * 6 + threadIdx.x];
            r = mx ? fmaxf(r, v) : fminf(r, v);
        }
        s_box[threadIdx.x] = r;
    }
    for (int f = threadIdx.x; f <= F; f += kEw) s_off[f] = off[f];
    __syncthreads();
    const int n = 1 << bits;
    float lo[3], sc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        lo[k] = s_box[k];
        const float ext = s_box[3 + k] - s_box[k];
        sc[k] = ext > 0.0f ? (float)n / ext : 0.0f;
    }
    const int64_t i0 = s_off[0], i1 = s_off[F];
    for (int64_t i = i0 + (int64_t)blockIdx.x * kEw + threadIdx.x; i < i1;
         i += (int64_t)gridDim.x * kEw) {
        int f = 0;
        while (f + 1 < F && i >= s_off[f + 1]) ++f;
        const float v[3] = {b.x[i], b.y[i], b.z[i]};
        int m = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            // NaN and out-of-range coordinates land in an edge cell
            const float q = fminf(fmaxf((v[k] - lo[k]) * sc[k], 0.0f), (float)(n - 1));
            m |= ord_spread((int)q, bits) << k;
        }
        const int kk = (f << (3 * bits)) | m;
        key[i - i0] = kk;
        atomicAdd(&cnt[kk], 1);
    }
}

__global__ void k_ord_scatter(const int64_t *__restrict__ off, int F, const int *__restrict__ key,
                              unsigned long long *__restrict__ cursor, int32_t *__restrict__ order) {
    const int64_t i0 = off[0], i1 = off[F];
    for (int64_t i = i0 + (int64_t)blockIdx.x * kEw + threadIdx.x; i < i1;
         i += (int64_t)gridDim.x * kEw) {
        const unsigned long long pos = atomicAdd(&cursor[key[i - i0]], 1ull);
        order[i0 + (int64_t)pos] = (int32_t)i;
    }
}

int order_bits(int F, int64_t B_cap) {
    if (F < 1 || B_cap < 1 || B_cap > INT32_MAX) return -1;
    // about one wave of balls per cell, at most 2^17 keys in all
    const double per = (double)B_cap / F / 64.0;
    int bits = per > 1.0 ? (int)lround(log2(per) / 3.0) : 0;
    if (bits > 5) bits = 5;
    while (bits > 0 && ((int64_t)F << (3 * bits)) > kOrdMaxKeys) --bits;
    return bits < 1 ? -1 : bits;
}

size_t order_ws_bytes(int F, int64_t B_cap) {
    const int bits = order_bits(F, B_cap);
    if (bits < 0) return 0;
    const int64_t nk = (int64_t)F << (3 * bits);
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return up((size_t)B_cap * 4) * 2 + up((size_t)nk * 4) + up((size_t)(nk + 1) * 8) +
           up((size_t)kOrdBoxBlocks * 6 * 4);
}

int launch_order(void *ws, const BallsP<float> &b, const int64_t *off, int F, int64_t B_cap,
                 int32_t **order, hipStream_t st) {
    *order = nullptr;
    const int bits = order_bits(F, B_cap);
    if (bits < 0) return SBP_OK;
    const int64_t nk = (int64_t)F << (3 * bits);
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char *p = (char *)ws;
    int32_t *ord = (int32_t *)p;
    p += up((size_t)B_cap * 4);
    int *key = (int *)p;
    p += up((size_t)B_cap * 4);
    int *cnt = (int *)p;
    p += up((size_t)nk * 4);
    int64_t *pre = (int64_t *)p;
    p += up((size_t)(nk + 1) * 8);
    float *part = (float *)p;
    int rc;
    if ((rc = launch_fill<int>(cnt, nk, 0, st))) return rc;
    hipLaunchKernelGGL(k_ord_box, dim3(kOrdBoxBlocks), dim3(kEw), 0, st, b, off, F, part);
    SBP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ord_key, dim3(ew_grid(B_cap)), dim3(kEw), 0, st, b, off, F, bits,
                       (const float *)part, key, cnt);
    SBP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, (const int *)cnt, (int)nk, pre);
    SBP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ord_scatter, dim3(ew_grid(B_cap)), dim3(kEw), 0, st, off, F,
                       (const int *)key, (unsigned long long *)pre, ord);
    SBP_HIP(hipGetLastError());
    *order = ord;
    return SBP_OK;
}

}  // namespace sbp
