// Plain growth rule (section 4.1 of SlingBAG Pro: split / destroy by thresholds
// on pressure and size in the coarse stage, plus duplication in the fine
// stage) on gfx950.  The paper gives no thresholds; sbp_growth_rule holds them.
//
// Every decision is taken in FP32 on the stored parameters (the duplication
// rank uses the exact FP64 sum of the squared FP32 position gradients), so the
// set of destroyed / split / duplicated balls is reproducible bit for bit.
//
// Passes (frames are independent; a ball's frame comes from a binary search in
// the frame offsets):
//   1. per-frame max p0                              (ordered-int atomicMax)
//   2. per-block sums of (emitted balls, candidates) -> exclusive scan
//   3. per frame: k = floor(n_candidates * dup_frac)
//   4. exact k-th largest key per frame by 8 radix passes of 8 bits over the
//      FP64 key, and how many balls equal to it must be taken (lowest index
//      first)
//   5. per-block sums of (key > threshold, key == threshold) -> exclusive scan
//   6. host reads the total (one synchronisation) and checks the capacity
//   7. scatter: survivors and children in input order, then the clones
#include <climits>

#include "sbp_internal.hpp"

namespace sbp {

constexpr int kGb = 256;

struct GrowIn {
    const float *x, *y, *z, *p0, *a;
    const float *gx, *gy, *gz;
    const float *m[5];
    const float *v[5];
    const int64_t *off;
    int F;
};

struct GrowOut {
    float *x, *y, *z, *p0, *a;
    float *m[5];
    float *v[5];
    int64_t *off;
};

struct GrowWs {
    int *pmax_key;        // [F]
    int64_t *blk;         // [4][nblk]   block sums of emit, cand, gt, eq
    int64_t *pre;         // [4][nblk+1] exclusive scans
    int64_t *kneed;       // [F] remaining count to select
    uint64_t *prefix;     // [F] threshold key bits being built
    int64_t *hist;        // [F][256]
    int64_t *frame_base;  // [F+1] output offsets
    int64_t *fpre;        // [4][F+1] prefix of each counter at the frame starts
};

__device__ inline int ordered_key(float x) {
    int k = __float_as_int(x);
    return k >= 0 ? k : (k ^ 0x7fffffff);
}
__device__ inline float ordered_val(int k) { return __int_as_float(k >= 0 ? k : (k ^ 0x7fffffff)); }

__device__ inline double dup_key(const GrowIn &in, int64_t i) {
    const double gx = in.gx[i], gy = in.gy[i], gz = in.gz[i];
    double k = gx * gx + gy * gy;
    k = k + gz * gz;
    return k;
}

struct Cls {
    bool alive, split, cand;
};

__device__ inline Cls classify(const GrowIn &in, const sbp_growth_rule &r, const int *pmax_key,
                               int f, int64_t i) {
    const float p0 = in.p0[i], a = in.a[i];
    const float thr = r.destroy_frac * ordered_val(pmax_key[f]);
    Cls c;
    c.alive = !((p0 < thr) || (a < r.a_min));
    c.split = c.alive && (a > r.a_split);
    c.cand = c.alive && !c.split;
    return c;
}

#define LOAD_OFFSETS()                                     \
    __shared__ int64_t s_off[SBP_MAX_FRAMES + 1];          \
    for (int i_ = threadIdx.x; i_ <= in.F; i_ += blockDim.x) s_off[i_] = in.off[i_]; \
    __syncthreads();                                       \
    const int64_t count = s_off[in.F];

// Grid (slices, F): block (s, f) reduces a slice of frame f, then one atomic.
__global__ void k_g_max(GrowIn in, int *pmax_key) {
    __shared__ int s_red[kGb / 64];
    const int f = blockIdx.y;
    const int64_t lo = in.off[f], hi = in.off[f + 1];
    int m = INT_MIN;
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, ordered_key(in.p0[i]));
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kGb / 64; ++w) m = max(m, s_red[w]);
        if (m != INT_MIN) atomicMax(pmax_key + f, m);
    }
}

// Block sums of up to four per-ball counters (which ones: `which` bits).
__global__ void k_g_blocksum(GrowIn in, sbp_growth_rule r, GrowWs ws, int nblk, int which) {
    LOAD_OFFSETS();
    __shared__ int64_t s_red[4][kGb / 64];
    const int64_t i = (int64_t)blockIdx.x * kGb + threadIdx.x;
    int64_t c[4] = {0, 0, 0, 0};
    if (i < count) {
        const int f = frame_of(s_off, in.F, i);
        const Cls k = classify(in, r, ws.pmax_key, f, i);
        c[0] = k.alive ? (k.split ? 2 : 1) : 0;
        c[1] = k.cand ? 1 : 0;
        if (which & 4) {
            if (k.cand && ws.kneed[f] > 0) {
                const uint64_t key = (uint64_t)__double_as_longlong(dup_key(in, i));
                c[2] = key > ws.prefix[f] ? 1 : 0;
                c[3] = key == ws.prefix[f] ? 1 : 0;
            }
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int64_t x = c[q];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if (lane == 0) s_red[q][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        int64_t t = 0;
        for (int w = 0; w < kGb / 64; ++w) t += s_red[q][w];
        if (which & (q < 2 ? 1 : 4)) ws.blk[(int64_t)q * nblk + blockIdx.x] = t;
    }
}

// Exclusive scan of blk[q] into pre[q] for the q selected by `which`, one workgroup.
__global__ void k_g_scan(GrowWs ws, int nblk, int which) {
    __shared__ int64_t s_carry;
    __shared__ int64_t s_wave[1024 / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int q = 0; q < 4; ++q) {
        if (!(which & (q < 2 ? 1 : 4))) continue;
        const int64_t *cnt = ws.blk + (int64_t)q * nblk;
        int64_t *pre = ws.pre + (int64_t)q * (nblk + 1);
        if (threadIdx.x == 0) s_carry = 0;
        __syncthreads();
        for (int base = 0; base < nblk; base += blockDim.x) {
            const int i = base + threadIdx.x;
            const int64_t x = i < nblk ? cnt[i] : 0;
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
        __syncthreads();
    }
}

// Exclusive prefix of counter q at ball index p (0 <= p <= count).
__device__ inline int64_t prefix_at(const GrowIn &in, const sbp_growth_rule &r, const GrowWs &ws,
                                    const int64_t *s_off, int64_t count, int nblk, int q, int64_t p) {
    const int64_t blk = p / kGb;
    const int64_t *pre = ws.pre + (int64_t)q * (nblk + 1);
    if (blk >= nblk) return pre[nblk];
    int64_t c = pre[blk];
    for (int64_t i = blk * kGb; i < p; ++i) {
        if (i >= count) break;
        const int f = frame_of(s_off, in.F, i);
        const Cls k = classify(in, r, ws.pmax_key, f, i);
        if (q == 0) c += k.alive ? (k.split ? 2 : 1) : 0;
        else if (q == 1) c += k.cand ? 1 : 0;
        else if (k.cand && ws.kneed[f] > 0) {
            const uint64_t key = (uint64_t)__double_as_longlong(dup_key(in, i));
            c += (q == 2) ? (key > ws.prefix[f] ? 1 : 0) : (key == ws.prefix[f] ? 1 : 0);
        }
    }
    return c;
}

// Per frame: k = floor(n_cand * dup_frac); reset the radix-select state.
__global__ void k_g_need(GrowIn in, sbp_growth_rule r, GrowWs ws, int nblk) {
    LOAD_OFFSETS();
    const int f = threadIdx.x;
    if (f >= in.F) return;
    const int64_t c0 = prefix_at(in, r, ws, s_off, count, nblk, 1, s_off[f]);
    const int64_t c1 = prefix_at(in, r, ws, s_off, count, nblk, 1, s_off[f + 1]);
    ws.kneed[f] = (int64_t)floor((double)(c1 - c0) * (double)r.dup_frac);
    ws.prefix[f] = 0;
}

// Histogram of the current 8-bit digit of the candidates' keys whose higher
// digits match the threshold prefix; LDS counts per frame, flushed once.
__global__ void k_g_hist(GrowIn in, sbp_growth_rule r, GrowWs ws, int shift) {
    LOAD_OFFSETS();
    extern __shared__ unsigned s_hist[];   // [F][256]
    for (int i = threadIdx.x; i < 256 * in.F; i += blockDim.x) s_hist[i] = 0u;
    __syncthreads();
    const uint64_t hi_mask = shift == 56 ? 0ull : (~0ull << (shift + 8));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int f = frame_of(s_off, in.F, i);
        if (ws.kneed[f] <= 0) continue;
        const Cls k = classify(in, r, ws.pmax_key, f, i);
        if (!k.cand) continue;
        const uint64_t key = (uint64_t)__double_as_longlong(dup_key(in, i));
        if ((key & hi_mask) == (ws.prefix[f] & hi_mask))
            atomicAdd(&s_hist[f * 256 + (int)((key >> shift) & 255)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 256 * in.F; i += blockDim.x)
        if (s_hist[i]) atomicAdd((unsigned long long *)(ws.hist + i), (unsigned long long)s_hist[i]);
}

// Choose the digit of the k-th largest key; kneed becomes the rank within it.
__global__ void k_g_pick(GrowWs ws, int F, int shift) {
    const int f = threadIdx.x;
    if (f >= F) return;
    int64_t need = ws.kneed[f];
    if (need <= 0) return;
    int64_t *h = ws.hist + (int64_t)f * 256;
    int digit = 0;
    for (int d = 255; d >= 0; --d) {
        if (h[d] >= need) { digit = d; break; }
        need -= h[d];
    }
    ws.prefix[f] |= (uint64_t)digit << shift;
    ws.kneed[f] = need;
    for (int d = 0; d < 256; ++d) h[d] = 0;
}

__global__ void k_g_frames(GrowIn in, sbp_growth_rule r, GrowWs ws, int nblk, int with_dup) {
    LOAD_OFFSETS();
    const int F = in.F;
    // prefixes of the counters at every frame start, one thread per (counter, frame)
    for (int t = threadIdx.x; t < 4 * (F + 1); t += blockDim.x) {
        const int q = t / (F + 1), f = t - q * (F + 1);
        int64_t v = 0;
        if (q == 0 || (with_dup && q >= 2)) v = prefix_at(in, r, ws, s_off, count, nblk, q, s_off[f]);
        ws.fpre[t] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    int64_t o = 0;
    for (int f = 0; f < F; ++f) {
        ws.frame_base[f] = o;
        const int64_t e = ws.fpre[f + 1] - ws.fpre[f];
        int64_t kd = 0;
        if (with_dup && ws.kneed[f] > 0)
            kd = (ws.fpre[2 * (F + 1) + f + 1] - ws.fpre[2 * (F + 1) + f]) + ws.kneed[f];
        o += e + kd;
    }
    ws.frame_base[F] = o;
}

__device__ inline int64_t block_excl_scan(int64_t x, int64_t *s_wave) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t s = x;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(s, o, 64);
        if (lane >= o) s += t;
    }
    if (lane == 63) s_wave[wid] = s;
    __syncthreads();
    int64_t wpre = 0;
    for (int w = 0; w < wid; ++w) wpre += s_wave[w];
    __syncthreads();
    return wpre + s - x;
}

__global__ void k_g_scatter(GrowIn in, sbp_growth_rule r, GrowWs ws, int nblk, int with_dup,
                            GrowOut out) {
    LOAD_OFFSETS();
    __shared__ int64_t s_wave[kGb / 64];
    const int64_t i = (int64_t)blockIdx.x * kGb + threadIdx.x;
    int emit = 0, gt = 0, eq = 0, f = 0;
    Cls k{false, false, false};
    if (i < count) {
        f = frame_of(s_off, in.F, i);
        k = classify(in, r, ws.pmax_key, f, i);
        emit = k.alive ? (k.split ? 2 : 1) : 0;
        if (with_dup && k.cand && ws.kneed[f] > 0) {
            const uint64_t key = (uint64_t)__double_as_longlong(dup_key(in, i));
            gt = key > ws.prefix[f] ? 1 : 0;
            eq = key == ws.prefix[f] ? 1 : 0;
        }
    }
    const int64_t e_loc = block_excl_scan(emit, s_wave);
    const int64_t g_loc = with_dup ? block_excl_scan(gt, s_wave) : 0;
    const int64_t q_loc = with_dup ? block_excl_scan(eq, s_wave) : 0;
    if (i >= count) return;
    const int64_t *pe = ws.pre;
    const int64_t *pg = ws.pre + 2 * (int64_t)(nblk + 1);
    const int64_t *pq = ws.pre + 3 * (int64_t)(nblk + 1);
    const int F = in.F;
    const int64_t e_lo = ws.fpre[f], e_hi = ws.fpre[f + 1];
    const int64_t e_i = pe[blockIdx.x] + e_loc;
    const int64_t base = ws.frame_base[f];
    const float x = in.x[i], y = in.y[i], z = in.z[i], p0 = in.p0[i], a = in.a[i];
    if (emit == 1) {
        const int64_t o = base + (e_i - e_lo);
        out.x[o] = x; out.y[o] = y; out.z[o] = z; out.p0[o] = p0; out.a[o] = a;
        for (int q = 0; q < 5; ++q) {
            if (out.m[q]) out.m[q][o] = in.m[q] ? in.m[q][i] : 0.0f;
            if (out.v[q]) out.v[q][o] = in.v[q] ? in.v[q][i] : 0.0f;
        }
    } else if (emit == 2) {
        const float ax = fabsf(in.gx[i]), ay = fabsf(in.gy[i]), az = fabsf(in.gz[i]);
        const int axis = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
        const float h = 0.5f * a;
        const float ac = a * 0.79370052598409973738f;  // a / 2^(1/3)
        for (int s = 0; s < 2; ++s) {
            const float sg = s == 0 ? -h : h;
            const int64_t o = base + (e_i - e_lo) + s;
            out.x[o] = axis == 0 ? x + sg : x;
            out.y[o] = axis == 1 ? y + sg : y;
            out.z[o] = axis == 2 ? z + sg : z;
            out.p0[o] = p0;
            out.a[o] = ac;
            for (int q = 0; q < 5; ++q) {
                if (out.m[q]) out.m[q][o] = 0.0f;
                if (out.v[q]) out.v[q][o] = 0.0f;
            }
        }
    }
    if (with_dup && (gt || eq)) {
        const int64_t g_i = pg[blockIdx.x] + g_loc;
        const int64_t q_i = pq[blockIdx.x] + q_loc;
        const int64_t g_lo = ws.fpre[2 * (F + 1) + f];
        const int64_t q_lo = ws.fpre[3 * (F + 1) + f];
        const int64_t take = ws.kneed[f];
        const int64_t eq_before = q_i - q_lo;
        if (gt || eq_before < take) {
            const int64_t rank = (g_i - g_lo) + (eq_before < take ? eq_before : take);
            const int64_t o = base + (e_hi - e_lo) + rank;
            const double gx = in.gx[i], gy = in.gy[i], gz = in.gz[i];
            const double nrm = sqrt(dup_key(in, i));
            const double s = nrm > 0.0 ? -(double)r.dup_offset * (double)a / nrm : 0.0;
            out.x[o] = (float)((double)x + s * gx);
            out.y[o] = (float)((double)y + s * gy);
            out.z[o] = (float)((double)z + s * gz);
            out.p0[o] = p0;
            out.a[o] = a;
            for (int q = 0; q < 5; ++q) {
                if (out.m[q]) out.m[q][o] = 0.0f;
                if (out.v[q]) out.v[q][o] = 0.0f;
            }
        }
    }
}

__global__ void k_g_offsets(const int64_t *frame_base, int F, int64_t *off_out) {
    const int f = threadIdx.x;
    if (f <= F) off_out[f] = frame_base[f];
}

int launch_grow(Ctx *c, const sbp_state *in, const sbp_growth_rule *rule, sbp_state *out,
                int64_t *count_out, hipStream_t st) {
    const int F = in->F;
    const int64_t B = in->B_cap;
    const int nblk = (int)((B + kGb - 1) / kGb);
    const int nb1 = nblk + 1;
    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 255) & ~(size_t)255; return o; };
    const size_t o_pmax = take(sizeof(int) * F);
    const size_t o_blk = take(sizeof(int64_t) * 4 * (size_t)(nblk > 0 ? nblk : 1));
    const size_t o_pre = take(sizeof(int64_t) * 4 * (size_t)nb1);
    const size_t o_kneed = take(sizeof(int64_t) * F);
    const size_t o_prefix = take(sizeof(uint64_t) * F);
    const size_t o_hist = take(sizeof(int64_t) * 256 * F);
    const size_t o_fb = take(sizeof(int64_t) * (F + 1));
    const size_t o_fpre = take(sizeof(int64_t) * 4 * (F + 1));
    int rc = ensure_scratch(c, off);
    if (rc) return rc;
    char *base = (char *)c->scratch;
    GrowWs ws;
    ws.pmax_key = (int *)(base + o_pmax);
    ws.blk = (int64_t *)(base + o_blk);
    ws.pre = (int64_t *)(base + o_pre);
    ws.kneed = (int64_t *)(base + o_kneed);
    ws.prefix = (uint64_t *)(base + o_prefix);
    ws.hist = (int64_t *)(base + o_hist);
    ws.frame_base = (int64_t *)(base + o_fb);
    ws.fpre = (int64_t *)(base + o_fpre);

    GrowIn gi;
    gi.x = in->balls.x; gi.y = in->balls.y; gi.z = in->balls.z; gi.p0 = in->balls.p0; gi.a = in->balls.a;
    gi.gx = in->grad.x; gi.gy = in->grad.y; gi.gz = in->grad.z;
    const float *im[5] = {in->m.x, in->m.y, in->m.z, in->m.p0, in->m.a};
    const float *iv[5] = {in->v.x, in->v.y, in->v.z, in->v.p0, in->v.a};
    for (int q = 0; q < 5; ++q) { gi.m[q] = im[q]; gi.v[q] = iv[q]; }
    gi.off = in->ball_off;
    gi.F = F;
    GrowOut go;
    go.x = out->balls.x; go.y = out->balls.y; go.z = out->balls.z; go.p0 = out->balls.p0; go.a = out->balls.a;
    float *om[5] = {out->m.x, out->m.y, out->m.z, out->m.p0, out->m.a};
    float *ov[5] = {out->v.x, out->v.y, out->v.z, out->v.p0, out->v.a};
    for (int q = 0; q < 5; ++q) { go.m[q] = om[q]; go.v[q] = ov[q]; }
    go.off = out->ball_off;

    const int with_dup = rule->dup_frac > 0.0f ? 1 : 0;
    const int grid = nblk > 0 ? nblk : 1;
    int rc2 = launch_fill<int32_t>(ws.pmax_key, F, (int32_t)0x80000000, st);
    if (rc2) return rc2;
    rc2 = launch_fill<int64_t>(ws.hist, 256 * (int64_t)F, 0, st);
    if (rc2) return rc2;
    rc2 = launch_fill<int64_t>(ws.blk, 4 * (int64_t)(nblk > 0 ? nblk : 1), 0, st);
    if (rc2) return rc2;
    rc2 = launch_fill<int64_t>(ws.pre, 4 * (int64_t)nb1, 0, st);
    if (rc2) return rc2;
    rc2 = launch_fill<uint64_t>(ws.prefix, F, 0ull, st);
    if (rc2) return rc2;
    hipLaunchKernelGGL(k_g_max, dim3(256, F), dim3(kGb), 0, st, gi, ws.pmax_key);
    SBP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_g_blocksum, dim3(grid), dim3(kGb), 0, st, gi, *rule, ws, nblk, 1);
    SBP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_g_scan, dim3(1), dim3(1024), 0, st, ws, nblk, 1);
    SBP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_g_need, dim3(1), dim3(SBP_MAX_FRAMES + 64), 0, st, gi, *rule, ws, nblk);
    SBP_HIP(hipGetLastError());
    if (with_dup) {
        for (int shift = 56; shift >= 0; shift -= 8) {
            hipLaunchKernelGGL(k_g_hist, dim3(grid < 1024 ? grid : 1024), dim3(kGb),
                               (size_t)256 * F * sizeof(unsigned), st, gi, *rule, ws, shift);
            SBP_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_g_pick, dim3(1), dim3(SBP_MAX_FRAMES), 0, st, ws, F, shift);
            SBP_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_g_blocksum, dim3(grid), dim3(kGb), 0, st, gi, *rule, ws, nblk, 4);
        SBP_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_g_scan, dim3(1), dim3(1024), 0, st, ws, nblk, 4);
        SBP_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_g_frames, dim3(1), dim3(256), 0, st, gi, *rule, ws, nblk,
                       with_dup);
    SBP_HIP(hipGetLastError());
    int64_t total = 0;
    SBP_HIP(hipMemcpyAsync(&total, ws.frame_base + F, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SBP_HIP(hipStreamSynchronize(st));
    if (count_out) *count_out = total;
    if (total > out->B_cap)
        return fail(SBP_E_CAPACITY, "growth needs %lld balls, output capacity is %lld",
                    (long long)total, (long long)out->B_cap);
    if (nblk > 0) {
        hipLaunchKernelGGL(k_g_scatter, dim3(nblk), dim3(kGb), 0, st, gi, *rule, ws, nblk, with_dup,
                           go);
        SBP_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_g_offsets, dim3(1), dim3(SBP_MAX_FRAMES + 64), 0, st, ws.frame_base, F,
                       out->ball_off);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

}  // namespace sbp
