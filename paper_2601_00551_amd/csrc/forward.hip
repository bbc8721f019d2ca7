// Forward model (Simulate of section 4.2 / 4.3 of SlingBAG Pro) on gfx950.
//
// Scatter form: a lane owns a ball, loops over a group of `dg` transducers
// whose traces it accumulates in LDS rows (the full record, or time tiles of
// it), and for each pair adds its bin values
//     amp * (max(q(u_n), 0) - max(q(u_{n+1}), 0))
// into the row with LDS atomics.  Adding bin values (which sum to zero per
// pair) rather than edge values avoids the cancellation a running
// antiderivative would suffer when many balls overlap in a bin.
//
// LDS accumulation.  gfx950 serialises LDS FP32 atomic adds (about 0.3 lanes
// per clock per CU, against ~7 for 64-bit integer adds), so the FP32 path
// accumulates in exact 64-bit fixed point: each bin value is rounded to an
// integer multiple of a power-of-two quantum q = 2^-k chosen per launch from
// a bound on |bin value| over all balls (|p0| a / (2 K c dt) for GAUSS,
// |p0| a / (4 c dt) for UNIFORM, using rho > support half-width), so that a
// single value never exceeds 2^30 q.  Flushed rows are added, still as
// integers, to a global int64 accumulator per sample, which one pass turns
// into FP32 at the end: every sum is exact, so the signals do not depend on
// how the work was split or scheduled (bitwise reproducible).  Each value is
// rounded to the nearest multiple of q (q <= 2^-29 of that bound): at most
// q / 2 per value, with no bias, so the errors of the many balls that reach a
// sample add like a random walk instead of in one direction.  The FP64 path
// keeps FP64 rows (LDS FP64 adds are not serialised) and flushes with FP64
// atomics.
//
// Work items are (frame, transducer group, time tile, chunk of block*bpt
// balls) in that order.  A persistent workgroup takes one contiguous range of
// items, so consecutive items share a group and tile and the rows are flushed
// (one global atomic per non-zero sample) only when those change.  Ball counts
// are read on the device, so the launch is sized by capacity and can be
// captured in a graph.
#include <climits>

#include "sbp_internal.hpp"

namespace sbp {

// LDS row element and how bin values are added to it, per precision.
template <typename R> struct FwdAcc;
template <> struct FwdAcc<float> {
    using T = unsigned long long;
    __device__ static void add(T *p, float v_scaled) {
        // to the nearest integer, floor(v + 1/2), in one instruction: |error|
        // <= half a quantum, without the bias truncation toward zero has
        int iv;
        asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(iv) : "v"(v_scaled));
        atomicAdd(p, (unsigned long long)(long long)iv);
    }
    __device__ static float value(T s, float inv_scale) {
        return (float)((double)(long long)s * (double)inv_scale);
    }
};
template <> struct FwdAcc<double> {
    using T = double;
    __device__ static void add(T *p, double v) { atomicAdd(p, v); }
    __device__ static double value(T s, double) { return s; }
};

// max over live balls of |p0| * a (a after softplus; |p0| alone under point
// sampling, where the peak pressure does not scale with a), as float bits in
// misc[kMiscBound] (zeroed before the launch; non-negative floats order like
// their bits).  A ball with a non-finite parameter (or bound term) sets its
// frame's flag misc[kMiscFlags + f] instead, so that the other frames keep a
// finite quantum and the flagged frames are written as NaN.
__global__ void k_amp_bound(BallsP<float> balls, const int64_t *__restrict__ ball_off, int F,
                            int a_softplus, int point, unsigned *misc) {
    __shared__ float s_red[8];
    __shared__ int64_t s_off[SBP_MAX_FRAMES + 1];
    for (int i = threadIdx.x; i <= F; i += blockDim.x) s_off[i] = ball_off[i];
    __syncthreads();
    const int64_t count = s_off[F];
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float p = balls.p0[i];
        const float ar = balls.a[i];
        const float a = a_softplus ? softplus_dev(ar) : ar;
        const float t = point ? fabsf(p) : fabsf(p) * a;
        if (!ball_finite(balls.x[i], balls.y[i], balls.z[i], p, ar) || !isfinite(t)) {
            atomicOr(misc + kMiscFlags + frame_of(s_off, F, i), 1u);
            continue;
        }
        if (a > 0.0f) m = fmaxf(m, t);
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, s_red[w]);
        atomicMax(misc + kMiscBound, __float_as_uint(m));
    }
}

// FP64 twin: the per-frame flags only (the FP64 rows need no quantum).
__global__ void k_nonfinite_flags(BallsP<double> balls, const int64_t *__restrict__ ball_off, int F,
                                  unsigned *misc) {
    __shared__ int64_t s_off[SBP_MAX_FRAMES + 1];
    for (int i = threadIdx.x; i <= F; i += blockDim.x) s_off[i] = ball_off[i];
    __syncthreads();
    const int64_t count = s_off[F];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!ball_finite(balls.x[i], balls.y[i], balls.z[i], balls.p0[i], balls.a[i]))
            atomicOr(misc + kMiscFlags + frame_of(s_off, F, i), 1u);
    }
}

// FP64 twin: every sample of a flagged frame becomes NaN (grid.y = frame).
__global__ void k_poison_frames(const unsigned *__restrict__ misc, int64_t nper, double *__restrict__ y) {
    if (misc[kMiscFlags + blockIdx.y] == 0) return;
    double *yf = y + (int64_t)blockIdx.y * nper;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nper;
         i += (int64_t)gridDim.x * blockDim.x)
        yf[i] = __builtin_nan("");
}

// Bins per unrolled block of the FP32 loops (the FP64 twin keeps the plain
// loop: its exponential is a call, not an instruction).
constexpr int kFwdBlock = 8;
template <typename R> struct FwdBlocks { static constexpr bool on = true; };
template <> struct FwdBlocks<double> { static constexpr bool on = false; };

// N consecutive GAUSS bins from edge m (u_m = ub): the right edge of bin k
// (k = 1..N) has shape value e_k = 2^(q0 (ub - k c)^2), evaluated as
// 2^(X0 + k (X1 + k X2)); bin k adds amp (e_{k-1} - e_k), e_0 = prev.
template <typename R, int N>
__device__ inline void gauss_bins(typename FwdAcc<R>::T *p, R ub, R q0, R X2, R Y1, R amp, R &prev) {
    const R X0 = q0 * ub * ub;
    const R X1 = Y1 * ub;
#pragma unroll
    for (int k = 1; k <= N; ++k) {
        const R e = ex2(fma(R(k), fma(R(k), X2, X1), X0));
        FwdAcc<R>::add(p + (k - 1), amp * (prev - e));
        prev = e;
    }
}

// N consecutive UNIFORM bins from edge m: shape value a^2 - u^2 at the edges,
// bins past the first linear in k (B0 + B1 k).
template <typename R, int N>
__device__ inline void uniform_bins(typename FwdAcc<R>::T *p, R ub, R q0, R c, R amp, R B1, R &prev) {
    const R u1 = ub - c;
    FwdAcc<R>::add(p, amp * (prev - (q0 - u1 * u1)));
    const R B0 = amp * fma(R(-2) * c, ub, -(c * c));
#pragma unroll
    for (int k = 2; k <= N; ++k) FwdAcc<R>::add(p + (k - 1), fma(B1, R(k), B0));
    const R ue = fma(R(-N), c, ub);
    prev = q0 - ue * ue;
}

// N consecutive point samples from sample m (u_m = ub): sample k (k = 0..N-1)
// adds amp u_k e_k, u_k = ub - k c, with e_k = 2^(q0 u_k^2) by the
// two-multiply recurrence e_{k+1} = e_k g_k, g_{k+1} = g_k h restarted here
// (e_0 = 2^(q0 ub^2), g_0 = 2^(Y1 ub + X2), h = 2^(2 X2)).  A sample is the
// value itself, not a difference of neighbours, so the recurrence's rounding
// over a block of eight (a few ulp of e) stays a few ulp of the sample.
template <typename R, int N>
__device__ inline void point_samples(typename FwdAcc<R>::T *p, R ub, R q0, R c, R X2, R Y1, R h,
                                     R amp) {
    R e = ex2(q0 * ub * ub);
    R g = ex2(fma(Y1, ub, X2));
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const R u = fma(R(-k), c, ub);
        FwdAcc<R>::add(p + k, amp * u * e);
        if (k + 1 < N) {
            e *= g;
            g *= h;
        }
    }
}

// Point sampling (GPOINT): adds p0 D u e(u) / (2 rho) at every sample of the
// tile [tlo, thi) whose time lies strictly inside the pulse's support.
template <typename R, int DIR>
__device__ inline void fwd_pair_point(const BallK<R, GPOINT> &b, R qx, R qy, R qz, R nx, R ny, R nz,
                                      const Level &lc, int tlo, int thi, R scale,
                                      typename FwdAcc<R>::T *__restrict__ row) {
    PairG<R> g;
    if (!pair_geometry<R, DIR>(b.x, b.y, b.z, b.w, qx, qy, qz, nx, ny, nz, lc, g)) return;
    const double lo = floor((g.s - (double)b.w) * lc.inv_cdt) + 1.0;
    const double hi = ceil((g.s + (double)b.w) * lc.inv_cdt) - 1.0;
    if (hi < (double)tlo || lo > (double)(thi - 1) || hi < lo) return;
    const int nb = lo < (double)tlo ? tlo : (int)lo;
    const int ne = hi > (double)(thi - 1) ? thi - 1 : (int)hi;
    const R amp = b.p * g.dir * R(0.5) * g.inv_rho * scale;
    const R c = LevelR<R>::cdt(lc);
    typename FwdAcc<R>::T *p = row - tlo + nb;
    int cnt = ne - nb + 1;
    int m = nb;
    if (FwdBlocks<R>::on) {
        const R X2 = b.q0 * c * c;
        const R Y1 = R(-2) * b.q0 * c;
        const R h = ex2(R(2) * X2);
        for (; cnt >= kFwdBlock; cnt -= kFwdBlock, p += kFwdBlock, m += kFwdBlock)
            point_samples<R, kFwdBlock>(p, (R)(g.s - (double)m * lc.cdt), b.q0, c, X2, Y1, h, amp);
        if (cnt & 4) {
            point_samples<R, 4>(p, (R)(g.s - (double)m * lc.cdt), b.q0, c, X2, Y1, h, amp);
            p += 4;
            m += 4;
        }
        if (cnt & 2) {
            point_samples<R, 2>(p, (R)(g.s - (double)m * lc.cdt), b.q0, c, X2, Y1, h, amp);
            p += 2;
            m += 2;
        }
        if (cnt & 1) point_samples<R, 1>(p, (R)(g.s - (double)m * lc.cdt), b.q0, c, X2, Y1, h, amp);
    } else {
        for (; cnt > 0; --cnt, ++p, ++m) {
            const R u = (R)(g.s - (double)m * lc.cdt);
            FwdAcc<R>::add(p, amp * u * ex2(u * u * b.q0));
        }
    }
}

// Adds the pair's bins that fall in the time tile [tlo, thi) to row[n - tlo];
// `scale` multiplies the bin values (the fixed-point quantum's inverse).
template <typename R, int PROF, int DIR>
__device__ inline void fwd_pair(const BallK<R, PROF> &b, R qx, R qy, R qz, R nx, R ny, R nz,
                                const Level &lc, int tlo, int thi, R scale,
                                typename FwdAcc<R>::T *__restrict__ row) {
    PairG<R> g;
    if (!pair_geometry<R, DIR>(b.x, b.y, b.z, b.w, qx, qy, qz, nx, ny, nz, lc, g)) return;
    const double lo = floor((g.s - (double)b.w) * lc.inv_cdt);
    const double hi = floor((g.s + (double)b.w) * lc.inv_cdt);
    if (hi < (double)tlo || lo > (double)(thi - 1)) return;
    const int nb = lo < (double)tlo ? tlo : (int)lo;
    const int ne = hi > (double)(thi - 1) ? thi - 1 : (int)hi;
    const R amp = b.ampk * g.dir * LevelR<R>::inv2cdt(lc) * g.inv_rho * scale;
    const R c = LevelR<R>::cdt(lc);
    // Bins nb..ne use edges nb..ne+1.  Edge lo and edge hi + 1 lie outside the
    // support (shape value: eK for GAUSS, 0 for UNIFORM) and every edge between
    // them inside, so only the inside edges are evaluated and none is clamped.
    const bool first_out = nb == (int)lo;
    const bool last_out = ne == (int)hi;
    typename FwdAcc<R>::T *p = row - tlo + nb;
    int cnt = ne - nb + 1 - (last_out ? 1 : 0);   // bins whose right edge is inside
    if (PROF == GAUSS) {
        // one exponential per edge: a recurrence drifts by ~1e-7 per step, and
        // bin differences amplify that by a / (c dt), up to ~10^2 here
        const R eK = LevelR<R>::eK(lc);
        R prev;
        int m = nb;   // left edge of the next bin
        {
            const R u0 = (R)(g.s - (double)nb * lc.cdt);
            prev = first_out ? eK : ex2(u0 * u0 * b.q0);
        }
        if (FwdBlocks<R>::on) {
            // blocks of kFwdBlock bins, then the remainder as blocks of 4, 2
            // and 1 (a typical support leaves 7): the edge offsets k are
            // constants, q0 (u_m - k c)^2 = X0 + k (X1 + k X2), u_m formed
            // exactly per block
            const R X2 = b.q0 * c * c;
            const R Y1 = R(-2) * b.q0 * c;
            for (; cnt >= kFwdBlock; cnt -= kFwdBlock, p += kFwdBlock, m += kFwdBlock)
                gauss_bins<R, kFwdBlock>(p, (R)(g.s - (double)m * lc.cdt), b.q0, X2, Y1, amp, prev);
            if (cnt & 4) {
                gauss_bins<R, 4>(p, (R)(g.s - (double)m * lc.cdt), b.q0, X2, Y1, amp, prev);
                p += 4;
                m += 4;
            }
            if (cnt & 2) {
                gauss_bins<R, 2>(p, (R)(g.s - (double)m * lc.cdt), b.q0, X2, Y1, amp, prev);
                p += 2;
                m += 2;
            }
            if (cnt & 1) {
                gauss_bins<R, 1>(p, (R)(g.s - (double)m * lc.cdt), b.q0, X2, Y1, amp, prev);
                p += 1;
            }
        } else {
            const R u0 = (R)(g.s - (double)m * lc.cdt);
            R j = R(1);
            // two bins per trip (no register copy of the carried edge value)
            for (; cnt >= 2; cnt -= 2, p += 2, j += R(2)) {
                const R u1 = fma(-j, c, u0);
                const R u2 = u1 - c;
                const R c1 = ex2(u1 * u1 * b.q0);
                const R c2 = ex2(u2 * u2 * b.q0);
                FwdAcc<R>::add(p, amp * (prev - c1));
                FwdAcc<R>::add(p + 1, amp * (c1 - c2));
                prev = c2;
            }
            if (cnt) {
                const R u1 = fma(-j, c, u0);
                const R c1 = ex2(u1 * u1 * b.q0);
                FwdAcc<R>::add(p, amp * (prev - c1));
                prev = c1;
                ++p;
            }
        }
        if (last_out) FwdAcc<R>::add(p, amp * (prev - eK));
    } else {
        R prev;
        int m = nb;
        {
            const R u0 = (R)(g.s - (double)nb * lc.cdt);
            prev = first_out ? R(0) : b.q0 - u0 * u0;
        }
        if (FwdBlocks<R>::on) {
            // (u_m - k c)^2 - (u_m - (k-1) c)^2 = -2 u_m c + (2k - 1) c^2: past
            // the block's first bin the bins are linear in k; remainder as
            // blocks of 4, 2 and 1
            const R B1 = amp * R(2) * c * c;
            for (; cnt >= kFwdBlock; cnt -= kFwdBlock, p += kFwdBlock, m += kFwdBlock)
                uniform_bins<R, kFwdBlock>(p, (R)(g.s - (double)m * lc.cdt), b.q0, c, amp, B1, prev);
            if (cnt & 4) {
                uniform_bins<R, 4>(p, (R)(g.s - (double)m * lc.cdt), b.q0, c, amp, B1, prev);
                p += 4;
                m += 4;
            }
            if (cnt & 2) {
                uniform_bins<R, 2>(p, (R)(g.s - (double)m * lc.cdt), b.q0, c, amp, B1, prev);
                p += 2;
                m += 2;
            }
            if (cnt & 1) {
                uniform_bins<R, 1>(p, (R)(g.s - (double)m * lc.cdt), b.q0, c, amp, B1, prev);
                p += 1;
            }
        } else {
            R u = (R)(g.s - (double)m * lc.cdt);
            for (; cnt >= 2; cnt -= 2, p += 2) {
                const R u1 = u - c;
                u = u1 - c;
                const R c1 = b.q0 - u1 * u1;
                const R c2 = b.q0 - u * u;
                FwdAcc<R>::add(p, amp * (prev - c1));
                FwdAcc<R>::add(p + 1, amp * (c1 - c2));
                prev = c2;
            }
            if (cnt) {
                u -= c;
                const R c1 = b.q0 - u * u;
                FwdAcc<R>::add(p, amp * (prev - c1));
                prev = c1;
                ++p;
            }
        }
        if (last_out) FwdAcc<R>::add(p, amp * prev);
    }
}

template <typename R>
__device__ inline void flush_rows(typename FwdAcc<R>::T *__restrict__ rows, int dg, int TT, int T,
                                  int g, int tile, int D, int f, R *__restrict__ y,
                                  unsigned long long *__restrict__ gacc) {
    using A = typename FwdAcc<R>::T;
    __syncthreads();
    const int tlo = tile * TT;
    const int len = min(TT, T - tlo);
    for (int dl = 0; dl < dg; ++dl) {
        const int d = g * dg + dl;
        if (d >= D) break;
        const int64_t o = ((int64_t)f * D + d) * (int64_t)T + tlo;
        A *row = rows + (int64_t)dl * TT;
        for (int n = threadIdx.x; n < len; n += blockDim.x) {
            const A v = row[n];
            if (v != A(0)) {
                if constexpr (sizeof(A) == sizeof(unsigned long long) && sizeof(R) == sizeof(float))
                    atomicAdd(gacc + o + n, (unsigned long long)v);
                else
                    atomicAdd(y + o + n, (R)v);
                row[n] = A(0);
            }
        }
    }
    __syncthreads();
}

// y = (accumulate ? y : 0) + q * sum, for every sample of the launch (grid.y =
// frame); a flagged frame gets NaN.
// Inside a step (y_ref given) the value written is v = 2 (y - y_ref), and the
// workgroup's sum of (y - y_ref)^2 goes to partial[frame][blockIdx.x]
// (gridDim.x = kLossBlocks); with `clear` each integer sum is zeroed once read.
__global__ void k_fwd_convert(unsigned long long *__restrict__ gacc, int64_t nper,
                              const unsigned *__restrict__ misc, int profile, Level lc,
                              int accumulate, float *__restrict__ y, int clear,
                              const float *__restrict__ y_ref, double *__restrict__ partial) {
    __shared__ double s_part[4];
    const bool bad = misc[kMiscFlags + blockIdx.y] != 0;
    const float inv_scale = 1.0f / fixed_scale(misc + kMiscBound, profile, lc);
    unsigned long long *g = gacc + (int64_t)blockIdx.y * nper;
    float *yf = y + (int64_t)blockIdx.y * nper;
    const float *rf = y_ref ? y_ref + (int64_t)blockIdx.y * nper : nullptr;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nper;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = bad ? __builtin_nanf("") : FwdAcc<float>::value(g[i], inv_scale);
        if (clear) g[i] = 0ull;
        if (rf) {
            const float e = v - rf[i];
            yf[i] = 2.0f * e;
            acc += (double)e * (double)e;
        } else {
            yf[i] = accumulate ? yf[i] + v : v;
        }
    }
    if (rf) {
        const double t = block_sum(acc, s_part);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

template <typename R, int PROF, int DIR>
__global__ __launch_bounds__(512, 4) void k_forward(ArrayP<R> arr, BallsP<R> balls,
                                                    const int64_t *__restrict__ ball_off, int F,
                                                    int G, int dg, int TT, int nt, int bpt,
                                                    Level lc, const unsigned *__restrict__ bound,
                                                    R *__restrict__ y,
                                                    unsigned long long *__restrict__ gacc) {
    using A = typename FwdAcc<R>::T;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    A *rows = reinterpret_cast<A *>(lds_raw);
    __shared__ int64_t s_off[SBP_MAX_FRAMES + 1];
    __shared__ int64_t s_ipre[SBP_MAX_FRAMES + 1];
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int T = lc.T;
    const int64_t CH = (int64_t)nth * bpt;
    const int64_t GT = (int64_t)G * nt;
    const R scale = bound ? (R)fixed_scale(bound, PROF, lc) : R(1);
    for (int i = tid; i <= F; i += nth) s_off[i] = ball_off[i];
    for (int i = tid; i < dg * TT; i += nth) rows[i] = A(0);
    __syncthreads();
    if (tid == 0) {
        s_ipre[0] = 0;
        for (int f = 0; f < F; ++f) {
            const int64_t nb = s_off[f + 1] - s_off[f];
            s_ipre[f + 1] = s_ipre[f] + ((nb + CH - 1) / CH) * GT;
        }
    }
    __syncthreads();
    const int64_t I = s_ipre[F];
    const int64_t i0 = I * (int64_t)blockIdx.x / gridDim.x;
    const int64_t i1 = I * (int64_t)(blockIdx.x + 1) / gridDim.x;
    const int D = arr.D;
    int f = 0, cur_f = -1, cur_gt = -1;
    for (int64_t it = i0; it < i1; ++it) {
        while (it >= s_ipre[f + 1]) ++f;
        const int64_t nch = (s_ipre[f + 1] - s_ipre[f]) / GT;
        const int64_t local = it - s_ipre[f];
        const int gt = __builtin_amdgcn_readfirstlane((int)(local / nch));
        const int64_t ck = local - (int64_t)gt * nch;
        if (f != cur_f || gt != cur_gt) {
            if (cur_f >= 0)
                flush_rows<R>(rows, dg, TT, T, cur_gt / nt, cur_gt % nt, D, cur_f, y, gacc);
            cur_f = f;
            cur_gt = gt;
        }
        const int g = gt / nt;
        const int tlo = (gt - g * nt) * TT;
        const int thi = min(tlo + TT, T);
        const int64_t base = s_off[f] + ck * CH;
        const int64_t end = min(base + CH, s_off[f + 1]);
        for (int jb = 0; jb < bpt; ++jb) {
            const int64_t i = base + (int64_t)jb * nth + tid;
            if (i >= end) break;
            const BallK<R, PROF> b = load_ball<R, PROF>(balls.x[i], balls.y[i], balls.z[i],
                                                        balls.p0[i], balls.a[i], lc);
            if (!b.live) continue;
            for (int dl = 0; dl < dg; ++dl) {
                const int d = __builtin_amdgcn_readfirstlane(g * dg + dl);
                if (d >= D) break;
                if constexpr (PROF == GPOINT)
                    fwd_pair_point<R, DIR>(b, arr.qx[d], arr.qy[d], arr.qz[d], arr.nx[d], arr.ny[d],
                                           arr.nz[d], lc, tlo, thi, scale, rows + (int64_t)dl * TT);
                else
                    fwd_pair<R, PROF, DIR>(b, arr.qx[d], arr.qy[d], arr.qz[d], arr.nx[d], arr.ny[d],
                                           arr.nz[d], lc, tlo, thi, scale, rows + (int64_t)dl * TT);
            }
        }
    }
    if (cur_f >= 0) flush_rows<R>(rows, dg, TT, T, cur_gt / nt, cur_gt % nt, D, cur_f, y, gacc);
}

// ---------------------------------------------------------------------------
// GAUSS bin means in FP32: edge form.
//
// Sample n of a pair is p0 G (psi(u_n) - psi(u_{n+1})) with G = D / (2 rho c
// dt_k), so a transducer's row is the difference of neighbouring entries of
// its edge row W_m = -sum_i p0_i G_i psi_i(u_m), m = 0 .. T:
//     y_n = W_{n+1} - W_n.
// A pair adds one value per edge strictly inside its support,
//     W = p0 a^2 G (e - e_K),  e = 2^(q0 u^2),  e_K = exp(-K^2 / 2),
// which is >= 0 for p0 >= 0.  The values are rounded to the nearest multiple
// of the same quantum as the bin values (|W| <= |p0| a^2 / (2 rho c dt_k),
// below the bound since rho > K a) and summed exactly; the last pass takes the
// differences exactly on the integers.  Per edge this is two multiplies of the
// Gaussian's recurrence (two exp2 per four edges restart it), one FMA, the
// conversion and one LDS add, and one LDS add fewer per pair than bin values.
// When no ball of a wave has p0 < 0 the 64-bit value needs no sign word.  Each
// sample carries two roundings per ball instead of one.
//
// The per-ball constants come from one pass over the cloud (k_fwd_prep),
// which also takes the fixed-point bound and the non-finite flags, so the
// pair loop reads six floats per ball and computes no size-dependent constant.
struct FwdPrepP {
    float *x, *y, *z, *w, *q0, *pa2;
};

constexpr int kPrepBlock = 256;

// w = K a (the support half-width, rounded from the FP64 product),
// q0 = -log2(e) / (2 a^2), pa2 = p0 a^2; a ball that adds nothing (a <= 0,
// p0 = 0) or has a non-finite parameter gets pa2 = 0, and the latter flags
// its frame.  misc[kMiscBound] receives max |p0| a over the finite live balls
// (zeroed before the launch).
__global__ __launch_bounds__(kPrepBlock) void k_fwd_prep(BallsP<float> balls,
                                                         const int64_t *__restrict__ ball_off,
                                                         int F, Level lc, unsigned *misc,
                                                         FwdPrepP out) {
    __shared__ float s_red[kPrepBlock / 64];
    __shared__ int64_t s_off[SBP_MAX_FRAMES + 1];
    for (int i = threadIdx.x; i <= F; i += blockDim.x) s_off[i] = ball_off[i];
    __syncthreads();
    const int64_t count = s_off[F];
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float x = balls.x[i], y = balls.y[i], z = balls.z[i];
        const float p = balls.p0[i];
        const float ar = balls.a[i];
        const float a = lc.a_softplus ? softplus_dev(ar) : ar;
        const float t = fabsf(p) * a;
        float w = 0.0f, q0 = 0.0f, pa2 = 0.0f;
        if (!ball_finite(x, y, z, p, ar) || !isfinite(t) || !isfinite(p * a * a)) {
            atomicOr(misc + kMiscFlags + frame_of(s_off, F, i), 1u);
        } else if (a > 0.0f) {
            m = fmaxf(m, t);
            w = (float)(lc.K_d * (double)a);
            q0 = -1.4426950408889634f / (2.0f * a * a);
            pa2 = p * a * a;
        }
        out.x[i] = x;
        out.y[i] = y;
        out.z[i] = z;
        out.w[i] = w;
        out.q0[i] = q0;
        out.pa2[i] = pa2;
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, s_red[w]);
        atomicMax(misc + kMiscBound, __float_as_uint(m));
    }
}

// Adds an edge value to an LDS row entry: vh is the scaled value plus 1/2, so
// its nearest integer is floor(vh).  NN: the value is >= 0 but for rounding
// just inside the support edge; v_cvt_u32_f32 truncates and clamps a negative
// input to 0, so the integer is floor(vh) >= 0 and the high word is 0.
template <bool NN>
__device__ inline void edge_add(unsigned long long *p, float vh) {
    if (NN) {
        unsigned iv;
        asm("v_cvt_u32_f32 %0, %1" : "=v"(iv) : "v"(vh));
        atomicAdd(p, (unsigned long long)iv);
    } else {
        int iv;
        asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(iv) : "v"(vh));
        atomicAdd(p, (unsigned long long)(long long)iv);
    }
}

// The block a lane starts from when it adds a pair's nb four-entry blocks in
// a rotated order (block j, j + 1, ..., wrapping to 0, ..., j - 1) starting at
// row entry m.  A wave's 64-bit LDS adds run faster when its lanes' entries
// spread over the residues modulo 16 (random entries: about 6.2 adds per clock
// per CU; four lanes on each residue: 9.3); a lane's entry at step s is
// m + 4 j + s until it wraps, so the lanes whose m has the same residue modulo
// 4 take, in lane order, the four starts m + 4 j that cover that residue's
// four classes modulo 16 (about 7.5 per clock with the wraps).  Lanes that are
// not active take no part.  The sums are integers, so the order changes no
// result.
__device__ inline int rotated_block(int m, int nb) {
    const unsigned cs = (unsigned)m & 3u;
    unsigned long long mine = 0;
#pragma unroll
    for (unsigned v = 0; v < 4; ++v) {
        const unsigned long long b = __ballot(cs == v);
        if (cs == v) mine = b;
    }
    const unsigned rank = (unsigned)__popcll(mine & ((1ull << __lane_id()) - 1ull));
    const int j = (int)(((cs + 4u * (rank & 3u) - (unsigned)m) & 15u) >> 2);
    return j < nb ? j : 0;
}

// N consecutive inside edges from offset u0 (edge k at u0 - k c), adding
// namp (e_k - e_K): the Gaussian e_k = 2^(q0 (u0 - k c)^2) by the two-multiply
// recurrence e_{k+1} = e_k g_k, g_{k+1} = g_k h restarted here, with
// e_0 = 2^(q0 u0^2), g_0 = 2^(q0 c (c - 2 u0)) = 2^(Y1 u0 + X2), h = 2^(2 X2).
template <bool NN, int N>
__device__ inline void gz_edges(unsigned long long *p, float u0, float q0, float X2, float Y1,
                                float h, float namp, float nampKh) {
    float e = __builtin_amdgcn_exp2f(q0 * u0 * u0);
    float g = __builtin_amdgcn_exp2f(fmaf(Y1, u0, X2));
#pragma unroll
    for (int k = 0; k < N; ++k) {
        edge_add<NN>(p + k, fmaf(namp, e, nampKh));
        if (k + 1 < N) {
            e *= g;
            g *= h;
        }
    }
}

// Adds the pair's inside edges that fall in the tile [tlo, thi) to
// row[m - tlo]; `scale` is the inverse of the fixed-point quantum.  The first
// edge's offset is formed exactly (FP64 difference, FP32 result), the later
// restarts' offsets by one FP32 fma from it; the recurrence restarts every
// four edges (its rounding grows with the run: about 1e-6 of a sample at 40
// edges per pair, several times that with eight).
template <int DIR, bool NN>
__device__ inline void gz_pair(float bx, float by, float bz, float w, float q0, float pa2,
                               float qx, float qy, float qz, float nx, float ny, float nz,
                               const Level &lc, int tlo, int thi, float scale,
                               unsigned long long *__restrict__ row) {
    PairG<float> g;
    if (!pair_geometry<float, DIR>(bx, by, bz, w, qx, qy, qz, nx, ny, nz, lc, g)) return;
    // edges strictly inside the support: floor((s - w) / c dt) + 1 .. floor((s + w) / c dt)
    const double lo = fmax(floor((g.s - (double)w) * lc.inv_cdt) + 1.0, (double)tlo);
    const double hi = fmin(floor((g.s + (double)w) * lc.inv_cdt), (double)(thi - 1));
    if (!(lo <= hi)) return;
    const int m = (int)lo;
    int cnt = (int)hi - m + 1;
    const float namp = pa2 * g.dir * lc.inv2cdt * g.inv_rho * scale;
    const float nampKh = fmaf(-namp, lc.eK, 0.5f);
    const float c = lc.cdt_f;
    const float X2 = q0 * c * c;
    const float Y1 = -2.0f * q0 * c;
    const float h = __builtin_amdgcn_exp2f(2.0f * X2);
    const float u0 = (float)(g.s - (double)m * lc.cdt);
    unsigned long long *p = row - tlo + m;
    // the whole four-edge blocks in a rotated order (rotated_block)
    const int nb = cnt >> 2;
    const int j = rotated_block(m, nb);
    if (nb > 0) {
        unsigned long long *const p0 = p + 4 * j, *const pend = p + 4 * nb;
        unsigned long long *q = p0;
        float kf = (float)(4 * j);
        do {
            gz_edges<NN, 4>(q, fmaf(-kf, c, u0), q0, X2, Y1, h, namp, nampKh);
            q += 4;
            kf += 4.0f;
            if (q == pend) {
                q = p;
                kf = 0.0f;
            }
        } while (q != p0);
    }
    p += 4 * nb;
    float k0 = (float)(4 * nb);
    if (cnt & 2) {
        gz_edges<NN, 2>(p, fmaf(-k0, c, u0), q0, X2, Y1, h, namp, nampKh);
        p += 2;
        k0 += 2.0f;
    }
    if (cnt & 1) gz_edges<NN, 1>(p, fmaf(-k0, c, u0), q0, X2, Y1, h, namp, nampKh);
}

// The edge-form forward: work items and flushes as in k_forward, over edge
// rows of T + 1 entries.
template <int DIR>
__global__ __launch_bounds__(512, 4) void k_forward_gz(ArrayP<float> arr, FwdPrepP pb,
                                                       const int64_t *__restrict__ ball_off, int F,
                                                       int G, int dg, int TT, int nt, int bpt,
                                                       Level lc, const unsigned *__restrict__ bound,
                                                       unsigned long long *__restrict__ gacc) {
    using A = unsigned long long;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    A *rows = reinterpret_cast<A *>(lds_raw);
    __shared__ int64_t s_off[SBP_MAX_FRAMES + 1];
    __shared__ int64_t s_ipre[SBP_MAX_FRAMES + 1];
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int TE = lc.T + 1;
    const int64_t CH = (int64_t)nth * bpt;
    const int64_t GT = (int64_t)G * nt;
    const float scale = fixed_scale(bound, GAUSS, lc);
    for (int i = tid; i <= F; i += nth) s_off[i] = ball_off[i];
    for (int i = tid; i < dg * TT; i += nth) rows[i] = A(0);
    __syncthreads();
    if (tid == 0) {
        s_ipre[0] = 0;
        for (int f = 0; f < F; ++f) {
            const int64_t nb = s_off[f + 1] - s_off[f];
            s_ipre[f + 1] = s_ipre[f] + ((nb + CH - 1) / CH) * GT;
        }
    }
    __syncthreads();
    const int64_t I = s_ipre[F];
    const int64_t i0 = I * (int64_t)blockIdx.x / gridDim.x;
    const int64_t i1 = I * (int64_t)(blockIdx.x + 1) / gridDim.x;
    const int D = arr.D;
    int f = 0, cur_f = -1, cur_gt = -1;
    for (int64_t it = i0; it < i1; ++it) {
        while (it >= s_ipre[f + 1]) ++f;
        const int64_t nch = (s_ipre[f + 1] - s_ipre[f]) / GT;
        const int64_t local = it - s_ipre[f];
        const int gt = __builtin_amdgcn_readfirstlane((int)(local / nch));
        const int64_t ck = local - (int64_t)gt * nch;
        if (f != cur_f || gt != cur_gt) {
            if (cur_f >= 0)
                flush_rows<float>(rows, dg, TT, TE, cur_gt / nt, cur_gt % nt, D, cur_f, nullptr, gacc);
            cur_f = f;
            cur_gt = gt;
        }
        const int g = gt / nt;
        const int tlo = (gt - g * nt) * TT;
        const int thi = min(tlo + TT, TE);
        const int64_t base = s_off[f] + ck * CH;
        const int64_t end = min(base + CH, s_off[f + 1]);
        // the next ball's constants load while this one's pairs are added
        float nbx = 0.0f, nby = 0.0f, nbz = 0.0f, nw = 0.0f, nq0 = 0.0f, npa2 = 0.0f;
        {
            const int64_t i = base + tid;
            if (i < end) {
                nbx = pb.x[i];
                nby = pb.y[i];
                nbz = pb.z[i];
                nw = pb.w[i];
                nq0 = pb.q0[i];
                npa2 = pb.pa2[i];
            }
        }
        for (int jb = 0; jb < bpt; ++jb) {
            const float bx = nbx, by = nby, bz = nbz, w = nw, q0 = nq0, pa2 = npa2;
            const int64_t i = base + (int64_t)(jb + 1) * nth + tid;
            nbx = nby = nbz = nw = nq0 = npa2 = 0.0f;
            if (jb + 1 < bpt && i < end) {
                nbx = pb.x[i];
                nby = pb.y[i];
                nbz = pb.z[i];
                nw = pb.w[i];
                nq0 = pb.q0[i];
                npa2 = pb.pa2[i];
            }
            const bool nn = __all(pa2 >= 0.0f);   // wave-uniform
            if (pa2 == 0.0f) continue;
            for (int dl = 0; dl < dg; ++dl) {
                const int d = __builtin_amdgcn_readfirstlane(g * dg + dl);
                if (d >= D) break;
                A *row = rows + (int64_t)dl * TT;
                if (nn)
                    gz_pair<DIR, true>(bx, by, bz, w, q0, pa2, arr.qx[d], arr.qy[d], arr.qz[d],
                                       arr.nx[d], arr.ny[d], arr.nz[d], lc, tlo, thi, scale, row);
                else
                    gz_pair<DIR, false>(bx, by, bz, w, q0, pa2, arr.qx[d], arr.qy[d], arr.qz[d],
                                        arr.nx[d], arr.ny[d], arr.nz[d], lc, tlo, thi, scale, row);
            }
        }
    }
    if (cur_f >= 0) flush_rows<float>(rows, dg, TT, TE, cur_gt / nt, cur_gt % nt, D, cur_f, nullptr, gacc);
}

// y[f][d][n] = (accumulate ? y : 0) + q (W[f][d][n+1] - W[f][d][n]); a flagged
// frame gets NaN.  grid.y = frame, workgroups stride over the transducers.
// Inside a step (y_ref given) the value written is v = 2 (y - y_ref) and the
// workgroup's sum of (y - y_ref)^2 goes to partial[frame][blockIdx.x]
// (gridDim.x = kLossBlocks); with `clear` a row's integer sums are zeroed once
// the whole workgroup has read them (each edge feeds two samples).
__global__ void k_fwd_convert_edges(unsigned long long *__restrict__ gacc, int D, int T,
                                    const unsigned *__restrict__ misc, Level lc, int accumulate,
                                    float *__restrict__ y, int clear,
                                    const float *__restrict__ y_ref, double *__restrict__ partial) {
    __shared__ double s_part[4];
    const bool bad = misc[kMiscFlags + blockIdx.y] != 0;
    const float inv_scale = 1.0f / fixed_scale(misc + kMiscBound, GAUSS, lc);
    double acc = 0.0;
    for (int d = blockIdx.x; d < D; d += gridDim.x) {
        const int64_t r = (int64_t)blockIdx.y * D + d;
        unsigned long long *w = gacc + r * (T + 1);
        float *yr = y + r * T;
        const float *rr = y_ref ? y_ref + r * T : nullptr;
        for (int n = threadIdx.x; n < T; n += blockDim.x) {
            const long long diff = (long long)(w[n + 1] - w[n]);
            const float v = bad ? __builtin_nanf("") : (float)((double)diff * (double)inv_scale);
            if (rr) {
                const float e = v - rr[n];
                yr[n] = 2.0f * e;
                acc += (double)e * (double)e;
            } else {
                yr[n] = accumulate ? yr[n] + v : v;
            }
        }
        if (clear) {
            __syncthreads();
            for (int n = threadIdx.x; n <= T; n += blockDim.x) w[n] = 0ull;
        }
    }
    if (y_ref) {
        const double t = block_sum(acc, s_part);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

template <int DIR>
static int run_forward_gz(Ctx *c, const ArrayP<float> &arr, const FwdPrepP &pb,
                          const int64_t *ball_off, int F, int64_t B_cap, const Level &lc,
                          const unsigned *bound, unsigned long long *gacc, hipStream_t st) {
    using A = unsigned long long;
    auto kern = k_forward_gz<DIR>;
    const size_t reserve = 2 * (SBP_MAX_FRAMES + 1) * sizeof(int64_t) + 256;
    const size_t avail = c->lds_max > reserve ? c->lds_max - reserve : 0;
    const int TE = lc.T + 1;
    int dg = c->tuning.fwd_dets;
    if (dg > arr.D) dg = arr.D;
    // edge tile: the whole row if the dg rows fit, else the longest that does
    int64_t TT = (int64_t)(avail / ((size_t)dg * sizeof(A)));
    if (TT > TE) TT = TE;
    if (TT < TE && TT < 64) return fail(SBP_E_DOMAIN, "LDS too small for %d rows", dg);
    if (c->tuning.fwd_tile > 0 && TT > c->tuning.fwd_tile) TT = c->tuning.fwd_tile;
    const int nt = (int)((TE + TT - 1) / TT);
    const int G = (arr.D + dg - 1) / dg;
    int block = c->tuning.fwd_block;
    int bpt = c->tuning.fwd_bpt;
    {
        const int64_t want = 2 * (int64_t)c->num_cus * (1024 / block > 0 ? 1024 / block : 1);
        auto items = [&](int blk, int b) {
            const int64_t ch = (int64_t)blk * b;
            return ((B_cap + ch - 1) / ch + F) * (int64_t)G * nt;
        };
        while (bpt > 1 && items(block, bpt) < want) --bpt;
        while (block > 128 && items(block, bpt) < want) block /= 2;
    }
    const size_t lds = (size_t)dg * (size_t)TT * sizeof(A);
    SBP_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    int grid = c->tuning.fwd_grid;
    if (grid <= 0) {
        int per_cu = 0;
        SBP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, block, lds));
        if (per_cu < 1) per_cu = 1;
        grid = per_cu * c->num_cus;
    }
    const int64_t CH = (int64_t)block * bpt;
    const int64_t max_items = ((B_cap + CH - 1) / CH + F) * (int64_t)G * nt;
    if (grid > max_items) grid = (int)max_items;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, st, arr, pb, ball_off, F, G, dg,
                       (int)TT, nt, bpt, lc, bound, gacc);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

template <typename R, int PROF, int DIR>
static int run_forward(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls,
                       const int64_t *ball_off, int F, int64_t B_cap, const Level &lc,
                       const unsigned *bound, R *y, unsigned long long *gacc, hipStream_t st) {
    using A = typename FwdAcc<R>::T;
    auto kern = k_forward<R, PROF, DIR>;
    const size_t reserve = 2 * (SBP_MAX_FRAMES + 1) * sizeof(int64_t) + 256;
    const size_t avail = c->lds_max > reserve ? c->lds_max - reserve : 0;
    int dg = c->tuning.fwd_dets;
    if (dg > arr.D) dg = arr.D;
    // time tile: the whole record if the dg rows fit, else the longest that does
    int64_t TT = (int64_t)(avail / ((size_t)dg * sizeof(A)));
    if (TT > lc.T) TT = lc.T;
    if (TT < lc.T && TT < 64) return fail(SBP_E_DOMAIN, "LDS too small for %d rows", dg);
    if (c->tuning.fwd_tile > 0 && TT > c->tuning.fwd_tile) TT = c->tuning.fwd_tile;
    const int nt = (int)((lc.T + TT - 1) / TT);
    const int G = (arr.D + dg - 1) / dg;
    // small clouds: fewer balls per item (bpt, then the block) until the chip
    // has about two work items per resident workgroup
    int block = c->tuning.fwd_block;
    int bpt = c->tuning.fwd_bpt;
    {
        const int64_t want = 2 * (int64_t)c->num_cus * (1024 / block > 0 ? 1024 / block : 1);
        auto items = [&](int blk, int b) {
            const int64_t ch = (int64_t)blk * b;
            return ((B_cap + ch - 1) / ch + F) * (int64_t)G * nt;
        };
        while (bpt > 1 && items(block, bpt) < want) --bpt;
        while (block > 128 && items(block, bpt) < want) block /= 2;
    }
    const size_t lds = (size_t)dg * (size_t)TT * sizeof(A);
    SBP_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    int grid = c->tuning.fwd_grid;
    if (grid <= 0) {
        int per_cu = 0;
        SBP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, block, lds));
        if (per_cu < 1) per_cu = 1;
        grid = per_cu * c->num_cus;
    }
    const int64_t CH = (int64_t)block * bpt;
    const int64_t max_items = ((B_cap + CH - 1) / CH + F) * (int64_t)G * nt;
    if (grid > max_items) grid = (int)max_items;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, st, arr, balls, ball_off, F, G, dg,
                       (int)TT, nt, bpt, lc, bound, y, gacc);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// FP32: [per-sample integer sums, T + 1 per row][six per-ball constant arrays]
size_t forward_ws_bytes(int F, int D, int T, int64_t B_cap, size_t elem) {
    if (elem != sizeof(float)) return 0;
    return up256((size_t)F * (size_t)D * (size_t)(T + 1) * sizeof(unsigned long long)) +
           6 * up256((size_t)B_cap * sizeof(float));
}

template <typename R>
int launch_forward(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls, const int64_t *ball_off,
                   int F, int64_t B_cap, const sbp_model *m, R *y, int accumulate,
                   unsigned *misc, void *ws, size_t ws_bytes, hipStream_t st,
                   const FwdStep *step) {
    const Level lc = make_level(m);
    const FwdStep none{};
    const FwdStep &sp = step ? *step : none;
    if (sp.y_ref && (sizeof(R) != sizeof(float) || !sp.partial))
        return fail(SBP_E_ARG, "the fused residual needs the FP32 forward and a partial buffer");
    if (sp.sums_only && (sizeof(R) != sizeof(float) || profile_code(m) != GAUSS || sp.y_ref || accumulate))
        return fail(SBP_E_ARG, "edge sums alone need the FP32 GAUSS bin forward");
    const int64_t nper = (int64_t)arr.D * m->T;
    const int64_t ns = (int64_t)F * nper;
    if (B_cap == 0 || sizeof(R) != sizeof(float)) {
        if (!accumulate) {
            int rc = launch_fill<R>(y, ns, R(0), st);
            if (rc) return rc;
        }
        if (B_cap == 0) return SBP_OK;
    }
    if (!misc) return fail(SBP_E_ARG, "forward needs the context's device words");
    // bound word and frame flags start at zero
    int rc = SBP_OK;
    if (!sp.ws_clean && (rc = launch_fill<int32_t>((int32_t *)misc, kMiscFlags + SBP_MAX_FRAMES, 0, st)))
        return rc;
    int64_t nbb = (B_cap + 255) / 256;
    if (nbb > 1024) nbb = 1024;
    unsigned long long *gacc = nullptr;
    const unsigned *bound = nullptr;
    if constexpr (sizeof(R) == sizeof(float)) {
      if (profile_code(m) == GAUSS) {
        if (!ws || ws_bytes < forward_ws_bytes(F, arr.D, m->T, B_cap, sizeof(float)))
            return fail(SBP_E_NOMEM, "forward workspace too small");
        gacc = (unsigned long long *)ws;
        const int64_t ne = (int64_t)F * arr.D * (m->T + 1);
        char *pp = (char *)ws + up256((size_t)ne * sizeof(unsigned long long));
        const size_t pb_bytes = up256((size_t)B_cap * sizeof(float));
        FwdPrepP pb;
        float **fields[6] = {&pb.x, &pb.y, &pb.z, &pb.w, &pb.q0, &pb.pa2};
        for (int k = 0; k < 6; ++k) *fields[k] = (float *)(pp + k * pb_bytes);
        if (!sp.ws_clean && (rc = launch_fill<uint64_t>((uint64_t *)gacc, ne, 0, st))) return rc;
        hipLaunchKernelGGL(k_fwd_prep, dim3((int)nbb), dim3(kPrepBlock), 0, st,
                           BallsP<float>{(float *)balls.x, (float *)balls.y, (float *)balls.z,
                                         (float *)balls.p0, (float *)balls.a},
                           ball_off, F, lc, misc, pb);
        SBP_HIP(hipGetLastError());
        bound = misc + kMiscBound;
        const ArrayP<float> af{(const float *)arr.qx, (const float *)arr.qy, (const float *)arr.qz,
                               (const float *)arr.nx, (const float *)arr.ny, (const float *)arr.nz,
                               arr.D};
        if (m->directivity == SBP_DIR_COS)
            rc = run_forward_gz<COS>(c, af, pb, ball_off, F, B_cap, lc, bound, gacc, st);
        else
            rc = run_forward_gz<OMNI>(c, af, pb, ball_off, F, B_cap, lc, bound, gacc, st);
        if (rc) return rc;
        if (sp.sums_only) return SBP_OK;
        int nbx = sp.y_ref ? kLossBlocks : (arr.D < 1024 ? arr.D : 1024);
        hipLaunchKernelGGL(k_fwd_convert_edges, dim3(nbx, F), dim3(256), 0, st, gacc, arr.D, m->T,
                           (const unsigned *)misc, lc, accumulate, (float *)y,
                           (int)sp.clear_after, sp.y_ref, sp.partial);
        SBP_HIP(hipGetLastError());
        return SBP_OK;
      }
    }
    if (sizeof(R) == sizeof(float)) {
        if (!ws || ws_bytes < (size_t)ns * sizeof(unsigned long long))
            return fail(SBP_E_NOMEM, "forward workspace too small");
        gacc = (unsigned long long *)ws;
        if (!sp.ws_clean && (rc = launch_fill<uint64_t>((uint64_t *)gacc, ns, 0, st))) return rc;
        hipLaunchKernelGGL(k_amp_bound, dim3((int)nbb), dim3(256), 0, st,
                           BallsP<float>{(float *)balls.x, (float *)balls.y, (float *)balls.z,
                                         (float *)balls.p0, (float *)balls.a},
                           ball_off, F, m->a_softplus, (int)(profile_code(m) == GPOINT), misc);
        SBP_HIP(hipGetLastError());
        bound = misc + kMiscBound;
    } else {
        hipLaunchKernelGGL(k_nonfinite_flags, dim3((int)nbb), dim3(256), 0, st,
                           BallsP<double>{(double *)balls.x, (double *)balls.y, (double *)balls.z,
                                          (double *)balls.p0, (double *)balls.a},
                           ball_off, F, misc);
        SBP_HIP(hipGetLastError());
    }
    if (profile_code(m) == GPOINT) {
        if (m->directivity == SBP_DIR_COS)
            rc = run_forward<R, GPOINT, COS>(c, arr, balls, ball_off, F, B_cap, lc, bound, y, gacc, st);
        else
            rc = run_forward<R, GPOINT, OMNI>(c, arr, balls, ball_off, F, B_cap, lc, bound, y, gacc, st);
    } else if (m->profile == SBP_PROFILE_GAUSS) {
        if constexpr (sizeof(R) == sizeof(double)) {
            if (m->directivity == SBP_DIR_COS)
                rc = run_forward<R, GAUSS, COS>(c, arr, balls, ball_off, F, B_cap, lc, bound, y, gacc, st);
            else
                rc = run_forward<R, GAUSS, OMNI>(c, arr, balls, ball_off, F, B_cap, lc, bound, y, gacc, st);
        }
    } else {
        if (m->directivity == SBP_DIR_COS)
            rc = run_forward<R, UNIFORM, COS>(c, arr, balls, ball_off, F, B_cap, lc, bound, y, gacc, st);
        else
            rc = run_forward<R, UNIFORM, OMNI>(c, arr, balls, ball_off, F, B_cap, lc, bound, y, gacc, st);
    }
    if (rc) return rc;
    int64_t nb = (nper + 255) / 256;
    if (nb > 4096 / F) nb = 4096 / F > 0 ? 4096 / F : 1;
    if (!gacc) {
        hipLaunchKernelGGL(k_poison_frames, dim3((int)nb, F), dim3(256), 0, st, (const unsigned *)misc,
                           nper, (double *)y);
        SBP_HIP(hipGetLastError());
        return SBP_OK;
    }
    if (sp.y_ref) nb = kLossBlocks;
    hipLaunchKernelGGL(k_fwd_convert, dim3((int)nb, F), dim3(256), 0, st, gacc, nper,
                       (const unsigned *)misc, profile_code(m), lc, accumulate, (float *)y,
                       (int)sp.clear_after, sp.y_ref, sp.partial);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

template int launch_forward<float>(Ctx *, const ArrayP<float> &, const BallsP<float> &,
                                   const int64_t *, int, int64_t, const sbp_model *, float *, int,
                                   unsigned *, void *, size_t, hipStream_t, const FwdStep *);
template int launch_forward<double>(Ctx *, const ArrayP<double> &, const BallsP<double> &,
                                    const int64_t *, int, int64_t, const sbp_model *, double *,
                                    int, unsigned *, void *, size_t, hipStream_t, const FwdStep *);

}  // namespace sbp
