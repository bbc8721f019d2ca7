// Adjoint (vector-Jacobian product) of the forward model on gfx950, and the
// p0-only variant that zero-gradient filtering (section 4.2) runs.
//
// Gather form, no atomics: a lane owns up to four balls and keeps their five
// gradient sums in registers while the workgroup streams every transducer's
// cotangent row through LDS, `ds` rows per pass.  Rows are staged pre-
// differenced, w_m = v_m - v_{m-1} (v_{-1} = v_T = 0), so that by summation by
// parts
//     sum_n v_n (h(u_n) - h(u_{n+1})) = sum_m h(u_m) w_m
// for any edge function h; one LDS read per support edge then serves the sums
// of w psi(u), w psi'(u) and w d psi / d a (psi, psi' = u fhat(u) and
// d psi / d a are written out per profile in adj_pair), from which the pair's
// gradients follow in closed form:
//     G = D / (2 rho c dt),  dL/dp0 = G S0,  dL/da = p0 G S2,
//     dL/dr = p0 G (S1 - S0 / rho) e_hat + p0 S0 / (2 rho c dt) (n_hat - D e_hat) / rho
// (the last term only for COS directivity and D > 0).
#include "adjoint_pair.hpp"
#include "sbp_internal.hpp"

namespace sbp {

constexpr int kMaxBpt = 3;

// Transducer data is read-only for the whole launch and indexed by a
// wave-uniform value: read it through the scalar cache.
template <typename R> __device__ __forceinline__ R ld_uniform(const R *p) {
    return *(const __attribute__((address_space(4))) R *)p;
}

// Stages edges [tlo, thi) of the nd cotangent rows d0.. into LDS rows of
// stride TS (a multiple of four): w_m = vscale (v_m - v_{m-1}) for bin means
// (v is zero outside [0, T)), w_m = vscale v_m for point samples.  FP32: a
// thread takes four consecutive edges at a time (one 16-byte load, one
// 16-byte LDS store) and issues the loads of kStageU such quads before it uses
// any, so a pass pays the global latency a few times rather than once per
// edge; the two quads at the record's ends load separately (one lane per row,
// loads ahead of use), and the tail of a tile or of a record that is not a
// multiple of four, and rows that are not 16-byte aligned, go edge by edge.
// The values are the same either way.
//
// kStageU, the quads in flight per thread: four covers a 4096-sample row in
// one round with 256 threads; the point-sampled OMNI and the UNIFORM / COS
// all-gradient kernels take three, which keeps them free of register spills
// at four waves per SIMD.
template <int PROF, int DIR, bool FULL> struct StageDepth {
    static constexpr int v = (FULL && ((PROF == GPOINT && DIR == OMNI) || (PROF == UNIFORM && DIR == COS))) ? 3 : 4;
};

template <typename R, bool DIFF>
__device__ inline R stage_edge(const R *__restrict__ vr, int m, int T, R vscale) {
    const R cur = m < T ? vr[m] : R(0);
    if (!DIFF) return vscale * cur;
    const R prv = m > 0 ? vr[m - 1] : R(0);
    return vscale * (cur - prv);
}

template <typename R, bool DIFF, int kStageU>
__device__ inline void stage_rows(const R *__restrict__ vf, int d0, int nd, int T, int tlo, int thi,
                                  R vscale, R *rows, int TS) {
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    if constexpr (sizeof(R) != sizeof(float)) {
        for (int dl = 0; dl < nd; ++dl) {
            const R *vr = vf + (int64_t)(d0 + dl) * T;
            R *wr = rows + (int64_t)dl * TS;
            for (int m = tlo + tid; m < thi; m += nth) wr[m - tlo] = stage_edge<R, DIFF>(vr, m, T, vscale);
        }
    } else {
        const int nq = (thi - tlo + 3) >> 2;
        for (int dl = 0; dl < nd; ++dl) {
            const float *vr = vf + (int64_t)(d0 + dl) * T;
            float *wr = rows + (int64_t)dl * TS;
            const bool vec = (reinterpret_cast<uintptr_t>(vr + tlo) & 15) == 0;
            for (int q0 = tid; q0 < nq; q0 += nth * kStageU) {
                float4 cv[kStageU];
                float pv[kStageU];
#pragma unroll
                for (int u = 0; u < kStageU; ++u) {
                    const int q = q0 + u * nth;
                    const int m = tlo + 4 * q;
                    if (vec && q < nq && m >= 1 && m + 4 <= T && m + 4 <= thi) {
                        cv[u] = *reinterpret_cast<const float4 *>(vr + m);
                        pv[u] = DIFF ? vr[m - 1] : 0.0f;
                    }
                }
#pragma unroll
                for (int u = 0; u < kStageU; ++u) {
                    const int q = q0 + u * nth;
                    const int m = tlo + 4 * q;
                    if (q >= nq) continue;
                    if (vec && m >= 1 && m + 4 <= T && m + 4 <= thi) {
                        float4 w;
                        if (DIFF) {
                            w.x = vscale * (cv[u].x - pv[u]);
                            w.y = vscale * (cv[u].y - cv[u].x);
                            w.z = vscale * (cv[u].z - cv[u].y);
                            w.w = vscale * (cv[u].w - cv[u].z);
                        } else {
                            w.x = vscale * cv[u].x;
                            w.y = vscale * cv[u].y;
                            w.z = vscale * cv[u].z;
                            w.w = vscale * cv[u].w;
                        }
                        *reinterpret_cast<float4 *>(wr + 4 * q) = w;
                    } else if (!(vec && (T & 3) == 0 && (m == 0 || m == T))) {
                        for (int k = 0; k < 4 && m + k < thi; ++k)
                            wr[m + k - tlo] = stage_edge<float, DIFF>(vr, m + k, T, vscale);
                    }
                }
            }
        }
        // The two end quads of aligned rows whose length is a multiple of
        // four, lane 0 of wave dl for row dl (addresses wave-uniform): edges
        // 0..3 (v_{-1} = 0) and edge T (v_T = 0), all loads ahead of use.
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int nwave = (nth + 63) >> 6;
        for (int dl = wave; dl < nd; dl += nwave) {
            if ((tid & 63) != 0) continue;
            const float *vr = vf + (int64_t)(d0 + dl) * T;
            float *wr = rows + (int64_t)dl * TS;
            if ((reinterpret_cast<uintptr_t>(vr + tlo) & 15) == 0 && (T & 3) == 0) {
                const bool head = tlo == 0;
                const bool tail = thi == T + 1;
                float4 h = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                float pt = 0.0f;
                if (head) h = *reinterpret_cast<const float4 *>(vr);
                if (tail && DIFF) pt = vr[T - 1];
                if (head) {
                    float4 w;
                    w.x = vscale * h.x;
                    w.y = DIFF ? vscale * (h.y - h.x) : vscale * h.y;
                    w.z = DIFF ? vscale * (h.z - h.y) : vscale * h.z;
                    w.w = DIFF ? vscale * (h.w - h.z) : vscale * h.w;
                    *reinterpret_cast<float4 *>(wr) = w;
                }
                if (tail) wr[T - tlo] = DIFF ? vscale * (0.0f - pt) : vscale * 0.0f;
            }
        }
    }
}

// Row stride of the staged tiles: the tile length rounded up to four floats.
__host__ __device__ inline int adj_row_stride(int TT) { return (TT + 3) & ~3; }

// Stages the nd whole rows d0.. of frame f from the forward's edge sums
// (AdjSrc): v_n = 2 (y_n - y_ref_n) with y_n = (W_{n+1} - W_n) q as the
// conversion forms it (NaN in a flagged frame) into vrows (stride T), then
// w_m = vscale (v_m - v_{m-1}) for m = 0..T into rows (stride TS).  A wave
// takes a row at a time, lane l its samples n = l, l + 64, ..., eight at a
// time with all their loads issued together (one round trip for 512
// samples); `first` (the frame's first ball chunk): the wave also
// writes v to y_work and the row's sum of (y - y_ref)^2 in FP64 (each lane in
// sample order, then a fixed tree), so the loss does not depend on the
// launch shape.
__device__ inline void stage_rows_from_sums(const AdjSrc &src, int f, int D, int d0, int nd, int T,
                                            const Level &lc, float vscale, float *rows, int TS,
                                            float *vrows, bool first) {
    constexpr int kU = 8;   // samples per lane whose loads are in flight together
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int lane = tid & 63;
    const bool bad = src.misc[kMiscFlags + f] != 0;
    const float inv_scale = 1.0f / fixed_scale(src.misc + kMiscBound, GAUSS, lc);
    for (int dl = tid >> 6; dl < nd; dl += (nth + 63) >> 6) {
        const int64_t r = (int64_t)f * D + d0 + dl;
        const unsigned long long *w = src.gacc + r * (T + 1);
        const float *rr = src.y_ref + r * T;
        float *yw = src.y_work + r * T;
        float *vr = vrows + (int64_t)dl * T;
        double acc = 0.0;
        for (int n0 = lane; n0 < T; n0 += 64 * kU) {
            unsigned long long wa[kU], wb[kU];
            float rv[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int n = n0 + 64 * u;
                if (n < T) {
                    wa[u] = w[n];
                    wb[u] = w[n + 1];
                    rv[u] = rr[n];
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int n = n0 + 64 * u;
                if (n < T) {
                    const long long diff = (long long)(wb[u] - wa[u]);
                    const float y = bad ? __builtin_nanf("") : (float)((double)diff * (double)inv_scale);
                    const float e = y - rv[u];
                    vr[n] = 2.0f * e;
                    if (first) {
                        yw[n] = 2.0f * e;
                        acc += (double)e * (double)e;
                    }
                }
            }
        }
        if (first) {
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
            if (lane == 0) src.row_loss[r] = acc;
        }
    }
    __syncthreads();
    for (int dl = 0; dl < nd; ++dl) {
        const float *vr = vrows + (int64_t)dl * T;
        float *wr = rows + (int64_t)dl * TS;
        for (int m = tid; m <= T; m += nth) {
            const float cur = m < T ? vr[m] : 0.0f;
            const float prv = m > 0 ? vr[m - 1] : 0.0f;
            wr[m] = vscale * (cur - prv);
        }
    }
}

// Work items are (frame, ball chunk, transducer slice).  With one slice the
// kernel writes the gradients; with nsl > 1 each item writes its slice's
// partial sums to part[(slice * NF + field) * pstride + ball] (NF = 5, or 1
// for the p0-only variant) and k_adj_reduce adds the slices in a fixed order,
// so results do not depend on scheduling.
// Occupancy target of the launch bounds (waves per SIMD): no instantiation may
// spill to scratch (the build checks the compiler's resource-usage remarks).
// FP32 kernels hold up to kMaxBpt = 3 balls per lane in 128 VGPRs (four
// waves); the FP64 twin, a correctness path, gets 256 (two waves).
template <typename R, int PROF, int DIR, bool FULL, bool SRC = false> struct AdjMinBlocks {
    // all-gradient GAUSS / OMNI needs more registers than four waves per SIMD
    // leave it: three waves rather than spilling (UNIFORM / COS fits four with
    // a staging depth of three); the variants that form the cotangent from
    // edge sums (small clouds, latency-bound) hold two, for their eight
    // samples per lane in flight while the balls load
    static constexpr int v = sizeof(R) == sizeof(double) ? 2
                             : SRC ? 2 : (FULL && PROF == GAUSS && DIR == OMNI) ? 3 : 4;
};

// S: NoSrc, or AdjSrc (FP32 GAUSS bins only) for the cotangent formed from
// the forward's edge sums (a separate instantiation, so that the other
// kernels carry neither its arguments nor its registers).
struct NoSrc {
    static constexpr bool on = false;
};
struct AdjSrcK : AdjSrc {
    static constexpr bool on = true;
};

template <typename R, int PROF, int DIR, bool FULL, typename S = NoSrc>
__global__ __launch_bounds__(512, (AdjMinBlocks<R, PROF, DIR, FULL, S::on>::v)) void k_adjoint(ArrayP<R> arr, BallsP<R> balls,
                                                 const int64_t *__restrict__ ball_off, int F,
                                                 int ds, int TT, int bpt, int nsl, int dsl,
                                                 Level lc, const R *__restrict__ v, R vscale,
                                                 uint32_t mask, BallsP<R> grad,
                                                 R *__restrict__ part, int64_t pstride,
                                                 const int32_t *__restrict__ order, S src) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    R *rows = reinterpret_cast<R *>(lds_raw);
    __shared__ int64_t s_off[SBP_MAX_FRAMES + 1];
    __shared__ int64_t s_cpre[SBP_MAX_FRAMES + 1];
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int T = lc.T;
    const int D = arr.D;
    const int64_t CH = (int64_t)nth * bpt;
    const int TS = adj_row_stride(TT);
    for (int i = tid; i <= F; i += nth) s_off[i] = ball_off[i];
    __syncthreads();
    if (tid == 0) {
        s_cpre[0] = 0;
        for (int f = 0; f < F; ++f)
            s_cpre[f + 1] = s_cpre[f] + (s_off[f + 1] - s_off[f] + CH - 1) / CH;
    }
    __syncthreads();
    const int64_t I = s_cpre[F] * nsl;
    for (int64_t it = blockIdx.x; it < I; it += gridDim.x) {
        const int64_t ci = it / nsl;
        const int sl = (int)(it - ci * nsl);
        int f = 0;
        while (ci >= s_cpre[f + 1]) ++f;
        [[maybe_unused]] const bool first = ci == s_cpre[f];   // the frame's first ball chunk
        const int64_t base = s_off[f] + (ci - s_cpre[f]) * CH;
        const int64_t end = min(base + CH, s_off[f + 1]);
        BallK<R, PROF> b[kMaxBpt];
        R acc[kMaxBpt][5];
        bool act[kMaxBpt];
        // (small clouds: the loads are only issued here; their arithmetic
        // waits until the rows are staged, so the two latencies overlap)
#pragma unroll
        for (int jb = 0; jb < kMaxBpt; ++jb) {
            const int64_t i0 = base + (int64_t)jb * nth + tid;
            act[jb] = jb < bpt && i0 < end;
#pragma unroll
            for (int k = 0; k < 5; ++k) acc[jb][k] = R(0);
            if (act[jb]) {
                const int64_t i = order ? (int64_t)order[i0] : i0;
                if constexpr (S::on) {
                    b[jb].x = balls.x[i];
                    b[jb].y = balls.y[i];
                    b[jb].z = balls.z[i];
                    b[jb].p = balls.p0[i];
                    b[jb].a = balls.a[i];
                } else {
                    b[jb] = load_ball<R, PROF>(balls.x[i], balls.y[i], balls.z[i], balls.p0[i],
                                               balls.a[i], lc);
                    act[jb] = b[jb].live;
                }
            }
        }
        [[maybe_unused]] bool pending = S::on;
        const R *vf = v + (int64_t)f * D * (int64_t)T;
        const int dbeg = sl * dsl;
        const int dend = min(D, dbeg + dsl);
        for (int d0 = dbeg; d0 < dend; d0 += ds) {
            const int nd = min(ds, dend - d0);
            for (int tlo = 0; tlo <= T; tlo += TT) {
                const int thi = min(tlo + TT, T + 1);
                __syncthreads();
                // point samples are staged as they are, bin edges differenced
                if constexpr (S::on)
                    stage_rows_from_sums(src, f, D, d0, nd, T, lc, vscale, rows, TS,
                                         rows + (int64_t)ds * TS, first);
                else
                    stage_rows<R, PROF != GPOINT, StageDepth<PROF, DIR, FULL>::v>(vf, d0, nd, T, tlo,
                                                                                  thi, vscale, rows, TS);
                __syncthreads();
                if constexpr (S::on) {
                    if (pending) {
#pragma unroll
                        for (int jb = 0; jb < kMaxBpt; ++jb)
                            if (act[jb]) {
                                finish_ball(b[jb], lc);
                                act[jb] = b[jb].live;
                            }
                        pending = false;
                    }
                }
                for (int dl = 0; dl < nd; ++dl) {
                    const int d = __builtin_amdgcn_readfirstlane(d0 + dl);
                    const R qx = ld_uniform(arr.qx + d), qy = ld_uniform(arr.qy + d),
                            qz = ld_uniform(arr.qz + d), nx = ld_uniform(arr.nx + d),
                            ny = ld_uniform(arr.ny + d), nz = ld_uniform(arr.nz + d);
                    const R *wrow = rows + (int64_t)dl * TS;
                    // the cotangent row: global, or staged after the rows when formed here
                    const R *vrow = S::on ? rows + (int64_t)ds * TS + (int64_t)dl * T
                                          : vf + (int64_t)d * T;
#pragma unroll
                    for (int jb = 0; jb < kMaxBpt; ++jb) {
                        if (!act[jb]) continue;
                        if constexpr (PROF == GPOINT)
                            adj_pair_point<R, DIR, FULL>(b[jb], qx, qy, qz, nx, ny, nz, lc, tlo, thi,
                                                         wrow, acc[jb]);
                        else
                            adj_pair<R, PROF, DIR, FULL>(b[jb], qx, qy, qz, nx, ny, nz, lc, tlo, thi,
                                                         wrow, vrow, vscale, acc[jb]);
                    }
                }
            }
        }
#pragma unroll
        for (int jb = 0; jb < kMaxBpt; ++jb) {
            const int64_t i0 = base + (int64_t)jb * nth + tid;
            if (!(jb < bpt && i0 < end)) continue;
            const int64_t i = order ? (int64_t)order[i0] : i0;
            // dead balls (a <= 0) get exact zeros, balls with a non-finite
            // parameter NaN
            {
                if (!ball_finite(balls.x[i], balls.y[i], balls.z[i], balls.p0[i], balls.a[i])) {
#pragma unroll
                    for (int k = 0; k < 5; ++k) acc[jb][k] = R(__builtin_nan(""));
                }
            }
            if (part) {
                if (FULL) {
#pragma unroll
                    for (int k = 0; k < 5; ++k) part[((int64_t)sl * 5 + k) * pstride + i] = acc[jb][k];
                } else {
                    part[(int64_t)sl * pstride + i] = acc[jb][3];
                }
                continue;
            }
            if (mask & SBP_X) grad.x[i] = acc[jb][0];
            if (mask & SBP_Y) grad.y[i] = acc[jb][1];
            if (mask & SBP_Z) grad.z[i] = acc[jb][2];
            if (mask & SBP_P0) grad.p0[i] = acc[jb][3];
            if (mask & SBP_A) {
                R ga = acc[jb][4];
                if (lc.a_softplus) ga *= sigmoid_dev(balls.a[i]);
                grad.a[i] = ga;
            }
        }
    }
}

// Sums the transducer slices of the partial gradients, slice 0 first;
// blockIdx.y is the parameter (the p0-only variant has one).
template <typename R, bool FULL>
__global__ void k_adj_reduce(const R *__restrict__ part, int nsl, int64_t pstride,
                             const int64_t *__restrict__ ball_off, int F, uint32_t mask,
                             int a_softplus, const R *__restrict__ a_arr, BallsP<R> grad) {
    const int k = FULL ? (int)blockIdx.y : 3;
    if (!(mask & (1u << k))) return;
    const int nf = FULL ? 5 : 1;
    R *out = k == 0 ? grad.x : k == 1 ? grad.y : k == 2 ? grad.z : k == 3 ? grad.p0 : grad.a;
    const R *pk = part + (int64_t)(FULL ? k : 0) * pstride;
    const int64_t lo = ball_off[0], hi = ball_off[F];
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
         i += (int64_t)gridDim.x * blockDim.x) {
        R s = slice_sum(pk + i, nsl, (int64_t)nf * pstride);
        if (k == 4 && a_softplus) s *= sigmoid_dev(a_arr[i]);
        out[i] = s;
    }
}

// Launch plan shared by the launcher and the workspace query: ball chunks of
// block * bpt balls (shrunk for small clouds), and as many transducer slices
// as it takes to give the chip about four work items per resident workgroup.
struct AdjPlan {
    int block, bpt, nsl, dsl;
};

// Workspace ceiling of the partial sums; plans that need more use fewer slices.
constexpr size_t kMaxAdjWs = size_t(512) << 20;

static AdjPlan adjoint_plan(const Ctx *c, int D, int64_t B_cap, int F, size_t slice_bytes) {
    AdjPlan p;
    p.block = c->tuning.adj_block;
    p.bpt = c->tuning.adj_bpt < kMaxBpt ? c->tuning.adj_bpt : kMaxBpt;
    int ds = c->tuning.adj_dets;
    if (ds > D) ds = D;
    const int64_t maxs = (D + ds - 1) / ds;
    const int64_t want = 4 * (int64_t)c->num_cus * (1024 / p.block > 0 ? 1024 / p.block : 1);
    auto chunks = [&](int blk, int bpt) {
        const int64_t ch = (int64_t)blk * bpt;
        return (B_cap + ch - 1) / ch + F;
    };
    while (p.bpt > 1 && chunks(p.block, p.bpt) * maxs < want) --p.bpt;
    while (p.block > 128 && chunks(p.block, p.bpt) * maxs < want) p.block /= 2;
    int64_t nsl = (want + chunks(p.block, p.bpt) - 1) / chunks(p.block, p.bpt);
    if (nsl > maxs) nsl = maxs;
    if (slice_bytes > 0 && (size_t)nsl * slice_bytes > kMaxAdjWs) nsl = (int64_t)(kMaxAdjWs / slice_bytes);
    if (nsl < 1) nsl = 1;
    int64_t dsl = ((D + nsl - 1) / nsl + ds - 1) / ds * ds;
    p.dsl = (int)dsl;
    p.nsl = (int)((D + dsl - 1) / dsl);
    return p;
}

size_t adjoint_ws_bytes(const Ctx *c, int D, int64_t B_cap, int F, uint32_t mask, size_t elem) {
    const int nf = (mask & ~SBP_P0) ? 5 : 1;
    const size_t slice = (size_t)nf * (size_t)B_cap * elem;
    const AdjPlan p = adjoint_plan(c, D, B_cap, F, slice);
    if (p.nsl <= 1) return 0;
    return ((size_t)p.nsl * slice + 255) & ~(size_t)255;
}

// LDS for the staged rows: what a workgroup may take, less the static arrays.
static size_t adj_lds_avail(const Ctx *c) {
    const size_t reserve = 2 * (SBP_MAX_FRAMES + 1) * sizeof(int64_t) + 256;
    return c->lds_max > reserve ? c->lds_max - reserve : 0;
}

bool adjoint_src_fits(const Ctx *c, int D, int T) {
    int ds = c->tuning.adj_dets;
    if (ds > D) ds = D;
    if (c->tuning.adj_tile > 0 && c->tuning.adj_tile < T + 1) return false;
    const size_t need = (size_t)ds * ((size_t)adj_row_stride(T + 1) + (size_t)T) * sizeof(float);
    return need <= adj_lds_avail(c);
}

template <typename R, int PROF, int DIR, bool FULL>
static int run_adjoint(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls,
                       const int64_t *ball_off, int F, int64_t B_cap, const Level &lc, const R *v,
                       R vscale, uint32_t mask, const BallsP<R> &grad, void *ws, size_t ws_bytes,
                       hipStream_t st, const int32_t *order, AdjDeferred *defer,
                       const AdjSrc *src) {
    auto kern = k_adjoint<R, PROF, DIR, FULL>;
    const size_t avail = adj_lds_avail(c);
    int ds = c->tuning.adj_dets;
    if (ds > arr.D) ds = arr.D;
    // edges 0..T staged per pass: the whole record if the ds rows fit (rows
    // padded to four floats)
    int64_t TT = (int64_t)(avail / ((size_t)ds * sizeof(R))) & ~(int64_t)3;
    if (TT > (int64_t)lc.T + 1) TT = (int64_t)lc.T + 1;
    if (TT < (int64_t)lc.T + 1 && TT < 64) return fail(SBP_E_DOMAIN, "LDS too small for %d rows", ds);
    if (c->tuning.adj_tile > 0 && TT > c->tuning.adj_tile) TT = c->tuning.adj_tile;
    constexpr bool CAN_SRC = sizeof(R) == sizeof(float) && PROF == GAUSS;
    if (src) {
        if (!CAN_SRC || !adjoint_src_fits(c, arr.D, lc.T))
            return fail(SBP_E_ARG, "the cotangent from edge sums needs FP32 GAUSS bins and whole rows");
        TT = (int64_t)lc.T + 1;
    }
    const int nf = FULL ? 5 : 1;
    AdjPlan pl = adjoint_plan(c, arr.D, B_cap, F, (size_t)nf * (size_t)B_cap * sizeof(R));
    if (pl.nsl > 1 && ws_bytes < (size_t)pl.nsl * nf * (size_t)B_cap * sizeof(R)) {
        pl.nsl = 1;
        pl.dsl = arr.D;
    }
    R *part = pl.nsl > 1 ? (R *)ws : nullptr;
    const int block = pl.block;
    // (with the cotangent formed here, its rows follow the staged edge rows)
    const size_t lds = (size_t)ds * ((size_t)adj_row_stride((int)TT) + (src ? (size_t)lc.T : 0)) *
                       sizeof(R);
    const void *kfun = (const void *)kern;
    if constexpr (CAN_SRC)
        if (src) kfun = (const void *)k_adjoint<R, PROF, DIR, FULL, AdjSrcK>;
    SBP_HIP(hipFuncSetAttribute(kfun, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int grid = c->tuning.adj_grid;
    if (grid <= 0) {
        int per_cu = 0;
        SBP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfun, block, lds));
        if (per_cu < 1) per_cu = 1;
        grid = per_cu * c->num_cus;
    }
    const int64_t CH = (int64_t)block * pl.bpt;
    const int64_t max_items = ((B_cap + CH - 1) / CH + F) * pl.nsl;
    if (grid > max_items) grid = (int)max_items;
    if (grid < 1) grid = 1;
    bool launched = false;
    if constexpr (CAN_SRC) {
        if (src) {
            AdjSrcK sk;
            static_cast<AdjSrc &>(sk) = *src;
            hipLaunchKernelGGL((k_adjoint<R, PROF, DIR, FULL, AdjSrcK>), dim3(grid), dim3(block), lds,
                               st, arr, balls, ball_off, F, ds, (int)TT, pl.bpt, pl.nsl, pl.dsl, lc,
                               v, vscale, mask, grad, part, B_cap, order, sk);
            launched = true;
        }
    }
    if (!launched)
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, st, arr, balls, ball_off, F, ds,
                           (int)TT, pl.bpt, pl.nsl, pl.dsl, lc, v, vscale, mask, grad, part, B_cap,
                           order, NoSrc{});
    SBP_HIP(hipGetLastError());
    if (defer) {
        *defer = AdjDeferred{};
        if constexpr (FULL && sizeof(R) == sizeof(float)) {
            if (part) {
                defer->part = (const float *)part;
                defer->nsl = pl.nsl;
                defer->pstride = B_cap;
                return SBP_OK;
            }
        }
    }
    if (part) {
        int64_t nb = (B_cap + 255) / 256;
        if (nb > 2048) nb = 2048;
        hipLaunchKernelGGL((k_adj_reduce<R, FULL>), dim3((int)nb, FULL ? 5 : 1), dim3(256), 0, st,
                           (const R *)part,
                           pl.nsl, B_cap, ball_off, F, mask, lc.a_softplus, (const R *)balls.a, grad);
        SBP_HIP(hipGetLastError());
    }
    return SBP_OK;
}

template <typename R, bool FULL>
static int dispatch_adjoint(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls,
                            const int64_t *ball_off, int F, int64_t B_cap, const sbp_model *m,
                            const R *v, R vscale, uint32_t mask, const BallsP<R> &grad, void *ws,
                            size_t ws_bytes, hipStream_t st, const int32_t *order,
                            AdjDeferred *defer, const AdjSrc *src) {
    const Level lc = make_level(m);
    if (profile_code(m) == GPOINT) {
        if (m->directivity == SBP_DIR_COS)
            return run_adjoint<R, GPOINT, COS, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v,
                                                     vscale, mask, grad, ws, ws_bytes, st, order, defer, src);
        return run_adjoint<R, GPOINT, OMNI, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v, vscale,
                                                  mask, grad, ws, ws_bytes, st, order, defer, src);
    }
    if (m->profile == SBP_PROFILE_GAUSS) {
        if (m->directivity == SBP_DIR_COS)
            return run_adjoint<R, GAUSS, COS, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v,
                                                    vscale, mask, grad, ws, ws_bytes, st, order, defer, src);
        return run_adjoint<R, GAUSS, OMNI, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v, vscale,
                                                 mask, grad, ws, ws_bytes, st, order, defer, src);
    }
    if (m->directivity == SBP_DIR_COS)
        return run_adjoint<R, UNIFORM, COS, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v, vscale,
                                                  mask, grad, ws, ws_bytes, st, order, defer, src);
    return run_adjoint<R, UNIFORM, OMNI, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v, vscale,
                                               mask, grad, ws, ws_bytes, st, order, defer, src);
}

template <typename R>
int launch_adjoint(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls, const int64_t *ball_off,
                   int F, int64_t B_cap, const sbp_model *m, const R *v, R vscale,
                   uint32_t mask, const BallsP<R> &grad, void *ws, size_t ws_bytes, hipStream_t st,
                   const int32_t *order, AdjDeferred *defer, const AdjSrc *src) {
    if (defer) *defer = AdjDeferred{};
    if (B_cap == 0) return SBP_OK;
    if ((mask & ~SBP_P0) == 0)
        return dispatch_adjoint<R, false>(c, arr, balls, ball_off, F, B_cap, m, v, vscale, mask,
                                          grad, ws, ws_bytes, st, order, defer, src);
    return dispatch_adjoint<R, true>(c, arr, balls, ball_off, F, B_cap, m, v, vscale, mask, grad,
                                     ws, ws_bytes, st, order, defer, src);
}

template int launch_adjoint<float>(Ctx *, const ArrayP<float> &, const BallsP<float> &,
                                   const int64_t *, int, int64_t, const sbp_model *, const float *,
                                   float, uint32_t, const BallsP<float> &, void *, size_t,
                                   hipStream_t, const int32_t *, AdjDeferred *, const AdjSrc *);
template int launch_adjoint<double>(Ctx *, const ArrayP<double> &, const BallsP<double> &,
                                    const int64_t *, int, int64_t, const sbp_model *,
                                    const double *, double, uint32_t, const BallsP<double> &,
                                    void *, size_t, hipStream_t, const int32_t *, AdjDeferred *,
                                    const AdjSrc *);

}  // namespace sbp
