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
#include "sbp_internal.hpp"

namespace sbp {

constexpr int kMaxBpt = 4;

// Edges per exact restart of the Gaussian recurrence below; the UNIFORM
// profile uses blocks of the same length for its moment sums.
constexpr int kRestart = 16;
// Staged values loaded together (one LDS latency per group, not per edge).
constexpr int kGroup = 8;
// FP32 unrolls a whole block with its edge offsets as constants; the FP64
// twin, which spills at this register budget, keeps a run-time loop.
template <typename R> struct BlockUnroll { static constexpr bool on = true; };
template <> struct BlockUnroll<double> { static constexpr bool on = false; };

// Transducer data is read-only for the whole launch and indexed by a
// wave-uniform value: read it through the scalar cache.
template <typename R> __device__ __forceinline__ R ld_uniform(const R *p) {
    return *(const __attribute__((address_space(4))) R *)p;
}

// Moment sums of one block of n <= kRestart edges starting at m0, j = m - m0:
//   Z = sum w_j f_j,  Z1 = sum w_j f_j j,  Z2 = sum w_j f_j j^2,  Z3 = sum w_j f_j j^3
// (the first NMOM of them) with f_j = e_j (GAUSS, e_{j+1} = e_j g_j,
// g_{j+1} = g_j h) or 1 (UNIFORM).  Along the edges u_j = u_0 - j c, so
// sum w f u = u_0 Z - c Z1, sum w f u^2 = u_0 (u_0 Z - 2 c Z1) + c^2 Z2, and
// likewise for u^3: a few sums per edge replace the running u and its powers.
template <typename R, int PROF, int NMOM>
__device__ inline void block_moments(const R *__restrict__ wb, int n, R e, R gq, R h, R &Z, R &Z1,
                                     R &Z2, R &Z3) {
    constexpr bool EXPO = PROF != UNIFORM;
    auto edge = [&](R w, R j, bool j0) {
        const R wf = EXPO ? w * e : w;
        Z += wf;
        if (NMOM >= 2 && !j0) Z1 = fma(wf, j, Z1);
        if (NMOM >= 3 && !j0) Z2 = fma(wf, j * j, Z2);
        if (NMOM >= 4 && !j0) Z3 = fma(wf, j * j * j, Z3);
        if (EXPO) {
            e *= gq;
            gq *= h;
        }
    };
    if (BlockUnroll<R>::on && n == kRestart) {
#pragma unroll
        for (int g0 = 0; g0 < kRestart; g0 += kGroup) {
            R w[kGroup];
#pragma unroll
            for (int k = 0; k < kGroup; ++k) w[k] = wb[g0 + k];
#pragma unroll
            for (int k = 0; k < kGroup; ++k) edge(w[k], R(g0 + k), g0 + k == 0);
        }
        return;
    }
    int k = 0;
    R j = R(0);
    if (BlockUnroll<R>::on) {
        for (; k + kGroup <= n; k += kGroup) {
            R w[kGroup];
#pragma unroll
            for (int i = 0; i < kGroup; ++i) w[i] = wb[k + i];
#pragma unroll
            for (int i = 0; i < kGroup; ++i) {
                edge(w[i], j, false);
                j += R(1);
            }
        }
    }
    for (; k < n; ++k) {
        edge(wb[k], j, false);
        j += R(1);
    }
}

// Point sampling (GPOINT): sample m carries p0 D g(u_m) / (2 rho) with
// g(u) = u e(u), e(u) = exp(-u^2 / (2 a^2)) for |u| < K a.  The staged row
// holds w_m = vscale v_m (not differenced), and
//   S0 = sum w g,  S1 = sum w g' = sum w e (1 - u^2 / a^2),
//   S2 = sum w dg/da = sum w e u^3 / a^3
// over the samples inside the support; the gradients then follow from the
// same closed forms as the bin means with G = D / (2 rho).
template <typename R, int DIR, bool FULL>
__device__ inline void adj_pair_point(const BallK<R, GPOINT> &b, R qx, R qy, R qz, R nx, R ny, R nz,
                                      const Level &lc, int tlo, int thi, const R *__restrict__ wr,
                                      R acc[5]) {
    PairG<R> g;
    if (!pair_geometry<R, DIR>(b.x, b.y, b.z, b.w, qx, qy, qz, nx, ny, nz, lc, g)) return;
    // samples inside the support: (s - w) / (c dt) < m < (s + w) / (c dt), m < T
    const double lo = floor((g.s - (double)b.w) * lc.inv_cdt) + 1.0;
    const double hi = ceil((g.s + (double)b.w) * lc.inv_cdt) - 1.0;
    const int top = min(thi, lc.T) - 1;
    if (hi < (double)tlo || lo > (double)top || hi < lo) return;
    const int mb = lo < (double)tlo ? tlo : (int)lo;
    const int me = hi > (double)top ? top : (int)hi;
    wr -= tlo;
    const R c = LevelR<R>::cdt(lc);
    constexpr int NMOM = FULL ? 4 : 2;
    // U1 = sum w e u, U2 = sum w e u^2, U3 = sum w e u^3, E0 = sum w e
    R E0 = R(0), U1 = R(0), U2 = R(0), U3 = R(0);
    for (int m0 = mb; m0 <= me; m0 += kRestart) {
        const R u0 = (R)(g.s - (double)m0 * lc.cdt);
        const int n = min(kRestart, me - m0 + 1);
        R e = ex2(u0 * u0 * b.q0);
        R gq = ex2(b.q0 * c * (c - R(2) * u0));
        R Z = R(0), Z1 = R(0), Z2 = R(0), Z3 = R(0);
        block_moments<R, GPOINT, NMOM>(wr + m0, n, e, gq, b.h, Z, Z1, Z2, Z3);
        const R cZ1 = c * Z1;
        U1 += u0 * Z - cZ1;
        if (FULL) {
            const R c2Z2 = c * c * Z2;
            E0 += Z;
            U2 += u0 * fma(u0, Z, R(-2) * cZ1) + c2Z2;
            // u0^3 Z - 3 u0^2 c Z1 + 3 u0 c^2 Z2 - c^3 Z3
            U3 += fma(u0, fma(u0, fma(u0, Z, R(-3) * cZ1), R(3) * c2Z2), -(c * c * c * Z3));
        }
    }
    const R inv_a2 = R(1) / (b.a * b.a);
    const R S0 = U1;
    const R G = g.dir * R(0.5) * g.inv_rho;
    acc[3] = fma(G, S0, acc[3]);
    if (FULL) {
        const R S1 = E0 - U2 * inv_a2;
        const R S2 = U3 * inv_a2 / b.a;
        const R pG = b.p * G;
        acc[4] = fma(pG, S2, acc[4]);
        const R radial = pG * (S1 - S0 * g.inv_rho);
        acc[0] = fma(radial, g.ex, acc[0]);
        acc[1] = fma(radial, g.ey, acc[1]);
        acc[2] = fma(radial, g.ez, acc[2]);
        if (DIR == COS) {
            const R ct = b.p * R(0.5) * S0 * g.inv_rho * g.inv_rho;
            acc[0] = fma(ct, nx - g.dir * g.ex, acc[0]);
            acc[1] = fma(ct, ny - g.dir * g.ey, acc[1]);
            acc[2] = fma(ct, nz - g.dir * g.ez, acc[2]);
        }
    }
}

// Accumulates the pair's support edges in the staged tile [tlo, thi)
// (wr[m - tlo]).  Everything is linear in (S0, S1, S2), so tiles add up.
//
// GAUSS: along the edges u_{m+1} = u_m - c, so e_m = exp(-u_m^2 / (2 a^2))
// obeys e_{m+1} = e_m g_m with g_{m+1} = g_m h, h = exp(-c^2 / a^2): two
// multiplies per edge instead of an exponential.  Both are recomputed
// exactly every kRestart edges (relative drift below 1e-5 in between).  The
// plain sum of w over the pair's edges telescopes, sum_{m=mb}^{me} w_m =
// vscale (v_me - v_{mb-1}), and is read from the cotangent row `vrow`.
template <typename R, int PROF, int DIR, bool FULL>
__device__ inline void adj_pair(const BallK<R, PROF> &b, R qx, R qy, R qz, R nx, R ny, R nz,
                                const Level &lc, int tlo, int thi, const R *__restrict__ wr,
                                const R *__restrict__ vrow, R vscale, R acc[5]) {
    PairG<R> g;
    if (!pair_geometry<R, DIR>(b.x, b.y, b.z, b.w, qx, qy, qz, nx, ny, nz, lc, g)) return;
    // support edges: |u_m| < w  <=>  (s - w) / (c dt) < m < (s + w) / (c dt)
    const double lo = floor((g.s - (double)b.w) * lc.inv_cdt) + 1.0;
    const double hi = ceil((g.s + (double)b.w) * lc.inv_cdt) - 1.0;
    if (hi < (double)tlo || lo > (double)(thi - 1) || hi < lo) return;
    const int mb = lo < (double)tlo ? tlo : (int)lo;
    const int me = hi > (double)(thi - 1) ? thi - 1 : (int)hi;
    R vhi = R(0), vlo = R(0);
    if (PROF == GAUSS) {
        vhi = me < lc.T ? vrow[me] : R(0);
        vlo = mb > 0 ? vrow[mb - 1] : R(0);
    }
    wr -= tlo;
    const R c = LevelR<R>::cdt(lc);
    // P = sum w f, A1 = sum w f u, A2 = sum w f u^2 (f = e for GAUSS, 1 for
    // UNIFORM), W = sum w
    R P = R(0), W = R(0), A1 = R(0), A2 = R(0);
    constexpr bool MOM = FULL || PROF == UNIFORM;
    for (int m0 = mb; m0 <= me; m0 += kRestart) {
        const R u0 = (R)(g.s - (double)m0 * lc.cdt);
        const int n = min(kRestart, me - m0 + 1);
        R e = R(1), gq = R(1);
        if (PROF == GAUSS) {
            e = ex2(u0 * u0 * b.q0);
            gq = ex2(b.q0 * c * (c - R(2) * u0));
        }
        R Z = R(0), Z1 = R(0), Z2 = R(0), Z3 = R(0);
        block_moments<R, PROF, MOM ? 3 : 1>(wr + m0, n, e, gq, b.h, Z, Z1, Z2, Z3);
        P += Z;
        if (MOM) {
            const R cZ1 = c * Z1;
            A1 += u0 * Z - cZ1;
            A2 += u0 * fma(u0, Z, R(-2) * cZ1) + c * c * Z2;
        }
    }
    R S0, S1, S2;
    if (PROF == GAUSS) {
        W = vscale * (vhi - vlo);
        const R A0 = P - LevelR<R>::eK(lc) * W;          // sum w (e - e^{-K^2/2})
        S0 = -(b.a * b.a) * A0;
        S1 = A1;
        S2 = R(-2) * b.a * A0 - A2 / b.a;
    } else {
        W = P;
        S0 = R(-0.5) * (b.q0 * W - A2);                  // -(1/2) sum w (a^2 - u^2)
        S1 = A1;
        S2 = -b.a * W;
    }
    const R G = g.dir * LevelR<R>::inv2cdt(lc) * g.inv_rho;
    acc[3] = fma(G, S0, acc[3]);
    if (FULL) {
        const R pG = b.p * G;
        acc[4] = fma(pG, S2, acc[4]);
        const R radial = pG * (S1 - S0 * g.inv_rho);
        acc[0] = fma(radial, g.ex, acc[0]);
        acc[1] = fma(radial, g.ey, acc[1]);
        acc[2] = fma(radial, g.ez, acc[2]);
        if (DIR == COS) {
            const R ct = b.p * LevelR<R>::inv2cdt(lc) * S0 * g.inv_rho * g.inv_rho;
            acc[0] = fma(ct, nx - g.dir * g.ex, acc[0]);
            acc[1] = fma(ct, ny - g.dir * g.ey, acc[1]);
            acc[2] = fma(ct, nz - g.dir * g.ez, acc[2]);
        }
    }
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
// one round with 256 threads; the point-sampled OMNI gradient kernel takes
// three, the most that keeps its pass loop free of register spills.
template <int PROF, int DIR, bool FULL> struct StageDepth {
    static constexpr int v = (PROF == GPOINT && DIR == OMNI && FULL) ? 3 : 4;
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

// Work items are (frame, ball chunk, transducer slice).  With one slice the
// kernel writes the gradients; with nsl > 1 each item writes its slice's
// partial sums to part[(slice * NF + field) * pstride + ball] (NF = 5, or 1
// for the p0-only variant) and k_adj_reduce adds the slices in a fixed order,
// so results do not depend on scheduling.
// Occupancy target of the launch bounds: the FP32 kernel is capped at 128
// VGPRs (four waves per SIMD); the FP64 twin, a correctness path, gets the
// registers it needs instead of spilling.
template <typename R> struct AdjMinBlocks { static constexpr int v = 4; };
template <> struct AdjMinBlocks<double> { static constexpr int v = 2; };

template <typename R, int PROF, int DIR, bool FULL>
__global__ __launch_bounds__(512, AdjMinBlocks<R>::v) void k_adjoint(ArrayP<R> arr, BallsP<R> balls,
                                                 const int64_t *__restrict__ ball_off, int F,
                                                 int ds, int TT, int bpt, int nsl, int dsl,
                                                 Level lc, const R *__restrict__ v, R vscale,
                                                 uint32_t mask, BallsP<R> grad,
                                                 R *__restrict__ part, int64_t pstride,
                                                 const int32_t *__restrict__ order) {
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
        const int64_t base = s_off[f] + (ci - s_cpre[f]) * CH;
        const int64_t end = min(base + CH, s_off[f + 1]);
        BallK<R, PROF> b[kMaxBpt];
        R acc[kMaxBpt][5];
        bool act[kMaxBpt];
#pragma unroll
        for (int jb = 0; jb < kMaxBpt; ++jb) {
            const int64_t i0 = base + (int64_t)jb * nth + tid;
            act[jb] = jb < bpt && i0 < end;
#pragma unroll
            for (int k = 0; k < 5; ++k) acc[jb][k] = R(0);
            if (act[jb]) {
                const int64_t i = order ? (int64_t)order[i0] : i0;
                b[jb] = load_ball<R, PROF>(balls.x[i], balls.y[i], balls.z[i], balls.p0[i],
                                           balls.a[i], lc);
                act[jb] = b[jb].live;
            }
        }
        const R *vf = v + (int64_t)f * D * (int64_t)T;
        const int dbeg = sl * dsl;
        const int dend = min(D, dbeg + dsl);
        for (int d0 = dbeg; d0 < dend; d0 += ds) {
            const int nd = min(ds, dend - d0);
            for (int tlo = 0; tlo <= T; tlo += TT) {
                const int thi = min(tlo + TT, T + 1);
                __syncthreads();
                // point samples are staged as they are, bin edges differenced
                stage_rows<R, PROF != GPOINT, StageDepth<PROF, DIR, FULL>::v>(vf, d0, nd, T, tlo, thi,
                                                                              vscale, rows, TS);
                __syncthreads();
                for (int dl = 0; dl < nd; ++dl) {
                    const int d = __builtin_amdgcn_readfirstlane(d0 + dl);
                    const R qx = ld_uniform(arr.qx + d), qy = ld_uniform(arr.qy + d),
                            qz = ld_uniform(arr.qz + d), nx = ld_uniform(arr.nx + d),
                            ny = ld_uniform(arr.ny + d), nz = ld_uniform(arr.nz + d);
                    const R *wrow = rows + (int64_t)dl * TS;
                    const R *vrow = vf + (int64_t)d * T;
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

// Sums the transducer slices of the partial gradients, slice 0 first.
template <typename R, bool FULL>
__global__ void k_adj_reduce(const R *__restrict__ part, int nsl, int64_t pstride,
                             const int64_t *__restrict__ ball_off, int F, uint32_t mask,
                             int a_softplus, const R *__restrict__ a_arr, BallsP<R> grad) {
    const int64_t lo = ball_off[0], hi = ball_off[F];
    R *out[5] = {grad.x, grad.y, grad.z, grad.p0, grad.a};
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (FULL) {
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                if (!(mask & (1u << k))) continue;
                R s = R(0);
                for (int sl = 0; sl < nsl; ++sl) s += part[((int64_t)sl * 5 + k) * pstride + i];
                if (k == 4 && a_softplus) s *= sigmoid_dev(a_arr[i]);
                out[k][i] = s;
            }
        } else {
            R s = R(0);
            for (int sl = 0; sl < nsl; ++sl) s += part[(int64_t)sl * pstride + i];
            grad.p0[i] = s;
        }
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
    p.bpt = c->tuning.adj_bpt;
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

template <typename R, int PROF, int DIR, bool FULL>
static int run_adjoint(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls,
                       const int64_t *ball_off, int F, int64_t B_cap, const Level &lc, const R *v,
                       R vscale, uint32_t mask, const BallsP<R> &grad, void *ws, size_t ws_bytes,
                       hipStream_t st, const int32_t *order) {
    auto kern = k_adjoint<R, PROF, DIR, FULL>;
    const size_t reserve = 2 * (SBP_MAX_FRAMES + 1) * sizeof(int64_t) + 256;
    const size_t avail = c->lds_max > reserve ? c->lds_max - reserve : 0;
    int ds = c->tuning.adj_dets;
    if (ds > arr.D) ds = arr.D;
    // edges 0..T staged per pass: the whole record if the ds rows fit (rows
    // padded to four floats)
    int64_t TT = (int64_t)(avail / ((size_t)ds * sizeof(R))) & ~(int64_t)3;
    if (TT > (int64_t)lc.T + 1) TT = (int64_t)lc.T + 1;
    if (TT < (int64_t)lc.T + 1 && TT < 64) return fail(SBP_E_DOMAIN, "LDS too small for %d rows", ds);
    if (c->tuning.adj_tile > 0 && TT > c->tuning.adj_tile) TT = c->tuning.adj_tile;
    const int nf = FULL ? 5 : 1;
    AdjPlan pl = adjoint_plan(c, arr.D, B_cap, F, (size_t)nf * (size_t)B_cap * sizeof(R));
    if (pl.nsl > 1 && ws_bytes < (size_t)pl.nsl * nf * (size_t)B_cap * sizeof(R)) {
        pl.nsl = 1;
        pl.dsl = arr.D;
    }
    R *part = pl.nsl > 1 ? (R *)ws : nullptr;
    const int block = pl.block;
    const size_t lds = (size_t)ds * (size_t)adj_row_stride((int)TT) * sizeof(R);
    SBP_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    int grid = c->tuning.adj_grid;
    if (grid <= 0) {
        int per_cu = 0;
        SBP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, block, lds));
        if (per_cu < 1) per_cu = 1;
        grid = per_cu * c->num_cus;
    }
    const int64_t CH = (int64_t)block * pl.bpt;
    const int64_t max_items = ((B_cap + CH - 1) / CH + F) * pl.nsl;
    if (grid > max_items) grid = (int)max_items;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, st, arr, balls, ball_off, F, ds,
                       (int)TT, pl.bpt, pl.nsl, pl.dsl, lc, v, vscale, mask, grad, part, B_cap,
                       order);
    SBP_HIP(hipGetLastError());
    if (part) {
        int64_t nb = (B_cap + 255) / 256;
        if (nb > 2048) nb = 2048;
        hipLaunchKernelGGL((k_adj_reduce<R, FULL>), dim3((int)nb), dim3(256), 0, st, (const R *)part,
                           pl.nsl, B_cap, ball_off, F, mask, lc.a_softplus, (const R *)balls.a, grad);
        SBP_HIP(hipGetLastError());
    }
    return SBP_OK;
}

template <typename R, bool FULL>
static int dispatch_adjoint(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls,
                            const int64_t *ball_off, int F, int64_t B_cap, const sbp_model *m,
                            const R *v, R vscale, uint32_t mask, const BallsP<R> &grad, void *ws,
                            size_t ws_bytes, hipStream_t st, const int32_t *order) {
    const Level lc = make_level(m);
    if (profile_code(m) == GPOINT) {
        if (m->directivity == SBP_DIR_COS)
            return run_adjoint<R, GPOINT, COS, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v,
                                                     vscale, mask, grad, ws, ws_bytes, st, order);
        return run_adjoint<R, GPOINT, OMNI, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v, vscale,
                                                  mask, grad, ws, ws_bytes, st, order);
    }
    if (m->profile == SBP_PROFILE_GAUSS) {
        if (m->directivity == SBP_DIR_COS)
            return run_adjoint<R, GAUSS, COS, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v,
                                                    vscale, mask, grad, ws, ws_bytes, st, order);
        return run_adjoint<R, GAUSS, OMNI, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v, vscale,
                                                 mask, grad, ws, ws_bytes, st, order);
    }
    if (m->directivity == SBP_DIR_COS)
        return run_adjoint<R, UNIFORM, COS, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v, vscale,
                                                  mask, grad, ws, ws_bytes, st, order);
    return run_adjoint<R, UNIFORM, OMNI, FULL>(c, arr, balls, ball_off, F, B_cap, lc, v, vscale,
                                               mask, grad, ws, ws_bytes, st, order);
}

template <typename R>
int launch_adjoint(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls, const int64_t *ball_off,
                   int F, int64_t B_cap, const sbp_model *m, const R *v, R vscale,
                   uint32_t mask, const BallsP<R> &grad, void *ws, size_t ws_bytes, hipStream_t st,
                   const int32_t *order) {
    if (B_cap == 0) return SBP_OK;
    if ((mask & ~SBP_P0) == 0)
        return dispatch_adjoint<R, false>(c, arr, balls, ball_off, F, B_cap, m, v, vscale, mask,
                                          grad, ws, ws_bytes, st, order);
    return dispatch_adjoint<R, true>(c, arr, balls, ball_off, F, B_cap, m, v, vscale, mask, grad,
                                     ws, ws_bytes, st, order);
}

template int launch_adjoint<float>(Ctx *, const ArrayP<float> &, const BallsP<float> &,
                                   const int64_t *, int, int64_t, const sbp_model *, const float *,
                                   float, uint32_t, const BallsP<float> &, void *, size_t,
                                   hipStream_t, const int32_t *);
template int launch_adjoint<double>(Ctx *, const ArrayP<double> &, const BallsP<double> &,
                                    const int64_t *, int, int64_t, const sbp_model *,
                                    const double *, double, uint32_t, const BallsP<double> &,
                                    void *, size_t, hipStream_t, const int32_t *);

}  // namespace sbp
