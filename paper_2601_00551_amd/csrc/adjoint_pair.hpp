// Per-pair arithmetic of the adjoint (vector-Jacobian product of the
// forward model of section 4.2 / 4.3) and of the filter's p0-only variant:
// the moment sums of one block of support edges and the closed-form
// gradients of one (ball, transducer) pair from the staged, pre-differenced
// cotangent row.  Included by adjoint.hip; host-and-device so that a test can
// run the FP64 instantiation against the CPU oracle on the host.
#pragma once

#include "sbp_internal.hpp"

namespace sbp {

// Edges per exact restart of the Gaussian recurrence below; the UNIFORM
// profile uses blocks of the same length for its moment sums.
constexpr int kRestart = 16;
// Staged values loaded together (one LDS latency per group, not per edge).
constexpr int kGroup = 8;
// FP32 unrolls a whole block with its edge offsets as constants; the FP64
// twin, which spills at this register budget, keeps a run-time loop.
template <typename R> struct BlockUnroll { static constexpr bool on = true; };
template <> struct BlockUnroll<double> { static constexpr bool on = false; };

// Moment sums of one block of n <= kRestart edges starting at m0, j = m - m0:
//   Z = sum w_j f_j,  Z1 = sum w_j f_j j,  Z2 = sum w_j f_j j^2,  Z3 = sum w_j f_j j^3
// (the first NMOM of them) with f_j = e_j (GAUSS, e_{j+1} = e_j g_j,
// g_{j+1} = g_j h) or 1 (UNIFORM).  Along the edges u_j = u_0 - j c, so
// sum w f u = u_0 Z - c Z1, sum w f u^2 = u_0 (u_0 Z - 2 c Z1) + c^2 Z2, and
// likewise for u^3: a few sums per edge replace the running u and its powers.
template <typename R, int PROF, int NMOM>
SBP_HD inline void block_moments(const R *__restrict__ wb, int n, R e, R gq, R h, R &Z, R &Z1,
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
SBP_HD inline void adj_pair_point(const BallK<R, GPOINT> &b, R qx, R qy, R qz, R nx, R ny, R nz,
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
SBP_HD inline void adj_pair(const BallK<R, PROF> &b, R qx, R qy, R qz, R nx, R ny, R nz,
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
        // -(1/2) sum w (a^2 - u^2); a^2 formed here (the same product as
        // b.q0) so that b.q0 is not held per ball across the transducers
        S0 = R(-0.5) * ((b.a * b.a) * W - A2);
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

}  // namespace sbp
