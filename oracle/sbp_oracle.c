/*
 * FP64 CPU oracle for the sliding-ball forward model and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper with
 * the HIP library: every formula below is written out again from the physics.
 *
 * What it computes (paper section 4.1 and 4.3, equations for Simulate with
 * Delta t_k = f_k Delta t and T_k = T / f_k):
 *
 *   A ball i is a radially symmetric initial pressure p0_i * fhat(|r - r_i|; a_i)
 *   (paper 4.1: Gaussian-distributed spherical sources with peak p0 and
 *   standard deviation a0).  In a lossless homogeneous medium with zero initial
 *   velocity the pressure at distance rho from the centre is (d'Alembert on
 *   w = rho*p, even extension of f):
 *
 *       p(rho, t) = [ (rho - ct) f(rho - ct) + (rho + ct) f(rho + ct) ] / (2 rho)
 *
 *   and for a transducer outside the support only the first term survives for
 *   t >= 0.  With u = rho - c t this is p = p0 * u * fhat(u) / (2 rho).
 *
 *   Readings taken where the paper is silent:
 *     - profile GAUSS: fhat(s) = exp(-s^2 / (2 a^2)), truncated at |s| < K a;
 *       profile UNIFORM: fhat(s) = 1 for |s| < a (the textbook N-shaped pulse).
 *     - sampling BIN: sample n is the mean of p over the bin
 *       [tau_n, tau_{n+1}), tau_m = t0 + m * dt_k.  Since dt = -du / c, the bin
 *       mean is p0 * [psi(u_n) - psi(u_{n+1})] / (2 rho c dt_k) with psi the
 *       compactly supported antiderivative of u * fhat(u).
 *       Sampling POINT (value at tau_n) is kept for the textbook comparison.
 *     - directivity COS: the trace is scaled by max(0, n_hat . e_hat) with
 *       e_hat the unit vector from transducer to ball centre; OMNI: factor 1.
 *     - near field: a pair with rho <= half-width of the support contributes 0;
 *       a ball with a <= 0 contributes 0.
 *     - record clipping: only bins 0 <= n < T_k exist.
 *
 * Gradients are taken by forward-mode dual numbers pushed through the same
 * definition (no hand-derived adjoint): for each pair the five tangents with
 * respect to (x, y, z, p0, a) of every bin value are formed and contracted
 * with the cotangent v.  The plain forward below is a separate, value-only
 * transcription so that the two can be checked against each other.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_UNIFORM 0
#define ORC_GAUSS 1
#define ORC_OMNI 0
#define ORC_COS 1
#define ORC_BIN 0
#define ORC_POINT 1

/* Time model of one level k: speed of sound c (mm/us), base interval dt (us),
 * time of the first edge t0 (us), samples T (= T_k), factor f (= f_k), profile,
 * directivity, truncation K (GAUSS, units of a) and sampling mode. */
typedef struct {
    double c, dt, t0, K;
    int32_t T, f, profile, directivity, sampling, pad_;
} orc_time;

/* ---------------------------------------------------------------- values -- */

/* Support half-width of a ball of size a. */
static double half_width(double a, const orc_time *tm)
{
    return tm->profile == ORC_UNIFORM ? a : tm->K * a;
}

/* Radial profile fhat(u) (peak 1). */
static double fhat(double u, double a, const orc_time *tm)
{
    if (tm->profile == ORC_UNIFORM)
        return fabs(u) < a ? 1.0 : 0.0;
    return fabs(u) < tm->K * a ? exp(-u * u / (2.0 * a * a)) : 0.0;
}

/* psi(u): antiderivative of u * fhat(u) in u, zero outside the support. */
static double psi(double u, double a, const orc_time *tm)
{
    if (tm->profile == ORC_UNIFORM)
        return fabs(u) < a ? -0.5 * (a * a - u * u) : 0.0;
    if (fabs(u) < tm->K * a)
        return -a * a * (exp(-u * u / (2.0 * a * a)) - exp(-0.5 * tm->K * tm->K));
    return 0.0;
}

/* Range of bins [*lo, *hi] that can be non-zero for a pair at distance rho:
 * edges m with |rho - c tau_m| < w, widened by one bin on each side (the
 * profile functions return exact zeros outside, so a generous range is safe). */
static void bin_range(double rho, double w, const orc_time *tm, int64_t *lo, int64_t *hi)
{
    double dtk = tm->f * tm->dt;
    double m_first = (rho - w - tm->c * tm->t0) / (tm->c * dtk);
    double m_last = (rho + w - tm->c * tm->t0) / (tm->c * dtk);
    int64_t a = (int64_t)floor(m_first) - 2;
    int64_t b = (int64_t)ceil(m_last) + 1;
    if (a < 0) a = 0;
    if (b > tm->T - 1) b = tm->T - 1;
    *lo = a;
    *hi = b;
}

/* Add one pair's trace into row[0..T). */
static void pair_trace(double bx, double by, double bz, double p0, double a,
                       double qx, double qy, double qz, double nx, double ny, double nz,
                       const orc_time *tm, double *row)
{
    if (!(a > 0.0)) return;
    double dx = bx - qx, dy = by - qy, dz = bz - qz;
    double rho = sqrt(dx * dx + dy * dy + dz * dz);
    double w = half_width(a, tm);
    if (rho <= w) return;
    double dir = 1.0;
    if (tm->directivity == ORC_COS) {
        double cosv = (nx * dx + ny * dy + nz * dz) / rho;
        dir = cosv > 0.0 ? cosv : 0.0;
    }
    if (dir == 0.0) return;
    double dtk = tm->f * tm->dt;
    int64_t lo, hi;
    bin_range(rho, w, tm, &lo, &hi);
    for (int64_t n = lo; n <= hi; ++n) {
        double tau0 = tm->t0 + (double)n * dtk;
        double tau1 = tm->t0 + (double)(n + 1) * dtk;
        double u0 = rho - tm->c * tau0;
        double u1 = rho - tm->c * tau1;
        if (tm->sampling == ORC_POINT) {
            row[n] += p0 * dir * u0 * fhat(u0, a, tm) / (2.0 * rho);
        } else {
            row[n] += p0 * dir * (psi(u0, a, tm) - psi(u1, a, tm)) / (2.0 * rho * tm->c * dtk);
        }
    }
}

/*
 * y[r][n] (rows r = 0..R-1, row r is transducer det_idx[r], or r itself when
 * det_idx is NULL) = sum over all balls of the pair traces.
 * Parallel over rows: each thread owns its rows, no shared writes.
 */
void orc_simulate(int64_t B, const double *bx, const double *by, const double *bz,
                  const double *bp, const double *ba,
                  int32_t D, const double *qx, const double *qy, const double *qz,
                  const double *nx, const double *ny, const double *nz,
                  const orc_time *tm, int32_t R, const int32_t *det_idx, double *y)
{
    memset(y, 0, sizeof(double) * (size_t)R * (size_t)tm->T);
    (void)D;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t r = 0; r < R; ++r) {
        int32_t d = det_idx ? det_idx[r] : r;
        double *row = y + (size_t)r * (size_t)tm->T;
        for (int64_t i = 0; i < B; ++i)
            pair_trace(bx[i], by[i], bz[i], bp[i], ba[i], qx[d], qy[d], qz[d],
                       nx[d], ny[d], nz[d], tm, row);
    }
}

/* ------------------------------------------------------------ dual numbers */

/* A value with its tangents along (x, y, z, p0, a) of one ball. */
typedef struct { double v; double d[5]; } dual;

static dual dc(double v) { dual r; r.v = v; for (int k = 0; k < 5; ++k) r.d[k] = 0.0; return r; }
static dual dvar(double v, int k) { dual r = dc(v); r.d[k] = 1.0; return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int k = 0; k < 5; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int k = 0; k < 5; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
static dual dmul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int k = 0; k < 5; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
static dual ddiv(dual a, dual b)
{
    dual r; r.v = a.v / b.v;
    for (int k = 0; k < 5; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
    return r;
}
static dual dscale(dual a, double s) { dual r; r.v = a.v * s; for (int k = 0; k < 5; ++k) r.d[k] = a.d[k] * s; return r; }
static dual dsqrt(dual a)
{
    dual r; r.v = sqrt(a.v);
    for (int k = 0; k < 5; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
    return r;
}
static dual dexp(dual a)
{
    dual r; r.v = exp(a.v);
    for (int k = 0; k < 5; ++k) r.d[k] = a.d[k] * r.v;
    return r;
}

/* psi(u; a) with both u and a carrying tangents. */
static dual dpsi(dual u, dual a, const orc_time *tm)
{
    if (tm->profile == ORC_UNIFORM) {
        if (!(fabs(u.v) < a.v)) return dc(0.0);
        return dscale(dsub(dmul(a, a), dmul(u, u)), -0.5);
    }
    if (!(fabs(u.v) < tm->K * a.v)) return dc(0.0);
    dual arg = ddiv(dmul(u, u), dscale(dmul(a, a), 2.0));
    dual e = dexp(dscale(arg, -1.0));
    dual inner = dsub(e, dc(exp(-0.5 * tm->K * tm->K)));
    return dscale(dmul(dmul(a, a), inner), -1.0);
}

/* fhat(u; a) * u with tangents (POINT sampling). */
static dual dufhat(dual u, dual a, const orc_time *tm)
{
    if (tm->profile == ORC_UNIFORM)
        return fabs(u.v) < a.v ? u : dc(0.0);
    if (!(fabs(u.v) < tm->K * a.v)) return dc(0.0);
    dual arg = ddiv(dmul(u, u), dscale(dmul(a, a), 2.0));
    return dmul(u, dexp(dscale(arg, -1.0)));
}

/* Contract one pair's bin tangents with the cotangent row vrow[0..T). */
static void pair_vjp(double bx, double by, double bz, double p0, double a,
                     double qx, double qy, double qz, double nx, double ny, double nz,
                     const orc_time *tm, const double *vrow, double g[5])
{
    if (!(a > 0.0)) return;
    dual X = dvar(bx, 0), Y = dvar(by, 1), Z = dvar(bz, 2), P = dvar(p0, 3), A = dvar(a, 4);
    dual dx = dsub(X, dc(qx)), dy = dsub(Y, dc(qy)), dz = dsub(Z, dc(qz));
    dual rho = dsqrt(dadd(dadd(dmul(dx, dx), dmul(dy, dy)), dmul(dz, dz)));
    double w = half_width(a, tm);
    if (rho.v <= w) return;
    dual dir = dc(1.0);
    if (tm->directivity == ORC_COS) {
        dual cosv = ddiv(dadd(dadd(dscale(dx, nx), dscale(dy, ny)), dscale(dz, nz)), rho);
        dir = cosv.v > 0.0 ? cosv : dc(0.0);
    }
    if (dir.v == 0.0) return;
    double dtk = tm->f * tm->dt;
    dual amp;
    if (tm->sampling == ORC_POINT)
        amp = ddiv(dmul(P, dir), dscale(rho, 2.0));
    else
        amp = ddiv(dmul(P, dir), dscale(rho, 2.0 * tm->c * dtk));
    int64_t lo, hi;
    bin_range(rho.v, w, tm, &lo, &hi);
    for (int64_t n = lo; n <= hi; ++n) {
        double vn = vrow[n];
        if (vn == 0.0) continue;
        dual u0 = dsub(rho, dc(tm->c * (tm->t0 + (double)n * dtk)));
        dual val;
        if (tm->sampling == ORC_POINT) {
            val = dmul(amp, dufhat(u0, A, tm));
        } else {
            dual u1 = dsub(rho, dc(tm->c * (tm->t0 + (double)(n + 1) * dtk)));
            val = dmul(amp, dsub(dpsi(u0, A, tm), dpsi(u1, A, tm)));
        }
        for (int k = 0; k < 5; ++k) g[k] += vn * val.d[k];
    }
}

/*
 * grad[k][j] (k over x, y, z, p0, a; j over the selected balls) =
 *   sum over transducers d and bins n of v[d][n] * d y[d][n] / d theta_k(ball).
 * Ball j is ball_idx[j] (or j when ball_idx is NULL).  v is [D][T].
 * Parallel over balls: each thread owns its balls' gradients.
 */
void orc_vjp(int64_t B, const double *bx, const double *by, const double *bz,
             const double *bp, const double *ba,
             int32_t D, const double *qx, const double *qy, const double *qz,
             const double *nx, const double *ny, const double *nz,
             const orc_time *tm, const double *v, int64_t J, const int64_t *ball_idx,
             double *grad)
{
    (void)B;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < J; ++j) {
        int64_t i = ball_idx ? ball_idx[j] : j;
        double g[5] = {0, 0, 0, 0, 0};
        for (int32_t d = 0; d < D; ++d)
            pair_vjp(bx[i], by[i], bz[i], bp[i], ba[i], qx[d], qy[d], qz[d],
                     nx[d], ny[d], nz[d], tm, v + (size_t)d * (size_t)tm->T, g);
        for (int k = 0; k < 5; ++k) grad[(size_t)k * (size_t)J + (size_t)j] = g[k];
    }
}

/* Number of OpenMP threads the oracle runs with (reported beside timings). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads (the single-thread timing beside the
 * all-core one); returns the number now in use. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return orc_num_threads();
}
