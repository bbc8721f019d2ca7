/*
 * Host-only driver that runs the C oracle (oracle/sbp_oracle.c) under
 * AddressSanitizer and UndefinedBehaviorSanitizer: the forward and the VJP for
 * every profile, directivity and sampling mode, on small scenes that include
 * the edge cases (a pulse clipped by either end of the record, a ball whose
 * support reaches the transducer, a ball of size zero, a one-sample record,
 * a selection of rows and of balls).  Besides the sanitizers' own checks it
 * requires finite outputs and, for bin means of pulses inside the record, a
 * zero sum over each row.  Test infrastructure, built and run by
 * tests/test_oracle_sanitizers.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    double c, dt, t0, K;
    int32_t T, f, profile, directivity, sampling, pad_;
} orc_time;

void orc_simulate(int64_t B, const double *bx, const double *by, const double *bz,
                  const double *bp, const double *ba, int32_t D, const double *qx,
                  const double *qy, const double *qz, const double *nx, const double *ny,
                  const double *nz, const orc_time *tm, int32_t R, const int32_t *det_idx,
                  double *y);
void orc_vjp(int64_t B, const double *bx, const double *by, const double *bz, const double *bp,
             const double *ba, int32_t D, const double *qx, const double *qy, const double *qz,
             const double *nx, const double *ny, const double *nz, const orc_time *tm,
             const double *v, int64_t J, const int64_t *ball_idx, double *grad);

static unsigned long long g_state = 88172645463325252ull;
static double urand(void) {
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) / 9007199254740992.0;
}

static int fail(const char *what, int a, int b, int c) {
    fprintf(stderr, "FAILED %s (profile %d directivity %d sampling %d)\n", what, a, b, c);
    return 1;
}

static int run_case(int profile, int directivity, int sampling, int T) {
    enum { B = 9, D = 5 };
    double bx[B], by[B], bz[B], bp[B], ba[B];
    double qx[D], qy[D], qz[D], nx[D], ny[D], nz[D];
    for (int d = 0; d < D; ++d) {
        const double th = 0.4 + 0.3 * d;
        qx[d] = 12.0 * sin(th);
        qy[d] = 0.5 * d;
        qz[d] = -12.0 * cos(th);
        const double r = sqrt(qx[d] * qx[d] + qy[d] * qy[d] + qz[d] * qz[d]);
        nx[d] = -qx[d] / r;
        ny[d] = -qy[d] / r;
        nz[d] = -qz[d] / r;
    }
    for (int i = 0; i < B; ++i) {
        bx[i] = 4.0 * (urand() - 0.5);
        by[i] = 4.0 * (urand() - 0.5);
        bz[i] = 4.0 * (urand() - 0.5);
        bp[i] = 0.5 + 0.5 * urand();
        ba[i] = 0.1 + 0.1 * urand();
    }
    /* edge cases: support reaching transducer 0, size zero, far enough that
     * the pulse leaves the end of the record */
    bx[6] = qx[0] + 0.05;
    by[6] = qy[0];
    bz[6] = qz[0];
    ba[7] = 0.0;
    bz[8] = 30.0;
    orc_time tm = {1.5, 0.05, 0.0, 5.0, T, 1, profile, directivity, sampling, 0};
    double *y = calloc((size_t)D * T, sizeof(double));
    double *v = calloc((size_t)D * T, sizeof(double));
    double *g = calloc((size_t)5 * B, sizeof(double));
    if (!y || !v || !g) return fail("allocation", profile, directivity, sampling);
    orc_simulate(B, bx, by, bz, bp, ba, D, qx, qy, qz, nx, ny, nz, &tm, D, NULL, y);
    for (int k = 0; k < D * T; ++k)
        if (!isfinite(y[k])) return fail("finite signal", profile, directivity, sampling);
    /* the record clips the far ball's pulse; without it every pulse lies inside
     * for T = 400, so each row of bin means sums to zero */
    if (sampling == 0 && T == 400) {
        double keep = bz[8];
        bz[8] = 0.0;
        orc_simulate(B, bx, by, bz, bp, ba, D, qx, qy, qz, nx, ny, nz, &tm, D, NULL, y);
        bz[8] = keep;
        for (int d = 1; d < D; ++d) {
            double s = 0.0, m = 0.0;
            for (int n = 0; n < T; ++n) {
                s += y[(size_t)d * T + n];
                m = fmax(m, fabs(y[(size_t)d * T + n]));
            }
            if (fabs(s) > 1e-12 * (m > 0 ? m : 1.0)) return fail("zero sum", profile, directivity, sampling);
        }
    }
    /* a selection of rows */
    int32_t rows[2] = {4, 1};
    orc_simulate(B, bx, by, bz, bp, ba, D, qx, qy, qz, nx, ny, nz, &tm, 2, rows, y);
    for (int k = 0; k < D * T; ++k) v[k] = urand() - 0.5;
    orc_vjp(B, bx, by, bz, bp, ba, D, qx, qy, qz, nx, ny, nz, &tm, v, B, NULL, g);
    for (int k = 0; k < 5 * B; ++k)
        if (!isfinite(g[k])) return fail("finite gradient", profile, directivity, sampling);
    int64_t sel[3] = {8, 0, 6};
    orc_vjp(B, bx, by, bz, bp, ba, D, qx, qy, qz, nx, ny, nz, &tm, v, 3, sel, g);
    for (int k = 0; k < 15; ++k)
        if (!isfinite(g[k])) return fail("finite selected gradient", profile, directivity, sampling);
    free(y);
    free(v);
    free(g);
    return 0;
}

int main(void) {
    int bad = 0, n = 0;
    for (int profile = 0; profile < 2; ++profile)
        for (int dir = 0; dir < 2; ++dir)
            for (int smp = 0; smp < 2; ++smp) {
                if (smp == 1 && profile == 0) continue;   /* point samples: GAUSS only */
                for (int T = 1; T <= 400; T += 399) {
                    bad |= run_case(profile, dir, smp, T);
                    ++n;
                }
            }
    printf("%d cases, %s\n", n, bad ? "failures" : "ok");
    return bad;
}
