// Host build of the adjoint's per-pair arithmetic (csrc/adjoint_pair.hpp),
// FP64 instantiation, driven the way the kernel drives it: for every ball and
// transducer the pre-differenced cotangent row is staged in time tiles of TT
// edges and adj_pair accumulates the five gradient sums tile by tile.  Test
// infrastructure: tests/test_adjoint_host.py compares the result with the
// CPU oracle.  Compiled for the host only (no GPU code).
#include <cstdint>
#include <vector>

#include "../../paper_2601_00551_amd/csrc/adjoint_pair.hpp"

using namespace sbp;

template <int PROF, int DIR>
static void run(int64_t B, const double *const *b, int D, const double *const *q, const Level &lc,
                const double *v, int TT, double *grad) {
    const int T = lc.T;
    std::vector<double> w((size_t)TT);
    for (int64_t i = 0; i < B; ++i) {
        double acc[5] = {0, 0, 0, 0, 0};
        const BallK<double, PROF> bk = load_ball<double, PROF>(b[0][i], b[1][i], b[2][i], b[3][i], b[4][i], lc);
        if (bk.live) {
            for (int d = 0; d < D; ++d) {
                const double *vr = v + (size_t)d * T;
                for (int tlo = 0; tlo <= T; tlo += TT) {
                    const int thi = tlo + TT < T + 1 ? tlo + TT : T + 1;
                    // staged edges w_m = v_m - v_{m-1}, v zero outside [0, T)
                    for (int m = tlo; m < thi; ++m)
                        w[m - tlo] = (m < T ? vr[m] : 0.0) - (m > 0 ? vr[m - 1] : 0.0);
                    adj_pair<double, PROF, DIR, true>(bk, q[0][d], q[1][d], q[2][d], q[3][d], q[4][d], q[5][d],
                                                      lc, tlo, thi, w.data(), vr, 1.0, acc);
                }
            }
        }
        for (int k = 0; k < 5; ++k) grad[(size_t)k * B + i] = acc[k];
    }
}

extern "C" int host_adjoint_f64(int64_t B, const double *x, const double *y, const double *z,
                                const double *p0, const double *a, int D, const double *qx,
                                const double *qy, const double *qz, const double *nx,
                                const double *ny, const double *nz, const sbp_model *m,
                                const double *v, int TT, double *grad) {
    const Level lc = make_level(m);
    const double *b[5] = {x, y, z, p0, a};
    const double *q[6] = {qx, qy, qz, nx, ny, nz};
    if (TT < 1) return -1;
    if (m->profile == SBP_PROFILE_GAUSS) {
        if (m->directivity == SBP_DIR_COS) run<GAUSS, COS>(B, b, D, q, lc, v, TT, grad);
        else run<GAUSS, OMNI>(B, b, D, q, lc, v, TT, grad);
    } else {
        if (m->directivity == SBP_DIR_COS) run<UNIFORM, COS>(B, b, D, q, lc, v, TT, grad);
        else run<UNIFORM, OMNI>(B, b, D, q, lc, v, TT, grad);
    }
    return 0;
}
