// Forward model (Simulate of section 4.2 / 4.3 of SlingBAG Pro) on gfx950.
//
// Scatter form: a lane owns a ball, loops over a group of `dg` transducers
// whose traces it accumulates in LDS rows (full record length, so no ball is
// culled against a time tile), and for each pair adds its bin values
//     amp * (max(q(u_n), 0) - max(q(u_{n+1}), 0))
// into the row with LDS atomics.  The rows are FP64: on gfx950 an LDS FP64
// atomic add sustains about ten times the rate of the FP32 one (which the
// hardware serialises), and it makes the accumulation over up to ~10^5 balls
// per sample exact to FP32 rounding.  Adding bin values (which sum to zero per
// pair) rather than edge values avoids the cancellation a running
// antiderivative would suffer when many balls overlap in a bin.
//
// Work items are (frame, transducer group, chunk of block*bpt balls), ordered
// frame-major, then group, then chunk.  A persistent workgroup takes one
// contiguous range of items, so consecutive items share a transducer group and
// the LDS rows are flushed to HBM (one global atomic per non-zero sample) only
// when the group or frame changes.  Ball counts are read on the device, so the
// launch is sized by capacity and can be captured in a graph.
#include "sbp_internal.hpp"

namespace sbp {

// Adds the pair's bins that fall in the time tile [tlo, thi) to row[n - tlo].
template <typename R, int PROF, int DIR>
__device__ inline void fwd_pair(const BallK<R, PROF> &b, R qx, R qy, R qz, R nx, R ny, R nz,
                                const Level &lc, int tlo, int thi, double *__restrict__ row) {
    PairG<R> g;
    if (!pair_geometry<R, DIR>(b.x, b.y, b.z, b.w, qx, qy, qz, nx, ny, nz, lc, g)) return;
    const double lo = floor((g.s - b.w) * lc.inv_cdt);
    const double hi = floor((g.s + b.w) * lc.inv_cdt);
    if (hi < (double)tlo || lo > (double)(thi - 1)) return;
    const int nb = lo < (double)tlo ? tlo : (int)lo;
    const int ne = hi > (double)(thi - 1) ? thi - 1 : (int)hi;
    const R amp = b.ampk * g.dir * LevelR<R>::inv2cdt(lc) * g.inv_rho;
    const R eK = LevelR<R>::eK(lc);
    const R cdt = LevelR<R>::cdt(lc);
    const R u0 = (R)(g.s - (double)nb * lc.cdt);
    R prev = amp * fmax(shape_q<R, PROF>(u0, b, eK), R(0));
    R j = R(1);
    double *out = row - tlo;
    for (int n = nb; n <= ne; ++n, j += R(1)) {
        const R u = fma(-j, cdt, u0);
        const R cur = amp * fmax(shape_q<R, PROF>(u, b, eK), R(0));
        atomicAdd(out + n, (double)(prev - cur));
        prev = cur;
    }
}

template <typename R>
__device__ inline void flush_rows(double *__restrict__ rows, int dg, int TT, int T, int g, int tile,
                                  int D, int f, R *__restrict__ y) {
    __syncthreads();
    const int tlo = tile * TT;
    const int len = min(TT, T - tlo);
    for (int dl = 0; dl < dg; ++dl) {
        const int d = g * dg + dl;
        if (d >= D) break;
        R *out = y + ((int64_t)f * D + d) * (int64_t)T + tlo;
        double *row = rows + (int64_t)dl * TT;
        for (int n = threadIdx.x; n < len; n += blockDim.x) {
            const double v = row[n];
            if (v != 0.0) {
                atomicAdd(out + n, (R)v);
                row[n] = 0.0;
            }
        }
    }
    __syncthreads();
}

// Work items are (frame, transducer group g, time tile, ball chunk), in that
// order; nt = number of time tiles of length TT.
template <typename R, int PROF, int DIR>
__global__ __launch_bounds__(512) void k_forward(ArrayP<R> arr, BallsP<R> balls,
                                                 const int64_t *__restrict__ ball_off, int F,
                                                 int G, int dg, int TT, int nt, int bpt, Level lc,
                                                 R *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double *rows = reinterpret_cast<double *>(lds_raw);
    __shared__ int64_t s_off[SBP_MAX_FRAMES + 1];
    __shared__ int64_t s_ipre[SBP_MAX_FRAMES + 1];
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int T = lc.T;
    const int64_t CH = (int64_t)nth * bpt;
    const int64_t GT = (int64_t)G * nt;
    for (int i = tid; i <= F; i += nth) s_off[i] = ball_off[i];
    for (int i = tid; i < dg * TT; i += nth) rows[i] = 0.0;
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
            if (cur_f >= 0) flush_rows(rows, dg, TT, T, cur_gt / nt, cur_gt % nt, D, cur_f, y);
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
                fwd_pair<R, PROF, DIR>(b, arr.qx[d], arr.qy[d], arr.qz[d], arr.nx[d], arr.ny[d],
                                       arr.nz[d], lc, tlo, thi, rows + (int64_t)dl * TT);
            }
        }
    }
    if (cur_f >= 0) flush_rows(rows, dg, TT, T, cur_gt / nt, cur_gt % nt, D, cur_f, y);
}

template <typename R, int PROF, int DIR>
static int run_forward(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls,
                       const int64_t *ball_off, int F, int64_t B_cap, const Level &lc, R *y,
                       hipStream_t st) {
    auto kern = k_forward<R, PROF, DIR>;
    const size_t reserve = 2 * (SBP_MAX_FRAMES + 1) * sizeof(int64_t) + 256;
    const size_t avail = c->lds_max > reserve ? c->lds_max - reserve : 0;
    int dg = c->tuning.fwd_dets;
    if (dg > arr.D) dg = arr.D;
    // time tile: the whole record if the dg rows fit, else the longest that does
    int64_t TT = (int64_t)(avail / ((size_t)dg * sizeof(double)));
    if (TT > lc.T) TT = lc.T;
    if (TT < lc.T && TT < 64) return fail(SBP_E_DOMAIN, "LDS too small for %d rows", dg);
    const int nt = (int)((lc.T + TT - 1) / TT);
    const int G = (arr.D + dg - 1) / dg;
    const int block = c->tuning.fwd_block;
    const int bpt = c->tuning.fwd_bpt;
    const size_t lds = (size_t)dg * (size_t)TT * sizeof(double);
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
                       (int)TT, nt, bpt, lc, y);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

template <typename R>
int launch_forward(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls, const int64_t *ball_off,
                   int F, int64_t B_cap, const sbp_model *m, R *y, int accumulate,
                   hipStream_t st) {
    const Level lc = make_level(m);
    if (!accumulate) {
        int rc = launch_fill<R>(y, (int64_t)F * arr.D * m->T, R(0), st);
        if (rc) return rc;
    }
    if (B_cap == 0) return SBP_OK;
    if (m->profile == SBP_PROFILE_GAUSS) {
        if (m->directivity == SBP_DIR_COS)
            return run_forward<R, GAUSS, COS>(c, arr, balls, ball_off, F, B_cap, lc, y, st);
        return run_forward<R, GAUSS, OMNI>(c, arr, balls, ball_off, F, B_cap, lc, y, st);
    }
    if (m->directivity == SBP_DIR_COS)
        return run_forward<R, UNIFORM, COS>(c, arr, balls, ball_off, F, B_cap, lc, y, st);
    return run_forward<R, UNIFORM, OMNI>(c, arr, balls, ball_off, F, B_cap, lc, y, st);
}

template int launch_forward<float>(Ctx *, const ArrayP<float> &, const BallsP<float> &,
                                   const int64_t *, int, int64_t, const sbp_model *, float *, int,
                                   hipStream_t);
template int launch_forward<double>(Ctx *, const ArrayP<double> &, const BallsP<double> &,
                                    const int64_t *, int, int64_t, const sbp_model *, double *,
                                    int, hipStream_t);

}  // namespace sbp
