// Internal declarations of the MI355X (gfx950) implementation behind sbp.h.
//
// Device-side physics of one (ball, transducer) pair.  A ball is a radially
// symmetric initial pressure p0 * fhat(s) (section 4.1 of SlingBAG Pro); at
// distance rho the pressure is p0 * u * fhat(u) / (2 rho), u = rho - c t, and
// the mean over the time bin [tau_n, tau_{n+1}) is
//     p0 * D * (psi(u_n) - psi(u_{n+1})) / (2 rho c dt_k),
// psi being the antiderivative of u * fhat(u) that vanishes outside the
// support.  Per profile (a = ball size, K = GAUSS truncation):
//     UNIFORM: psi(u) = -(a^2 - u^2) / 2                   for |u| < a
//     GAUSS:   psi(u) = -a^2 (exp(-u^2 / (2 a^2)) - e^{-K^2/2}) for |u| < K a
// Both are written below as amp * max(q(u), 0) so that the support test is a
// single max.  The distance rho and the offset rho - c t of the first edge are
// formed in FP64 (a FP32 rho would move the pulse by up to 4e-6 mm at 70 mm,
// several 1e-5 of its width); the per-edge work is FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "../../include/sbp.h"

// The per-pair arithmetic is also compiled for the host (a test checks its
// FP64 instantiation against the CPU oracle there).
#define SBP_HD __host__ __device__

namespace sbp {

enum { UNIFORM = SBP_PROFILE_UNIFORM, GAUSS = SBP_PROFILE_GAUSS };
// Kernel-internal profile code of GAUSS balls under point sampling (the
// samples are pressure values u fhat(u) p0 D / (2 rho) at the sample times,
// not bin means); its ball constants are GAUSS's.
enum { GPOINT = 2 };

// Internal profile code of a model.
inline int profile_code(const sbp_model *m) {
    return m->sampling == SBP_SAMPLING_POINT ? GPOINT : m->profile;
}
enum { OMNI = SBP_DIR_OMNI, COS = SBP_DIR_COS };

// Per-launch constants of one temporal level.
struct Level {
    double ct0;      // c * t0
    double cdt;      // c * dt_k
    double inv_cdt;  // 1 / (c dt_k)
    double inv2cdt_d;  // 1 / (2 c dt_k)
    double eK_d;     // exp(-K^2 / 2)
    double K_d;      // GAUSS truncation, units of a
    float cdt_f;     // the same, rounded to float
    float inv2cdt;
    float K;
    float eK;
    int T;           // samples at this level
    int a_softplus;  // a arrays hold a~ with a = softplus(a~)
};

// Level constants in the precision R of the kernel instantiation.
template <typename R> struct LevelR;
template <> struct LevelR<float> {
    __device__ static float cdt(const Level &l) { return l.cdt_f; }
    __device__ static float inv2cdt(const Level &l) { return l.inv2cdt; }
    __device__ static float eK(const Level &l) { return l.eK; }
};
template <> struct LevelR<double> {
    SBP_HD static double cdt(const Level &l) { return l.cdt; }
    SBP_HD static double inv2cdt(const Level &l) { return l.inv2cdt_d; }
    SBP_HD static double eK(const Level &l) { return l.eK_d; }
};

inline Level make_level(const sbp_model *m) {
    Level lc;
    const double dtk = (double)m->f * m->dt;
    lc.ct0 = m->c * m->t0;
    lc.cdt = m->c * dtk;
    lc.inv_cdt = 1.0 / lc.cdt;
    lc.inv2cdt_d = 1.0 / (2.0 * lc.cdt);
    lc.K_d = m->gauss_K;
    lc.eK_d = std::exp(-0.5 * m->gauss_K * m->gauss_K);
    lc.cdt_f = (float)lc.cdt;
    lc.inv2cdt = (float)lc.inv2cdt_d;
    lc.K = (float)lc.K_d;
    lc.eK = (float)lc.eK_d;
    lc.T = m->T;
    lc.a_softplus = m->a_softplus;
    return lc;
}

// ------------------------------------------------------------ device math --

// FP32: the hardware instructions (device only); FP64: the library functions.
__device__ inline float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
SBP_HD inline double ex2(double x) { return exp2(x); }
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
SBP_HD inline double rcp(double x) { return 1.0 / x; }

// a = softplus(a~) (identity above 20, as PyTorch) and d a / d a~ = sigmoid(a~).
template <typename R> SBP_HD inline R softplus_dev(R x) {
    return x > R(20) ? x : log1p(exp(x));
}
template <typename R> SBP_HD inline R sigmoid_dev(R x) { return R(1) / (R(1) + exp(-x)); }

// Per-ball constants.
template <typename R, int PROF>
struct BallK {
    R x, y, z;        // centre (widened to FP64 per pair: the difference is exact)
    R w;              // support half-width (a or K a)
    R p, a;           // peak pressure, size
    R q0;             // UNIFORM: a^2        GAUSS: -log2(e) / (2 a^2)
    R ampk;           // UNIFORM: -p / 2     GAUSS: -p a^2
    R h;              // GAUSS: 2^(2 q0 (c dt)^2), the ratio of successive edge ratios
    bool live;        // a > 0
};

// The derived fields of a ball whose x, y, z, p and stored size parameter
// (in b.a) are set.
template <typename R, int PROF>
SBP_HD inline void finish_ball(BallK<R, PROF> &b, const Level &lc) {
    const R a = lc.a_softplus ? softplus_dev(b.a) : b.a;
    const R p = b.p;
    b.a = a;
    b.live = a > R(0);
    if (PROF == UNIFORM) {
        b.w = a;
        b.q0 = a * a;
        b.ampk = R(-0.5) * p;
        b.h = R(1);
    } else {
        b.w = (R)(lc.K_d * (double)a);
        b.q0 = R(-1.4426950408889634) / (R(2) * a * a);
        b.ampk = -p * a * a;
        const R c = LevelR<R>::cdt(lc);
        b.h = ex2(R(2) * b.q0 * c * c);
    }
}

template <typename R, int PROF>
SBP_HD inline BallK<R, PROF> load_ball(R x, R y, R z, R p, R araw, const Level &lc) {
    BallK<R, PROF> b;
    b.x = x;
    b.y = y;
    b.z = z;
    b.p = p;
    b.a = araw;
    finish_ball(b, lc);
    return b;
}

// q(u) such that psi(u) = amp * max(q(u), 0) with amp = ampk * D / (2 rho c dt).
template <typename R, int PROF>
SBP_HD inline R shape_q(R u, const BallK<R, PROF> &b, R eK) {
    if (PROF == UNIFORM) return b.q0 - u * u;
    return ex2(u * u * b.q0) - eK;
}

// Geometry of one pair, shared by the forward and the adjoint.
template <typename R>
struct PairG {
    double s;    // rho - c t0
    R rho;       // distance
    R inv_rho;
    R ex, ey, ez;  // unit vector transducer -> ball
    R dir;       // directivity factor
};

// Returns false if the pair contributes nothing (near field, facing away).
template <typename R, int DIR>
SBP_HD inline bool pair_geometry(R bx, R by, R bz, R w, R qx, R qy, R qz,
                                     R nx, R ny, R nz, const Level &lc, PairG<R> &g) {
    const double dx = (double)bx - (double)qx, dy = (double)by - (double)qy,
                 dz = (double)bz - (double)qz;
    const double r2 = dx * dx + dy * dy + dz * dz;
    double rho;
    R inv_rho;
    if constexpr (sizeof(R) == 4) {
        // FP32 square root refined by one Newton step in FP64: relative error
        // about 1e-14, from a half-rate FP32 root instead of the FP64 one
        const float r0 = __builtin_amdgcn_sqrtf((float)r2);
        const float i0 = __builtin_amdgcn_rcpf(r0);
        rho = fma(fma(-(double)r0, (double)r0, r2), (double)(0.5f * i0), (double)r0);
        inv_rho = (R)i0;
    } else {
        rho = sqrt(r2);
        inv_rho = rcp((R)rho);
    }
    if (!(rho > (double)w)) return false;
    g.s = rho - lc.ct0;
    g.rho = (R)rho;
    g.inv_rho = inv_rho;
    g.ex = (R)dx * g.inv_rho;
    g.ey = (R)dy * g.inv_rho;
    g.ez = (R)dz * g.inv_rho;
    if (DIR == COS) {
        g.dir = nx * g.ex + ny * g.ey + nz * g.ez;
        if (!(g.dir > R(0))) return false;
    } else {
        g.dir = R(1);
    }
    return true;
}

// ------------------------------------------------------------- host side --

struct Ctx {
    int device = 0;
    int num_cus = 0;
    size_t lds_max = 0;
    sbp_tuning tuning{};
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    unsigned *misc = nullptr;  // kMiscBytes persistent bytes (layout below)
    void *fixed_ws = nullptr;  // this device's fixed workspace (device address), see api.hip
};

// Persistent device words of a context (and of a captured graph): word
// kMiscBound holds the forward's fixed-point bound, words kMiscScales.. the
// proposal features' three scales, words kMiscFlags + f one flag per frame
// (set when a ball of frame f has a non-finite parameter).
constexpr size_t kMiscBytes = 512;
constexpr int kMiscBound = 0;
constexpr int kMiscScales = 4;
constexpr int kMiscFlags = 64;
static_assert((kMiscFlags + SBP_MAX_FRAMES) * sizeof(unsigned) <= kMiscBytes, "misc words");

// A ball with a non-finite stored parameter (centre, peak, or the size array
// as stored, a or a~) poisons its frame: the forward writes NaN to every
// sample of that frame and the adjoint writes NaN to every gradient of that
// ball.
template <typename R>
SBP_HD inline bool ball_finite(R x, R y, R z, R p, R a) {
    return isfinite(x) && isfinite(y) && isfinite(z) && isfinite(p) && isfinite(a);
}

// Frame of ball i given the frame offsets (off[0] <= i < off[F]): the largest
// f with off[f] <= i (empty frames are skipped over).
__device__ inline int frame_of(const int64_t *off, int F, int64_t i) {
    int lo = 0, hi = F;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int ensure_scratch(Ctx *c, size_t bytes);

#define SBP_HIP(call)                                          \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return ::sbp::hip_fail(e_, #call); \
    } while (0)

// Launchers (forward.hip, adjoint.hip, elementwise.hip).
template <typename R>
struct ArrayP {
    const R *qx, *qy, *qz, *nx, *ny, *nz;
    int D;
};
template <typename R>
struct BallsP {
    R *x, *y, *z, *p0, *a;
};

// Sum of x over the workgroup in a fixed order (lanes, then waves); the
// result is valid in thread 0.  s_part holds one double per wave.
__device__ inline double block_sum(double x, double *s_part) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) s_part[wid] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += s_part[w];
    return t;
}

// p[0] + p[step] + ... + p[(nsl - 1) step], added in that order (the result
// does not depend on how the loads are issued: eight at a time here, since the
// slices of small clouds are many and the sum is latency-bound).
template <typename R>
__device__ inline R slice_sum(const R *__restrict__ p, int nsl, int64_t step) {
    R s = R(0);
    int sl = 0;
    for (; sl + 8 <= nsl; sl += 8) {
        R v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = p[(int64_t)(sl + j) * step];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; sl < nsl; ++sl) s += p[(int64_t)sl * step];
    return s;
}

// Power-of-two scale with |bin value| * scale <= 2^30 (FP32 path).
__device__ inline float fixed_scale(const unsigned *slot, int profile, const Level &lc) {
    const float pa = __uint_as_float(*slot);
    // point samples: |u e(u)| <= a e^{-1/2} and rho > K a, so |p| < |p0| / (2 K)
    const float bound = profile == GPOINT ? pa * 0.5f / lc.K
                                          : pa * lc.inv2cdt * (profile == GAUSS ? 1.0f / lc.K : 0.5f);
    if (!(bound > 0.0f) || !(bound < 3.0e38f)) return 1.0f;
    int e = 0;
    frexpf(bound, &e);              // bound < 2^e
    int k = 30 - e;
    if (k > 120) k = 120;
    if (k < -120) k = -120;
    return ldexpf(1.0f, k);
}

// b^t for an integer step t >= 0 by repeated squaring: at most 2 log2(t)
// FP64 products, a relative error of about that many ulp (far below the FP32
// rounding of the bias corrections it feeds), where the general pow costs a
// lane about two microseconds of dependent FP64 work.
__device__ inline double step_power(double b, int t) {
    double r = 1.0, x = b;
    for (unsigned n = (unsigned)t; n; n >>= 1) {
        if (n & 1u) r *= x;
        x *= x;
    }
    return r;
}

// Partial sums of the loss per frame (a fixed count: a deterministic order).
constexpr int kLossBlocks = 512;

// The forward inside a reconstruction step (FP32):
//   ws_clean     misc and the integer sums are zero on entry (no fills);
//   clear_after  the conversion zeroes each integer sum once it has read it;
//   sums_only    (GAUSS bins) no conversion: the edge sums stay in the
//                workspace for an adjoint that forms the cotangent from them
//                (AdjSrc);
//   y_ref        when set, the conversion writes v = 2 (y - y_ref) instead of y,
//                and the sums of (y - y_ref)^2 (FP64, kLossBlocks per frame)
//                to partial[F][kLossBlocks].
struct FwdStep {
    bool ws_clean = false;
    bool clear_after = false;
    bool sums_only = false;
    const float *y_ref = nullptr;
    double *partial = nullptr;
};

// misc: kMiscBytes of device words (the fixed-point bound of the FP32 path and
// the per-frame non-finite flags); ws: the FP32 path's per-sample integer sums
// (forward_ws_bytes; none for FP64).
size_t forward_ws_bytes(int F, int D, int T, int64_t B_cap, size_t elem);
template <typename R>
int launch_forward(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls, const int64_t *ball_off,
                   int F, int64_t B_cap, const sbp_model *m, R *y, int accumulate,
                   unsigned *misc, void *ws, size_t ws_bytes, hipStream_t st,
                   const FwdStep *step = nullptr);

// An all-gradient FP32 adjoint that splits the transducers into slices can
// leave the sum of the slices to the Adam kernel that follows it: with
// `defer` given, the launch skips its reduction and reports the partial sums
// (part == NULL when it did not split and wrote the gradients itself).
struct AdjDeferred {
    const float *part = nullptr;
    int nsl = 0;
    int64_t pstride = 0;
};

// The cotangent of a reconstruction step formed inside the adjoint (GAUSS
// bins, FP32, small clouds): each work item stages its rows as
// v = 2 (y - y_ref) from the forward's edge sums (y as the conversion forms
// it, NaN in a flagged frame) and keeps v itself in LDS (for the telescoped
// sum over a pair's edges); the items of each frame's first ball chunk also
// write v to y_work and each row's sum of (y - y_ref)^2 (FP64, in a fixed
// order) to row_loss[f][d].  Rows are staged whole (adjoint_src_fits).
struct AdjSrc {
    const unsigned long long *gacc = nullptr;   // [F][D][T + 1] edge sums
    const float *y_ref = nullptr;               // [F][D][T]
    const unsigned *misc = nullptr;             // fixed-point bound, frame flags
    float *y_work = nullptr;                    // [F][D][T] receives v
    double *row_loss = nullptr;                 // [F][D]
};
// Whether the adjoint can stage whole rows with their cotangents (LDS and the
// tile limit) for this many transducers and samples.
bool adjoint_src_fits(const Ctx *c, int D, int T);

// vscale multiplies v (the filter passes y_ref with vscale = -2).  ws holds the
// per-slice partial gradients when the launch splits the transducers into
// slices (adjoint_ws_bytes of them; with less, the launch does not split).
size_t adjoint_ws_bytes(const Ctx *c, int D, int64_t B_cap, int F, uint32_t mask, size_t elem);
template <typename R>
int launch_adjoint(Ctx *c, const ArrayP<R> &arr, const BallsP<R> &balls, const int64_t *ball_off,
                   int F, int64_t B_cap, const sbp_model *m, const R *v, R vscale,
                   uint32_t mask, const BallsP<R> &grad, void *ws, size_t ws_bytes, hipStream_t st,
                   const int32_t *order = nullptr, AdjDeferred *defer = nullptr,
                   const AdjSrc *src = nullptr);

template <typename R>
int launch_fill(R *p, int64_t n, R value, hipStream_t st);

int launch_downsample(const float *y, int64_t R_, int T, int f, float *out, hipStream_t st);
int launch_decimate(const float *y, int64_t R_, int T, int f, float *out, hipStream_t st);
size_t residual_ws_bytes(int F);
int launch_residual_loss(double *partial_ws, const float *ys, const float *yr, int64_t n, int F,
                         float *v, double *loss, hipStream_t st);
// What the Adam kernel of a reconstruction step also does:
//   part/nsl/pstride  sum the adjoint's transducer slices into the gradients
//                     (in slice order, as the adjoint's own reduction) first;
//   a_softplus        the size gradient then takes the softplus chain factor;
//   loss_partial      reduce partial[F][kLossBlocks] into loss[F] (F extra
//                     workgroups);
//   misc_clear        zero the forward's device words afterwards (so that the
//                     next forward needs no fill);
//   step_add          the step count is *step_dev + step_add.
struct AdamFuse {
    AdjDeferred adj;
    int a_softplus = 0;
    const double *loss_partial = nullptr;
    double *loss = nullptr;
    unsigned *misc_clear = nullptr;
    int step_add = 0;
    // with an AdjSrc adjoint: the loss of a frame is the sum of its D row
    // sums (row_loss); a frame without balls (no adjoint items) gets v and
    // its loss here from y_ref; gacc (n_gacc words) is zeroed for the next
    // forward when set
    const double *row_loss = nullptr;
    int D = 0, T = 0;
    const float *y_ref = nullptr;
    float *y_work = nullptr;
    unsigned long long *gacc = nullptr;
    int64_t n_gacc = 0;
};
int launch_adam(const sbp_state *s, const sbp_adam_params *p, const int32_t *step_dev,
                int a_softplus, hipStream_t st, const AdamFuse *fuse = nullptr);
int launch_incr_by(int32_t *p, int32_t by, hipStream_t st);
size_t compact_ws_bytes(int64_t B_cap);
int launch_compact(void *ws, const float *g, int strict, const BallsP<float> &in,
                   const int64_t *off_in, int F, int64_t B_cap, const BallsP<float> &out,
                   int64_t *off_out, const BallsP<float> *m_in, const BallsP<float> *v_in,
                   const BallsP<float> *m_out, const BallsP<float> *v_out, hipStream_t st);
int launch_incr(int32_t *p, hipStream_t st);
// Spatial visiting order for the gather-form kernels (elementwise.hip):
// order[off[0] + k] lists the frames' balls cell by cell; *order is set to
// NULL (visit in storage order) when the cloud is too large for int32 indices.
size_t order_ws_bytes(int F, int64_t B_cap);
int launch_order(void *ws, const BallsP<float> &b, const int64_t *off, int F, int64_t B_cap,
                 int32_t **order, hipStream_t st);
int launch_reparam(float *a, float *m, float *v, const int64_t *ball_off, int F, int64_t B_cap,
                   int to_softplus, hipStream_t st);
int launch_grow(Ctx *c, const sbp_state *in, const sbp_growth_rule *rule, sbp_state *out,
                int64_t *count, hipStream_t st);

// Transducer response (response.hip): rows records of T samples, record r
// using tap row (rows_h == 1 ? 0 : r mod D); adjoint = 0 convolves, 1
// correlates.  out must not overlap y.
template <typename R>
int launch_response(const float *h, int rows_h, int L, int zero, const R *y, int64_t rows, int D,
                    int T, int adjoint, int accumulate, R *out, hipStream_t st);
int launch_response_taps(const float *fc, const float *bw, int rows, double dt, int L, int zero,
                         float *h, hipStream_t st);

}  // namespace sbp

// The opaque context of the C-ABI.
struct sbp_ctx {
    sbp::Ctx c;
};
