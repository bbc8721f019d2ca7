// Host side of the C-ABI declared in include/sbp.h: argument validation (all
// of it before anything is enqueued), the context, error reporting, and the
// composition of the kernels into the calls of the reconstruction loop.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "sbp_internal.hpp"

struct sbp_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *ws = nullptr;  // residual partial sums, forward bound and integer sums, adjoint slices (owned)
    int device = 0;
};

namespace sbp {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(SBP_E_HIP, "%s failed: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------ fixed device workspace --
// The workspace of sbp_simulate_signals_noalloc: a file-scope device array,
// one copy per GPU for the life of the process, so that the call allocates
// nothing.  In host code `scratch` names a host-side stand-in, not device
// memory; its device address on each GPU is looked up once per device (with
// that device current) when a context is created there, kept in
// g_fixed_ws[device] and in the context, and only that address is handed to
// kernels.  Every call on one GPU shares the array: the call clears what must
// start at zero, and calls that overlap on one GPU race.
constexpr size_t kFixedWsBytes = (size_t)128 << 20;
constexpr int kFixedWsDevices = 64;
static __device__ __align__(256) unsigned char scratch[kFixedWsBytes];
static std::mutex g_fixed_ws_mu;
static void *g_fixed_ws[kFixedWsDevices];

// Device address of `scratch` on `device`, which must be current.
static int fixed_ws_address(int device, void **out) {
    *out = nullptr;
    if (device >= kFixedWsDevices)
        return fail(SBP_E_ARG, "device %d: the fixed workspace supports devices 0..%d", device,
                    kFixedWsDevices - 1);
    std::lock_guard<std::mutex> lock(g_fixed_ws_mu);
    if (!g_fixed_ws[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(SBP_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_fixed_ws[device] = p;
    }
    *out = g_fixed_ws[device];
    return SBP_OK;
}

int ensure_scratch(Ctx *c, size_t bytes) {
    if (bytes <= c->scratch_bytes) return SBP_OK;
    size_t nb = c->scratch_bytes * 2;
    if (nb < bytes) nb = bytes;
    nb = (nb + 4095) & ~(size_t)4095;
    if (c->scratch) {
        hipError_t e = hipFree(c->scratch);
        c->scratch = nullptr;
        c->scratch_bytes = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree(scratch)");
    }
    if (hipMalloc(&c->scratch, nb) != hipSuccess) {
        c->scratch = nullptr;
        (void)hipGetLastError();
        return fail(SBP_E_NOMEM, "could not allocate %zu bytes of scratch", nb);
    }
    c->scratch_bytes = nb;
    return SBP_OK;
}


// ----------------------------------------------------------- validation --

constexpr double kMaxGaussK = 12.0;

static int check_model(const sbp_model *m) {
    if (!m) return fail(SBP_E_ARG, "model is NULL");
    if (!(m->c > 0.0) || !std::isfinite(m->c)) return fail(SBP_E_DOMAIN, "c must be > 0");
    if (!(m->dt > 0.0) || !std::isfinite(m->dt)) return fail(SBP_E_DOMAIN, "dt must be > 0");
    if (!std::isfinite(m->t0)) return fail(SBP_E_DOMAIN, "t0 must be finite");
    if (m->f < 1) return fail(SBP_E_DOMAIN, "f must be >= 1");
    if (m->T < 1) return fail(SBP_E_DOMAIN, "T must be >= 1");
    if (m->profile != SBP_PROFILE_UNIFORM && m->profile != SBP_PROFILE_GAUSS)
        return fail(SBP_E_DOMAIN, "unknown profile %d", m->profile);
    if (m->directivity != SBP_DIR_OMNI && m->directivity != SBP_DIR_COS)
        return fail(SBP_E_DOMAIN, "unknown directivity %d", m->directivity);
    if (m->a_softplus != 0 && m->a_softplus != 1) return fail(SBP_E_DOMAIN, "a_softplus must be 0 or 1");
    if (m->sampling != SBP_SAMPLING_BIN && m->sampling != SBP_SAMPLING_POINT)
        return fail(SBP_E_DOMAIN, "unknown sampling %d", m->sampling);
    if (m->sampling == SBP_SAMPLING_POINT && m->profile != SBP_PROFILE_GAUSS)
        return fail(SBP_E_DOMAIN, "point sampling is implemented for the GAUSS profile only");
    // the Gaussian recurrences' first ratio reaches exp(K^2 / 2) for balls with
    // a = c dt_k / K: K <= 12 keeps it inside the FP32 range
    if (m->profile == SBP_PROFILE_GAUSS &&
        (!(m->gauss_K > 0.0) || !(m->gauss_K <= kMaxGaussK)))
        return fail(SBP_E_DOMAIN, "gauss_K must be in (0, %g]", kMaxGaussK);
    if (m->reserved != 0) return fail(SBP_E_ARG, "model.reserved must be 0");
    if (m->response) {
        if (m->response_taps < 1 || m->response_taps > SBP_MAX_TAPS)
            return fail(SBP_E_DOMAIN, "response_taps must be in [1, %d]", SBP_MAX_TAPS);
        if (m->response_zero < 0 || m->response_zero >= m->response_taps)
            return fail(SBP_E_DOMAIN, "response_zero must be in [0, response_taps)");
    }
    return SBP_OK;
}

// The response rows must match the array (checked where D is known).
static int check_response_rows(const sbp_model *m, int D) {
    if (m->response && m->response_rows != 1 && m->response_rows != D)
        return fail(SBP_E_ARG, "response_rows must be 1 or D (%d), not %d", D, m->response_rows);
    return SBP_OK;
}

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Scratch for the record before (forward) or after (adjoint) the response.
static size_t response_ws_bytes(const sbp_model *m, int F, int D, size_t elem) {
    return m->response ? up256((size_t)F * (size_t)D * (size_t)m->T * elem) : 0;
}

template <typename R>
static int apply_response(const sbp_model *m, const R *y, int F, int D, int adjoint, int accumulate,
                          R *out, hipStream_t st) {
    return launch_response<R>(m->response, m->response_rows, m->response_taps, m->response_zero,
                              y, (int64_t)F * D, D, m->T, adjoint, accumulate, out, st);
}

// Forward with the model's response: the simulated record goes to `sim`
// (F D T elements of scratch), then its convolution to y.
template <typename R>
static int forward_with_response(Ctx *c, const ArrayP<R> &a, const BallsP<R> &b, const int64_t *off,
                                 int F, int64_t B_cap, const sbp_model *m, R *y, int accumulate,
                                 unsigned *misc, void *ws, size_t ws_bytes, R *sim, hipStream_t st) {
    if (!m->response)
        return launch_forward<R>(c, a, b, off, F, B_cap, m, y, accumulate, misc, ws, ws_bytes, st);
    int rc = launch_forward<R>(c, a, b, off, F, B_cap, m, sim, 0, misc, ws, ws_bytes, st);
    if (rc) return rc;
    return apply_response<R>(m, sim, F, a.D, 0, accumulate, y, st);
}

// Adjoint with the model's response: the cotangent of y is correlated with
// the taps into `vsim` (F D T elements of scratch) first.
template <typename R>
static int adjoint_with_response(Ctx *c, const ArrayP<R> &a, const BallsP<R> &b, const int64_t *off,
                                 int F, int64_t B_cap, const sbp_model *m, const R *v, R vscale,
                                 uint32_t mask, const BallsP<R> &g, void *ws, size_t ws_bytes,
                                 R *vsim, hipStream_t st, const int32_t *order = nullptr) {
    if (m->response) {
        int rc = apply_response<R>(m, v, F, a.D, 1, 0, vsim, st);
        if (rc) return rc;
        v = vsim;
    }
    return launch_adjoint<R>(c, a, b, off, F, B_cap, m, v, vscale, mask, g, ws, ws_bytes, st, order);
}

template <typename A>
static int check_array(const A *a) {
    if (!a) return fail(SBP_E_ARG, "array is NULL");
    if (!a->qx || !a->qy || !a->qz || !a->nx || !a->ny || !a->nz)
        return fail(SBP_E_ARG, "array has a NULL coordinate pointer");
    if (a->D < 1) return fail(SBP_E_ARG, "array D must be >= 1");
    return SBP_OK;
}

// Ball arrays may be NULL only when the capacity is zero.
template <typename B>
static int check_balls(const B *b, const char *what, int64_t B_cap = 1) {
    if (!b) return fail(SBP_E_ARG, "%s is NULL", what);
    if (B_cap == 0) return SBP_OK;
    if (!b->x || !b->y || !b->z || !b->p0 || !b->a) return fail(SBP_E_ARG, "%s has a NULL array", what);
    return SBP_OK;
}

static int check_frames(const int64_t *off, int32_t F, int64_t B_cap) {
    if (!off) return fail(SBP_E_ARG, "ball_off is NULL");
    if (F < 1 || F > SBP_MAX_FRAMES) return fail(SBP_E_ARG, "F must be in [1, %d]", SBP_MAX_FRAMES);
    if (B_cap < 0) return fail(SBP_E_ARG, "B_cap must be >= 0");
    return SBP_OK;
}

template <typename B>
static int check_grad(const B *g, uint32_t mask, int64_t B_cap) {
    if (mask == 0 || (mask & ~SBP_ALL)) return fail(SBP_E_ARG, "mask must be a non-empty subset of SBP_ALL");
    if (!g) return fail(SBP_E_ARG, "grad is NULL");
    if (B_cap == 0) return SBP_OK;
    if (((mask & SBP_X) && !g->x) || ((mask & SBP_Y) && !g->y) || ((mask & SBP_Z) && !g->z) ||
        ((mask & SBP_P0) && !g->p0) || ((mask & SBP_A) && !g->a))
        return fail(SBP_E_ARG, "grad array for a masked parameter is NULL");
    return SBP_OK;
}

static int check_ctx(const sbp_ctx *ctx) {
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    return SBP_OK;
}

static int check_adam(const sbp_adam_params *p, bool need_step) {
    if (!p) return fail(SBP_E_ARG, "adam params are NULL");
    if (p->mask == 0 || (p->mask & ~SBP_ALL)) return fail(SBP_E_ARG, "adam mask must be a non-empty subset of SBP_ALL");
    if (!(p->beta1 >= 0.0f && p->beta1 < 1.0f) || !(p->beta2 >= 0.0f && p->beta2 < 1.0f))
        return fail(SBP_E_DOMAIN, "betas must be in [0, 1)");
    if (!(p->eps >= 0.0f)) return fail(SBP_E_DOMAIN, "eps must be >= 0");
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(p->lr[k])) return fail(SBP_E_DOMAIN, "lr must be finite");
    if (need_step && p->step < 1) return fail(SBP_E_DOMAIN, "step must be >= 1");
    return SBP_OK;
}

static int check_state(const sbp_state *s, uint32_t mask, bool need_moments) {
    if (!s) return fail(SBP_E_ARG, "state is NULL");
    int rc = check_frames(s->ball_off, s->F, s->B_cap);
    if (rc) return rc;
    rc = check_balls(&s->balls, "state.balls", s->B_cap);
    if (rc) return rc;
    if (s->B_cap == 0) return SBP_OK;
    const float *g[5] = {s->grad.x, s->grad.y, s->grad.z, s->grad.p0, s->grad.a};
    const float *m[5] = {s->m.x, s->m.y, s->m.z, s->m.p0, s->m.a};
    const float *v[5] = {s->v.x, s->v.y, s->v.z, s->v.p0, s->v.a};
    for (int k = 0; k < 5; ++k) {
        if (!(mask & (1u << k))) continue;
        if (!g[k]) return fail(SBP_E_ARG, "state.grad array for a masked parameter is NULL");
        if (need_moments && (!m[k] || !v[k]))
            return fail(SBP_E_ARG, "state moment array for a masked parameter is NULL");
    }
    return SBP_OK;
}

template <typename R, typename A>
static ArrayP<R> arrp(const A *a) {
    return ArrayP<R>{a->qx, a->qy, a->qz, a->nx, a->ny, a->nz, a->D};
}

template <typename R, typename B>
static BallsP<R> ballsp(const B *b) {
    return BallsP<R>{b->x, b->y, b->z, b->p0, b->a};
}

static int set_device(const Ctx &c) {
    SBP_HIP(hipSetDevice(c.device));
    return SBP_OK;
}

static int check_tuning(const sbp_tuning *t) {
    if (!t) return fail(SBP_E_ARG, "tuning is NULL");
    auto okb = [](int b) { return b == 64 || b == 128 || b == 256 || b == 512; };
    if (t->fwd_dets < 1 || t->fwd_dets > 16 || t->adj_dets < 1 || t->adj_dets > 16)
        return fail(SBP_E_DOMAIN, "dets must be in [1, 16]");
    if (!okb(t->fwd_block) || !okb(t->adj_block)) return fail(SBP_E_DOMAIN, "block must be 64, 128, 256 or 512");
    if (t->fwd_bpt < 1 || t->fwd_bpt > 16) return fail(SBP_E_DOMAIN, "fwd_bpt must be in [1, 16]");
    if (t->adj_bpt < 1 || t->adj_bpt > 3) return fail(SBP_E_DOMAIN, "adj_bpt must be in [1, 3]");
    if (t->fwd_grid < 0 || t->adj_grid < 0) return fail(SBP_E_DOMAIN, "grid must be >= 0");
    if ((t->fwd_tile != 0 && t->fwd_tile < 64) || (t->adj_tile != 0 && t->adj_tile < 64))
        return fail(SBP_E_DOMAIN, "tile must be 0 or >= 64");
    return SBP_OK;
}

// One iteration, shared by sbp_step and the graph capture: forward, residual
// and loss, adjoint, Adam.  Without a transducer response it runs as four
// kernels after the forward's prep: the forward's conversion writes
// v = 2 (y - y_ref) and the loss partial sums, and the Adam kernel adds the
// adjoint's transducer slices and reduces the loss (the same bits as the
// separate kernels).  On a small GAUSS-bin cloud whose rows the adjoint can
// stage whole (adjoint_src_fits) there is no conversion: the adjoint forms
// v from the edge sums as it stages its rows (AdjSrc; the frames' first ball
// chunks write y_work and each row's loss sum to `partial`, which then holds
// F x D row sums), and Adam sums the rows, covers the frames without balls
// and, in a captured sequence, zeroes the edge sums.  y_aux: F D T floats of scratch
// when the model has a response (the simulated record before it, then the
// correlated cotangent).  `captured`: the forward's integer sums and device
// words are zero on entry and are left zero (the conversion clears the sums,
// Adam the words), so a captured sequence fills them once per launch; the
// step count is *step_dev + step_add.
// Pairs (balls x transducers) up to which a step forms the cotangent inside
// the adjoint (clouds whose kernels cost about their launch and latency).
constexpr double kSrcPairs = 2.0e7;

// Bytes of a step's loss sums: F x kLossBlocks partial sums, or F x D row sums.
static size_t step_res_bytes(int F, int D) {
    return (size_t)F * (size_t)(D > kLossBlocks ? D : kLossBlocks) * sizeof(double);
}

static int step_body(Ctx *c, const sbp_array *arr, sbp_state *s, const sbp_model *model,
                     const float *y_ref, float *y_work, const sbp_adam_params *p,
                     const int32_t *step_dev, double *loss, double *partial, unsigned *misc,
                     void *fwd_ws, size_t fwd_ws_bytes, void *adj_ws, size_t adj_ws_bytes,
                     float *y_aux, hipStream_t st, bool captured = false, int step_add = 0) {
    const ArrayP<float> a = arrp<float>(arr);
    const BallsP<float> b = ballsp<float>(&s->balls);
    const BallsP<float> g = ballsp<float>(&s->grad);
    const int64_t n = (int64_t)arr->D * model->T;
    const bool fused = !model->response && s->B_cap > 0;
    const bool src_mode = fused && profile_code(model) == GAUSS &&
                          (double)s->B_cap * arr->D <= kSrcPairs &&
                          adjoint_src_fits(c, arr->D, model->T);
    int rc;
    if (fused) {
        FwdStep fs;
        fs.ws_clean = captured;
        fs.clear_after = captured;
        fs.sums_only = src_mode;
        fs.y_ref = src_mode ? nullptr : y_ref;
        fs.partial = src_mode ? nullptr : partial;
        rc = launch_forward<float>(c, a, b, s->ball_off, s->F, s->B_cap, model, y_work, 0, misc,
                                   fwd_ws, fwd_ws_bytes, st, &fs);
    } else {
        rc = forward_with_response<float>(c, a, b, s->ball_off, s->F, s->B_cap, model, y_work, 0,
                                          misc, fwd_ws, fwd_ws_bytes, y_aux, st);
        if (!rc) rc = launch_residual_loss(partial, y_work, y_ref, n, s->F, y_work, loss, st);
    }
    if (rc) return rc;
    AdamFuse af;
    if (model->response) {
        rc = adjoint_with_response<float>(c, a, b, s->ball_off, s->F, s->B_cap, model, y_work,
                                          1.0f, p->mask, g, adj_ws, adj_ws_bytes, y_aux, st);
    } else {
        AdjSrc src;
        if (src_mode) {
            src.gacc = (const unsigned long long *)fwd_ws;
            src.y_ref = y_ref;
            src.misc = misc;
            src.y_work = y_work;
            src.row_loss = partial;
        }
        rc = launch_adjoint<float>(c, a, b, s->ball_off, s->F, s->B_cap, model, y_work, 1.0f,
                                   p->mask, g, adj_ws, adj_ws_bytes, st, nullptr, &af.adj,
                                   src_mode ? &src : nullptr);
    }
    if (rc) return rc;
    af.a_softplus = model->a_softplus;
    if (fused) {
        af.loss = loss;
        if (src_mode) {
            af.row_loss = partial;
            af.D = arr->D;
            af.T = model->T;
            af.y_ref = y_ref;
            af.y_work = y_work;
            if (captured) {
                af.gacc = (unsigned long long *)fwd_ws;
                af.n_gacc = (int64_t)s->F * arr->D * ((int64_t)model->T + 1);
            }
        } else {
            af.loss_partial = partial;
        }
    }
    // the forward left its device words set; in a captured sequence Adam
    // clears them for the next forward (with fills skipped on entry).  Any
    // forward that did not clear its sums (no fused conversion) breaks that,
    // so a captured step always fuses or fills.
    if (captured && fused) af.misc_clear = misc;
    af.step_add = step_add;
    return launch_adam(s, p, step_dev, model->a_softplus, st, &af);
}

}  // namespace sbp

using namespace sbp;

extern "C" {

const char *sbp_last_error(void) { return g_err; }

int sbp_ctx_create(sbp_ctx **out, int device) {
    g_err[0] = 0;
    if (!out) return fail(SBP_E_ARG, "out is NULL");
    *out = nullptr;
    if (device < 0) return fail(SBP_E_ARG, "device must be >= 0");
    int n = 0;
    SBP_HIP(hipGetDeviceCount(&n));
    if (device >= n) return fail(SBP_E_HIP, "device %d does not exist (%d visible)", device, n);
    SBP_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    SBP_HIP(hipGetDeviceProperties(&prop, device));
    sbp_ctx *ctx = new sbp_ctx();
    ctx->c.device = device;
    ctx->c.num_cus = prop.multiProcessorCount;
    size_t lds = prop.sharedMemPerBlock;
    if (prop.maxSharedMemoryPerMultiProcessor > lds) lds = prop.maxSharedMemoryPerMultiProcessor;
    ctx->c.lds_max = lds;
    ctx->c.tuning = sbp_tuning{4, 512, 4, 0, 4, 512, 3, 0, 0, 0};
    if (hipMalloc((void **)&ctx->c.misc, kMiscBytes) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return fail(SBP_E_NOMEM, "could not allocate the context's device words");
    }
    int rc = fixed_ws_address(device, &ctx->c.fixed_ws);
    if (rc) {
        (void)hipFree(ctx->c.misc);
        delete ctx;
        return rc;
    }
    *out = ctx;
    return SBP_OK;
}

int sbp_ctx_destroy(sbp_ctx *ctx) {
    if (!ctx) return SBP_OK;
    int rc = SBP_OK;
    if (ctx->c.scratch || ctx->c.misc) {
        if (hipSetDevice(ctx->c.device) != hipSuccess) rc = fail(SBP_E_HIP, "hipSetDevice failed");
        if (ctx->c.scratch && hipFree(ctx->c.scratch) != hipSuccess)
            rc = fail(SBP_E_HIP, "hipFree(scratch) failed");
        if (ctx->c.misc && hipFree(ctx->c.misc) != hipSuccess)
            rc = fail(SBP_E_HIP, "hipFree(misc) failed");
    }
    delete ctx;
    return rc;
}

int sbp_ctx_num_cus(const sbp_ctx *ctx, int32_t *out) {
    if (!out) return fail(SBP_E_ARG, "out is NULL");
    int rc = check_ctx(ctx);
    if (rc) return rc;
    *out = ctx->c.num_cus;
    return SBP_OK;
}

int sbp_ctx_set_tuning(sbp_ctx *ctx, const sbp_tuning *t) {
    int rc = check_tuning(t);
    if (rc) return rc;
    rc = check_ctx(ctx);
    if (rc) return rc;
    ctx->c.tuning = *t;
    return SBP_OK;
}

int sbp_ctx_get_tuning(const sbp_ctx *ctx, sbp_tuning *t) {
    if (!t) return fail(SBP_E_ARG, "tuning is NULL");
    int rc = check_ctx(ctx);
    if (rc) return rc;
    *t = ctx->c.tuning;
    return SBP_OK;
}

int sbp_downsample(sbp_ctx *ctx, const float *y, int64_t R, int32_t T, int32_t f, float *y_out,
                   void *stream) {
    if (!y || !y_out) return fail(SBP_E_ARG, "y or y_out is NULL");
    if (R < 1) return fail(SBP_E_ARG, "R must be >= 1");
    if (f < 1) return fail(SBP_E_DOMAIN, "f must be >= 1");
    if (T < 1 || T / f < 1) return fail(SBP_E_DOMAIN, "T / f must be >= 1");
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = set_device(ctx->c))) return rc;
    return launch_downsample(y, R, T, f, y_out, (hipStream_t)stream);
}

int sbp_decimate(sbp_ctx *ctx, const float *y, int64_t R, int32_t T, int32_t f, float *y_out,
                 void *stream) {
    if (!y || !y_out) return fail(SBP_E_ARG, "y or y_out is NULL");
    if (R < 1) return fail(SBP_E_ARG, "R must be >= 1");
    if (f < 1) return fail(SBP_E_DOMAIN, "f must be >= 1");
    if (T < 1 || T / f < 1) return fail(SBP_E_DOMAIN, "T / f must be >= 1");
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = set_device(ctx->c))) return rc;
    return launch_decimate(y, R, T, f, y_out, (hipStream_t)stream);
}

int sbp_simulate_signals(sbp_ctx *ctx, const sbp_array *arr, const sbp_balls *balls,
                         const int64_t *ball_off, int32_t F, int64_t B_cap, const sbp_model *model,
                         float *y, int32_t accumulate, void *stream) {
    int rc;
    if ((rc = check_array(arr)) || (rc = check_frames(ball_off, F, B_cap)) ||
        (rc = check_balls(balls, "balls", B_cap)))
        return rc;
    if (!y) return fail(SBP_E_ARG, "y is NULL");
    if (accumulate != 0 && accumulate != 1) return fail(SBP_E_ARG, "accumulate must be 0 or 1");
    if ((rc = check_model(model)) || (rc = check_response_rows(model, arr->D)) ||
        (rc = check_ctx(ctx)))
        return rc;
    if ((rc = set_device(ctx->c))) return rc;
    // scratch: [forward integer sums and ball constants][record before the response]
    const size_t wsb = up256(forward_ws_bytes(F, arr->D, model->T, B_cap, sizeof(float)));
    const size_t rb = response_ws_bytes(model, F, arr->D, sizeof(float));
    if ((rc = ensure_scratch(&ctx->c, wsb + rb))) return rc;
    return forward_with_response<float>(&ctx->c, arrp<float>(arr), ballsp<float>(balls), ball_off,
                                        F, B_cap, model, y, accumulate, ctx->c.misc,
                                        ctx->c.scratch, wsb,
                                        (float *)((char *)ctx->c.scratch + wsb),
                                        (hipStream_t)stream);
}

int sbp_simulate_signals_noalloc(sbp_ctx *ctx, const sbp_array *arr, const sbp_balls *balls,
                                 const int64_t *ball_off, int32_t F, int64_t B_cap,
                                 const sbp_model *model, float *y, int32_t accumulate,
                                 void *stream) {
    int rc;
    if ((rc = check_array(arr)) || (rc = check_frames(ball_off, F, B_cap)) ||
        (rc = check_balls(balls, "balls", B_cap)))
        return rc;
    if (!y) return fail(SBP_E_ARG, "y is NULL");
    if (accumulate != 0 && accumulate != 1) return fail(SBP_E_ARG, "accumulate must be 0 or 1");
    if ((rc = check_model(model)) || (rc = check_response_rows(model, arr->D))) return rc;
    const size_t wsb = up256(forward_ws_bytes(F, arr->D, model->T, B_cap, sizeof(float)));
    const size_t rb = response_ws_bytes(model, F, arr->D, sizeof(float));
    if (wsb + rb > kFixedWsBytes - kMiscBytes)
        return fail(SBP_E_CAPACITY,
                    "this call needs %zu bytes of workspace; the fixed workspace holds %zu "
                    "(8 (T + 1) F D + 24 B_cap bytes, plus 4 T F D with a response, rounded, "
                    "must fit)",
                    wsb + rb, kFixedWsBytes - kMiscBytes);
    if ((rc = check_ctx(ctx))) return rc;
    if (!ctx->c.fixed_ws) return fail(SBP_E_HIP, "the context has no fixed workspace address");
    if ((rc = set_device(ctx->c))) return rc;
    // [device words (bound, frame flags)][forward integer sums and ball constants]
    // [record before the response]
    char *base = (char *)ctx->c.fixed_ws;
    return forward_with_response<float>(&ctx->c, arrp<float>(arr), ballsp<float>(balls), ball_off,
                                        F, B_cap, model, y, accumulate, (unsigned *)base,
                                        base + kMiscBytes, wsb,
                                        (float *)(base + kMiscBytes + wsb), (hipStream_t)stream);
}

int sbp_response_length(double fc, double bw, double dt_k, double n_sigma, int32_t *L,
                        int32_t *zero) {
    if (!L || !zero) return fail(SBP_E_ARG, "L or zero is NULL");
    auto pos = [](double v) { return v > 0.0 && std::isfinite(v); };
    if (!pos(fc) || !pos(bw) || !pos(dt_k) || !pos(n_sigma))
        return fail(SBP_E_DOMAIN, "fc, bw, dt_k and n_sigma must be positive and finite");
    const double s_f = bw * fc / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const double s_t = 1.0 / (2.0 * M_PI * s_f);
    const double half = std::ceil(n_sigma * s_t / dt_k);
    if (!(2.0 * half + 1.0 <= SBP_MAX_TAPS))
        return fail(SBP_E_CAPACITY, "the response needs %.0f taps (at most %d)", 2.0 * half + 1.0,
                    SBP_MAX_TAPS);
    *zero = (int32_t)half;
    *L = 2 * (int32_t)half + 1;
    return SBP_OK;
}

int sbp_response_taps(sbp_ctx *ctx, const float *fc, const float *bw, int32_t rows, double dt_k,
                      int32_t L, int32_t zero, float *h, void *stream) {
    if (!fc || !bw || !h) return fail(SBP_E_ARG, "fc, bw or h is NULL");
    if (rows < 1) return fail(SBP_E_ARG, "rows must be >= 1");
    if (!(dt_k > 0.0) || !std::isfinite(dt_k)) return fail(SBP_E_DOMAIN, "dt_k must be > 0");
    if (L < 1 || L > SBP_MAX_TAPS) return fail(SBP_E_DOMAIN, "L must be in [1, %d]", SBP_MAX_TAPS);
    if (zero < 0 || zero >= L) return fail(SBP_E_DOMAIN, "zero must be in [0, L)");
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = set_device(ctx->c))) return rc;
    return launch_response_taps(fc, bw, rows, dt_k, L, zero, h, (hipStream_t)stream);
}

int sbp_response_apply(sbp_ctx *ctx, const float *h, int32_t rows_h, int32_t L, int32_t zero,
                       const float *y, int64_t R, int32_t D, int32_t T, int32_t adjoint,
                       int32_t accumulate, float *out, void *stream) {
    if (!h || !y || !out) return fail(SBP_E_ARG, "h, y or out is NULL");
    if (R < 1 || D < 1) return fail(SBP_E_ARG, "R and D must be >= 1");
    if (rows_h != 1 && rows_h != D) return fail(SBP_E_ARG, "rows_h must be 1 or D");
    if (rows_h == D && R % D) return fail(SBP_E_ARG, "R must be a multiple of D");
    if ((adjoint != 0 && adjoint != 1) || (accumulate != 0 && accumulate != 1))
        return fail(SBP_E_ARG, "adjoint and accumulate must be 0 or 1");
    if (T < 1) return fail(SBP_E_DOMAIN, "T must be >= 1");
    if (L < 1 || L > SBP_MAX_TAPS) return fail(SBP_E_DOMAIN, "L must be in [1, %d]", SBP_MAX_TAPS);
    if (zero < 0 || zero >= L) return fail(SBP_E_DOMAIN, "zero must be in [0, L)");
    const uintptr_t y0 = (uintptr_t)y, o0 = (uintptr_t)out;
    const uintptr_t nbytes = (uintptr_t)R * (uintptr_t)T * sizeof(float);
    if (y0 < o0 + nbytes && o0 < y0 + nbytes) return fail(SBP_E_ARG, "out overlaps y");
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = set_device(ctx->c))) return rc;
    return launch_response<float>(h, rows_h, L, zero, y, R, D, T, adjoint, accumulate, out,
                                  (hipStream_t)stream);
}

int sbp_simulate_signals_f64(sbp_ctx *ctx, const sbp_array_f64 *arr, const sbp_balls_f64 *balls,
                             const int64_t *ball_off, int32_t F, int64_t B_cap,
                             const sbp_model *model, double *y, int32_t accumulate, void *stream) {
    int rc;
    if ((rc = check_array(arr)) || (rc = check_frames(ball_off, F, B_cap)) ||
        (rc = check_balls(balls, "balls", B_cap)))
        return rc;
    if (!y) return fail(SBP_E_ARG, "y is NULL");
    if (accumulate != 0 && accumulate != 1) return fail(SBP_E_ARG, "accumulate must be 0 or 1");
    if ((rc = check_model(model)) || (rc = check_response_rows(model, arr->D)) ||
        (rc = check_ctx(ctx)))
        return rc;
    if ((rc = set_device(ctx->c))) return rc;
    const size_t rb = response_ws_bytes(model, F, arr->D, sizeof(double));
    if ((rc = ensure_scratch(&ctx->c, rb))) return rc;
    return forward_with_response<double>(&ctx->c, arrp<double>(arr), ballsp<double>(balls),
                                         ball_off, F, B_cap, model, y, accumulate, ctx->c.misc,
                                         nullptr, 0, (double *)ctx->c.scratch, (hipStream_t)stream);
}

int sbp_residual_loss(sbp_ctx *ctx, const float *y_sim, const float *y_ref, int64_t n_per_frame,
                      int32_t F, float *v_out, double *loss, void *stream) {
    if (!y_sim || !y_ref || !loss) return fail(SBP_E_ARG, "y_sim, y_ref or loss is NULL");
    if (n_per_frame < 0) return fail(SBP_E_ARG, "n_per_frame must be >= 0");
    if (F < 1 || F > SBP_MAX_FRAMES) return fail(SBP_E_ARG, "F must be in [1, %d]", SBP_MAX_FRAMES);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = set_device(ctx->c))) return rc;
    if ((rc = ensure_scratch(&ctx->c, residual_ws_bytes(F)))) return rc;
    return launch_residual_loss((double *)ctx->c.scratch, y_sim, y_ref, n_per_frame, F, v_out, loss,
                                (hipStream_t)stream);
}

int sbp_adjoint_gradients(sbp_ctx *ctx, const sbp_array *arr, const sbp_balls *balls,
                          const int64_t *ball_off, int32_t F, int64_t B_cap,
                          const sbp_model *model, const float *v, uint32_t mask, sbp_balls *grad,
                          void *stream) {
    int rc;
    if ((rc = check_array(arr)) || (rc = check_frames(ball_off, F, B_cap)) ||
        (rc = check_balls(balls, "balls", B_cap)) || (rc = check_grad(grad, mask, B_cap)))
        return rc;
    if (!v) return fail(SBP_E_ARG, "v is NULL");
    if ((rc = check_model(model)) || (rc = check_response_rows(model, arr->D)) ||
        (rc = check_ctx(ctx)))
        return rc;
    if ((rc = set_device(ctx->c))) return rc;
    // scratch: [adjoint slices][cotangent before the response]
    const size_t wsb = up256(adjoint_ws_bytes(&ctx->c, arr->D, B_cap, F, mask, sizeof(float)));
    const size_t rb = response_ws_bytes(model, F, arr->D, sizeof(float));
    if ((rc = ensure_scratch(&ctx->c, wsb + rb))) return rc;
    return adjoint_with_response<float>(&ctx->c, arrp<float>(arr), ballsp<float>(balls), ball_off,
                                        F, B_cap, model, v, 1.0f, mask, ballsp<float>(grad),
                                        ctx->c.scratch, wsb,
                                        (float *)((char *)ctx->c.scratch + wsb),
                                        (hipStream_t)stream);
}

int sbp_adjoint_gradients_f64(sbp_ctx *ctx, const sbp_array_f64 *arr, const sbp_balls_f64 *balls,
                              const int64_t *ball_off, int32_t F, int64_t B_cap,
                              const sbp_model *model, const double *v, uint32_t mask,
                              sbp_balls_f64 *grad, void *stream) {
    int rc;
    if ((rc = check_array(arr)) || (rc = check_frames(ball_off, F, B_cap)) ||
        (rc = check_balls(balls, "balls", B_cap)) || (rc = check_grad(grad, mask, B_cap)))
        return rc;
    if (!v) return fail(SBP_E_ARG, "v is NULL");
    if ((rc = check_model(model)) || (rc = check_response_rows(model, arr->D)) ||
        (rc = check_ctx(ctx)))
        return rc;
    if ((rc = set_device(ctx->c))) return rc;
    const size_t wsb = up256(adjoint_ws_bytes(&ctx->c, arr->D, B_cap, F, mask, sizeof(double)));
    const size_t rb = response_ws_bytes(model, F, arr->D, sizeof(double));
    if ((rc = ensure_scratch(&ctx->c, wsb + rb))) return rc;
    return adjoint_with_response<double>(&ctx->c, arrp<double>(arr), ballsp<double>(balls),
                                         ball_off, F, B_cap, model, v, 1.0, mask,
                                         ballsp<double>(grad), ctx->c.scratch, wsb,
                                         (double *)((char *)ctx->c.scratch + wsb),
                                         (hipStream_t)stream);
}

int sbp_filter_zero_grad(sbp_ctx *ctx, const sbp_array *arr, const sbp_balls *in,
                         const int64_t *off_in, int32_t F, int64_t B_cap, const sbp_model *model,
                         const float *y_ref, int32_t strict, sbp_balls *out, int64_t *off_out,
                         float *g_out, const sbp_balls *m_in, const sbp_balls *v_in,
                         sbp_balls *m_out, sbp_balls *v_out, void *stream) {
    int rc;
    if ((rc = check_array(arr)) || (rc = check_frames(off_in, F, B_cap)) ||
        (rc = check_balls(in, "in", B_cap)) || (rc = check_balls(out, "out", B_cap)))
        return rc;
    if (!y_ref || !off_out) return fail(SBP_E_ARG, "y_ref or off_out is NULL");
    if (strict != 0 && strict != 1) return fail(SBP_E_ARG, "strict must be 0 or 1");
    const bool any_mom = m_in || v_in || m_out || v_out;
    if (any_mom) {
        if ((rc = check_balls(m_in, "m_in", B_cap)) || (rc = check_balls(v_in, "v_in", B_cap)) ||
            (rc = check_balls(m_out, "m_out", B_cap)) || (rc = check_balls(v_out, "v_out", B_cap)))
            return rc;
    }
    if ((rc = check_model(model)) || (rc = check_response_rows(model, arr->D)) ||
        (rc = check_ctx(ctx)))
        return rc;
    if ((rc = set_device(ctx->c))) return rc;
    // scratch: [filter gradient (if g_out is NULL)][compaction workspace][adjoint slices]
    //          [visiting order][reference correlated with the response]
    const size_t g_bytes = g_out ? 0 : up256((size_t)B_cap * sizeof(float));
    const size_t c_bytes = up256(compact_ws_bytes(B_cap));
    const size_t a_bytes = up256(adjoint_ws_bytes(&ctx->c, arr->D, B_cap, F, SBP_P0, sizeof(float)));
    const size_t o_bytes = up256(order_ws_bytes(F, B_cap));
    const size_t r_bytes = response_ws_bytes(model, F, arr->D, sizeof(float));
    if ((rc = ensure_scratch(&ctx->c, g_bytes + c_bytes + a_bytes + o_bytes + r_bytes))) return rc;
    float *g = g_out ? g_out : (float *)ctx->c.scratch;
    void *ws = (char *)ctx->c.scratch + g_bytes;
    hipStream_t st = (hipStream_t)stream;
    // the p0-only gradient visits the balls cell by cell (same values, fewer
    // LDS bank conflicts and divergent lanes)
    int32_t *order = nullptr;
    if (o_bytes &&
        (rc = launch_order((char *)ws + c_bytes + a_bytes, ballsp<float>(in), off_in, F, B_cap,
                           &order, st)))
        return rc;
    BallsP<float> gp{nullptr, nullptr, nullptr, g, nullptr};
    rc = adjoint_with_response<float>(&ctx->c, arrp<float>(arr), ballsp<float>(in), off_in, F, B_cap,
                                      model, y_ref, -2.0f, SBP_P0, gp, (char *)ws + c_bytes,
                                      a_bytes, (float *)((char *)ws + c_bytes + a_bytes + o_bytes),
                                      st, order);
    if (rc) return rc;
    BallsP<float> mi, vi, mo, vo;
    if (any_mom) {
        mi = ballsp<float>(m_in);
        vi = ballsp<float>(v_in);
        mo = ballsp<float>(m_out);
        vo = ballsp<float>(v_out);
    }
    return launch_compact(ws, g, strict, ballsp<float>(in), off_in, F, B_cap, ballsp<float>(out),
                          off_out, any_mom ? &mi : nullptr, any_mom ? &vi : nullptr,
                          any_mom ? &mo : nullptr, any_mom ? &vo : nullptr, st);
}

int sbp_adam_update(sbp_ctx *ctx, sbp_state *state, const sbp_adam_params *p,
                    const int32_t *step_dev, void *stream) {
    int rc;
    if ((rc = check_adam(p, step_dev == nullptr))) return rc;
    if ((rc = check_state(state, p->mask, true))) return rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = set_device(ctx->c))) return rc;
    return launch_adam(state, p, step_dev, 0, (hipStream_t)stream);
}

int sbp_step(sbp_ctx *ctx, const sbp_array *arr, sbp_state *state, const sbp_model *model,
             const float *y_ref, float *y_work, const sbp_adam_params *p, double *loss,
             void *stream) {
    int rc;
    if ((rc = check_array(arr)) || (rc = check_adam(p, true)) ||
        (rc = check_state(state, p->mask, true)))
        return rc;
    if (!y_ref || !y_work || !loss) return fail(SBP_E_ARG, "y_ref, y_work or loss is NULL");
    if ((rc = check_model(model)) || (rc = check_response_rows(model, arr->D)) ||
        (rc = check_ctx(ctx)))
        return rc;
    if ((rc = set_device(ctx->c))) return rc;
    // scratch: [residual partial sums][forward integer sums][adjoint slices][record before
    //          the response]
    const size_t r_bytes = up256(step_res_bytes(state->F, arr->D));
    const size_t f_bytes = up256(forward_ws_bytes(state->F, arr->D, model->T, state->B_cap, sizeof(float)));
    const size_t a_bytes = up256(adjoint_ws_bytes(&ctx->c, arr->D, state->B_cap, state->F, p->mask, sizeof(float)));
    const size_t x_bytes = response_ws_bytes(model, state->F, arr->D, sizeof(float));
    if ((rc = ensure_scratch(&ctx->c, r_bytes + f_bytes + a_bytes + x_bytes))) return rc;
    char *sc = (char *)ctx->c.scratch;
    return step_body(&ctx->c, arr, state, model, y_ref, y_work, p, nullptr, loss, (double *)sc,
                     ctx->c.misc, sc + r_bytes, f_bytes, sc + r_bytes + f_bytes, a_bytes,
                     (float *)(sc + r_bytes + f_bytes + a_bytes), (hipStream_t)stream);
}

int sbp_step_graph_create(sbp_ctx *ctx, const sbp_array *arr, sbp_state *state,
                          const sbp_model *model, const float *y_ref, float *y_work,
                          const sbp_adam_params *p, int32_t *step_dev, double *loss, int32_t iters,
                          sbp_graph **out, void *stream) {
    int rc;
    if (!out) return fail(SBP_E_ARG, "out is NULL");
    *out = nullptr;
    if ((rc = check_array(arr)) || (rc = check_adam(p, false)) ||
        (rc = check_state(state, p->mask, true)))
        return rc;
    if (!y_ref || !y_work || !loss || !step_dev) return fail(SBP_E_ARG, "y_ref, y_work, loss or step_dev is NULL");
    if (iters < 1) return fail(SBP_E_ARG, "iters must be >= 1");
    if (!stream) return fail(SBP_E_ARG, "graph capture needs a non-null stream");
    if ((rc = check_model(model)) || (rc = check_response_rows(model, arr->D)) ||
        (rc = check_ctx(ctx)))
        return rc;
    if ((rc = set_device(ctx->c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    sbp_graph *g = new sbp_graph();
    g->device = ctx->c.device;
    // graph workspace: [residual partial sums][device words][forward integer sums][adjoint slices]
    //                  [record before the response]
    const size_t ws_res = up256(step_res_bytes(state->F, arr->D));
    const size_t ws_fwd = up256(forward_ws_bytes(state->F, arr->D, model->T, state->B_cap, sizeof(float)));
    const size_t ws_adj = up256(adjoint_ws_bytes(&ctx->c, arr->D, state->B_cap, state->F, p->mask, sizeof(float)));
    const size_t ws_aux = response_ws_bytes(model, state->F, arr->D, sizeof(float));
    if (hipMalloc(&g->ws, ws_res + kMiscBytes + ws_fwd + ws_adj + ws_aux) != hipSuccess) {
        delete g;
        (void)hipGetLastError();
        return fail(SBP_E_NOMEM, "could not allocate the graph workspace");
    }
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipFree(g->ws);
        delete g;
        return hip_fail(e, "hipStreamBeginCapture");
    }
    // Each launch starts by zeroing the forward's device words and integer
    // sums (fill kernels, not memset nodes); the iterations then leave them
    // zero for each other, and one increment advances the step count by iters.
    unsigned *g_misc = (unsigned *)((char *)g->ws + ws_res);
    char *g_fwd = (char *)g->ws + ws_res + kMiscBytes;
    int body = launch_fill<int32_t>((int32_t *)g_misc, kMiscFlags + SBP_MAX_FRAMES, 0, st);
    if (body == SBP_OK)
        body = launch_fill<uint64_t>((uint64_t *)g_fwd,
                                     (int64_t)state->F * arr->D * ((int64_t)model->T + 1), 0, st);
    for (int it = 0; it < iters && body == SBP_OK; ++it)
        body = step_body(&ctx->c, arr, state, model, y_ref, y_work, p, step_dev,
                         loss + (int64_t)it * state->F, (double *)g->ws, g_misc, g_fwd, ws_fwd,
                         g_fwd + ws_fwd, ws_adj, (float *)(g_fwd + ws_fwd + ws_adj), st,
                         /*captured=*/true, /*step_add=*/it);
    if (body == SBP_OK) body = launch_incr_by(step_dev, iters, st);
    e = hipStreamEndCapture(st, &g->graph);
    if (body != SBP_OK || e != hipSuccess) {
        char msg[512];
        snprintf(msg, sizeof msg, "%s", g_err);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        (void)hipFree(g->ws);
        delete g;
        if (body != SBP_OK) return fail(body, "during capture: %s", msg);
        return hip_fail(e, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        (void)hipFree(g->ws);
        delete g;
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = g;
    return SBP_OK;
}

int sbp_graph_launch(sbp_graph *g, void *stream) {
    if (!g) return fail(SBP_E_ARG, "graph is NULL");
    SBP_HIP(hipSetDevice(g->device));
    SBP_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return SBP_OK;
}

int sbp_graph_destroy(sbp_graph *g) {
    if (!g) return SBP_OK;
    int rc = SBP_OK;
    if (hipSetDevice(g->device) != hipSuccess) rc = fail(SBP_E_HIP, "hipSetDevice failed");
    if (g->exec && hipGraphExecDestroy(g->exec) != hipSuccess) rc = fail(SBP_E_HIP, "hipGraphExecDestroy failed");
    if (g->graph && hipGraphDestroy(g->graph) != hipSuccess) rc = fail(SBP_E_HIP, "hipGraphDestroy failed");
    if (g->ws && hipFree(g->ws) != hipSuccess) rc = fail(SBP_E_HIP, "hipFree failed");
    delete g;
    return rc;
}

int sbp_softplus_reparam(sbp_ctx *ctx, sbp_state *state, int32_t to_softplus, void *stream) {
    int rc;
    if (!state) return fail(SBP_E_ARG, "state is NULL");
    if ((rc = check_frames(state->ball_off, state->F, state->B_cap))) return rc;
    if (state->B_cap > 0 && !state->balls.a) return fail(SBP_E_ARG, "state.balls.a is NULL");
    if (to_softplus != 0 && to_softplus != 1) return fail(SBP_E_ARG, "to_softplus must be 0 or 1");
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = set_device(ctx->c))) return rc;
    return launch_reparam(state->balls.a, state->m.a, state->v.a, state->ball_off, state->F,
                          state->B_cap, to_softplus, (hipStream_t)stream);
}

int sbp_grow(sbp_ctx *ctx, const sbp_state *in, const sbp_growth_rule *rule, sbp_state *out,
             int64_t *count, void *stream) {
    int rc;
    if (!in || !out || !rule) return fail(SBP_E_ARG, "in, out or rule is NULL");
    if ((rc = check_frames(in->ball_off, in->F, in->B_cap)) ||
        (rc = check_balls(&in->balls, "in.balls", in->B_cap)) ||
        (rc = check_frames(out->ball_off, out->F, out->B_cap)) ||
        (rc = check_balls(&out->balls, "out.balls", out->B_cap)))
        return rc;
    if (in->B_cap > 0 && (!in->grad.x || !in->grad.y || !in->grad.z))
        return fail(SBP_E_ARG, "in.grad x, y, z are needed");
    if (out->F != in->F) return fail(SBP_E_ARG, "out.F must equal in.F");
    if (!(rule->destroy_frac >= 0.0f) || !(rule->a_min >= 0.0f) || !(rule->a_split > 0.0f) ||
        !(rule->dup_frac >= 0.0f && rule->dup_frac <= 1.0f) || !std::isfinite(rule->dup_offset) ||
        rule->reserved != 0)
        return fail(SBP_E_DOMAIN, "growth rule out of range");
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = set_device(ctx->c))) return rc;
    return launch_grow(&ctx->c, in, rule, out, count, (hipStream_t)stream);
}

}  // extern "C"
