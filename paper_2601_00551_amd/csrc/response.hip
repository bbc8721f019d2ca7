// Transducer impulse response: the Gaussian-envelope taps of each element and
// the per-row time convolution of a record with them, and its adjoint (the
// correlation).  The elements of the in vivo array of section 2.2 have a
// 2.02 MHz mean centre frequency and 54 % bandwidth; the amplitude spectrum
// is taken as a Gaussian of that centre whose full width at half the peak
// (-6 dB) is bw * fc, with unit gain at fc.
//
// The convolution does 2 L flops per output sample on 8 bytes of HBM traffic
// (one read, one write), so for the responses of interest (L of 30 to 140
// taps at 10-40 MHz) it is bound by VALU FMA issue, not by HBM.  One workgroup
// takes kRespTile consecutive outputs of one row: it stages the input window
// (tile + L - 1 samples) in LDS once, then each lane slides a register window
// of kRespP samples across it, one LDS read per tap feeding kRespP FMAs.  The
// taps are wave-uniform (scalar loads).  Lanes own kRespP consecutive outputs,
// so a wave's LDS reads have stride kRespP words: odd, hence every lane of a
// read hits a different bank.  The outputs go back through LDS and leave as
// coalesced rows.
#include "sbp_internal.hpp"

namespace sbp {

constexpr int kRespBlock = 256;
constexpr int kRespP = 7;
constexpr int kRespTile = kRespBlock * kRespP;

static int round_up(int x, int m) { return (x + m - 1) / m * m; }

// out[row][n] (+)= sum_{i<L} tap_i * x[n - n0 + i] with the staged window
// x[i] = y[row][s0 + i]: a convolution (ADJ false: tap_i = h[L-1-i],
// s0 = n0 + zero - L + 1) or its adjoint, the correlation (tap_i = h[i],
// s0 = n0 - zero).  Taps are read kRespP at a time (one scalar wait per
// block instead of one per tap).
template <typename R, bool ADJ>
__global__ __launch_bounds__(kRespBlock) void k_resp_apply(
    const float *__restrict__ h, int rows_h, int L, int zero, const R *__restrict__ y, int D, int T,
    int ntiles, int accumulate, R *__restrict__ out) {
    extern __shared__ __align__(16) unsigned char resp_smem[];
    R *x = reinterpret_cast<R *>(resp_smem);
    const int64_t row = blockIdx.x / ntiles;
    const int n0 = (int)(blockIdx.x - row * ntiles) * kRespTile;
    const float *hr = h + (rows_h == 1 ? 0 : (row % D) * (int64_t)L);
    const R *yr = y + row * (int64_t)T;
    const int Lp = (L + kRespP - 1) / kRespP * kRespP;
    const int W = kRespTile + L - 1;          // samples the tile reads
    const int Wl = kRespTile + Lp + kRespP;   // staged (the tail beyond W is zero)
    const int s0 = ADJ ? n0 - zero : n0 + zero - (L - 1);
    for (int i = threadIdx.x; i < Wl; i += kRespBlock) {
        const int64_t n = (int64_t)s0 + i;
        x[i] = (i < W && n >= 0 && n < T) ? yr[n] : R(0);
    }
    __syncthreads();
    const int base = threadIdx.x * kRespP;
    R acc[kRespP], w[kRespP];
#pragma unroll
    for (int k = 0; k < kRespP; ++k) {
        acc[k] = R(0);
        w[k] = x[base + k];
    }
    // before tap i, slot (k + i) mod P holds x[base + i + k]
    int i0 = 0;
    for (; i0 + kRespP <= L; i0 += kRespP) {
        float tap[kRespP];
#pragma unroll
        for (int s = 0; s < kRespP; ++s) tap[s] = ADJ ? hr[i0 + s] : hr[L - 1 - i0 - s];
#pragma unroll
        for (int s = 0; s < kRespP; ++s) {
#pragma unroll
            for (int k = 0; k < kRespP; ++k) acc[k] = fma((R)tap[s], w[(k + s) % kRespP], acc[k]);
            w[s] = x[base + i0 + s + kRespP];
        }
    }
    if (i0 < L) {   // the last L mod P taps
#pragma unroll
        for (int s = 0; s < kRespP; ++s) {
            const int i = i0 + s;
            if (i < L) {
                const R tap = (R)(ADJ ? hr[i] : hr[L - 1 - i]);
#pragma unroll
                for (int k = 0; k < kRespP; ++k) acc[k] = fma(tap, w[(k + s) % kRespP], acc[k]);
            }
            w[s] = x[base + i + kRespP];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRespP; ++k) x[base + k] = acc[k];
    __syncthreads();
    R *orow = out + row * (int64_t)T;
    for (int i = threadIdx.x; i < kRespTile; i += kRespBlock) {
        const int n = n0 + i;
        if (n < T) orow[n] = accumulate ? orow[n] + x[i] : x[i];
    }
}

// h[r][j] = dt A exp(-t^2 / (2 s_t^2)) cos(2 pi fc t), t = (j - zero) dt, with
// s_f = bw fc / (2 sqrt(2 ln 2)), s_t = 1 / (2 pi s_f), A = 2 / (s_t sqrt(2 pi));
// computed in FP64 and rounded once.  A row whose fc or bw is not a positive
// finite number gets NaN taps.
__global__ void k_resp_taps(const float *__restrict__ fc, const float *__restrict__ bw, int rows,
                            double dt, int L, int zero, float *__restrict__ h) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * L) return;
    const int r = (int)(idx / L);
    const int j = (int)(idx - (int64_t)r * L);
    const double f = fc[r], b = bw[r];
    if (!(f > 0.0) || !(b > 0.0) || !isfinite(f) || !isfinite(b)) {
        h[idx] = __builtin_nanf("");
        return;
    }
    const double kPi = 3.14159265358979323846;
    const double s_f = b * f / (2.0 * sqrt(2.0 * log(2.0)));
    const double s_t = 1.0 / (2.0 * kPi * s_f);
    const double amp = 2.0 / (s_t * sqrt(2.0 * kPi));
    const double t = (double)(j - zero) * dt;
    h[idx] = (float)(dt * amp * exp(-(t * t) / (2.0 * s_t * s_t)) * cos(2.0 * kPi * f * t));
}

size_t response_lds_bytes(int L, size_t elem) {
    return (size_t)(kRespTile + round_up(L, kRespP) + kRespP) * elem;
}

template <typename R>
int launch_response(const float *h, int rows_h, int L, int zero, const R *y, int64_t rows, int D,
                    int T, int adjoint, int accumulate, R *out, hipStream_t st) {
    if (rows < 1 || T < 1) return SBP_OK;
    const int ntiles = (T + kRespTile - 1) / kRespTile;
    const int64_t nblocks = rows * ntiles;
    if (nblocks > INT32_MAX) return fail(SBP_E_ARG, "response: %lld rows x %d samples is too many",
                                         (long long)rows, T);
    if (adjoint)
        hipLaunchKernelGGL((k_resp_apply<R, true>), dim3((unsigned)nblocks), dim3(kRespBlock),
                           response_lds_bytes(L, sizeof(R)), st, h, rows_h, L, zero, y, D, T,
                           ntiles, accumulate, out);
    else
        hipLaunchKernelGGL((k_resp_apply<R, false>), dim3((unsigned)nblocks), dim3(kRespBlock),
                           response_lds_bytes(L, sizeof(R)), st, h, rows_h, L, zero, y, D, T,
                           ntiles, accumulate, out);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

template int launch_response<float>(const float *, int, int, int, const float *, int64_t, int, int,
                                    int, int, float *, hipStream_t);
template int launch_response<double>(const float *, int, int, int, const double *, int64_t, int,
                                     int, int, int, double *, hipStream_t);

int launch_response_taps(const float *fc, const float *bw, int rows, double dt, int L, int zero,
                         float *h, hipStream_t st) {
    const int64_t n = (int64_t)rows * L;
    hipLaunchKernelGGL(k_resp_taps, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, fc, bw,
                       rows, dt, L, zero, h);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

}  // namespace sbp
