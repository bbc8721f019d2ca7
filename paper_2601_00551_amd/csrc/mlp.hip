// Growth-proposal MLP on gfx950 matrix cores (declared in include/sbp_mlp.h).
//
// Every GEMM uses v_mfma_f32_16x16x32_bf16 (C[16x16] += A[16x32] B[32x16],
// FP32 accumulation).  Lane l of a wave holds A[row l%16][k (l/16)*8 .. +7],
// B[k (l/16)*8 .. +7][col l%16] and C[rows (l/16)*4 .. +3][col l%16], so both
// operands are read as 16 contiguous bytes when A is stored [rows][k] and B is
// stored transposed, [cols][k].  The working copies of the weights are kept in
// exactly those layouts: W^T ([out][in]) for the forward pass and W ([in][out])
// for the backward pass.  Activations saved for the weight gradients are
// transposed ([features][rows]), which is also how a C tile is naturally
// written (four consecutive rows of one column per lane).
#include "../../include/sbp_mlp.h"
#include "sbp_internal.hpp"

namespace sbp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 32;      // 31 features + one zero column
constexpr int kH = 256;
constexpr int kOP = 16;      // output layer padded to one 16-wide tile
constexpr int kTM = 64;      // rows per workgroup in the fused kernels
constexpr int kLd = kH + 8;  // LDS row stride (bf16) of activation tiles, breaks bank conflicts
constexpr int kLdIn = kIn + 8;

// flat FP32 parameter offsets
constexpr int oW1 = 0, oB1 = 8192, oW2 = 8448, oB2 = 73984, oW3 = 74240, oB3 = 139776,
              oW4 = 140032, oB4 = 140544;
// bf16 working-copy offsets
constexpr int wW1t = 0, wW2t = 8192, wW3t = 73728, wW4t = 139264, wW2r = 143360, wW3r = 208896,
              wW4r = 274432;

static_assert(oB4 + 2 == SBP_MLP_NPARAM, "parameter layout");
static_assert(wW4r + kH * kOP == SBP_MLP_NWORK, "work layout");

__device__ inline floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 16 contiguous bytes = 8 bf16 (k-contiguous operand fragment of one lane)
__device__ inline bf16x8 frag(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

static int64_t padded(int64_t M) { return (M + kTM - 1) / kTM * kTM; }

// ------------------------------------------------------------------- sync --

__global__ void k_mlp_sync(const float *__restrict__ P, __bf16 *__restrict__ W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    // W1t [256][32] <- W1 [32][256]
    if (i < kH * kIn) {
        const int n = i / kIn, k = i % kIn;
        W[wW1t + i] = (__bf16)P[oW1 + k * kH + n];
    }
    // W2t, W3t [256][256] <- W [256][256]; W2r, W3r row-major copies
    if (i < kH * kH) {
        const int n = i / kH, k = i % kH;
        W[wW2t + i] = (__bf16)P[oW2 + k * kH + n];
        W[wW3t + i] = (__bf16)P[oW3 + k * kH + n];
        W[wW2r + i] = (__bf16)P[oW2 + i];
        W[wW3r + i] = (__bf16)P[oW3 + i];
    }
    // W4t [16][256] (rows >= 2 zero) and W4r [256][16] (cols >= 2 zero)
    if (i < kOP * kH) {
        const int n = i / kH, k = i % kH;
        W[wW4t + i] = n < SBP_MLP_OUT ? (__bf16)P[oW4 + k * SBP_MLP_OUT + n] : (__bf16)0.0f;
        const int k2 = i / kOP, n2 = i % kOP;
        W[wW4r + i] = n2 < SBP_MLP_OUT ? (__bf16)P[oW4 + k2 * SBP_MLP_OUT + n2] : (__bf16)0.0f;
    }
}

static int launch_sync(const float *P, uint16_t *W, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_sync, dim3(kH * kH / 256), dim3(256), 0, st, P, (__bf16 *)W);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

// ---------------------------------------------------------------- forward --

// One hidden layer of the workgroup's 64 rows: out = bf16(relu(A W + b)) into
// LDS (and transposed into acts if given).  Wave w owns output columns
// [64 w, 64 w + 64) for all 64 rows (4 x 4 accumulator tiles), so per k-step
// it reads 4 A fragments from LDS and 4 B fragments (W^T rows) from global
// memory for 16 matrix-core products, and the weights' columns are read by one
// wave only.
template <int K>
__device__ inline void hidden_layer(const __bf16 *__restrict__ A, int lda, const __bf16 *__restrict__ Wt,
                                    const float *__restrict__ bias, __bf16 *__restrict__ O,
                                    __bf16 *__restrict__ acts_t, int64_t Mp, int64_t m_base,
                                    int64_t M) {
    const int l = threadIdx.x & 63;
    const int c0 = (threadIdx.x >> 6) * 64;
    floatx4 acc[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int ks = 0; ks < K / 32; ++ks) {
        bf16x8 a[4], bq[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) bq[ct] = frag(Wt + (c0 + ct * 16 + (l & 15)) * K + ks * 32 + (l >> 4) * 8);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) a[rt] = frag(A + (rt * 16 + (l & 15)) * lda + ks * 32 + (l >> 4) * 8);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = mfma(a[rt], bq[ct], acc[rt][ct]);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int col = c0 + ct * 16 + (l & 15);
        const float bb = bias[col];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            bf16x4 h4;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = rt * 16 + (l >> 4) * 4 + i;
                const bool valid = m_base + r < M;
                const float v = valid ? fmaxf(acc[rt][ct][i] + bb, 0.0f) : 0.0f;
                const __bf16 h = (__bf16)v;
                O[r * kLd + col] = h;
                h4[i] = h;
            }
            if (acts_t)
                *reinterpret_cast<bf16x4 *>(acts_t + (int64_t)col * Mp + m_base + rt * 16 + (l >> 4) * 4) = h4;
        }
    }
}

__global__ __launch_bounds__(256, 2) void k_mlp_fwd(const float *__restrict__ P, const __bf16 *__restrict__ W,
                                                 const float *__restrict__ X, int64_t M, int64_t Mp,
                                                 float *__restrict__ out, __bf16 *__restrict__ acts) {
    __shared__ __align__(16) __bf16 s_x[kTM * kLdIn];
    __shared__ __align__(16) __bf16 s_a[kTM * kLd];
    __shared__ __align__(16) __bf16 s_b[kTM * kLd];
    const int tid = threadIdx.x;
    const int wrow = (tid >> 6) * 16;
    const int64_t m_base = (int64_t)blockIdx.x * kTM;
    // inputs -> bf16 tile (feature 31 and rows beyond M are zero)
    for (int i = tid; i < kTM * kIn; i += blockDim.x) {
        const int r = i / kIn, k = i % kIn;
        const int64_t m = m_base + r;
        const float v = (m < M && k < SBP_MLP_IN) ? X[m * SBP_MLP_IN + k] : 0.0f;
        s_x[r * kLdIn + k] = (__bf16)v;
    }
    __syncthreads();
    if (acts)   // transposed copy for the weight gradients, rows contiguous
        for (int i = tid; i < kTM * kIn; i += blockDim.x) {
            const int k = i / kTM, r = i % kTM;
            acts[(int64_t)k * Mp + m_base + r] = s_x[r * kLdIn + k];
        }
    __bf16 *a1 = acts ? acts + (int64_t)kIn * Mp : nullptr;
    __bf16 *a2 = acts ? a1 + (int64_t)kH * Mp : nullptr;
    __bf16 *a3 = acts ? a2 + (int64_t)kH * Mp : nullptr;
    hidden_layer<kIn>(s_x, kLdIn, W + wW1t, P + oB1, s_a, a1, Mp, m_base, M);
    __syncthreads();
    hidden_layer<kH>(s_a, kLd, W + wW2t, P + oB2, s_b, a2, Mp, m_base, M);
    __syncthreads();
    hidden_layer<kH>(s_b, kLd, W + wW3t, P + oB3, s_a, a3, Mp, m_base, M);
    __syncthreads();
    // output layer: one 16x16 tile per wave, columns 0..1 are real
    const int l = tid & 63;
    floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kH / 32; ++ks) {
        const bf16x8 a = frag(s_a + (wrow + (l & 15)) * kLd + ks * 32 + (l >> 4) * 8);
        const bf16x8 b = frag(W + wW4t + (l & 15) * kH + ks * 32 + (l >> 4) * 8);
        acc = mfma(a, b, acc);
    }
    const int col = l & 15;
    if (col < SBP_MLP_OUT) {
        const float bb = P[oB4 + col];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t m = m_base + wrow + (l >> 4) * 4 + i;
            if (m < M) out[m * SBP_MLP_OUT + col] = acc[i] + bb;
        }
    }
}

// ------------------------------------------------------------------- loss --

__global__ void k_mlp_loss(const float *__restrict__ out, const float *__restrict__ yg,
                           const float *__restrict__ yp, int64_t M, int64_t Mp, float pos_weight,
                           double *__restrict__ partial, float *__restrict__ dout,
                           __bf16 *__restrict__ dout_t) {
    __shared__ double s_red[4];
    double acc = 0.0;
    const float invM = 1.0f / (float)(M > 0 ? M : 1);
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < Mp;
         m += (int64_t)gridDim.x * blockDim.x) {
        float dz = 0.0f, dp = 0.0f;
        if (m < M) {
            const float z = out[m * 2], p = out[m * 2 + 1];
            const float y = yg[m], t = yp[m];
            const float sp_pos = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));   // softplus(z)
            const float sp_neg = sp_pos - z;                                  // softplus(-z)
            const float sig = 1.0f / (1.0f + expf(-z));
            acc += (double)(pos_weight * y * sp_neg + (1.0f - y) * sp_pos + y * (p - t) * (p - t));
            dz = (pos_weight * y * (sig - 1.0f) + (1.0f - y) * sig) * invM;
            dp = 2.0f * y * (p - t) * invM;
        }
        dout[m * 2] = dz;
        dout[m * 2 + 1] = dp;
        dout_t[m] = (__bf16)dz;
        dout_t[Mp + m] = (__bf16)dp;
        for (int r = 2; r < kOP; ++r) dout_t[(int64_t)r * Mp + m] = (__bf16)0.0f;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

__global__ void k_mlp_loss_final(const double *__restrict__ partial, int n, int64_t M,
                                 double *__restrict__ loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += partial[i];
        *loss = s / (double)(M > 0 ? M : 1);
    }
}

// ----------------------------------------------------------- backward data --

// dH_l = (dH_{l+1} W_{l+1}^T) * 1[H_l > 0] for the workgroup's 64 rows; A is
// the row-major dH_{l+1} tile in LDS, Wr the row-major W_{l+1} ([k_l][k_{l+1}],
// i.e. the B operand with k_{l+1} contiguous).  Wave w owns columns
// [64 w, 64 w + 64) of dH_l, as in the forward's hidden layers.
__device__ inline void back_layer(const __bf16 *__restrict__ A, const __bf16 *__restrict__ Wr,
                                  const __bf16 *__restrict__ h_t, __bf16 *__restrict__ O,
                                  __bf16 *__restrict__ d_t, int64_t Mp, int64_t m_base) {
    const int l = threadIdx.x & 63;
    const int c0 = (threadIdx.x >> 6) * 64;
    floatx4 acc[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int ks = 0; ks < kH / 32; ++ks) {
        bf16x8 a[4], bq[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) bq[ct] = frag(Wr + (c0 + ct * 16 + (l & 15)) * kH + ks * 32 + (l >> 4) * 8);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) a[rt] = frag(A + (rt * 16 + (l & 15)) * kLd + ks * 32 + (l >> 4) * 8);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = mfma(a[rt], bq[ct], acc[rt][ct]);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int col = c0 + ct * 16 + (l & 15);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            const int64_t m0 = m_base + rt * 16 + (l >> 4) * 4;
            const bf16x4 h4 = *reinterpret_cast<const bf16x4 *>(h_t + (int64_t)col * Mp + m0);
            bf16x4 d4;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const __bf16 d = (float)h4[i] > 0.0f ? (__bf16)acc[rt][ct][i] : (__bf16)0.0f;
                if (O) O[(rt * 16 + (l >> 4) * 4 + i) * kLd + col] = d;
                d4[i] = d;
            }
            *reinterpret_cast<bf16x4 *>(d_t + (int64_t)col * Mp + m0) = d4;
        }
    }
}

__global__ __launch_bounds__(256, 2) void k_mlp_bwd(const __bf16 *__restrict__ W, const __bf16 *__restrict__ acts,
                                                 const float *__restrict__ dout, int64_t Mp,
                                                 __bf16 *__restrict__ dacts) {
    __shared__ __align__(16) __bf16 s_a[kTM * kLd];
    __shared__ __align__(16) __bf16 s_b[kTM * kLd];
    const int tid = threadIdx.x;
    const int wrow = (tid >> 6) * 16;
    const int64_t m_base = (int64_t)blockIdx.x * kTM;
    const __bf16 *h1 = acts + (int64_t)kIn * Mp;
    const __bf16 *h2 = h1 + (int64_t)kH * Mp;
    const __bf16 *h3 = h2 + (int64_t)kH * Mp;
    __bf16 *d1 = dacts, *d2 = dacts + (int64_t)kH * Mp, *d3 = d2 + (int64_t)kH * Mp;
    // dH3 = dout W4^T * 1[H3 > 0]: an inner dimension of 2, plain FMAs
    const __bf16 *w4r = W + wW4r;
    for (int i = tid; i < kTM * kH; i += blockDim.x) {
        const int k = i / kTM, r = i % kTM;      // rows fastest: the transposed arrays are read contiguously
        const int64_t m = m_base + r;
        const float g = dout[m * 2] * (float)w4r[k * kOP] + dout[m * 2 + 1] * (float)w4r[k * kOP + 1];
        const __bf16 d = (float)h3[(int64_t)k * Mp + m] > 0.0f ? (__bf16)g : (__bf16)0.0f;
        s_a[r * kLd + k] = d;
        d3[(int64_t)k * Mp + m] = d;
    }
    __syncthreads();
    back_layer(s_a, W + wW3r, h2, s_b, d2, Mp, m_base);
    __syncthreads();
    back_layer(s_b, W + wW2r, h1, nullptr, d1, Mp, m_base);
}

// ------------------------------------------------------- weight gradients --

// G[k][n] (row-major, ldg) += sum over rows m in this block's slice of
// At[k][m] * Bt[n][m]   (At: [K][Mp], Bt: [N][Mp], BF16, m-contiguous).
// Block = 4 waves on a 64 x 64 tile of G (4 C tiles per wave); grid.z splits m.
__global__ __launch_bounds__(256) void k_mlp_wgrad(const __bf16 *__restrict__ At, const __bf16 *__restrict__ Bt,
                                                   int K, int N, int64_t Mp, int64_t m_per,
                                                   float *__restrict__ G, int ldg) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kb = blockIdx.x * 64 + w * 16;
    if (kb >= K) return;
    const int64_t m0 = (int64_t)blockIdx.z * m_per;
    const int64_t m1 = min(m0 + m_per, Mp);
    floatx4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int64_t m = m0; m < m1; m += 32) {
        const bf16x8 a = frag(At + (int64_t)(kb + (l & 15)) * Mp + m + (l >> 4) * 8);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int nb = blockIdx.y * 64 + t * 16;
            if (nb >= N) break;
            const bf16x8 b = frag(Bt + (int64_t)(nb + (l & 15)) * Mp + m + (l >> 4) * 8);
            acc[t] = mfma(a, b, acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int n = blockIdx.y * 64 + t * 16 + (l & 15);
        if (n >= N || n >= ldg) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = kb + (l >> 4) * 4 + i;
            atomicAdd(G + (int64_t)k * ldg + n, acc[t][i]);
        }
    }
}

// bias gradient: g[n] += sum of Bt[n][m] over this block's slice of m
// (grid: n x slices; g is zeroed beforehand)
__global__ void k_mlp_bgrad(const __bf16 *__restrict__ Bt, int64_t Mp, int64_t m_per, float *__restrict__ g) {
    __shared__ float s_red[4];
    float acc = 0.0f;
    const __bf16 *row = Bt + (int64_t)blockIdx.x * Mp;
    const int64_t m0 = (int64_t)blockIdx.y * m_per, m1 = min(m0 + m_per, Mp);
    for (int64_t m = m0 + threadIdx.x; m < m1; m += blockDim.x) acc += (float)row[m];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(g + blockIdx.x, s_red[0] + s_red[1] + s_red[2] + s_red[3]);
}

// bias gradient of the output layer from the FP32 output gradient [Mp][2]
__global__ void k_mlp_bgrad_out(const float *__restrict__ dout, int64_t Mp, int64_t m_per, float *__restrict__ g) {
    __shared__ float s_red[2][4];
    float a0 = 0.0f, a1 = 0.0f;
    const int64_t m0 = (int64_t)blockIdx.x * m_per, m1 = min(m0 + m_per, Mp);
    for (int64_t m = m0 + threadIdx.x; m < m1; m += blockDim.x) {
        a0 += dout[m * 2];
        a1 += dout[m * 2 + 1];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_down(a0, o, 64);
        a1 += __shfl_down(a1, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_red[0][threadIdx.x >> 6] = a0;
        s_red[1][threadIdx.x >> 6] = a1;
    }
    __syncthreads();
    if (threadIdx.x < 2)
        atomicAdd(g + threadIdx.x, s_red[threadIdx.x][0] + s_red[threadIdx.x][1] + s_red[threadIdx.x][2] +
                                       s_red[threadIdx.x][3]);
}

static int launch_wgrad(const __bf16 *At, const __bf16 *Bt, int K, int N, int64_t Mp, float *G,
                        int ldg, hipStream_t st) {
    int64_t splits = Mp / 4096;
    if (splits < 1) splits = 1;
    if (splits > 64) splits = 64;
    int64_t m_per = (Mp + splits - 1) / splits;
    m_per = (m_per + 31) / 32 * 32;
    splits = (Mp + m_per - 1) / m_per;
    dim3 grid((K + 63) / 64, (N + 63) / 64, (unsigned)splits);
    hipLaunchKernelGGL(k_mlp_wgrad, grid, dim3(256), 0, st, At, Bt, K, N, Mp, m_per, G, ldg);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

// ------------------------------------------------------------------- Adam --

__global__ void k_mlp_adam(float *__restrict__ P, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                           int step) {
    const double bc1 = 1.0 - pow((double)b1, (double)step);
    const double bc2 = 1.0 - pow((double)b2, (double)step);
    const float bc2s = (float)sqrt(bc2);
    const float ss = (float)(-(double)lr / bc1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        float mi = m[i], vi = v[i];
        mi = mi + (1.0f - b1) * (gi - mi);
        vi = vi * b2 + (1.0f - b2) * gi * gi;
        P[i] = P[i] + ss * (mi / (sqrtf(vi) / bc2s + eps));
        m[i] = mi;
        v[i] = vi;
    }
}

}  // namespace sbp

using namespace sbp;

extern "C" {

int sbp_mlp_sync(sbp_ctx *ctx, const float *params, uint16_t *work, void *stream) {
    if (!params || !work) return fail(SBP_E_ARG, "params or work is NULL");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    return launch_sync(params, work, (hipStream_t)stream);
}

int sbp_mlp_forward(sbp_ctx *ctx, const float *params, const uint16_t *work, const float *X,
                    int64_t M, float *out, uint16_t *acts, void *stream) {
    if (!params || !work || !out || (M > 0 && !X)) return fail(SBP_E_ARG, "a required pointer is NULL");
    if (M < 0) return fail(SBP_E_ARG, "M must be >= 0");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    if (M == 0) return SBP_OK;
    const int64_t Mp = padded(M);
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)(Mp / kTM)), dim3(256), 0, (hipStream_t)stream, params,
                       (const __bf16 *)work, X, M, Mp, out, (__bf16 *)acts);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

int sbp_mlp_loss(sbp_ctx *ctx, const float *out, const float *label_grow, const float *label_p0,
                 int64_t M, float pos_weight, double *loss, float *dout, uint16_t *dout_t,
                 void *stream) {
    if (!out || !label_grow || !label_p0 || !loss || !dout || !dout_t)
        return fail(SBP_E_ARG, "a required pointer is NULL");
    if (M < 1) return fail(SBP_E_ARG, "M must be >= 1");
    if (!(pos_weight >= 0.0f)) return fail(SBP_E_DOMAIN, "pos_weight must be >= 0");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    const int64_t Mp = padded(M);
    const int nb = 256;
    int rc = ensure_scratch(&ctx->c, nb * sizeof(double));
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_loss, dim3(nb), dim3(256), 0, st, out, label_grow, label_p0, M, Mp,
                       pos_weight, (double *)ctx->c.scratch, dout, (__bf16 *)dout_t);
    SBP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mlp_loss_final, dim3(1), dim3(64), 0, st, (const double *)ctx->c.scratch, nb, M, loss);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

int sbp_mlp_backward(sbp_ctx *ctx, const uint16_t *work, const uint16_t *acts, const float *dout,
                     const uint16_t *dout_t, int64_t M, uint16_t *dacts, float *grad,
                     void *stream) {
    if (!work || !acts || !dout || !dout_t || !dacts || !grad)
        return fail(SBP_E_ARG, "a required pointer is NULL");
    if (M < 1) return fail(SBP_E_ARG, "M must be >= 1");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    const int64_t Mp = padded(M);
    hipStream_t st = (hipStream_t)stream;
    const __bf16 *W = (const __bf16 *)work;
    const __bf16 *A = (const __bf16 *)acts;
    __bf16 *dA = (__bf16 *)dacts;
    int rc = launch_fill<float>(grad, SBP_MLP_NPARAM, 0.0f, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mlp_bwd, dim3((unsigned)(Mp / kTM)), dim3(256), 0, st, W, A, dout, Mp, dA);
    SBP_HIP(hipGetLastError());
    const __bf16 *x_t = A, *h1 = A + (int64_t)kIn * Mp, *h2 = h1 + (int64_t)kH * Mp,
                 *h3 = h2 + (int64_t)kH * Mp;
    const __bf16 *d1 = dA, *d2 = dA + (int64_t)kH * Mp, *d3 = d2 + (int64_t)kH * Mp;
    if ((rc = launch_wgrad(x_t, d1, kIn, kH, Mp, grad + oW1, kH, st))) return rc;
    if ((rc = launch_wgrad(h1, d2, kH, kH, Mp, grad + oW2, kH, st))) return rc;
    if ((rc = launch_wgrad(h2, d3, kH, kH, Mp, grad + oW3, kH, st))) return rc;
    if ((rc = launch_wgrad(h3, (const __bf16 *)dout_t, kH, SBP_MLP_OUT, Mp, grad + oW4, SBP_MLP_OUT, st)))
        return rc;
    // bias gradients: slices of 8192 rows, summed with FP32 atomics into the zeroed grad
    const int64_t m_per = 8192;
    const unsigned nsl = (unsigned)((Mp + m_per - 1) / m_per);
    hipLaunchKernelGGL(k_mlp_bgrad, dim3(kH, nsl), dim3(256), 0, st, d1, Mp, m_per, grad + oB1);
    hipLaunchKernelGGL(k_mlp_bgrad, dim3(kH, nsl), dim3(256), 0, st, d2, Mp, m_per, grad + oB2);
    hipLaunchKernelGGL(k_mlp_bgrad, dim3(kH, nsl), dim3(256), 0, st, d3, Mp, m_per, grad + oB3);
    hipLaunchKernelGGL(k_mlp_bgrad_out, dim3(nsl), dim3(256), 0, st, dout, Mp, m_per, grad + oB4);
    SBP_HIP(hipGetLastError());
    return SBP_OK;
}

int sbp_mlp_adam(sbp_ctx *ctx, float *params, const float *grad, float *m, float *v,
                 const sbp_adam_params *p, uint16_t *work, void *stream) {
    if (!params || !grad || !m || !v || !p || !work) return fail(SBP_E_ARG, "a required pointer is NULL");
    if (!(p->beta1 >= 0.0f && p->beta1 < 1.0f) || !(p->beta2 >= 0.0f && p->beta2 < 1.0f) || p->step < 1)
        return fail(SBP_E_DOMAIN, "betas must be in [0, 1) and step >= 1");
    if (!ctx) return fail(SBP_E_ARG, "ctx is NULL");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_adam, dim3(256), dim3(256), 0, st, params, grad, m, v,
                       (int64_t)SBP_MLP_NPARAM, p->lr[0], p->beta1, p->beta2, p->eps, p->step);
    SBP_HIP(hipGetLastError());
    return launch_sync(params, work, st);
}

}  // extern "C"
