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
// wave only.  The next k-step's B fragments and the layer's bias values are
// loaded ahead of use, so their latency overlaps the products (with two waves
// per SIMD there is little else to hide it; two steps ahead gained nothing).
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
    float bb4[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) bb4[ct] = bias[c0 + ct * 16 + (l & 15)];
    bf16x8 bn[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) bn[ct] = frag(Wt + (c0 + ct * 16 + (l & 15)) * K + (l >> 4) * 8);
#pragma unroll 2
    for (int ks = 0; ks < K / 32; ++ks) {
        bf16x8 a[4], bq[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) bq[ct] = bn[ct];
        if (ks + 1 < K / 32) {
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                bn[ct] = frag(Wt + (c0 + ct * 16 + (l & 15)) * K + (ks + 1) * 32 + (l >> 4) * 8);
        }
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
        const float bb = bb4[ct];
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
            // transposed copy for the weight gradients (four rows of one column)
            if (acts_t)
                *reinterpret_cast<bf16x4 *>(acts_t + (int64_t)col * Mp + m_base + rt * 16 + (l >> 4) * 4) = h4;
        }
    }
}

constexpr int kFwdThreads = 256;     // the forward's workgroup size (its loops assume it)

__global__ __launch_bounds__(kFwdThreads, 2) void k_mlp_fwd(const float *__restrict__ P, const __bf16 *__restrict__ W,
                                                 const float *__restrict__ X, int64_t M, int64_t Mp,
                                                 float *__restrict__ out, __bf16 *__restrict__ acts) {
    __shared__ __align__(16) __bf16 s_x[kTM * kLdIn];
    __shared__ __align__(16) __bf16 s_a[kTM * kLd];
    __shared__ __align__(16) __bf16 s_b[kTM * kLd];
    const int tid = threadIdx.x;
    const int wrow = (tid >> 6) * 16;
    const int64_t m_base = (int64_t)blockIdx.x * kTM;
    // inputs -> bf16 tile (feature 31 and rows beyond M are zero): every
    // thread loads all its values (indices clamped into X, M >= 1) before it
    // uses any, one latency instead of one per value
    constexpr int kXPer = kTM * kIn / kFwdThreads;
    float xv[kXPer];
#pragma unroll
    for (int j = 0; j < kXPer; ++j) {
        const int i = tid + j * kFwdThreads;
        const int64_t m = m_base + i / kIn;
        const int k = i % kIn;
        xv[j] = X[(m < M ? m : M - 1) * SBP_MLP_IN + (k < SBP_MLP_IN ? k : SBP_MLP_IN - 1)];
    }
#pragma unroll
    for (int j = 0; j < kXPer; ++j) {
        const int i = tid + j * kFwdThreads;
        const int k = i % kIn;
        const bool real = m_base + i / kIn < M && k < SBP_MLP_IN;
        s_x[(i / kIn) * kLdIn + k] = (__bf16)(real ? xv[j] : 0.0f);
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
    // output layer: one 16x16 tile per wave, columns 0..1 are real; the bias
    // is loaded ahead and the four results stored back to back
    const int l = tid & 63;
    const int col = l & 15;
    const float bb = P[oB4 + (col < SBP_MLP_OUT ? col : 0)];
    floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kH / 32; ++ks) {
        const bf16x8 a = frag(s_a + (wrow + (l & 15)) * kLd + ks * 32 + (l >> 4) * 8);
        const bf16x8 b = frag(W + wW4t + (l & 15) * kH + ks * 32 + (l >> 4) * 8);
        acc = mfma(a, b, acc);
    }
    if (col < SBP_MLP_OUT) {
        const int64_t m0 = m_base + wrow + (l >> 4) * 4;
        float o0 = acc[0] + bb, o1 = acc[1] + bb, o2 = acc[2] + bb, o3 = acc[3] + bb;
        // four live registers: otherwise one register is refilled between the
        // stores and each store waits for the previous one to complete
        asm volatile("" : "+v"(o0), "+v"(o1), "+v"(o2), "+v"(o3));
        float *po = out + m0 * SBP_MLP_OUT + col;
        if (m0 < M) po[0] = o0;
        if (m0 + 1 < M) po[SBP_MLP_OUT] = o1;
        if (m0 + 2 < M) po[2 * SBP_MLP_OUT] = o2;
        if (m0 + 3 < M) po[3 * SBP_MLP_OUT] = o3;
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

// Writes the workgroup's 64 x 256 row-major LDS tile O transposed into
// dst_t[col][Mp] (rows m_base .. m_base + 63): thread t owns column t and
// stores its 64 values as eight 16-byte vectors, 128 contiguous bytes per
// column (lane-scattered 8-byte stores of the MFMA layout waste most of each
// memory transaction).  If h_t is given, a value is kept only where the
// saved activation h_t[col][m] is positive (the ReLU derivative), and O is
// updated with the masked values.  Call between barriers.  The forward keeps
// the MFMA-layout stores: measured faster there, where they overlap the next
// layer's loads; the backward's masked read-modify-write is faster this way.
__device__ inline void store_tile_t(__bf16 *__restrict__ O, const __bf16 *__restrict__ h_t,
                                    __bf16 *__restrict__ dst_t, int64_t Mp, int64_t m_base) {
    const int col = threadIdx.x;
    __bf16 *dst = dst_t + (int64_t)col * Mp + m_base;
    const __bf16 *hp = h_t ? h_t + (int64_t)col * Mp + m_base : nullptr;
    bf16x8 h[kTM / 8];
    if (hp) {
#pragma unroll
        for (int v = 0; v < kTM / 8; ++v) h[v] = frag(hp + v * 8);   // all issued before any store
    }
#pragma unroll
    for (int v = 0; v < kTM / 8; ++v) {
        bf16x8 d;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int r = v * 8 + e;
            __bf16 x = O[r * kLd + col];
            if (hp) {
                x = (float)h[v][e] > 0.0f ? x : (__bf16)0.0f;
                O[r * kLd + col] = x;
            }
            d[e] = x;
        }
        *reinterpret_cast<bf16x8 *>(dst + v * 8) = d;
    }
}

// dH_l = (dH_{l+1} W_{l+1}^T) * 1[H_l > 0] for the workgroup's 64 rows; A is
// the row-major dH_{l+1} tile in LDS, Wr the row-major W_{l+1} ([k_l][k_{l+1}],
// i.e. the B operand with k_{l+1} contiguous).  Wave w owns columns
// [64 w, 64 w + 64) of dH_l, as in the forward's hidden layers.  This writes
// the unmasked product (BF16) into the LDS tile O; store_tile_t then applies
// the ReLU mask and writes dH_l transposed.
__device__ inline void back_layer(const __bf16 *__restrict__ A, const __bf16 *__restrict__ Wr,
                                  __bf16 *__restrict__ O) {
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
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) O[(rt * 16 + (l >> 4) * 4 + i) * kLd + col] = (__bf16)acc[rt][ct][i];
    }
}

__global__ __launch_bounds__(256, 2) void k_mlp_bwd(const __bf16 *__restrict__ W, const __bf16 *__restrict__ acts,
                                                 const float *__restrict__ dout, int64_t Mp,
                                                 __bf16 *__restrict__ dacts) {
    __shared__ __align__(16) __bf16 s_a[kTM * kLd];
    __shared__ __align__(16) __bf16 s_b[kTM * kLd];
    const int tid = threadIdx.x;
    const int64_t m_base = (int64_t)blockIdx.x * kTM;
    const __bf16 *h1 = acts + (int64_t)kIn * Mp;
    const __bf16 *h2 = h1 + (int64_t)kH * Mp;
    const __bf16 *h3 = h2 + (int64_t)kH * Mp;
    __bf16 *d1 = dacts, *d2 = dacts + (int64_t)kH * Mp, *d3 = d2 + (int64_t)kH * Mp;
    // dH3 = dout W4^T * 1[H3 > 0]: an inner dimension of 2, plain FMAs.  Thread
    // t owns column t: its 64 saved activations are read as eight 16-byte
    // vectors issued together (one memory latency, not 64), the tile's output
    // gradients come from LDS.
    __shared__ float s_dout[kTM * 2];
    if (tid < kTM * 2) s_dout[tid] = dout[m_base * 2 + tid];
    const __bf16 *w4r = W + wW4r;
    {
        const int k = tid;
        const float w0 = (float)w4r[k * kOP], w1 = (float)w4r[k * kOP + 1];
        const __bf16 *hk = h3 + (int64_t)k * Mp + m_base;
        __bf16 *dk = d3 + (int64_t)k * Mp + m_base;
        bf16x8 h[kTM / 8];
#pragma unroll
        for (int v = 0; v < kTM / 8; ++v) h[v] = frag(hk + v * 8);
        __syncthreads();
#pragma unroll
        for (int v = 0; v < kTM / 8; ++v) {
            bf16x8 dv;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int r = v * 8 + e;
                const float g = s_dout[2 * r] * w0 + s_dout[2 * r + 1] * w1;
                const __bf16 d = (float)h[v][e] > 0.0f ? (__bf16)g : (__bf16)0.0f;
                s_a[r * kLd + k] = d;
                dv[e] = d;
            }
            *reinterpret_cast<bf16x8 *>(dk + v * 8) = dv;
        }
    }
    __syncthreads();
    back_layer(s_a, W + wW3r, s_b);
    __syncthreads();
    store_tile_t(s_b, h2, d2, Mp, m_base);
    __syncthreads();
    back_layer(s_b, W + wW2r, s_a);
    __syncthreads();
    store_tile_t(s_a, h1, d1, Mp, m_base);
}

// ------------------------------------------------------- weight gradients --

// Partial weight (and bias) gradients of one slice of rows m:
//   part[s][k][n] = sum over m in slice s of At[k][m] * Bt[n][m]   (k < K, n < NP)
//   part[s][K][n] = sum over m in slice s of Bt[n][m]              (bias, if BIAS)
// At: [K][Mp], Bt: [NP][Mp] (BF16, m-contiguous, NP a multiple of 16).  One
// workgroup takes the whole K x NP block for its slice, so At and Bt are read
// from memory once per call; wave w owns a WK x WN sub-block (waves laid out
// K/WK by NP/WN) and per 32-wide m-step loads WK/16 + WN/16 fragments for
// (WK/16)(WN/16) matrix-core products.  The bias sums ride along as products
// of a ones fragment with the B fragments, in the waves that own k = 0.
// Slices are added in a fixed order by k_mlp_wgrad_reduce (no atomics:
// gradients are reproducible).
template <int WK, int WN, bool BIAS>
__global__ __launch_bounds__(512) void k_mlp_wgrad(const __bf16 *__restrict__ At,
                                                   const __bf16 *__restrict__ Bt, int K, int NP,
                                                   int64_t Mp, int64_t m_per,
                                                   float *__restrict__ part) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nwn = NP / WN;
    const int k0 = (w / nwn) * WK, n0 = (w % nwn) * WN;
    if (k0 >= K) return;
    const int64_t m0 = (int64_t)blockIdx.x * m_per;
    const int64_t m1 = min(m0 + m_per, Mp);
    floatx4 acc[WK / 16][WN / 16];
    floatx4 accb[WN / 16];
#pragma unroll
    for (int i = 0; i < WK / 16; ++i)
#pragma unroll
        for (int j = 0; j < WN / 16; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < WN / 16; ++j) accb[j] = floatx4{0.f, 0.f, 0.f, 0.f};
    bf16x8 ones;
#pragma unroll
    for (int e = 0; e < 8; ++e) ones[e] = (__bf16)1.0f;
    const bool bias_wave = BIAS && k0 == 0;
    const __bf16 *pa = At + (int64_t)(k0 + (l & 15)) * Mp + (l >> 4) * 8;
    const __bf16 *pb = Bt + (int64_t)(n0 + (l & 15)) * Mp + (l >> 4) * 8;
    for (int64_t m = m0; m < m1; m += 32) {
        bf16x8 a[WK / 16], b[WN / 16];
#pragma unroll
        for (int i = 0; i < WK / 16; ++i) a[i] = frag(pa + (int64_t)i * 16 * Mp + m);
#pragma unroll
        for (int j = 0; j < WN / 16; ++j) b[j] = frag(pb + (int64_t)j * 16 * Mp + m);
#pragma unroll
        for (int i = 0; i < WK / 16; ++i)
#pragma unroll
            for (int j = 0; j < WN / 16; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
        if (bias_wave) {
#pragma unroll
            for (int j = 0; j < WN / 16; ++j) accb[j] = mfma(ones, b[j], accb[j]);
        }
    }
    const int rows = K + (BIAS ? 1 : 0);
    float *ps = part + (int64_t)blockIdx.x * rows * NP;
#pragma unroll
    for (int i = 0; i < WK / 16; ++i)
#pragma unroll
        for (int j = 0; j < WN / 16; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                ps[(int64_t)(k0 + i * 16 + (l >> 4) * 4 + r) * NP + n0 + j * 16 + (l & 15)] = acc[i][j][r];
    if (bias_wave && (l >> 4) == 0) {
        // every row of the ones product holds the column sums; row 0 is lane l < 16
#pragma unroll
        for (int j = 0; j < WN / 16; ++j) ps[(int64_t)K * NP + n0 + j * 16 + l] = accb[j][0];
    }
}

// G[k][n] = sum over slices of part[s][k][n] for k < K, n < N (G row stride
// ldg), slice 0 first; the bias row k = K, if present, goes to gb[n].
__global__ void k_mlp_wgrad_reduce(const float *__restrict__ part, int nsl, int rows, int NP, int K,
                                   int N, float *__restrict__ G, int ldg, float *__restrict__ gb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * NP) return;
    const int k = i / NP, n = i % NP;
    if (n >= N) return;
    // eight interleaved running sums (slices sl = j mod 8), added in a fixed
    // order: more loads in flight than one dependent chain
    const int64_t stride = (int64_t)rows * NP;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int sl = 0;
    for (; sl + 8 <= nsl; sl += 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] += part[(int64_t)(sl + j) * stride + i];
    }
    for (int j = 0; sl < nsl; ++sl, ++j) acc[j] += part[(int64_t)sl * stride + i];
    const float s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    if (k < K)
        G[(int64_t)k * ldg + n] = s;
    else if (gb)
        gb[n] = s;
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

// Rows per slice of the weight gradients: at least 1024 (so that a slice's
// matrix-core work outweighs writing its partial block), and no more slices
// than CUs (the partial-sum buffer stays below 256 x (K + 1) x NP floats).
static int64_t wgrad_slices(const Ctx *c, int64_t Mp, int64_t *m_per) {
    int64_t cus = c->num_cus > 0 ? c->num_cus : 256;
    if (cus > 256) cus = 256;
    int64_t mp = (Mp + cus - 1) / cus;
    mp = (mp + 31) / 32 * 32;
    if (mp < 1024) mp = 1024;
    *m_per = mp;
    return (Mp + mp - 1) / mp;
}

template <int WK, int WN, bool BIAS>
static int launch_wgrad(Ctx *c, const __bf16 *At, const __bf16 *Bt, int K, int NP, int N, int64_t Mp,
                        float *G, int ldg, float *gb, hipStream_t st) {
    if ((K / WK) * (NP / WN) > 8 || K % WK || NP % WN) return fail(SBP_E_ARG, "wgrad tiling");
    int64_t m_per = 0;
    const int64_t nsl = wgrad_slices(c, Mp, &m_per);
    const int rows = K + (BIAS ? 1 : 0);
    const size_t bytes = (size_t)nsl * rows * NP * sizeof(float);
    int rc = ensure_scratch(c, bytes);
    if (rc) return rc;
    float *part = (float *)c->scratch;
    hipLaunchKernelGGL((k_mlp_wgrad<WK, WN, BIAS>), dim3((unsigned)nsl), dim3(512), 0, st, At, Bt, K, NP,
                       Mp, m_per, part);
    SBP_HIP(hipGetLastError());
    const int n = rows * NP;
    hipLaunchKernelGGL(k_mlp_wgrad_reduce, dim3((n + 255) / 256), dim3(256), 0, st, (const float *)part,
                       (int)nsl, rows, NP, K, N, G, ldg, gb);
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
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)(Mp / kTM)), dim3(kFwdThreads), 0, (hipStream_t)stream, params,
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
    // weight gradients and, folded into the same pass, the hidden-layer bias gradients
    Ctx *c = &ctx->c;
    if ((rc = launch_wgrad<32, 32, true>(c, x_t, d1, kIn, kH, kH, Mp, grad + oW1, kH, grad + oB1, st))) return rc;
    if ((rc = launch_wgrad<64, 128, true>(c, h1, d2, kH, kH, kH, Mp, grad + oW2, kH, grad + oB2, st))) return rc;
    if ((rc = launch_wgrad<64, 128, true>(c, h2, d3, kH, kH, kH, Mp, grad + oW3, kH, grad + oB3, st))) return rc;
    if ((rc = launch_wgrad<32, 16, false>(c, h3, (const __bf16 *)dout_t, kH, kOP, SBP_MLP_OUT, Mp, grad + oW4,
                                          SBP_MLP_OUT, nullptr, st)))
        return rc;
    // output-layer bias gradient from the FP32 output gradient: slices of 8192 rows,
    // FP32 atomics into the zeroed grad
    const int64_t m_per = 8192;
    const unsigned nsl = (unsigned)((Mp + m_per - 1) / m_per);
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
