// Issue-rate microbenchmark for the roofline of the VALU-bound kernels:
// lane-operations per second on this device for FP32 FMA and multiply, the
// FP32 transcendentals the physics kernels use (exp2, reciprocal, square
// root), FP64 FMA, and LDS 64/32-bit integer and FP64 atomic adds and
// 32/64/128-bit reads at pseudo-random addresses inside one row (the access
// pattern of the forward's accumulation and of the adjoint's staged rows; wide
// reads count every dword as one lane-operation), and atomic adds at
// consecutive addresses (no bank conflict) and with four lanes per address.
//
// Every lane runs eight independent chains so that latency is hidden; the
// grid fills every CU with eight 256-thread workgroups.  Output: one JSON
// line with lane-ops/s and lane-ops per clock per CU at the nominal clock.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#define CHECK(x)                                                                      \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

enum { OP_FMA, OP_MUL, OP_EXP, OP_RCP, OP_SQRT };

template <int OP>
__device__ __forceinline__ float op(float x, float a, float b) {
    if (OP == OP_FMA) return fmaf(x, a, b);
    if (OP == OP_MUL) return x * a;
    if (OP == OP_EXP) return __builtin_amdgcn_exp2f(x);
    if (OP == OP_RCP) return __builtin_amdgcn_rcpf(x);
    return __builtin_amdgcn_sqrtf(x);
}

template <int OP>
__global__ __launch_bounds__(256) void k_f32(float *out, int iters, float a, float b) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = 1.0f + 1e-3f * (float)(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = op<OP>(x[k], a, b);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_f64(double *out, int iters, double a, double b) {
    double x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = 1.0 + 1e-3 * (double)(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = fma(x[k], a, b);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// READ = false: atomic adds; READ = true: plain loads summed in registers.
template <typename T, bool READ>
__global__ __launch_bounds__(256) void k_lds(unsigned long long *out, int iters) {
    __shared__ T row[4096];
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) row[i] = (T)i;
    __syncthreads();
    uint32_t h = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 12345u;
    T acc = 0;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            h = h * 1664525u + 1013904223u;
            const uint32_t idx = (h >> 16) & 4095u;
            if (READ)
                acc += row[idx];
            else
                atomicAdd(&row[idx], (T)(h & 7u));
        }
    }
    __syncthreads();
    unsigned long long s = (unsigned long long)acc;
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) s += (unsigned long long)row[i];
    atomicAdd(out, s);
}

// Atomic adds with a wave-uniform random base and a lane pattern: CONSEC, lane
// l at base + l (consecutive entries: no two lanes share a bank or an
// address); CLUSTER4, four lanes per entry (base + l / 4).  Every address is
// taken modulo the 4096-entry row.
enum { PAT_CONSEC, PAT_CLUSTER4 };

template <typename T, int PAT>
__global__ __launch_bounds__(256) void k_lds_pattern(unsigned long long *out, int iters) {
    __shared__ T row[4096];
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) row[i] = (T)0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t h = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 12345u;
    uint32_t hw = __builtin_amdgcn_readfirstlane((blockIdx.x * 4u + (threadIdx.x >> 6)) * 2246822519u + 777u);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            h = h * 1664525u + 1013904223u;
            hw = hw * 1664525u + 1013904223u;
            const uint32_t base = (hw >> 16) & 4095u;
            const uint32_t idx = (base + (PAT == PAT_CONSEC ? lane : lane >> 2)) & 4095u;
            atomicAdd(&row[idx], (T)(h & 7u));
        }
    }
    __syncthreads();
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) s += (unsigned long long)row[i];
    atomicAdd(out, s);
}

// Random 64-bit atomic adds with the address residue fixed by the lane:
// RES entries in a row of the same residue modulo RES are lane l's (l mod RES)
// (RES = 8: eight lanes per residue class; 16: four), and with only the first
// ACTIVE lanes of each wave taking part (ACTIVE < 64: a partly masked
// instruction, as at the end of a pair's edges).
// Random 64-bit atomic adds confined to a span of SPAN consecutive entries
// (a wave-uniform random base): more lanes of an instruction share an entry
// as the span narrows (a transducer sees a chunk's balls over a few hundred
// edges).
template <int SPAN>
__global__ __launch_bounds__(256) void k_lds_span(unsigned long long *out, int iters) {
    __shared__ unsigned long long row[4096];
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) row[i] = 0ull;
    __syncthreads();
    uint32_t h = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 12345u;
    uint32_t hw = __builtin_amdgcn_readfirstlane((blockIdx.x * 4u + (threadIdx.x >> 6)) * 2246822519u + 777u);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            h = h * 1664525u + 1013904223u;
            hw = hw * 1664525u + 1013904223u;
            const uint32_t idx = (((hw >> 16) & 4095u) + ((h >> 16) % (uint32_t)SPAN)) & 4095u;
            atomicAdd(&row[idx], (unsigned long long)(h & 7u));
        }
    }
    __syncthreads();
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) s += row[i];
    atomicAdd(out, s);
}

template <int RES, int ACTIVE>
__global__ __launch_bounds__(256) void k_lds_residue(unsigned long long *out, int iters) {
    __shared__ unsigned long long row[4096];
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) row[i] = 0ull;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t h = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 12345u;
    if (lane < (uint32_t)ACTIVE) {
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                h = h * 1664525u + 1013904223u;
                const uint32_t idx = RES > 1 ? (((h >> 16) & 4095u & ~(uint32_t)(RES - 1)) | (lane & (RES - 1)))
                                             : ((h >> 16) & 4095u);
                atomicAdd(&row[idx], (unsigned long long)(h & 7u));
            }
        }
    }
    __syncthreads();
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) s += row[i];
    atomicAdd(out, s);
}

// 64-bit adds at random entries done as a returning 32-bit add to the low
// word and, where it wrapped, a 32-bit add of the carry to the high word (the
// sum is the same 64-bit integer).  Values are uniform below 2^VBITS, so a
// carry follows about 2^(VBITS-33) of the adds once the low words are busy;
// eight adds are issued before their carries are checked.
template <int VBITS>
__global__ __launch_bounds__(256) void k_lds_split(unsigned long long *out, int iters) {
    __shared__ unsigned int row[2 * 4096];
    for (int i = threadIdx.x; i < 2 * 4096; i += blockDim.x) row[i] = 0u;
    __syncthreads();
    uint32_t h = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 12345u;
    uint32_t g = (blockIdx.x * 256u + threadIdx.x) * 2246822519u + 777u;
    for (int i = 0; i < iters; ++i) {
        uint32_t idx[8], v[8], old[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            h = h * 1664525u + 1013904223u;
            g = g * 22695477u + 1u;
            idx[r] = (h >> 16) & 4095u;
            v[r] = g >> (32 - VBITS);
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) old[r] = atomicAdd(&row[2 * idx[r]], v[r]);
#pragma unroll
        for (int r = 0; r < 8; ++r)
            if (old[r] + v[r] < old[r]) atomicAdd(&row[2 * idx[r] + 1], 1u);
    }
    __syncthreads();
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < 4096; i += blockDim.x)
        s += ((unsigned long long)row[2 * i + 1] << 32) | row[2 * i];
    atomicAdd(out, s);
}

// The forward's edge pattern: a lane adds 40 consecutive entries from a
// random first entry m, as ten blocks of four.  ROT = 0 takes the blocks in
// order (the entries of a wave's lanes at one step have random residues
// modulo 16); ROT = 1 starts each lane at block beta and wraps, beta chosen so
// that the lanes whose m has one residue modulo 4 take, in lane order, the four
// starts m + 4 beta covering that residue's classes modulo 16.
template <int ROT>
__global__ __launch_bounds__(256) void k_lds_blocks(unsigned long long *out, int iters) {
    __shared__ unsigned long long row[4096];
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) row[i] = 0ull;
    __syncthreads();
    uint32_t h = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 12345u;
    const unsigned long long below = (1ull << (threadIdx.x & 63u)) - 1ull;
    for (int it = 0; it < iters; ++it) {
        h = h * 1664525u + 1013904223u;
        const uint32_t m = h >> 20;
        uint32_t beta = 0;
        if (ROT) {
            const uint32_t cs = m & 3u;
            unsigned long long mine = 0;
#pragma unroll
            for (uint32_t v = 0; v < 4; ++v) {
                const unsigned long long b = __ballot(cs == v);
                if (cs == v) mine = b;
            }
            const uint32_t rank = (uint32_t)__popcll(mine & below);
            beta = ((cs + 4u * (rank & 3u) - m) & 15u) >> 2;
        }
#pragma unroll
        for (int t = 0; t < 10; ++t) {
            uint32_t j = beta + t;
            if (j >= 10u) j -= 10u;
#pragma unroll
            for (int i = 0; i < 4; ++i) atomicAdd(&row[(m + 4u * j + i) & 4095u], (unsigned long long)(i + 1));
        }
    }
    __syncthreads();
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) s += row[i];
    atomicAdd(out, s);
}

// The same 40 edges per lane started at any edge: lane l begins at the edge
// whose entry is congruent to l modulo 16 and wraps (what steering to the
// exact residue would give; the forward cannot start inside a four-edge block
// without restarting its recurrence there).
__global__ __launch_bounds__(256) void k_lds_edges_exact(unsigned long long *out, int iters) {
    __shared__ unsigned long long row[4096];
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) row[i] = 0ull;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t h = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 12345u;
    for (int it = 0; it < iters; ++it) {
        h = h * 1664525u + 1013904223u;
        const uint32_t m = h >> 20;
        const uint32_t r = ((lane & 15u) - m) & 15u;
#pragma unroll
        for (int t = 0; t < 40; ++t) {
            uint32_t k = r + t;
            if (k >= 40u) k -= 40u;
            atomicAdd(&row[(m + k) & 4095u], (unsigned long long)(t & 7) + 1ull);
        }
    }
    __syncthreads();
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) s += row[i];
    atomicAdd(out, s);
}

// Aligned random reads of W dwords per lane (the row holds 4096 dwords).
template <int W>
__global__ __launch_bounds__(256) void k_lds_wide(unsigned long long *out, int iters) {
    typedef unsigned int vec __attribute__((ext_vector_type(W)));
    __shared__ vec row[4096 / W];
    for (int i = threadIdx.x; i < 4096 / W; i += blockDim.x) row[i] = (vec)(unsigned)i;
    __syncthreads();
    uint32_t h = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 12345u;
    vec acc = (vec)0u;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            h = h * 1664525u + 1013904223u;
            acc += row[(h >> 16) & (4096u / W - 1u)];
        }
    }
    unsigned long long s = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) s += acc[k];
    atomicAdd(out, s);
}

int main() {
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const double clk = 2.4e9;
    const int blocks = cus * 8, threads = 256;
    float *out = nullptr;
    double *outd = nullptr;
    unsigned long long *outl = nullptr;
    CHECK(hipMalloc(&out, (size_t)blocks * threads * sizeof(float)));
    CHECK(hipMalloc(&outd, (size_t)blocks * threads * sizeof(double)));
    CHECK(hipMalloc(&outl, sizeof(unsigned long long)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    printf("{\"cus\": %d, \"nominal_clock_hz\": %.3e, \"rates\": {", cus, clk);
    bool first = true;
    auto run = [&](const char *name, auto launch, double lane_ops) -> int {
        launch();
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(e0));
        launch();
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.0f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        const double r = lane_ops / (ms * 1e-3);
        printf("%s\"%s\": {\"lane_ops_per_s\": %.4e, \"per_clk_per_cu\": %.2f, \"ms\": %.3f}",
               first ? "" : ", ", name, r, r / cus / clk, ms);
        first = false;
        return 0;
    };
    const int it = 20000;
    const double nv = (double)blocks * threads * it * 32;
    if (run("fma_f32", [&] { hipLaunchKernelGGL(k_f32<OP_FMA>, dim3(blocks), dim3(threads), 0, 0, out, it, 0.999f, 1e-3f); }, nv)) return 1;
    if (run("mul_f32", [&] { hipLaunchKernelGGL(k_f32<OP_MUL>, dim3(blocks), dim3(threads), 0, 0, out, it, 0.999f, 1e-3f); }, nv)) return 1;
    if (run("exp2_f32", [&] { hipLaunchKernelGGL(k_f32<OP_EXP>, dim3(blocks), dim3(threads), 0, 0, out, it / 4, 0.f, 0.f); }, nv / 4)) return 1;
    if (run("rcp_f32", [&] { hipLaunchKernelGGL(k_f32<OP_RCP>, dim3(blocks), dim3(threads), 0, 0, out, it / 4, 0.f, 0.f); }, nv / 4)) return 1;
    if (run("sqrt_f32", [&] { hipLaunchKernelGGL(k_f32<OP_SQRT>, dim3(blocks), dim3(threads), 0, 0, out, it / 4, 0.f, 0.f); }, nv / 4)) return 1;
    if (run("fma_f64", [&] { hipLaunchKernelGGL(k_f64, dim3(blocks), dim3(threads), 0, 0, outd, it, 0.999, 1e-3); }, nv)) return 1;
    const int li = 2000;
    const double nl = (double)blocks * threads * li * 8;
    if (run("lds_add_u64_random", [&] { hipLaunchKernelGGL((k_lds<unsigned long long, false>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u32_random", [&] { hipLaunchKernelGGL((k_lds<unsigned int, false>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_consecutive", [&] { hipLaunchKernelGGL((k_lds_pattern<unsigned long long, PAT_CONSEC>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_four_lanes_per_entry", [&] { hipLaunchKernelGGL((k_lds_pattern<unsigned long long, PAT_CLUSTER4>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_random_residue8", [&] { hipLaunchKernelGGL((k_lds_residue<8, 64>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_random_residue16", [&] { hipLaunchKernelGGL((k_lds_residue<16, 64>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_random_span1024", [&] { hipLaunchKernelGGL(k_lds_span<1024>, dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_random_span512", [&] { hipLaunchKernelGGL(k_lds_span<512>, dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_random_span256", [&] { hipLaunchKernelGGL(k_lds_span<256>, dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_random_48_lanes", [&] { hipLaunchKernelGGL((k_lds_residue<1, 48>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl * 48 / 64)) return 1;
    if (run("lds_add_u64_random_32_lanes", [&] { hipLaunchKernelGGL((k_lds_residue<1, 32>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl * 32 / 64)) return 1;
    if (run("lds_add_u64_random_16_lanes", [&] { hipLaunchKernelGGL((k_lds_residue<1, 16>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl * 16 / 64)) return 1;
    if (run("lds_add_u64_as_u32_carry_v22", [&] { hipLaunchKernelGGL(k_lds_split<22>, dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_as_u32_carry_v26", [&] { hipLaunchKernelGGL(k_lds_split<26>, dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_as_u32_carry_v29", [&] { hipLaunchKernelGGL(k_lds_split<29>, dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_u64_forward_blocks_in_order", [&] { hipLaunchKernelGGL(k_lds_blocks<0>, dim3(blocks), dim3(threads), 0, 0, outl, li / 5); }, (double)blocks * threads * (li / 5) * 40)) return 1;
    if (run("lds_add_u64_forward_blocks_rotated", [&] { hipLaunchKernelGGL(k_lds_blocks<1>, dim3(blocks), dim3(threads), 0, 0, outl, li / 5); }, (double)blocks * threads * (li / 5) * 40)) return 1;
    if (run("lds_add_u64_forward_edges_exact_start", [&] { hipLaunchKernelGGL(k_lds_edges_exact, dim3(blocks), dim3(threads), 0, 0, outl, li / 5); }, (double)blocks * threads * (li / 5) * 40)) return 1;
    if (run("lds_add_u32_consecutive", [&] { hipLaunchKernelGGL((k_lds_pattern<unsigned int, PAT_CONSEC>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_f64_random", [&] { hipLaunchKernelGGL((k_lds<double, false>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_add_f64_consecutive", [&] { hipLaunchKernelGGL((k_lds_pattern<double, PAT_CONSEC>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_read_b32_random", [&] { hipLaunchKernelGGL((k_lds<unsigned int, true>), dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl)) return 1;
    if (run("lds_read_b64_random", [&] { hipLaunchKernelGGL(k_lds_wide<2>, dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl * 2)) return 1;
    if (run("lds_read_b128_random", [&] { hipLaunchKernelGGL(k_lds_wide<4>, dim3(blocks), dim3(threads), 0, 0, outl, li); }, nl * 4)) return 1;
    printf("}}\n");
    CHECK(hipFree(out));
    CHECK(hipFree(outd));
    CHECK(hipFree(outl));
    return 0;
}
