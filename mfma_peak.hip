// Microbenchmark of the matrix-core issue rate on one GPU, used by bench.py
// to report roofline fractions against a measured peak beside the spec one.
// Every wave runs a loop of independent matrix instructions (eight
// accumulator chains, enough to cover the instruction latency) of one form;
// flops = waves x iterations x 8 x (2 M N K) of that form.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <type_traits>

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int CHAINS = 8;

template <int KIND>
__global__ __launch_bounds__(256) void k_peak(int iters, float seed, float *out) {
    const int lane = threadIdx.x & 63;
    const float x = seed + 1e-3f * (float)lane;
    float sum = 0.f;
    if constexpr (KIND == 0) {   // v_mfma_f32_16x16x4_f32
        floatx4 acc[CHAINS];
        for (int c = 0; c < CHAINS; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
        const float a = x, b = 1.f - x;
        for (int t = 0; t < iters; ++t)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
        for (int c = 0; c < CHAINS; ++c) sum += acc[c][0] + acc[c][3];
    } else if constexpr (KIND == 1) {   // v_mfma_f64_16x16x4_f64
        doublex4 acc[CHAINS];
        for (int c = 0; c < CHAINS; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
        const double a = x, b = 1.0 - x;
        for (int t = 0; t < iters; ++t)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
        for (int c = 0; c < CHAINS; ++c) sum += (float)(acc[c][0] + acc[c][3]);
    } else if constexpr (KIND == 2 || KIND == 3) {   // v_mfma_f32_16x16x32_{bf16,f16}
        typedef typename std::conditional<KIND == 2, bf16x8, f16x8>::type h8;
        typedef typename std::conditional<KIND == 2, __bf16, _Float16>::type H;
        h8 a, b;
        for (int e = 0; e < 8; ++e) {
            a[e] = (H)(x + 0.01f * e);
            b[e] = (H)(1.f - 0.01f * e);
        }
        floatx4 acc[CHAINS];
        for (int c = 0; c < CHAINS; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int t = 0; t < iters; ++t)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) {
                if constexpr (KIND == 2) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
                else acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[c], 0, 0, 0);
            }
        for (int c = 0; c < CHAINS; ++c) sum += acc[c][0] + acc[c][3];
    } else {   // v_mfma_f32_32x32x16_{bf16,f16}
        typedef typename std::conditional<KIND == 4, bf16x8, f16x8>::type h8;
        typedef typename std::conditional<KIND == 4, __bf16, _Float16>::type H;
        h8 a, b;
        for (int e = 0; e < 8; ++e) {
            a[e] = (H)(x + 0.01f * e);
            b[e] = (H)(1.f - 0.01f * e);
        }
        floatx16 acc[CHAINS / 2];
        for (int c = 0; c < CHAINS / 2; ++c)
            for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;
        for (int t = 0; t < iters; ++t)
#pragma unroll
            for (int c = 0; c < CHAINS / 2; ++c) {
                if constexpr (KIND == 4) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
                else acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[c], 0, 0, 0);
            }
        for (int c = 0; c < CHAINS / 2; ++c) sum += acc[c][0] + acc[c][15];
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = sum;
}

// flops of one instruction and instructions per wave per iteration
constexpr double FLOPS[6] = {2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 32, 2.0 * 16 * 16 * 32,
                             2.0 * 32 * 32 * 16, 2.0 * 32 * 32 * 16};
constexpr int PER_ITER[6] = {CHAINS, CHAINS, CHAINS, CHAINS, CHAINS / 2, CHAINS / 2};

}  // namespace

// kind: 0 FP32 16x16x4, 1 FP64 16x16x4, 2 bf16 16x16x32, 3 fp16 16x16x32,
// 4 bf16 32x32x16, 5 fp16 32x32x16.  Runs `blocks` workgroups of four waves, `iters` loop
// iterations each, `reps` timed launches after one warm-up; writes the best
// launch's TFLOP/s and milliseconds.  Returns 0, or the HIP error code.
extern "C" int mfma_peak(int kind, int blocks, int iters, int reps, double *tflops, double *ms) {
    if (kind < 0 || kind > 5 || blocks < 1 || iters < 1 || reps < 1 || !tflops || !ms) return -1;
    float *out = nullptr;
    hipError_t e = hipMalloc((void **)&out, (size_t)blocks * 256 * sizeof(float));
    if (e != hipSuccess) return (int)e;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 1e30;
    for (int r = 0; r <= reps && e == hipSuccess; ++r) {
        (void)hipEventRecord(e0, nullptr);
        switch (kind) {
        case 0: hipLaunchKernelGGL(k_peak<0>, dim3(blocks), dim3(256), 0, nullptr, iters, 0.5f, out); break;
        case 1: hipLaunchKernelGGL(k_peak<1>, dim3(blocks), dim3(256), 0, nullptr, iters, 0.5f, out); break;
        case 2: hipLaunchKernelGGL(k_peak<2>, dim3(blocks), dim3(256), 0, nullptr, iters, 0.5f, out); break;
        case 3: hipLaunchKernelGGL(k_peak<3>, dim3(blocks), dim3(256), 0, nullptr, iters, 0.5f, out); break;
        case 4: hipLaunchKernelGGL(k_peak<4>, dim3(blocks), dim3(256), 0, nullptr, iters, 0.5f, out); break;
        default: hipLaunchKernelGGL(k_peak<5>, dim3(blocks), dim3(256), 0, nullptr, iters, 0.5f, out); break;
        }
        e = hipGetLastError();
        (void)hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess && r > 0 && hipEventElapsedTime(&t, e0, e1) == hipSuccess) best = t < best ? t : best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (e != hipSuccess) return (int)e;
    const double waves = 4.0 * blocks;
    *ms = best;
    *tflops = waves * iters * PER_ITER[kind] * FLOPS[kind] / (best * 1e-3) / 1e12;
    return 0;
}
