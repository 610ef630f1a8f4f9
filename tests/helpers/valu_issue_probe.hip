// valu_issue_probe.hip -- issue rate of single VALU instruction kinds on the
// device (measurement aid for the kernels' instruction-issue roofline; not
// part of the library).
//
// Every lane runs eight independent chains of one instruction kind (float32
// FMA, float64 FMA, 32 x 32 -> 64-bit integer multiply-add with an xor, the
// hardware 2^x with an xor, xor-add) over 8192 work-groups of 256 threads,
// timed with HIP events; it prints lane operations per second beside 3.93e13,
// the rate of one wave64 instruction per four clocks on each of the 4 x 256
// SIMDs at 2.4 GHz. Build: hipcc --offload-arch=gfx950 -O3 -Xclang
// -target-feature -Xclang -packed-fp32-ops (as the library).
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdint.h>
#define CHK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("err %s line %d\n", hipGetErrorString(e_), __LINE__); return 1; } } while (0)

template <int K>
__global__ __launch_bounds__(256) void k_fma32(float *out, int iters, float b, float c) {
    float a[K];
#pragma unroll
    for (int i = 0; i < K; ++i) a[i] = threadIdx.x * 1e-3f + i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < K; ++i) a[i] = __builtin_fmaf(a[i], b, c);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < K; ++i) s += a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
template <int K>
__global__ __launch_bounds__(256) void k_fma64(double *out, int iters, double b, double c) {
    double a[K];
#pragma unroll
    for (int i = 0; i < K; ++i) a[i] = threadIdx.x * 1e-3 + i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < K; ++i) a[i] = __builtin_fma(a[i], b, c);
    }
    double s = 0.;
#pragma unroll
    for (int i = 0; i < K; ++i) s += a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
template <int K>
__global__ __launch_bounds__(256) void k_mad64(uint32_t *out, int iters, uint32_t b) {
    uint32_t a[K];
#pragma unroll
    for (int i = 0; i < K; ++i) a[i] = threadIdx.x * 7u + i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < K; ++i) { uint64_t p = (uint64_t)a[i] * b; a[i] = (uint32_t)(p >> 32) ^ (uint32_t)p; }
    }
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) s ^= a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
template <int K>
__global__ __launch_bounds__(256) void k_exp(float *out, int iters) {
    float a[K];
#pragma unroll
    for (int i = 0; i < K; ++i) a[i] = -(threadIdx.x * 1e-4f + i * 1e-2f);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < K; ++i) a[i] = -__builtin_amdgcn_exp2f(a[i]);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < K; ++i) s += a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
template <int K>
__global__ __launch_bounds__(256) void k_xor3(uint32_t *out, int iters, uint32_t b, uint32_t c) {
    uint32_t a[K];
#pragma unroll
    for (int i = 0; i < K; ++i) a[i] = threadIdx.x * 7u + i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < K; ++i) a[i] = (a[i] ^ b ^ c) + i;
    }
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) s ^= a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int main() {
    const int blocks = 256 * 8 * 4, threads = 256, iters = 4096;
    const size_t n = (size_t)blocks * threads;
    void *buf;
    CHK(hipMalloc(&buf, n * 8));
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0)); CHK(hipEventCreate(&e1));
    float ms;
    const double lanes = (double)n * iters * 8;
#define RUN(name, launch, per)                                                  \
    for (int rep = 0; rep < 3; ++rep) {                                         \
        CHK(hipEventRecord(e0));                                                \
        launch;                                                                 \
        CHK(hipGetLastError());                                                 \
        CHK(hipEventRecord(e1));                                                \
        CHK(hipEventSynchronize(e1));                                           \
        CHK(hipEventElapsedTime(&ms, e0, e1));                                  \
        if (rep == 2) printf("%-8s %8.3f ms  %.3e lane-ops/s (x%d instr each)\n", name, ms, lanes / (ms * 1e-3), per); \
    }
    RUN("fma32", (k_fma32<8><<<blocks, threads>>>((float *)buf, iters, 0.999f, 1e-3f)), 1);
    RUN("fma64", (k_fma64<8><<<blocks, threads>>>((double *)buf, iters, 0.999, 1e-3)), 1);
    RUN("mad64+x", (k_mad64<8><<<blocks, threads>>>((uint32_t *)buf, iters, 0xD2511F53u)), 2);
    RUN("exp2", (k_exp<8><<<blocks, threads>>>((float *)buf, iters)), 1);
    RUN("xor3+a", (k_xor3<8><<<blocks, threads>>>((uint32_t *)buf, iters, 0x9E3779B9u, 0xBB67AE85u)), 2);
    CHK(hipFree(buf));
    printf("peak if 4 cycles per wave64 instr: %.3e lane-ops/s\n", 256.0 * 4 * 16 * 2.4e9);
    return 0;
}
