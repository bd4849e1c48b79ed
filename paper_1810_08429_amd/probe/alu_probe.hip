// ALU throughput probe for the roofline of the pair-quadrature kernels:
//   fma_only : independent FP32 FMA chains        -> VALU lane-ops per second
//   rsq_only : independent v_rsq_f32 chains       -> transcendental rate
//   eval_mix : w * rsq(|x - y|^2) accumulated, the instruction mix of one
//              kernel evaluation (3 sub, mul, 2 fma, rsq, fma)
// Grid 4096 x 256 threads, 4096 iterations, 8 chains per thread; results are
// written to a buffer of exactly grid x block floats.
#include <hip/hip_runtime.h>

#include <cstdio>

#define NCH 8

__global__ void __launch_bounds__(256) fma_only(float *out, int iters)
{
    float a[NCH];
    for (int k = 0; k < NCH; ++k) a[k] = threadIdx.x * 1e-3f + k;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < NCH; ++k) a[k] = fmaf(a[k], 0.999f, 1e-3f);
    float s = 0;
    for (int k = 0; k < NCH; ++k) s += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) rsq_only(float *out, int iters)
{
    float a[NCH];
    for (int k = 0; k < NCH; ++k) a[k] = 1.0f + threadIdx.x * 1e-3f + k;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < NCH; ++k) a[k] = __builtin_amdgcn_rsqf(a[k]);
    float s = 0;
    for (int k = 0; k < NCH; ++k) s += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) eval_mix(float *out, int iters)
{
    float x0 = threadIdx.x * 1e-3f, x1 = 0.5f, x2 = 0.25f;
    float acc[NCH], y0[NCH], y1[NCH], y2[NCH];
    for (int k = 0; k < NCH; ++k) {
        acc[k] = 0;
        y0[k] = 3.0f + k;
        y1[k] = 1.0f + k;
        y2[k] = 2.0f - k;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            float dx = x0 - y0[k], dy = x1 - y1[k], dz = x2 - y2[k];
            float r2 = dx * dx + dy * dy + dz * dz;
            acc[k] = fmaf(0.5f, __builtin_amdgcn_rsqf(r2), acc[k]);
        }
        x0 += 1e-7f;
        x1 -= 1e-7f;
        x2 += 2e-7f;
    }
    float s = 0;
    for (int k = 0; k < NCH; ++k) s += acc[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

#define CHECK(x)                                                            \
    do {                                                                    \
        hipError_t e_ = (x);                                                \
        if (e_ != hipSuccess) {                                             \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));         \
            return 1;                                                       \
        }                                                                   \
    } while (0)

int main()
{
    const int blocks = 4096, threads = 256, iters = 4096;
    float *out;
    CHECK(hipMalloc(&out, sizeof(float) * blocks * threads));
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    const char *names[3] = {"fma_only (FMA lane-ops/s)", "rsq_only (v_rsq_f32 lane-ops/s)",
                            "eval_mix (evaluations/s)"};
    for (int kind = 0; kind < 3; ++kind) {
        for (int rep = 0; rep < 3; ++rep) {
            CHECK(hipEventRecord(a));
            if (kind == 0) hipLaunchKernelGGL(fma_only, dim3(blocks), dim3(threads), 0, 0, out, iters);
            if (kind == 1) hipLaunchKernelGGL(rsq_only, dim3(blocks), dim3(threads), 0, 0, out, iters);
            if (kind == 2) hipLaunchKernelGGL(eval_mix, dim3(blocks), dim3(threads), 0, 0, out, iters);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(b));
            CHECK(hipEventSynchronize(b));
            float ms;
            CHECK(hipEventElapsedTime(&ms, a, b));
            double ops = (double)blocks * threads * iters * NCH;
            if (rep == 2) printf("%s: %.3f ms, %.3e per s\n", names[kind], ms, ops / (ms * 1e-3));
        }
    }
    CHECK(hipFree(out));
    return 0;
}
