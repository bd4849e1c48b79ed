// ALU throughput probe for the roofline of the pair-quadrature kernels.
// Every kernel runs NCH independent chains per thread so that issue rate, not
// latency, is measured:
//   fma_only : FP32 FMA with literal operands         -> VALU lane-ops per second
//   fma_vv   : FP32 FMA with register operands (VOP3)
//   add_vv   : FP32 add with register operands
//   mul_vv   : FP32 multiply with register operands
//   rsq_only : v_rsq_f32                               -> transcendental rate
//   eval_mix : w * rsq(|x - y|^2) accumulated, the direct evaluation
//              (3 sub, mul, 2 fma, rsq, fma)
//   exp_mix  : the expanded evaluation |x|^2 + |y|^2 - 2 x.y
//              (add, 3 fma, rsq, fma)
// Grid 4096 x 256 threads, 4096 iterations; results are written to a buffer
// of exactly grid x block floats.
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

__global__ void __launch_bounds__(256) fma_vv(float *out, int iters)
{
    float a[NCH];
    const float b = 0.999f + threadIdx.x * 1e-9f, c = 1e-3f - threadIdx.x * 1e-9f;
    for (int k = 0; k < NCH; ++k) a[k] = threadIdx.x * 1e-3f + k;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < NCH; ++k) a[k] = __builtin_fmaf(b, a[k], c);
    float s = 0;
    for (int k = 0; k < NCH; ++k) s += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) add_vv(float *out, int iters)
{
    float a[NCH];
    const float b = 1e-7f + threadIdx.x * 1e-12f;
    for (int k = 0; k < NCH; ++k) a[k] = threadIdx.x * 1e-3f + k;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < NCH; ++k) a[k] = a[k] + b;
    float s = 0;
    for (int k = 0; k < NCH; ++k) s += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) mul_vv(float *out, int iters)
{
    float a[NCH];
    const float b = 0.9999999f + threadIdx.x * 1e-12f;
    for (int k = 0; k < NCH; ++k) a[k] = threadIdx.x * 1e-3f + k;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < NCH; ++k) a[k] = a[k] * b;
    float s = 0;
    for (int k = 0; k < NCH; ++k) s += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) exp_mix(float *out, int iters)
{
    float x0 = threadIdx.x * 1e-3f, x1 = 0.5f, x2 = 0.25f, xn = x0 * x0 + 0.3125f;
    float acc[NCH], m0[NCH], m1[NCH], m2[NCH], yn[NCH];
    for (int k = 0; k < NCH; ++k) {
        acc[k] = 0;
        m0[k] = -2.0f * (3.0f + k);
        m1[k] = -2.0f * (1.0f + k);
        m2[k] = -2.0f * (2.0f - k);
        yn[k] = 0.25f * (m0[k] * m0[k] + m1[k] * m1[k] + m2[k] * m2[k]);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            float r2 = xn + yn[k];
            r2 = __builtin_fmaf(x2, m2[k], r2);
            r2 = __builtin_fmaf(x1, m1[k], r2);
            r2 = __builtin_fmaf(x0, m0[k], r2);
            acc[k] = __builtin_fmaf(0.5f, __builtin_amdgcn_rsqf(r2), acc[k]);
        }
        x0 += 1e-7f;
        x1 -= 1e-7f;
        x2 += 2e-7f;
        xn += 1e-7f;
    }
    float s = 0;
    for (int k = 0; k < NCH; ++k) s += acc[k];
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
    const char *names[7] = {"fma_only (FMA lane-ops/s)", "rsq_only (v_rsq_f32 lane-ops/s)",
                            "eval_mix (evaluations/s)", "fma_vv (FMA lane-ops/s)",
                            "add_vv (add lane-ops/s)", "mul_vv (mul lane-ops/s)",
                            "exp_mix (evaluations/s)"};
    void (*kern[7])(float *, int) = {fma_only, rsq_only, eval_mix, fma_vv, add_vv, mul_vv, exp_mix};
    for (int kind = 0; kind < 7; ++kind) {
        for (int rep = 0; rep < 3; ++rep) {
            CHECK(hipEventRecord(a));
            hipLaunchKernelGGL(kern[kind], dim3(blocks), dim3(threads), 0, 0, out, iters);
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
