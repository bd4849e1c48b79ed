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
//   mfma_only: v_mfma_f32_16x16x4_f32 chains            -> matrix FLOP/s
//   mfma_eval: point-pair evaluation with |x - y|^2 from the matrix core
//              (one 16x16x4 MFMA per 256 pairs) and, on the VALU, rsq and two
//              FMAs (row and column sums) per pair      -> evaluations/s
//   valu_eval: the same VALU work with |x - y|^2 from one add instead of the
//              MFMA (what the VALU alone sustains)     -> evaluations/s
// mfma_layout checks the operand/result lane layout of the 16x16x4 FP32 MFMA
// that the point-pair kernels assume: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives D[4 (l / 16) + r][l % 16] in result r.
// Grid 4096 x 256 threads, 4096 iterations; results are written to a buffer
// of exactly grid x block floats.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#define NCH 8

typedef float f4 __attribute__((ext_vector_type(4)));

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


__global__ void __launch_bounds__(256) mfma_only(float *out, int iters)
{
    f4 d[4];
    float a = threadIdx.x * 1e-3f, b = 0.5f;
    for (int k = 0; k < 4; ++k) d[k] = f4{1.0f * k, 2, 3, 4};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d[k], 0, 0, 0);
        b += 1e-7f;
    }
    float s = 0;
    for (int k = 0; k < 4; ++k) s += d[k][0] + d[k][1] + d[k][2] + d[k][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 4 row blocks x one 16-column tile per iteration: 4 MFMAs, 16 rsq, 32 FMAs per lane
__global__ void __launch_bounds__(256) mfma_eval(float *out, int iters)
{
    const int lane = threadIdx.x & 63;
    float a[4];
    f4 c[4], z[4], v[4];
    for (int k = 0; k < 4; ++k) {
        a[k] = (lane >> 4) == 3 ? 1.0f : 0.1f * (k + 1) + lane * 1e-3f;
        for (int r = 0; r < 4; ++r) {
            c[k][r] = 4.0f + r + k;
            z[k][r] = 0;
            v[k][r] = 0.5f + 0.01f * r;
        }
    }
    float b = -0.2f + lane * 1e-4f, u = 0.75f;
    float t = 0;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const f4 r2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], b, c[k], 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float K = __builtin_amdgcn_rsqf(r2[r]);
                z[k][r] = __builtin_fmaf(u, K, z[k][r]);
                t = __builtin_fmaf(v[k][r], K, t);
            }
        }
        b += 1e-7f;
        u -= 1e-7f;
    }
    float s = t;
    for (int k = 0; k < 4; ++k) s += z[k][0] + z[k][1] + z[k][2] + z[k][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) valu_eval(float *out, int iters)
{
    const int lane = threadIdx.x & 63;
    f4 c[4], z[4], v[4];
    for (int k = 0; k < 4; ++k)
        for (int r = 0; r < 4; ++r) {
            c[k][r] = 4.0f + 0.37f * r + 1.13f * k + lane * 1e-3f;
            z[k][r] = 0;
            v[k][r] = 0.5f + 0.01f * r;
        }
    float b = 0.2f, u = 0.75f;
    float t = 0;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float K = __builtin_amdgcn_rsqf(c[k][r] + b);
                z[k][r] = __builtin_fmaf(u, K, z[k][r]);
                t = __builtin_fmaf(v[k][r], K, t);
            }
        }
        b += 1e-7f;
        u -= 1e-7f;
    }
    float s = t;
    for (int k = 0; k < 4; ++k) s += z[k][0] + z[k][1] + z[k][2] + z[k][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// one wavefront: A (16 x 4) and B (4 x 16) from their index patterns
__global__ void __launch_bounds__(64) mfma_layout(float *out)
{
    const int l = threadIdx.x;
    const float a = 1.0f + (l % 16) + 0.25f * (l / 16);   // A[i][k] = 1 + i + k / 4
    const float b = 2.0f - 0.5f * (l / 16) + (l % 16);    // B[k][j] = 2 - k / 2 + j
    const f4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, f4{0, 0, 0, 0}, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = d[r];
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
    const char *names[10] = {"fma_only (FMA lane-ops/s)", "rsq_only (v_rsq_f32 lane-ops/s)",
                             "eval_mix (evaluations/s)", "fma_vv (FMA lane-ops/s)",
                             "add_vv (add lane-ops/s)", "mul_vv (mul lane-ops/s)",
                             "exp_mix (evaluations/s)", "mfma_only (matrix FLOP/s)",
                             "mfma_eval (evaluations/s)", "valu_eval (evaluations/s)"};
    void (*kern[10])(float *, int) = {fma_only, rsq_only, eval_mix, fma_vv, add_vv, mul_vv, exp_mix,
                                      mfma_only, mfma_eval, valu_eval};
    // per thread and iteration: NCH ops, except the MFMA kernels
    // (mfma_only: 4 MFMAs of 2048 FLOPs per wavefront = 128 FLOPs per lane;
    //  mfma_eval / valu_eval: 16 evaluations per lane)
    const double per_iter[10] = {NCH, NCH, NCH, NCH, NCH, NCH, NCH, 128, 16, 16};
    {
        float h[256];
        hipLaunchKernelGGL(mfma_layout, dim3(1), dim3(64), 0, 0, out);
        CHECK(hipGetLastError());
        CHECK(hipMemcpy(h, out, sizeof(h), hipMemcpyDeviceToHost));
        double err = 0;
        for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * (l / 16) + r, j = l % 16;
                double ref = 0;
                for (int k = 0; k < 4; ++k) ref += (1.0 + i + 0.25 * k) * (2.0 - 0.5 * k + j);
                err = fmax(err, fabs(h[l * 4 + r] - ref));
            }
        printf("mfma_layout: max |D - A B| = %.3g (%s)\n", err, err < 1e-3 ? "layout as assumed" : "LAYOUT DIFFERS");
    }
    for (int kind = 0; kind < 10; ++kind) {
        for (int rep = 0; rep < 3; ++rep) {
            CHECK(hipEventRecord(a));
            hipLaunchKernelGGL(kern[kind], dim3(blocks), dim3(threads), 0, 0, out, iters);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(b));
            CHECK(hipEventSynchronize(b));
            float ms;
            CHECK(hipEventElapsedTime(&ms, a, b));
            double ops = (double)blocks * threads * iters * per_iter[kind];
            if (rep == 2) printf("%s: %.3f ms, %.3e per s\n", names[kind], ms, ops / (ms * 1e-3));
        }
    }
    CHECK(hipFree(out));
    return 0;
}
