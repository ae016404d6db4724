// Sustained fused multiply-add rate of the device (akra_fma_rate): the practical ceiling of
// ALU-bound kernels beside the published peak, under the same clock and power limits they run at.
// Sustained matrix-core rate of v_mfma_f32_32x32x2_f32 with and without plain FP32 FMAs between the
// products (akra_mfma_rate): the ceiling of the batched Legendre kernels, whose recurrence is such
// VALU work.
#include "akra_internal.h"

namespace akra {

// C independent chains acc = acc * a + b per thread; the sum of the chains is stored so that no
// chain is dead.  out holds one value per thread of the grid.
template <typename T, int C>
__global__ __launch_bounds__(256) void k_fma_rate(T *__restrict__ out, T a, T b, int iters)
{
    T acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = (T)(threadIdx.x + c);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = fma(acc[c], a, b);
    }
    T s = (T)0;
#pragma unroll
    for (int c = 0; c < C; ++c) s += acc[c];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

typedef float v16f __attribute__((ext_vector_type(16)));

// K independent 32 x 32 accumulators per wave; after each product, V pairs of plain FP32 FMAs on two
// chains of the lane.  The accumulators and the chains are summed and stored so that none is dead.
template <int K, int V>
__global__ __launch_bounds__(64) void k_mfma_rate(float *__restrict__ out, float a0, int iters)
{
    v16f acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[k][r] = 0.f;
    float a = a0 + threadIdx.x * 1e-6f, b = a0 * 0.5f, y = a, z = b;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[k], 0, 0, 0);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                y = fmaf(y, 0.999f, 1e-3f);
                z = fmaf(z, 0.998f, 1e-3f);
            }
        }
        a += 1e-7f;
    }
    float s = y + z;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) s += acc[k][r];
    out[(int64_t)blockIdx.x * 64 + threadIdx.x] = s;
}

template <int K, int V> static void launch_mfma_rate(int blocks, hipStream_t s, float *buf, int iters)
{
    k_mfma_rate<K, V><<<blocks, 64, 0, s>>>(buf, 1.0f, iters);
}

}  // namespace akra

using namespace akra;

akra_status akra_mfma_rate(int chains, int valu, int waves, double *tflops)
{
    if (!tflops || (chains != 1 && chains != 2 && chains != 4) || (valu != 0 && valu != 4 && valu != 8) ||
        (waves != 1 && waves != 2)) {
        set_error("akra_mfma_rate: null output, chains not 1, 2 or 4, valu not 0, 4 or 8, or waves not 1 or 2");
        return AKRA_ERR_ARG;
    }
    constexpr int ITERS = 4096, REPS = 6;
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "akra_mfma_rate: device query");
    const int blocks = ncu * 4 * waves;  // one wave per workgroup: waves per SIMD on four SIMDs per CU
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *buf = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMalloc(&buf, (size_t)blocks * 64 * sizeof(float));
    float best = 0.0f;
    for (int rep = 0; rep < REPS && e == hipSuccess; ++rep) {
        float ms = 0.0f;
        e = hipEventRecord(e0, s);
        const int key = chains * 100 + valu;
        float *f = (float *)buf;
        switch (key) {
        case 100: launch_mfma_rate<1, 0>(blocks, s, f, ITERS); break;
        case 104: launch_mfma_rate<1, 4>(blocks, s, f, ITERS); break;
        case 108: launch_mfma_rate<1, 8>(blocks, s, f, ITERS); break;
        case 200: launch_mfma_rate<2, 0>(blocks, s, f, ITERS); break;
        case 204: launch_mfma_rate<2, 4>(blocks, s, f, ITERS); break;
        case 208: launch_mfma_rate<2, 8>(blocks, s, f, ITERS); break;
        case 400: launch_mfma_rate<4, 0>(blocks, s, f, ITERS); break;
        case 404: launch_mfma_rate<4, 4>(blocks, s, f, ITERS); break;
        default: launch_mfma_rate<4, 8>(blocks, s, f, ITERS);
        }
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms > 0.0f && (best == 0.0f || ms < best)) best = ms;
    }
    if (buf) (void)hipFree(buf);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (e != hipSuccess) return hip_fail(e, "akra_mfma_rate");
    if (best <= 0.0f) {
        set_error("akra_mfma_rate: no launch was timed");
        return AKRA_ERR_HIP;
    }
    *tflops = (double)blocks * ITERS * chains * (32.0 * 32.0 * 2.0 * 2.0) / (best * 1e-3) / 1e12;
    return AKRA_OK;
}

akra_status akra_fma_rate(int precision, double *tflops)
{
    if (!tflops || (precision != AKRA_FP64 && precision != AKRA_FP32)) {
        set_error("akra_fma_rate: null output or unknown precision");
        return AKRA_ERR_ARG;
    }
    constexpr int C = 16, ITERS = 4096, REPS = 12;
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "akra_fma_rate: device query");
    const int blocks = ncu * 4 * 8;  // 8 waves of 64 threads per SIMD, four SIMDs per compute unit
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *buf = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMalloc(&buf, (size_t)blocks * 256 * sizeof(double));
    // back-to-back launches of a few ms each: the clock settles under the load within the first
    // ones; the fastest launch gives the rate
    float best = 0.0f;
    for (int rep = 0; rep < REPS && e == hipSuccess; ++rep) {
        float ms = 0.0f;
        e = hipEventRecord(e0, s);
        if (precision == AKRA_FP64) k_fma_rate<double, C><<<blocks, 256, 0, s>>>((double *)buf, 0.999, 0.001, ITERS);
        else k_fma_rate<float, C><<<blocks, 256, 0, s>>>((float *)buf, 0.999f, 0.001f, ITERS);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms > 0.0f && (best == 0.0f || ms < best)) best = ms;
    }
    if (buf) (void)hipFree(buf);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (e != hipSuccess) return hip_fail(e, "akra_fma_rate");
    if (best <= 0.0f) {
        set_error("akra_fma_rate: no launch was timed");
        return AKRA_ERR_HIP;
    }
    *tflops = 2.0 * blocks * 256.0 * ITERS * C / (best * 1e-3) / 1e12;
    return AKRA_OK;
}
