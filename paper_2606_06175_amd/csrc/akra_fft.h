// Complex arithmetic and in-place radix-4 FFTs in LDS for the ring stage and the flat-sky
// transforms (device code, gfx950).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace akra {

template <typename T> struct V2;
template <> struct V2<double> { using type = double2; };
template <> struct V2<float> { using type = float2; };
template <typename T> using cplx = typename V2<T>::type;
template <typename T> __device__ __forceinline__ cplx<T> mk(T a, T b) { cplx<T> r; r.x = a; r.y = b; return r; }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b)
{
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T> __device__ __forceinline__ cplx<T> cmuli(cplx<T> a) { return mk<T>(-a.y, a.x); }  // i a
template <typename T> __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }

// e^{i pi k / den} for an integer k (reduced exactly modulo 2 den), evaluated in FP64.
template <typename T> __device__ __forceinline__ cplx<T> cis_pi(int64_t k, int64_t den)
{
    int64_t p = 2 * den;
    k %= p;
    if (k < 0) k += p;
    double s, c;
    sincospi((double)k / (double)den, &s, &c);
    return mk<T>((T)c, (T)s);
}

constexpr int RT = 256;  // default thread count of the FFT helpers (and the chirp-spectrum kernel)
constexpr int RU = 8;    // default elements per thread of dft_forward

__device__ __forceinline__ unsigned brev(unsigned n, int logM) { return logM ? (__builtin_bitreverse32(n) >> (32 - logM)) : 0u; }

// LDS slot of FFT element i: one pad slot per 32 elements, so that the bit-reversed and strided
// accesses of the radix-2 passes do not all fall into one bank
__device__ __forceinline__ int pd(int i) { return i + (i >> 5); }

// (-+ i) z for sign -1 / +1: the twiddle W_4^{+-1} of a radix-4 step
template <typename T> __device__ __forceinline__ cplx<T> rot4(cplx<T> z, int sign)
{
    return sign < 0 ? mk<T>(z.y, -z.x) : mk<T>(-z.y, z.x);
}

// In-place FFT of length M (a power of two) in LDS, bit-reversed input -> natural output, sign -1:
// e^{-2 pi i/M}.  Two radix-2 stages h, 2h are done as one radix-4 step on the elements i0 + {0, h,
// 2h, 3h} (twiddles u = W_{4h}^pos and u^2 = W_{2h}^pos from the table), so a length-M transform
// takes ceil(log2 M / 2) passes through LDS; an odd log2 M starts with one radix-2 stage.
template <typename T, int NT = RT>
__device__ void fft_dit(cplx<T> *buf, int M, const cplx<T> *__restrict__ tw, int twn, int sign)
{
    const int logM = 31 - __builtin_clz(M);
    int h = 1;
    if (logM & 1) {
        for (int b = threadIdx.x; b < M / 2; b += NT) {
            const cplx<T> a = buf[pd(2 * b)], c = buf[pd(2 * b + 1)];
            buf[pd(2 * b)] = cadd<T>(a, c);
            buf[pd(2 * b + 1)] = csub<T>(a, c);
        }
        __syncthreads();
        h = 2;
    }
    for (; h < M; h <<= 2) {
        const int s4 = twn / (4 * h);
        for (int b = threadIdx.x; b < M / 4; b += NT) {
            const int pos = b & (h - 1);
            const int i0 = ((b - pos) << 2) + pos;
            cplx<T> u = tw[pos * s4], w = tw[2 * pos * s4];
            if (sign > 0) {
                u.y = -u.y;
                w.y = -w.y;
            }
            const cplx<T> a0 = buf[pd(i0)], a1 = buf[pd(i0 + h)], a2 = buf[pd(i0 + 2 * h)], a3 = buf[pd(i0 + 3 * h)];
            const cplx<T> t1 = cmul<T>(w, a1), t3 = cmul<T>(w, a3);
            const cplx<T> b0 = cadd<T>(a0, t1), b1 = csub<T>(a0, t1), b2 = cadd<T>(a2, t3), b3 = csub<T>(a2, t3);
            const cplx<T> x2 = cmul<T>(u, b2), y3 = rot4<T>(cmul<T>(u, b3), sign);
            buf[pd(i0)] = cadd<T>(b0, x2);
            buf[pd(i0 + 2 * h)] = csub<T>(b0, x2);
            buf[pd(i0 + h)] = cadd<T>(b1, y3);
            buf[pd(i0 + 3 * h)] = csub<T>(b1, y3);
        }
        __syncthreads();
    }
}

// In-place FFT, natural input -> bit-reversed output: the radix-2 stages h = M/2 .. 1 in pairs
// (2h, h) as radix-4 steps; an odd log2 M ends with the radix-2 stage h = 1.
template <typename T, int NT = RT>
__device__ void fft_dif(cplx<T> *buf, int M, const cplx<T> *__restrict__ tw, int twn, int sign)
{
    int h = M >> 2;
    for (; h >= 1; h >>= 2) {
        const int s4 = twn / (4 * h);
        for (int b = threadIdx.x; b < M / 4; b += NT) {
            const int pos = b & (h - 1);
            const int i0 = ((b - pos) << 2) + pos;
            cplx<T> u = tw[pos * s4], w = tw[2 * pos * s4];
            if (sign > 0) {
                u.y = -u.y;
                w.y = -w.y;
            }
            const cplx<T> a0 = buf[pd(i0)], a1 = buf[pd(i0 + h)], a2 = buf[pd(i0 + 2 * h)], a3 = buf[pd(i0 + 3 * h)];
            const cplx<T> b0 = cadd<T>(a0, a2), b2 = cmul<T>(csub<T>(a0, a2), u);
            const cplx<T> b1 = cadd<T>(a1, a3), b3 = rot4<T>(cmul<T>(csub<T>(a1, a3), u), sign);
            buf[pd(i0)] = cadd<T>(b0, b1);
            buf[pd(i0 + h)] = cmul<T>(csub<T>(b0, b1), w);
            buf[pd(i0 + 2 * h)] = cadd<T>(b2, b3);
            buf[pd(i0 + 3 * h)] = cmul<T>(csub<T>(b2, b3), w);
        }
        __syncthreads();
    }
    if ((31 - __builtin_clz(M)) & 1) {
        for (int b = threadIdx.x; b < M / 2; b += NT) {
            const cplx<T> a = buf[pd(2 * b)], c = buf[pd(2 * b + 1)];
            buf[pd(2 * b)] = cadd<T>(a, c);
            buf[pd(2 * b + 1)] = csub<T>(a, c);
        }
        __syncthreads();
    }
}

}  // namespace akra
