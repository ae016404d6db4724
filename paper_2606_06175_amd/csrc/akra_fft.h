// Complex arithmetic and in-place radix-8 FFTs in LDS for the ring stage and the flat-sky
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

// W_8^{+-1} z and W_8^{+-3} z for sign -1 / +1 (the twiddles e^{-+ i pi / 4}, e^{-+ 3 i pi / 4})
template <typename T> __device__ __forceinline__ cplx<T> rot8(cplx<T> z, int sign)
{
    const T r = (T)0.70710678118654752440;
    return sign < 0 ? mk<T>(r * (z.x + z.y), r * (z.y - z.x)) : mk<T>(r * (z.x - z.y), r * (z.x + z.y));
}
template <typename T> __device__ __forceinline__ cplx<T> rot8_3(cplx<T> z, int sign)
{
    const T r = (T)0.70710678118654752440;
    return sign < 0 ? mk<T>(r * (z.y - z.x), -r * (z.x + z.y)) : mk<T>(-r * (z.x + z.y), r * (z.x - z.y));
}

// twiddle of the table for sign -1 (e^{-2 pi i k / twn}) or its conjugate for sign +1
template <typename T> __device__ __forceinline__ cplx<T> twid(const cplx<T> *__restrict__ tw, int k, int sign)
{
    cplx<T> u = tw[k];
    if (sign > 0) u.y = -u.y;
    return u;
}

// Radix-2 stage of span 1 on adjacent pairs (the same for both orders: its twiddle is 1).
template <typename T, int NT> __device__ __forceinline__ void fft_r2_span1(cplx<T> *buf, int M)
{
    for (int b = threadIdx.x; b < M / 2; b += NT) {
        const cplx<T> a = buf[pd(2 * b)], c = buf[pd(2 * b + 1)];
        buf[pd(2 * b)] = cadd<T>(a, c);
        buf[pd(2 * b + 1)] = csub<T>(a, c);
    }
    __syncthreads();
}

// In-place FFT of length M (a power of two) in LDS, bit-reversed input -> natural output, sign -1:
// e^{-2 pi i/M}.  Decimation in time: radix-2 stages of span h = 1, 2, 4, ..., each pair
// (a, b) -> (a + t b, a - t b) with t = W_{2h}^pos, pos the position in its block of 2h.  Three
// stages h, 2h, 4h are done as one radix-8 step in registers on the elements i0 + j h, j < 8 (block
// of 8h, position pos): twiddles W_{2h}^pos, W_{4h}^pos and W_{8h}^pos from the table, the others
// from them by the constant factors W_4 and W_8.  A length-M transform takes floor(log2 M / 3)
// radix-8 passes through LDS, after one radix-2 stage (log2 M = 1 mod 3) or one radix-4 step
// (log2 M = 2 mod 3).
template <typename T, int NT = RT>
__device__ void fft_dit(cplx<T> *buf, int M, const cplx<T> *__restrict__ tw, int twn, int sign)
{
    const int logM = 31 - __builtin_clz(M);
    int h = 1;
    if (logM % 3 == 1) {
        fft_r2_span1<T, NT>(buf, M);
        h = 2;
    } else if (logM % 3 == 2) {
        // radix-4 step at h = 1: spans 1 and 2, twiddles 1 and W_4
        for (int b = threadIdx.x; b < M / 4; b += NT) {
            const int i0 = 4 * b;
            const cplx<T> a0 = buf[pd(i0)], a1 = buf[pd(i0 + 1)], a2 = buf[pd(i0 + 2)], a3 = buf[pd(i0 + 3)];
            const cplx<T> b0 = cadd<T>(a0, a1), b1 = csub<T>(a0, a1), b2 = cadd<T>(a2, a3), b3 = csub<T>(a2, a3);
            const cplx<T> y3 = rot4<T>(b3, sign);
            buf[pd(i0)] = cadd<T>(b0, b2);
            buf[pd(i0 + 2)] = csub<T>(b0, b2);
            buf[pd(i0 + 1)] = cadd<T>(b1, y3);
            buf[pd(i0 + 3)] = csub<T>(b1, y3);
        }
        __syncthreads();
        h = 4;
    }
    for (; h < M; h <<= 3) {
        const int s8 = twn / (8 * h);
        for (int b = threadIdx.x; b < M / 8; b += NT) {
            const int pos = b & (h - 1);
            const int i0 = ((b - pos) << 3) + pos;
            const cplx<T> t8 = twid<T>(tw, pos * s8, sign), t4 = twid<T>(tw, 2 * pos * s8, sign),
                          t2 = twid<T>(tw, 4 * pos * s8, sign);
            cplx<T> e[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) e[j] = buf[pd(i0 + j * h)];
            // span h: pairs (2k, 2k + 1), twiddle W_{2h}^pos
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const cplx<T> x = cmul<T>(t2, e[2 * k + 1]);
                e[2 * k + 1] = csub<T>(e[2 * k], x);
                e[2 * k] = cadd<T>(e[2 * k], x);
            }
            // span 2h: pairs (j, j + 2), twiddle W_{4h}^{pos + (j & 1) h} = W_{4h}^pos W_4^{j & 1}
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = (q & 1) + 4 * (q >> 1);  // 0, 1, 4, 5
                cplx<T> x = cmul<T>(t4, e[j + 2]);
                if (j & 1) x = rot4<T>(x, sign);
                e[j + 2] = csub<T>(e[j], x);
                e[j] = cadd<T>(e[j], x);
            }
            // span 4h: pairs (j, j + 4), twiddle W_{8h}^{pos + j h} = W_{8h}^pos W_8^j
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                cplx<T> x = cmul<T>(t8, e[j + 4]);
                if (j == 1) x = rot8<T>(x, sign);
                if (j == 2) x = rot4<T>(x, sign);
                if (j == 3) x = rot8_3<T>(x, sign);
                e[j + 4] = csub<T>(e[j], x);
                e[j] = cadd<T>(e[j], x);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) buf[pd(i0 + j * h)] = e[j];
        }
        __syncthreads();
    }
}

// In-place FFT, natural input -> bit-reversed output: decimation in frequency, radix-2 stages of
// span h = M/2, M/4, ..., 1, each pair (a, b) -> (a + b, (a - b) t) with t = W_{2h}^pos.  Three
// stages 4h, 2h, h are done as one radix-8 step (the mirror of the one above); one radix-4 step
// (spans 2, 1) or one radix-2 stage (span 1) ends the transform when log2 M is not a multiple of 3.
template <typename T, int NT = RT>
__device__ void fft_dif(cplx<T> *buf, int M, const cplx<T> *__restrict__ tw, int twn, int sign)
{
    const int logM = 31 - __builtin_clz(M);
    int h = M >> 3;
    for (int q = 0; q < logM / 3; ++q, h >>= 3) {
        const int s8 = twn / (8 * h);
        for (int b = threadIdx.x; b < M / 8; b += NT) {
            const int pos = b & (h - 1);
            const int i0 = ((b - pos) << 3) + pos;
            const cplx<T> t8 = twid<T>(tw, pos * s8, sign), t4 = twid<T>(tw, 2 * pos * s8, sign),
                          t2 = twid<T>(tw, 4 * pos * s8, sign);
            cplx<T> e[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) e[j] = buf[pd(i0 + j * h)];
            // span 4h: pairs (j, j + 4), twiddle W_{8h}^{pos + j h}
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const cplx<T> a = e[j], c = e[j + 4];
                e[j] = cadd<T>(a, c);
                cplx<T> d = cmul<T>(csub<T>(a, c), t8);
                if (j == 1) d = rot8<T>(d, sign);
                if (j == 2) d = rot4<T>(d, sign);
                if (j == 3) d = rot8_3<T>(d, sign);
                e[j + 4] = d;
            }
            // span 2h: pairs (j, j + 2), twiddle W_{4h}^{pos + (j & 1) h}
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = (q & 1) + 4 * (q >> 1);  // 0, 1, 4, 5
                const cplx<T> a = e[j], c = e[j + 2];
                e[j] = cadd<T>(a, c);
                cplx<T> d = cmul<T>(csub<T>(a, c), t4);
                if (j & 1) d = rot4<T>(d, sign);
                e[j + 2] = d;
            }
            // span h: pairs (2k, 2k + 1), twiddle W_{2h}^pos
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const cplx<T> a = e[2 * k], c = e[2 * k + 1];
                e[2 * k] = cadd<T>(a, c);
                e[2 * k + 1] = cmul<T>(csub<T>(a, c), t2);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) buf[pd(i0 + j * h)] = e[j];
        }
        __syncthreads();
    }
    if (logM % 3 == 2) {
        // radix-4 step at h = 1: spans 2 and 1
        for (int b = threadIdx.x; b < M / 4; b += NT) {
            const int i0 = 4 * b;
            const cplx<T> a0 = buf[pd(i0)], a1 = buf[pd(i0 + 1)], a2 = buf[pd(i0 + 2)], a3 = buf[pd(i0 + 3)];
            const cplx<T> b0 = cadd<T>(a0, a2), b2 = csub<T>(a0, a2);
            const cplx<T> b1 = cadd<T>(a1, a3), b3 = rot4<T>(csub<T>(a1, a3), sign);
            buf[pd(i0)] = cadd<T>(b0, b1);
            buf[pd(i0 + 1)] = csub<T>(b0, b1);
            buf[pd(i0 + 2)] = cadd<T>(b2, b3);
            buf[pd(i0 + 3)] = csub<T>(b2, b3);
        }
        __syncthreads();
    } else if (logM % 3 == 1) {
        fft_r2_span1<T, NT>(buf, M);
    }
}

}  // namespace akra
