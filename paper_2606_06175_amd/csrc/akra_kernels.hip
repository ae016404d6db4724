// Device kernels of libakra for CDNA4 (gfx950).
//
// Operator chain of the matrix-free H v (paper Sec. II.B, storage problem):
//   prologue      x -> K_l x                                   (harmonic diagonal, eq. Dl_kernel)
//   leg_synth     alm -> F_r(+-m) per ring                      (inverse SHT, Legendre stage)
//   ring          F -> fold -> inverse DFT -> x W -> DFT -> unfold -> G     (SHT ring stage + N^-1 M)
//   leg_adj       G -> partial sums of 2h_lm, -2h_lm            (adjoint SHT, Legendre stage)
//   epilogue      E/B combination (eq. EB_decomp), K_l, + lambda_eff x   (eq. ML_estimator_reg)
#include <type_traits>

#include "akra_leg.h"

namespace akra {

// ------------------------------------------------------------------------------------------------
// Entry states (plan build).  One wave per (m, 64-pair group) runs the FP64 recurrence from the
// seeds at l0 = max(m, 2) with the same steps and rescaling as the Legendre kernels' ramp (two
// steps, then a rescale), and stops at the first degree where some pair of the group contributes:
// it has left the scaled range and reaches `live`.  FP64 plans take live = 2^-100: the values are
// of order one where they oscillate, so the terms of a group that is still below 2^-100 everywhere
// change a sum by less than 2^-100 of its scale, far under FP64 rounding (2^-53), and skipping them
// saves about 5% of the triples at lmax 4096.  FP32 plans take 2^-44, the bound below which the
// FP32 kernels' scaled values are still masked.  The state at the last degree l0 + 8q
// before it is stored with that degree; a group that never contributes up to lmax is marked
// ENT_SKIP.
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_entry(const double *__restrict__ seed2, const double *__restrict__ seedm2,
                                               const int *__restrict__ seedk, const double *__restrict__ pair_z,
                                               const Coef64 *__restrict__ coef, Ent64 *__restrict__ ent,
                                               int *__restrict__ entk, int *__restrict__ entl, int lmax, int npairs,
                                               int ng, int gpb, double live)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int m = blockIdx.x / gpb;
    const int g = (blockIdx.x - m * gpb) * 4 + wave;
    if (m > lmax || g >= ng) return;
    const int p = g * 64 + lane;
    const bool valid = p < npairs;
    const int64_t idx = (int64_t)m * npairs + p;
    double x = 0, c2 = 0, p2 = 0, cm = 0, pm = 0;
    int k = 0;
    if (valid) {
        x = pair_z[p];
        c2 = seed2[idx];
        cm = seedm2[idx];
        k = seedk[idx];
    }
    const int l0 = m > 2 ? m : 2;
    const Coef64 *cf = coef + (int64_t)m * (2 * lmax + 1 - m) / 2;
    double s2 = c2, sp2 = p2, sm = cm, spm = pm;
    int sk = k, sl = l0, res = ENT_SKIP;
    for (int l = l0; l <= lmax;) {
        if (wave_any(valid && k == 0 && fmax(fabs(c2), fabs(cm)) >= live)) {
            res = sl;
            break;
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const Coef64 c = cf[l + t];
            const double u = c.a * x;
            const double n2 = fma(u + c.b, c2, -(c.g * p2));
            const double nm = fma(u - c.b, cm, -(c.g * pm));
            p2 = c2;
            c2 = n2;
            pm = cm;
            cm = nm;
        }
        l += 2;
        if (k < 0) {
            const double big = fmax(fabs(c2), fabs(cm));
            if (big > scale_hi<double>()) {
                const double d = scale_down<double>();
                c2 *= d;
                p2 *= d;
                cm *= d;
                pm *= d;
                k += 1;
            }
        }
        if (((l - l0) & 7) == 0) {
            s2 = c2;
            sp2 = p2;
            sm = cm;
            spm = pm;
            sk = k;
            sl = l;
        }
    }
    if (valid) {
        Ent64 e;
        e.c2 = s2;
        e.p2 = sp2;
        e.cm = sm;
        e.pm = spm;
        ent[idx] = e;
        entk[idx] = sk;
    }
    if (lane == 0) entl[(int64_t)m * ng + g] = res;
}

// ================================================================================================
// prologue / epilogue / weights
// ================================================================================================
// records of the scaled plain form (c_l times the u combinations of K_l alm, FP64 arithmetic; see
// SynRec) and, when recu is given, the unscaled u combinations for the difference form
template <typename T>
__global__ void k_prologue(const double *__restrict__ xE, const double *__restrict__ xB, const double *__restrict__ kern,
                           const int *__restrict__ lof, const typename CoefT<T, 0>::type *__restrict__ coef,
                           const Coef64S *__restrict__ cs64, int lmax, int64_t nalm, int64_t rec_stride,
                           SynRec<T> *__restrict__ rec, float4 *__restrict__ recu)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (i >= nalm) return;
    const int64_t o = rhs * nalm + i;
    const double K = kern ? kern[lof[i]] : 1.0;
    const bool m0 = i <= lmax;
    const auto c = coef[i];
    const double er = K * xE[2 * o], ei = m0 ? 0.0 : K * xE[2 * o + 1];
    const double br = K * xB[2 * o], bi = m0 ? 0.0 : K * xB[2 * o + 1];
    const double s = cs64[i].c;
    const double u0 = er - bi, u1 = ei + br, u2 = er + bi, u3 = br - ei;
    SynRec<T> r;
    r.a = c.a;
    r.b = c.b;
    r.g = (T)0;
    r.pad = (T)0;
    r.u0 = (T)(s * u0);
    r.u1 = (T)(s * u1);
    r.u2 = (T)(s * u2);
    r.u3 = (T)(s * u3);
    rec[rhs * rec_stride + i] = r;
    if (recu) recu[rhs * rec_stride + i] = make_float4((float)u0, (float)u1, (float)u2, (float)u3);
}

// m of the alm index i = m (2 lmax + 1 - m)/2 + l
__device__ __forceinline__ int m_of(int64_t i, int l, int lmax)
{
    const int64_t b = i - l;
    const double A = 2.0 * lmax + 1.0;
    int m = (int)((A - sqrt(A * A - 8.0 * (double)b)) * 0.5);
    if (m < 0) m = 0;
    if (m > lmax) m = lmax;
    while (m > 0 && (int64_t)m * (2 * lmax + 1 - m) / 2 > b) --m;
    while (m < lmax && (int64_t)(m + 1) * (2 * lmax - m) / 2 <= b) ++m;
    return m;
}

// Workgroup sum of 256 threads' values in a fixed order (deterministic); the result in thread 0.
__device__ __forceinline__ double block_sum256(double s, double *sh)
{
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int q = 128; q > 0; q >>= 1) {
        if ((int)threadIdx.x < q) sh[threadIdx.x] += sh[threadIdx.x + q];
        __syncthreads();
    }
    return sh[0];
}

// One alm index of the epilogue; returns the full-m weighted Re<x, out> of the index (for the
// fused inner product of a CG iteration).
template <typename T>
__device__ __forceinline__ double epilogue_one(int64_t i, const T *__restrict__ part, const int *__restrict__ wgstart,
                                               int nrb, int64_t nalm, const int *__restrict__ lof, int lmax,
                                               const double *__restrict__ kern, double lam,
                                               const double *__restrict__ xE, const double *__restrict__ xB,
                                               double *__restrict__ outE, double *__restrict__ outB, int proj)
{
    const int l = lof[i];
    const bool m0 = i <= lmax;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    if (l >= 2) {
        // ring blocks that started above l wrote nothing for it
        const int *ws = wgstart + (int64_t)m_of(i, l, lmax) * nrb;
        for (int rb = 0; rb < nrb; ++rb) {
            if (l < ws[rb]) continue;
            const T *q = part + ((int64_t)rb * nalm + i) * 4;
            s0 += (double)q[0];
            s1 += (double)q[1];
            s2 += (double)q[2];
            s3 += (double)q[3];
        }
    }
    // cE = -(2h + -2h)/2,  cB = (i/2)(2h - -2h)
    double eR = -0.5 * (s0 + s2), eI = -0.5 * (s1 + s3);
    double bR = -0.5 * (s1 - s3), bI = 0.5 * (s0 - s2);
    if (m0) eI = bI = 0.0;
    const double K = kern ? kern[l] : 1.0;
    eR *= K; eI *= K; bR *= K; bI *= K;
    if (xE) {
        eR += lam * xE[2 * i];
        bR += lam * xB[2 * i];
        if (!m0) {
            eI += lam * xE[2 * i + 1];
            bI += lam * xB[2 * i + 1];
        }
    }
    // block systems: the output block of the unknowns held at zero is zero
    if (proj == 1) bR = bI = 0.0;
    if (proj == 2) eR = eI = 0.0;
    outE[2 * i] = eR;
    outE[2 * i + 1] = eI;
    outB[2 * i] = bR;
    outB[2 * i + 1] = bI;
    if (!xE) return 0.0;
    const double wgt = m0 ? 1.0 : 2.0;
    return wgt * ((eR * xE[2 * i] + eI * xE[2 * i + 1]) + (bR * xB[2 * i] + bI * xB[2 * i + 1]));
}

// E/B combination of the adjoint's partial sums, harmonic diagonal and + lambda x (grid-stride over
// the alm indices).  With dot_red, also the workgroup partials of the full-m inner product <x, out>
// (one per workgroup, summed in a fixed order by the CG scalar kernel).
template <typename T>
__global__ __launch_bounds__(256) void k_epilogue(const T *__restrict__ part, const int *__restrict__ wgstart, int nrb,
                                                  int64_t nalm, const int *__restrict__ lof, int lmax,
                                                  const double *__restrict__ kern, double lam,
                                                  const double *__restrict__ xE, const double *__restrict__ xB,
                                                  double *__restrict__ outE, double *__restrict__ outB, int proj,
                                                  double *__restrict__ dot_red)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x)
        s += epilogue_one<T>(i, part, wgstart, nrb, nalm, lof, lmax, kern, lam, xE, xB, outE, outB, proj);
    if (dot_red) {
        const double t = block_sum256(s, sh);
        if (threadIdx.x == 0) dot_red[blockIdx.x] = t;
    }
}

// W = mask * ninv; block partials of sum(M N^-1), sum(M), #non-finite, #negative, sum over all pixels
__global__ void k_weights(const double *__restrict__ ninv, const uint8_t *__restrict__ mask, double *__restrict__ W,
                          int64_t npix, int ncount, double *__restrict__ red)
{
    // right-hand side rhs takes the N^-1 map rhs mod ncount
    const int rhs = blockIdx.y;
    const int64_t nofs = (int64_t)(rhs % ncount) * npix;
    __shared__ double sh[5][256];
    double a = 0, b = 0, c = 0, d = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = ninv[nofs + i];
        const bool obs = mask[i] != 0;
        if (!isfinite(v)) c += 1;
        if (v < 0) d += 1;
        const double w = obs ? v : 0.0;
        W[rhs * npix + i] = w;
        a += w;
        b += obs ? 1.0 : 0.0;
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    sh[2][threadIdx.x] = c;
    sh[3][threadIdx.x] = d;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) red[((int64_t)rhs * gridDim.x + blockIdx.x) * 4 + q] = sh[q][0];
}

// ================================================================================================
// Ring stage.  One workgroup per ring of N pixels.  Synthesis direction: fold F(m), |m| <= lmax,
// into the N bins (phase e^{i m phi0}), inverse DFT -> gamma at the pixels.  Adjoint direction:
// weight, forward DFT, unfold into every |m| <= lmax (phase e^{-i m phi0}) and multiply by the pixel
// area.  Three kernels cover the rings: a radix-8 FFT of the whole ring in LDS when N is a power of
// two, Bluestein's chirp-z over the whole ring when its convolution (a power-of-two length
// M >= 2N - 1) fits in LDS, else two interleaved sub-transforms of length N / 2, each by Bluestein.
// ================================================================================================
// e^{-i pi n^2 / L}
template <typename T> __device__ __forceinline__ cplx<T> chirp(int n, int L)
{
    return cconj<T>(cis_pi<T>(((int64_t)n * n) % (2 * (int64_t)L), L));
}

// Forward DFT of length L: y_k = sum_n x_n e^{-2 pi i n k / L}; x_n = get(u) for n = tid + NT u,
// y_k delivered as put(u, y) for k = tid + NT u (NT threads, L <= NT NU).
template <typename T, int NT = RT, int NU = RU, class Get, class Put>
__device__ __forceinline__ void dft_forward(cplx<T> *buf, const cplx<T> *bhat, int L, int M, int logM, bool blu,
                                            const cplx<T> *__restrict__ tw, int twn, Get &&get, Put &&put)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int n = tid + NT * u;
        if (n < L) {
            cplx<T> v = get(u);
            if (blu) v = cmul<T>(v, chirp<T>(n, L));
            buf[pd(brev(n, logM))] = v;
        }
    }
    for (int n = L + tid; n < M; n += NT) buf[pd(brev(n, logM))] = mk<T>(0, 0);
    __syncthreads();
    fft_dit<T, NT>(buf, M, tw, twn, -1);
    if (blu) {
        for (int n = tid; n < M; n += NT) buf[pd(n)] = cmul<T>(buf[pd(n)], bhat[n]);
        __syncthreads();
        fft_dif<T, NT>(buf, M, tw, twn, +1);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int kk = tid + NT * u;
            if (kk < L) put(u, cmul<T>(buf[pd(brev(kk, logM))], chirp<T>(kk, L)));
        }
    } else {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int kk = tid + NT * u;
            if (kk < L) put(u, buf[pd(kk)]);
        }
    }
    __syncthreads();
}

// Ring kernels.  MODE 0: F -> maps (o1, o2).  MODE 1: maps (g1, g2) x W -> G.  MODE 2: F -> maps x W -> G
// in place.  MODE 3 (gradient of the solve): F = Y K x as maps px; with o1, o2 holding q = Y K u, per
// pixel  o3 = M (omega q . (g - px) - c),   (o1, o2) = omega W q.
// ================================================================================================
// Ring stage for rings whose length N is a power of two (the equatorial belt when Nside is one):
// the length-N transforms run directly in LDS, one workgroup of RF threads per ring.  F is folded
// and G unfolded in m order, so neighbouring threads read and write neighbouring entries of the
// ring's row; each direction is one FFT of radix-8 passes (floor(log2 N / 3) of them, plus one
// radix-2 or radix-4 step for the remainder), both directions taking natural input to bit-reversed
// output.
// MODE as above.
// ================================================================================================
constexpr int RF = 1024;  // threads per ring workgroup
constexpr int RFU = 8;    // elements per thread: N <= RF * RFU

template <typename T> __device__ __forceinline__ cplx<T> to_t(double2 z) { return mk<T>((T)z.x, (T)z.y); }

// e^{i pi (k0 + k1 u) / den} for u = 0, 1, ... as a running FP64 product (one rounding per step)
struct PhaseSeq {
    double2 cur, step;
    __device__ __forceinline__ PhaseSeq(int64_t k0, int64_t k1, int64_t den)
        : cur(cis_pi<double>(k0, den)), step(cis_pi<double>(k1, den))
    {
    }
    __device__ __forceinline__ double2 next()
    {
        const double2 r = cur;
        cur = cmul<double>(cur, step);
        return r;
    }
};

// a / N for 0 <= a < 2^24 from a float reciprocal rN = 1 / N and one correction
__device__ __forceinline__ int udiv(int a, int N, float rN)
{
    int q = (int)((float)a * rN);
    const int r = a - q * N;
    if (r < 0) --q;
    else if (r >= N) ++q;
    return q;
}

// fold_bin / unfold_bin with the phase ph = e^{i pi bin / N} supplied (used when shift)
template <typename T>
__device__ __forceinline__ cplx<T> fold_bin_ph(const cplx<T> *__restrict__ F, int bin, int N, float rN, int shift,
                                               int lmax, const double2 &ph)
{
    const int tlo = -udiv(lmax + bin, N, rN);
    const int thi = (lmax >= bin) ? udiv(lmax - bin, N, rN) : -1;
    T sr = 0, si = 0;
    for (int t = tlo; t <= thi; ++t) {
        const int m = bin + N * t;
        cplx<T> f = (m >= 0) ? F[2 * m] : F[2 * (-m) + 1];
        if (shift && (t & 1)) f = mk<T>(-f.x, -f.y);
        sr += f.x;
        si += f.y;
    }
    cplx<T> s = mk<T>(sr, si);
    if (shift) s = cmul<T>(s, mk<T>((T)ph.x, (T)ph.y));
    return s;
}
template <typename T>
__device__ __forceinline__ void unfold_bin_ph(cplx<T> *__restrict__ G, int bin, int N, float rN, int shift, int lmax,
                                              cplx<T> y, const double2 &ph)
{
    if (shift) y = cmul<T>(y, mk<T>((T)ph.x, (T)-ph.y));
    const int tlo = -udiv(lmax + bin, N, rN);
    const int thi = (lmax >= bin) ? udiv(lmax - bin, N, rN) : -1;
    for (int t = tlo; t <= thi; ++t) {
        const int m = bin + N * t;
        const cplx<T> g = (shift && (t & 1)) ? mk<T>(-y.x, -y.y) : y;
        if (m > 0) G[2 * m] = g;
        else if (m < 0) G[2 * (-m) + 1] = g;
        else {
            G[0] = g;
            G[1] = g;
        }
    }
}

// Short rings (many orders per bin: 2 lmax + 1 > 8 N): the fold and the unfold run over the orders
// with the whole workgroup instead of one thread per bin.  Thread tau < Q N (Q = floor(RF / N)) takes
// the orders m = tau - lmax + Q N u, which all fall into one bin, sums them in order, and the Q
// partial sums of a bin are added in a fixed tree in LDS.  The unfold gives every order its own
// thread.  Both read and write F / G in m order, neighbouring threads on neighbouring entries.
__device__ __forceinline__ bool short_ring(int N, int lmax) { return 2 * lmax + 1 > 8 * N; }

// X_b = e^{i pi b shift / N} sum_{m = b + N t, |m| <= lmax} (-1)^{t shift} F(m) into buf[pd(b)], b < N;
// buf must hold RF complex entries; ends with a barrier
template <typename T>
__device__ void fold_short(const cplx<T> *__restrict__ F, cplx<T> *buf, int N, int shift, int lmax)
{
    const int tid = threadIdx.x, Q = RF / N, RFp = Q * N;
    if (tid < RFp) {
        const int r = tid - (tid / N) * N;
        const int b = ((r - lmax) % N + N) % N;             // bin of every order of this thread
        int t = (tid - lmax - b) / N;                         // m = b + N t for m = tid - lmax
        const bool flip = shift && (Q & 1);                   // t advances by Q per step
        bool neg = shift && (t & 1);
        T sr = 0, si = 0;
        for (int mm = tid; mm <= 2 * lmax; mm += RFp) {
            const int m = mm - lmax;
            const cplx<T> f = (m >= 0) ? F[2 * m] : F[2 * (-m) + 1];
            sr += neg ? -f.x : f.x;
            si += neg ? -f.y : f.y;
            neg ^= flip;
        }
        buf[tid] = mk<T>(sr, si);
    }
    for (int st = 1; st < Q; st <<= 1) {
        __syncthreads();
        if (tid < RFp) {
            const int q = tid / N;
            if ((q % (2 * st)) == 0 && q + st < Q) buf[tid] = cadd<T>(buf[tid], buf[tid + st * N]);
        }
    }
    __syncthreads();
    cplx<T> x = mk<T>(0, 0);
    int b = 0;
    if (tid < N) {
        b = ((tid - lmax) % N + N) % N;
        x = buf[tid];
        if (shift) x = cmul<T>(x, to_t<T>(cis_pi<double>(b, N)));
    }
    __syncthreads();
    if (tid < N) buf[pd(b)] = x;
    __syncthreads();
}

// G(m) = (-1)^{t shift} e^{-i pi b shift / N} Y_b for every |m| <= lmax, m = b + N t, from Y_b in
// buf[pd(b)] (already scaled); G(0) goes to both components
template <typename T>
__device__ void unfold_short(cplx<T> *__restrict__ G, cplx<T> *buf, int N, int shift, int lmax)
{
    const int tid = threadIdx.x;
    if (shift) {
        for (int b = tid; b < N; b += RF) buf[pd(b)] = cmul<T>(buf[pd(b)], to_t<T>(cis_pi<double>(-b, N)));
        __syncthreads();
    }
    for (int mm = tid; mm <= 2 * lmax; mm += RF) {
        const int m = mm - lmax;
        const int b = ((m % N) + N) % N, t = (m - b) / N;
        cplx<T> g = buf[pd(b)];
        if (shift && (t & 1)) g = mk<T>(-g.x, -g.y);
        if (m > 0) G[2 * m] = g;
        else if (m < 0) G[2 * (-m) + 1] = g;
        else {
            G[0] = g;
            G[1] = g;
        }
    }
}

template <typename T, int MODE>
__global__ __launch_bounds__(RF) void k_ring_full(cplx<T> *__restrict__ FG, int64_t fg_stride,
                                                  const double *__restrict__ g1, const double *__restrict__ g2,
                                                  double *__restrict__ o1, double *__restrict__ o2, int64_t map_stride,
                                                  const double *__restrict__ Wt, const RingInfo *__restrict__ rings,
                                                  const int *__restrict__ order, const cplx<T> *__restrict__ tw,
                                                  int twn, int lmax, double omega, double *__restrict__ o3,
                                                  const uint8_t *__restrict__ mask, const double *__restrict__ cdev)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    const int r = order[blockIdx.x];
    const int rhs = blockIdx.y;
    const RingInfo ri = rings[r];
    const int N = ri.nphi, shift = ri.shift;
    const int logN = 31 - __builtin_clz(N);
    cplx<T> *F = FG + rhs * fg_stride + (int64_t)r * (lmax + 1) * 2;
    const int tid = threadIdx.x;
    const int64_t pofs = rhs * map_stride + ri.ofs;
    const float rN = 1.0f / (float)N;
    cplx<T> v[RFU];

    const bool shortr = short_ring(N, lmax);
    if (MODE != 1) {
        // bin b collects F(m) e^{i m phi0} over m = b + N t, |m| <= lmax (phi0 = pi shift / N)
        if (shortr) {
            fold_short<T>(F, buf, N, shift, lmax);
        } else {
            PhaseSeq ph(tid, RF, N);  // e^{i pi b / N}
#pragma unroll
            for (int u = 0; u < RFU; ++u) {
                const int b = tid + RF * u;
                const double2 e = ph.next();
                if (b < N) buf[pd(b)] = fold_bin_ph<T>(F, b, N, rN, shift, lmax, e);
            }
            __syncthreads();
        }
        fft_dif<T, RF>(buf, N, tw, twn, +1);  // gamma_j = sum_b X_b e^{+2 pi i b j / N}, at brev(j)
#pragma unroll
        for (int u = 0; u < RFU; ++u) {
            const int j = tid + RF * u;
            if (j < N) v[u] = buf[pd(brev(j, logN))];
        }
        __syncthreads();
    }
    if (MODE == 0) {
#pragma unroll
        for (int u = 0; u < RFU; ++u) {
            const int j = tid + RF * u;
            if (j >= N) continue;
            o1[pofs + j] = (double)v[u].x;
            o2[pofs + j] = (double)v[u].y;
        }
        return;
    }
    if (MODE == 3) {
        const double c = *cdev;
#pragma unroll
        for (int u = 0; u < RFU; ++u) {
            const int j = tid + RF * u;
            if (j >= N) continue;
            const int64_t pix = pofs + j;
            const int64_t pm = ri.ofs + j;  // the mask is shared by all right-hand sides
            const double q1 = o1[pix], q2 = o2[pix];
            const double r1 = g1[pix] - (double)v[u].x, r2 = g2[pix] - (double)v[u].y;
            o3[pix] = mask[pm] ? omega * (q1 * r1 + q2 * r2) - c : 0.0;
            const double w = omega * Wt[pix];
            o1[pix] = w * q1;
            o2[pix] = w * q2;
        }
        return;
    }
    // h_j = W_j gamma_j (MODE 2) or W_j (g1 + i g2)_j (MODE 1), in natural order
#pragma unroll
    for (int u = 0; u < RFU; ++u) {
        const int j = tid + RF * u;
        if (j >= N) continue;
        const int64_t pix = pofs + j;
        if (MODE == 1) {
            const T w = Wt ? (T)Wt[pix] : (T)1;
            buf[pd(j)] = mk<T>((T)g1[pix] * w, (T)g2[pix] * w);
        } else {
            buf[pd(j)] = cscale<T>(v[u], (T)Wt[pix]);
        }
    }
    __syncthreads();
    fft_dif<T, RF>(buf, N, tw, twn, -1);  // Y_b = sum_j h_j e^{-2 pi i b j / N}, at brev(b)
    const T om = (T)omega;
    if (shortr) {
        // bins to natural order, scaled (read all, then write: the two orders overlap)
#pragma unroll
        for (int u = 0; u < RFU; ++u) {
            const int b = tid + RF * u;
            if (b < N) v[u] = cscale<T>(buf[pd(brev(b, logN))], om);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < RFU; ++u) {
            const int b = tid + RF * u;
            if (b < N) buf[pd(b)] = v[u];
        }
        __syncthreads();
        unfold_short<T>(F, buf, N, shift, lmax);
        return;
    }
    PhaseSeq ph(tid, RF, N);
#pragma unroll
    for (int u = 0; u < RFU; ++u) {
        const int b = tid + RF * u;
        const double2 e = ph.next();
        if (b < N) unfold_bin_ph<T>(F, b, N, rN, shift, lmax, cscale<T>(buf[pd(brev(b, logN))], om), e);
    }
}

// ================================================================================================
// Ring stage for rings of any length N whose Bluestein convolution (length M >= 2N - 1, a power of
// two) fits in LDS: one DFT of the whole ring per direction by Bluestein's chirp-z, with the chirp
// spectrum of length N from the plan's table; fold and unfold in m order as in k_ring_full.
// MODE as above.
// ================================================================================================
constexpr int RBU = 4;  // elements per thread: N <= RF * RBU

template <typename T, int MODE>
__global__ __launch_bounds__(RF) void k_ring_bfull(cplx<T> *__restrict__ FG, int64_t fg_stride,
                                                   const double *__restrict__ g1, const double *__restrict__ g2,
                                                   double *__restrict__ o1, double *__restrict__ o2, int64_t map_stride,
                                                   const double *__restrict__ Wt, const RingInfo *__restrict__ rings,
                                                   const int *__restrict__ order, const cplx<T> *__restrict__ tw,
                                                   int twn, int lmax, double omega, double *__restrict__ o3,
                                                   const uint8_t *__restrict__ mask, const double *__restrict__ cdev,
                                                   const cplx<T> *__restrict__ bhat_all)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    const int r = order[blockIdx.x];
    const int rhs = blockIdx.y;
    const RingInfo ri = rings[r];
    const int N = ri.nphi, shift = ri.shift, M = ri.M;
    const int logM = 31 - __builtin_clz(M);
    const cplx<T> *bhat = bhat_all + ri.bofs;
    cplx<T> *F = FG + rhs * fg_stride + (int64_t)r * (lmax + 1) * 2;
    const int tid = threadIdx.x;
    const int64_t pofs = rhs * map_stride + ri.ofs;
    const float rN = 1.0f / (float)N;
    cplx<T> v[RBU];

    const bool shortr = short_ring(N, lmax);
    if (MODE != 1) {
        // gamma_j = sum_b X_b e^{+2 pi i b j / N} = conj(DFT(conj X))_j; get and put run in u order
        if (shortr) {
            fold_short<T>(F, buf, N, shift, lmax);
#pragma unroll
            for (int u = 0; u < RBU; ++u) {
                const int b = tid + RF * u;
                v[u] = b < N ? buf[pd(b)] : mk<T>(0, 0);
            }
            __syncthreads();
            dft_forward<T, RF, RBU>(
                buf, bhat, N, M, logM, true, tw, twn, [&](int u) { return cconj<T>(v[u]); },
                [&](int u, cplx<T> y) { v[u] = cconj<T>(y); });
        } else {
            PhaseSeq ph(tid, RF, N);  // e^{i pi b / N} along b = tid + RF u
            dft_forward<T, RF, RBU>(
                buf, bhat, N, M, logM, true, tw, twn,
                [&](int u) {
                    const double2 e = ph.next();
                    return cconj<T>(fold_bin_ph<T>(F, tid + RF * u, N, rN, shift, lmax, e));
                },
                [&](int u, cplx<T> y) { v[u] = cconj<T>(y); });
        }
    }
    if (MODE == 0) {
#pragma unroll
        for (int u = 0; u < RBU; ++u) {
            const int j = tid + RF * u;
            if (j >= N) continue;
            o1[pofs + j] = (double)v[u].x;
            o2[pofs + j] = (double)v[u].y;
        }
        return;
    }
    if (MODE == 3) {
        const double c = *cdev;
#pragma unroll
        for (int u = 0; u < RBU; ++u) {
            const int j = tid + RF * u;
            if (j >= N) continue;
            const int64_t pix = pofs + j;
            const int64_t pm = ri.ofs + j;  // the mask is shared by all right-hand sides
            const double q1 = o1[pix], q2 = o2[pix];
            const double r1 = g1[pix] - (double)v[u].x, r2 = g2[pix] - (double)v[u].y;
            o3[pix] = mask[pm] ? omega * (q1 * r1 + q2 * r2) - c : 0.0;
            const double w = omega * Wt[pix];
            o1[pix] = w * q1;
            o2[pix] = w * q2;
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < RBU; ++u) {
        const int j = tid + RF * u;
        if (j >= N) continue;
        const int64_t pix = pofs + j;
        if (MODE == 1) {
            const T w = Wt ? (T)Wt[pix] : (T)1;
            v[u] = mk<T>((T)g1[pix] * w, (T)g2[pix] * w);
        } else {
            v[u] = cscale<T>(v[u], (T)Wt[pix]);
        }
    }
    const T om = (T)omega;
    if (shortr) {
        dft_forward<T, RF, RBU>(
            buf, bhat, N, M, logM, true, tw, twn, [&](int u) { return v[u]; },
            [&](int u, cplx<T> y) { v[u] = cscale<T>(y, om); });
#pragma unroll
        for (int u = 0; u < RBU; ++u) {
            const int b = tid + RF * u;
            if (b < N) buf[pd(b)] = v[u];
        }
        __syncthreads();
        unfold_short<T>(F, buf, N, shift, lmax);
        return;
    }
    PhaseSeq ph(tid, RF, N);
    dft_forward<T, RF, RBU>(
        buf, bhat, N, M, logM, true, tw, twn, [&](int u) { return v[u]; },
        [&](int u, cplx<T> y) {
            const double2 e = ph.next();
            unfold_bin_ph<T>(F, tid + RF * u, N, rN, shift, lmax, cscale<T>(y, om), e);
        });
}

// ================================================================================================
// Ring stage for the remaining rings (whole-ring convolution too long for LDS): the length-N DFT
// (N even) splits into two interleaved sub-DFTs of length L = N / 2 over the even and odd bins, each
// by Bluestein with the chirp spectrum of length L; the radix-2 step in registers combines them:
//   synthesis  gamma[j1] = Y0[j1] + w^j1 Y1[j1],  gamma[j1 + L] = Y0[j1] - w^j1 Y1[j1],  w = e^{2 pi i/N}
//   adjoint    u_q[j1] = w^{-q j1} (h[j1] + (-1)^q h[j1 + L]),  bins 2 k + q = DFT_L(u_q)[k].
// MODE as above.
// ================================================================================================
template <typename T, int MODE>
__global__ __launch_bounds__(RF) void k_ring_b2(cplx<T> *__restrict__ FG, int64_t fg_stride,
                                                const double *__restrict__ g1, const double *__restrict__ g2,
                                                double *__restrict__ o1, double *__restrict__ o2, int64_t map_stride,
                                                const double *__restrict__ Wt, const RingInfo *__restrict__ rings,
                                                const int *__restrict__ order, const cplx<T> *__restrict__ tw,
                                                int twn, int lmax, double omega, double *__restrict__ o3,
                                                const uint8_t *__restrict__ mask, const double *__restrict__ cdev,
                                                const cplx<T> *__restrict__ bhat_all)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    const int r = order[blockIdx.x];
    const int rhs = blockIdx.y;
    const RingInfo ri = rings[r];
    const int N = ri.nphi, L = N / 2, shift = ri.shift, M = ri.M;
    const int logM = 31 - __builtin_clz(M);
    const cplx<T> *bhat = bhat_all + ri.bofs;
    cplx<T> *F = FG + rhs * fg_stride + (int64_t)r * (lmax + 1) * 2;
    const int tid = threadIdx.x;
    const int64_t pofs = rhs * map_stride + ri.ofs;
    const float rN = 1.0f / (float)N;
    cplx<T> v[RBU][2];

    if (MODE != 1) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            // Y_q = inverse DFT_L of the bins 2 k + q; get and put run in u order
            PhaseSeq ph(2 * tid + q, 2 * RF, N);  // e^{i pi b / N} along b = 2 (tid + RF u) + q
            dft_forward<T, RF, RBU>(
                buf, bhat, L, M, logM, true, tw, twn,
                [&](int u) {
                    const double2 e = ph.next();
                    return cconj<T>(fold_bin_ph<T>(F, 2 * (tid + RF * u) + q, N, rN, shift, lmax, e));
                },
                [&](int u, cplx<T> y) { v[u][q] = cconj<T>(y); });
        }
        PhaseSeq pw(2 * tid, 2 * RF, N);  // e^{2 pi i j1 / N}
#pragma unroll
        for (int u = 0; u < RBU; ++u) {
            const int j1 = tid + RF * u;
            const double2 w = pw.next();
            if (j1 >= L) continue;
            const cplx<T> t = cmul<T>(to_t<T>(w), v[u][1]), a = v[u][0];
            v[u][0] = cadd<T>(a, t);
            v[u][1] = csub<T>(a, t);
        }
    }
    if (MODE == 0) {
#pragma unroll
        for (int u = 0; u < RBU; ++u) {
            const int j1 = tid + RF * u;
            if (j1 >= L) continue;
#pragma unroll
            for (int j2 = 0; j2 < 2; ++j2) {
                o1[pofs + j1 + L * j2] = (double)v[u][j2].x;
                o2[pofs + j1 + L * j2] = (double)v[u][j2].y;
            }
        }
        return;
    }
    if (MODE == 3) {
        const double c = *cdev;
#pragma unroll
        for (int u = 0; u < RBU; ++u) {
            const int j1 = tid + RF * u;
            if (j1 >= L) continue;
#pragma unroll
            for (int j2 = 0; j2 < 2; ++j2) {
                const int64_t pix = pofs + j1 + L * j2;
                const int64_t pm = ri.ofs + j1 + L * j2;  // the mask is shared by all right-hand sides
                const double q1 = o1[pix], q2 = o2[pix];
                const double r1 = g1[pix] - (double)v[u][j2].x, r2 = g2[pix] - (double)v[u][j2].y;
                o3[pix] = mask[pm] ? omega * (q1 * r1 + q2 * r2) - c : 0.0;
                const double w = omega * Wt[pix];
                o1[pix] = w * q1;
                o2[pix] = w * q2;
            }
        }
        return;
    }
    PhaseSeq pw(2 * tid, 2 * RF, N);
#pragma unroll
    for (int u = 0; u < RBU; ++u) {
        const int j1 = tid + RF * u;
        const double2 w = pw.next();
        if (j1 >= L) continue;
#pragma unroll
        for (int j2 = 0; j2 < 2; ++j2) {
            const int64_t pix = pofs + j1 + L * j2;
            if (MODE == 1) {
                const T wt = Wt ? (T)Wt[pix] : (T)1;
                v[u][j2] = mk<T>((T)g1[pix] * wt, (T)g2[pix] * wt);
            } else {
                v[u][j2] = cscale<T>(v[u][j2], (T)Wt[pix]);
            }
        }
        const cplx<T> h0 = v[u][0], h1 = v[u][1];
        v[u][0] = cadd<T>(h0, h1);
        v[u][1] = cmul<T>(cconj<T>(to_t<T>(w)), csub<T>(h0, h1));
    }
    const T om = (T)omega;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        PhaseSeq pf(2 * tid + q, 2 * RF, N);  // put runs in u order
        dft_forward<T, RF, RBU>(
            buf, bhat, L, M, logM, true, tw, twn, [&](int u) { return v[u][q]; },
            [&](int u, cplx<T> y) {
                const double2 e = pf.next();
                unfold_bin_ph<T>(F, 2 * (tid + RF * u) + q, N, rN, shift, lmax, cscale<T>(y, om), e);
            });
    }
}

// ================================================================================================
// Register-resident ring transforms for transform lengths M = 2^LOGM, LOGM = 12 or 13 (the equatorial
// belt and the long cap rings of Nside 1024 and 2048).  A workgroup of NT = M / 16 threads holds the
// M points of a transform in registers, 16 per thread, and runs the radix-2 stages four at a time
// in registers.  Between the three register passes the points move through LDS in two exchanges;
// every access pattern is contiguous across lanes (or has stride 2 with one pad slot per 32), so the
// exchanges are free of bank conflicts.  With the LDS holding one component at a time in FP64, two
// rings share a compute unit.
//
// Layouts: in the layout of stride S, register k of thread t holds position
//   pos = (t mod S) + S k + 16 S (t div S),
// so the register index runs over the four position bits log2 S .. log2 S + 3.  The three layouts
// have S0 = M / 16 (bits LOGM-1 .. LOGM-4: thread t holds t + NT k, the natural order of the fold
// and the unfold), S1 = M / 256 and S2 = M / 4096 (bits 3..0 for LOGM = 12; bits 4..1 for
// LOGM = 13, whose bit 0 is the lane's bit 0 and is crossed with a DPP swap of neighbouring lanes).
//
// A decimation-in-frequency transform (natural input, bit-reversed output) runs the passes S0, S1,
// S2; a decimation-in-time transform (bit-reversed input, natural output) runs them back.  Between
// the two the values sit at bit-reversed positions, where the pointwise step of each use happens:
// the pixel weights W (belt rings: inverse DFT, x W, forward DFT) or the chirp spectrum of a
// Bluestein convolution (forward FFT, x bhat, inverse FFT).
// ================================================================================================
template <int LOGM> struct R16 {
    static constexpr int M = 1 << LOGM, NT = M / 16;
    static constexpr int S0 = NT, S1 = 1 << (LOGM - 8), S2 = 1 << (LOGM - 12);
};

template <int S> __device__ __forceinline__ int lpos(int t, int k) { return (t & (S - 1)) + S * k + 16 * S * (t / S); }

template <int LOGM> __device__ __forceinline__ int brevm(int p) { return (int)(__builtin_bitreverse32((unsigned)p) >> (32 - LOGM)); }

// x, made opaque to the compiler at this point: loads indexed by it are not hoisted above it (keeps
// the twiddle, weight and chirp-spectrum loads of a later phase from holding registers early)
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// z W_16^q, W_16 = e^{-2 pi i / 16} for sign -1 (its conjugate for +1), q in [0, 8) a constant after
// unrolling
template <typename T> __device__ __forceinline__ cplx<T> mul_w16(cplx<T> z, int q, int sign)
{
    switch (q) {
    case 0: return z;
    case 2: return rot8<T>(z, sign);
    case 4: return rot4<T>(z, sign);
    case 6: return rot8_3<T>(z, sign);
    default: {
        const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
        const T c = q == 1 ? c1 : q == 3 ? s1 : q == 5 ? -s1 : -c1;
        const T s = q == 1 ? s1 : q == 3 ? c1 : q == 5 ? c1 : s1;
        return cmul<T>(z, mk<T>(c, sign < 0 ? -s : s));
    }
    }
}

// base twiddles of a pass at stride S: B[j] = W_{2 S 2^j}^u, u = t mod S (table e^{-2 pi i k / twn})
template <typename T, int S>
__device__ __forceinline__ void pass_tw(cplx<T> (&B)[4], const cplx<T> *__restrict__ tw, int twn, int t, int sign)
{
    const int u = opaque(t) & (S - 1);
#pragma unroll
    for (int j = 0; j < 4; ++j) B[j] = twid<T>(tw, u * (twn / (S << (j + 1))), sign);
}

// four DIF stages of spans 8S, 4S, 2S, S: (a, b) -> (a + b, (a - b) W_{2h}^pos), pos = u + S (k mod 2^j)
template <typename T, int S>
__device__ __forceinline__ void dif_pass(cplx<T> (&v)[16], const cplx<T> *__restrict__ tw, int twn, int t, int sign)
{
    cplx<T> B[4];
    if (S > 1) pass_tw<T, S>(B, tw, twn, t, sign);
#pragma unroll
    for (int j = 3; j >= 0; --j) {
        const int s = 1 << j;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k & s) continue;
            const cplx<T> a = v[k], b = v[k + s];
            v[k] = cadd<T>(a, b);
            cplx<T> d = csub<T>(a, b);
            if (S > 1) d = cmul<T>(d, B[j]);
            v[k + s] = mul_w16<T>(d, (k & (s - 1)) << (3 - j), sign);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

// four DIT stages of spans S, 2S, 4S, 8S: (a, b) -> (a + w b, a - w b), w = W_{2h}^pos
template <typename T, int S>
__device__ __forceinline__ void dit_pass(cplx<T> (&v)[16], const cplx<T> *__restrict__ tw, int twn, int t, int sign)
{
    cplx<T> B[4];
    if (S > 1) pass_tw<T, S>(B, tw, twn, t, sign);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int s = 1 << j;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k & s) continue;
            cplx<T> b = v[k + s];
            if (S > 1) b = cmul<T>(b, B[j]);
            b = mul_w16<T>(b, (k & (s - 1)) << (3 - j), sign);
            const cplx<T> a = v[k];
            v[k] = cadd<T>(a, b);
            v[k + s] = csub<T>(a, b);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

// move the 16 registers of every thread from layout SA to layout SB through LDS (lds: M + M / 32
// scalars of T when SPLIT, else as many complex values); the leading barrier retires the reads of
// the previous exchange.  In every layout the padded slot of register k is the padded slot of
// register 0 plus pd(S k), so each access is a base register plus a constant offset.
template <typename T, bool SPLIT, int SA, int SB>
__device__ __forceinline__ void exchange16(cplx<T> (&v)[16], T *lds, int t)
{
    const int tt = opaque(t);
    const int ba = pd(lpos<SA>(tt, 0)), bb = pd(lpos<SB>(tt, 0));
    if constexpr (SPLIT) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) lds[ba + pd(SA * k)] = v[k].x;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k].x = lds[bb + pd(SB * k)];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) lds[ba + pd(SA * k)] = v[k].y;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k].y = lds[bb + pd(SB * k)];
    } else {
        cplx<T> *b = reinterpret_cast<cplx<T> *>(lds);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) b[ba + pd(SA * k)] = v[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = b[bb + pd(SB * k)];
    }
}

// the value of the neighbouring lane (lane ^ 1)
template <typename T> __device__ __forceinline__ cplx<T> lane_swap1(cplx<T> z)
{
    return mk<T>(dpp_mov<0xB1>(z.x), dpp_mov<0xB1>(z.y));
}

// radix-2 stage on position bit 0 held across neighbouring lanes (LOGM = 13): (a, b) -> (a + b, a - b)
// with a in the even lane; its twiddle is 1 in both directions
template <typename T> __device__ __forceinline__ void lane_stage(cplx<T> (&v)[16], int c)
{
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const cplx<T> p = lane_swap1<T>(v[k]);
        v[k] = c ? csub<T>(p, v[k]) : cadd<T>(v[k], p);
    }
    __builtin_amdgcn_sched_barrier(0);
}

// full DIF from layout S0 (natural) to the bit-reversed positions of layout S2, all stages done
template <typename T, int LOGM, bool SPLIT>
__device__ __forceinline__ void fft16_dif(cplx<T> (&v)[16], T *lds, const cplx<T> *__restrict__ tw, int twn, int t,
                                          int sign)
{
    using G = R16<LOGM>;
    dif_pass<T, G::S0>(v, tw, twn, t, sign);
    exchange16<T, SPLIT, G::S0, G::S1>(v, lds, t);
    dif_pass<T, G::S1>(v, tw, twn, t, sign);
    exchange16<T, SPLIT, G::S1, G::S2>(v, lds, t);
    dif_pass<T, G::S2>(v, tw, twn, t, sign);
    if constexpr (LOGM == 13) lane_stage<T>(v, t & 1);
}

// full DIT from the bit-reversed positions of layout S2 to the natural layout S0
template <typename T, int LOGM, bool SPLIT>
__device__ __forceinline__ void fft16_dit(cplx<T> (&v)[16], T *lds, const cplx<T> *__restrict__ tw, int twn, int t,
                                          int sign)
{
    using G = R16<LOGM>;
    if constexpr (LOGM == 13) lane_stage<T>(v, t & 1);
    dit_pass<T, G::S2>(v, tw, twn, t, sign);
    exchange16<T, SPLIT, G::S2, G::S1>(v, lds, t);
    dit_pass<T, G::S1>(v, tw, twn, t, sign);
    exchange16<T, SPLIT, G::S1, G::S0>(v, lds, t);
    dit_pass<T, G::S0>(v, tw, twn, t, sign);
}

// e^{-i pi n^2 / N} along n = t + NT k, k = 0, 1, ... as running FP64 products (exact start values):
// c_{k+1} = c_k r_k, r_{k+1} = r_k q
struct ChirpSeq {
    double2 c, r, q;
    __device__ __forceinline__ ChirpSeq(int t, int NT, int N)
    {
        const int64_t twoN = 2 * (int64_t)N, tt = t, nt = NT;
        c = cis_pi<double>(-((tt * tt) % twoN), N);
        r = cis_pi<double>(-((2 * nt * tt + nt * nt) % twoN), N);
        q = cis_pi<double>(-((2 * nt * nt) % twoN), N);
    }
    __device__ __forceinline__ double2 next()
    {
        const double2 o = c;
        c = cmul<double>(c, r);
        r = cmul<double>(r, q);
        return o;
    }
};

// keeps the compiler from moving memory accesses across this point: the per-register loops over
// global memory run in groups of four, which bounds the registers that loads in flight hold
__device__ __forceinline__ void mem_fence_compiler()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// One Bluestein DFT of length L on v (natural order n = t + NT k, zero from n = L): chirp, forward
// FFT, x bhat (the chirp spectrum in register order), inverse FFT, chirp
template <typename T, int LOGM, bool SPLIT>
__device__ __forceinline__ void bluestein16(cplx<T> (&v)[16], T *lds, const cplx<T> *__restrict__ tw, int twn, int t,
                                            int L, const cplx<T> *__restrict__ bh)
{
    // the input is zero from n = L and L <= M / 2: registers 8 .. 15 start at zero, and their outputs
    // (n >= M / 2) are not used
    constexpr int NT = R16<LOGM>::NT;
    {
        ChirpSeq ch(opaque(t), NT, L);
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = cmul<T>(v[k], to_t<T>(ch.next()));
    }
#pragma unroll
    for (int k = 8; k < 16; ++k) v[k] = mk<T>(0, 0);
    fft16_dif<T, LOGM, SPLIT>(v, lds, tw, twn, t, -1);
    const int tt = opaque(t);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        v[k] = cmul<T>(v[k], bh[k * NT + tt]);
        if ((k & 3) == 3) mem_fence_compiler();
    }
    fft16_dit<T, LOGM, SPLIT>(v, lds, tw, twn, t, +1);
    ChirpSeq ch(opaque(t), NT, L);
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = cmul<T>(v[k], to_t<T>(ch.next()));
}

// fold of the bins b = NH n + q, n = t + NT k < L, into v (conjugated: the synthesis transform is
// conj(DFT(conj X)))
template <typename T, int NT, int NH>
__device__ __forceinline__ void fold16_conj(cplx<T> (&v)[16], const cplx<T> *__restrict__ F, int t, int q, int L,
                                            int N, float rN, int shift, int lmax)
{
    PhaseSeq ph(NH * t + q, NH * NT, N);  // e^{i pi b / N} along b = NH (t + NT k) + q
#pragma unroll
    for (int k = 0; k < 8; ++k) {  // n < L <= 8 NT
        const int n = t + NT * k, b = NH * n + q;
        const double2 e = ph.next();
        v[k] = n < L ? cconj<T>(fold_bin_ph<T>(F, b, N, rN, shift, lmax, e)) : mk<T>(0, 0);
        if ((k & 3) == 3) mem_fence_compiler();
    }
}

// unfold of the bins b = NH n + q, n = t + NT k < L, from v with the pixel area
template <typename T, int NT, int NH, int K>
__device__ __forceinline__ void unfold16(const cplx<T> (&v)[16], cplx<T> *__restrict__ G, int t, int q, int L, int N,
                                         float rN, int shift, int lmax, T om)
{
    PhaseSeq ph(NH * t + q, NH * NT, N);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int n = t + NT * k;
        const double2 e = ph.next();
        if (n < L) unfold_bin_ph<T>(G, NH * n + q, N, rN, shift, lmax, cscale<T>(v[k], om), e);
        if ((k & 3) == 3) mem_fence_compiler();
    }
}

// The per-pixel step of one half of the registers: MODE 0 stores gamma, MODE 3 the gradient
// epilogue, MODE 1 loads W (g1 + i g2), MODE 2 multiplies by W.  Pixel of register k: brev(pos) of
// layout S2 (BREV), else p0 + NT k (below lim).
template <typename T, int MODE, int LOGM, bool BREV, int K, int KA>
__device__ __forceinline__ void pixels16(cplx<T> (&v)[KA], int tp, int p0, int lim, int64_t pofs, int64_t mofs,
                                         const double *__restrict__ g1, const double *__restrict__ g2,
                                         double *__restrict__ o1, double *__restrict__ o2, const double *__restrict__ Wt,
                                         double omega, double *__restrict__ o3, const uint8_t *__restrict__ mask,
                                         double cc)
{
    constexpr int NT = R16<LOGM>::NT;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int j = BREV ? brevm<LOGM>(lpos<R16<LOGM>::S2>(tp, k)) : p0 + NT * k;
        const bool live = BREV || tp + NT * k < lim;
        if (MODE == 0) {
            if (live) {
                o1[pofs + j] = (double)v[k].x;
                o2[pofs + j] = (double)v[k].y;
            }
        } else if (MODE == 3) {
            if (live) {
                const int64_t pix = pofs + j;
                const double q1 = o1[pix], q2 = o2[pix];
                const double r1 = g1[pix] - (double)v[k].x, r2 = g2[pix] - (double)v[k].y;
                o3[pix] = mask[mofs + j] ? omega * (q1 * r1 + q2 * r2) - cc : 0.0;
                const double w = omega * Wt[pix];
                o1[pix] = w * q1;
                o2[pix] = w * q2;
            }
        } else if (!live) {
            v[k] = mk<T>(0, 0);
        } else if (MODE == 1) {
            const int64_t pix = pofs + j;
            const T w = Wt ? (T)Wt[pix] : (T)1;
            v[k] = mk<T>((T)g1[pix] * w, (T)g2[pix] * w);
        } else {
            v[k] = cscale<T>(v[k], (T)Wt[pofs + j]);
        }
        if ((k & 3) == 3) mem_fence_compiler();
    }
}

// Ring kernel of the register engine.  KIND 0: rings whose length N is the transform length M (an
// inverse DIF FFT to the pixels, a forward DIT FFT back).  KIND 1: rings transformed whole by
// Bluestein's chirp-z with a convolution of length M >= 2N - 1.  KIND 2: rings of even length N = 2L
// split into two interleaved sub-transforms of length L over the even and odd bins, each by Bluestein
// with M >= 2L - 1, combined by a radix-2 step in registers:
//   synthesis  gamma[j] = Y0[j] + w^j Y1[j],  gamma[j + L] = Y0[j] - w^j Y1[j],  w = e^{2 pi i / N}
//   adjoint    u_q[j] = w^{-q j} (h[j] + (-1)^q h[j + L]),  bins 2 k + q = DFT_L(u_q)[k].
// bhat_r holds the chirp spectrum of the transformed length in register order (thread t, register k
// of layout S2 at index k NT + t).  MODE as for the other ring kernels.
template <typename T> struct Ring16Waves {
    // FP64 holds 16 complex values and, in the split form, a second set of 16 per thread
    static constexpr int value = std::is_same<T, double>::value ? 2 : 4;
};

template <typename T, int MODE, int LOGM, int KIND>
__global__ __launch_bounds__(R16<LOGM>::NT) __attribute__((amdgpu_waves_per_eu(Ring16Waves<T>::value))) void k_ring16(
    cplx<T> *__restrict__ FG, int64_t fg_stride, const double *__restrict__ g1, const double *__restrict__ g2,
    double *__restrict__ o1, double *__restrict__ o2, int64_t map_stride, const double *__restrict__ Wt,
    const RingInfo *__restrict__ rings, const int *__restrict__ order, const cplx<T> *__restrict__ tw, int twn,
    int lmax, double omega, double *__restrict__ o3, const uint8_t *__restrict__ mask, const double *__restrict__ cdev,
    const cplx<T> *__restrict__ bhat_r)
{
    using G = R16<LOGM>;
    constexpr int NT = G::NT;
    constexpr int NH = KIND == 2 ? 2 : 1;  // sub-transforms per ring
    // exchanges one component at a time in FP64, and in FP32 for the split rings, which also keep
    // one half-ring in LDS (two workgroups per compute unit either way)
    constexpr bool SPLIT = std::is_same<T, double>::value || KIND == 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    // KIND 2: the half-ring waiting while the other is transformed, thread t's register k at k NT + t
    cplx<T> *stash = reinterpret_cast<cplx<T> *>(lds + (G::M + G::M / 32));
    const int r = order[blockIdx.x];
    const int rhs = blockIdx.y;
    const RingInfo ri = rings[r];
    const int N = ri.nphi, shift = ri.shift;
    const int L = KIND == 2 ? N / 2 : N;  // transformed length
    cplx<T> *F = FG + rhs * fg_stride + (int64_t)r * (lmax + 1) * 2;
    const int t = threadIdx.x;
    const int64_t pofs = rhs * map_stride + ri.ofs;
    const float rN = 1.0f / (float)N;
    const cplx<T> *bh = KIND ? bhat_r + ri.rofs : nullptr;
    cplx<T> v[16];
    cplx<T> u[KIND == 2 ? 8 : 1];  // KIND 2: the values at pixels n + L (n = t + NT k < L <= 8 NT)
    auto stash_put = [&](const cplx<T> *a) {
#pragma unroll
        for (int k = 0; k < 8; ++k) stash[k * NT + t] = a[k];
    };
    auto stash_get = [&](cplx<T> *a) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = stash[k * NT + t];
    };

    if (MODE != 1) {
        // gamma_j = sum_b X_b e^{+2 pi i b j / N}
        if constexpr (KIND == 0) {
            PhaseSeq ph(t, NT, N);  // e^{i pi b / N} along b = t + NT k
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                v[k] = fold_bin_ph<T>(F, t + NT * k, N, rN, shift, lmax, ph.next());
                if ((k & 3) == 3) mem_fence_compiler();
            }
            fft16_dif<T, LOGM, SPLIT>(v, lds, tw, twn, t, +1);  // gamma at pixel brev(pos)
        } else {
            fold16_conj<T, NT, NH>(v, F, t, 0, L, N, rN, shift, lmax);
            bluestein16<T, LOGM, SPLIT>(v, lds, tw, twn, t, L, bh);
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = cconj<T>(v[k]);
            if constexpr (KIND == 2) {
                // Y0 waits in LDS while Y1 is transformed in v (each thread reads back its own slots)
                stash_put(v);
                fold16_conj<T, NT, NH>(v, F, t, 1, L, N, rN, shift, lmax);
                bluestein16<T, LOGM, SPLIT>(v, lds, tw, twn, t, L, bh);
                stash_get(u);
                PhaseSeq pw(2 * t, 2 * NT, N);  // e^{2 pi i n / N}
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const cplx<T> a = u[k], b = cmul<T>(to_t<T>(pw.next()), cconj<T>(v[k]));
                    v[k] = cadd<T>(a, b);
                    u[k] = csub<T>(a, b);
                }
            }
        }
    }
    const int tp = opaque(t);
    const double cc = MODE == 3 ? *cdev : 0.0;
    pixels16<T, MODE, LOGM, KIND == 0, KIND == 0 ? 16 : 8, 16>(v, tp, tp, L, pofs, ri.ofs, g1, g2, o1, o2, Wt, omega,
                                                               o3, mask, cc);
    if constexpr (KIND == 2)
        pixels16<T, MODE, LOGM, false, 8, 8>(u, tp, tp + L, L, pofs, ri.ofs, g1, g2, o1, o2, Wt, omega, o3, mask, cc);
    if (MODE == 0 || MODE == 3) return;
    // Y_b = sum_j h_j e^{-2 pi i b j / N}, then unfold with the pixel area
    const T om = (T)omega;
    if constexpr (KIND == 0) {
        fft16_dit<T, LOGM, SPLIT>(v, lds, tw, twn, t, -1);  // natural bins b = t + NT k
        unfold16<T, NT, 1, 16>(v, F, t, 0, N, N, rN, shift, lmax, om);
    } else {
        if constexpr (KIND == 2) {
            PhaseSeq pw(2 * t, 2 * NT, N);  // e^{2 pi i n / N}
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const cplx<T> a = v[k], b = u[k];
                v[k] = cadd<T>(a, b);
                u[k] = cmul<T>(cconj<T>(to_t<T>(pw.next())), csub<T>(a, b));
            }
        }
        if constexpr (KIND == 2) stash_put(u);
        bluestein16<T, LOGM, SPLIT>(v, lds, tw, twn, t, L, bh);
        unfold16<T, NT, NH, 8>(v, F, t, 0, L, N, rN, shift, lmax, om);
        if constexpr (KIND == 2) {
            stash_get(v);
            bluestein16<T, LOGM, SPLIT>(v, lds, tw, twn, t, L, bh);
            unfold16<T, NT, NH, 8>(v, F, t, 1, L, N, rN, shift, lmax, om);
        }
    }
}

// Chirp spectra of the register-engine Bluestein rings in register order: out[o + k NT + t] =
// bhat[brev(pos)] with pos the layout-S2 position of register k of thread t (one block per length).
template <typename T, int LOGM>
__global__ void k_bhat_reorder(const cplx<T> *__restrict__ bhat, const int64_t *__restrict__ src_ofs,
                               const int64_t *__restrict__ dst_ofs, cplx<T> *__restrict__ out)
{
    using G = R16<LOGM>;
    const int64_t so = src_ofs[blockIdx.x], d = dst_ofs[blockIdx.x];
    for (int t = threadIdx.x; t < G::NT; t += blockDim.x)
#pragma unroll
        for (int k = 0; k < 16; ++k) out[d + k * G::NT + t] = bhat[so + brevm<LOGM>(lpos<G::S2>(t, k))];
}

// ================================================================================================
// vector kernels (FP64): full-m inner product and the CG updates
// ================================================================================================
constexpr int RED_BLOCKS = 512;

__global__ void k_dot_part(const double *__restrict__ a, const double *__restrict__ b, int64_t n, int64_t nalm, int lmax,
                           double *__restrict__ red)
{
    __shared__ double sh[256];
    double s = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double w = ((i % nalm) <= lmax) ? 1.0 : 2.0;
        s += w * (a[2 * i] * b[2 * i] + a[2 * i + 1] * b[2 * i + 1]);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int q = 128; q > 0; q >>= 1) {
        if ((int)threadIdx.x < q) sh[threadIdx.x] += sh[threadIdx.x + q];
        __syncthreads();
    }
    if (threadIdx.x == 0) red[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum_part(const double *__restrict__ red, int n, int stride, int ncomp,
                                                  double *__restrict__ out)
{
    // deterministic: per component, thread t sums the block partials t, t + 256, ... in order, then
    // a fixed tree over the threads
    __shared__ double sh[256];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0;
        for (int i = threadIdx.x; i < n; i += 256) s += red[(int64_t)i * stride + c];
        const double t = block_sum256(s, sh);
        if (threadIdx.x == 0) out[c] = t;
        __syncthreads();
    }
}

// x += alpha p, r -= alpha w on complex elements (re, im pairs), with the workgroup partials of the
// full-m <r, r> of the updated r
__global__ __launch_bounds__(256) void k_cg_xr_rr(double2 *__restrict__ x, double2 *__restrict__ r,
                                                  const double2 *__restrict__ p, const double2 *__restrict__ w,
                                                  const double *__restrict__ alpha, int64_t nc, int64_t nalm, int lmax,
                                                  double *__restrict__ rr_red)
{
    __shared__ double sh[256];
    const double a = *alpha;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 pi = p[i], wi = w[i];
        double2 xi = x[i], ri = r[i];
        xi.x = fma(a, pi.x, xi.x);
        xi.y = fma(a, pi.y, xi.y);
        ri.x = fma(-a, wi.x, ri.x);
        ri.y = fma(-a, wi.y, ri.y);
        x[i] = xi;
        r[i] = ri;
        const double wgt = ((i % nalm) <= lmax) ? 1.0 : 2.0;
        s += wgt * (ri.x * ri.x + ri.y * ri.y);
    }
    const double t = block_sum256(s, sh);
    if (threadIdx.x == 0) rr_red[blockIdx.x] = t;
}

// Fixed-order sum of n workgroup partials by one workgroup of 256 threads (thread t sums partials
// t, t + 256, ... in order, then a tree), the total in thread 0
__device__ __forceinline__ double sum_partials256(const double *__restrict__ red, int n, double *sh)
{
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) s += red[j];
    return block_sum256(s, sh);
}

// scal[1] = <p, w> from the epilogue's partials, then alpha = rz / <p, w> into scal[2]; breakdown
// (p^T H p <= 0 or non-finite) sets the flag, which is sticky: alpha = 0 until the host reads it
__global__ __launch_bounds__(256) void k_cg_alpha_sum(const double *__restrict__ red, int n, double *__restrict__ scal,
                                                      int *__restrict__ flag)
{
    __shared__ double sh[256];
    const double pw = sum_partials256(red, n, sh);
    if (threadIdx.x != 0) return;
    scal[1] = pw;
    if (flag[0] || !(pw > 0.0) || !isfinite(pw)) {
        flag[0] = 1;
        scal[2] = 0.0;
    } else {
        scal[2] = scal[0] / pw;
    }
}

// Single-right-hand-side iteration with the scalar steps inside the vector kernels: every
// workgroup sums the same partials in the same fixed order, so all hold the same alpha (beta), and
// workgroup 0 records the scalars.  The x/r update reads rz at scal[0] and keeps it at scal[7] for
// the p update, which then owns scal[0].
__global__ __launch_bounds__(256) void k_cg_xr_alpha(double2 *__restrict__ x, double2 *__restrict__ r,
                                                     const double2 *__restrict__ p, const double2 *__restrict__ w,
                                                     const double *__restrict__ red_pw, int n_pw,
                                                     double *__restrict__ scal, int *__restrict__ flag, int64_t nc,
                                                     int64_t nalm, int lmax, double *__restrict__ rr_red)
{
    __shared__ double sh[256];
    const double pw = sum_partials256(red_pw, n_pw, sh);
    __syncthreads();
    const double rz = scal[0];
    const bool bad = flag[0] != 0 || !(pw > 0.0) || !isfinite(pw);
    const double a = bad ? 0.0 : rz / pw;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 pi = p[i], wi = w[i];
        double2 xi = x[i], ri = r[i];
        xi.x = fma(a, pi.x, xi.x);
        xi.y = fma(a, pi.y, xi.y);
        ri.x = fma(-a, wi.x, ri.x);
        ri.y = fma(-a, wi.y, ri.y);
        x[i] = xi;
        r[i] = ri;
        const double wgt = ((i % nalm) <= lmax) ? 1.0 : 2.0;
        s += wgt * (ri.x * ri.x + ri.y * ri.y);
    }
    const double t = block_sum256(s, sh);
    if (threadIdx.x == 0) {
        rr_red[blockIdx.x] = t;
        if (blockIdx.x == 0) {
            scal[1] = pw;
            scal[2] = a;
            scal[7] = rz;
            if (bad) flag[0] = 1;
        }
    }
}

// p = P r + beta p with beta = P <r, r> / rz (rz from scal[7]); workgroup 0 records <r, r> at scal[3],
// beta at scal[4] and the new rz = P <r, r> at scal[0]
__global__ __launch_bounds__(256) void k_cg_p_beta(double2 *__restrict__ p, const double2 *__restrict__ r,
                                                   const double *__restrict__ red_rr, int n_rr,
                                                   double *__restrict__ scal, double pc, int64_t nc)
{
    __shared__ double sh[256];
    const double rr = sum_partials256(red_rr, n_rr, sh);
    const double rz_old = scal[7];
    const double rz = pc * rr;
    const double bt = (rz_old > 0.0) ? rz / rz_old : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 ri = r[i];
        double2 pi = p[i];
        pi.x = fma(bt, pi.x, pc * ri.x);
        pi.y = fma(bt, pi.y, pc * ri.y);
        p[i] = pi;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[3] = rr;
        scal[4] = bt;
        scal[0] = rz;
    }
}

// scal[3] = <r, r> from the update's partials, then beta = P <r, r> / rz into scal[4], rz <- P <r, r>
__global__ __launch_bounds__(256) void k_cg_beta_sum(const double *__restrict__ red, int n, double *__restrict__ scal,
                                                     double pc)
{
    __shared__ double sh[256];
    const double rr = sum_partials256(red, n, sh);
    if (threadIdx.x != 0) return;
    scal[3] = rr;
    const double rz = pc * rr;
    scal[4] = (scal[0] > 0.0) ? rz / scal[0] : 0.0;
    scal[0] = rz;
}

__global__ void k_cg_p(double *__restrict__ p, const double *__restrict__ r, const double *__restrict__ beta,
                       double precond, int64_t n2)
{
    const double bt = *beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = fma(bt, p[i], precond * r[i]);
}

__global__ void k_axpby(double *__restrict__ y, double a, const double *__restrict__ x, double b, int64_t n2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

__global__ void k_scalar_div(double *out, const double *num, const double *den) { *out = *num / *den; }

// ================================================================================================
// launchers
// ================================================================================================
bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// ================================================================================================
// Batched synthesis (FP32 plans with several right-hand sides): for one m, a group of 64 ring pairs
// (one per lane) and NBR = 8 right-hand sides, the sums over l of lambda(l, pair) a(l, rhs, c) are a
// matrix product [pairs x l] x [l x (rhs, c)] with the lambda generated on the fly, accumulated on
// the matrix cores (v_mfma_f32_32x32x2_f32: D[32 x 32] += A[32 x 2] B[2 x 32]), per half of the pairs.
//   A[i][k]  lambda of pair i (of the half) at degree l + 2k (even offsets from the step l of four) or
//            l + 1 + 2k (odd), held by lane i + 32k.  Every lane runs the recurrence of its own pair;
//            one v_permlane32_swap per pair of degrees (l, l+2) moves the values into that layout:
//            [low lanes at l | low lanes at l+2] for the first half, [high at l | high at l+2] for
//            the second.
//   B[k][j]  record value j = 4 rhs + c (c = Re/Im of aE, Re/Im of aB) at the same degree
//   D        per half four accumulators: spin +2 / -2 times even / odd offsets from the start degree
// Lane l, register r of D holds pair i = 8 (r/4) + 4 (l/32) + r%4 of the half and column j = l%32.
// ================================================================================================
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr int NBR = 8;  // right-hand sides per batched group

// per (l, m): the NBR x 4 kernel-scaled alm values of one group (Im(a_l0) zeroed), zero past nrhs
__global__ void k_prologue_b(const double *__restrict__ xE, const double *__restrict__ xB, int64_t rstride,
                             const double *__restrict__ kern, const int *__restrict__ lof, int lmax, int64_t nalm,
                             int nrhs, int q, float *__restrict__ brec)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (alm, rhs-in-group)
    if (t >= nalm * NBR) return;
    const int64_t i = t / NBR;
    const int rr = (int)(t - i * NBR), rhs = q * NBR + rr;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (rhs < nrhs) {
        const int64_t o = (int64_t)rhs * rstride + i;  // rstride: complex elements between right-hand sides
        const double K = kern ? kern[lof[i]] : 1.0;
        const bool m0 = i <= lmax;
        v.x = (float)(K * xE[2 * o]);
        v.y = m0 ? 0.f : (float)(K * xE[2 * o + 1]);
        v.z = (float)(K * xB[2 * o]);
        v.w = m0 ? 0.f : (float)(K * xB[2 * o + 1]);
    }
    reinterpret_cast<float4 *>(brec)[t] = v;
}

// quad sum over the four lanes 4 rhs + (0..3) that hold c = 0..3 of one right-hand side
__device__ __forceinline__ float quad_sum(float v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    return v;
}

// exchange the upper half of a's lanes with the lower half of b's: a = [a_lo | b_lo], b = [a_hi | b_hi]
__device__ __forceinline__ void swap_halves(float &a, float &b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(a), __float_as_int(b), false, false);
    a = __int_as_float(r[0]);
    b = __int_as_float(r[1]);
}

// SW waves (64-pair groups) per workgroup, a launch shape of the autotuner
template <int F, int SW>
__global__ __launch_bounds__(64 * SW) __attribute__((amdgpu_waves_per_eu(2))) void k_leg_synth_b(const float *__restrict__ brec,
                                                     const typename CoefB<F>::type *__restrict__ coef,
                                                     float2 *__restrict__ FG, int64_t fg_stride,
                                                     const Ent64 *__restrict__ ent, const int *__restrict__ entk,
                                                     const int *__restrict__ entl, int ng64,
                                                     const double *__restrict__ pair_z, int lmax, int npairs,
                                                     int nrings, int nrhs, int q, const int *__restrict__ glist,
                                                     int ngl, int nbm)
{
    const int lane = threadIdx.x & 63, h = lane >> 5, i = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    int m, blk;
    xcd_map((int)blockIdx.x, nbm, m, blk);
    const int wi = blk * SW + wave;  // list entry of the wave
    if (m > lmax || wi >= ngl) return;
    const int w = uniform_ptr(glist)[wi];  // 64-pair group: pairs 64 w .. 64 w + 63
    const int l0 = m > 2 ? m : 2;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const int p = 64 * w + lane;
    // a group that never enters still writes its (zero) F
    const int ls = __builtin_amdgcn_readfirstlane(uniform_ptr(entl + (int64_t)m * ng64)[w]);

    typename PosT<float, F>::type x;
    float c2 = 0.f, p2 = 0.f, cm = 0.f, pm = 0.f;
    int k = 0;
    setpos(x, 0.0);
    if (p < npairs && ls <= lmax) {
        setpos(x, pair_z[p]);
        load_entry<float, F>(ent, entk, (int64_t)m * npairs + p, c2, p2, cm, pm, k);
    }
    v16f D2e[2], D2o[2], Dme[2], Dmo[2];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int r = 0; r < 16; ++r) D2e[s2][r] = D2o[s2][r] = Dme[s2][r] = Dmo[s2][r] = 0.f;
    bool ramp = wave_any(k < 0);
    using C = typename CoefB<F>::type;
    const_as<C> *cp = uniform_ptr(coef + base);
    const float *bl = brec + base * (NBR * 4) + i;  // column i of the group's records
    // four degrees from l: records and recurrence values, then the eight products.  RAMP: some lane is
    // still in the scaled range (its values count as zero until its exponent reaches zero, and the
    // exponents are checked once per four steps); once no lane is, none returns to it, and the loop
    // without the selects and the checks takes over.
    auto four = [&](int l, auto ramp_tag) {
        constexpr bool RAMP = decltype(ramp_tag)::value;
        // B rows l + 2h (even offsets) and l + 1 + 2h (odd), zero past lmax
        const int re = l + 2 * h, ro = re + 1;
        const float be = re <= lmax ? bl[(int64_t)re * (NBR * 4)] : 0.f;
        const float bo = ro <= lmax ? bl[(int64_t)ro * (NBR * 4)] : 0.f;
        float v2[4], vm[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bool live = !RAMP || k == 0;
            v2[t] = live ? c2 : 0.f;
            vm[t] = live ? cm : 0.f;
            rstep(ld_coef(cp + l + t), x, c2, p2, cm, pm);
        }
        // degrees (l, l+2) and (l+1, l+3) of both halves of the pairs
        swap_halves(v2[0], v2[2]);
        swap_halves(v2[1], v2[3]);
        swap_halves(vm[0], vm[2]);
        swap_halves(vm[1], vm[3]);
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
            D2e[s2] = __builtin_amdgcn_mfma_f32_32x32x2f32(v2[2 * s2], be, D2e[s2], 0, 0, 0);
            D2o[s2] = __builtin_amdgcn_mfma_f32_32x32x2f32(v2[2 * s2 + 1], bo, D2o[s2], 0, 0, 0);
            Dme[s2] = __builtin_amdgcn_mfma_f32_32x32x2f32(vm[2 * s2], be, Dme[s2], 0, 0, 0);
            Dmo[s2] = __builtin_amdgcn_mfma_f32_32x32x2f32(vm[2 * s2 + 1], bo, Dmo[s2], 0, 0, 0);
        }
        if constexpr (RAMP) {
            // once per four steps (the growth over four steps stays far from overflow)
            if (k < 0 && fmaxf(fabsf(c2), fabsf(cm)) > scale_hi<float>()) {
                const float d = scale_down<float>();
                c2 *= d;
                p2 *= d;
                cm *= d;
                pm *= d;
                k += 1;
            }
            ramp = wave_any(k < 0);
        }
    };
    int l = ls;
    for (; l <= lmax && ramp; l += 4) four(l, std::true_type{});
    for (; l <= lmax; l += 4) four(l, std::false_type{});
    // F of the north and south ring of every (pair, rhs): quad sums over c, written by lane c = 0
    const bool odd0 = ((l0 + m) & 1) != 0;  // entries are l0 + 8 q: D2e holds degrees of parity l0 + m
    const int c = i & 3, rl = i >> 2, rhs = q * NBR + rl;
    const float s0r = c == 0 ? -1.f : (c == 3 ? 1.f : 0.f), s0i = (c == 1 || c == 2) ? -1.f : 0.f;
    const float s1r = (c == 0 || c == 3) ? -1.f : 0.f, s1i = c == 2 ? -1.f : (c == 1 ? 1.f : 0.f);
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int pi = 64 * w + 32 * s2 + 8 * (r >> 2) + 4 * h + (r & 3);
            const float E2 = odd0 ? D2o[s2][r] : D2e[s2][r], O2 = odd0 ? D2e[s2][r] : D2o[s2][r];
            const float Em = odd0 ? Dmo[s2][r] : Dme[s2][r], Om = odd0 ? Dme[s2][r] : Dmo[s2][r];
            // north: S2 = E2 + O2, Sm = Em + Om;  south: S2 = Em - Om, Sm = E2 - O2
            const float S2n = E2 + O2, Smn = Em + Om, S2s = Em - Om, Sms = E2 - O2;
            // f0 = -(S2[0] - S2[3], S2[1] + S2[2]),  f1 = -(Sm[0] + Sm[3], Sm[2] - Sm[1])
            const float fn0r = quad_sum(s0r * S2n), fn0i = quad_sum(s0i * S2n);
            const float fn1r = quad_sum(s1r * Smn), fn1i = quad_sum(s1i * Smn);
            const float fs0r = quad_sum(s0r * S2s), fs0i = quad_sum(s0i * S2s);
            const float fs1r = quad_sum(s1r * Sms), fs1i = quad_sum(s1i * Sms);
            if (c == 0 && rhs < nrhs && pi < npairs) {
                float2 *Fb = FG + (int64_t)rhs * fg_stride;
                const int rn = pi, rs = nrings - 1 - pi;
                float2 *f = Fb + ((int64_t)rn * (lmax + 1) + m) * 2;
                f[0] = make_float2(fn0r, fn0i);
                f[1] = make_float2(fn1r, fn1i);
                if (rs != rn) {
                    float2 *g = Fb + ((int64_t)rs * (lmax + 1) + m) * 2;
                    g[0] = make_float2(fs0r, fs0i);
                    g[1] = make_float2(fs1r, fs1i);
                }
            }
        }
    }
}

// ================================================================================================
// Batched FP32 Legendre adjoint on the matrix cores.  For one m, a block of AW 64-pair groups (one per
// wave) and the NBR right-hand sides of group q, the partial sums over the block's ring pairs
//   out_rhs[l][c],  c = 0..3 as in k_leg_adj (2h_lm and -2h_lm, Re and Im).
// Per chunk of ABL = 32 degrees each wave writes the recurrence values of its pairs to LDS (one row
// per degree), then v_mfma_f32_32x32x2_f32 contracts over the pairs, two per instruction:
//   D+ = Lambda+ [GN.x, GN.y, HS.x, HS.y],   D- = Lambda- [HN.x, HN.y, GS.x, GS.y]
// (columns 4 rhs + c, G of the north ring GN, HN = conj of its second component, S the south ring),
// and the south terms take the sign s = (-1)^(l+m) of their row:
//   out_0,1 = D+[c] + s D-[c+2],   out_2,3 = D-[c-2] + s D+[c].
// G is loaded once per wave into registers (it does not depend on l).  The waves of the block are
// summed in LDS and one slab per (right-hand side of the group, block) is written,
// [rhs - NBR q][nrb][nalm][4], rows from the chunk holding the block's first entry degree (recorded in
// wgstart) to lmax.
// ================================================================================================
// AW waves (64-pair groups) per workgroup is a launch shape of the autotuner (2, 4 or 8)
constexpr int ABL = 32;  // degrees per chunk: the rows of the MFMA
constexpr int ABS = 33;  // LDS stride of one pair's 32 rows (bank-conflict-free writes)

template <int F, int AW>
__global__ __launch_bounds__(64 * AW) __attribute__((amdgpu_waves_per_eu(2))) void k_leg_adj_b(const float2 *__restrict__ FG, int64_t fg_stride,
                                                        const typename CoefB<F>::type *__restrict__ coef,
                                                        const Ent64 *__restrict__ ent, const int *__restrict__ entk,
                                                        const int *__restrict__ entl, int ng64,
                                                        const double *__restrict__ pair_z, float *__restrict__ part,
                                                        int *__restrict__ wgstart, int64_t nalm, int lmax, int npairs,
                                                        int nrings, int nrhs, int q, const int *__restrict__ glist,
                                                        int ngl, const uint8_t *__restrict__ live, int rb0,
                                                        int nrbl, int nrb)
{
    __shared__ float lam[AW][2][64 * ABS];  // per wave: lambda+ and lambda- of its 64 pairs x 32 rows
    __shared__ float red[8 * AW * 64];      // the cross-wave sum, eight output registers at a time
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    int m, rbl;
    xcd_map((int)blockIdx.x, nrbl, m, rbl);
    if (m > lmax) return;
    const int rb = rb0 + rbl;
    const int lb = rbl * AW;  // first list entry of the block
    const int l0 = m > 2 ? m : 2;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const_as<int> *el = uniform_ptr(entl + (int64_t)m * ng64);
    const_as<int> *gl = uniform_ptr(glist);
    int ls = ENT_SKIP;
    for (int li = lb; li < lb + AW && li < ngl; ++li) ls = el[gl[li]] < ls ? el[gl[li]] : ls;
    if (threadIdx.x == 0) wgstart[(int64_t)m * nrb + rb] = ls;
    if (ls > lmax) return;
    const int g = lb + wave < ngl ? gl[lb + wave] : -1;  // this wave's group
    const int e = g >= 0 ? el[g] : ENT_SKIP;             // and its entry degree
    const int p = g * 64 + lane;
    const bool valid = g >= 0 && p < npairs;

    // B operands: lane l holds, for pair-pair kk, pair 64 g + 2 kk + l / 32 and column j = l % 32
    const int j = lane & 31, c = j & 3, rhs = q * NBR + (j >> 2);
    float Bp[32], Bm[32];
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) {
        Bp[kk] = Bm[kk] = 0.f;
        const int pk = g * 64 + 2 * kk + (lane >> 5);
        if (e > lmax || g < 0 || pk >= npairs || rhs >= nrhs) continue;
        const float2 *Fb = FG + rhs * fg_stride;
        if (c < 2) {
            if (live && !live[pk]) continue;  // a ring without weight has G = 0
            const float2 *fn = Fb + ((int64_t)pk * (lmax + 1) + m) * 2;
            const float2 gn = fn[0], hn = fn[1];  // HN = conj(hn)
            Bp[kk] = c ? gn.y : gn.x;
            Bm[kk] = c ? -hn.y : hn.x;
        } else {
            const int rs = nrings - 1 - pk;
            if (rs != pk && (!live || live[rs])) {
                const float2 *fs = Fb + ((int64_t)rs * (lmax + 1) + m) * 2;
                const float2 gs = fs[0], hs = fs[1];  // HS = conj(hs)
                Bp[kk] = (c & 1) ? -hs.y : hs.x;
                Bm[kk] = (c & 1) ? gs.y : gs.x;
            }
        }
    }

    typename PosT<float, F>::type x;
    setpos(x, valid ? pair_z[p] : 0.0);
    float c2 = 0.f, p2 = 0.f, cm = 0.f, pm = 0.f;
    int k = 0;
    bool ramp = false;
    using C = typename CoefB<F>::type;
    const_as<C> *cp = uniform_ptr(coef + base);
    float *lp = &lam[wave][0][lane * ABS], *lmn = &lam[wave][1][lane * ABS];
    const float *ap = &lam[wave][0][(lane >> 5) * ABS + (lane & 31)], *am = &lam[wave][1][(lane >> 5) * ABS + (lane & 31)];
    // the wave's recurrence covers the chunk starting at lx (zero before the wave's entry, for lanes
    // still in the scaled range and past lmax)
    auto is_active = [&](int lx) { return lx <= lmax && e <= lx + ABL - 1 && e <= lmax; };
    // rows t8 .. t8 + 7 of the chunk at lx into the wave's LDS rows (entry degrees are l0 + 8 q and
    // chunks start at l0 + 32 j, so an entry falls on a block of 8)
    auto rows8 = [&](int lx, int t8, auto &&after) {
        const int lb = lx + t8;
        if (lb == e) {
            if (valid) load_entry<float, F>(ent, entk, (int64_t)m * npairs + p, c2, p2, cm, pm, k);
            ramp = wave_any(k < 0);
        }
        if (lb < e || lb > lmax) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                lp[t8 + t] = lmn[t8 + t] = 0.f;
                after(t);
            }
            return;
        }
        C cc[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) cc[t] = ld_coef(cp + lb + t);  // padded past lmax
        if (!ramp && lb + 7 <= lmax) {
            // every lane out of the scaled range and every row in range: no selects, no checks
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                lp[t8 + t] = c2;
                lmn[t8 + t] = cm;
                rstep(cc[t], x, c2, p2, cm, pm);
                after(t);
            }
            return;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bool live = k == 0 && lb + t <= lmax;
            lp[t8 + t] = live ? c2 : 0.f;
            lmn[t8 + t] = live ? cm : 0.f;
            rstep(cc[t], x, c2, p2, cm, pm);
            after(t);
            if (ramp && (t & 3) == 3) {
                // every four steps (the growth over four steps stays far from overflow)
                if (k < 0 && fmaxf(fabsf(c2), fabsf(cm)) > scale_hi<float>()) {
                    const float d = scale_down<float>();
                    c2 *= d;
                    p2 *= d;
                    cm *= d;
                    pm *= d;
                    k += 1;
                }
                ramp = wave_any(k < 0);
            }
        }
    };
    // Software pipeline over chunks: the A operands of chunk lc are read from LDS into registers, then
    // the recurrence writes the rows of the next chunk into the same LDS rows while the matrix cores
    // contract chunk lc (eight rows, then the sixteen products of eight pair-pairs).  A wave reads and
    // writes only its own rows, and its LDS accesses run in program order, so the reads return the
    // rows of chunk lc.
    const int lstart = l0 + ((ls - l0) / ABL) * ABL;
    if (is_active(lstart)) {
#pragma unroll
        for (int t8 = 0; t8 < ABL; t8 += 8) rows8(lstart, t8, [](int) {});
    }
    for (int lc = lstart; lc <= lmax; lc += ABL) {
        const bool act = is_active(lc), actn = is_active(lc + ABL);
        wg_lds_sync<1>();
        float a[32], b[32];
        if (act) {
#pragma unroll
            for (int kk = 0; kk < 32; ++kk) {
                a[kk] = ap[2 * kk * ABS];
                b[kk] = am[2 * kk * ABS];
            }
        }
        wg_lds_sync<1>();
        v16f Dp, Dm;
#pragma unroll
        for (int r = 0; r < 16; ++r) Dp[r] = Dm[r] = 0.f;
        // the products of pair-pair kk follow row kk % 8 of block kk / 8 of the next chunk
        auto mm = [&](int kk) {
            Dp = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kk], Bp[kk], Dp, 0, 0, 0);
            Dm = __builtin_amdgcn_mfma_f32_32x32x2f32(b[kk], Bm[kk], Dm, 0, 0, 0);
        };
        if (act && actn) {
#pragma unroll
            for (int t8 = 0; t8 < ABL; t8 += 8) rows8(lc + ABL, t8, [&](int t) { mm(t8 + t); });
        } else if (act) {
#pragma unroll
            for (int kk = 0; kk < 32; ++kk) mm(kk);
        } else if (actn) {
#pragma unroll
            for (int t8 = 0; t8 < ABL; t8 += 8) rows8(lc + ABL, t8, [](int) {});
        }
        // D row of register r in lane l: 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
        float o[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const float s = ((lc + i + m) & 1) ? -1.f : 1.f;
            const float t2 = dpp_mov<0x4E>(Dm[r]);  // D- of column j ^ 2
            o[r] = c < 2 ? fmaf(s, t2, Dp[r]) : fmaf(s, Dp[r], t2);
        }
        // sum over the block's waves in LDS, eight registers at a time
#pragma unroll
        for (int h = 0; h < 16; h += 8) {
            __syncthreads();
#pragma unroll
            for (int r8 = 0; r8 < 8; ++r8) red[(wave * 8 + r8) * 64 + lane] = o[h + r8];
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 8 / AW; ++u) {
                const int r = h + wave * (8 / AW) + u;  // this thread's register index, lane as it was
                float sum = 0.f;
#pragma unroll
                for (int w = 0; w < AW; ++w) sum += red[(w * 8 + r - h) * 64 + lane];
                const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), l = lc + i;
                if (l <= lmax && rhs < nrhs)
                    part[(((int64_t)(j >> 2) * nrb + rb) * nalm + base + l) * 4 + c] = sum;
            }
        }
    }
}


void launch_prologue(Plan &P, bool fp32, const double *xE, const double *xB, const double *kern, int nrhs)
{
    dim3 g((unsigned)cdiv(P.nalm, 256), nrhs);
    if (fp32)
        k_prologue<float><<<g, 256, 0, P.stream>>>(xE, xB, kern, P.d_lof, P.d_coef32s, P.d_coef64s, P.lmax, P.nalm,
                                                   P.rec_stride, (SynRec<float> *)P.d_rec, P.d_recu);
    else
        k_prologue<double><<<g, 256, 0, P.stream>>>(xE, xB, kern, P.d_lof, P.d_coef64s, P.d_coef64s, P.lmax, P.nalm,
                                                    P.rec_stride, (SynRec<double> *)P.d_rec, nullptr);
}

// the near-polar groups list[0 .. npol) in the difference form and list[npol .. npol + nmain) in the
// plain form, SW groups per workgroup
template <int SW>
static void synth_b_launch(Plan &P, int q, int64_t fg_stride, int64_t lblocks, const int *list, int npol, int nmain)
{
    if (npol > 0) {
        const int nbm = (int)cdiv(npol, SW);
        k_leg_synth_b<1, SW><<<(unsigned)(8 * nbm * lblocks), 64 * SW, 0, P.stream>>>(
            P.d_brec, P.d_coef32d, (float2 *)P.d_FG, fg_stride, P.d_ent, P.d_entk, P.d_entl, P.ng64, P.d_pair_z,
            P.lmax, P.npairs, P.nrings, P.nrhs, q, list, npol, nbm);
    }
    if (nmain > 0) {
        const int nbm = (int)cdiv(nmain, SW);
        k_leg_synth_b<0, SW><<<(unsigned)(8 * nbm * lblocks), 64 * SW, 0, P.stream>>>(
            P.d_brec, P.d_coef32, (float2 *)P.d_FG, fg_stride, P.d_ent, P.d_entk, P.d_entl, P.ng64, P.d_pair_z,
            P.lmax, P.npairs, P.nrings, P.nrhs, q, list + npol, nmain, nbm);
    }
}

// ring blocks of AW groups: the near-polar groups first (difference form), then the others
template <int AW>
static void adj_b_launch(Plan &P, int q, int64_t fg_stride, int64_t lblocks, const int *list, int npol, int nmain,
                         const uint8_t *live, int nrb)
{
    const int nbp = (int)cdiv(npol, AW), nbn = (int)cdiv(nmain, AW);
    if (nbp > 0)
        k_leg_adj_b<1, AW><<<(unsigned)(8 * nbp * lblocks), 64 * AW, 0, P.stream>>>(
            (const float2 *)P.d_FG, fg_stride, P.d_coef32d, P.d_ent, P.d_entk, P.d_entl, P.ng64, P.d_pair_z,
            (float *)P.d_part, P.d_wgstart_b, P.nalm, P.lmax, P.npairs, P.nrings, P.nrhs, q, list, npol, live, 0, nbp,
            nrb);
    if (nbn > 0)
        k_leg_adj_b<0, AW><<<(unsigned)(8 * nbn * lblocks), 64 * AW, 0, P.stream>>>(
            (const float2 *)P.d_FG, fg_stride, P.d_coef32, P.d_ent, P.d_entk, P.d_entl, P.ng64, P.d_pair_z,
            (float *)P.d_part, P.d_wgstart_b, P.nalm, P.lmax, P.npairs, P.nrings, P.nrhs, q, list + npol, nmain, live,
            nbp, nbn, nrb);
}

// batched synthesis of FP32 plans: records and matrix-core sums per group of NBR right-hand sides, over
// every 64-pair group (live false) or those with a ring that carries weight (live true)
void launch_synth_batched(Plan &P, const double *xE, const double *xB, int64_t rstride, const double *kern, bool live)
{
    const int64_t fg_stride = (int64_t)P.nrings * (P.lmax + 1) * 2;
    const GroupSet &G = live && P.skip_rings ? P.gs_live : P.gs_all;
    const int64_t lblocks = xcd_slots(P.lmax);
    for (int q = 0; q * NBR < P.nrhs; ++q) {
        k_prologue_b<<<(unsigned)cdiv(P.nalm * NBR, 256), 256, 0, P.stream>>>(xE, xB, rstride, kern, P.d_lof, P.lmax,
                                                                             P.nalm, P.nrhs, q, P.d_brec);
        switch (P.bat_SW) {
        case 1: synth_b_launch<1>(P, q, fg_stride, lblocks, G.list_any, G.npol_any, G.nmain_any); break;
        case 2: synth_b_launch<2>(P, q, fg_stride, lblocks, G.list_any, G.npol_any, G.nmain_any); break;
        case 8: synth_b_launch<8>(P, q, fg_stride, lblocks, G.list_any, G.npol_any, G.nmain_any); break;
        default: synth_b_launch<4>(P, q, fg_stride, lblocks, G.list_any, G.npol_any, G.nmain_any);
        }
    }
}

// batched adjoint of the right-hand-side group q into the [rhs - NBR q][nrb_cur_b][nalm][4] slabs of
// d_part, over every 64-pair group (live false) or those with a ring that carries weight, reading
// only such rings (live true)
void launch_adj_batched(Plan &P, int q, bool live)
{
    live = live && P.skip_rings;
    const int64_t fg_stride = (int64_t)P.nrings * (P.lmax + 1) * 2;
    const GroupSet &G = live ? P.gs_live : P.gs_all;
    const uint8_t *lv = live ? P.d_ring_live : nullptr;
    const int64_t lblocks = xcd_slots(P.lmax);
    const int nrb = (int)(cdiv(G.npol_any, P.bat_AW) + cdiv(G.nmain_any, P.bat_AW));
    switch (P.bat_AW) {
    case 2: adj_b_launch<2>(P, q, fg_stride, lblocks, G.list_any, G.npol_any, G.nmain_any, lv, nrb); break;
    case 8: adj_b_launch<8>(P, q, fg_stride, lblocks, G.list_any, G.npol_any, G.nmain_any, lv, nrb); break;
    default: adj_b_launch<4>(P, q, fg_stride, lblocks, G.list_any, G.npol_any, G.nmain_any, lv, nrb);
    }
    P.nrb_b_cur = nrb;
}

void launch_epilogue_batched(Plan &P, int rhs, const double *kern, double lam, const double *xE, const double *xB,
                             double *outE, double *outB, double *dot_red)
{
    const float *part = (const float *)P.d_part + (int64_t)(rhs % NBR) * P.nrb_b_cur * P.nalm * 4;
    const unsigned g = dot_red ? (unsigned)cg_red_blocks(P) : (unsigned)cdiv(P.nalm, 256);
    k_epilogue<float><<<g, 256, 0, P.stream>>>(part, P.d_wgstart_b, P.nrb_b_cur, P.nalm, P.d_lof, P.lmax, kern, lam, xE,
                                              xB, outE, outB, P.proj, dot_red);
}

void launch_entry(Plan &P)
{
    const int gpb = (int)cdiv(P.ng64, 4);
    k_entry<<<(unsigned)((int64_t)gpb * (P.lmax + 1)), 256, 0, P.stream>>>(
        P.d_seed2, P.d_seedm2, P.d_seedk, P.d_pair_z, P.d_coef64, P.d_ent, P.d_entk, P.d_entl, P.lmax, P.npairs, P.ng64,
        gpb, P.prec == AKRA_FP32 ? 0x1p-44 : 0x1p-100);
}

// Legendre synthesis of the prologue's records: every 64-pair group (live false), or the groups of
// the current weights by class (live true)
void launch_leg_synth(Plan &P, bool fp32, int nrhs, bool live)
{
    const GroupSet &G = live && P.skip_rings ? P.gs_live : P.gs_all;
    auto n = [&](int c) { return G.npol[c] + G.nmain[c]; };
    auto two = [&]() {
        if (n(GCLS_BOTH)) leg_synth_cls<GCLS_BOTH>(P, fp32, nrhs, G.list[GCLS_BOTH], G.npol[GCLS_BOTH], G.nmain[GCLS_BOTH]);
    };
    auto one = [&]() {
        if (n(GCLS_NORTH))
            leg_synth_cls<GCLS_NORTH>(P, fp32, nrhs, G.list[GCLS_NORTH], G.npol[GCLS_NORTH], G.nmain[GCLS_NORTH]);
        if (n(GCLS_SOUTH))
            leg_synth_cls<GCLS_SOUTH>(P, fp32, nrhs, G.list[GCLS_SOUTH], G.npol[GCLS_SOUTH], G.nmain[GCLS_SOUTH]);
    };
    // the classes write F of disjoint rings: the two-sided groups on the side stream
    if (n(GCLS_BOTH) && n(GCLS_NORTH) + n(GCLS_SOUTH)) fork_join(P, two, one);
    else {
        two();
        one();
    }
}

bool adj_shape_supported(int r, int w, int l)
{
#define AKRA_ADJ_SUP(a, b, c) \
    if (r == a && w == b && l == c) return true;
    AKRA_ADJ_SHAPES(AKRA_ADJ_SUP)
#undef AKRA_ADJ_SUP
    return false;
}

int adj_blocks_total(const Plan &P, bool live)
{
    const GroupSet &G = live && P.skip_rings ? P.gs_live : P.gs_all;
    int n = 0;
    for (int c = 0; c < GCLS_N; ++c) n += adj_blocks(P, c, G.npol[c], G.nmain[c]);
    return n;
}

// Legendre adjoint of d_FG (right-hand side rhs) into the partial sums, over every 64-pair group
// (live false) or the groups of the current weights by class, reading only rings that carry weight
// (live true).  The near-polar groups of FP32 plans form their own blocks of at most adj_Rpol in
// FP32 and in FP64 applies alike; the epilogue sums the nrb_cur blocks written.
void launch_leg_adj(Plan &P, bool fp32, int rhs, bool live)
{
    live = live && P.skip_rings;
    const GroupSet &G = live ? P.gs_live : P.gs_all;
    const uint8_t *lv = live ? P.d_ring_live : nullptr;
    const int nrb = adj_blocks_total(P, live);
    auto n = [&](int c) { return G.npol[c] + G.nmain[c]; };
    // ring blocks: the two-sided class first, then north, then south (the slabs are disjoint)
    const int rb1 = adj_blocks(P, GCLS_BOTH, G.npol[GCLS_BOTH], G.nmain[GCLS_BOTH]);
    const int rb2 = rb1 + adj_blocks(P, GCLS_NORTH, G.npol[GCLS_NORTH], G.nmain[GCLS_NORTH]);
    auto two = [&]() {
        if (n(GCLS_BOTH))
            leg_adj_cls<GCLS_BOTH>(P, fp32, rhs, G.list[GCLS_BOTH], G.npol[GCLS_BOTH], G.nmain[GCLS_BOTH], lv, 0, nrb);
    };
    auto one = [&]() {
        if (n(GCLS_NORTH))
            leg_adj_cls<GCLS_NORTH>(P, fp32, rhs, G.list[GCLS_NORTH], G.npol[GCLS_NORTH], G.nmain[GCLS_NORTH], lv,
                                    rb1, nrb);
        if (n(GCLS_SOUTH))
            leg_adj_cls<GCLS_SOUTH>(P, fp32, rhs, G.list[GCLS_SOUTH], G.npol[GCLS_SOUTH], G.nmain[GCLS_SOUTH], lv,
                                    rb2, nrb);
    };
    if (n(GCLS_BOTH) && n(GCLS_NORTH) + n(GCLS_SOUTH)) fork_join(P, two, one);
    else {
        two();
        one();
    }
    P.nrb_cur = nrb;
}

int cg_red_blocks(const Plan &P) { return (int)std::min<int64_t>(CG_RED_BLOCKS, cdiv(P.nalm, 256)); }

void launch_epilogue(Plan &P, bool fp32, const double *kern, double lam, const double *xE, const double *xB,
                     double *outE, double *outB, double *dot_red)
{
    const dim3 g(dot_red ? (unsigned)cg_red_blocks(P) : (unsigned)cdiv(P.nalm, 256));
    if (fp32)
        k_epilogue<float><<<g, 256, 0, P.stream>>>((const float *)P.d_part, P.d_wgstart, P.nrb_cur, P.nalm, P.d_lof,
                                                   P.lmax, kern, lam, xE, xB, outE, outB, P.proj, dot_red);
    else
        k_epilogue<double><<<g, 256, 0, P.stream>>>((const double *)P.d_part, P.d_wgstart, P.nrb_cur, P.nalm,
                                                    P.d_lof, P.lmax, kern, lam, xE, xB, outE, outB, P.proj, dot_red);
}

void launch_cg_alpha_sum(Plan &P, const double *red, double *scal, int *flag)
{
    k_cg_alpha_sum<<<1, 256, 0, P.stream>>>(red, cg_red_blocks(P), scal, flag);
}

void launch_cg_xr_rr(Plan &P, double *x, double *r, const double *p, const double *w, const double *alpha_dev,
                     int64_t n_complex, double *rr_red)
{
    k_cg_xr_rr<<<cg_red_blocks(P), 256, 0, P.stream>>>((double2 *)x, (double2 *)r, (const double2 *)p,
                                                       (const double2 *)w, alpha_dev, n_complex, P.nalm, P.lmax,
                                                       rr_red);
}

void launch_cg_xr_alpha(Plan &P, double *x, double *r, const double *p, const double *w, const double *red_pw,
                        double *scal, int *flag, int64_t n_complex, double *rr_red)
{
    const int nb = cg_red_blocks(P);
    k_cg_xr_alpha<<<nb, 256, 0, P.stream>>>((double2 *)x, (double2 *)r, (const double2 *)p, (const double2 *)w, red_pw,
                                            nb, scal, flag, n_complex, P.nalm, P.lmax, rr_red);
}

void launch_cg_p_beta(Plan &P, double *p, const double *r, const double *red_rr, double *scal, double precond,
                      int64_t n_complex)
{
    const int nb = cg_red_blocks(P);
    k_cg_p_beta<<<nb, 256, 0, P.stream>>>((double2 *)p, (const double2 *)r, red_rr, nb, scal, precond, n_complex);
}

void launch_cg_beta_sum(Plan &P, const double *red, double *scal, double precond)
{
    k_cg_beta_sum<<<1, 256, 0, P.stream>>>(red, cg_red_blocks(P), scal, precond);
}

// The ring kinds of a RingSet: RK_P2 whole power-of-two rings (LDS FFT), RK_BF whole-ring Bluestein,
// RK_BL rings split into two half-length Bluestein transforms, RK_REG + q the register engine's
// lists (see Plan::d_order_r)
template <typename T, int MODE>
static void ring_launch_t(Plan &P, const RingSet &RS, const double *g1, const double *g2, double *o1, double *o2,
                          const double *W, double *o3, const uint8_t *mask, const double *cdev, int nrhs,
                          bool split = true)
{
    const int64_t fg_stride = (int64_t)P.nrings * (P.lmax + 1) * 2;
    const void *tw = std::is_same<T, double>::value ? P.d_tw64 : P.d_tw32;
    const cplx<T> *bh = (const cplx<T> *)(std::is_same<T, double>::value ? P.d_bhat64 : P.d_bhat32);
    if (RS.n[RK_P2]) {
        // whole rings: N = 4 sub <= 4 nside <= 8192 = RF RFU (nside <= 2048 is enforced at plan creation)
        const size_t nmax = std::max((size_t)RF, 4 * (size_t)P.maxM_p2);  // RF: the short-ring fold
        size_t sm = sizeof(cplx<T>) * (nmax + nmax / 32);
        k_ring_full<T, MODE><<<dim3(RS.n[RK_P2], nrhs), RF, sm, P.stream>>>(
            (cplx<T> *)P.d_FG, fg_stride, g1, g2, o1, o2, P.npix, W, P.d_rings, RS.order[RK_P2], (const cplx<T> *)tw,
            P.twn, P.lmax, P.omega, o3, mask, cdev);
    }
    if (RS.n[RK_BF]) {
        const size_t nmax = std::max((size_t)RF, (size_t)P.maxM_bf);  // RF: the short-ring fold
        size_t sm = sizeof(cplx<T>) * (nmax + nmax / 32);
        k_ring_bfull<T, MODE><<<dim3(RS.n[RK_BF], nrhs), RF, sm, P.stream>>>(
            (cplx<T> *)P.d_FG, fg_stride, g1, g2, o1, o2, P.npix, W, P.d_rings, RS.order[RK_BF], (const cplx<T> *)tw,
            P.twn, P.lmax, P.omega, o3, mask, cdev, bh);
    }
    if (RS.n[RK_BL]) {
        size_t sm = sizeof(cplx<T>) * (size_t)(P.maxM_bl + P.maxM_bl / 32);
        k_ring_b2<T, MODE><<<dim3(RS.n[RK_BL], nrhs), RF, sm, P.stream>>>(
            (cplx<T> *)P.d_FG, fg_stride, g1, g2, o1, o2, P.npix, W, P.d_rings, RS.order[RK_BL], (const cplx<T> *)tw,
            P.twn, P.lmax, P.omega, o3, mask, cdev, bh);
    }
    // register engine: LDS of M + M / 32 components (FP64, one component at a time) or complex values (FP32)
    const cplx<T> *bhr = (const cplx<T> *)(std::is_same<T, double>::value ? P.d_bhatr64 : P.d_bhatr32);
    auto reg = [&](auto kern, int q, int M) {
        if (!RS.n[RK_REG + q]) return;
        const bool split_ring = q >= 4;  // KIND 2: one-component exchanges and a half-ring stash
        const size_t sm = ((std::is_same<T, double>::value || split_ring) ? sizeof(T) : sizeof(cplx<T>)) *
                              (size_t)(M + M / 32) +
                          (split_ring ? sizeof(cplx<T>) * (size_t)(M / 2) : 0);
        kern<<<dim3(RS.n[RK_REG + q], nrhs), M / 16, sm, P.stream>>>(
            (cplx<T> *)P.d_FG, fg_stride, g1, g2, o1, o2, P.npix, W, P.d_rings, RS.order[RK_REG + q],
            (const cplx<T> *)tw, P.twn, P.lmax, P.omega, o3, mask, cdev, bhr);
    };
    // the kinds touch disjoint rings: the largest direct kind on the plan stream, the others beside it
    // (split false: all on the plan stream)
    auto side = [&]() {
        reg(k_ring16<T, MODE, 13, 2>, 5, 8192);
        reg(k_ring16<T, MODE, 13, 1>, 3, 8192);
        reg(k_ring16<T, MODE, 12, 0>, 0, 4096);
    };
    auto main = [&]() {
        reg(k_ring16<T, MODE, 13, 0>, 1, 8192);
        reg(k_ring16<T, MODE, 12, 2>, 4, 4096);
        reg(k_ring16<T, MODE, 12, 1>, 2, 4096);
    };
    if (split) {
        fork_join(P, side, main);
    } else {
        side();
        main();
    }
}

// Spectra of the Bluestein chirps, one per distinct sub-transform length L (plan creation):
//   bhat = FFT_M(b) / M,  b_n = e^{+i pi n^2 / L} for n in (-L, L) (wrapped mod M), in FP64 and FP32.
__global__ __launch_bounds__(RT) void k_bhat(const int *__restrict__ Ls, const int *__restrict__ Ms,
                                             const int64_t *__restrict__ ofs, const double2 *__restrict__ tw,
                                             int twn, double2 *__restrict__ b64, float2 *__restrict__ b32)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double2 *buf = reinterpret_cast<double2 *>(smem_raw);
    const int L = Ls[blockIdx.x], M = Ms[blockIdx.x];
    const int64_t o = ofs[blockIdx.x];
    const int logM = 31 - __builtin_clz(M);
    for (int n = threadIdx.x; n < M; n += RT) {
        double2 v = make_double2(0.0, 0.0);
        if (n < L) v = cconj<double>(chirp<double>(n, L));
        else if (n > M - L) v = cconj<double>(chirp<double>(M - n, L));
        buf[pd(brev(n, logM))] = v;
    }
    __syncthreads();
    fft_dit<double>(buf, M, tw, twn, -1);
    const double inv = 1.0 / (double)M;
    for (int n = threadIdx.x; n < M; n += RT) {
        const double2 v = cscale<double>(buf[pd(n)], inv);
        b64[o + n] = v;
        b32[o + n] = make_float2((float)v.x, (float)v.y);
    }
}

void launch_bhat_reorder(Plan &P, int logm, const int64_t *src_ofs, const int64_t *dst_ofs, int n)
{
    if (logm == 13) {
        k_bhat_reorder<double, 13><<<n, 256, 0, P.stream>>>((const double2 *)P.d_bhat64, src_ofs, dst_ofs,
                                                            (double2 *)P.d_bhatr64);
        k_bhat_reorder<float, 13><<<n, 256, 0, P.stream>>>((const float2 *)P.d_bhat32, src_ofs, dst_ofs,
                                                           (float2 *)P.d_bhatr32);
    } else {
        k_bhat_reorder<double, 12><<<n, 256, 0, P.stream>>>((const double2 *)P.d_bhat64, src_ofs, dst_ofs,
                                                            (double2 *)P.d_bhatr64);
        k_bhat_reorder<float, 12><<<n, 256, 0, P.stream>>>((const float2 *)P.d_bhat32, src_ofs, dst_ofs,
                                                           (float2 *)P.d_bhatr32);
    }
}

void launch_bhat(Plan &P, const int *Ls, const int *Ms, const int64_t *ofs, int n, int maxM)
{
    k_bhat<<<n, RT, sizeof(double2) * (size_t)(maxM + maxM / 32), P.stream>>>(Ls, Ms, ofs, (const double2 *)P.d_tw64,
                                                                              P.twn, (double2 *)P.d_bhat64,
                                                                              (float2 *)P.d_bhat32);
}

// every ring (live false), or the rings that carry weight in the current weights (live true)
void launch_ring(Plan &P, bool fp32, int mode, const double *g1, const double *g2, double *o1, double *o2,
                 const double *W, int nrhs, bool live)
{
    const RingSet &RS = live && P.skip_rings ? P.rs_live : P.rs_all;
    if (fp32) {
        if (mode == 0) ring_launch_t<float, 0>(P, RS, g1, g2, o1, o2, W, nullptr, nullptr, nullptr, nrhs);
        else if (mode == 1) ring_launch_t<float, 1>(P, RS, g1, g2, o1, o2, W, nullptr, nullptr, nullptr, nrhs);
        else ring_launch_t<float, 2>(P, RS, g1, g2, o1, o2, W, nullptr, nullptr, nullptr, nrhs);
    } else {
        if (mode == 0) ring_launch_t<double, 0>(P, RS, g1, g2, o1, o2, W, nullptr, nullptr, nullptr, nrhs);
        else if (mode == 1) ring_launch_t<double, 1>(P, RS, g1, g2, o1, o2, W, nullptr, nullptr, nullptr, nrhs);
        else ring_launch_t<double, 2>(P, RS, g1, g2, o1, o2, W, nullptr, nullptr, nullptr, nrhs);
    }
}

// Two chains, one per class of ring groups, each running synthesis, ring stage and adjoint of its
// class: the groups weighted on both sides on the side stream, those weighted on one side on the
// plan stream.  A chain's rings are those of its groups, so the chains write F and G of disjoint
// rings and partial sums of disjoint ring blocks; a chain's ring stage needs only its own
// synthesis, and its adjoint only its own rings, so no stage waits for the other class.
void launch_weighted_chains(Plan &P, bool fp32, const double *W)
{
    const GroupSet &G = P.gs_live;
    const uint8_t *lv = P.d_ring_live;
    const int nrb = adj_blocks_total(P, true);
    const int rb1 = adj_blocks(P, GCLS_BOTH, G.npol[GCLS_BOTH], G.nmain[GCLS_BOTH]);
    const int rb2 = rb1 + adj_blocks(P, GCLS_NORTH, G.npol[GCLS_NORTH], G.nmain[GCLS_NORTH]);
    auto n = [&](int c) { return G.npol[c] + G.nmain[c]; };
    auto ring = [&](const RingSet &RS) {
        if (fp32) ring_launch_t<float, 2>(P, RS, nullptr, nullptr, nullptr, nullptr, W, nullptr, nullptr, nullptr, 1, false);
        else ring_launch_t<double, 2>(P, RS, nullptr, nullptr, nullptr, nullptr, W, nullptr, nullptr, nullptr, 1, false);
    };
    auto two = [&]() {
        leg_synth_cls<GCLS_BOTH>(P, fp32, 1, G.list[GCLS_BOTH], G.npol[GCLS_BOTH], G.nmain[GCLS_BOTH]);
        ring(P.rs_cls[0]);
        leg_adj_cls<GCLS_BOTH>(P, fp32, 0, G.list[GCLS_BOTH], G.npol[GCLS_BOTH], G.nmain[GCLS_BOTH], lv, 0, nrb);
    };
    auto one = [&]() {
        if (n(GCLS_NORTH))
            leg_synth_cls<GCLS_NORTH>(P, fp32, 1, G.list[GCLS_NORTH], G.npol[GCLS_NORTH], G.nmain[GCLS_NORTH]);
        if (n(GCLS_SOUTH))
            leg_synth_cls<GCLS_SOUTH>(P, fp32, 1, G.list[GCLS_SOUTH], G.npol[GCLS_SOUTH], G.nmain[GCLS_SOUTH]);
        ring(P.rs_cls[1]);
        if (n(GCLS_NORTH))
            leg_adj_cls<GCLS_NORTH>(P, fp32, 0, G.list[GCLS_NORTH], G.npol[GCLS_NORTH], G.nmain[GCLS_NORTH], lv,
                                    rb1, nrb);
        if (n(GCLS_SOUTH))
            leg_adj_cls<GCLS_SOUTH>(P, fp32, 0, G.list[GCLS_SOUTH], G.npol[GCLS_SOUTH], G.nmain[GCLS_SOUTH], lv,
                                    rb2, nrb);
    };
    fork_join(P, two, one);
    P.nrb_cur = nrb;
}

void launch_ring_grad(Plan &P, const double *g1, const double *g2, double *q1, double *q2, const double *W,
                      double *dninv, const uint8_t *mask, const double *cdev)
{
    ring_launch_t<double, 3>(P, P.rs_all, g1, g2, q1, q2, W, dninv, mask, cdev, 1);
}

// right-hand side of the backward solve: the upstream gradient on the stored (Re, Im) of the alm,
// divided by the full-m weight (1 for m = 0, 2 for m > 0), Im(a_l0) dropped
__global__ void k_vjp_rhs(const double *__restrict__ vE, const double *__restrict__ vB, double *__restrict__ bE,
                          double *__restrict__ bB, int64_t nalm, int lmax)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nalm) return;
    const bool m0 = i <= lmax;
    const double s = m0 ? 1.0 : 0.5;
    bE[2 * i] = s * vE[2 * i];
    bE[2 * i + 1] = m0 ? 0.0 : s * vE[2 * i + 1];
    bB[2 * i] = s * vB[2 * i];
    bB[2 * i + 1] = m0 ? 0.0 : s * vB[2 * i + 1];
}

void launch_vjp_rhs(Plan &P, const double *vE, const double *vB, double *bE, double *bB)
{
    k_vjp_rhs<<<(unsigned)cdiv(P.nalm, 256), 256, 0, P.stream>>>(vE, vB, bE, bB, P.nalm, P.lmax);
}

__global__ void k_scale_scalar(double *out, const double *in, double f) { *out = f * *in; }

void launch_scale_scalar(Plan &P, double *out, const double *in, double f)
{
    k_scale_scalar<<<1, 1, 0, P.stream>>>(out, in, f);
}

// one workgroup per ring: 1 when any of the nrhs weight maps has a nonzero weight on the ring
__global__ __launch_bounds__(256) void k_ring_live(const double *__restrict__ W, const RingInfo *__restrict__ rings,
                                                   int64_t npix, int nrhs, uint8_t *__restrict__ live)
{
    const RingInfo ri = rings[blockIdx.x];
    int any = 0;
    for (int r = 0; r < nrhs; ++r)
        for (int j = threadIdx.x; j < ri.nphi; j += blockDim.x) any |= W[r * npix + ri.ofs + j] != 0.0;
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) live[blockIdx.x] = any ? 1 : 0;
}

void launch_ring_live(Plan &P, int nrhs)
{
    k_ring_live<<<P.nrings, 256, 0, P.stream>>>(P.d_W, P.d_rings, P.npix, nrhs, P.d_ring_live);
}

void launch_weights(Plan &P, const double *ninv, const uint8_t *mask, int nrhs, int ncount)
{
    k_weights<<<dim3(RED_BLOCKS, nrhs), 256, 0, P.stream>>>(ninv, mask, P.d_W, P.npix, ncount, P.d_red);
    for (int r = 0; r < nrhs; ++r)
        k_sum_part<<<1, 256, 0, P.stream>>>(P.d_red + (int64_t)r * RED_BLOCKS * 4, RED_BLOCKS, 4, 4, P.d_scal + 8 + 4 * r);
}

void launch_dot(Plan &P, const double *a, const double *b, double *out_dev, int64_t n_complex)
{
    k_dot_part<<<RED_BLOCKS, 256, 0, P.stream>>>(a, b, n_complex, P.nalm, P.lmax, P.d_red);
    k_sum_part<<<1, 256, 0, P.stream>>>(P.d_red, RED_BLOCKS, 1, 1, out_dev);
}

void launch_cg_p(Plan &P, double *p, const double *r, const double *beta_dev, double precond, int64_t n_complex)
{
    k_cg_p<<<1024, 256, 0, P.stream>>>(p, r, beta_dev, precond, 2 * n_complex);
}

void launch_axpby(Plan &P, double *y, double a, const double *x, double b, int64_t n_complex)
{
    k_axpby<<<1024, 256, 0, P.stream>>>(y, a, x, b, 2 * n_complex);
}

void launch_scalar_div(Plan &P, double *out, const double *num, const double *den)
{
    k_scalar_div<<<1, 1, 0, P.stream>>>(out, num, den);
}

}  // namespace akra
