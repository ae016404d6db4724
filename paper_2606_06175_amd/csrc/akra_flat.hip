// Flat-sky variant of the operator (Sec. II.B, storage problem: on a flat field each spherical
// harmonic transform becomes a 2-D FFT, the four-step operator and the CG solver are unchanged).
//
// Unknown: the complex convergence z = kappa_E + i kappa_B on an nx x ny periodic grid, held by the
// solver as its unitary 2-D Fourier transform x = F z.  With the flat-sky Kaiser-Squires kernel
// D(k) = (k1 + i k2)^2 / |k|^2 (D(0) = 0):
//   A z = F^-1 (D x),   H x = conj(D) F (W F^-1 (D x)) + lambda_eff x,   b = conj(D) F (W gamma_obs).
// CG on x is CG on z (F is unitary), with two 2-D FFTs per apply instead of four.
//
// Layouts: maps are [ny][nx] float64 (i1 fast); the solver's Fourier vectors are stored transposed,
// [nx][ny] complex (rows indexed by the x frequency n1), so each 2-D transform is one row pass, one
// tiled transpose and one row pass, and the pixel-space weighting sits between an inverse and a
// forward row transform of the same row in LDS:
//   H x:  rows n1: x.D -> iFFT along n2 | transpose | rows i2: iFFT along n1, x W, FFT along i1 |
//         transpose | rows n1: FFT along i2, x conj(D) / (nx ny), + lambda x.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "akra_fft.h"
#include "akra_internal.h"

#define FK_HIP(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return akra::hip_fail(e_, what); \
    } while (0)

namespace akra {

constexpr int FL_MAXN = 8192;  // longest row a workgroup transforms in LDS (FP64)
constexpr int FL_RED = 1024;   // partial sums of the dot products

struct FlatPlan {
    int nx = 0, ny = 0;
    int64_t n = 0;
    hipStream_t stream = nullptr;
    double2 *d_tw = nullptr;  // e^{-2 pi i k / twn}, k < twn / 2
    int twn = 1;
    double *d_W = nullptr;  // [ny][nx]
    double2 *d_x = nullptr, *d_r = nullptr, *d_p = nullptr, *d_w = nullptr, *d_b = nullptr;  // [nx][ny]
    double2 *d_t1 = nullptr, *d_t2 = nullptr;  // transposition buffers
    double *d_red = nullptr, *d_scal = nullptr;
    int *d_flag = nullptr;
    double *h_pin = nullptr;
    int64_t device_bytes = 0;
    double step_lam = 0, step_pc = 1;  // lambda_eff and P of the step-wise solve
    bool step_ready = false;
};

// signed frequency of index k of a length-n transform, divided by n
__device__ __forceinline__ double ffreq(int k, int n) { return (double)(k < n / 2 ? k : k - n) / (double)n; }

// D(k) = (k1 + i k2)^2 / |k|^2 at frequency indices (n1, n2); 0 at k = 0
__device__ __forceinline__ double2 ks_D(int n1, int nx, int n2, int ny)
{
    const double a = ffreq(n1, nx), b = ffreq(n2, ny);
    const double k2 = a * a + b * b;
    if (k2 == 0.0) return make_double2(0.0, 0.0);
    return make_double2((a * a - b * b) / k2, 2.0 * a * b / k2);
}

// row-pass modes
enum { FR_INV_D = 0, FR_PIX_W = 1, FR_FWD_MAPS = 2, FR_FWD_OUT = 3, FR_INV_MAPS = 4 };

struct FRowArgs {
    const double2 *in;          // complex rows [rows][L]
    const double *in1, *in2;    // real maps [rows][L] (FR_FWD_MAPS)
    double2 *out;               // complex rows [rows][L]
    double *out1, *out2;        // real maps (FR_INV_MAPS)
    const double *W;            // weights [rows][L] (FR_PIX_W; FR_FWD_MAPS when non-null)
    const double2 *xadd;        // FR_FWD_OUT: + lam * xadd when non-null
    double *dot_part;           // FR_FWD_OUT: per-row Re sum conj(xadd) out when non-null
    double lam, scale;
    int L;                      // row length (power of two)
    int dmode;                  // FR_INV_D / FR_FWD_OUT: 0 times D, 1 times conj(D), -1 none
    int nx, ny;                 // grid: in FR_INV_D / FR_FWD_OUT the row is n1, the position n2
    const double2 *tw;
    int twn;
};

__device__ __forceinline__ double2 dfac(int mode, int n1, int nx, int n2, int ny)
{
    const double2 d = ks_D(n1, nx, n2, ny);
    return mode == 1 ? make_double2(d.x, -d.y) : d;
}

// One workgroup of NT threads transforms one row of length L <= FL_MAXN in LDS.
template <int NT, int MODE>
__global__ __launch_bounds__(NT) void k_frow(FRowArgs a)
{
    extern __shared__ double2 buf[];
    const int r = blockIdx.x, L = a.L, tid = threadIdx.x;
    const int logL = 31 - __builtin_clz(L);
    const int64_t base = (int64_t)r * L;
    if constexpr (MODE == FR_INV_D || MODE == FR_PIX_W || MODE == FR_INV_MAPS) {
        // natural order in, inverse transform (sign +1), bit-reversed out
        for (int k = tid; k < L; k += NT) {
            double2 v = a.in[base + k];
            if (MODE == FR_INV_D && a.dmode >= 0) v = cmul<double>(v, dfac(a.dmode, r, a.nx, k, a.ny));
            buf[pd(k)] = v;
        }
        __syncthreads();
        fft_dif<double, NT>(buf, L, a.tw, a.twn, +1);
        if constexpr (MODE == FR_INV_D) {
            for (int k = tid; k < L; k += NT) {
                const double2 v = buf[pd(brev(k, logL))];
                a.out[base + k] = make_double2(v.x * a.scale, v.y * a.scale);
            }
        } else if constexpr (MODE == FR_INV_MAPS) {
            for (int k = tid; k < L; k += NT) {
                const double2 v = buf[pd(brev(k, logL))];
                a.out1[base + k] = v.x * a.scale;
                a.out2[base + k] = v.y * a.scale;
            }
        } else {
            // pixel row: weight, then the forward transform back (bit-reversed in, natural out)
            for (int k = tid; k < L; k += NT) {
                const int s = pd(brev(k, logL));
                const double w = a.W[base + k];
                const double2 v = buf[s];
                buf[s] = make_double2(v.x * w, v.y * w);
            }
            __syncthreads();
            fft_dit<double, NT>(buf, L, a.tw, a.twn, -1);
            for (int k = tid; k < L; k += NT) {
                const double2 v = buf[pd(k)];
                a.out[base + k] = make_double2(v.x * a.scale, v.y * a.scale);
            }
        }
    } else {
        // bit-reversed in, forward transform (sign -1), natural out
        for (int k = tid; k < L; k += NT) {
            double2 v;
            if constexpr (MODE == FR_FWD_MAPS) {
                v = make_double2(a.in1[base + k], a.in2[base + k]);
                if (a.W) {
                    const double w = a.W[base + k];
                    v = make_double2(v.x * w, v.y * w);
                }
            } else {
                v = a.in[base + k];
            }
            buf[pd(brev(k, logL))] = v;
        }
        __syncthreads();
        fft_dit<double, NT>(buf, L, a.tw, a.twn, -1);
        double dot = 0.0;
        for (int k = tid; k < L; k += NT) {
            double2 v = buf[pd(k)];
            v = make_double2(v.x * a.scale, v.y * a.scale);
            if constexpr (MODE == FR_FWD_OUT) {
                if (a.dmode >= 0) v = cmul<double>(v, dfac(a.dmode, r, a.nx, k, a.ny));
                if (a.xadd) {
                    const double2 x = a.xadd[base + k];
                    v = make_double2(v.x + a.lam * x.x, v.y + a.lam * x.y);
                    dot += x.x * v.x + x.y * v.y;
                }
            }
            a.out[base + k] = v;
        }
        if constexpr (MODE == FR_FWD_OUT) {
            if (a.dot_part) {
                // row sum in a fixed order: within waves by butterfly, then the waves in order
                __shared__ double wsum[NT / 64];
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o, 64);
                if ((tid & 63) == 0) wsum[tid >> 6] = dot;
                __syncthreads();
                if (tid == 0) {
                    double t = 0.0;
                    for (int w = 0; w < NT / 64; ++w) t += wsum[w];
                    a.dot_part[r] = t;
                }
            }
        }
    }
}

// out[c][r] = in[r][c] for an [R][C] complex array, through 32 x 32 LDS tiles
__global__ __launch_bounds__(256) void k_ftranspose(const double2 *__restrict__ in, double2 *__restrict__ out, int R,
                                                    int C)
{
    __shared__ double2 tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = 0; k < 32; k += 8) {
        const int r = r0 + ty + k, c = c0 + tx;
        if (r < R && c < C) tile[ty + k][tx] = in[(int64_t)r * C + c];
    }
    __syncthreads();
    for (int k = 0; k < 32; k += 8) {
        const int c = c0 + ty + k, r = r0 + tx;
        if (r < R && c < C) out[(int64_t)c * R + r] = tile[tx][ty + k];
    }
}

// ---- reductions and CG vector updates --------------------------------------------------------------
__device__ __forceinline__ double block_sum256(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// partials of Re sum conj(a) b
__global__ __launch_bounds__(256) void k_fdot_part(const double2 *__restrict__ a, const double2 *__restrict__ b,
                                                   int64_t n, double *__restrict__ part)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double2 u = a[i], v = b[i];
        s += u.x * v.x + u.y * v.y;
    }
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sums of np partial rows of width k, in a fixed order: out[q] = sum_b part[b * k + q]
__global__ __launch_bounds__(256) void k_fsum(const double *__restrict__ part, int np, int k, double *__restrict__ out)
{
    __shared__ double sh[256];
    for (int q = 0; q < k; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < np; b += 256) s += part[(int64_t)b * k + q];
        s = block_sum256(s, sh);
        if (threadIdx.x == 0) out[q] = s;
    }
}

// W = M N^-1 and the sums sum W, sum M, non-finite count, negative count
__global__ __launch_bounds__(256) void k_fweights(const double *__restrict__ ninv, const uint8_t *__restrict__ mask,
                                                  double *__restrict__ W, int64_t n, double *__restrict__ part)
{
    __shared__ double sh[256];
    double sw = 0, sm = 0, nf = 0, ng = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = ninv[i];
        const bool obs = mask[i] != 0;
        if (!isfinite(v)) nf += 1;
        if (v < 0) ng += 1;
        const double w = obs ? v : 0.0;
        W[i] = w;
        sw += w;
        sm += obs ? 1.0 : 0.0;
    }
    sw = block_sum256(sw, sh);
    sm = block_sum256(sm, sh);
    nf = block_sum256(nf, sh);
    ng = block_sum256(ng, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = sw;
        part[blockIdx.x * 4 + 1] = sm;
        part[blockIdx.x * 4 + 2] = nf;
        part[blockIdx.x * 4 + 3] = ng;
    }
}

// scalars s: [0] rz, [1] <p, w>, [2] alpha, [3] <r, r>, [4] beta, [7] rz of the iteration in progress

__global__ void k_fcg_beta(double *s, double pc)
{
    const double rz = pc * s[3];
    s[4] = s[0] > 0.0 ? rz / s[0] : 0.0;
    s[0] = rz;
}

// r -= alpha w, with per-block partials of <r, r>.  Every workgroup forms alpha = rz / <p, w> itself;
// breakdown (p^T H p <= 0 or non-finite) gives alpha = 0 and raises the flag, which is sticky (alpha
// stays 0 until the host reads it).  Workgroup 0 records alpha, keeps rz at s[7] for the p update
// and raises the flag.
__global__ __launch_bounds__(256) void k_fcg_r_alpha(double2 *__restrict__ r, const double2 *__restrict__ w,
                                                     double *__restrict__ s, int *__restrict__ flag, int64_t n,
                                                     double *__restrict__ part)
{
    __shared__ double sh[256];
    const double pw = s[1], rz = s[0];
    const bool bad = flag[0] != 0 || !(pw > 0.0) || !isfinite(pw);
    const double al = bad ? 0.0 : rz / pw;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double2 wv = w[i];
        double2 rv = r[i];
        rv.x -= al * wv.x;
        rv.y -= al * wv.y;
        r[i] = rv;
        acc += rv.x * rv.x + rv.y * rv.y;
    }
    acc = block_sum256(acc, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc;
        if (blockIdx.x == 0) {
            s[2] = al;
            s[7] = rz;
            if (bad) flag[0] = 1;
        }
    }
}

// <r, r> from the np partials (every workgroup, in the order of k_fsum), beta = P <r, r> / rz with rz
// from s[7], then x += alpha p and p = P r + beta p in one pass; workgroup 0 records <r, r>, beta and
// the new rz = P <r, r>
__global__ __launch_bounds__(256) void k_fcg_px_beta(double2 *__restrict__ x, double2 *__restrict__ p,
                                                     const double2 *__restrict__ r, const double *__restrict__ part,
                                                     int np, double *__restrict__ s, double pc, int64_t n)
{
    __shared__ double sh[256];
    double t = 0.0;
    for (int b = threadIdx.x; b < np; b += 256) t += part[b];
    const double rr = block_sum256(t, sh);
    const double rzn = pc * rr;
    const double rz_old = s[7];
    const double be = rz_old > 0.0 ? rzn / rz_old : 0.0;
    const double al = s[2];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s[3] = rr;
        s[4] = be;
        s[0] = rzn;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 pv = p[i], rv = r[i];
        double2 xv = x[i];
        xv.x += al * pv.x;
        xv.y += al * pv.y;
        x[i] = xv;
        p[i] = make_double2(pc * rv.x + be * pv.x, pc * rv.y + be * pv.y);
    }
}

// y = a x + b y
__global__ void k_faxpby(double2 *__restrict__ y, double a, const double2 *__restrict__ x, double b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 xv = x[i], yv = y[i];
        y[i] = make_double2(a * xv.x + b * yv.x, a * xv.y + b * yv.y);
    }
}

// ---- launch helpers ---------------------------------------------------------------------------------
static int vgrid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

// LDS bytes of a row of length L with the pad slot of pd() every 32 elements
static size_t row_lds(int L) { return (size_t)(L + (L - 1) / 32) * sizeof(double2); }

template <int MODE> static void row_pass_nt(FlatPlan &F, FRowArgs a, int rows)
{
    const size_t lds = row_lds(a.L);
    if (a.L >= 4096)
        k_frow<1024, MODE><<<rows, 1024, lds, F.stream>>>(a);
    else if (a.L >= 1024)
        k_frow<256, MODE><<<rows, 256, lds, F.stream>>>(a);
    else
        k_frow<64, MODE><<<rows, 64, lds, F.stream>>>(a);
}

template <int MODE> static hipError_t allow_lds()
{
    hipError_t e = hipFuncSetAttribute((const void *)k_frow<1024, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)row_lds(FL_MAXN));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_frow<256, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)row_lds(FL_MAXN));
    return e;
}

static FRowArgs row_args(FlatPlan &F, int L)
{
    FRowArgs a{};
    a.L = L;
    a.scale = 1.0;
    a.dmode = -1;
    a.nx = F.nx;
    a.ny = F.ny;
    a.tw = F.d_tw;
    a.twn = F.twn;
    return a;
}

static void transpose(FlatPlan &F, const double2 *in, double2 *out, int R, int C)
{
    k_ftranspose<<<dim3((C + 31) / 32, (R + 31) / 32), 256, 0, F.stream>>>(in, out, R, C);
}

// x = F (m1 + i m2) [x W] [x conj(D) or D] (unitary), into the transposed layout [nx][ny]
static void to_fourier(FlatPlan &F, const double *m1, const double *m2, const double *W, int dmode, double2 *x)
{
    FRowArgs a = row_args(F, F.nx);
    a.in1 = m1;
    a.in2 = m2;
    a.W = W;
    a.out = F.d_t1;
    row_pass_nt<FR_FWD_MAPS>(F, a, F.ny);
    transpose(F, F.d_t1, F.d_t2, F.ny, F.nx);
    FRowArgs b = row_args(F, F.ny);
    b.in = F.d_t2;
    b.out = x;
    b.dmode = dmode;
    b.scale = 1.0 / std::sqrt((double)F.n);
    row_pass_nt<FR_FWD_OUT>(F, b, F.nx);
}

// (o1 + i o2) = F^-1 ([D or conj(D)] x) (unitary)
static void to_maps(FlatPlan &F, const double2 *x, int dmode, double *o1, double *o2)
{
    FRowArgs a = row_args(F, F.ny);
    a.in = x;
    a.out = F.d_t1;
    a.dmode = dmode;
    row_pass_nt<FR_INV_D>(F, a, F.nx);
    transpose(F, F.d_t1, F.d_t2, F.nx, F.ny);
    FRowArgs b = row_args(F, F.nx);
    b.in = F.d_t2;
    b.out1 = o1;
    b.out2 = o2;
    b.scale = 1.0 / std::sqrt((double)F.n);
    row_pass_nt<FR_INV_MAPS>(F, b, F.ny);
}

// y = conj(D) F (W F^-1 (D x)) + lam x, with the weights in d_W; with dot_out, also <x, y> there
static void apply_H(FlatPlan &F, const double2 *x, double2 *y, double lam, double *dot_out = nullptr)
{
    FRowArgs a = row_args(F, F.ny);
    a.in = x;
    a.out = F.d_t1;
    a.dmode = 0;
    row_pass_nt<FR_INV_D>(F, a, F.nx);
    transpose(F, F.d_t1, F.d_t2, F.nx, F.ny);
    FRowArgs b = row_args(F, F.nx);
    b.in = F.d_t2;
    b.out = F.d_t1;
    b.W = F.d_W;
    row_pass_nt<FR_PIX_W>(F, b, F.ny);
    transpose(F, F.d_t1, F.d_t2, F.ny, F.nx);
    FRowArgs c = row_args(F, F.ny);
    c.in = F.d_t2;
    c.out = y;
    c.dmode = 1;
    c.scale = 1.0 / (double)F.n;
    c.xadd = (lam != 0.0 || dot_out) ? x : nullptr;
    c.lam = lam;
    c.dot_part = dot_out ? F.d_red : nullptr;
    row_pass_nt<FR_FWD_OUT>(F, c, F.nx);
    if (dot_out) k_fsum<<<1, 256, 0, F.stream>>>(F.d_red, F.nx, 1, dot_out);
}

// one PCG iteration on device-resident state (scalars in d_scal):
//   w = H p and <p, w> in one pass, alpha, r -= alpha w and <r, r>, beta, x += alpha p and
//   p = P r + beta p in one pass
static void cg_iteration(FlatPlan &F, double lam, double pc)
{
    double *s = F.d_scal;
    const int vg = vgrid(F.n);
    apply_H(F, F.d_p, F.d_w, lam, s + 1);
    k_fcg_r_alpha<<<FL_RED, 256, 0, F.stream>>>(F.d_r, F.d_w, s, F.d_flag, F.n, F.d_red);
    k_fcg_px_beta<<<vg, 256, 0, F.stream>>>(F.d_x, F.d_p, F.d_r, F.d_red, FL_RED, s, pc, F.n);
}

static void fdot(FlatPlan &F, const double2 *a, const double2 *b, double *out)
{
    k_fdot_part<<<FL_RED, 256, 0, F.stream>>>(a, b, F.n, F.d_red);
    k_fsum<<<1, 256, 0, F.stream>>>(F.d_red, FL_RED, 1, out);
}

static hipError_t read_dev(FlatPlan &F, const double *src, int k, double *dst)
{
    hipError_t e = hipMemcpyAsync(F.h_pin, src, sizeof(double) * k, hipMemcpyDeviceToHost, F.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(F.stream);
    if (e == hipSuccess) std::memcpy(dst, F.h_pin, sizeof(double) * k);
    return e;
}

// W from ninv and mask (validated), lambda_eff and the scalar preconditioner
static akra_status weights(FlatPlan &F, const double *ninv, const uint8_t *mask, double lam, double *lam_eff, double *pc)
{
    if (!ninv || !mask) {
        set_error("ninv and mask must be device pointers");
        return AKRA_ERR_ARG;
    }
    k_fweights<<<FL_RED, 256, 0, F.stream>>>(ninv, mask, F.d_W, F.n, F.d_red);
    k_fsum<<<1, 256, 0, F.stream>>>(F.d_red, FL_RED, 4, F.d_scal + 8);
    double s[4];
    FK_HIP(read_dev(F, F.d_scal + 8, 4, s), "weights");
    if (s[2] > 0) {
        set_error("ninv holds NaN or Inf");
        return AKRA_ERR_NUMERIC;
    }
    if (s[3] > 0) {
        set_error("ninv holds negative weights");
        return AKRA_ERR_ARG;
    }
    *lam_eff = s[1] > 0 ? lam * s[0] / s[1] : 0.0;
    *pc = 1.0 / (s[0] / (double)F.n + *lam_eff);
    return AKRA_OK;
}

static void free_flat(FlatPlan *F)
{
    void *ptrs[] = {F->d_tw, F->d_W, F->d_x, F->d_r, F->d_p, F->d_w, F->d_b, F->d_t1, F->d_t2, F->d_red, F->d_scal,
                    F->d_flag};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (F->h_pin) (void)hipHostFree(F->h_pin);
    delete F;
}

}  // namespace akra

using namespace akra;

extern "C" {

struct akra_flat_plan_s {
    FlatPlan *F;
};

static bool pow2_in(int n) { return n >= 4 && n <= FL_MAXN && (n & (n - 1)) == 0; }

akra_status akra_flat_plan_create(int nx, int ny, void *hip_stream, akra_flat_plan *out)
{
    TraceRange trace_range("akra_flat_plan_create");
    if (!out) {
        set_error("out is NULL");
        return AKRA_ERR_ARG;
    }
    *out = nullptr;
    if (!pow2_in(nx) || !pow2_in(ny)) {
        set_error("nx and ny must be powers of two in [4, 8192]");
        return AKRA_ERR_ARG;
    }
    FlatPlan *F = new FlatPlan();
    F->nx = nx;
    F->ny = ny;
    F->n = (int64_t)nx * ny;
    F->stream = (hipStream_t)hip_stream;
    F->twn = std::max(nx, ny);
    auto al = [&](void **p, size_t b) -> bool {
        if (hipMalloc(p, std::max<size_t>(b, 16)) != hipSuccess) {
            *p = nullptr;
            return false;
        }
        F->device_bytes += (int64_t)b;
        return true;
    };
    const size_t cb = (size_t)F->n * sizeof(double2);
    bool ok = al((void **)&F->d_tw, sizeof(double2) * (F->twn / 2)) && al((void **)&F->d_W, sizeof(double) * F->n) &&
              al((void **)&F->d_x, cb) && al((void **)&F->d_r, cb) && al((void **)&F->d_p, cb) &&
              al((void **)&F->d_w, cb) && al((void **)&F->d_b, cb) && al((void **)&F->d_t1, cb) &&
              al((void **)&F->d_t2, cb) && al((void **)&F->d_red, sizeof(double) * std::max(FL_RED * 4, nx)) &&
              al((void **)&F->d_scal, sizeof(double) * 64) && al((void **)&F->d_flag, sizeof(int) * 4);
    if (ok && hipHostMalloc((void **)&F->h_pin, 64 * sizeof(double)) != hipSuccess) {
        F->h_pin = nullptr;
        ok = false;
    }
    if (!ok) {
        free_flat(F);
        set_error("device allocation failed");
        return AKRA_ERR_ALLOC;
    }
    std::vector<double2> tw(F->twn / 2);
    for (int k = 0; k < F->twn / 2; ++k) {
        const long double t = -2.0L * 3.141592653589793238462643383279502884L * k / F->twn;
        tw[k] = make_double2((double)cosl(t), (double)sinl(t));
    }
    if (hipMemcpy(F->d_tw, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice) != hipSuccess ||
        allow_lds<FR_INV_D>() != hipSuccess || allow_lds<FR_PIX_W>() != hipSuccess ||
        allow_lds<FR_FWD_MAPS>() != hipSuccess || allow_lds<FR_FWD_OUT>() != hipSuccess ||
        allow_lds<FR_INV_MAPS>() != hipSuccess || hipMemset(F->d_flag, 0, sizeof(int) * 4) != hipSuccess) {
        free_flat(F);
        set_error("plan set-up failed");
        return AKRA_ERR_HIP;
    }
    *out = new akra_flat_plan_s{F};
    return AKRA_OK;
}

void akra_flat_plan_destroy(akra_flat_plan plan)
{
    if (!plan) return;
    (void)hipStreamSynchronize(plan->F->stream);
    free_flat(plan->F);
    delete plan;
}

int64_t akra_flat_plan_device_bytes(akra_flat_plan plan) { return plan ? plan->F->device_bytes : 0; }

#define FL_PLAN()                          \
    if (!plan) {                           \
        set_error("plan is NULL");         \
        return AKRA_ERR_ARG;               \
    }                                      \
    FlatPlan &F = *plan->F

static akra_status fl_check(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return AKRA_OK;
}

akra_status akra_flat_synth(akra_flat_plan plan, const double *kE, const double *kB, double *g1, double *g2)
{
    TraceRange trace_range("akra_flat_synth");
    FL_PLAN();
    if (!kE || !kB || !g1 || !g2) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    to_fourier(F, kE, kB, nullptr, -1, F.d_x);
    to_maps(F, F.d_x, 0, g1, g2);
    return fl_check("flat_synth");
}

akra_status akra_flat_adjoint(akra_flat_plan plan, const double *g1, const double *g2, double *yE, double *yB)
{
    TraceRange trace_range("akra_flat_adjoint");
    FL_PLAN();
    if (!g1 || !g2 || !yE || !yB) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    to_fourier(F, g1, g2, nullptr, 1, F.d_x);
    to_maps(F, F.d_x, -1, yE, yB);
    return fl_check("flat_adjoint");
}

akra_status akra_flat_apply_H(akra_flat_plan plan, const double *ninv, const uint8_t *mask, double lambda_eff,
                              const double *kE, const double *kB, double *yE, double *yB)
{
    TraceRange trace_range("akra_flat_apply_H");
    FL_PLAN();
    if (!kE || !kB || !yE || !yB) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    double le, pc;
    akra_status st = weights(F, ninv, mask, 0.0, &le, &pc);
    if (st) return st;
    to_fourier(F, kE, kB, nullptr, -1, F.d_x);
    apply_H(F, F.d_x, F.d_w, lambda_eff);
    to_maps(F, F.d_w, -1, yE, yB);
    return fl_check("flat_apply_H");
}

akra_status akra_flat_rhs(akra_flat_plan plan, const double *g1, const double *g2, const double *ninv,
                          const uint8_t *mask, double *bE, double *bB)
{
    TraceRange trace_range("akra_flat_rhs");
    FL_PLAN();
    if (!g1 || !g2 || !bE || !bB) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    double le, pc;
    akra_status st = weights(F, ninv, mask, 0.0, &le, &pc);
    if (st) return st;
    to_fourier(F, g1, g2, F.d_W, 1, F.d_b);
    to_maps(F, F.d_b, -1, bE, bB);
    return fl_check("flat_rhs");
}

akra_status akra_flat_cg_solve(akra_flat_plan plan, const double *g1, const double *g2, const double *ninv,
                               const uint8_t *mask, const akra_cg_opts *opts, double *kE, double *kB,
                               akra_cg_info *info_out)
{
    TraceRange trace_range("akra_flat_cg_solve");
    FL_PLAN();
    auto t0 = std::chrono::steady_clock::now();
    akra_cg_opts o;
    akra_cg_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.tol > 0) || o.maxiter < 0 || !(o.lambda >= 0) || o.mode != AKRA_JOINT_EB || o.kernel_l ||
        o.stall_iters < 0 || o.check_every < 0) {
        set_error("flat solve: tol > 0, maxiter >= 0, lambda >= 0, stall_iters >= 0, check_every >= 0, joint mode "
                  "and no kernel_l are required");
        return AKRA_ERR_ARG;
    }
    if (!g1 || !g2 || !kE || !kB) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    double le, pc;
    akra_status st = weights(F, ninv, mask, o.lambda, &le, &pc);
    if (st) return st;
    const int64_t n = F.n;
    const int vg = vgrid(n);
    double *s = F.d_scal;
    to_fourier(F, g1, g2, F.d_W, 1, F.d_b);
    if (o.use_x0) {
        to_fourier(F, kE, kB, nullptr, -1, F.d_x);
        apply_H(F, F.d_x, F.d_w, le);
        FK_HIP(hipMemcpyAsync(F.d_r, F.d_b, sizeof(double2) * n, hipMemcpyDeviceToDevice, F.stream), "copy");
        k_faxpby<<<vg, 256, 0, F.stream>>>(F.d_r, -1.0, F.d_w, 1.0, n);
    } else {
        FK_HIP(hipMemsetAsync(F.d_x, 0, sizeof(double2) * n, F.stream), "memset");
        FK_HIP(hipMemcpyAsync(F.d_r, F.d_b, sizeof(double2) * n, hipMemcpyDeviceToDevice, F.stream), "copy");
    }
    FK_HIP(hipMemsetAsync(F.d_flag, 0, sizeof(int), F.stream), "memset");
    fdot(F, F.d_b, F.d_b, s + 5);
    fdot(F, F.d_r, F.d_r, s + 3);
    double hs[6];
    FK_HIP(read_dev(F, s, 6, hs), "cg");
    if (!std::isfinite(hs[5])) {
        set_error("right-hand side is not finite");
        return AKRA_ERR_NUMERIC;
    }
    akra_cg_info info{};
    info.lambda_eff = le;
    info.precond = pc;
    const double bn = std::sqrt(hs[5]);
    int result = AKRA_OK;
    int it = 0;
    if (bn > 0) {
        // p = P r, rz = P <r, r>
        FK_HIP(hipMemsetAsync(F.d_p, 0, sizeof(double2) * n, F.stream), "memset");
        k_faxpby<<<vg, 256, 0, F.stream>>>(F.d_p, pc, F.d_r, 0.0, n);
        double rr = hs[3], rel = std::sqrt(rr) / bn;
        const double rz0 = pc * rr;
        FK_HIP(hipMemcpyAsync(s, &rz0, sizeof(double), hipMemcpyHostToDevice, F.stream), "copy");
        result = AKRA_NOT_CONVERGED;
        StallWatch stall(o.stall_iters, rel);
        while (true) {
            if (rel < o.tol) {
                result = AKRA_OK;
                break;
            }
            if (it >= o.maxiter) break;
            const int nb = std::min(o.check_every > 1 ? o.check_every : 1, o.maxiter - it);
            for (int b = 0; b < nb; ++b) cg_iteration(F, le, pc);
            it += nb;
            st = fl_check("flat_cg");
            if (st) return st;
            FK_HIP(hipMemcpyAsync(F.h_pin, s + 3, sizeof(double), hipMemcpyDeviceToHost, F.stream), "copy");
            FK_HIP(hipMemcpyAsync(F.h_pin + 1, F.d_flag, sizeof(int), hipMemcpyDeviceToHost, F.stream), "copy");
            FK_HIP(hipStreamSynchronize(F.stream), "sync");
            rr = F.h_pin[0];
            int flag = 0;
            std::memcpy(&flag, F.h_pin + 1, sizeof(int));
            if (flag || !std::isfinite(rr)) {
                set_error("CG breakdown (p^T H p <= 0 or a non-finite residual)");
                return AKRA_ERR_NUMERIC;
            }
            rel = std::sqrt(rr) / bn;
            if (o.resid_hist && it <= o.resid_hist_len) o.resid_hist[it - 1] = rel;
            if (rel >= o.tol && stall.step(rel)) {
                result = AKRA_STAGNATED;
                set_error("CG stagnated: no new smallest residual in stall_iters iterations");
                break;
            }
        }
        info.rel_resid = rel;
        // true residual
        apply_H(F, F.d_x, F.d_w, le);
        FK_HIP(hipMemcpyAsync(F.d_r, F.d_b, sizeof(double2) * n, hipMemcpyDeviceToDevice, F.stream), "copy");
        k_faxpby<<<vg, 256, 0, F.stream>>>(F.d_r, -1.0, F.d_w, 1.0, n);
        fdot(F, F.d_r, F.d_r, s + 6);
        double tr;
        FK_HIP(read_dev(F, s + 6, 1, &tr), "cg");
        info.rel_resid_true = std::sqrt(tr) / bn;
    } else {
        FK_HIP(hipMemsetAsync(F.d_x, 0, sizeof(double2) * n, F.stream), "memset");
    }
    to_maps(F, F.d_x, -1, kE, kB);
    st = fl_check("flat_cg");
    if (st) return st;
    FK_HIP(hipStreamSynchronize(F.stream), "sync");
    info.iters = it;
    info.status = result;
    info.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info_out) *info_out = info;
    if (result == AKRA_NOT_CONVERGED) set_error("maxiter reached");
    return (akra_status)result;
}

// ---- step-wise form for timing: start, steps without synchronisation ----------------------------
akra_status akra_flat_cg_start(akra_flat_plan plan, const double *g1, const double *g2, const double *ninv,
                               const uint8_t *mask, double lambda)
{
    TraceRange trace_range("akra_flat_cg_start");
    FL_PLAN();
    if (!g1 || !g2) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    double le, pc;
    akra_status st = weights(F, ninv, mask, lambda, &le, &pc);
    if (st) return st;
    const int vg = vgrid(F.n);
    to_fourier(F, g1, g2, F.d_W, 1, F.d_b);
    FK_HIP(hipMemsetAsync(F.d_x, 0, sizeof(double2) * F.n, F.stream), "memset");
    FK_HIP(hipMemcpyAsync(F.d_r, F.d_b, sizeof(double2) * F.n, hipMemcpyDeviceToDevice, F.stream), "copy");
    FK_HIP(hipMemsetAsync(F.d_p, 0, sizeof(double2) * F.n, F.stream), "memset");
    k_faxpby<<<vg, 256, 0, F.stream>>>(F.d_p, pc, F.d_r, 0.0, F.n);
    fdot(F, F.d_r, F.d_r, F.d_scal + 3);
    k_fcg_beta<<<1, 1, 0, F.stream>>>(F.d_scal, pc);  // rz = P <r, r>
    FK_HIP(hipStreamSynchronize(F.stream), "sync");
    F.step_lam = le;
    F.step_pc = pc;
    F.step_ready = true;
    return fl_check("flat_cg_start");
}

akra_status akra_flat_cg_step(akra_flat_plan plan, int nsteps)
{
    TraceRange trace_range("akra_flat_cg_step");
    FL_PLAN();
    if (nsteps < 0 || !F.step_ready) {
        set_error("nsteps must be >= 0, after akra_flat_cg_start");
        return AKRA_ERR_ARG;
    }
    const double le = F.step_lam, pc = F.step_pc;
    for (int k = 0; k < nsteps; ++k) cg_iteration(F, le, pc);
    return fl_check("flat_cg_step");
}

}  // extern "C"
