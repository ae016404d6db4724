// Shape-noise realisations and power spectra of reconstructed convergence fields (Sec. IV, power
// spectrum results): the list of unmasked pixels, the shear permuted among them, the spectra
// C_l^{XY} of coefficient pairs and the moments of a set of realisations.
//
// All of it is HBM-bound bookkeeping next to the solves it feeds; the kernels keep the access
// patterns coalesced where the data allow (contiguous mask tiles, contiguous degree runs of the
// m-major coefficient layout) and make every result independent of scheduling (no atomics, fixed
// summation order).
#include "akra_internal.h"

#include <mutex>

namespace akra {

// ---- unmasked pixel list --------------------------------------------------------------------
// One block of CMP_T threads covers a tile of CMP_TILE pixels, CMP_PER contiguous per thread, so a
// block-wide exclusive scan of the per-thread counts orders the tile's unmasked pixels.

template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int *sh, int &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
        const int s = sh[k];
        before += (k < w) ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + inc - v;
}

__device__ __forceinline__ int tile_count(const uint8_t *__restrict__ mask, int64_t p0, int64_t npix)
{
    int c = 0;
#pragma unroll
    for (int i = 0; i < CMP_PER; ++i) {
        const int64_t p = p0 + i;
        c += (p < npix && mask[p] != 0) ? 1 : 0;
    }
    return c;
}

__global__ __launch_bounds__(CMP_T) void k_mask_count(const uint8_t *__restrict__ mask, int64_t npix,
                                                      int *__restrict__ cnt)
{
    __shared__ int sh[CMP_T / 64];
    const int64_t p0 = (int64_t)blockIdx.x * CMP_TILE + (int64_t)threadIdx.x * CMP_PER;
    int total;
    (void)block_excl_scan<CMP_T>(tile_count(mask, p0, npix), sh, total);
    if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// exclusive scan of the tile counts (one workgroup, chunks of 1024 with a running carry);
// offs[t] = first list position of tile t, *nobs = number of unmasked pixels
__global__ __launch_bounds__(1024) void k_mask_scan(const int *__restrict__ cnt, int ntile,
                                                    int64_t *__restrict__ offs, int64_t *__restrict__ nobs)
{
    __shared__ int sh[16];
    int64_t carry = 0;
    for (int base = 0; base < ntile; base += 1024) {
        const int t = base + (int)threadIdx.x;
        const int v = t < ntile ? cnt[t] : 0;
        int total;
        const int ex = block_excl_scan<1024>(v, sh, total);
        if (t < ntile) offs[t] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) nobs[0] = carry;
}

__global__ __launch_bounds__(CMP_T) void k_mask_write(const uint8_t *__restrict__ mask, int64_t npix,
                                                      const int64_t *__restrict__ offs, int32_t *__restrict__ idx)
{
    __shared__ int sh[CMP_T / 64];
    const int64_t p0 = (int64_t)blockIdx.x * CMP_TILE + (int64_t)threadIdx.x * CMP_PER;
    int total;
    int64_t pos = offs[blockIdx.x] + block_excl_scan<CMP_T>(tile_count(mask, p0, npix), sh, total);
#pragma unroll
    for (int i = 0; i < CMP_PER; ++i) {
        const int64_t p = p0 + i;
        if (p < npix && mask[p] != 0) idx[pos++] = (int32_t)p;
    }
}

// ---- shuffled shear -------------------------------------------------------------------------
__global__ void k_fill2(double *__restrict__ a, double *__restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a[i] = 0.0;
        b[i] = 0.0;
    }
}

// o[idx[j]] = g[idx[perm[j]]] for j < n_obs; an index out of range sets *flag and skips the entry
__global__ void k_shuffle(const double *__restrict__ g1, const double *__restrict__ g2,
                          const int32_t *__restrict__ idx, int64_t n_obs, int64_t npix,
                          const int32_t *__restrict__ perm, double *__restrict__ o1, double *__restrict__ o2,
                          int *__restrict__ flag)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_obs;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = perm[j];
        if (s < 0 || (int64_t)s >= n_obs) {
            flag[0] = 1;
            continue;
        }
        const int32_t d = idx[j], src = idx[s];
        if (d < 0 || (int64_t)d >= npix || src < 0 || (int64_t)src >= npix) {
            flag[0] = 2;
            continue;
        }
        o1[d] = g1[src];
        o2[d] = g2[src];
    }
}

// ---- spectra ----------------------------------------------------------------------------------
// Partial sums over m-chunks of SPEC_MC orders for degree tiles of SPEC_LT: block (tile, chunk,
// pair), thread = degree.  For one order m the tile's degrees are contiguous in the m-major
// layout, so each step reads SPEC_LT consecutive coefficients of X and Y.  Chunks beyond the
// tile's last degree hold nothing and are skipped (the sum kernel never reads them).
__global__ __launch_bounds__(SPEC_LT) void k_spec_part(SpecArgs a, int lmax, int nmc, double *__restrict__ part)
{
    const int l0 = blockIdx.x * SPEC_LT, l = l0 + (int)threadIdx.x;
    const int m0 = blockIdx.y * SPEC_MC, q = blockIdx.z;
    const int lhi = min(l0 + SPEC_LT - 1, lmax);
    if (m0 > lhi) return;
    const double2 *__restrict__ X = a.x[q];
    const double2 *__restrict__ Y = a.y[q];
    const int mend = min(m0 + SPEC_MC, lhi + 1);
    double acc = 0.0;
    for (int m = m0; m < mend; ++m) {
        if (l >= m && l <= lmax) {
            const int64_t i = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
            const double2 u = X[i], v = Y[i];
            const double t = u.x * v.x + u.y * v.y;  // Re(X conj Y)
            acc += (m == 0) ? t : 2.0 * t;
        }
    }
    if (l <= lmax) part[((int64_t)q * nmc + blockIdx.y) * (lmax + 1) + l] = acc;
}

__global__ __launch_bounds__(SPEC_LT) void k_spec_sum(SpecArgs a, int lmax, int nmc, const double *__restrict__ part)
{
    const int l = blockIdx.x * SPEC_LT + (int)threadIdx.x, q = blockIdx.y;
    if (l > lmax) return;
    double s = 0.0;
    if (l >= 2)
        for (int c = 0; c <= l / SPEC_MC; ++c) s += part[((int64_t)q * nmc + c) * (lmax + 1) + l];
    a.cl[q][l] = (l >= 2) ? s / (double)(2 * l + 1) : 0.0;
}

// mean and sample standard deviation over n realisations of len values each (two passes)
__global__ void k_cl_moments(const double *__restrict__ cl, int n, int64_t len, double *__restrict__ mean,
                             double *__restrict__ sd)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += cl[(int64_t)k * len + i];
    const double mu = n > 0 ? s / n : 0.0;
    double v = 0.0;
    for (int k = 0; k < n; ++k) {
        const double d = cl[(int64_t)k * len + i] - mu;
        v += d * d;
    }
    if (mean) mean[i] = mu;
    if (sd) sd[i] = n > 1 ? sqrt(v / (n - 1)) : 0.0;
}

// ---- launchers ----------------------------------------------------------------------------------
void launch_unmasked_index(Plan &P, const uint8_t *mask, int32_t *idx)
{
    const int nt = (int)P.cmp_ntile;
    k_mask_count<<<nt, CMP_T, 0, P.stream>>>(mask, P.npix, P.d_cmp_cnt);
    k_mask_scan<<<1, 1024, 0, P.stream>>>(P.d_cmp_cnt, nt, P.d_cmp_offs, P.d_cmp_nobs);
    k_mask_write<<<nt, CMP_T, 0, P.stream>>>(mask, P.npix, P.d_cmp_offs, idx);
}

void launch_shuffle(Plan &P, const double *g1, const double *g2, const int32_t *idx, int64_t n_obs,
                    const int32_t *perm, double *o1, double *o2)
{
    k_fill2<<<1024, 256, 0, P.stream>>>(o1, o2, P.npix);
    if (perm && n_obs > 0) {
        const int64_t nb = std::min<int64_t>((n_obs + 255) / 256, 8192);
        k_shuffle<<<(int)nb, 256, 0, P.stream>>>(g1, g2, idx, n_obs, P.npix, perm, o1, o2, P.d_cmp_flag);
    }
}

// partial sums in part[n][nmc][lmax + 1]; every entry the sum kernel reads is written first by the
// part kernel of the same launch pair, so part needs no clearing
static void spectra_on(const SpecArgs &a, int n, int lmax, int nmc, double *part, hipStream_t stream)
{
    const int nlt = (lmax + SPEC_LT) / SPEC_LT;
    k_spec_part<<<dim3(nlt, nmc, n), SPEC_LT, 0, stream>>>(a, lmax, nmc, part);
    k_spec_sum<<<dim3(nlt, n), SPEC_LT, 0, stream>>>(a, lmax, nmc, part);
}

void launch_spectra(Plan &P, const SpecArgs &a, int n)
{
    spectra_on(a, n, P.lmax, P.spec_nmc, P.d_spec, P.stream);
}

void launch_cl_moments(Plan &P, const double *cl, int n, int64_t len, double *mean, double *sd)
{
    k_cl_moments<<<(int)((len + 255) / 256), 256, 0, P.stream>>>(cl, n, len, mean, sd);
}

// ---- spectra without allocation --------------------------------------------------------------
// The partial sums of akra_alm_spectra_noalloc live in this file-scope device array, one copy per
// GPU for the life of the process, sized for SPEC_NP pairs at lmax = AKRA_NOALLOC_LMAX_MAX.  Host code
// never uses the array's name as an address: the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current, and only that address is
// passed to the kernels.
constexpr int64_t NOALLOC_NMC = (AKRA_NOALLOC_LMAX_MAX + SPEC_MC) / SPEC_MC;
constexpr int64_t NOALLOC_DOUBLES = (int64_t)SPEC_NP * NOALLOC_NMC * (AKRA_NOALLOC_LMAX_MAX + 1);
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEV = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[NOALLOC_MAX_DEV] = {};

// device address of the current device's scratch array (set up on the first call on that device)
static akra_status scratch_address(int dev, double **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return AKRA_ERR_HIP;
        }
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return AKRA_OK;
}

}  // namespace akra

using namespace akra;

extern "C" akra_status akra_alm_spectra_noalloc(int lmax, const double *x, int nx, const double *y, int ny,
                                                const int32_t *pairs, int npairs, double *cl, void *hip_stream)
{
    TraceRange trace_range("akra_alm_spectra_noalloc");
    // every argument is checked before the first HIP call
    if (lmax < 0 || lmax > AKRA_NOALLOC_LMAX_MAX) {
        set_error("lmax " + std::to_string(lmax) + " is outside [0, " + std::to_string(AKRA_NOALLOC_LMAX_MAX) +
                  "], the largest band limit the static scratch of akra_alm_spectra_noalloc holds");
        return AKRA_ERR_ARG;
    }
    if (npairs < 0 || nx < 0 || ny < 0) {
        set_error("counts must be >= 0");
        return AKRA_ERR_ARG;
    }
    if (npairs == 0) return AKRA_OK;
    if (!x || !y || !pairs || !cl) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    if (((uintptr_t)x | (uintptr_t)y) % 16) {
        set_error("coefficient arrays must be 16-byte aligned (complex128)");
        return AKRA_ERR_ARG;
    }
    for (int q = 0; q < npairs; ++q)
        if (pairs[2 * q] < 0 || pairs[2 * q] >= nx || pairs[2 * q + 1] < 0 || pairs[2 * q + 1] >= ny) {
            set_error("pair " + std::to_string(q) + " is out of range");
            return AKRA_ERR_ARG;
        }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEV) {
        set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return AKRA_ERR_HIP;
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    if (stream) {
        int sdev = -1;
        e = hipStreamGetDevice(stream, &sdev);
        if (e != hipSuccess || sdev != dev) {
            set_error("the stream does not belong to the current device");
            return AKRA_ERR_ARG;
        }
    }
    double *part = nullptr;
    const akra_status st = scratch_address(dev, &part);
    if (st != AKRA_OK) return st;
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    const int nmc = (lmax + SPEC_MC) / SPEC_MC;
    const double2 *X = (const double2 *)x, *Y = (const double2 *)y;
    for (int q0 = 0; q0 < npairs; q0 += SPEC_NP) {
        SpecArgs a{};
        const int n = std::min(SPEC_NP, npairs - q0);
        for (int i = 0; i < n; ++i) {
            a.x[i] = X + (int64_t)pairs[2 * (q0 + i)] * nalm;
            a.y[i] = Y + (int64_t)pairs[2 * (q0 + i) + 1] * nalm;
            a.cl[i] = cl + (int64_t)(q0 + i) * (lmax + 1);
        }
        spectra_on(a, n, lmax, nmc, part, stream);
    }
    e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("spectra launch: ") + hipGetErrorString(e));
        return AKRA_ERR_HIP;
    }
    return AKRA_OK;
}
