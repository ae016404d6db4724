// Shape-noise realisations and power spectra of reconstructed convergence fields (Sec. IV, power
// spectrum results): the list of unmasked pixels, the shear permuted among them, the spectra
// C_l^{XY} of coefficient pairs and the moments of a set of realisations.
//
// All of it is HBM-bound bookkeeping next to the solves it feeds; the kernels keep the access
// patterns coalesced where the data allow (contiguous mask tiles, contiguous degree runs of the
// m-major coefficient layout) and make every result independent of scheduling (no atomics, fixed
// summation order).
#include "akra_internal.h"

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

void launch_spectra(Plan &P, const SpecArgs &a, int n)
{
    const int nlt = (P.lmax + SPEC_LT) / SPEC_LT;
    k_spec_part<<<dim3(nlt, P.spec_nmc, n), SPEC_LT, 0, P.stream>>>(a, P.lmax, P.spec_nmc, P.d_spec);
    k_spec_sum<<<dim3(nlt, n), SPEC_LT, 0, P.stream>>>(a, P.lmax, P.spec_nmc, P.d_spec);
}

void launch_cl_moments(Plan &P, const double *cl, int n, int64_t len, double *mean, double *sd)
{
    k_cl_moments<<<(int)((len + 255) / 256), 256, 0, P.stream>>>(cl, n, len, mean, sd);
}

}  // namespace akra
