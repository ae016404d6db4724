// Catalogue pixelisation (Sec. III.B pixelization): galaxies binned onto the HEALPix RING grid, and
// per pixel the weighted shear (eq. gamma_obs), the effective count N_eff (eq. Neff_pixel), the
// inverse noise N^-1 = N_eff / sigma_e^2 (eq. noise_var) and the threshold mask (eq. mask).
//
// The sums of a pixel run over its galaxies in catalogue order: a stable radix sort of (pixel,
// galaxy) pairs groups them, and one thread per pixel accumulates sequentially with contraction
// off.  Every output is therefore a fixed, IEEE-rounded function of the catalogue -- no atomics,
// no dependence on scheduling -- and the threshold decision N_eff >= N_th is reproducible.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "akra_internal.h"

namespace akra {

// RING index of the direction (z = cos theta, phi in [0, 2 pi)) from the inverse of the HEALPix
// pixel boundaries (Gorski et al. 2005): in the equatorial belt |z| <= 2/3 the pixel edges are the
// lines Nside (1/2 + t) -+ (3/4) Nside z of t = phi / (pi/2), whose integer parts jp, jm give the
// ring ir = Nside + 1 + jp - jm (counted from z = 2/3) and the position in it; in the caps the edges
// are f h and (1 - f) h with f = frac(t), h = Nside sqrt(3 (1 - |z|)), giving the ring from the pole
// ir = jp + jm + 1 and the position floor(t ir) mod 4 ir.  Each product and sum is rounded on its own.
__device__ int64_t ang2pix_ring(int nside, double z, double phi)
{
#pragma clang fp contract(off)
    const int64_t n = nside;
    const double dn = (double)nside;
    const double za = fabs(z), tt = phi / (M_PI / 2);
    if (za <= 2.0 / 3.0) {
        const double t1 = dn * (0.5 + tt);
        const double t2 = dn * (z * 0.75);
        const int64_t jp = (int64_t)floor(t1 - t2), jm = (int64_t)floor(t1 + t2);
        const int64_t ir = n + 1 + jp - jm;
        const int64_t kshift = 1 - (ir & 1);
        const int64_t m4 = 4 * n;
        const int64_t ip = (((jp + jm - n + kshift + 1) >> 1) % m4 + m4) % m4;
        return 2 * n * (n - 1) + (ir - 1) * m4 + ip;
    }
    const double tp = tt - floor(tt);
    const double tmp = dn * sqrt(3.0 * (1.0 - za));
    const int64_t jp = (int64_t)floor(tp * tmp), jm = (int64_t)floor((1.0 - tp) * tmp);
    const int64_t ir = jp + jm + 1;
    const int64_t ip = ((int64_t)floor(tt * (double)ir)) % (4 * ir);
    return z > 0 ? 2 * ir * (ir - 1) + ip : 12 * n * n - 2 * ir * (ir + 1) + ip;
}

// pixel of every galaxy; inputs out of range set flag (1: position, 2: weight or ellipticity) and
// give pixel 0, so later stages stay in bounds.  With ellipticities, also the galaxy's record
// {w, w e1, w e2, w^2} (each product rounded once), so that the per-pixel pass gathers one 32-byte
// record per galaxy instead of three scattered values.
__global__ void k_ang2pix(const double *__restrict__ z, const double *__restrict__ phi,
                          const double *__restrict__ e1, const double *__restrict__ e2,
                          const double *__restrict__ w, int64_t n, int nside, uint32_t *__restrict__ pix,
                          double4 *__restrict__ rec, int *__restrict__ flag)
{
#pragma clang fp contract(off)
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double zz = z[j], pp = phi[j];
        int64_t p = 0;
        if (!(zz >= -1.0 && zz <= 1.0 && pp >= 0.0 && pp < 2.0 * M_PI)) {
            flag[0] = 1;
        } else {
            p = ang2pix_ring(nside, zz, pp);
        }
        if (e1) {
            const double ww = w[j], a = e1[j], b = e2[j];
            if (!(ww >= 0.0) || !isfinite(ww) || !isfinite(a) || !isfinite(b)) flag[1] = 2;
            rec[j] = make_double4(ww, ww * a, ww * b, ww * ww);
        }
        pix[j] = (uint32_t)p;
    }
}

__global__ void k_fill_i32(int32_t *__restrict__ a, int32_t *__restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a[i] = 0;
        b[i] = 0;
    }
}

// [start, end) of every pixel's run in the sorted keys (empty pixels keep 0, 0)
__global__ void k_seg_bounds(const uint32_t *__restrict__ keys, int64_t n, int32_t *__restrict__ start,
                             int32_t *__restrict__ end)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = keys[i];
        if (i == 0 || keys[i - 1] != p) start[p] = (int32_t)i;
        if (i == n - 1 || keys[i + 1] != p) end[p] = (int32_t)(i + 1);
    }
}

// per pixel: sums over its galaxies in catalogue order, then eq. gamma_obs, Neff_pixel, noise_var,
// mask (sum w = 0: no shear; sum w^2 = 0: N_eff = 0)
__global__ void k_pix_accum(const int32_t *__restrict__ start, const int32_t *__restrict__ end,
                            const uint32_t *__restrict__ gal, const double4 *__restrict__ rec, int64_t npix, double R,
                            double se2, double n_th, double *__restrict__ g1, double *__restrict__ g2,
                            double *__restrict__ ninv, double *__restrict__ neff, uint8_t *__restrict__ mask)
{
#pragma clang fp contract(off)
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
        double sw = 0.0, s1 = 0.0, s2 = 0.0, sww = 0.0;
        const int32_t b = start[p], e = end[p];
        for (int32_t i = b; i < e; ++i) {
            const double4 g = rec[gal[i]];
            sw = sw + g.x;
            s1 = s1 + g.y;
            s2 = s2 + g.z;
            sww = sww + g.w;
        }
        const double den = R * sw;
        const double ne = (sww != 0.0) ? (sw * sw) / sww : 0.0;
        g1[p] = (sw != 0.0) ? s1 / den : 0.0;
        g2[p] = (sw != 0.0) ? s2 / den : 0.0;
        neff[p] = ne;
        ninv[p] = ne / se2;
        mask[p] = ne >= n_th ? 1 : 0;
    }
}

static int key_bits(int64_t npix)
{
    int b = 1;
    while (((int64_t)1 << b) < npix) ++b;
    return b;
}

static int grid_for(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384));
}

// workspace: galaxy records, unsorted keys, sorted keys, sorted galaxy indices, pixel runs,
// radix-sort storage
struct PixWork {
    double4 *rec;
    uint32_t *keys, *keys_s, *gal_s;
    int32_t *seg_a, *seg_b;
    void *tmp;
    size_t tmp_bytes;
};

static int64_t a256(int64_t b) { return (b + 255) / 256 * 256; }

static hipError_t pixelize_work(Plan &P, int64_t n_gal, void *base, int64_t *bytes, PixWork *pw)
{
    size_t tb = 0;
    const uint32_t *kin = nullptr;
    uint32_t *kout = nullptr, *vout = nullptr;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, tb, kin, kout, rocprim::counting_iterator<uint32_t>(0u), vout,
                                             (size_t)std::max<int64_t>(n_gal, 1), 0u, (unsigned)key_bits(P.npix),
                                             P.stream);
    if (e != hipSuccess) return e;
    const int64_t ng = std::max<int64_t>(n_gal, 1);
    const int64_t total = a256(32 * ng) + 3 * a256(4 * ng) + 2 * a256(4 * P.npix) + a256((int64_t)tb);
    if (bytes) *bytes = total;
    if (pw && base) {
        char *c = (char *)base;
        pw->rec = (double4 *)c;
        c += a256(32 * ng);
        pw->keys = (uint32_t *)c;
        c += a256(4 * ng);
        pw->keys_s = (uint32_t *)c;
        c += a256(4 * ng);
        pw->gal_s = (uint32_t *)c;
        c += a256(4 * ng);
        pw->seg_a = (int32_t *)c;
        c += a256(4 * P.npix);
        pw->seg_b = (int32_t *)c;
        c += a256(4 * P.npix);
        pw->tmp = c;
        pw->tmp_bytes = tb;
    }
    return hipSuccess;
}

void launch_ang2pix(Plan &P, const double *z, const double *phi, const double *e1, const double *e2, const double *w,
                    int64_t n, uint32_t *pix, double4 *rec)
{
    if (n > 0) k_ang2pix<<<grid_for(n), 256, 0, P.stream>>>(z, phi, e1, e2, w, n, P.nside, pix, rec, P.d_cmp_flag);
}

hipError_t launch_pixelize(Plan &P, int64_t n, double R, double se2, double n_th, void *work, double *g1, double *g2,
                           double *ninv, double *neff, uint8_t *mask)
{
    PixWork pw;
    int64_t total = 0;
    hipError_t e = pixelize_work(P, n, work, &total, &pw);
    if (e != hipSuccess) return e;
    k_fill_i32<<<grid_for(P.npix), 256, 0, P.stream>>>(pw.seg_a, pw.seg_b, P.npix);
    if (n > 0) {
        size_t tb = pw.tmp_bytes;
        e = rocprim::radix_sort_pairs(pw.tmp, tb, pw.keys, pw.keys_s, rocprim::counting_iterator<uint32_t>(0u),
                                      pw.gal_s, (size_t)n, 0u, (unsigned)key_bits(P.npix), P.stream);
        if (e != hipSuccess) return e;
        k_seg_bounds<<<grid_for(n), 256, 0, P.stream>>>(pw.keys_s, n, pw.seg_a, pw.seg_b);
    }
    k_pix_accum<<<grid_for(P.npix), 256, 0, P.stream>>>(pw.seg_a, pw.seg_b, pw.gal_s, pw.rec, P.npix, R, se2, n_th, g1,
                                                        g2, ninv, neff, mask);
    return hipGetLastError();
}

hipError_t pixelize_work_bytes(Plan &P, int64_t n_gal, int64_t *bytes)
{
    return pixelize_work(P, n_gal, nullptr, bytes, nullptr);
}

uint32_t *pixelize_keys(Plan &P, int64_t n, void *work, double4 **rec)
{
    PixWork pw;
    if (pixelize_work(P, n, work, nullptr, &pw) != hipSuccess) return nullptr;
    *rec = pw.rec;
    return pw.keys;
}

}  // namespace akra
