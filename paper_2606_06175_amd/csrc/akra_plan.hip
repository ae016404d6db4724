// Host side of libakra: plan (geometry, recurrence tables, seeds, workspaces), the C ABI and
// the conjugate-gradient drivers (paper Sec. II.B, inversion problem; eq. ML_estimator_reg,
// eq. precond).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "akra_internal.h"

// FP32 plans run the spin-weighted recurrences of ring pairs within AKRA_DIFF_THETA radians of a pole
// in the difference form.  Near a pole the per-step phase advance of the recurrence is of the order
// of theta; in the plain form the FP32 rounding of each step moves the phase by ~eps/theta, an
// error that grows like sqrt(l) eps/theta.  The difference form keeps it at ~sqrt(l) eps there but
// rounds more at large theta; the two errors cross near 0.45 rad.
#ifndef AKRA_DIFF_THETA
#define AKRA_DIFF_THETA 0.45
#endif

namespace akra {

static thread_local std::string g_err;
// largest whole-ring Bluestein convolution of plans created afterwards (akra_set_ring_whole_maxm)
static int g_ring_whole_maxm = 8192;
static int g_ring_register = 1;
void set_error(const std::string &msg) { g_err = msg; }
akra_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return AKRA_ERR_HIP;
}

#define AK_HIP(call, what)                         \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

template <class F> static void parallel_for(int n, F f)
{
    int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nt = std::min(nt, std::max(1, n));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([=]() {
            for (int i = t; i < n; i += nt) f(i);
        });
    for (auto &x : th) x.join();
}

// ---------------------------------------------------------------------------------------------
// HEALPix RING geometry (Gorski et al. 2005; the pixelisation of Sec. III.B).  A ring is defined
// by its double-precision z computed exactly as below.
// ---------------------------------------------------------------------------------------------
static void build_rings(Plan &P)
{
    const int ns = P.nside;
    P.nrings = 4 * ns - 1;
    P.npairs = 2 * ns;
    P.npix = 12LL * ns * ns;
    P.omega = 4.0 * M_PI / (double)P.npix;
    P.h_rings.resize(P.nrings);
    int64_t ofs = 0;
    for (int k = 0; k < P.nrings; ++k) {
        const int i = k + 1;
        RingInfo r{};
        if (i < ns || i > 3 * ns) {
            const int ii = (i < ns) ? i : 4 * ns - i;
            const double d = (double)((int64_t)ii * ii) / (3.0 * ns * ns);
            r.z = (i < ns) ? (1.0 - d) : -(1.0 - d);
            r.nphi = 4 * ii;
            r.shift = 1;
        } else {
            r.z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns);
            r.nphi = 4 * ns;
            r.shift = (i - ns + 1) % 2;
        }
        r.ofs = ofs;
        r.sub = r.nphi / 4;
        r.M = 0;
        if (!pow2(r.sub)) {
            int M = 1;
            while (M < 2 * r.sub - 1) M <<= 1;
            r.M = M;
        }
        ofs += r.nphi;
        P.h_rings[k] = r;
    }
}

// ---------------------------------------------------------------------------------------------
// Recurrence coefficients of lambda_l = sqrt((2l+1)/(4pi)) d^l_{m,mp}(theta), mp = -+2, from the
// three-term recurrence of the Wigner d-functions:
//   a_l = (l+1) sqrt((2l+1)(2l+3)) / R_{l+1},  b_l = 2m sqrt((2l+1)(2l+3)) / (l R_{l+1}),
//   g_l = (l+1) R_l sqrt((2l+3)/(2l-1)) / (l R_{l+1}),   R_l = sqrt((l^2 - m^2)(l^2 - 4)).
// ---------------------------------------------------------------------------------------------
// Entries past the last column (ALM_PAD) keep the kernels' look-ahead loads in bounds.
// The scaled form (Coef64S) divides out c_l with c_{l0} = c_{l0+1} = 1, c_{l+1} = g_l c_{l-1}: entries
// below l0 and the padding carry c = 1, the entry at lmax its c with a' = b' = 0.
static void build_coef(int lmax, std::vector<Coef64> &c64, std::vector<Coef32> &c32, std::vector<Coef32D> &c32d,
                       std::vector<Coef64S> &c64s, std::vector<Coef32S> &c32s)
{
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    c64.assign(nalm + ALM_PAD, Coef64{0, 0, 0, 0});
    c32.assign(nalm + ALM_PAD, Coef32{0, 0, 0, 0});
    c32d.assign(nalm + ALM_PAD, Coef32D{0, 0, 0, 0});
    c64s.assign(nalm + ALM_PAD, Coef64S{0, 0, 1, 1});
    c32s.assign(nalm + ALM_PAD, Coef32S{0, 0, 1, 1});
    parallel_for(lmax + 1, [&](int m) {
        const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
        const int l0 = std::max(m, 2);
        typedef long double ld;
        auto R = [&](int l) { return sqrtl(((ld)l * l - (ld)m * m) * ((ld)l * l - 4.0L)); };
        std::vector<ld> cs(lmax + 2, 1.0L);  // c_l, l0 <= l <= lmax
        for (int l = l0; l < lmax; ++l) {
            const ld L = l;
            const ld r1 = R(l + 1), r0 = R(l);
            const ld q = sqrtl((2 * L + 1) * (2 * L + 3));
            const ld a = (L + 1) * q / r1;
            const ld b = 2.0L * m * q / (L * r1);
            const ld g = (L + 1) * r0 * sqrtl((2 * L + 3) / (2 * L - 1)) / (L * r1);
            c64[base + l] = Coef64{(double)a, (double)b, (double)g, 0.0};
            c32[base + l] = Coef32{(float)a, (float)b, (float)g, 0.0f};
            c32d[base + l] = Coef32D{(float)a, (float)(a + b - g - 1), (float)(a - b - g - 1), (float)g};
            if (l > l0) cs[l + 1] = g * cs[l - 1];
            const ld f = cs[l] / cs[l + 1];
            c64s[base + l] = Coef64S{(double)(a * f), (double)(b * f), (double)cs[l], (double)(1.0L / cs[l])};
            c32s[base + l] = Coef32S{(float)(a * f), (float)(b * f), (float)cs[l], (float)(1.0L / cs[l])};
        }
        c64s[base + lmax] = Coef64S{0.0, 0.0, (double)cs[lmax], (double)(1.0L / cs[lmax])};
        c32s[base + lmax] = Coef32S{0.0f, 0.0f, (float)cs[lmax], (float)(1.0L / cs[lmax])};
    });
}

// ---------------------------------------------------------------------------------------------
// Seeds lambda_{l0,m}, l0 = max(m,2), for the north ring of every pair, by a recurrence in m:
//   t_2 = d^2_{22} = c^4,  t_{m+1} = -t_m sqrt((2m+2)(2m+1)/((m+3)(m-1))) c s   (t_m = d^m_{m,2}),
//   d^m_{m,-2} = t_m (s/c)^4;  for m < 2: d^2_{0,+-2} = sqrt6 c^2 s^2, d^2_{1,2} = 2 c^3 s, d^2_{1,-2} = -2 c s^3.
// c = cos(theta/2), s = sin(theta/2).  Long double with explicit binary exponents; stored as
// mant * 2^(512 k) (see Scale<double>).
// ---------------------------------------------------------------------------------------------
static void build_seeds(Plan &P, std::vector<double> &s2, std::vector<double> &sm, std::vector<int> &sk)
{
    typedef long double ld;
    const int lmax = P.lmax, np = P.npairs;
    s2.assign((size_t)(lmax + 1) * np, 0.0);
    sm.assign((size_t)(lmax + 1) * np, 0.0);
    sk.assign((size_t)(lmax + 1) * np, 0);
    std::vector<ld> fac(lmax + 2, 0.0L);
    for (int m = 2; m <= lmax; ++m) fac[m] = sqrtl((ld)(2 * m + 2) * (2 * m + 1) / ((ld)(m + 3) * (m - 1)));
    const ld inv4pi = 1.0L / (4.0L * 3.141592653589793238462643383279502884L);
    parallel_for(np, [&](int p) {
        const ld z = P.h_rings[p].z;
        const ld c = sqrtl((1 + z) / 2), s = sqrtl((1 - z) / 2);
        const ld cs = c * s, t4 = (s / c) * (s / c) * (s / c) * (s / c);
        auto store = [&](int m, ld mant_m2, int e_m2, ld mant_2, int e_2) {
            // value_m2 = mant_m2 2^e_m2 is -2lambda (mp = +2), value_2 = 2lambda (mp = -2)
            const int l0 = std::max(m, 2);
            const ld nrm = sqrtl((2 * l0 + 1) * inv4pi);
            int ea, eb;
            ld fa = frexpl(mant_m2 * nrm, &ea), fb = frexpl(mant_2 * nrm, &eb);
            ea += e_m2;
            eb += e_2;
            if (fa == 0) ea = -1000000;
            if (fb == 0) eb = -1000000;
            const int ebig = std::max(ea, eb);
            int k = 0;
            if (ebig < -400) k = (int)std::floor((ebig + 300) / 512.0);
            const size_t idx = (size_t)m * np + p;
            sm[idx] = (double)ldexpl(fa, ea - 512 * k);
            s2[idx] = (double)ldexpl(fb, eb - 512 * k);
            sk[idx] = k;
        };
        store(0, sqrtl(6.0L) * c * c * s * s, 0, sqrtl(6.0L) * c * c * s * s, 0);
        if (lmax >= 1) store(1, 2.0L * c * c * c * s, 0, -2.0L * c * s * s * s, 0);
        int e = 0;
        ld t = frexpl(c * c * c * c, &e);  // t_2
        for (int m = 2; m <= lmax; ++m) {
            if (m > 2) {
                int de;
                t = frexpl(-t * fac[m - 1] * cs, &de);
                e += de;
            }
            int de2;
            ld u = frexpl(t * t4, &de2);
            store(m, t, e, u, e + de2);
        }
    });
}

// Triples (l, m, ring pair) the Legendre kernels evaluate with the current launch shapes: a wave of
// the synthesis starts at the earliest entry degree of its slots' groups, a workgroup of the adjoint
// at the earliest of its groups; every lane of a started wave or workgroup steps to lmax.
static void compute_work(Plan &P)
{
    const int lmax = P.lmax, np = P.npairs, ng = P.ng64, gp = P.polar_groups;
    auto pairs_in = [&](int g0, int g1) { return (int64_t)std::max(0, std::min(np, 64 * g1) - 64 * g0); };
    int64_t all = 0, syn = 0, adj = 0, bat = 0;
    // blocks of gs groups over [g0, g1): each starts at the earliest entry degree of its groups
    auto seg = [&](const int *e, int g0, int g1, int gs) {
        int64_t w = 0;
        for (int b = g0; b < g1; b += gs) {
            int ls = ENT_SKIP;
            for (int g = b; g < std::min(g1, b + gs); ++g) ls = std::min(ls, e[g]);
            if (ls <= lmax) w += pairs_in(b, std::min(g1, b + gs)) * (lmax - ls + 1);
        }
        return w;
    };
    // adjoint workgroups over [g0, g1) as adj_split places them
    auto seg_adj = [&](const int *e, int g0, int g1, int R, int W) {
        const AdjSplit sp = adj_split(g1 - g0, R, W);
        int64_t w = 0;
        for (int b = 0; b < sp.q; ++b) {
            int first, count;
            adj_block(sp, g1 - g0, W, b, first, count);
            const int a0 = g0 + first, a1 = a0 + count;
            int ls = ENT_SKIP;
            for (int g = a0; g < a1; ++g) ls = std::min(ls, e[g]);
            if (ls <= lmax) w += pairs_in(a0, a1) * (lmax - ls + 1);
        }
        return w;
    };
    for (int m = 0; m <= lmax; ++m) {
        all += (int64_t)np * (lmax - std::max(m, 2) + 1);
        const int *e = P.h_entl.data() + (size_t)m * ng;
        syn += seg(e, 0, gp, 1) + seg(e, gp, ng, P.syn_R);
        adj += seg_adj(e, 0, gp, P.adj_Rpol, 1) + seg_adj(e, gp, ng, P.adj_R, P.adj_W);
        bat += seg(e, 0, ng, 1);
    }
    P.work[0] = all;
    P.work[1] = syn;
    P.work[2] = adj;
    P.work_b = bat;
}

static akra_status upload(void **dst, const void *src, size_t bytes, Plan &P)
{
    AK_HIP(hipMalloc(dst, std::max<size_t>(bytes, 16)), "hipMalloc");
    P.device_bytes += (int64_t)bytes;
    if (src) AK_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy");
    return AKRA_OK;
}

static akra_status alloc(void **dst, size_t bytes, Plan &P)
{
    AK_HIP(hipMalloc(dst, std::max<size_t>(bytes, 16)), "hipMalloc");
    P.device_bytes += (int64_t)bytes;
    return AKRA_OK;
}

static void default_kernel(int lmax, std::vector<double> &k)
{
    // K_l = sigma_D D_l, sigma_D = -1, D_l = -sqrt((l-1)(l+2)/(l(l+1))) (eq. Dl_kernel), K_0 = K_1 = 0
    k.assign(lmax + 1, 0.0);
    for (int l = 2; l <= lmax; ++l) k[l] = std::sqrt((double)(l - 1) * (l + 2) / ((double)l * (l + 1)));
}

// ---- rings and groups that carry weight -------------------------------------------------------
// ints of the device list buffer: the ring lists of every kind, then GCLS_N + 1 group lists
static size_t live_list_ints(const Plan &P) { return (size_t)RING_KINDS * P.nrings + (GCLS_N + 1) * (size_t)P.ng64; }
// pinned bytes: the ring flags (padded to 16), then the staged lists
static size_t live_stage_bytes(const Plan &P) { return (size_t)(P.nrings + 15) / 16 * 16 + 4 * live_list_ints(P); }

// Evaluated (l, m, pair) triples of the Legendre kernels over the weighted group lists: a synthesis
// wave of syn_R list entries (one for near-polar groups) and an adjoint workgroup of adj_R adj_W
// entries (four near-polar) start at the earliest entry degree among their groups; every pair of
// their groups steps to lmax.  Split into two-ring and one-ring classes; the last count is that of
// the batched kernels (every weighted group from its own entry degree).
static void compute_work_live(Plan &P)
{
    const GroupSet &G = P.gs_live;
    const int lmax = P.lmax, ng = P.ng64, np = P.npairs;
    std::vector<int> hl[GCLS_N];
    const int *base = (const int *)(P.h_live + (P.nrings + 15) / 16 * 16) + (size_t)RING_KINDS * P.nrings;
    for (int c = 0; c < GCLS_N; ++c) hl[c].assign(base + (size_t)c * ng, base + (size_t)c * ng + G.npol[c] + G.nmain[c]);
    auto seg = [&](const int *e, const int *gl, int n, int gs) {
        int64_t w = 0;
        for (int b = 0; b < n; b += gs) {
            int ls = ENT_SKIP;
            int64_t pairs = 0;
            for (int i = b; i < std::min(n, b + gs); ++i) {
                ls = std::min(ls, e[gl[i]]);
                pairs += std::min(64, np - 64 * gl[i]);
            }
            if (ls <= lmax) w += pairs * (lmax - ls + 1);
        }
        return w;
    };
    auto seg_adj = [&](const int *e, const int *gl, int n, int R, int W) {
        const AdjSplit sp = adj_split(n, R, W);
        int64_t w = 0;
        for (int b = 0; b < sp.q; ++b) {
            int first, count;
            adj_block(sp, n, W, b, first, count);
            int ls = ENT_SKIP;
            int64_t pairs = 0;
            for (int i = first; i < first + count; ++i) {
                ls = std::min(ls, e[gl[i]]);
                pairs += std::min(64, np - 64 * gl[i]);
            }
            if (ls <= lmax) w += pairs * (lmax - ls + 1);
        }
        return w;
    };
    const int *any = base + (size_t)GCLS_N * ng;
    const int nany = G.npol_any + G.nmain_any;
    int64_t w[5] = {0, 0, 0, 0, 0};
    for (int m = 0; m <= lmax; ++m) {
        const int *e = P.h_entl.data() + (size_t)m * ng;
        w[4] += seg(e, any, nany, 1);
        for (int c = 0; c < GCLS_N; ++c) {
            const int *gl = hl[c].data();
            const int npol = G.npol[c], nmain = G.nmain[c];
            const bool two = c == GCLS_BOTH;
            const int64_t s = seg(e, gl, npol, 1) + seg(e, gl + npol, nmain, two ? P.syn_R : P.syn_R1);
            const int64_t a = seg_adj(e, gl, npol, P.adj_Rpol, 1) + seg_adj(e, gl + npol, nmain, two ? P.adj_R : P.adj_R1,
                                                                 two ? P.adj_W : P.adj_W1);
            w[c == GCLS_BOTH ? 0 : 1] += s;
            w[c == GCLS_BOTH ? 2 : 3] += a;
        }
    }
    for (int i = 0; i < 5; ++i) P.work_live[i] = w[i];
}

// From the ring flags in h_live: the ring lists of every kind and the group lists of every class,
// staged after the flags and uploaded to d_live_lists (stream-ordered before the next launches);
// rs_live and gs_live then describe them.
static akra_status build_live_lists(Plan &P)
{
    const uint8_t *flag = P.h_live;
    // the same rings as at the last set-up: the lists on the device (and recorded graphs) still hold
    if (P.live_gen && P.h_live_prev.size() == (size_t)P.nrings &&
        std::memcmp(P.h_live_prev.data(), flag, (size_t)P.nrings) == 0)
        return AKRA_OK;
    P.h_live_prev.assign(flag, flag + P.nrings);
    int *stage = (int *)(P.h_live + (P.nrings + 15) / 16 * 16);
    // class of every 64-pair group by the rings of its pairs that carry weight (-1: none)
    std::vector<int> gcls(P.ng64, -1);
    for (int g = 0; g < P.ng64; ++g) {
        bool n = false, s = false;
        for (int p = 64 * g; p < std::min(P.npairs, 64 * g + 64); ++p) {
            const int rs = P.nrings - 1 - p;
            n = n || flag[p];
            s = s || (rs != p && flag[rs]);
        }
        if (n || s) gcls[g] = (n && s) ? GCLS_BOTH : n ? GCLS_NORTH : GCLS_SOUTH;
    }
    // ring lists per kind: the weighted rings of two-sided groups, then those of one-sided groups
    for (int k = 0; k < RING_KINDS; ++k) {
        int *o = stage + (size_t)k * P.nrings;
        int n = 0, n2 = 0;
        for (int two = 1; two >= 0; --two) {
            for (int r : P.h_order[k]) {
                const int p = std::min(r, P.nrings - 1 - r);
                if (flag[r] && (gcls[p / 64] == GCLS_BOTH) == (two == 1)) o[n++] = r;
            }
            if (two) n2 = n;
        }
        int *d = P.d_live_lists + (size_t)k * P.nrings;
        P.rs_live.order[k] = d;
        P.rs_live.n[k] = n;
        P.rs_cls[0].order[k] = d;
        P.rs_cls[0].n[k] = n2;
        P.rs_cls[1].order[k] = d + n2;
        P.rs_cls[1].n[k] = n - n2;
    }
    int *gbase = stage + (size_t)RING_KINDS * P.nrings;
    int cnt[GCLS_N + 1] = {0, 0, 0, 0}, pol[GCLS_N + 1] = {0, 0, 0, 0};
    for (int g = 0; g < P.ng64; ++g) {
        if (gcls[g] < 0) continue;
        const int c = gcls[g];
        for (int cc : {c, (int)GCLS_N}) {
            gbase[(size_t)cc * P.ng64 + cnt[cc]++] = g;
            if (g < P.polar_groups) pol[cc]++;
        }
    }
    GroupSet &G = P.gs_live;
    for (int c = 0; c < GCLS_N; ++c) {
        G.list[c] = P.d_live_lists + (size_t)RING_KINDS * P.nrings + (size_t)c * P.ng64;
        G.npol[c] = pol[c];
        G.nmain[c] = cnt[c] - pol[c];
    }
    G.list_any = P.d_live_lists + (size_t)RING_KINDS * P.nrings + (size_t)GCLS_N * P.ng64;
    G.npol_any = pol[GCLS_N];
    G.nmain_any = cnt[GCLS_N] - pol[GCLS_N];
    AK_HIP(hipMemcpyAsync(P.d_live_lists, stage, live_list_ints(P) * sizeof(int), hipMemcpyHostToDevice, P.stream),
           "hipMemcpyAsync");
    P.live_gen++;
    P.n_live_rings = 0;
    for (int r = 0; r < P.nrings; ++r) P.n_live_rings += flag[r] != 0;
    compute_work_live(P);
    return AKRA_OK;
}

static void free_plan(Plan *P)
{
    void *ptrs[] = {P->d_rings, P->d_pair_z, P->d_coef64, P->d_coef32, P->d_coef64s, P->d_coef32s, P->d_recu,
                    P->d_seed2, P->d_seedm2, P->d_seedk,
                    P->d_ent, P->d_entk, P->d_entl, P->d_wgstart, P->d_wgstart_b, P->d_coef32d, P->d_brec,
                    P->d_tw64, P->d_tw32, P->d_bhat64, P->d_bhat32, P->d_bhatr64, P->d_bhatr32, P->d_order_r[0], P->d_order_r[1],
                    P->d_order_r[2], P->d_order_r[3], P->d_order_r[4], P->d_order_r[5], P->d_lof, P->d_order_p2, P->d_order_bl, P->d_order_bf, P->d_FG, P->d_part, P->d_rec, P->d_W, P->d_kern, P->d_kuser, P->d_red, P->d_red_cg, P->d_scal, P->d_flag, P->d_x, P->d_r,
                    P->d_p, P->d_w, P->d_b, P->d_xs, P->d_cmp, P->d_spec, P->d_gl_all, P->d_live_lists,
                    P->d_ring_live};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (P->h_pin) (void)hipHostFree(P->h_pin);
    if (P->h_live) (void)hipHostFree(P->h_live);
    for (auto &e : P->ev_pool) {
        (void)hipEventDestroy(e[0]);
        (void)hipEventDestroy(e[1]);
    }
    if (P->cg_graph) (void)hipGraphExecDestroy(P->cg_graph);
    if (P->cg_graph_b) (void)hipGraphExecDestroy(P->cg_graph_b);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    if (P->side_stream) (void)hipStreamDestroy(P->side_stream);
    if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
    if (P->ev_join) (void)hipEventDestroy(P->ev_join);
    delete P;
}

static akra_status create(int nside, int lmax, int nrhs, int prec, void *stream, Plan **out)
{
    if (nside < 1 || nside > 2048) {
        set_error("nside must be in [1, 2048]");
        return AKRA_ERR_ARG;
    }
    if (lmax < 2 || lmax > 4 * nside) {
        set_error("lmax must be in [2, 4 nside]");
        return AKRA_ERR_ARG;
    }
    if (nrhs < 1 || nrhs > 64) {
        set_error("nrhs must be in [1, 64]");
        return AKRA_ERR_ARG;
    }
    if (prec != AKRA_FP64 && prec != AKRA_FP32) {
        set_error("precision must be AKRA_FP64 or AKRA_FP32");
        return AKRA_ERR_ARG;
    }
    Plan *P = new Plan();
    P->nside = nside;
    P->lmax = lmax;
    P->nrhs = nrhs;
    P->prec = prec;
    P->stream = (hipStream_t)stream;
    (void)hipGetDevice(&P->dev);
    P->nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    build_rings(*P);

    // ring launch lists, largest first: power-of-two rings (whole-ring FFT), rings whose whole-ring
    // Bluestein convolution fits in LDS (M <= BF_MAXM), and the rest as two sub-transforms of length
    // N / 2, each by Bluestein (M <= 8192 since N <= 4 nside <= 8192)
    // Rings whose transform length is 4096 or 8192 (a whole power-of-two ring, or a whole-ring
    // Bluestein convolution) go to the register engine unless it is switched off.
    const int BF_MAXM = g_ring_whole_maxm;
    std::vector<int> p2, bl, bf, rl[6];
    int maxp2 = 1, maxbl = 1, maxbf = 1, maxreg = 1;  // the LDS kernels' lists, and the register engine
    for (int r = 0; r < P->nrings; ++r) {
        RingInfo &ri = P->h_rings[r];
        if (!ri.M) {
            if (g_ring_register && (ri.nphi == 4096 || ri.nphi == 8192)) {
                rl[ri.nphi == 4096 ? 0 : 1].push_back(r);
                maxreg = std::max(maxreg, ri.nphi);
            } else {
                p2.push_back(r);
                maxp2 = std::max(maxp2, ri.sub);
            }
            continue;
        }
        int MF = 1;
        while (MF < 2 * ri.nphi - 1) MF <<= 1;
        if (MF <= BF_MAXM) {
            ri.M = MF;  // the whole ring's convolution length
            if (g_ring_register && (MF == 4096 || MF == 8192)) {
                rl[MF == 4096 ? 2 : 3].push_back(r);
                maxreg = std::max(maxreg, MF);
            } else {
                bf.push_back(r);
                maxbf = std::max(maxbf, MF);
            }
        } else {
            int M2 = 1;
            while (M2 < ri.nphi - 1) M2 <<= 1;  // 2 (N / 2) - 1
            ri.M = M2;
            if (g_ring_register && (M2 == 4096 || M2 == 8192)) {
                rl[M2 == 4096 ? 4 : 5].push_back(r);
                maxreg = std::max(maxreg, M2);
            } else {
                bl.push_back(r);
                maxbl = std::max(maxbl, M2);
            }
        }
    }
    auto bysize = [&](int a, int b) { return P->h_rings[a].nphi > P->h_rings[b].nphi; };
    std::stable_sort(p2.begin(), p2.end(), bysize);
    std::stable_sort(bl.begin(), bl.end(), bysize);
    std::stable_sort(bf.begin(), bf.end(), bysize);
    for (auto &v : rl) std::stable_sort(v.begin(), v.end(), bysize);
    for (int q = 0; q < 6; ++q) P->n_r[q] = (int)rl[q].size();
    P->h_order[RK_P2] = p2;
    P->h_order[RK_BF] = bf;
    P->h_order[RK_BL] = bl;
    for (int q = 0; q < 6; ++q) P->h_order[RK_REG + q] = rl[q];
    P->n_p2 = (int)p2.size();
    P->n_bl = (int)bl.size();
    P->n_bf = (int)bf.size();
    P->maxM_p2 = maxp2;
    P->maxM_bl = maxbl;
    P->maxM_bf = maxbf;
    // twiddles for the Bluestein convolutions and for whole power-of-two rings (N = 4 sub)
    P->twn = std::max(std::max(2, maxreg), std::max(4 * maxp2, std::max(maxbl, maxbf)));
    // one chirp spectrum per distinct chirp length: N / 2 for the split rings, N for the whole-ring
    // ones (the two caps share them)
    std::vector<int> bL, bM;
    std::vector<int64_t> bO;
    int64_t btot = 0;
    {
        std::vector<int64_t> at(4 * (size_t)P->nside + 1, -1);
        auto key = [&](int r, int len) {
            RingInfo &ri = P->h_rings[r];
            if (at[len] < 0) {
                at[len] = btot;
                bL.push_back(len);
                bM.push_back(ri.M);
                bO.push_back(btot);
                btot += ri.M;
            }
            ri.bofs = at[len];
        };
        for (int r : bl) key(r, P->h_rings[r].nphi / 2);
        for (int r : bf) key(r, P->h_rings[r].nphi);
        for (int q = 2; q < 6; ++q)
            for (int r : rl[q]) key(r, q < 4 ? P->h_rings[r].nphi : P->h_rings[r].nphi / 2);
    }
    // the register engine's chirp spectra in register order, one per distinct transformed length
    // (lists 2 and 4 transform in 4096 points, 3 and 5 in 8192)
    std::vector<int64_t> rsrc[2], rdst[2];
    int64_t rtot = 0;
    {
        std::vector<int64_t> at(4 * (size_t)P->nside + 1, -1);
        for (int q = 2; q < 6; ++q)
            for (int r : rl[q]) {
                RingInfo &ri = P->h_rings[r];
                const int len = q < 4 ? ri.nphi : ri.nphi / 2;
                if (at[len] < 0) {
                    at[len] = rtot;
                    rsrc[(q & 1) ? 1 : 0].push_back(ri.bofs);
                    rdst[(q & 1) ? 1 : 0].push_back(rtot);
                    rtot += ri.M;
                }
                ri.rofs = at[len];
            }
    }

    // near-polar groups of FP32 plans: first pair of the group within theta_c of a pole
    P->ng64 = (P->npairs + 63) / 64;
    if (prec == AKRA_FP32) {
        const double theta_c = AKRA_DIFF_THETA;
        int g = 0;
        while (g < P->ng64 && std::acos(P->h_rings[64 * g].z) < theta_c) ++g;
        P->polar_groups = std::min(P->ng64, (g + 3) / 4 * 4);
        // blocks of four need some 8192 waves (8 per SIMD) to fill the device; fewer, and each wave's
        // long difference-form recurrence leaves the launch latency-bound: then one group per block
        P->adj_Rpol = (int64_t)((P->polar_groups + 3) / 4) * (lmax + 1) >= 8192 ? 4 : 1;
        P->adj_nrb_polar = (P->polar_groups + P->adj_Rpol - 1) / P->adj_Rpol;
    }

    // Legendre launch shapes
    P->syn_R = P->npairs >= 256 ? 2 : 1;
    P->syn_groups = (P->npairs + 64 * P->syn_R - 1) / (64 * P->syn_R);
    const int caps[5][2] = {{1, 1}, {1, 2}, {1, 4}, {2, 4}, {4, 4}};
    int ci = 4;
    for (int i = 0; i < 5; ++i)
        if (64 * caps[i][0] * caps[i][1] >= P->npairs) {
            ci = i;
            break;
        }
    P->adj_R = caps[ci][0];
    P->adj_W = caps[ci][1];
    P->adj_nrb = P->adj_nrb_polar + (P->ng64 - P->polar_groups + P->adj_R * P->adj_W - 1) / (P->adj_R * P->adj_W);
    P->syn_V1 = P->syn_V;
    P->syn_R1 = P->syn_R;
    P->adj_R1 = P->adj_R;
    P->adj_W1 = P->adj_W;
    P->adj_L1 = P->adj_L;

    akra_status st;
#define AK_TRY(x)                \
    do {                         \
        st = (x);                \
        if (st != AKRA_OK) {     \
            free_plan(P);        \
            return st;           \
        }                        \
    } while (0)

    // tables
    {
        std::vector<Coef64> c64;
        std::vector<Coef32> c32;
        std::vector<Coef32D> c32d;
        std::vector<Coef64S> c64s;
        std::vector<Coef32S> c32s;
        build_coef(lmax, c64, c32, c32d, c64s, c32s);
        AK_TRY(upload((void **)&P->d_coef64, c64.data(), c64.size() * sizeof(Coef64), *P));
        AK_TRY(upload((void **)&P->d_coef32, c32.data(), c32.size() * sizeof(Coef32), *P));
        AK_TRY(upload((void **)&P->d_coef64s, c64s.data(), c64s.size() * sizeof(Coef64S), *P));
        AK_TRY(upload((void **)&P->d_coef32s, c32s.data(), c32s.size() * sizeof(Coef32S), *P));
        AK_TRY(upload((void **)&P->d_coef32d, c32d.data(), c32d.size() * sizeof(Coef32D), *P));
    }
    {
        std::vector<double> s2, sm;
        std::vector<int> sk;
        build_seeds(*P, s2, sm, sk);
        AK_TRY(upload((void **)&P->d_seed2, s2.data(), s2.size() * sizeof(double), *P));
        AK_TRY(upload((void **)&P->d_seedm2, sm.data(), sm.size() * sizeof(double), *P));
        AK_TRY(upload((void **)&P->d_seedk, sk.data(), sk.size() * sizeof(int), *P));
    }
    {
        std::vector<double> pz(P->npairs);
        for (int p = 0; p < P->npairs; ++p) pz[p] = P->h_rings[p].z;
        AK_TRY(upload((void **)&P->d_pair_z, pz.data(), pz.size() * sizeof(double), *P));
        AK_TRY(upload((void **)&P->d_rings, P->h_rings.data(), P->h_rings.size() * sizeof(RingInfo), *P));
        AK_TRY(upload((void **)&P->d_order_p2, p2.data(), p2.size() * sizeof(int), *P));
        AK_TRY(upload((void **)&P->d_order_bl, bl.data(), bl.size() * sizeof(int), *P));
        AK_TRY(upload((void **)&P->d_order_bf, bf.data(), bf.size() * sizeof(int), *P));
        for (int q = 0; q < 6; ++q)
            if (!rl[q].empty()) AK_TRY(upload((void **)&P->d_order_r[q], rl[q].data(), rl[q].size() * sizeof(int), *P));
        P->rs_all.order[RK_P2] = P->d_order_p2;
        P->rs_all.order[RK_BF] = P->d_order_bf;
        P->rs_all.order[RK_BL] = P->d_order_bl;
        for (int q = 0; q < 6; ++q) P->rs_all.order[RK_REG + q] = P->d_order_r[q];
        for (int k = 0; k < RING_KINDS; ++k) P->rs_all.n[k] = (int)P->h_order[k].size();
        // every group in one list (the transforms without weights), polar groups first
        std::vector<int> ids(P->ng64);
        for (int g = 0; g < P->ng64; ++g) ids[g] = g;
        AK_TRY(upload((void **)&P->d_gl_all, ids.data(), ids.size() * sizeof(int), *P));
        GroupSet &A = P->gs_all;
        A.list[GCLS_BOTH] = A.list_any = P->d_gl_all;
        A.npol[GCLS_BOTH] = A.npol_any = P->polar_groups;
        A.nmain[GCLS_BOTH] = A.nmain_any = P->ng64 - P->polar_groups;
        // until a weight set-up, the weighted sets are the full ones
        P->rs_live = P->rs_all;
        P->rs_cls[0] = P->rs_all;  // every group counts as two-sided
        P->gs_live = P->gs_all;
        AK_TRY(alloc((void **)&P->d_live_lists, live_list_ints(*P) * sizeof(int), *P));
        AK_TRY(alloc((void **)&P->d_ring_live, (size_t)P->nrings, *P));
        if (hipHostMalloc((void **)&P->h_live, live_stage_bytes(*P)) != hipSuccess) {
            P->h_live = nullptr;
            free_plan(P);
            set_error("hipHostMalloc failed");
            return AKRA_ERR_ALLOC;
        }
    }
    // entry states of the recurrence (the seeds are only needed to build them)
    {
        const size_t nmp = (size_t)(lmax + 1) * P->npairs;
        AK_TRY(alloc((void **)&P->d_ent, nmp * sizeof(Ent64), *P));
        AK_TRY(alloc((void **)&P->d_entk, nmp * sizeof(int), *P));
        AK_TRY(alloc((void **)&P->d_entl, (size_t)(lmax + 1) * P->ng64 * sizeof(int), *P));
        launch_entry(*P);
        P->h_entl.resize((size_t)(lmax + 1) * P->ng64);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(P->stream) != hipSuccess ||
            hipMemcpy(P->h_entl.data(), P->d_entl, P->h_entl.size() * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
            free_plan(P);
            set_error("entry-state kernel failed");
            return AKRA_ERR_HIP;
        }
        for (void **q : {(void **)&P->d_seed2, (void **)&P->d_seedm2, (void **)&P->d_seedk}) {
            (void)hipFree(*q);
            *q = nullptr;
        }
        P->device_bytes -= (int64_t)nmp * (2 * sizeof(double) + sizeof(int));
    }
    {
        const int n = P->twn / 2;
        std::vector<double2> t64(n);
        std::vector<float2> t32(n);
        for (int k = 0; k < n; ++k) {
            long double a = -2.0L * 3.141592653589793238462643383279502884L * k / P->twn;
            t64[k] = make_double2((double)cosl(a), (double)sinl(a));
            t32[k] = make_float2((float)cosl(a), (float)sinl(a));
        }
        AK_TRY(upload(&P->d_tw64, t64.data(), n * sizeof(double2), *P));
        AK_TRY(upload(&P->d_tw32, t32.data(), n * sizeof(float2), *P));
    }
    if (!bL.empty()) {
        int *dL = nullptr, *dM = nullptr;
        int64_t *dO = nullptr;
        AK_TRY(alloc(&P->d_bhat64, (size_t)btot * sizeof(double2), *P));
        AK_TRY(alloc(&P->d_bhat32, (size_t)btot * sizeof(float2), *P));
        const size_t nb = bL.size();
        bool ok = hipMalloc((void **)&dL, nb * sizeof(int)) == hipSuccess &&
                  hipMalloc((void **)&dM, nb * sizeof(int)) == hipSuccess &&
                  hipMalloc((void **)&dO, nb * sizeof(int64_t)) == hipSuccess &&
                  hipMemcpy(dL, bL.data(), nb * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(dM, bM.data(), nb * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(dO, bO.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess;
        if (ok) {
            launch_bhat(*P, dL, dM, dO, (int)nb, std::max(std::max(P->maxM_bl, P->maxM_bf), maxreg));
            ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(P->stream) == hipSuccess;
        }
        for (void *q : {(void *)dL, (void *)dM, (void *)dO})
            if (q) (void)hipFree(q);
        if (!ok) {
            free_plan(P);
            set_error("chirp-spectrum kernel failed");
            return AKRA_ERR_HIP;
        }
    }
    if (rtot > 0) {
        AK_TRY(alloc(&P->d_bhatr64, (size_t)rtot * sizeof(double2), *P));
        AK_TRY(alloc(&P->d_bhatr32, (size_t)rtot * sizeof(float2), *P));
        bool ok = true;
        for (int q = 0; q < 2 && ok; ++q) {
            const size_t nb = rsrc[q].size();
            if (!nb) continue;
            int64_t *dS = nullptr, *dD = nullptr;
            ok = hipMalloc((void **)&dS, nb * sizeof(int64_t)) == hipSuccess &&
                 hipMalloc((void **)&dD, nb * sizeof(int64_t)) == hipSuccess &&
                 hipMemcpy(dS, rsrc[q].data(), nb * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(dD, rdst[q].data(), nb * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess;
            if (ok) {
                launch_bhat_reorder(*P, q ? 13 : 12, dS, dD, (int)nb);
                ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(P->stream) == hipSuccess;
            }
            for (void *d : {(void *)dS, (void *)dD})
                if (d) (void)hipFree(d);
        }
        if (!ok) {
            free_plan(P);
            set_error("chirp-spectrum reordering kernel failed");
            return AKRA_ERR_HIP;
        }
    }
    {
        std::vector<int> lof(P->nalm);
        for (int m = 0; m <= lmax; ++m)
            for (int l = m; l <= lmax; ++l) lof[(int64_t)m * (2 * lmax + 1 - m) / 2 + l] = l;
        AK_TRY(upload((void **)&P->d_lof, lof.data(), lof.size() * sizeof(int), *P));
        std::vector<double> kd, ones(lmax + 1, 1.0);
        default_kernel(lmax, kd);
        AK_TRY(upload((void **)&P->d_kern, kd.data(), kd.size() * sizeof(double), *P));
        AK_TRY(upload((void **)&P->d_kuser, ones.data(), ones.size() * sizeof(double), *P));
    }
    // workspaces
    const size_t fg = (size_t)nrhs * P->nrings * (lmax + 1) * 2 * sizeof(double2);
    AK_TRY(alloc(&P->d_FG, fg, *P));
    // the class lists of a weighted apply split the groups in up to three polar and three main parts,
    // each rounded up to whole blocks: at most LIVE_NRB_EXTRA blocks more than the unsplit layout
    P->part_rb_cap = (size_t)std::max(P->adj_nrb, P->adj_nrb_polar + (P->npairs <= 1024 ? P->ng64 : (P->ng64 + 3) / 4)) +
                     LIVE_NRB_EXTRA;
    if (prec == AKRA_FP32 && nrhs > 1) {
        // batched adjoint: blocks of four groups (polar blocks apart), 8 right-hand sides of FP32 slabs
        // ring blocks of bat_AW groups (polar blocks apart); room for the smallest supported bat_AW, 2
        P->nrb_b = (P->polar_groups + P->bat_AW - 1) / P->bat_AW + (P->ng64 - P->polar_groups + P->bat_AW - 1) / P->bat_AW;
        P->nrb_b_cap = (P->polar_groups + 1) / 2 + (P->ng64 - P->polar_groups + 1) / 2;
        P->part_rb_cap = std::max(P->part_rb_cap, (size_t)4 * P->nrb_b_cap);
        AK_TRY(alloc((void **)&P->d_wgstart_b, (size_t)P->nrb_b_cap * (lmax + 1) * sizeof(int), *P));
    }
    AK_TRY(alloc(&P->d_part, P->part_rb_cap * P->nalm * 4 * sizeof(double), *P));
    AK_TRY(alloc((void **)&P->d_wgstart, P->part_rb_cap * (lmax + 1) * sizeof(int), *P));
    compute_work(*P);
    // before any weight set-up every ring counts, in two-ring groups
    P->n_live_rings = P->nrings;
    P->work_live[0] = P->work[1];
    P->work_live[2] = P->work[2];
    P->work_live[4] = P->work_b;
    P->rec_stride = P->nalm + ALM_PAD;
    AK_TRY(alloc(&P->d_rec, (size_t)nrhs * P->rec_stride * 64, *P));
    if (prec == AKRA_FP32 && P->polar_groups > 0) {
        AK_TRY(alloc((void **)&P->d_recu, (size_t)nrhs * P->rec_stride * sizeof(float4), *P));
        if (hipMemset(P->d_recu, 0, (size_t)nrhs * P->rec_stride * sizeof(float4)) != hipSuccess) {
            free_plan(P);
            set_error("hipMemset failed");
            return AKRA_ERR_HIP;
        }
    }
    if (prec == AKRA_FP32 && nrhs > 1) AK_TRY(alloc((void **)&P->d_brec, (size_t)P->rec_stride * 8 * 4 * sizeof(float), *P));
    if (hipMemset(P->d_rec, 0, (size_t)nrhs * P->rec_stride * 64) != hipSuccess) {
        free_plan(P);
        set_error("hipMemset failed");
        return AKRA_ERR_HIP;
    }
    AK_TRY(alloc((void **)&P->d_W, (size_t)nrhs * P->npix * sizeof(double), *P));
    AK_TRY(alloc((void **)&P->d_red, (size_t)512 * 4 * nrhs * sizeof(double), *P));
    AK_TRY(alloc((void **)&P->d_red_cg, (size_t)2 * CG_RED_BLOCKS * nrhs * sizeof(double), *P));
    AK_TRY(alloc((void **)&P->d_scal, (size_t)(64 + 16 * nrhs) * sizeof(double), *P));
    AK_TRY(alloc((void **)&P->d_flag, 64 * sizeof(int), *P));
    // unmasked-pixel list scratch: count and flag, then per-tile counts and offsets
    P->cmp_ntile = (P->npix + CMP_TILE - 1) / CMP_TILE;
    {
        const size_t nt = (size_t)P->cmp_ntile, cnt_b = (nt * sizeof(int) + 255) / 256 * 256;
        AK_TRY(alloc(&P->d_cmp, 256 + cnt_b + nt * sizeof(int64_t), *P));
        char *b = (char *)P->d_cmp;
        P->d_cmp_nobs = (int64_t *)b;
        P->d_cmp_flag = (int *)(b + 64);
        P->d_cmp_cnt = (int *)(b + 256);
        P->d_cmp_offs = (int64_t *)(b + 256 + cnt_b);
        if (hipMemset(P->d_cmp, 0, 256) != hipSuccess) {
            free_plan(P);
            set_error("hipMemset failed");
            return AKRA_ERR_HIP;
        }
    }
    P->spec_nmc = (lmax + SPEC_MC) / SPEC_MC;
    AK_TRY(alloc((void **)&P->d_spec, (size_t)SPEC_NP * P->spec_nmc * (lmax + 1) * sizeof(double), *P));
    const size_t vb = (size_t)nrhs * 2 * P->nalm * sizeof(double2);
    AK_TRY(alloc((void **)&P->d_x, vb, *P));
    AK_TRY(alloc((void **)&P->d_r, vb, *P));
    AK_TRY(alloc((void **)&P->d_p, vb, *P));
    AK_TRY(alloc((void **)&P->d_w, vb, *P));
    AK_TRY(alloc((void **)&P->d_b, vb, *P));
    AK_TRY(alloc((void **)&P->d_xs, vb, *P));
    if (hipStreamCreateWithFlags(&P->side_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming) != hipSuccess) {
        free_plan(P);
        set_error("stream or event creation failed");
        return AKRA_ERR_HIP;
    }
    if (hipHostMalloc((void **)&P->h_pin, 256 * sizeof(double)) != hipSuccess) {
        P->h_pin = nullptr;
        free_plan(P);
        set_error("hipHostMalloc failed");
        return AKRA_ERR_ALLOC;
    }
#undef AK_TRY
    *out = P;
    return AKRA_OK;
}

// ---------------------------------------------------------------------------------------------
// operator pieces
// ---------------------------------------------------------------------------------------------
static bool plan_fp32(const Plan &P) { return P.prec == AKRA_FP32; }

static akra_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return AKRA_OK;
}

// W from ninv/mask, validated; returns lambda_eff and P for every rhs (host).  ninv holds ncount
// maps (0: one per right-hand side); right-hand side r takes map r mod ncount.
static akra_status setup_weights(Plan &P, const double *ninv, const uint8_t *mask, double lam, std::vector<double> &lam_eff,
                                 std::vector<double> &pc, std::vector<double> *msum = nullptr, int ncount = 0)
{
    if (!ninv || !mask) {
        set_error("ninv and mask must be device pointers");
        return AKRA_ERR_ARG;
    }
    launch_weights(P, ninv, mask, P.nrhs, ncount > 0 ? ncount : P.nrhs);
    launch_ring_live(P, P.nrhs);
    akra_status st = check_launch("weights");
    if (st) return st;
    AK_HIP(hipMemcpyAsync(P.h_pin, P.d_scal + 8, sizeof(double) * 4 * P.nrhs, hipMemcpyDeviceToHost, P.stream),
           "hipMemcpyAsync");
    AK_HIP(hipMemcpyAsync(P.h_live, P.d_ring_live, (size_t)P.nrings, hipMemcpyDeviceToHost, P.stream),
           "hipMemcpyAsync");
    AK_HIP(hipStreamSynchronize(P.stream), "hipStreamSynchronize");
    st = build_live_lists(P);
    if (st) return st;
    lam_eff.resize(P.nrhs);
    pc.resize(P.nrhs);
    if (msum) msum->resize(P.nrhs);
    for (int r = 0; r < P.nrhs; ++r) {
        const double sw = P.h_pin[4 * r], sm = P.h_pin[4 * r + 1], nonfin = P.h_pin[4 * r + 2], negs = P.h_pin[4 * r + 3];
        if (nonfin > 0) {
            set_error("ninv holds NaN or Inf");
            return AKRA_ERR_NUMERIC;
        }
        if (negs > 0) {
            set_error("ninv holds negative weights");
            return AKRA_ERR_ARG;
        }
        lam_eff[r] = (sm > 0) ? lam * sw / sm : 0.0;  // lambda <N^-1>_M
        if (msum) (*msum)[r] = sm;
        pc[r] = 1.0 / (sw / (double)P.npix + lam_eff[r]);  // (<M^2 N^-1> + lambda_eff)^-1
    }
    return AKRA_OK;
}

static akra_status kernel_to_device(Plan &P, const double *kernel_l, const double **kdev)
{
    if (!kernel_l) {
        *kdev = P.d_kern;
        return AKRA_OK;
    }
    // a caller-supplied kernel goes into the plan's second kernel table
    AK_HIP(hipMemcpyAsync(P.d_kuser, kernel_l, sizeof(double) * (P.lmax + 1), hipMemcpyHostToDevice, P.stream),
           "hipMemcpyAsync");
    *kdev = P.d_kuser;
    return AKRA_OK;
}

static double read_scalar(Plan &P, const double *dev, hipError_t *err)
{
    *err = hipMemcpyAsync(P.h_pin, dev, sizeof(double), hipMemcpyDeviceToHost, P.stream);
    if (*err == hipSuccess) *err = hipStreamSynchronize(P.stream);
    return P.h_pin[0];
}

__global__ void k_cg_beta(double *scal, double pc)
{
    // scal[3] = <r, r> (new), scal[0] = rz (old) -> scal[4] = beta, scal[0] = P <r, r>
    const double rz = pc * scal[3];
    scal[4] = (scal[0] > 0.0) ? rz / scal[0] : 0.0;
    scal[0] = rz;
}

__global__ void k_set(double *p, double v) { *p = v; }

// after a residual replacement: rz = P <r, r> for the next alpha; the search direction is kept
__global__ void k_cg_rz(double *scal, double pc) { scal[0] = pc * scal[3]; }

// ---- block systems (App. A) ---------------------------------------------------------------------
// Sets the unknowns of a solve for its duration; every apply, right-hand side and gradient formed
// meanwhile has the block of the held unknowns zeroed by the epilogue.
struct ProjScope {
    Plan &P;
    ProjScope(Plan &p, int mode) : P(p) { P.proj = mode; }
    ~ProjScope() { P.proj = 0; }
};

// zero the held block of an (E, B) pair of alm vectors (v: E at v, B at v + 2 nalm)
static akra_status zero_held(Plan &P, double *v)
{
    if (P.proj == 1) AK_HIP(hipMemsetAsync(v + 2 * P.nalm, 0, sizeof(double2) * P.nalm, P.stream), "memset");
    if (P.proj == 2) AK_HIP(hipMemsetAsync(v, 0, sizeof(double2) * P.nalm, P.stream), "memset");
    return AKRA_OK;
}

// ---- stage marks: trace ranges, and timing with HIP events on the plan stream ------------------
static const char *const k_stage_names[AKRA_NSTAGES] = {"akra.prologue", "akra.leg_synth", "akra.ring",
                                                         "akra.leg_adj", "akra.epilogue", "akra.cg_vec"};
static void stage_mark(Plan &P, int stage, bool begin)
{
    if (!P.capturing) {
        if (begin) roctxRangePushA(k_stage_names[stage]);
        else roctxRangePop();
    }
    if (!P.timing) return;
    if (begin) {
        if (P.ev_used == (int)P.ev_pool.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
            P.ev_pool.push_back({a, b});
            P.ev_stage.push_back(0);
        }
        P.ev_stage[P.ev_used] = stage;
        (void)hipEventRecord(P.ev_pool[P.ev_used][0], P.stream);
    } else {
        (void)hipEventRecord(P.ev_pool[P.ev_used][1], P.stream);
        P.ev_used++;
    }
}

// w = H p style apply with timing marks; W of right-hand side `rhs` must be in P.d_W.  With dot_red,
// the epilogue also leaves the partials of <x, y>.
static akra_status apply_H_timed(Plan &P, bool fp32, const double *kern_dev, double lam, const double *xE,
                                 const double *xB, double *yE, double *yB, int rhs, double *dot_red = nullptr)
{
    stage_mark(P, 0, true);
    launch_prologue(P, fp32, xE, xB, kern_dev, 1);
    stage_mark(P, 0, false);
    const GroupSet &G = P.gs_live;
    const bool two = G.npol[GCLS_BOTH] + G.nmain[GCLS_BOTH] > 0,
               one = G.npol[GCLS_NORTH] + G.nmain[GCLS_NORTH] + G.npol[GCLS_SOUTH] + G.nmain[GCLS_SOUTH] > 0;
    if (!P.timing && P.skip_rings && P.side_stream && two && one) {
        // untimed: one chain per class of ring groups (stage times need the staged order below)
        launch_weighted_chains(P, fp32, P.d_W + (int64_t)rhs * P.npix);
        launch_epilogue(P, fp32, kern_dev, lam, xE, xB, yE, yB, dot_red);
        return check_launch("apply_H");
    }
    stage_mark(P, 1, true);
    launch_leg_synth(P, fp32, 1, true);
    stage_mark(P, 1, false);
    stage_mark(P, 2, true);
    launch_ring(P, fp32, 2, nullptr, nullptr, nullptr, nullptr, P.d_W + (int64_t)rhs * P.npix, 1, true);
    stage_mark(P, 2, false);
    stage_mark(P, 3, true);
    launch_leg_adj(P, fp32, 0, true);
    stage_mark(P, 3, false);
    stage_mark(P, 4, true);
    launch_epilogue(P, fp32, kern_dev, lam, xE, xB, yE, yB, dot_red);
    stage_mark(P, 4, false);
    return check_launch("apply_H");
}

// H applied to all right-hand sides of an FP32 plan at once: batched matrix-core synthesis, ring
// stage of every right-hand side with its own W, then per group of 8 right-hand sides the batched
// matrix-core adjoint and the epilogue of each.  lam_host (per rhs) overrides lam when given.
// With dot_red, right-hand side r's epilogue also leaves the partials of <x_r, y_r> at
// dot_red + r 2 CG_RED_BLOCKS.
static akra_status apply_H_batched(Plan &P, const double *kern_dev, const double *lam_host, double lam,
                                   const double *xE, const double *xB, double *yE, double *yB, int64_t rstride,
                                   double *dot_red = nullptr)
{
    stage_mark(P, 1, true);
    launch_synth_batched(P, xE, xB, rstride, kern_dev, true);
    stage_mark(P, 1, false);
    stage_mark(P, 2, true);
    launch_ring(P, true, 2, nullptr, nullptr, nullptr, nullptr, P.d_W, P.nrhs, true);
    stage_mark(P, 2, false);
    for (int q = 0; q * 8 < P.nrhs; ++q) {
        stage_mark(P, 3, true);
        launch_adj_batched(P, q, true);
        stage_mark(P, 3, false);
        for (int r = 8 * q; r < P.nrhs && r < 8 * q + 8; ++r) {
            const int64_t o = (int64_t)r * 2 * rstride;
            stage_mark(P, 4, true);
            launch_epilogue_batched(P, r, kern_dev, lam_host ? lam_host[r] : lam, xE + o, xB + o, yE + o, yB + o,
                                    dot_red ? dot_red + (int64_t)r * 2 * CG_RED_BLOCKS : nullptr);
            stage_mark(P, 4, false);
        }
    }
    return check_launch("apply_H_batched");
}

static akra_status true_residual(Plan &P, double *rdst)
{
    const int64_t nc = 2 * P.nalm;
    double *x = P.d_x, *w = P.d_w;
    akra_status st = apply_H_timed(P, false, P.cg_kern, P.cg_lam, x, x + 2 * P.nalm, w, w + 2 * P.nalm, P.cg_rhs);
    if (st) return st;
    P.cg_fp64_applies++;
    AK_HIP(hipMemcpyAsync(rdst, P.d_b, sizeof(double2) * nc, hipMemcpyDeviceToDevice, P.stream), "copy");
    launch_axpby(P, rdst, -1.0, w, 1.0, nc);
    return AKRA_OK;
}

// Initialise PCG on the right-hand side already in P.d_b (x0 in P.d_x when use_x0):
//   r0 = b - H x0, p0 = P r0, rz0 = P <r0, r0>.  One host synchronisation (||b||, ||r0||).
static akra_status cg_begin(Plan &P, bool use_x0)
{
    const int64_t nc = 2 * P.nalm;
    hipError_t he;
    P.cg_ready = false;
    P.cg_iters = 0;
    P.cg_fp64_applies = 0;
    launch_dot(P, P.d_b, P.d_b, P.d_scal + 5, nc);
    const double bn2 = read_scalar(P, P.d_scal + 5, &he);
    if (he != hipSuccess) return hip_fail(he, "cg");
    if (!std::isfinite(bn2)) {
        set_error("right-hand side is not finite");
        return AKRA_ERR_NUMERIC;
    }
    P.cg_bn = std::sqrt(bn2);
    if (use_x0) {
        akra_status st = true_residual(P, P.d_r);
        if (st) return st;
    } else {
        AK_HIP(hipMemsetAsync(P.d_x, 0, sizeof(double2) * nc, P.stream), "memset");
        AK_HIP(hipMemcpyAsync(P.d_r, P.d_b, sizeof(double2) * nc, hipMemcpyDeviceToDevice, P.stream), "copy");
    }
    AK_HIP(hipMemsetAsync(P.d_flag, 0, sizeof(int), P.stream), "memset");
    launch_dot(P, P.d_r, P.d_r, P.d_scal + 3, nc);
    AK_HIP(hipMemsetAsync(P.d_p, 0, sizeof(double2) * nc, P.stream), "memset");
    k_set<<<1, 1, 0, P.stream>>>(P.d_scal + 0, 0.0);
    k_cg_beta<<<1, 1, 0, P.stream>>>(P.d_scal, P.cg_pc);
    k_set<<<1, 1, 0, P.stream>>>(P.d_scal + 4, 0.0);
    launch_cg_p(P, P.d_p, P.d_r, P.d_scal + 4, P.cg_pc, nc);
    const double rr = read_scalar(P, P.d_scal + 3, &he);
    if (he != hipSuccess) return hip_fail(he, "cg");
    P.cg_rr = rr;
    P.cg_ready = true;
    return check_launch("cg_begin");
}

// One PCG iteration on device-resident state, no host synchronisation:
//   w = H p, alpha = rz / <p, w>, x += alpha p, r -= alpha w, rr = <r, r>,
//   beta = P rr / rz, p = P r + beta p.
// The inner products ride on the kernels that already stream the vectors: the epilogue forms the
// partials of <p, w> as it writes w, the x/r update those of <r, r> as it writes r; each workgroup
// of the x/r update (of the p update) sums the <p, w> (<r, r>) partials in the same fixed order and
// forms alpha (beta) itself.
static akra_status cg_iterate(Plan &P, bool fp32)
{
    const int64_t nc = 2 * P.nalm;
    double *x = P.d_x, *r = P.d_r, *p = P.d_p, *w = P.d_w;
    double *red_pw = P.d_red_cg, *red_rr = P.d_red_cg + CG_RED_BLOCKS;
    akra_status st =
        apply_H_timed(P, fp32, P.cg_kern, P.cg_lam, p, p + 2 * P.nalm, w, w + 2 * P.nalm, P.cg_rhs, red_pw);
    if (st) return st;
    stage_mark(P, 5, true);
    launch_cg_xr_alpha(P, x, r, p, w, red_pw, P.d_scal, P.d_flag, nc, red_rr);
    launch_cg_p_beta(P, p, r, red_rr, P.d_scal, P.cg_pc, nc);
    stage_mark(P, 5, false);
    P.cg_iters++;
    return check_launch("cg_step");
}

// Every value the launches of one iteration take by value, besides plan-constant pointers and
// sizes: precision, right-hand side, projection, lambda_eff, P, the K_l table and the Legendre
// launch shapes.  A recorded iteration is valid while these are unchanged.
static void iter_key(const Plan &P, bool fp32, double *k)
{
    const double v[ITER_KEY_N] = {(double)fp32, (double)P.cg_rhs, (double)P.proj, P.cg_lam, P.cg_pc,
                                  (double)(uintptr_t)P.cg_kern, (double)P.syn_V, (double)P.syn_R, (double)P.adj_R,
                                  (double)P.adj_W, (double)P.adj_L, (double)P.adj_nrb, (double)P.live_gen,
                                  (double)P.syn_V1, (double)P.syn_R1, (double)P.adj_R1, (double)P.adj_W1,
                                  (double)P.adj_L1};
    std::memcpy(k, v, sizeof v);
}

static void drop_graph(Plan &P)
{
    if (P.cg_graph) (void)hipGraphExecDestroy(P.cg_graph);
    P.cg_graph = nullptr;
    if (P.cg_graph_b) (void)hipGraphExecDestroy(P.cg_graph_b);
    P.cg_graph_b = nullptr;
    P.cg_graph_b_key.clear();
}

// Records the launches of fn() into exec: they go to the private capture stream (the plan stream
// may be the legacy default stream, which cannot be captured).  Nothing executes here.
template <class Fn> static akra_status record_graph(Plan &P, hipGraphExec_t &exec, Fn &&fn)
{
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    if (!P.cap_stream) AK_HIP(hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    AK_HIP(hipGetLastError(), "launch");
    const hipStream_t s = P.stream;
    AK_HIP(hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    P.stream = P.cap_stream;
    P.capturing = true;
    akra_status st = fn();
    P.capturing = false;
    P.stream = s;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(P.cap_stream, &g);
    if (st == AKRA_OK && e != hipSuccess) st = hip_fail(e, "hipStreamEndCapture");
    if (st == AKRA_OK) {
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            exec = nullptr;
            st = hip_fail(e, "hipGraphInstantiate");
        }
    }
    if (g) (void)hipGraphDestroy(g);
    return st;
}

// Records one cg_iterate (the iteration count is not advanced by the recording)
static akra_status record_iteration(Plan &P, bool fp32)
{
    const int iters = P.cg_iters;
    akra_status st = record_graph(P, P.cg_graph, [&]() { return cg_iterate(P, fp32); });
    P.cg_iters = iters;
    if (st == AKRA_OK) iter_key(P, fp32, P.cg_graph_key);
    return st;
}

// One PCG iteration: a replay of the recorded graph (recorded again when a by-value argument has
// changed), or direct launches when stage timing is on or graphs are switched off.
static akra_status cg_step1(Plan &P, bool fp32)
{
    if (P.timing || !P.use_graph) return cg_iterate(P, fp32);
    double k[ITER_KEY_N];
    iter_key(P, fp32, k);
    if (!P.cg_graph || std::memcmp(k, P.cg_graph_key, sizeof k) != 0) {
        akra_status st = record_iteration(P, fp32);
        if (st) return st;
    }
    TraceRange tr("akra.cg_iteration_graph");
    AK_HIP(hipGraphLaunch(P.cg_graph, P.stream), "hipGraphLaunch");
    P.cg_iters++;
    return AKRA_OK;
}

// host view of <r, r> and the breakdown flag (one synchronisation)
static akra_status cg_poll(Plan &P, double *rr, int *flag)
{
    AK_HIP(hipMemcpyAsync(P.h_pin, P.d_scal + 3, sizeof(double), hipMemcpyDeviceToHost, P.stream), "copy");
    AK_HIP(hipMemcpyAsync(P.h_pin + 1, P.d_flag, sizeof(int), hipMemcpyDeviceToHost, P.stream), "copy");
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    *rr = P.h_pin[0];
    std::memcpy(flag, P.h_pin + 1, sizeof(int));
    return AKRA_OK;
}

// Full solve on the state prepared by cg_begin.  FP32 plans iterate with the FP32 operator and
// replace the recursive residual by the FP64 true residual whenever it has dropped by
// reliable_delta since the last replacement (reliable updates); convergence is only accepted
// on a true residual.  The search direction is kept across replacements.  If the FP32 operator
// can no longer resolve a search direction (p^T H p <= 0 near the tolerance of an ill-conditioned
// system) the solve restarts from the true residual and finishes with the FP64 operator.
static akra_status cg_run(Plan &P, const akra_cg_opts &o, akra_cg_info *info)
{
    const int64_t nc = 2 * P.nalm;
    bool fp32 = P.prec == AKRA_FP32;
    hipError_t he;
    info->lambda_eff = P.cg_lam;
    info->precond = P.cg_pc;
    if (P.cg_bn == 0.0) {
        info->iters = 0;
        info->rel_resid = info->rel_resid_true = 0.0;
        return AKRA_OK;
    }
    const double bn = P.cg_bn;
    double rr = P.cg_rr, rel = std::sqrt(rr) / bn, rmax = std::sqrt(rr);
    bool fresh = true;
    akra_status result = AKRA_NOT_CONVERGED;
    StallWatch stall(o.stall_iters, rel);
    auto refresh = [&]() -> akra_status {
        akra_status s2 = true_residual(P, P.d_r);
        if (s2) return s2;
        launch_dot(P, P.d_r, P.d_r, P.d_scal + 3, nc);
        rr = read_scalar(P, P.d_scal + 3, &he);
        if (he != hipSuccess) return hip_fail(he, "cg");
        rel = std::sqrt(rr) / bn;
        rmax = std::sqrt(rr);
        fresh = true;
        return AKRA_OK;
    };
    while (true) {
        if (rel < o.tol) {
            if (!fp32 || fresh) {
                result = AKRA_OK;
                break;
            }
            akra_status st = refresh();
            if (st) return st;
            if (rel < o.tol) {
                result = AKRA_OK;
                break;
            }
            // continue from the true residual with the kept direction
            k_cg_rz<<<1, 1, 0, P.stream>>>(P.d_scal, P.cg_pc);
        }
        if (P.cg_iters >= o.maxiter) break;
        const int nb = std::min(o.check_every > 1 ? o.check_every : 1, o.maxiter - P.cg_iters);
        akra_status st = AKRA_OK;
        for (int b = 0; b < nb; ++b) {
            st = cg_step1(P, fp32);
            if (st) return st;
            if (!fp32 && P.prec == AKRA_FP32) P.cg_fp64_applies++;
        }
        int flag = 0;
        st = cg_poll(P, &rr, &flag);
        if (st) return st;
        fresh = false;
        if ((flag || !std::isfinite(rr)) && fp32) {
            // x is the last iterate (alpha was set to 0): restart p = P r from the true residual
            fp32 = false;
            AK_HIP(hipMemsetAsync(P.d_flag, 0, sizeof(int), P.stream), "memset");
            st = refresh();
            if (st) return st;
            k_set<<<1, 1, 0, P.stream>>>(P.d_scal + 4, 0.0);
            launch_cg_p(P, P.d_p, P.d_r, P.d_scal + 4, P.cg_pc, nc);
            k_cg_rz<<<1, 1, 0, P.stream>>>(P.d_scal, P.cg_pc);
            continue;
        }
        if ((flag || !std::isfinite(rr)) && P.prec == AKRA_FP32) {
            // the FP64 iterations of an FP32 plan stalled too: tol is below the attainable accuracy
            // of the system; x is the last iterate
            AK_HIP(hipMemsetAsync(P.d_flag, 0, sizeof(int), P.stream), "memset");
            set_error("CG stalled below the attainable accuracy (p^T H p <= 0 after the FP64 restart)");
            break;
        }
        if (flag || !std::isfinite(rr)) {
            set_error("CG breakdown: p^T H p <= 0 or non-finite scalar");
            info->iters = P.cg_iters;
            return AKRA_ERR_NUMERIC;
        }
        rel = std::sqrt(rr) / bn;
        if (o.resid_hist && P.cg_iters - 1 < o.resid_hist_len) o.resid_hist[P.cg_iters - 1] = rel;
        if (rel >= o.tol && stall.step(rel)) {
            result = AKRA_STAGNATED;
            set_error("CG stagnated: no new smallest residual in stall_iters iterations");
            break;
        }
        if (fp32 && std::sqrt(rr) < o.reliable_delta * rmax && rel >= o.tol) {
            st = refresh();
            if (st) return st;
            k_cg_rz<<<1, 1, 0, P.stream>>>(P.d_scal, P.cg_pc);
        }
    }
    info->iters = P.cg_iters;
    info->rel_resid = rel;
    {
        akra_status st = true_residual(P, P.d_xs);
        if (st) return st;
        launch_dot(P, P.d_xs, P.d_xs, P.d_scal + 6, nc);
        const double tr = read_scalar(P, P.d_scal + 6, &he);
        if (he != hipSuccess) return hip_fail(he, "cg");
        info->rel_resid_true = std::sqrt(tr) / bn;
    }
    info->fp64_applies = P.cg_fp64_applies;
    if (result == AKRA_NOT_CONVERGED && P.cg_iters >= o.maxiter) set_error("maxiter reached");
    return result;
}

}  // namespace akra

using namespace akra;

// =================================================================================================
// C ABI
// =================================================================================================
extern "C" {

struct akra_plan_s {
    Plan *P;
};

const char *akra_last_error(void) { return g_err.c_str(); }

void akra_cg_opts_default(akra_cg_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->lambda = 1e-3;
    o->tol = 1e-3;
    o->maxiter = 1000;
    o->use_x0 = 0;
    o->kernel_l = nullptr;
    o->reliable_delta = 0.1;
}

akra_status akra_plan_create(int nside, int lmax, int nrhs, int precision, void *hip_stream, akra_plan *out)
{
    TraceRange trace_range("akra_plan_create");
    if (!out) {
        set_error("out is NULL");
        return AKRA_ERR_ARG;
    }
    *out = nullptr;
    Plan *P = nullptr;
    akra_status st;
    try {
        st = create(nside, lmax, nrhs, precision, hip_stream, &P);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return AKRA_ERR_ALLOC;
    }
    if (st != AKRA_OK) return st;
    *out = new akra_plan_s{P};
    return AKRA_OK;
}

void akra_plan_destroy(akra_plan plan)
{
    if (!plan) return;
    (void)hipStreamSynchronize(plan->P->stream);
    free_plan(plan->P);
    delete plan;
}

int64_t akra_plan_device_bytes(akra_plan plan) { return plan ? plan->P->device_bytes : 0; }

#define AK_PLAN()                          \
    if (!plan) {                           \
        set_error("plan is NULL");         \
        return AKRA_ERR_ARG;               \
    }                                      \
    Plan &P = *plan->P

akra_status akra_synth2(akra_plan plan, const double *almE, const double *almB, double *g1, double *g2)
{
    TraceRange trace_range("akra_synth2");
    AK_PLAN();
    if (!almE || !almB || !g1 || !g2) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    const bool fp32 = plan_fp32(P);
    if (fp32 && P.nrhs > 1) {
        launch_synth_batched(P, almE, almB, P.nalm, nullptr, false);
    } else {
        launch_prologue(P, fp32, almE, almB, nullptr, P.nrhs);
        launch_leg_synth(P, fp32, P.nrhs, false);
    }
    launch_ring(P, fp32, 0, nullptr, nullptr, g1, g2, nullptr, P.nrhs, false);
    return check_launch("synth2");
}

akra_status akra_adjoint2(akra_plan plan, const double *g1, const double *g2, double *almE, double *almB)
{
    TraceRange trace_range("akra_adjoint2");
    AK_PLAN();
    if (!almE || !almB || !g1 || !g2) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    const bool fp32 = plan_fp32(P);
    launch_ring(P, fp32, 1, g1, g2, nullptr, nullptr, nullptr, P.nrhs, false);
    for (int r = 0; r < P.nrhs; ++r) {
        launch_leg_adj(P, fp32, r, false);
        launch_epilogue(P, fp32, nullptr, 0.0, nullptr, nullptr, almE + (int64_t)r * 2 * P.nalm,
                        almB + (int64_t)r * 2 * P.nalm);
    }
    return check_launch("adjoint2");
}

akra_status akra_apply_H(akra_plan plan, const double *ninv, const uint8_t *mask, const double *kernel_l,
                         double lambda_eff, const double *xE, const double *xB, double *yE, double *yB)
{
    TraceRange trace_range("akra_apply_H");
    AK_PLAN();
    if (!xE || !xB || !yE || !yB) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    std::vector<double> le, pc;
    akra_status st = setup_weights(P, ninv, mask, 0.0, le, pc);
    if (st) return st;
    const double *kd;
    st = kernel_to_device(P, kernel_l, &kd);
    if (st) return st;
    const bool fp32 = plan_fp32(P);
    if (fp32 && P.nrhs > 1) return apply_H_batched(P, kd, nullptr, lambda_eff, xE, xB, yE, yB, P.nalm);
    for (int r = 0; r < P.nrhs; ++r) {
        const int64_t o = (int64_t)r * 2 * P.nalm;
        st = apply_H_timed(P, fp32, kd, lambda_eff, xE + o, xB + o, yE + o, yB + o, r);
        if (st) return st;
    }
    return AKRA_OK;
}

static akra_status rhs_core(Plan &P, const double *g1, const double *g2, const double *kd, double *bE, double *bB)
{
    const bool fp32 = plan_fp32(P);
    // W gamma_obs, adjoint ring stage in the plan precision would lose FP64 accuracy of b for the
    // refined solve: the right-hand side is always formed in FP64.
    (void)fp32;
    launch_ring(P, false, 1, g1, g2, nullptr, nullptr, P.d_W, P.nrhs, true);
    for (int r = 0; r < P.nrhs; ++r) {
        launch_leg_adj(P, false, r, true);
        launch_epilogue(P, false, kd, 0.0, nullptr, nullptr, bE + (int64_t)r * 2 * P.nalm, bB + (int64_t)r * 2 * P.nalm);
    }
    return check_launch("rhs");
}

akra_status akra_rhs(akra_plan plan, const double *g1, const double *g2, const double *ninv, const uint8_t *mask,
                     const double *kernel_l, double *bE, double *bB)
{
    TraceRange trace_range("akra_rhs");
    AK_PLAN();
    if (!g1 || !g2 || !bE || !bB) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    std::vector<double> le, pc;
    akra_status st = setup_weights(P, ninv, mask, 0.0, le, pc);
    if (st) return st;
    const double *kd;
    st = kernel_to_device(P, kernel_l, &kd);
    if (st) return st;
    return rhs_core(P, g1, g2, kd, bE, bB);
}

// Load right-hand side `r` (from maps, or given b) and x0 into the solver state and run cg_begin.
static akra_status cg_prepare(Plan &P, const double *g1, const double *g2, const double *bE, const double *bB,
                              const double *xE, const double *xB, const akra_cg_opts &o, const double *kd,
                              const std::vector<double> &le, const std::vector<double> &pc, int r)
{
    const int64_t off = (int64_t)r * 2 * P.nalm;
    P.cg_kern = kd;
    P.cg_lam = le[r];
    P.cg_pc = pc[r];
    P.cg_rhs = r;
    if (g1) {
        launch_ring(P, false, 1, g1 + r * P.npix, g2 + r * P.npix, nullptr, nullptr, P.d_W + r * P.npix, 1, true);
        launch_leg_adj(P, false, 0, true);
        launch_epilogue(P, false, kd, 0.0, nullptr, nullptr, P.d_b, P.d_b + 2 * P.nalm);
    } else {
        AK_HIP(hipMemcpyAsync(P.d_b, bE + off, sizeof(double2) * P.nalm, hipMemcpyDeviceToDevice, P.stream), "copy");
        AK_HIP(hipMemcpyAsync(P.d_b + 2 * P.nalm, bB + off, sizeof(double2) * P.nalm, hipMemcpyDeviceToDevice,
                              P.stream),
               "copy");
    }
    akra_status st = zero_held(P, P.d_b);
    if (st) return st;
    if (o.use_x0) {
        AK_HIP(hipMemcpyAsync(P.d_x, xE + off, sizeof(double2) * P.nalm, hipMemcpyDeviceToDevice, P.stream), "copy");
        AK_HIP(hipMemcpyAsync(P.d_x + 2 * P.nalm, xB + off, sizeof(double2) * P.nalm, hipMemcpyDeviceToDevice,
                              P.stream),
               "copy");
        st = zero_held(P, P.d_x);
        if (st) return st;
    }
    return cg_begin(P, o.use_x0 != 0);
}

static akra_status read_opts(const akra_cg_opts *opts, akra_cg_opts &o)
{
    akra_cg_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.tol > 0) || o.maxiter < 0 || !(o.lambda >= 0) || !(o.reliable_delta > 0 && o.reliable_delta < 1) ||
        o.mode < AKRA_JOINT_EB || o.mode > AKRA_B_ONLY || o.stall_iters < 0 || o.check_every < 0) {
        set_error("invalid solver options");
        return AKRA_ERR_ARG;
    }
    return AKRA_OK;
}

// Lockstep PCG of all right-hand sides of an FP32 plan with nrhs > 1: one batched operator apply per
// iteration (matrix-core synthesis shared by all right-hand sides), per-right-hand-side scalars on
// the device, reliable updates and convergence tests per right-hand side.  A right-hand side that
// has converged keeps its iterate and takes no further updates.
static akra_status solve_batched(Plan &P, const double *g1, const double *g2, const double *bE, const double *bB,
                                 const akra_cg_opts &o, const double *kd, const std::vector<double> &le,
                                 const std::vector<double> &pc, double *xE, double *xB, akra_cg_info &info)
{
    const int nr = P.nrhs;
    const int64_t na = P.nalm, nc = 2 * na;
    hipError_t he;
    auto V = [&](double *base, int r) { return base + (int64_t)r * 2 * nc; };  // [rhs][E, B][nalm] complex
    double *scb = P.d_scal + 16 + 4 * nr;
    auto S = [&](int r) { return scb + 8 * r; };
    // right-hand sides (FP64) and starting residuals
    for (int r = 0; r < nr; ++r) {
        const int64_t off = (int64_t)r * 2 * na;
        if (g1) {
            launch_ring(P, false, 1, g1 + r * P.npix, g2 + r * P.npix, nullptr, nullptr, P.d_W + r * P.npix, 1, true);
            launch_leg_adj(P, false, 0, true);
            launch_epilogue(P, false, kd, 0.0, nullptr, nullptr, V(P.d_b, r), V(P.d_b, r) + 2 * na);
        } else {
            AK_HIP(hipMemcpyAsync(V(P.d_b, r), bE + off, sizeof(double2) * na, hipMemcpyDeviceToDevice, P.stream), "copy");
            AK_HIP(hipMemcpyAsync(V(P.d_b, r) + 2 * na, bB + off, sizeof(double2) * na, hipMemcpyDeviceToDevice,
                                  P.stream),
                   "copy");
        }
        akra_status s0 = zero_held(P, V(P.d_b, r));
        if (s0) return s0;
        if (o.use_x0) {
            AK_HIP(hipMemcpyAsync(V(P.d_x, r), xE + off, sizeof(double2) * na, hipMemcpyDeviceToDevice, P.stream), "copy");
            AK_HIP(hipMemcpyAsync(V(P.d_x, r) + 2 * na, xB + off, sizeof(double2) * na, hipMemcpyDeviceToDevice,
                                  P.stream),
                   "copy");
            s0 = zero_held(P, V(P.d_x, r));
            if (s0) return s0;
        } else {
            AK_HIP(hipMemsetAsync(V(P.d_x, r), 0, sizeof(double2) * nc, P.stream), "memset");
        }
    }
    // true residual of right-hand side r (FP64 apply): r_r = b_r - H x_r
    auto true_res = [&](int r, double *dst) -> akra_status {
        akra_status s2 = apply_H_timed(P, false, kd, le[r], V(P.d_x, r), V(P.d_x, r) + 2 * na, V(P.d_w, r),
                                       V(P.d_w, r) + 2 * na, r);
        if (s2) return s2;
        P.cg_fp64_applies++;
        AK_HIP(hipMemcpyAsync(dst, V(P.d_b, r), sizeof(double2) * nc, hipMemcpyDeviceToDevice, P.stream), "copy");
        launch_axpby(P, dst, -1.0, V(P.d_w, r), 1.0, nc);
        return AKRA_OK;
    };
    std::vector<double> bn(nr), rel(nr), rmax(nr), rr(nr);
    std::vector<char> active(nr, 1), fresh(nr, 1), restarted(nr, 0);
    std::vector<int> status(nr, AKRA_NOT_CONVERGED);
    std::vector<StallWatch> stall(nr);
    P.cg_fp64_applies = 0;
    AK_HIP(hipMemsetAsync(P.d_flag, 0, sizeof(int) * nr, P.stream), "memset");
    for (int r = 0; r < nr; ++r) {
        launch_dot(P, V(P.d_b, r), V(P.d_b, r), S(r) + 5, nc);
        if (o.use_x0) {
            akra_status st = true_res(r, V(P.d_r, r));
            if (st) return st;
        } else {
            AK_HIP(hipMemcpyAsync(V(P.d_r, r), V(P.d_b, r), sizeof(double2) * nc, hipMemcpyDeviceToDevice, P.stream),
                   "copy");
        }
        launch_dot(P, V(P.d_r, r), V(P.d_r, r), S(r) + 3, nc);
        k_set<<<1, 1, 0, P.stream>>>(S(r) + 0, 0.0);
        k_cg_beta<<<1, 1, 0, P.stream>>>(S(r), pc[r]);
        k_set<<<1, 1, 0, P.stream>>>(S(r) + 4, 0.0);
        AK_HIP(hipMemsetAsync(V(P.d_p, r), 0, sizeof(double2) * nc, P.stream), "memset");
        launch_cg_p(P, V(P.d_p, r), V(P.d_r, r), S(r) + 4, pc[r], nc);
    }
    std::vector<double> hs(8 * nr);
    std::vector<int> hf(nr);
    auto pull = [&]() -> akra_status {
        AK_HIP(hipMemcpyAsync(hs.data(), scb, sizeof(double) * 8 * nr, hipMemcpyDeviceToHost, P.stream), "copy");
        AK_HIP(hipMemcpyAsync(hf.data(), P.d_flag, sizeof(int) * nr, hipMemcpyDeviceToHost, P.stream), "copy");
        AK_HIP(hipStreamSynchronize(P.stream), "sync");
        return AKRA_OK;
    };
    akra_status st = pull();
    if (st) return st;
    for (int r = 0; r < nr; ++r) {
        if (!std::isfinite(hs[8 * r + 5])) {
            set_error("right-hand side is not finite");
            return AKRA_ERR_NUMERIC;
        }
        bn[r] = std::sqrt(hs[8 * r + 5]);
        rr[r] = hs[8 * r + 3];
        rel[r] = bn[r] > 0 ? std::sqrt(rr[r]) / bn[r] : 0.0;
        rmax[r] = std::sqrt(rr[r]);
        stall[r] = StallWatch(o.stall_iters, rel[r]);
        if (bn[r] == 0.0) {
            active[r] = 0;
            status[r] = AKRA_OK;
        }
    }
    auto refresh = [&](int r) -> akra_status {
        akra_status s2 = true_res(r, V(P.d_r, r));
        if (s2) return s2;
        launch_dot(P, V(P.d_r, r), V(P.d_r, r), S(r) + 3, nc);
        rr[r] = read_scalar(P, S(r) + 3, &he);
        if (he != hipSuccess) return hip_fail(he, "cg");
        rel[r] = std::sqrt(rr[r]) / bn[r];
        rmax[r] = std::sqrt(rr[r]);
        fresh[r] = 1;
        return AKRA_OK;
    };
    int iters = 0;
    while (true) {
        // convergence (accepted on a true residual)
        for (int r = 0; r < nr; ++r) {
            if (!active[r] || rel[r] >= o.tol) continue;
            if (!fresh[r]) {
                st = refresh(r);
                if (st) return st;
                if (rel[r] >= o.tol) {
                    k_cg_rz<<<1, 1, 0, P.stream>>>(S(r), pc[r]);
                    continue;
                }
            }
            active[r] = 0;
            status[r] = AKRA_OK;
        }
        bool any = false;
        for (int r = 0; r < nr; ++r) any |= active[r] != 0;
        if (!any || iters >= o.maxiter) break;
        // one lockstep iteration: the batched apply, then the updates of the active right-hand sides
        auto iterate = [&]() -> akra_status {
            akra_status s2 = apply_H_batched(P, kd, le.data(), 0.0, P.d_p, P.d_p + 2 * na, P.d_w, P.d_w + 2 * na,
                                             2 * na, P.d_red_cg);
            if (s2) return s2;
            for (int r = 0; r < nr; ++r) {
                if (!active[r]) continue;
                // the epilogue left the partials of <p, w>; the update leaves those of <r, r>
                double *red_pw = P.d_red_cg + (int64_t)r * 2 * CG_RED_BLOCKS, *red_rr = red_pw + CG_RED_BLOCKS;
                stage_mark(P, 5, true);
                launch_cg_alpha_sum(P, red_pw, S(r), P.d_flag + r);
                launch_cg_xr_rr(P, V(P.d_x, r), V(P.d_r, r), V(P.d_p, r), V(P.d_w, r), S(r) + 2, nc, red_rr);
                launch_cg_beta_sum(P, red_rr, S(r), pc[r]);
                launch_cg_p(P, V(P.d_p, r), V(P.d_r, r), S(r) + 4, pc[r], nc);
                stage_mark(P, 5, false);
            }
            return check_launch("cg_batched");
        };
        if (P.timing || !P.use_graph) {
            st = iterate();
        } else {
            // replay of the recorded iteration; recorded again when a by-value argument or the active
            // set has changed
            std::vector<double> key;
            key.reserve(9 + 3 * (size_t)nr);
            key.push_back((double)(uintptr_t)kd);
            key.push_back((double)P.proj);
            key.push_back((double)nr);
            for (int v : {P.syn_V, P.syn_R, P.adj_R, P.adj_W, P.adj_L, P.adj_nrb, P.live_gen, P.syn_V1, P.syn_R1,
                          P.adj_R1, P.adj_W1, P.adj_L1})
                key.push_back((double)v);
            for (int r = 0; r < nr; ++r) {
                key.push_back(le[r]);
                key.push_back(pc[r]);
                key.push_back((double)active[r]);
            }
            st = AKRA_OK;
            if (!P.cg_graph_b || key != P.cg_graph_b_key) {
                st = record_graph(P, P.cg_graph_b, iterate);
                if (st == AKRA_OK) P.cg_graph_b_key = key;
            }
            if (st == AKRA_OK) {
                TraceRange tr("akra.cg_batched_iteration_graph");
                AK_HIP(hipGraphLaunch(P.cg_graph_b, P.stream), "hipGraphLaunch");
            }
        }
        if (st) return st;
        ++iters;
        st = pull();
        if (st) return st;
        for (int r = 0; r < nr; ++r) {
            if (!active[r]) continue;
            fresh[r] = 0;
            rr[r] = hs[8 * r + 3];
            if (hf[r] || !std::isfinite(rr[r])) {
                // p^T H p <= 0 with the FP32 operator: restart once from the true residual,
                // a second breakdown stops this right-hand side at its last iterate
                AK_HIP(hipMemsetAsync(P.d_flag + r, 0, sizeof(int), P.stream), "memset");
                if (restarted[r]) {
                    active[r] = 0;
                    continue;
                }
                restarted[r] = 1;
                st = refresh(r);
                if (st) return st;
                k_set<<<1, 1, 0, P.stream>>>(S(r) + 4, 0.0);
                launch_cg_p(P, V(P.d_p, r), V(P.d_r, r), S(r) + 4, pc[r], nc);
                k_cg_rz<<<1, 1, 0, P.stream>>>(S(r), pc[r]);
                continue;
            }
            rel[r] = std::sqrt(rr[r]) / bn[r];
            if (rel[r] >= o.tol && stall[r].step(rel[r])) {
                active[r] = 0;
                status[r] = AKRA_STAGNATED;
                continue;
            }
            if (std::sqrt(rr[r]) < o.reliable_delta * rmax[r] && rel[r] >= o.tol) {
                st = refresh(r);
                if (st) return st;
                k_cg_rz<<<1, 1, 0, P.stream>>>(S(r), pc[r]);
            }
        }
    }
    // results and the true residual of every right-hand side
    double worst_true = 0.0, worst_rel = 0.0;
    int result = AKRA_OK;
    for (int r = 0; r < nr; ++r) {
        const int64_t off = (int64_t)r * 2 * na;
        double tr = 0.0;
        if (bn[r] > 0) {
            st = true_res(r, P.d_xs);
            if (st) return st;
            launch_dot(P, P.d_xs, P.d_xs, S(r) + 6, nc);
            tr = std::sqrt(read_scalar(P, S(r) + 6, &he)) / bn[r];
            if (he != hipSuccess) return hip_fail(he, "cg");
        }
        worst_true = std::max(worst_true, tr);
        worst_rel = std::max(worst_rel, bn[r] > 0 ? rel[r] : 0.0);
        result = merge_stops((akra_status)result, (akra_status)status[r]);
        if (xE)
            AK_HIP(hipMemcpyAsync(xE + off, V(P.d_x, r), sizeof(double2) * na, hipMemcpyDeviceToDevice, P.stream),
                   "copy");
        AK_HIP(hipMemcpyAsync(xB + off, V(P.d_x, r) + 2 * na, sizeof(double2) * na, hipMemcpyDeviceToDevice,
                              P.stream),
               "copy");
    }
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    info.iters = iters;
    info.fp64_applies = P.cg_fp64_applies;
    info.rel_resid = worst_rel;
    info.rel_resid_true = worst_true;
    info.lambda_eff = le[0];
    info.precond = pc[0];
    if (result == AKRA_NOT_CONVERGED) set_error("maxiter reached or stalled for some right-hand side");
    if (result == AKRA_STAGNATED) set_error("CG stagnated for some right-hand side");
    return (akra_status)result;
}

static akra_status solve_common(Plan &P, const double *g1, const double *g2, const double *ninv, const uint8_t *mask,
                                const double *bE, const double *bB, const akra_cg_opts *opts, double *xE, double *xB,
                                akra_cg_info *info_out, int ninv_count = 0)
{
    auto t0 = std::chrono::steady_clock::now();
    akra_cg_opts o;
    akra_status st = read_opts(opts, o);
    if (st) return st;
    akra_cg_info info{};
    std::vector<double> le, pc;
    st = setup_weights(P, ninv, mask, o.lambda, le, pc, nullptr, ninv_count);
    if (st) return st;
    const double *kd;
    st = kernel_to_device(P, o.kernel_l, &kd);
    if (st) return st;
    ProjScope scope(P, o.mode);
    akra_status worst = AKRA_OK;
    if (P.prec == AKRA_FP32 && P.nrhs > 1) {
        worst = solve_batched(P, g1, g2, bE, bB, o, kd, le, pc, xE, xB, info);
        if (worst != AKRA_OK && !stopped_early(worst)) return worst;
        info.status = worst;
        info.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (info_out) *info_out = info;
        return worst;
    }
    for (int r = 0; r < P.nrhs; ++r) {
        const int64_t off = (int64_t)r * 2 * P.nalm;
        st = cg_prepare(P, g1, g2, bE, bB, xE, xB, o, kd, le, pc, r);
        if (st) return st;
        st = cg_run(P, o, &info);
        if (st == AKRA_OK || stopped_early(st)) {
            if (xE)
                AK_HIP(hipMemcpyAsync(xE + off, P.d_x, sizeof(double2) * P.nalm, hipMemcpyDeviceToDevice, P.stream),
                       "copy");
            AK_HIP(hipMemcpyAsync(xB + off, P.d_x + 2 * P.nalm, sizeof(double2) * P.nalm, hipMemcpyDeviceToDevice,
                                  P.stream),
                   "copy");
            AK_HIP(hipStreamSynchronize(P.stream), "sync");
        }
        if (st != AKRA_OK && !stopped_early(st)) return st;
        worst = merge_stops(worst, st);
    }
    info.status = worst;
    info.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info_out) *info_out = info;
    return worst;
}

akra_status akra_cg_solve(akra_plan plan, const double *g1, const double *g2, const double *ninv, const uint8_t *mask,
                          const akra_cg_opts *opts, double *xE, double *xB, akra_cg_info *info)
{
    TraceRange trace_range("akra_cg_solve");
    AK_PLAN();
    if (!g1 || !g2 || !xE || !xB) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    return solve_common(P, g1, g2, ninv, mask, nullptr, nullptr, opts, xE, xB, info);
}

akra_status akra_cg_solve_b(akra_plan plan, const double *ninv, const uint8_t *mask, const double *bE, const double *bB,
                            const akra_cg_opts *opts, double *xE, double *xB, akra_cg_info *info)
{
    TraceRange trace_range("akra_cg_solve_b");
    AK_PLAN();
    if (!bE || !bB || !xE || !xB) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    return solve_common(P, nullptr, nullptr, ninv, mask, bE, bB, opts, xE, xB, info);
}

// Conditional B-mode solve (App. A): b~_B = b_B - H_BE kE, then (H_BB + lambda_eff) kB = b~_B.
// b~_B of every right-hand side is formed in FP64 into kB, which then serves as the given
// right-hand side of a B-only solve (the E block of a given b is zeroed by the B-only scope).
akra_status akra_cg_solve_cond_b(akra_plan plan, const double *g1, const double *g2, const double *ninv,
                                 const uint8_t *mask, const akra_cg_opts *opts, const double *kE, double *kB,
                                 akra_cg_info *info)
{
    TraceRange trace_range("akra_cg_solve_cond_b");
    AK_PLAN();
    if (!g1 || !g2 || !kE || !kB) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    akra_cg_opts o;
    akra_status st = read_opts(opts, o);
    if (st) return st;
    if (o.use_x0) {
        set_error("use_x0 is not supported by the conditional B-mode solve");
        return AKRA_ERR_ARG;
    }
    if (kE == kB) {
        set_error("kB must not alias kE");
        return AKRA_ERR_ARG;
    }
    std::vector<double> le, pc;
    st = setup_weights(P, ninv, mask, o.lambda, le, pc);
    if (st) return st;
    const double *kd;
    st = kernel_to_device(P, o.kernel_l, &kd);
    if (st) return st;
    const int64_t na = P.nalm, nc = 2 * na;
    {
        ProjScope scope(P, AKRA_JOINT_EB);
        for (int r = 0; r < P.nrhs; ++r) {
            const int64_t off = (int64_t)r * 2 * na;
            // b of this right-hand side (both blocks) into d_b
            launch_ring(P, false, 1, g1 + r * P.npix, g2 + r * P.npix, nullptr, nullptr, P.d_W + r * P.npix, 1, true);
            launch_leg_adj(P, false, 0, true);
            launch_epilogue(P, false, kd, 0.0, nullptr, nullptr, P.d_b, P.d_b + nc);
            // H (kE, 0) into d_w; the B block is H_BE kE (the regulariser term of a zero B is zero)
            AK_HIP(hipMemsetAsync(P.d_xs + nc, 0, sizeof(double2) * na, P.stream), "memset");
            st = apply_H_timed(P, false, kd, le[r], kE + off, P.d_xs + nc, P.d_w, P.d_w + nc, r);
            if (st) return st;
            launch_axpby(P, P.d_b + nc, -1.0, P.d_w + nc, 1.0, na);
            AK_HIP(hipMemcpyAsync(kB + off, P.d_b + nc, sizeof(double2) * na, hipMemcpyDeviceToDevice, P.stream),
                   "copy");
        }
        st = check_launch("cond_b rhs");
        if (st) return st;
    }
    akra_cg_opts ob = o;
    ob.mode = AKRA_B_ONLY;
    // the given right-hand side: B block in kB, its E block is zeroed by the B-only scope
    return solve_common(P, nullptr, nullptr, ninv, mask, kB, kB, &ob, nullptr, kB, info);
}

__global__ void k_sum2_scaled(double *out, const double *a, const double *b, double f) { *out = f * (*a + *b); }

// Gradient of L(x(g, ninv)) for x = H^-1 b(g, ninv) (differentiable form of the solve).  With the
// upstream gradient v on the stored (Re, Im) of x and the full-m product <,>_w under which H is
// self-adjoint:
//   u = H^-1 (v / w)                                   (one more solve with the same operator)
//   dL/dg     = Omega W (Y K u)
//   dL/dninv  = M [Omega (Y K u) . (g - Y K x) - (lambda / sum M) <u, x>_w]
// the last term from lambda_eff = lambda <ninv>_M.  Y K u and Y K x are formed in FP64.
akra_status akra_cg_solve_vjp(akra_plan plan, const double *g1, const double *g2, const double *ninv,
                              const uint8_t *mask, const akra_cg_opts *opts, const double *xE, const double *xB,
                              const double *vE, const double *vB, double *dg1, double *dg2, double *dninv,
                              akra_cg_info *info_out)
{
    TraceRange trace_range("akra_cg_solve_vjp");
    AK_PLAN();
    if (!g1 || !g2 || !xE || !xB || !vE || !vB || !dg1 || !dg2 || !dninv) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    if (opts && opts->use_x0) {
        set_error("use_x0 is not supported by the gradient solve");
        return AKRA_ERR_ARG;
    }
    auto t0 = std::chrono::steady_clock::now();
    akra_cg_opts o;
    akra_status st = read_opts(opts, o);
    if (st) return st;
    akra_cg_info info{};
    std::vector<double> le, pc, ms;
    st = setup_weights(P, ninv, mask, o.lambda, le, pc, &ms);
    if (st) return st;
    const double *kd;
    st = kernel_to_device(P, o.kernel_l, &kd);
    if (st) return st;
    akra_status worst = AKRA_OK;
    const int64_t na = P.nalm;
    ProjScope scope(P, o.mode);
    for (int r = 0; r < P.nrhs; ++r) {
        const int64_t off = (int64_t)r * 2 * na, mo = (int64_t)r * P.npix;
        launch_vjp_rhs(P, vE + off, vB + off, P.d_b, P.d_b + 2 * na);
        st = zero_held(P, P.d_b);
        if (st) return st;
        P.cg_kern = kd;
        P.cg_lam = le[r];
        P.cg_pc = pc[r];
        P.cg_rhs = r;
        st = cg_begin(P, false);
        if (st) return st;
        st = cg_run(P, o, &info);
        if (st != AKRA_OK && !stopped_early(st)) return st;
        worst = merge_stops(worst, st);
        // c = lambda / sum M * <u, x>_w, in scalar slots past the per-rhs weight sums
        double *sc = P.d_scal + 8 + 4 * P.nrhs;
        launch_dot(P, P.d_x, xE + off, sc, na);
        launch_dot(P, P.d_x + 2 * na, xB + off, sc + 1, na);
        k_sum2_scaled<<<1, 1, 0, P.stream>>>(sc + 2, sc, sc + 1, ms[r] > 0 ? o.lambda / ms[r] : 0.0);
        // q = Y K u into the gradient maps
        launch_prologue(P, false, P.d_x, P.d_x + 2 * na, kd, 1);
        launch_leg_synth(P, false, 1, false);
        launch_ring(P, false, 0, nullptr, nullptr, dg1 + mo, dg2 + mo, nullptr, 1, false);
        // Y K x, consumed per pixel together with q, g, W and the mask
        launch_prologue(P, false, xE + off, xB + off, kd, 1);
        launch_leg_synth(P, false, 1, false);
        launch_ring_grad(P, g1 + mo, g2 + mo, dg1 + mo, dg2 + mo, P.d_W + mo, dninv + mo, mask, sc + 2);
        st = check_launch("solve_vjp");
        if (st) return st;
    }
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    info.status = worst;
    info.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info_out) *info_out = info;
    return worst;
}

akra_status akra_cg_start(akra_plan plan, const double *g1, const double *g2, const double *ninv, const uint8_t *mask,
                          const akra_cg_opts *opts)
{
    TraceRange trace_range("akra_cg_start");
    AK_PLAN();
    if (!g1 || !g2) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    akra_cg_opts o;
    akra_status st = read_opts(opts, o);
    if (st) return st;
    if (o.use_x0) {
        set_error("akra_cg_start starts from x0 = 0");
        return AKRA_ERR_ARG;
    }
    std::vector<double> le, pc;
    st = setup_weights(P, ninv, mask, o.lambda, le, pc);
    if (st) return st;
    const double *kd;
    st = kernel_to_device(P, o.kernel_l, &kd);
    if (st) return st;
    P.cg_proj = o.mode;
    ProjScope scope(P, o.mode);
    return cg_prepare(P, g1, g2, nullptr, nullptr, nullptr, nullptr, o, kd, le, pc, 0);
}

akra_status akra_cg_step(akra_plan plan, int nsteps)
{
    TraceRange trace_range("akra_cg_step");
    AK_PLAN();
    if (!P.cg_ready) {
        set_error("akra_cg_step before akra_cg_start");
        return AKRA_ERR_ARG;
    }
    ProjScope scope(P, P.cg_proj);
    for (int i = 0; i < nsteps; ++i) {
        akra_status st = cg_step1(P, P.prec == AKRA_FP32);
        if (st) return st;
    }
    return AKRA_OK;
}

akra_status akra_cg_state(akra_plan plan, double *rel_resid, int *iters, double *xE, double *xB)
{
    TraceRange trace_range("akra_cg_state");
    AK_PLAN();
    if (!P.cg_ready) {
        set_error("akra_cg_state before akra_cg_start");
        return AKRA_ERR_ARG;
    }
    double rr;
    int flag;
    akra_status st = cg_poll(P, &rr, &flag);
    if (st) return st;
    if (rel_resid) *rel_resid = P.cg_bn > 0 ? std::sqrt(rr) / P.cg_bn : 0.0;
    if (iters) *iters = P.cg_iters;
    if (xE && xB) {
        AK_HIP(hipMemcpyAsync(xE, P.d_x, sizeof(double2) * P.nalm, hipMemcpyDeviceToDevice, P.stream), "copy");
        AK_HIP(hipMemcpyAsync(xB, P.d_x + 2 * P.nalm, sizeof(double2) * P.nalm, hipMemcpyDeviceToDevice, P.stream),
               "copy");
        AK_HIP(hipStreamSynchronize(P.stream), "sync");
    }
    if (flag || !std::isfinite(rr)) {
        set_error("CG breakdown: p^T H p <= 0 or non-finite scalar");
        return AKRA_ERR_NUMERIC;
    }
    return AKRA_OK;
}

// the largest adjoint ring-block count any weighted apply can reach with the two shapes: the
// groups of every class under the smaller group count per block, plus the rounding of the split
static int nrb_bound(const Plan &P, int gpw0, int gpw1)
{
    const int gpw = std::min(gpw0, gpw1);
    return P.adj_nrb_polar + (P.ng64 - P.polar_groups + gpw - 1) / gpw + LIVE_NRB_EXTRA;
}

static akra_status set_tuning_class(Plan &P, int one_sided, int syn_variant, int syn_rings, int adj_rings,
                                    int adj_waves, int adj_chunk)
{
    const bool sv = syn_variant == 0 || syn_variant == 1;
    const bool sr = syn_rings == 1 || syn_rings == 2 || syn_rings == 4;
    if (!sv || !sr || !adj_shape_supported(adj_rings, adj_waves, adj_chunk)) {
        set_error("unsupported tuning (see akra.h for the supported launch shapes)");
        return AKRA_ERR_ARG;
    }
    const int gpw = adj_rings * adj_waves;
    const int other = one_sided ? P.adj_R * P.adj_W : P.adj_R1 * P.adj_W1;
    if ((size_t)nrb_bound(P, gpw, other) > P.part_rb_cap) {
        set_error("adjoint shape needs more ring blocks than the plan's partial-sum buffer holds");
        return AKRA_ERR_ARG;
    }
    if (one_sided) {
        P.syn_V1 = syn_variant;
        P.syn_R1 = syn_rings;
        P.adj_R1 = adj_rings;
        P.adj_W1 = adj_waves;
        P.adj_L1 = adj_chunk;
    } else {
        P.syn_V = syn_variant;
        P.syn_R = syn_rings;
        P.adj_R = adj_rings;
        P.adj_W = adj_waves;
        P.adj_L = adj_chunk;
        P.adj_nrb = P.adj_nrb_polar + (P.ng64 - P.polar_groups + gpw - 1) / gpw;
    }
    compute_work(P);
    if (P.live_gen) compute_work_live(P);  // the staged lists of the last weight set-up
    return AKRA_OK;
}

akra_status akra_plan_set_tuning(akra_plan plan, int syn_variant, int syn_rings, int adj_rings, int adj_waves,
                                 int adj_chunk)
{
    AK_PLAN();
    return set_tuning_class(P, 0, syn_variant, syn_rings, adj_rings, adj_waves, adj_chunk);
}

akra_status akra_plan_set_tuning_one_sided(akra_plan plan, int syn_variant, int syn_rings, int adj_rings,
                                           int adj_waves, int adj_chunk)
{
    AK_PLAN();
    return set_tuning_class(P, 1, syn_variant, syn_rings, adj_rings, adj_waves, adj_chunk);
}

akra_status akra_plan_get_tuning_one_sided(akra_plan plan, int *out5)
{
    AK_PLAN();
    if (!out5) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    out5[0] = P.syn_V1;
    out5[1] = P.syn_R1;
    out5[2] = P.adj_R1;
    out5[3] = P.adj_W1;
    out5[4] = P.adj_L1;
    return AKRA_OK;
}

akra_status akra_plan_set_tuning_batched(akra_plan plan, int syn_waves, int adj_waves)
{
    AK_PLAN();
    const bool sw = syn_waves == 1 || syn_waves == 2 || syn_waves == 4 || syn_waves == 8;
    const bool aw = adj_waves == 2 || adj_waves == 4 || adj_waves == 8;
    if (!sw || !aw) {
        set_error("unsupported batched tuning: syn_waves in {1, 2, 4, 8}, adj_waves in {2, 4, 8}");
        return AKRA_ERR_ARG;
    }
    if (P.prec != AKRA_FP32 || P.nrhs < 2) {
        set_error("batched tuning applies to FP32 plans with several right-hand sides");
        return AKRA_ERR_ARG;
    }
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    P.bat_SW = syn_waves;
    P.bat_AW = adj_waves;
    P.nrb_b = (P.polar_groups + adj_waves - 1) / adj_waves + (P.ng64 - P.polar_groups + adj_waves - 1) / adj_waves;
    drop_graph(P);  // recorded iterations hold the old launch shapes
    return AKRA_OK;
}

akra_status akra_plan_get_tuning_batched(akra_plan plan, int *out2)
{
    AK_PLAN();
    if (!out2) {
        set_error("out2 is NULL");
        return AKRA_ERR_ARG;
    }
    out2[0] = P.bat_SW;
    out2[1] = P.bat_AW;
    return AKRA_OK;
}

akra_status akra_set_ring_register_engine(int on)
{
    g_ring_register = on != 0;
    return AKRA_OK;
}

akra_status akra_set_ring_whole_maxm(int maxm)
{
    if (maxm < 2 || maxm > 8192 || (maxm & (maxm - 1))) {
        set_error("ring whole-transform bound must be a power of two in [2, 8192]");
        return AKRA_ERR_ARG;
    }
    g_ring_whole_maxm = maxm;
    return AKRA_OK;
}

akra_status akra_plan_work(akra_plan plan, int64_t *out3)
{
    AK_PLAN();
    if (!out3) {
        set_error("out3 is NULL");
        return AKRA_ERR_ARG;
    }
    for (int i = 0; i < 3; ++i) out3[i] = P.work[i];
    return AKRA_OK;
}

akra_status akra_plan_work_weighted(akra_plan plan, int64_t *out6)
{
    AK_PLAN();
    int64_t *out5 = out6;
    if (!out5) {
        set_error("out6 is NULL");
        return AKRA_ERR_ARG;
    }
    out5[0] = P.n_live_rings;
    for (int i = 0; i < 5; ++i) out5[1 + i] = P.work_live[i];
    return AKRA_OK;
}

akra_status akra_plan_set_skip_unweighted(akra_plan plan, int on)
{
    AK_PLAN();
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    P.skip_rings = on != 0;
    drop_graph(P);  // recorded iterations hold the launch sets
    return AKRA_OK;
}

akra_status akra_plan_work_batched(akra_plan plan, int64_t *out1)
{
    AK_PLAN();
    if (!out1) {
        set_error("out1 is NULL");
        return AKRA_ERR_ARG;
    }
    *out1 = P.work_b;
    return AKRA_OK;
}

akra_status akra_plan_get_tuning(akra_plan plan, int *out5)
{
    AK_PLAN();
    if (!out5) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    out5[0] = P.syn_V;
    out5[1] = P.syn_R;
    out5[2] = P.adj_R;
    out5[3] = P.adj_W;
    out5[4] = P.adj_L;
    return AKRA_OK;
}

akra_status akra_plan_set_timing(akra_plan plan, int on)
{
    AK_PLAN();
    P.timing = on != 0;
    P.ev_used = 0;
    return AKRA_OK;
}

akra_status akra_plan_set_graph(akra_plan plan, int on)
{
    AK_PLAN();
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    P.use_graph = on != 0;
    if (!P.use_graph) drop_graph(P);
    return AKRA_OK;
}

akra_status akra_plan_stage_times(akra_plan plan, double *ms, int *calls)
{
    AK_PLAN();
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    for (int s = 0; s < AKRA_NSTAGES; ++s) {
        if (ms) ms[s] = 0.0;
        if (calls) calls[s] = 0;
    }
    for (int i = 0; i < P.ev_used; ++i) {
        float t = 0;
        AK_HIP(hipEventElapsedTime(&t, P.ev_pool[i][0], P.ev_pool[i][1]), "hipEventElapsedTime");
        const int s = P.ev_stage[i];
        if (ms) ms[s] += t;
        if (calls) calls[s] += 1;
    }
    P.ev_used = 0;
    return AKRA_OK;
}


// ---- shape-noise realisations and power spectra (Sec. IV, power spectrum results) ---------------
static bool overlaps(const void *a, int64_t na, const void *b, int64_t nb)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

static akra_status read_nobs(Plan &P, int64_t *n)
{
    AK_HIP(hipMemcpyAsync(P.h_pin, P.d_cmp_nobs, sizeof(int64_t), hipMemcpyDeviceToHost, P.stream), "copy");
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    std::memcpy(n, P.h_pin, sizeof(int64_t));
    return AKRA_OK;
}

// range check of the shuffles since the flag was last cleared
static akra_status shuffle_flag(Plan &P)
{
    akra_status st = check_launch("shuffle");
    if (st) return st;
    int f = 0;
    AK_HIP(hipMemcpyAsync(P.h_pin, P.d_cmp_flag, sizeof(int), hipMemcpyDeviceToHost, P.stream), "copy");
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    std::memcpy(&f, P.h_pin, sizeof(int));
    if (f) {
        AK_HIP(hipMemsetAsync(P.d_cmp_flag, 0, sizeof(int), P.stream), "memset");
        set_error(f == 1 ? "perm holds an entry outside [0, n_obs)" : "idx holds a pixel index outside [0, Npix)");
        return AKRA_ERR_ARG;
    }
    return AKRA_OK;
}

akra_status akra_unmasked_index(akra_plan plan, const uint8_t *mask, int32_t *idx, int64_t *n_obs)
{
    TraceRange trace_range("akra_unmasked_index");
    AK_PLAN();
    if (!mask || !idx || !n_obs) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    launch_unmasked_index(P, mask, idx);
    akra_status st = check_launch("unmasked_index");
    if (st) return st;
    return read_nobs(P, n_obs);
}

akra_status akra_shuffle_shear(akra_plan plan, const double *g1, const double *g2, const int32_t *idx, int64_t n_obs,
                               const int32_t *perm, int n_real, double *g1_out, double *g2_out)
{
    TraceRange trace_range("akra_shuffle_shear");
    AK_PLAN();
    if (n_real < 0 || n_obs < 0 || n_obs > P.npix) {
        set_error("n_real must be >= 0 and n_obs in [0, Npix]");
        return AKRA_ERR_ARG;
    }
    if (n_real == 0) return AKRA_OK;
    if (!g1 || !g2 || !g1_out || !g2_out || (n_obs > 0 && (!idx || !perm))) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    const int64_t mb = P.npix * (int64_t)sizeof(double), ob = mb * n_real;
    if (overlaps(g1_out, ob, g1, mb) || overlaps(g1_out, ob, g2, mb) || overlaps(g2_out, ob, g1, mb) ||
        overlaps(g2_out, ob, g2, mb) || overlaps(g1_out, ob, g2_out, ob)) {
        set_error("outputs alias inputs or each other");
        return AKRA_ERR_ARG;
    }
    AK_HIP(hipMemsetAsync(P.d_cmp_flag, 0, sizeof(int), P.stream), "memset");
    for (int k = 0; k < n_real; ++k)
        launch_shuffle(P, g1, g2, idx, n_obs, perm ? perm + (int64_t)k * n_obs : nullptr, g1_out + (int64_t)k * P.npix,
                       g2_out + (int64_t)k * P.npix);
    return shuffle_flag(P);
}

akra_status akra_alm_spectra(akra_plan plan, const double *x, int nx, const double *y, int ny, const int32_t *pairs,
                             int npairs, double *cl)
{
    TraceRange trace_range("akra_alm_spectra");
    AK_PLAN();
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
    const double2 *X = (const double2 *)x, *Y = (const double2 *)y;
    for (int q0 = 0; q0 < npairs; q0 += SPEC_NP) {
        SpecArgs a{};
        const int n = std::min(SPEC_NP, npairs - q0);
        for (int i = 0; i < n; ++i) {
            a.x[i] = X + (int64_t)pairs[2 * (q0 + i)] * P.nalm;
            a.y[i] = Y + (int64_t)pairs[2 * (q0 + i) + 1] * P.nalm;
            a.cl[i] = cl + (int64_t)(q0 + i) * (P.lmax + 1);
        }
        launch_spectra(P, a, n);
    }
    return check_launch("spectra");
}

static int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

akra_status akra_noise_work_size(akra_plan plan, int nset, int64_t *bytes)
{
    AK_PLAN();
    if ((nset != 1 && nset != 2) || !bytes) {
        set_error("nset must be 1 or 2 and bytes non-NULL");
        return AKRA_ERR_ARG;
    }
    const int64_t gx = std::max(P.nrhs, nset);
    *bytes = align256(P.npix * 4) + 2 * align256(gx * P.npix * 8) + 2 * align256(gx * P.nalm * 16);
    return AKRA_OK;
}

akra_status akra_noise_spectra(akra_plan plan, int nset, const double *g1, const double *g2, const double *ninv,
                               const uint8_t *mask, const int32_t *perm, int64_t n_obs, int n_real,
                               const akra_cg_opts *opts, void *work, int64_t work_bytes, double *cl, double *cl_mean,
                               double *cl_std, akra_cg_info *info_out)
{
    TraceRange trace_range("akra_noise_spectra");
    AK_PLAN();
    auto t0 = std::chrono::steady_clock::now();
    if (nset != 1 && nset != 2) {
        set_error("nset must be 1 or 2");
        return AKRA_ERR_ARG;
    }
    if (n_real < 0 || n_obs < 0 || n_obs > P.npix) {
        set_error("n_real must be >= 0 and n_obs in [0, Npix]");
        return AKRA_ERR_ARG;
    }
    const int G = P.nrhs, gx = std::max(G, nset);
    if (nset == 2 && G > 1 && G % 2) {
        set_error("split halves need an even nrhs (or nrhs = 1)");
        return AKRA_ERR_ARG;
    }
    akra_cg_opts o;
    akra_status st = read_opts(opts, o);
    if (st) return st;
    const int nspec = o.mode == AKRA_JOINT_EB ? 3 : 1;
    int64_t need = 0;
    st = akra_noise_work_size(plan, nset, &need);
    if (st) return st;
    if (!g1 || !g2 || !ninv || !mask || !work || (n_real > 0 && !cl) || (n_obs > 0 && n_real > 0 && !perm)) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    if (work_bytes < need) {
        set_error("workspace too small: " + std::to_string(need) + " bytes needed");
        return AKRA_ERR_ARG;
    }
    if ((uintptr_t)work % 256) {
        set_error("workspace must be 256-byte aligned");
        return AKRA_ERR_ARG;
    }
    const int64_t npix = P.npix, na = P.nalm, L1 = P.lmax + 1;
    char *w = (char *)work;
    int32_t *idx = (int32_t *)w;
    w += align256(npix * 4);
    double *m1 = (double *)w;
    w += align256(gx * npix * 8);
    double *m2 = (double *)w;
    w += align256(gx * npix * 8);
    double *xE = (double *)w;
    w += align256(gx * na * 16);
    double *xB = (double *)w;

    launch_unmasked_index(P, mask, idx);
    st = check_launch("unmasked_index");
    if (st) return st;
    int64_t nob = 0;
    st = read_nobs(P, &nob);
    if (st) return st;
    if (nob != n_obs) {
        set_error("n_obs (" + std::to_string(n_obs) + ") differs from the unmasked pixels of the mask (" +
                  std::to_string(nob) + ")");
        return AKRA_ERR_ARG;
    }
    AK_HIP(hipMemsetAsync(P.d_cmp_flag, 0, sizeof(int), P.stream), "memset");
    akra_cg_info agg{};
    akra_status worst = AKRA_OK;
    bool first = true;
    const int R = gx / nset;  // realisations per pass
    for (int k0 = 0; k0 < n_real; k0 += R) {
        // shuffled maps of the pass: slot s = realisation k0 + s / nset, set s % nset (zero past n_real)
        for (int s = 0; s < gx; ++s) {
            const int k = k0 + s / nset, q = s % nset;
            const int32_t *pr = (k < n_real && n_obs > 0) ? perm + ((int64_t)q * n_real + k) * n_obs : nullptr;
            launch_shuffle(P, g1 + (int64_t)q * npix, g2 + (int64_t)q * npix, idx, n_obs, pr, m1 + (int64_t)s * npix,
                           m2 + (int64_t)s * npix);
        }
        st = shuffle_flag(P);
        if (st) return st;
        // solves in groups of nrhs slots; slot s takes N^-1 map s mod nset
        for (int g0 = 0; g0 < gx; g0 += G) {
            akra_cg_info gi{};
            st = solve_common(P, m1 + (int64_t)g0 * npix, m2 + (int64_t)g0 * npix, ninv + (int64_t)(g0 % nset) * npix,
                              mask, nullptr, nullptr, &o, xE + (int64_t)g0 * 2 * na, xB + (int64_t)g0 * 2 * na, &gi,
                              G == 1 ? 1 : nset);
            if (st != AKRA_OK && !stopped_early(st)) return st;
            worst = merge_stops(worst, st);
            agg.iters += gi.iters;
            agg.fp64_applies += gi.fp64_applies;
            agg.rel_resid = std::max(agg.rel_resid, gi.rel_resid);
            agg.rel_resid_true = std::max(agg.rel_resid_true, gi.rel_resid_true);
            if (first) {
                agg.lambda_eff = gi.lambda_eff;
                agg.precond = gi.precond;
                first = false;
            }
        }
        // spectra of the pass's realisations: sets A (slot r nset) and B (slot r nset + nset - 1)
        SpecArgs a{};
        int n = 0;
        auto add = [&](const double2 *u, const double2 *v, double *c) {
            a.x[n] = u;
            a.y[n] = v;
            a.cl[n] = c;
            if (++n == SPEC_NP) {
                launch_spectra(P, a, n);
                n = 0;
            }
        };
        for (int r = 0; r < R && k0 + r < n_real; ++r) {
            const int64_t sa = (int64_t)r * nset, sb = sa + nset - 1;
            const double2 *EA = (const double2 *)xE + sa * na, *EB = (const double2 *)xE + sb * na;
            const double2 *BA = (const double2 *)xB + sa * na, *BB = (const double2 *)xB + sb * na;
            double *c = cl + (int64_t)(k0 + r) * nspec * L1;
            if (o.mode == AKRA_E_ONLY) {
                add(EA, EB, c);
            } else if (o.mode == AKRA_B_ONLY) {
                add(BA, BB, c);
            } else {
                add(EA, EB, c);
                add(BA, BB, c + L1);
                add(EA, BB, c + 2 * L1);
            }
        }
        if (n) launch_spectra(P, a, n);
        st = check_launch("spectra");
        if (st) return st;
    }
    if (cl_mean || cl_std) launch_cl_moments(P, cl, n_real, (int64_t)nspec * L1, cl_mean, cl_std);
    st = check_launch("cl_moments");
    if (st) return st;
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    agg.status = worst;
    agg.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info_out) *info_out = agg;
    if (worst == AKRA_NOT_CONVERGED) set_error("maxiter reached or stalled for some realisation");
    if (worst == AKRA_STAGNATED) set_error("CG stagnated for some realisation");
    return worst;
}

// ---- catalogue pixelisation (Sec. III.B) -----------------------------------------------------------
static akra_status read_flags2(Plan &P, int *f)
{
    AK_HIP(hipMemcpyAsync(P.h_pin, P.d_cmp_flag, 2 * sizeof(int), hipMemcpyDeviceToHost, P.stream), "copy");
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    std::memcpy(f, P.h_pin, 2 * sizeof(int));
    if (f[0] || f[1]) AK_HIP(hipMemsetAsync(P.d_cmp_flag, 0, 2 * sizeof(int), P.stream), "memset");
    return AKRA_OK;
}

akra_status akra_ang2pix(akra_plan plan, const double *z, const double *phi, int64_t n, int32_t *pix)
{
    TraceRange trace_range("akra_ang2pix");
    AK_PLAN();
    if (n < 0) {
        set_error("n must be >= 0");
        return AKRA_ERR_ARG;
    }
    if (n == 0) return AKRA_OK;
    if (!z || !phi || !pix) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    AK_HIP(hipMemsetAsync(P.d_cmp_flag, 0, 2 * sizeof(int), P.stream), "memset");
    launch_ang2pix(P, z, phi, nullptr, nullptr, nullptr, n, (uint32_t *)pix, nullptr);
    akra_status st = check_launch("ang2pix");
    if (st) return st;
    int f[2];
    st = read_flags2(P, f);
    if (st) return st;
    if (f[0]) {
        set_error("a direction lies outside z in [-1, 1], phi in [0, 2 pi)");
        return AKRA_ERR_ARG;
    }
    return AKRA_OK;
}

akra_status akra_pixelize_work_size(akra_plan plan, int64_t n_gal, int64_t *bytes)
{
    AK_PLAN();
    if (n_gal < 0 || n_gal > INT32_MAX || !bytes) {
        set_error("n_gal must be in [0, 2^31 - 1] and bytes non-NULL");
        return AKRA_ERR_ARG;
    }
    AK_HIP(pixelize_work_bytes(P, n_gal, bytes), "radix sort storage query");
    return AKRA_OK;
}

akra_status akra_pixelize(akra_plan plan, const double *z, const double *phi, const double *e1, const double *e2,
                          const double *w, int64_t n_gal, double R, double sigma_e, double n_th, void *work,
                          int64_t work_bytes, double *g1, double *g2, double *ninv, double *neff, uint8_t *mask)
{
    TraceRange trace_range("akra_pixelize");
    AK_PLAN();
    if (n_gal < 0 || n_gal > INT32_MAX) {
        set_error("n_gal must be in [0, 2^31 - 1]");
        return AKRA_ERR_ARG;
    }
    if (!(std::isfinite(R) && R != 0.0) || !(std::isfinite(sigma_e) && sigma_e > 0.0) || !std::isfinite(n_th)) {
        set_error("R must be finite and nonzero, sigma_e finite and > 0, n_th finite");
        return AKRA_ERR_ARG;
    }
    if (!work || !g1 || !g2 || !ninv || !neff || !mask || (n_gal > 0 && (!z || !phi || !e1 || !e2 || !w))) {
        set_error("null pointer argument");
        return AKRA_ERR_ARG;
    }
    int64_t need = 0;
    akra_status st = akra_pixelize_work_size(plan, n_gal, &need);
    if (st) return st;
    if (work_bytes < need) {
        set_error("workspace too small: " + std::to_string(need) + " bytes needed");
        return AKRA_ERR_ARG;
    }
    if ((uintptr_t)work % 256) {
        set_error("workspace must be 256-byte aligned");
        return AKRA_ERR_ARG;
    }
    AK_HIP(hipMemsetAsync(P.d_cmp_flag, 0, 2 * sizeof(int), P.stream), "memset");
    double4 *rec = nullptr;
    uint32_t *keys = pixelize_keys(P, n_gal, work, &rec);
    if (!keys) {
        set_error("radix sort storage query failed");
        return AKRA_ERR_HIP;
    }
    launch_ang2pix(P, z, phi, e1, e2, w, n_gal, keys, rec);
    st = check_launch("ang2pix");
    if (st) return st;
    int f[2];
    st = read_flags2(P, f);
    if (st) return st;
    if (f[0] || f[1]) {
        set_error(f[0] ? "a direction lies outside z in [-1, 1], phi in [0, 2 pi)"
                       : "a weight is negative or not finite, or an ellipticity is not finite");
        return AKRA_ERR_ARG;
    }
    AK_HIP(launch_pixelize(P, n_gal, R, sigma_e * sigma_e, n_th, work, g1, g2, ninv, neff, mask), "pixelize");
    AK_HIP(hipStreamSynchronize(P.stream), "sync");
    return AKRA_OK;
}

}  // extern "C"
