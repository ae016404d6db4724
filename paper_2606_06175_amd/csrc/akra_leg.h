// Legendre stages of the operator chain (device code, gfx950): the on-the-fly spin-weighted
// recurrence with exponent rescaling, the synthesis kernel (alm -> F per ring pair) and the adjoint
// kernel (G -> partial sums per ring block), plus the launch helpers shared by the translation units
// that instantiate them.  Not part of the public ABI.
#pragma once
#include <type_traits>

#include "akra_fft.h"
#include "akra_internal.h"

namespace akra {
// Recurrence forms of the Legendre kernels: 0 the plain three-term form in its scaled variant (FP64,
// and FP32 away from the poles; see Coef64S), 1 the difference form of FP32 near the poles (see
// Coef32D).  The batched matrix-core synthesis runs the unscaled plain form (CoefB).
template <typename T, int F> struct CoefT;
template <> struct CoefT<double, 0> { using type = Coef64S; };
template <> struct CoefT<float, 0> { using type = Coef32S; };
template <> struct CoefT<float, 1> { using type = Coef32D; };
template <int F> struct CoefB;
template <> struct CoefB<0> { using type = Coef32; };
template <> struct CoefB<1> { using type = Coef32D; };

// ------------------------------------------------------------------------------------------------
// Entry states: stored in FP64 as mant * 2^(512 k).  FP32 kernels re-express them in their own unit.
// ------------------------------------------------------------------------------------------------
// i0, i1: 1 / c_l and 1 / c_{l-1} at the entry degree l for the scaled plain form (mu = lambda / c);
// the difference form and the unscaled plain form pass 1.  refl = +-1 gives the state of the
// reflected ring (theta -> pi - theta) instead: with s = refl = (-1)^(l+m) at the entry degree l,
// +2lambda_l(pi - theta) = s -2lambda_l(theta) and +2lambda_{l-1}(pi - theta) = -s -2lambda_{l-1}(theta),
// and the same with the spins exchanged.
template <typename T, int F>
__device__ __forceinline__ void load_entry(const Ent64 *__restrict__ ent, const int *__restrict__ entk, int64_t idx,
                                           T &c2, T &p2, T &cm, T &pm, int &k, double i0 = 1.0, double i1 = 1.0,
                                           int refl = 0)
{
    Ent64 e = ent[idx];
    const int k64 = entk[idx];
    if (refl != 0) {
        const double sg = (double)refl;
        const Ent64 n = e;
        e.c2 = sg * n.cm;
        e.cm = sg * n.c2;
        e.p2 = -sg * n.pm;
        e.pm = -sg * n.p2;
    }
    if constexpr (F == 0) {
        e.c2 *= i0;
        e.cm *= i0;
        e.p2 *= i1;
        e.pm *= i1;
    }
    if constexpr (std::is_same<T, double>::value) {
        c2 = e.c2;
        p2 = e.p2;
        cm = e.cm;
        pm = e.pm;
        k = k64;
    } else {
        // difference form: p2, pm carry lambda_l - lambda_{l-1}
        const double d2 = F ? e.c2 - e.p2 : e.p2, dm = F ? e.cm - e.pm : e.pm;
        const double big = fmax(fmax(fabs(e.c2), fabs(e.cm)), fmax(fabs(d2), fabs(dm)));
        if (big == 0.0) {
            c2 = p2 = cm = pm = 0.0f;
            k = 0;
            return;
        }
        const int ex = ilogb(big) + 512 * k64;
        const int k32 = (ex >= -40) ? 0 : -((20 - ex) / 64);
        const int sh = 512 * k64 - 64 * k32;
        c2 = (float)ldexp(e.c2, sh);
        p2 = (float)ldexp(d2, sh);
        cm = (float)ldexp(e.cm, sh);
        pm = (float)ldexp(dm, sh);
        k = k32;
    }
}

template <typename T> __device__ __forceinline__ T scale_hi();
template <> __device__ __forceinline__ double scale_hi<double>() { return 0x1p256; }
template <> __device__ __forceinline__ float scale_hi<float>() { return 0x1p32f; }
template <typename T> __device__ __forceinline__ T scale_down();
template <> __device__ __forceinline__ double scale_down<double>() { return 0x1p-512; }
template <> __device__ __forceinline__ float scale_down<float>() { return 0x1p-64f; }

// A read-only pointer that is the same in every lane, made explicit for the compiler: the value is
// taken from the first lane and the result lives in the constant address space, so uniform loads
// through it become scalar loads.
template <typename P> using const_as = const __attribute__((address_space(4))) P;
template <typename P> __device__ __forceinline__ const_as<P> *uniform_ptr(const P *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const_as<P> *)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ Coef64 ld_coef(const_as<Coef64> *p)
{
    Coef64 c;
    c.a = p->a;
    c.b = p->b;
    c.g = p->g;
    c.pad = 0;
    return c;
}
__device__ __forceinline__ Coef32 ld_coef(const_as<Coef32> *p)
{
    Coef32 c;
    c.a = p->a;
    c.b = p->b;
    c.g = p->g;
    c.pad = 0;
    return c;
}
// the recurrence reads a' and b' only (scalar registers are scarce in the adjoint's look-ahead)
__device__ __forceinline__ Coef64S ld_coef(const_as<Coef64S> *p)
{
    Coef64S c;
    c.a = p->a;
    c.b = p->b;
    c.c = c.ic = 0.0;
    return c;
}
__device__ __forceinline__ Coef32S ld_coef(const_as<Coef32S> *p)
{
    Coef32S c;
    c.a = p->a;
    c.b = p->b;
    c.c = c.ic = 0.0f;
    return c;
}
__device__ __forceinline__ Coef32D ld_coef(const_as<Coef32D> *p)
{
    Coef32D c;
    c.a = p->a;
    c.ep = p->ep;
    c.em = p->em;
    c.g = p->g;
    return c;
}

// The ring pair's position as the recurrences use it.  FP64: x = cos(theta).  FP32 carries its
// coordinate as an unevaluated sum hi + lo of two floats, x = cos(theta) in the plain form and
// y = 1 - cos(theta) (exact in double for the ring's defining z) in the difference form: rounding
// it to one float would move the ring by a fixed angle, an error that grows linearly along l.
struct XF {
    float hi, lo;
};
struct YF {
    float hi, lo;
};
template <typename T, int F> struct PosT;
template <> struct PosT<double, 0> { using type = double; };
template <> struct PosT<float, 0> { using type = XF; };
template <> struct PosT<float, 1> { using type = YF; };
__device__ __forceinline__ void setpos(double &x, double z) { x = z; }
__device__ __forceinline__ void setpos(XF &x, double z)
{
    x.hi = (float)z;
    x.lo = (float)(z - (double)x.hi);
}
__device__ __forceinline__ void setpos(YF &y, double z)
{
    const double v = 1.0 - z;
    y.hi = (float)v;
    y.lo = (float)(v - (double)y.hi);
}

// One step l -> l+1 of the spin +2 and spin -2 recurrences.  Plain form: (c2, p2) = (lambda_l,
// lambda_{l-1}).  Difference form: (c2, p2) = (lambda_l, lambda_l - lambda_{l-1}).
template <class C>
__device__ __forceinline__ void rstep(const C &c, double x, double &c2, double &p2, double &cm, double &pm)
{
    const double u = c.a * x;
    const double n2 = fma(u + c.b, c2, -(c.g * p2));
    const double nm = fma(u - c.b, cm, -(c.g * pm));
    p2 = c2;
    c2 = n2;
    pm = cm;
    cm = nm;
}
template <class C>
__device__ __forceinline__ void rstep(const C &c, XF x, float &c2, float &p2, float &cm, float &pm)
{
    const float u = fmaf(c.a, x.hi, c.a * x.lo);
    const float n2 = fmaf(u + c.b, c2, -(c.g * p2));
    const float nm = fmaf(u - c.b, cm, -(c.g * pm));
    p2 = c2;
    c2 = n2;
    pm = cm;
    cm = nm;
}
template <class C>
__device__ __forceinline__ void rstep(const C &c, YF y, float &c2, float &p2, float &cm, float &pm)
{
    const float t = c.a * y.lo;
    const float kp = fmaf(-c.a, y.hi, c.ep - t), km = fmaf(-c.a, y.hi, c.em - t);
    p2 = fmaf(kp, c2, c.g * p2);
    pm = fmaf(km, cm, c.g * pm);
    c2 += p2;
    cm += pm;
}

// Scaled plain form (Coef64S): mu_{l+1} = (a' x +- b') mu_l - mu_{l-1}, two FMAs per spin.
__device__ __forceinline__ void rstep_s(double a, double b, double x, double &c2, double &p2, double &cm, double &pm)
{
    const double n2 = fma(fma(a, x, b), c2, -p2);
    const double nm = fma(fma(a, x, -b), cm, -pm);
    p2 = c2;
    c2 = n2;
    pm = cm;
    cm = nm;
}
__device__ __forceinline__ void rstep_s(float a, float b, XF x, float &c2, float &p2, float &cm, float &pm)
{
    const float up = fmaf(a, x.hi, fmaf(a, x.lo, b)), um = fmaf(a, x.hi, fmaf(a, x.lo, -b));
    const float n2 = fmaf(up, c2, -p2);
    const float nm = fmaf(um, cm, -pm);
    p2 = c2;
    c2 = n2;
    pm = cm;
    cm = nm;
}
__device__ __forceinline__ void rstep(const Coef64S &c, double x, double &c2, double &p2, double &cm, double &pm)
{
    rstep_s(c.a, c.b, x, c2, p2, cm, pm);
}
__device__ __forceinline__ void rstep(const Coef32S &c, XF x, float &c2, float &p2, float &cm, float &pm)
{
    rstep_s(c.a, c.b, x, c2, p2, cm, pm);
}

// wave-uniform "any lane"
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// ================================================================================================
// Legendre synthesis: for every (m, ring pair) accumulate
//   P2[par] += 2lambda_lm * (aE, aB),  Pm[par] += -2lambda_lm * (aE, aB)       par = (l + m) mod 2
// over l = max(m,2) .. lmax, with the recurrence values of the north ring in registers.  The south
// ring follows from 2lambda_lm(pi - theta) = (-1)^(l+m) -2lambda_lm(theta).  Then
//   F(m) = -(sum 2lambda (aE + i aB)),  F(-m) = -(sum -2lambda (conj aE + i conj aB)).
// One wave handles 64*R ring pairs of one m; per-l data (alm, coefficients) are wave-uniform.
// ================================================================================================
// Per-(l, m) wave-uniform input of the synthesis, written by the prologue: the coefficients a', b'
// of the scaled plain form next to c_l times four combinations of the kernel-scaled alm,
//   u0 = aE.re - aB.im,  u1 = aE.im + aB.re,  u2 = aE.re + aB.im,  u3 = aB.re - aE.im
// (Im(a_l0) zeroed), one record of 8 values so that a step is a single scalar load.  In this basis
// each ring of a pair needs four of the eight products of the two recurrence values with the record
// (see syn_step), so a pair with one weighted ring contracts with four FMAs per degree.  The record
// buffer is padded so look-ahead loads stay in bounds.
template <typename T> struct SynRec;
template <> struct alignas(64) SynRec<double> {
    double a, b, g, pad, u0, u1, u2, u3;
};
template <> struct alignas(32) SynRec<float> {
    float a, b, g, pad, u0, u1, u2, u3;
};
// record of the difference form, assembled from the coefficient table and the alm records
struct SynRecD {
    float a, ep, em, g, u0, u1, u2, u3;
};
template <typename T> using SynIn = SynRec<T>;
__device__ __forceinline__ void rstep(const SynRec<double> &c, double x, double &c2, double &p2, double &cm, double &pm)
{
    rstep_s(c.a, c.b, x, c2, p2, cm, pm);
}
__device__ __forceinline__ void rstep(const SynRec<float> &c, XF x, float &c2, float &p2, float &cm, float &pm)
{
    rstep_s(c.a, c.b, x, c2, p2, cm, pm);
}

__device__ __forceinline__ SynRec<double> ld_rec(const_as<SynRec<double>> *p)
{
    SynRec<double> r;
    r.a = p->a;
    r.b = p->b;
    r.g = p->g;
    r.pad = 0.0;
    r.u0 = p->u0;
    r.u1 = p->u1;
    r.u2 = p->u2;
    r.u3 = p->u3;
    return r;
}
__device__ __forceinline__ SynRec<float> ld_rec(const_as<SynRec<float>> *p)
{
    SynRec<float> r;
    r.a = p->a;
    r.b = p->b;
    r.g = p->g;
    r.pad = 0.0f;
    r.u0 = p->u0;
    r.u1 = p->u1;
    r.u2 = p->u2;
    r.u3 = p->u3;
    return r;
}


template <typename T>
__device__ __forceinline__ SynIn<T> syn_load(const SynRec<T> *__restrict__ rec, int l)
{
    return rec[l];
}

// Wave-uniform source of the synthesis records of form F: the prologue's records for the plain form;
// for the FP32 difference form the coefficients come from their own table and the unscaled alm
// values from the prologue's second record buffer.
template <typename T, int F> struct SynSrc;
template <typename T> struct SynSrc<T, 0> {
    const_as<SynRec<T>> *r;
    __device__ __forceinline__ SynSrc(const SynRec<T> *rec, const float4 *, const Coef32D *) : r(uniform_ptr(rec)) {}
    __device__ __forceinline__ SynRec<T> at(int i) const { return ld_rec(r + i); }
    __device__ __forceinline__ void adv(int n) { r += n; }
};
template <> struct SynSrc<float, 1> {
    const_as<float4> *r;
    const_as<Coef32D> *c;
    __device__ __forceinline__ SynSrc(const SynRec<float> *, const float4 *recu, const Coef32D *cf)
        : r(uniform_ptr(recu)), c(uniform_ptr(cf))
    {
    }
    __device__ __forceinline__ SynRecD at(int i) const
    {
        SynRecD o;
        o.a = c[i].a;
        o.ep = c[i].ep;
        o.em = c[i].em;
        o.g = c[i].g;
        o.u0 = r[i].x;
        o.u1 = r[i].y;
        o.u2 = r[i].z;
        o.u3 = r[i].w;
        return o;
    }
    __device__ __forceinline__ void adv(int n)
    {
        r += n;
        c += n;
    }
};

// XCD-aware placement: workgroups are dealt to the 8 XCDs round-robin, so all blocks of one m
// are mapped to blocks with the same index mod 8 (they share that XCD's L2 for the per-m data),
// and each XCD walks its m values in increasing order (decreasing work).  XCD x takes the orders
// m = 32 j + 4 x + i (i < 4): the four orders whose (Q, U) entries of one ring share a 128-byte
// line of F or G are placed on the same XCD, so the line is fetched into one L2, not four.  A
// launch covers m < 32 ceil((lmax + 1) / 32) (xcd_slots below); blocks past lmax return at once.
__device__ __forceinline__ void xcd_map(int b, int nbm, int &m, int &blk)
{
    const int xcd = b & 7, local = b >> 3;
    const int q = local / nbm;
    m = 32 * (q >> 2) + 4 * xcd + (q & 3);
    blk = local - q * nbm;
}

// Classes of 64-pair groups by the rings that carry weight (GCLS_BOTH, GCLS_NORTH, GCLS_SOUTH in
// akra_internal.h).  With the records in the u basis the sums of the north ring are
//   S+(u0), S+(u1) (spin +2 values times u0, u1) and S-(u2), S-(u3),
// and those of the south ring (through the reflection, with the parity sign) are
//   S-(u0), S-(u1) and S+(u2), S+(u3):
// a one-ring class runs the four FMAs of its ring only.  acc[c] holds S+(u_c), acc[4 + c] S-(u_c).
// DIRECT: a one-ring class whose recurrence runs on that ring itself (the south ring at its own
// cos(theta)): the four sums of the north-ring formula, S+(u0), S+(u1), S-(u2), S-(u3), in acc[0..3].
template <typename T, int R, bool MASK, int CLS, bool DIRECT = false, typename In, typename X>
__device__ __forceinline__ void syn_step(const In &in, const X (&x)[R], T (&c2)[R], T (&p2)[R], T (&cm)[R],
                                         T (&pm)[R], const int (&k)[R], T (&acc)[8][R])
{
#pragma unroll
    for (int j = 0; j < R; ++j) {
        T v2 = c2[j], vm = cm[j];
        if (MASK) {
            if (k[j] != 0) v2 = vm = (T)0;
        }
        if constexpr (DIRECT) {
            acc[0][j] = fma(v2, in.u0, acc[0][j]);
            acc[1][j] = fma(v2, in.u1, acc[1][j]);
            acc[2][j] = fma(vm, in.u2, acc[2][j]);
            acc[3][j] = fma(vm, in.u3, acc[3][j]);
            rstep(in, x[j], c2[j], p2[j], cm[j], pm[j]);
            continue;
        }
        if (CLS != GCLS_SOUTH) {
            acc[0][j] = fma(v2, in.u0, acc[0][j]);
            acc[1][j] = fma(v2, in.u1, acc[1][j]);
        }
        if (CLS != GCLS_NORTH) {
            acc[2][j] = fma(v2, in.u2, acc[2][j]);
            acc[3][j] = fma(v2, in.u3, acc[3][j]);
            acc[4][j] = fma(vm, in.u0, acc[4][j]);
            acc[5][j] = fma(vm, in.u1, acc[5][j]);
        }
        if (CLS != GCLS_SOUTH) {
            acc[6][j] = fma(vm, in.u2, acc[6][j]);
            acc[7][j] = fma(vm, in.u3, acc[7][j]);
        }
        rstep(in, x[j], c2[j], p2[j], cm[j], pm[j]);
    }
}

template <typename T, int R>
__device__ __forceinline__ bool rescale(T (&c2)[R], T (&p2)[R], T (&cm)[R], T (&pm)[R], int (&k)[R])
{
    bool any_neg = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (k[j] < 0) {
            T big = fmax(fabs(c2[j]), fabs(cm[j]));
            if (big > scale_hi<T>()) {
                const T d = scale_down<T>();
                c2[j] *= d;
                p2[j] *= d;
                cm[j] *= d;
                pm[j] *= d;
                k[j] += 1;
            }
            any_neg |= (k[j] < 0);
        }
    }
    return wave_any(any_neg);
}

// Rescale check of the synthesis ramp: a lane whose exponent reaches zero restarts its sums (what it
// accumulated while scaled is discarded).  Returns whether any lane of the wave is still scaled.
template <typename T, int R>
__device__ __forceinline__ bool rescale_restart(T (&c2)[R], T (&p2)[R], T (&cm)[R], T (&pm)[R], int (&k)[R],
                                                T (&acc0)[8][R], T (&acc1)[8][R])
{
    bool any_neg = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (k[j] < 0) {
            const T big = fmax(fabs(c2[j]), fabs(cm[j]));
            if (big > scale_hi<T>()) {
                const T d = scale_down<T>();
                c2[j] *= d;
                p2[j] *= d;
                cm[j] *= d;
                pm[j] *= d;
                k[j] += 1;
                if (k[j] == 0) {
#pragma unroll
                    for (int c = 0; c < 8; ++c) acc0[c][j] = acc1[c][j] = (T)0;
                }
            }
            any_neg |= (k[j] < 0);
        }
    }
    return wave_any(any_neg);
}


// Start of a slot j whose group enters later than the wave (its values are zero until then).
// ct: the m's row of the scaled table (1 / c_l for the entry of the scaled plain form)
// REFL: the slots run on the reflected (south) ring of their pair, m the order.
template <typename T, int R, int F, bool REFL = false>
__device__ __forceinline__ void inject(int l, const int (&e)[R], const int (&pr)[R], const Ent64 *__restrict__ ent,
                                       const int *__restrict__ entk, int64_t row, int npairs, T (&c2)[R], T (&p2)[R],
                                       T (&cm)[R], T (&pm)[R], int (&k)[R], const_as<Coef64S> *ct, int m = 0)
{
    const int refl = REFL ? (((l + m) & 1) ? -1 : 1) : 0;
#pragma unroll
    for (int j = 0; j < R; ++j)
        if (e[j] == l && pr[j] < npairs)
            load_entry<T, F>(ent, entk, row + pr[j], c2[j], p2[j], cm[j], pm[j], k[j], ct[l].ic, ct[l - 1].ic, refl);
}

template <int R> __device__ __forceinline__ bool pending(int l, int lmax, const int (&e)[R])
{
    bool q = false;
#pragma unroll
    for (int j = 0; j < R; ++j) q |= (e[j] > l && e[j] <= lmax);
    return q;
}

// Synthesis over a list of 64-pair groups: wave w of the launch holds the groups glist[w R + j],
// j < R, of every m (ngl entries; a slot past the list holds nothing).  CLS selects the rings it
// writes F for (GCLS_BOTH, GCLS_NORTH, GCLS_SOUTH).
template <typename T, int R, int V, int F, int CLS>
__global__ __launch_bounds__(256) void k_leg_synth(const SynRec<T> *__restrict__ recs, int64_t rec_stride,
                                                   const float4 *__restrict__ recus, const Coef64S *__restrict__ cs64,
                                                   const Coef32D *__restrict__ coefd, cplx<T> *__restrict__ FG,
                                                   int64_t fg_stride, const Ent64 *__restrict__ ent,
                                                   const int *__restrict__ entk, const int *__restrict__ entl,
                                                   int ng64, const double *__restrict__ pair_z, int lmax, int npairs,
                                                   int nrings, const int *__restrict__ glist, int ngl, int nbm)
{
    const int rhs = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    int m, blk;
    xcd_map((int)blockIdx.x, nbm, m, blk);
    const int li0 = (blk * 4 + wave) * R;  // first list entry of the wave
    if (m > lmax || li0 >= ngl) return;
    const int l0 = m > 2 ? m : 2;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const SynRec<T> *rec = recs + rhs * rec_stride + base;
    const float4 *recu = F ? recus + rhs * rec_stride + base : nullptr;
    const Coef32D *cfd = coefd + base;
    const_as<Coef64S> *ct = uniform_ptr(cs64 + base);
    const SynSrc<T, F> src(rec, recu, cfd);
    // one-ring classes of the plain form run on their own ring (the south class from reflected entry
    // states at the south ring's cos(theta)) and need no split of the sums by the parity of l + m
    constexpr bool DIRECT = CLS != GCLS_BOTH && F == 0, REFL = DIRECT && CLS == GCLS_SOUTH;
    auto rload = [&](int i) {
        if constexpr (F == 0) return rec[i];
        else return src.at(i);
    };

    typename PosT<T, F>::type x[R];
    T c2[R], p2[R], cm[R], pm[R];
    int k[R], pr[R], e[R];
    T acc0[8][R], acc1[8][R];
    // entry degree of each slot's 64-pair group; the wave starts at the earliest
    const_as<int> *el = uniform_ptr(entl + (int64_t)m * ng64);
    const_as<int> *gl = uniform_ptr(glist);
    int ls = ENT_SKIP;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int g = li0 + j < ngl ? gl[li0 + j] : -1;
        e[j] = g >= 0 ? el[g] : ENT_SKIP;
        ls = e[j] < ls ? e[j] : ls;
        pr[j] = g >= 0 ? g * 64 + lane : npairs;  // pairs at or past npairs hold nothing
    }
    const int64_t row = (int64_t)m * npairs;
    bool neg = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int p = pr[j];
        setpos(x[j], 0.0);
        c2[j] = p2[j] = cm[j] = pm[j] = (T)0;
        k[j] = 0;
        if (p < npairs) {
            setpos(x[j], REFL ? -pair_z[p] : pair_z[p]);
            if (e[j] == ls && ls <= lmax)
                load_entry<T, F>(ent, entk, row + p, c2[j], p2[j], cm[j], pm[j], k[j], ct[ls].ic, ct[ls - 1].ic,
                                 REFL ? (((ls + m) & 1) ? -1 : 1) : 0);
        }
        neg |= (k[j] < 0);
#pragma unroll
        for (int c = 0; c < 8; ++c) acc0[c][j] = acc1[c][j] = (T)0;
    }
    // Lanes whose scale exponent is still negative ("ramp") run the same unmasked steps: their
    // scaled values accumulate garbage that is discarded when the lane's exponent reaches zero (its
    // sums restart there) or at the end; the check runs once per trip of S steps, which the growth
    // of the recurrence over S steps keeps far from overflow.
    bool pend = R > 1 && pending<R>(ls, lmax, e);
    bool ramp = wave_any(neg);
    constexpr int S = V == 0 ? 2 : 4;
    int l = __builtin_amdgcn_readfirstlane(ls <= lmax ? ls : lmax + 1);
    SynSrc<T, F> rp(rec + l, F ? recu + l : nullptr, cfd + l);
    T(&accB)[8][R] = DIRECT ? acc0 : acc1;  // sums of the second step of a pair of steps
    auto a0 = rp.at(0), a1 = rp.at(1), b0 = a0, b1 = a1;
    for (; l + S - 1 <= lmax; l += S, rp.adv(S)) {
        if (pend) {
            // a slot enters at its group's entry degree (entries are l0 + 8q, trips start at ls + S q)
            inject<T, R, F, REFL>(l, e, pr, ent, entk, row, npairs, c2, p2, cm, pm, k, ct, m);
            pend = pending<R>(l, lmax, e);
            bool ng = false;
#pragma unroll
            for (int j = 0; j < R; ++j) ng |= (k[j] < 0);
            ramp = ramp || wave_any(ng);
        }
        if constexpr (S == 4) {
            // Scalar loads return out of order, so the wait before a record's first use covers
            // every load then in flight: each pair's loads are issued after the first step of the
            // pair before it (the scheduling barriers keep them there) and have that pair's second
            // step to arrive.
            syn_step<T, R, false, CLS, DIRECT>(a0, x, c2, p2, cm, pm, k, acc0);
            __builtin_amdgcn_sched_barrier(0);
            b0 = rp.at(2);
            b1 = rp.at(3);
            __builtin_amdgcn_sched_barrier(0);
            syn_step<T, R, false, CLS, DIRECT>(a1, x, c2, p2, cm, pm, k, accB);
            __builtin_amdgcn_sched_barrier(0);
            syn_step<T, R, false, CLS, DIRECT>(b0, x, c2, p2, cm, pm, k, acc0);
            __builtin_amdgcn_sched_barrier(0);
            a0 = rp.at(4);
            a1 = rp.at(5);
            __builtin_amdgcn_sched_barrier(0);
            syn_step<T, R, false, CLS, DIRECT>(b1, x, c2, p2, cm, pm, k, accB);
        } else {
            syn_step<T, R, false, CLS, DIRECT>(a0, x, c2, p2, cm, pm, k, acc0);
            syn_step<T, R, false, CLS, DIRECT>(a1, x, c2, p2, cm, pm, k, accB);
            a0 = rp.at(2);
            a1 = rp.at(3);
        }
        if (ramp) ramp = rescale_restart<T, R>(c2, p2, cm, pm, k, acc0, acc1);
    }
    // tail (fewer than S steps)
    for (int t = 0; l <= lmax; ++l, ++t) {
        if (pend) inject<T, R, F, REFL>(l, e, pr, ent, entk, row, npairs, c2, p2, cm, pm, k, ct, m);
        if (t & 1) syn_step<T, R, false, CLS, DIRECT>(rload(l), x, c2, p2, cm, pm, k, accB);
        else syn_step<T, R, false, CLS, DIRECT>(rload(l), x, c2, p2, cm, pm, k, acc0);
    }
    // lanes that never left the scaled range contribute nothing
#pragma unroll
    for (int j = 0; j < R; ++j)
        if (k[j] < 0) {
#pragma unroll
            for (int c = 0; c < 8; ++c) acc0[c][j] = acc1[c][j] = (T)0;
        }

    const bool odd0 = ((l0 + m) & 1) != 0;  // acc0 holds l + m odd terms when true
    cplx<T> *Fb = FG + rhs * fg_stride;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (pr[j] >= npairs) continue;
        if constexpr (DIRECT) {
            // F(m) = -(S+(u0), S+(u1)), F(-m) part = -(S-(u2), S-(u3)) on the ring the slot ran on
            const int r = REFL ? nrings - 1 - pr[j] : pr[j];
            if (REFL && r == pr[j]) continue;  // the equator ring belongs to the north side
            cplx<T> *f = Fb + ((int64_t)r * (lmax + 1) + m) * 2;
            f[0] = mk<T>(-acc0[0][j], -acc0[1][j]);
            f[1] = mk<T>(-acc0[2][j], -acc0[3][j]);
            continue;
        }
        T E[8], O[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            E[c] = odd0 ? acc1[c][j] : acc0[c][j];
            O[c] = odd0 ? acc0[c][j] : acc1[c][j];
        }
        const int rn = pr[j], rs = nrings - 1 - pr[j];
        // F(m) = -(S+(u0), S+(u1)), F(-m) part = -(S-(u2), S-(u3)) on the north ring; the south ring
        // takes the spin -2 sums for F(m) and spin +2 for the other, with the parity sign
        if (CLS != GCLS_SOUTH) {
            cplx<T> *f = Fb + ((int64_t)rn * (lmax + 1) + m) * 2;
            f[0] = mk<T>(-(E[0] + O[0]), -(E[1] + O[1]));
            f[1] = mk<T>(-(E[6] + O[6]), -(E[7] + O[7]));
        }
        if (CLS != GCLS_NORTH && rs != rn) {
            cplx<T> *f = Fb + ((int64_t)rs * (lmax + 1) + m) * 2;
            f[0] = mk<T>(-(E[4] - O[4]), -(E[5] - O[5]));
            f[1] = mk<T>(-(E[2] - O[2]), -(E[3] - O[3]));
        }
    }
}

// ================================================================================================
// Legendre adjoint: for one m and a block of ring pairs, the partial sums
//   2h_lm  = sum_r 2lambda_lm(theta_r) G_r(m),      -2h_lm = sum_r -2lambda_lm(theta_r) conj(G_r(-m))
// (south rings through the reflection symmetry).  Each lane sums its R ring pairs in registers;
// every L steps of l the per-lane partials go through LDS and are reduced over the workgroup.
// ================================================================================================
// CLS: GCLS_NORTH adds the north ring's four products only, GCLS_SOUTH the south ring's
template <typename T, int R, bool MASK, bool ODD, int CLS, typename C, typename X>
__device__ __forceinline__ void adj_step(const C &c, const X (&x)[R], T (&c2)[R],
                                         T (&p2)[R], T (&cm)[R], T (&pm)[R], const int (&k)[R],
                                         const cplx<T> (&GN)[R], const cplx<T> (&GS)[R], const cplx<T> (&HN)[R],
                                         const cplx<T> (&HS)[R], T (&out)[4])
{
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        T v2 = c2[j], vm = cm[j];
        if (MASK) {
            if (k[j] != 0) v2 = vm = (T)0;
        }
        const T s = ODD ? (T)-1 : (T)1;
        if (CLS != GCLS_SOUTH) {
            a0 = fma(v2, GN[j].x, a0);
            a1 = fma(v2, GN[j].y, a1);
            a2 = fma(vm, HN[j].x, a2);
            a3 = fma(vm, HN[j].y, a3);
        }
        if (CLS != GCLS_NORTH) {
            a0 = fma(s * vm, GS[j].x, a0);
            a1 = fma(s * vm, GS[j].y, a1);
            a2 = fma(s * v2, HS[j].x, a2);
            a3 = fma(s * v2, HS[j].y, a3);
        }
        rstep(c, x[j], c2[j], p2[j], cm[j], pm[j]);
    }
    out[0] = a0;
    out[1] = a1;
    out[2] = a2;
    out[3] = a3;
}

// Occupancy the adjoint is compiled for (waves per SIMD): the FP64 form with four ring pairs per
// lane would otherwise use about 175 registers and run two waves per SIMD, too few to hide its LDS
// round trips; at three the compiler spills only registers of the rarely taken group-entry path.
// The one-sided classes hold half of the G values (four registers less per pair in FP64) and fit
// four waves.  Eight pairs per lane cannot fit three waves without spilling in the inner loop: no
// target there.
template <typename T, int R, int CLS = GCLS_BOTH> struct AdjWaves {
    static constexpr bool two = CLS == GCLS_BOTH, fp64 = std::is_same<T, double>::value;
    static constexpr int value = R > 4 ? (two ? 1 : 2) : (fp64 && two) ? 3 : 4;
};
// Column reads the reduction of a chunk issues before it waits for them: each batch is one LDS
// round trip.  The one-sided FP64 forms with 5 to 7 pairs per lane run at two waves per SIMD with
// registers to spare for 16 values; the others keep 8.
template <typename T, int R, int CLS> struct AdjBatch {
    static constexpr int value = (std::is_same<T, double>::value && CLS != GCLS_BOTH && R >= 5 && R <= 7) ? 16 : 8;
};
// LDS hand-over between the lanes of a workgroup.  A single-wave workgroup needs no s_barrier: the
// LDS unit executes one wave's instructions in order, so a fence that keeps the compiler from moving
// LDS accesses across it suffices, and no full wait for outstanding LDS operations is forced.
// value of lane l ^ 1, l ^ 2 (DPP quad permutations) and of the mirrored lane in the half-row of
// 8 or the row of 16 lanes (row_half_mirror, row_mirror)
template <int CTRL> __device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_mov(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
// sum over the aligned group of G lanes (G = 1, 2, 4, 8, 16), in every lane of the group
template <int G, typename T> __device__ __forceinline__ T group_sum(T s)
{
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group size");
    if constexpr (G >= 2) s += dpp_mov<0xB1>(s);   // quad_perm [1, 0, 3, 2]
    if constexpr (G >= 4) s += dpp_mov<0x4E>(s);   // quad_perm [2, 3, 0, 1]
    if constexpr (G >= 8) s += dpp_mov<0x141>(s);  // row_half_mirror: lane 7 - i of the half-row
    if constexpr (G >= 16) s += dpp_mov<0x140>(s); // row_mirror: lane 15 - i of the row
    return s;
}

template <int W> __device__ __forceinline__ void wg_lds_sync()
{
    if constexpr (W == 1) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// The adjoint of one workgroup: m, its ring block rb, and its groups glist[lw .. lw + W R) (wave w
// the R of them from lw + w R; entries at or past ngl hold nothing).  red: the workgroup's LDS.
template <typename T, int R, int W, int L, int F, int CLS>
__device__ __forceinline__ void adj_body(T *__restrict__ red, const cplx<T> *__restrict__ FG,
                                         const typename CoefT<T, F>::type *__restrict__ coef,
                                         const Coef64S *__restrict__ cs64, const Ent64 *__restrict__ ent,
                                         const int *__restrict__ entk, const int *__restrict__ entl, int ng64,
                                         const double *__restrict__ pair_z, T *__restrict__ part,
                                         int *__restrict__ wgstart, int64_t nalm, int lmax, int npairs, int nrings,
                                         const int *__restrict__ glist, int ngl, const uint8_t *__restrict__ live,
                                         int nrb, int m, int rb, int lw)
{
    // LDS columns (wave, l, c) of 64 lanes, padded to CS entries: the G threads that sum one column
    // read entries gi + G t of it, and with CS = 64 + G (mod 32 double-banks) the 64 threads of a
    // wave spread over the banks twice each, as do the lane-contiguous writes
    constexpr int GR = 16 * W / L, CS = 64 + GR;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l0 = m > 2 ? m : 2;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const auto *cf = coef + base;
    const_as<Coef64S> *ct = uniform_ptr(cs64 + base);
    const T sgn0 = ((l0 + m) & 1) ? (T)-1 : (T)1;

    // entry degrees of the workgroup's 64-pair groups: the workgroup starts at the earliest, a slot
    // whose group enters later holds zeros until its entry (always at a chunk start: entries are
    // l0 + 8q and chunks start at l0 + Lq)
    const_as<int> *el = uniform_ptr(entl + (int64_t)m * ng64);
    const_as<int> *gl = uniform_ptr(glist);
    int ls = ENT_SKIP;
    for (int li = lw; li < lw + W * R && li < ngl; ++li) ls = el[gl[li]] < ls ? el[gl[li]] : ls;
    if (threadIdx.x == 0) wgstart[(int64_t)m * nrb + rb] = ls;
    if (ls > lmax) return;
    int e[R], pr[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int li = lw + wave * R + j;
        const int g = li < ngl ? gl[li] : -1;
        e[j] = g >= 0 ? el[g] : ENT_SKIP;
        pr[j] = g >= 0 ? g * 64 + lane : npairs;  // pairs at or past npairs hold nothing
    }
    const int64_t row = (int64_t)m * npairs;

    typename PosT<T, F>::type x[R];
    T c2[R], p2[R], cm[R], pm[R];
    int k[R];
    cplx<T> GN[R], GS[R], HN[R], HS[R];
    bool neg = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int p = pr[j];
        const cplx<T> z = mk<T>(0, 0);
        GN[j] = GS[j] = HN[j] = HS[j] = z;
        setpos(x[j], 0.0);
        c2[j] = cm[j] = p2[j] = pm[j] = (T)0;
        k[j] = 0;
        if (p < npairs) {
            setpos(x[j], pair_z[p]);
            if (e[j] == ls)
                load_entry<T, F>(ent, entk, row + p, c2[j], p2[j], cm[j], pm[j], k[j], ct[ls].ic, ct[ls - 1].ic);
        }
        neg |= (k[j] < 0);
    }
    // G of slot j's ring pair; lanes still in the scaled range (k < 0) hold G = 0, so the unmasked
    // steps add nothing for them until their exponent reaches zero and G is loaded
    auto load_g = [&](int j) {
        const int p = pr[j];
        if (p >= npairs || k[j] < 0) return;
        const int rn = p, rs = nrings - 1 - p;
        if (CLS != GCLS_SOUTH && (!live || live[rn])) {
            const cplx<T> *fn = FG + ((int64_t)rn * (lmax + 1) + m) * 2;
            GN[j] = fn[0];
            HN[j] = cconj<T>(fn[1]);
        }
        if (CLS != GCLS_NORTH && rs != rn && (!live || live[rs])) {
            const cplx<T> *fs = FG + ((int64_t)rs * (lmax + 1) + m) * 2;
            GS[j] = cscale<T>(fs[0], sgn0);
            HS[j] = cscale<T>(cconj<T>(fs[1]), sgn0);
        }
    };
#pragma unroll
    for (int j = 0; j < R; ++j)
        if (e[j] == ls) load_g(j);
    bool ramp = wave_any(neg);
    bool pend = (R > 1 || W > 1) && pending<R>(ls, lmax, e);
    constexpr int NT = 64 * W, NO = 4 * L, G = NT / NO;
    static_assert(G == GR && G >= 1 && 64 % G == 0 && NT % (4 * G) == 0, "reduction layout");
    const int t = threadIdx.x, o = t / G, gi = t - o * G;
    const int oli = o >> 2, oc = o & 3;
    const T *col = red + o * CS + gi;                                   // column o, entry gi
    T *pout = part + ((int64_t)rb * nalm + base + ls + oli) * 4 + oc;  // output of the first chunk

    using C = typename CoefT<T, F>::type;
    // coefficient records through an explicitly uniform pointer (scalar loads); the table is padded
    // past its last column, so the look-ahead loads stay in bounds
    const_as<C> *cp = uniform_ptr(cf + ls);
    C cc[L];
#pragma unroll
    for (int li = 0; li < L; ++li) cc[li] = ld_coef(cp + li);
    for (int lc = ls; lc <= lmax; lc += L, cp += L) {
        if (pend) {
            inject<T, R, F>(lc, e, pr, ent, entk, row, npairs, c2, p2, cm, pm, k, ct);
            bool ng = false;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (e[j] == lc) load_g(j);
                ng |= (k[j] < 0);
            }
            ramp = ramp || wave_any(ng);
            pend = pending<R>(lc, lmax, e);
        }
        // the next chunk's coefficients (scalar loads) are issued before this chunk's steps: they
        // share the LDS wait counter, and must have arrived by the time the reduction waits on LDS
        C nc[L];
#pragma unroll
        for (int li = 0; li < L; ++li) nc[li] = ld_coef(cp + L + li);
        // c_l of this thread's output row for the scaled plain form (a vector load, used at the store)
        T sc = (T)1;
        if constexpr (F == 0) sc = cf[lc + oli < lmax ? lc + oli : lmax].c;
        // all L steps unmasked: rows past lmax (last chunk) are reduced but not stored, and the
        // coefficient table is padded past its last column
#pragma unroll
        for (int li = 0; li < L; li += 2) {
            T out[4];
            adj_step<T, R, false, false, CLS>(cc[li], x, c2, p2, cm, pm, k, GN, GS, HN, HS, out);
#pragma unroll
            for (int c = 0; c < 4; ++c) red[((wave * L + li) * 4 + c) * CS + lane] = out[c];
            adj_step<T, R, false, true, CLS>(cc[li + 1], x, c2, p2, cm, pm, k, GN, GS, HN, HS, out);
#pragma unroll
            for (int c = 0; c < 4; ++c) red[((wave * L + li + 1) * 4 + c) * CS + lane] = out[c];
        }
        wg_lds_sync<W>();
        // column sums over the workgroup's lanes: thread (o, gi) reads the entries q = gi + G t of
        // column o (wave q / 64, lane q % 64) at compile-time offsets from its column base, all
        // reads first, adds them in four independent partial sums, then sums over the G adjacent
        // threads sharing the output with DPP lane moves
        // (in batches of AdjBatch reads, which bounds the registers they hold)
        constexpr int NR = NT / G, BR = NR < AdjBatch<T, R, CLS>::value ? NR : AdjBatch<T, R, CLS>::value;
        static_assert(NR >= 4 && NR % BR == 0, "four partial sums");
        T ps[4];
#pragma unroll
        for (int b0 = 0; b0 < NR; b0 += BR) {
            T rv[BR];
#pragma unroll
            for (int u = 0; u < BR; ++u) rv[u] = col[(G * (b0 + u) / 64) * (L * 4 * CS) + (G * (b0 + u)) % 64];
#pragma unroll
            for (int u = 0; u < BR; ++u) {
                if (b0 + u < 4) ps[u] = rv[u];
                else ps[(b0 + u) & 3] += rv[u];
            }
        }
        const T s = group_sum<G>((ps[0] + ps[1]) + (ps[2] + ps[3]));
        // the scaled plain form sums mu: the output of degree lc + oli is c_l times the sum
        if (gi == 0 && lc + oli <= lmax) pout[(int64_t)(lc - ls) * 4] = s * sc;
#pragma unroll
        for (int li = 0; li < L; ++li) cc[li] = nc[li];
        if (ramp) {
            // once per chunk (the growth over L steps stays far from overflow): rescale, and load
            // G for lanes whose exponent reached zero
            bool any_neg = false;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (k[j] < 0) {
                    const T big = fmax(fabs(c2[j]), fabs(cm[j]));
                    if (big > scale_hi<T>()) {
                        const T d = scale_down<T>();
                        c2[j] *= d;
                        p2[j] *= d;
                        cm[j] *= d;
                        pm[j] *= d;
                        k[j] += 1;
                        if (k[j] == 0) load_g(j);
                    }
                    any_neg |= (k[j] < 0);
                }
            }
            ramp = wave_any(any_neg);
        }
        wg_lds_sync<W>();
    }
}

// Adjoint over a list of 64-pair groups: workgroup b of the launch writes ring block rb0 + b of the
// nrb blocks of every m, from the groups adj_block gives it (glist[b W R ..] for W > 1; for W = 1
// the first nA workgroups take R groups each and the others R - 1, so that no slot is empty).  CLS
// selects the rings it reads (GCLS_BOTH, GCLS_NORTH, GCLS_SOUTH); a ring whose flag in live is zero
// is read as G = 0 (live null: every ring is read).
template <typename T, int R, int W, int L, int F, int CLS>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(AdjWaves<T, R, CLS>::value))) void k_leg_adj(const cplx<T> *__restrict__ FG,
                                                    const typename CoefT<T, F>::type *__restrict__ coef,
                                                    const Coef64S *__restrict__ cs64,
                                                    const Ent64 *__restrict__ ent, const int *__restrict__ entk,
                                                    const int *__restrict__ entl, int ng64,
                                                    const double *__restrict__ pair_z, T *__restrict__ part,
                                                    int *__restrict__ wgstart, int64_t nalm, int lmax, int npairs,
                                                    int nrings, const int *__restrict__ glist, int ngl,
                                                    const uint8_t *__restrict__ live, int rb0, int nrbl, int nrb,
                                                    int nA)
{
    constexpr int GR = 16 * W / L, CS = 64 + GR;
    __shared__ T red[W * L * 4 * CS];
    int m, rbl;
    xcd_map((int)blockIdx.x, nrbl, m, rbl);
    if (m > lmax) return;
    if constexpr (W == 1 && R > 1) {
        if (rbl >= nA) {
            adj_body<T, R - 1, 1, L, F, CLS>(red, FG, coef, cs64, ent, entk, entl, ng64, pair_z, part, wgstart, nalm,
                                             lmax, npairs, nrings, glist, ngl, live, nrb, m, rb0 + rbl,
                                             nA * R + (rbl - nA) * (R - 1));
            return;
        }
    }
    adj_body<T, R, W, L, F, CLS>(red, FG, coef, cs64, ent, entk, entl, ng64, pair_z, part, wgstart, nalm, lmax,
                                 npairs, nrings, glist, ngl, live, nrb, m, rb0 + rbl, rbl * W * R);
}

// ================================================================================================
// launch helpers (host): the translation units akra_leg_both/north/south.hip instantiate
// leg_synth_cls and leg_adj_cls for one class each
// ================================================================================================
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
// orders per XCD of a launch placed by xcd_map: 8 of them cover 32 ceil((lmax + 1) / 32) >= lmax + 1
inline int64_t xcd_slots(int lmax) { return 4 * cdiv(lmax + 1, 32); }

// synthesis waves (four per workgroup, R list entries each) over glist[0 .. ngl)
template <typename T, int R, int V, int F, int CLS>
void syn_launch(Plan &P, int nrhs, int64_t fg_stride, const int *glist, int ngl)
{
    if (ngl <= 0) return;
    const int nbm = (int)cdiv(cdiv(ngl, R), 4);  // workgroups per m
    dim3 g((unsigned)(8 * nbm * xcd_slots(P.lmax)), nrhs);
    k_leg_synth<T, R, V, F, CLS><<<g, 256, 0, P.stream>>>((const SynRec<T> *)P.d_rec, P.rec_stride, P.d_recu,
                                                          P.d_coef64s, P.d_coef32d, (cplx<T> *)P.d_FG, fg_stride,
                                                          P.d_ent, P.d_entk, P.d_entl, P.ng64, P.d_pair_z, P.lmax,
                                                          P.npairs, P.nrings, glist, ngl, nbm);
}

// launch shape of a class: the two-sided class takes (syn_V, syn_R, adj_R, adj_W, adj_L), the
// one-sided classes (syn_V1, syn_R1, adj_R1, adj_W1, adj_L1)
inline int syn_V_of(const Plan &P, int cls) { return cls == GCLS_BOTH ? P.syn_V : P.syn_V1; }
inline int syn_R_of(const Plan &P, int cls) { return cls == GCLS_BOTH ? P.syn_R : P.syn_R1; }
inline void adj_shape_of(const Plan &P, int cls, int &R, int &W, int &L)
{
    R = cls == GCLS_BOTH ? P.adj_R : P.adj_R1;
    W = cls == GCLS_BOTH ? P.adj_W : P.adj_W1;
    L = cls == GCLS_BOTH ? P.adj_L : P.adj_L1;
}

template <typename T, int V, int CLS>
void syn_dispatch_r(Plan &P, int nrhs, int64_t fg_stride, const int *glist, int ngl)
{
    const int R = syn_R_of(P, CLS);
    if (R == 1) syn_launch<T, 1, V, 0, CLS>(P, nrhs, fg_stride, glist, ngl);
    else if (R == 2) syn_launch<T, 2, V, 0, CLS>(P, nrhs, fg_stride, glist, ngl);
    else syn_launch<T, 4, V, 0, CLS>(P, nrhs, fg_stride, glist, ngl);
}

// Legendre synthesis of the groups list[0 .. npol + nmain) of class CLS: the first npol are
// near-polar groups of FP32 plans (difference form), the others run the plan's tuned shape
template <int CLS>
void leg_synth_cls(Plan &P, bool fp32, int nrhs, const int *list, int npol, int nmain)
{
    const int64_t fg_stride = (int64_t)P.nrings * (P.lmax + 1) * 2;
    const int V = syn_V_of(P, CLS);
    if (fp32) {
        // the near-polar and the other groups write F of disjoint rings: the near-polar launch (few
        // waves, long recurrences) beside the main one
        auto pol = [&]() { syn_launch<float, 1, 1, 1, CLS>(P, nrhs, fg_stride, list, npol); };
        auto rest = [&]() {
            if (V == 0) syn_dispatch_r<float, 0, CLS>(P, nrhs, fg_stride, list + npol, nmain);
            else syn_dispatch_r<float, 1, CLS>(P, nrhs, fg_stride, list + npol, nmain);
        };
        if (npol > 0 && nmain > 0) fork_join(P, pol, rest);
        else {
            pol();
            rest();
        }
    } else if (V == 0) {
        syn_dispatch_r<double, 0, CLS>(P, nrhs, fg_stride, list, npol + nmain);
    } else {
        syn_dispatch_r<double, 1, CLS>(P, nrhs, fg_stride, list, npol + nmain);
    }
}

// adjoint workgroups over glist[0 .. ngl) as split by sp (adj_split with this R, or RA, and W),
// writing ring blocks rb0 .. of the apply's nrb; returns the blocks written
template <typename T, int R, int W, int L, int F, int CLS>
int adj_launch(Plan &P, int rhs, const int *glist, int ngl, const AdjSplit &sp, const uint8_t *live, int rb0,
               int nrb)
{
    if (sp.q <= 0) return 0;
    const int64_t fg_stride = (int64_t)P.nrings * (P.lmax + 1) * 2;
    const void *coef = std::is_same<T, double>::value ? (const void *)P.d_coef64s
                       : F                              ? (const void *)P.d_coef32d
                                                        : (const void *)P.d_coef32s;
    dim3 g((unsigned)(8 * sp.q * xcd_slots(P.lmax)));
    k_leg_adj<T, R, W, L, F, CLS><<<g, 64 * W, 0, P.stream>>>(
        (const cplx<T> *)P.d_FG + rhs * fg_stride, (const typename CoefT<T, F>::type *)coef, P.d_coef64s, P.d_ent,
        P.d_entk, P.d_entl, P.ng64, P.d_pair_z, (T *)P.d_part, P.d_wgstart, P.nalm, P.lmax, P.npairs, P.nrings, glist,
        ngl, live, rb0, sp.q, nrb, sp.nA);
    return sp.q;
}

// single-wave workgroups of at most RMAX groups, spread evenly (adj_split): the kernel of RA = sp.RA
// groups per workgroup, whose later workgroups take RA - 1
template <typename T, int RMAX, int L, int F, int CLS>
int adj_launch_even(Plan &P, int rhs, const int *glist, int ngl, const AdjSplit &sp, const uint8_t *live, int rb0,
                    int nrb)
{
    if constexpr (RMAX > 1) {
        if (sp.RA < RMAX) return adj_launch_even<T, RMAX - 1, L, F, CLS>(P, rhs, glist, ngl, sp, live, rb0, nrb);
    }
    return adj_launch<T, RMAX, 1, L, F, CLS>(P, rhs, glist, ngl, sp, live, rb0, nrb);
}

// supported adjoint shapes (ring pairs per lane, waves per workgroup, l-chunk); the single-wave ones
// run through adj_launch_even
#define AKRA_ADJ_SHAPES_W1(X)                                                                          \
    X(1, 1, 8) X(2, 1, 8) X(3, 1, 8) X(4, 1, 8) X(5, 1, 8) X(6, 1, 8) X(7, 1, 8) X(8, 1, 8) X(1, 1, 4) X(2, 1, 4) \
        X(3, 1, 4) X(4, 1, 4) X(5, 1, 4) X(6, 1, 4) X(7, 1, 4) X(8, 1, 4)
#define AKRA_ADJ_SHAPES_WN(X) \
    X(1, 2, 8) X(1, 4, 8) X(2, 2, 8) X(2, 4, 8) X(4, 2, 8) X(4, 4, 8) X(8, 2, 8) X(2, 4, 4) X(4, 2, 4) X(4, 4, 4)
#define AKRA_ADJ_SHAPES(X) AKRA_ADJ_SHAPES_W1(X) AKRA_ADJ_SHAPES_WN(X)

template <typename T, int CLS>
int adj_dispatch(Plan &P, int rhs, const int *glist, int ngl, const uint8_t *live, int rb0, int nrb)
{
    int R, W, L;
    adj_shape_of(P, CLS, R, W, L);
    const AdjSplit sp = adj_split(ngl, R, W);
    if (W == 1) {
        if (L == 4) return adj_launch_even<T, 8, 4, 0, CLS>(P, rhs, glist, ngl, sp, live, rb0, nrb);
        return adj_launch_even<T, 8, 8, 0, CLS>(P, rhs, glist, ngl, sp, live, rb0, nrb);
    }
#define AKRA_ADJ_CASE(r, w, l) \
    if (R == r && W == w && L == l) return adj_launch<T, r, w, l, 0, CLS>(P, rhs, glist, ngl, sp, live, rb0, nrb);
    AKRA_ADJ_SHAPES_WN(AKRA_ADJ_CASE)
#undef AKRA_ADJ_CASE
    return adj_launch<T, 4, 4, 8, 0, CLS>(P, rhs, glist, ngl, adj_split(ngl, 4, 4), live, rb0, nrb);
}

// ring blocks the adjoint of a class list of npol near-polar and nmain other groups writes: the
// near-polar groups form blocks of at most adj_Rpol (difference form in FP32 plans; FP64 applies of
// such plans keep the same layout), the others blocks of the class's tuned adj_R adj_W
inline int adj_blocks(const Plan &P, int cls, int npol, int nmain)
{
    int R, W, L;
    adj_shape_of(P, cls, R, W, L);
    return adj_split(npol, P.adj_Rpol, 1).q + adj_split(nmain, R, W).q;
}

// Legendre adjoint of right-hand side rhs over list[0 .. npol + nmain) of class CLS into ring blocks
// rb0 .. of nrb; returns the blocks written
template <int CLS>
int leg_adj_cls(Plan &P, bool fp32, int rhs, const int *list, int npol, int nmain, const uint8_t *live, int rb0,
                int nrb)
{
    // the near-polar blocks first, then the others (in order: side by side the two launches took
    // longer than one after the other)
    const AdjSplit pol = adj_split(npol, P.adj_Rpol, 1);
    int n = 0;
    if (fp32) {
        n += adj_launch_even<float, 4, 4, 1, CLS>(P, rhs, list, npol, pol, live, rb0, nrb);
        n += adj_dispatch<float, CLS>(P, rhs, list + npol, nmain, live, rb0 + n, nrb);
    } else {
        n += adj_launch_even<double, 4, 4, 0, CLS>(P, rhs, list, npol, pol, live, rb0, nrb);
        n += adj_dispatch<double, CLS>(P, rhs, list + npol, nmain, live, rb0 + n, nrb);
    }
    return n;
}

extern template void leg_synth_cls<GCLS_BOTH>(Plan &, bool, int, const int *, int, int);
extern template void leg_synth_cls<GCLS_NORTH>(Plan &, bool, int, const int *, int, int);
extern template void leg_synth_cls<GCLS_SOUTH>(Plan &, bool, int, const int *, int, int);
extern template int leg_adj_cls<GCLS_BOTH>(Plan &, bool, int, const int *, int, int, const uint8_t *, int, int);
extern template int leg_adj_cls<GCLS_NORTH>(Plan &, bool, int, const int *, int, int, const uint8_t *, int, int);
extern template int leg_adj_cls<GCLS_SOUTH>(Plan &, bool, int, const int *, int, int, const uint8_t *, int, int);

}  // namespace akra
