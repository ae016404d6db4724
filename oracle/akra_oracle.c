/*
 * CPU oracle for the AKRA 3.0 spin-2 operator -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load
 * this library.  It shares no code with the HIP path and is deliberately plain
 * and slow: every sum is evaluated directly as it is defined.
 *
 *   * Spin-weighted harmonics (shear expansion, Sec. II.A, eq. shear_SH):
 *       sY_lm(theta, phi) = (-1)^s sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta) e^{i m phi}
 *     with the Wigner d^l_{m'm}(b) = <l m'| exp(-i b J_y) |l m>.  For s = +-2 the
 *     (-1)^s factor is 1, so  2lambda_lm = n_l d^l_{m,-2},  -2lambda_lm = n_l d^l_{m,+2}.
 *   * d^l is produced by the standard three-term recurrence in l, started from
 *     the closed form at l = max(|m|, |m'|), in x87 long double.  Values are kept
 *     as mantissa * 2^(SC_UNIT * k) with an integer k <= 0; a value is used only
 *     once k == 0 (anything smaller is below 2^-4096 and contributes nothing).
 *   * Negative m is computed explicitly (no symmetry shortcut), using the
 *     reality relation of a real field,  a_{l,-m} = (-1)^m conj(a_lm)  (Sec. II.A).
 *   * Ring transforms are direct sums over pixels / over m (no FFT).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

#define SC_UNIT 8192 /* binary exponent of one scale step */
#define SC_HI 4096   /* rescale once |mantissa| exceeds 2^SC_HI */

static const ld PI_L = 3.141592653589793238462643383279502884L;

static ld log2_binom(int n, int k)
{
    return (lgammal((ld)n + 1) - lgammal((ld)k + 1) - lgammal((ld)(n - k) + 1)) / logl(2.0L);
}

/* cos(theta/2), sin(theta/2) of the ring at z = cos(theta).  A ring is defined by
 * its double-precision z; 1 -+ z is exact in long double, so both half angles are
 * accurate to long-double precision even next to the poles. */
static void half_angles(ld z, ld *c, ld *s)
{
    *c = sqrtl((1 + z) / 2);
    *s = sqrtl((1 - z) / 2);
}

/* Closed form of d^j_{m,mp} at j = max(|m|,|mp|):
 *   d = sgn * sqrt(C(2j, kb)) * c^a * s^b,   c = cos(theta/2), s = sin(theta/2).
 * Returns sgn (0 when d vanishes exactly) and log2|d| in *l2. */
static int wigner_seed(int m, int mp, ld c, ld s, ld *l2)
{
    int am = abs(m), amp = abs(mp);
    int j = am > amp ? am : amp;
    int sgn, kb, a, b;
    if (j == m) { /* d^j_{j,mp} = (-1)^(j-mp) sqrt(C(2j,j+mp)) c^(j+mp) s^(j-mp) */
        sgn = ((j - mp) & 1) ? -1 : 1;
        kb = j + mp; a = j + mp; b = j - mp;
    } else if (j == -m) { /* d^j_{-j,mp} = sqrt(C(2j,j-mp)) c^(j-mp) s^(j+mp) */
        sgn = 1;
        kb = j - mp; a = j - mp; b = j + mp;
    } else if (j == mp) { /* d^j_{m,j} = sqrt(C(2j,j+m)) c^(j+m) s^(j-m) */
        sgn = 1;
        kb = j + m; a = j + m; b = j - m;
    } else { /* j == -mp:  d^j_{m,-j} = (-1)^(j+m) sqrt(C(2j,j-m)) c^(j-m) s^(j+m) */
        sgn = ((j + m) & 1) ? -1 : 1;
        kb = j - m; a = j - m; b = j + m;
    }
    if ((a > 0 && c == 0) || (b > 0 && s == 0)) return 0;
    *l2 = 0.5L * log2_binom(2 * j, kb) + (a ? (ld)a * log2l(c) : 0) + (b ? (ld)b * log2l(s) : 0);
    return sgn;
}

/* d^l_{m,mp}(theta) for l = 0..lmax (times sqrt((2l+1)/(4pi)) when norm != 0).
 * Entries with l < max(|m|,|mp|) are zero. */
static void wigner_column(int lmax, int m, int mp, ld c, ld s, ld z, int norm, ld *out)
{
    for (int l = 0; l <= lmax; l++) out[l] = 0;
    int am = abs(m), amp = abs(mp);
    int j = am > amp ? am : amp;
    if (j > lmax) return;
    ld l2 = 0;
    int sgn = wigner_seed(m, mp, c, s, &l2);
    if (!sgn) return;
    int k = (int)ceill(l2 / SC_UNIT);
    ld cur = (ld)sgn * exp2l(l2 - (ld)SC_UNIT * k), prev = 0;
    const ld hi = exp2l((ld)SC_HI);
    const ld mm = (ld)m * m, mpmp = (ld)mp * mp, mmp = (ld)m * mp;
    for (int l = j; l <= lmax; l++) {
        if (k == 0) out[l] = norm ? cur * sqrtl((2.0L * l + 1) / (4 * PI_L)) : cur;
        if (l == lmax) break;
        ld L = l, next;
        if (l == 0) {
            next = z * cur; /* m = mp = 0:  d^1_00 = cos(theta) */
        } else {
            /* l sqrt(((l+1)^2-m^2)((l+1)^2-mp^2)) d^{l+1}
             *   = (2l+1)(l(l+1) cos(theta) - m mp) d^l - (l+1) sqrt((l^2-m^2)(l^2-mp^2)) d^{l-1} */
            ld num1 = (2 * L + 1) * (L * (L + 1) * z - mmp);
            ld num2 = (L + 1) * sqrtl((L * L - mm) * (L * L - mpmp));
            ld den = L * sqrtl(((L + 1) * (L + 1) - mm) * ((L + 1) * (L + 1) - mpmp));
            next = (num1 * cur - num2 * prev) / den;
        }
        prev = cur;
        cur = next;
        if (k < 0 && fabsl(cur) > hi) {
            cur = ldexpl(cur, -SC_UNIT);
            prev = ldexpl(prev, -SC_UNIT);
            k++;
        }
    }
}

/* Public: one Wigner column in double precision (for the oracle's own pins). */
void orc_wigner_d(int lmax, int m, int mp, double z, int norm, double *out)
{
    ld c, s;
    ld *tmp = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
    half_angles(z, &c, &s);
    wigner_column(lmax, m, mp, c, s, z, norm, tmp);
    for (int l = 0; l <= lmax; l++) out[l] = (double)tmp[l];
    free(tmp);
}

static inline int64_t alm_index(int lmax, int l, int m)
{
    return (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
}

/* Full-m coefficient a_lm of a real field from its m >= 0 storage
 * (interleaved re, im); Im(a_l0) is not a degree of freedom and is ignored. */
static void alm_full(const double *a, int lmax, int l, int m, ld *re, ld *im)
{
    int am = abs(m);
    int64_t i = alm_index(lmax, l, am);
    ld r = a[2 * i], q = a[2 * i + 1];
    if (m == 0) q = 0;
    if (m < 0) {
        ld sg = (am & 1) ? -1 : 1;
        *re = sg * r;
        *im = -sg * q;
    } else {
        *re = r;
        *im = q;
    }
}

/* e^{i pi k / den}, k taken modulo 2*den. */
static void cis_frac(int64_t k, int64_t den, ld *c, ld *s)
{
    int64_t p = 2 * den;
    k %= p;
    if (k < 0) k += p;
    ld ang = PI_L * (ld)k / (ld)den;
    *c = cosl(ang);
    *s = sinl(ang);
}

/*
 * Synthesis Y: gamma = gamma_1 + i gamma_2 = sum_{l>=2} sum_{m=-l..l} 2a_lm 2Y_lm at pixel centres,
 * with 2a_lm = -(aE_lm + i aB_lm) (E/B decomposition, eq. EB_decomp).
 * Ring r has nphi[r] pixels at phi_j = pi*p0num/p0den + 2 pi j / nphi, starting at map offset ofs[r].
 * Only the nr rings passed are computed.
 */
void orc_synth(int lmax, const double *aE, const double *aB, int nr, const double *z,
               const int64_t *nphi, const int64_t *p0num, const int64_t *p0den, const int64_t *ofs,
               double *g1, double *g2)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < nr; r++) {
        ld c, s;
        half_angles(z[r], &c, &s);
        int nm = 2 * lmax + 1;
        ld *lam = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
        ld *Fr = (ld *)calloc((size_t)nm, sizeof(ld));
        ld *Fi = (ld *)calloc((size_t)nm, sizeof(ld));
        for (int m = -lmax; m <= lmax; m++) {
            wigner_column(lmax, m, -2, c, s, z[r], 1, lam); /* 2lambda_lm */
            ld sr = 0, si = 0;
            int l0 = abs(m) > 2 ? abs(m) : 2;
            for (int l = l0; l <= lmax; l++) {
                ld er, ei, br, bi;
                alm_full(aE, lmax, l, m, &er, &ei);
                alm_full(aB, lmax, l, m, &br, &bi);
                /* 2a = -(aE + i aB) */
                ld ar = -(er - bi), ai = -(ei + br);
                sr += ar * lam[l];
                si += ai * lam[l];
            }
            Fr[m + lmax] = sr;
            Fi[m + lmax] = si;
        }
        int64_t N = nphi[r];
        ld *ec = (ld *)malloc(sizeof(ld) * (size_t)N), *es = (ld *)malloc(sizeof(ld) * (size_t)N);
        for (int64_t k = 0; k < N; k++) cis_frac(2 * k, N, &ec[k], &es[k]); /* e^{2 pi i k / N} */
        /* fold the ring phase e^{i m phi0} into F */
        for (int m = -lmax; m <= lmax; m++) {
            ld pc, ps;
            cis_frac((int64_t)m * p0num[r], p0den[r], &pc, &ps);
            ld xr = Fr[m + lmax], xi = Fi[m + lmax];
            Fr[m + lmax] = xr * pc - xi * ps;
            Fi[m + lmax] = xr * ps + xi * pc;
        }
        for (int64_t j = 0; j < N; j++) {
            ld gr = 0, gi = 0;
            for (int m = -lmax; m <= lmax; m++) {
                int64_t k = ((int64_t)m * j) % N;
                if (k < 0) k += N;
                gr += Fr[m + lmax] * ec[k] - Fi[m + lmax] * es[k];
                gi += Fr[m + lmax] * es[k] + Fi[m + lmax] * ec[k];
            }
            g1[ofs[r] + j] = (double)gr;
            g2[ofs[r] + j] = (double)gi;
        }
        free(ec); free(es); free(lam); free(Fr); free(Fi);
    }
}

/*
 * Adjoint Y^H with respect to the pixel product  <g,h> = sum_p Omega_p Re(conj(g_p) h_p)
 * and the full-m harmonic product:
 *   2h_lm  = sum_p Omega_p conj(2Y_lm(p)) h_p,     -2h_lm = sum_p Omega_p conj(-2Y_lm(p)) conj(h_p),
 *   cE = -(2h + -2h)/2,   cB = (i/2)(2h - -2h)     (the E/B combination of eq. EB_decomp).
 * Computed for the m values in mlist (all l), summing over the nr rings passed.
 * cE, cB use the m >= 0 storage; entries for other m are left untouched.
 */
void orc_adjoint(int lmax, const double *g1, const double *g2, int nr, const double *z,
                 const int64_t *nphi, const int64_t *p0num, const int64_t *p0den, const int64_t *ofs,
                 const double *omega, int nmsel, const int *mlist, double *cE, double *cB)
{
    /* Step 1: per ring and per m, G = Omega sum_j h_j e^{-i m phi_j} and Gc = Omega sum_j conj(h_j) e^{-i m phi_j}. */
    double *G = (double *)malloc(sizeof(double) * 4 * (size_t)nr * (size_t)nmsel);
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < nr; r++) {
        int64_t N = nphi[r];
        ld *ec = (ld *)malloc(sizeof(ld) * (size_t)N), *es = (ld *)malloc(sizeof(ld) * (size_t)N);
        for (int64_t k = 0; k < N; k++) cis_frac(2 * k, N, &ec[k], &es[k]);
        for (int mi = 0; mi < nmsel; mi++) {
            int m = mlist[mi];
            ld pc, ps; /* e^{-i m phi0} */
            cis_frac(-(int64_t)m * p0num[r], p0den[r], &pc, &ps);
            ld ar = 0, ai = 0, br = 0, bi = 0;
            for (int64_t j = 0; j < N; j++) {
                int64_t k = ((int64_t)m * j) % N; /* e^{-i m 2 pi j/N} = conj(e^{2 pi i k/N}) */
                if (k < 0) k += N;
                ld cr = ec[k], ci = -es[k];
                ld hr = g1[ofs[r] + j], hi = g2[ofs[r] + j];
                ar += hr * cr - hi * ci;
                ai += hr * ci + hi * cr;
                br += hr * cr + hi * ci; /* conj(h) */
                bi += hr * ci - hi * cr;
            }
            ld w = omega[r];
            size_t o = 4 * ((size_t)r * (size_t)nmsel + (size_t)mi);
            G[o + 0] = (double)(w * (ar * pc - ai * ps));
            G[o + 1] = (double)(w * (ar * ps + ai * pc));
            G[o + 2] = (double)(w * (br * pc - bi * ps));
            G[o + 3] = (double)(w * (br * ps + bi * pc));
        }
        free(ec); free(es);
    }
    /* Step 2: per m, sum over rings of the Wigner columns against G. */
#pragma omp parallel for schedule(dynamic, 1)
    for (int mi = 0; mi < nmsel; mi++) {
        int m = mlist[mi];
        ld *l2 = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
        ld *lm2 = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
        ld *acc = (ld *)calloc(4 * (size_t)(lmax + 1), sizeof(ld));
        for (int r = 0; r < nr; r++) {
            ld c, s;
            half_angles(z[r], &c, &s);
            wigner_column(lmax, m, -2, c, s, z[r], 1, l2);  /* 2lambda  */
            wigner_column(lmax, m, +2, c, s, z[r], 1, lm2); /* -2lambda */
            size_t o = 4 * ((size_t)r * (size_t)nmsel + (size_t)mi);
            ld Gr = G[o], Gi = G[o + 1], Cr = G[o + 2], Ci = G[o + 3];
            for (int l = 2; l <= lmax; l++) {
                acc[4 * l + 0] += l2[l] * Gr;
                acc[4 * l + 1] += l2[l] * Gi;
                acc[4 * l + 2] += lm2[l] * Cr;
                acc[4 * l + 3] += lm2[l] * Ci;
            }
        }
        for (int l = 0; l <= lmax; l++) {
            if (l < m) continue;
            int64_t i = alm_index(lmax, l, m);
            ld pr = acc[4 * l], pi = acc[4 * l + 1], qr = acc[4 * l + 2], qi = acc[4 * l + 3];
            if (l < 2) pr = pi = qr = qi = 0;
            ld eR = -(pr + qr) / 2, eI = -(pi + qi) / 2;
            ld dR = pr - qr, dI = pi - qi; /* cB = (i/2) d */
            ld bR = -dI / 2, bI = dR / 2;
            if (m == 0) eI = bI = 0;
            cE[2 * i] = (double)eR;
            cE[2 * i + 1] = (double)eI;
            cB[2 * i] = (double)bR;
            cB[2 * i + 1] = (double)bI;
        }
        free(l2); free(lm2); free(acc);
    }
    free(G);
}
