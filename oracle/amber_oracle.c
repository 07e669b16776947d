/*
 * amber_oracle.c -- plain, slow, FP64 CPU oracle for the reionization-redshift
 * hot path of AMBER (Trac, Chen, Holst, Alvarez & Cen, "AMBER: A
 * Semi-numerical Abundance Matching Box for the Epoch of Reionization",
 * arXiv:2109.10375).
 *
 * TEST INFRASTRUCTURE.  This file exists to check the GPU library.  Only the
 * test suite, the package smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or constant generator with the
 * GPU library, and it never reads anything the GPU library produced.
 *
 * Every routine is the plain definition of what the method computes, written
 * out in FP64 (FP32 inputs are exact in FP64):
 *   - reionization history points   : Sec. 3.1.1, Eqs. (zear), (zlat)
 *   - Weibull history and inverse   : Sec. 3.1.2, Eq. (weibull) and its inverse
 *   - Weibull coefficient solve     : Appendix A (secant on f(c_w), then the
 *                                     algebraic a_w, b_w)
 *   - radiation field               : Sec. 3.4.1, Eq. (intensity), evaluated as
 *                                     a periodic convolution through discrete
 *                                     Fourier transforms, with the kernel's
 *                                     closed-form transform atan(k l)/k
 *   - abundance matching            : Sec. 3.4.2, the cumulative-mass equation
 *                                     (unnumbered) with weights 1+delta
 *   - two-point statistics          : Sec. 2.3, Eqs. (deltaz), (Pk), (Dk), (bias),
 *                                     (rcc): shell-averaged auto and cross spectra
 *   - halo source construction      : Sec. 3.2.1, Eqs. (interlace), (Wofk): mass
 *                                     assignment (NGP, CIC, TSC) to two meshes
 *                                     staggered by half a cell, combined and
 *                                     deconvolved in Fourier space
 *   - growth-rescaled matching      : Sec. 3.4.2, the cumulative-mass equation
 *                                     with delta_m(z_n) = D(z_n)/D(z_mid) delta_m,
 *                                     D the linear growth factor of the paper's
 *                                     flat cosmology (Sec. 2)
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *   R1 the spectral kernel is atan(k l_mfp)/k sampled at the discrete
 *      wavenumbers k_m = (2 pi / L)|m~|, m~ the signed integer frequency, with
 *      value l_mfp at k = 0;
 *   R2 the inverse transform carries the 1/N^3 normalisation;
 *   Z1 z_lat = z_ear - Delta_z (the middle expression printed for z_lat in
 *      Sec. 3.1.1 contradicts its own right-hand side and Table 1);
 *   Z2 a history is accepted when a_w, b_w, c_w > 0 and 0 < A_z <= 15;
 *   Z3 rank order: intensity descending, ties by ascending row-major cell
 *      index, -0 equal to +0, NaN rejected;
 *   Z4 the cumulative mass is the exact sum (fixed point), F_n = RN(C_n)/RN(C_N);
 *   Z5 F = 1 maps to z = a_w;
 *   Z6 contract inversion by monotone table interpolation (geometry below);
 *   Z7 weights are 1+delta at z_mid (growth factor ratio 1);
 *   D1 a field enters the spectra as given, as an overdensity f/mean - 1, or as
 *      the normalised redshift (f - mean)/(1 + mean) of Eq. (deltaz), the mean
 *      being the volume average;
 *   D2 spectra are shell averages over the full N^3 DFT grid: bin i holds the
 *      modes with i - 1/2 <= |m~| < i + 1/2, P = (L^3/N^6) <Re(A_m conj B_m)>,
 *      and the bin's k is (2 pi / L) times the mean |m~| of its modes;
 *   A1 halo positions are in length units in [0, L), periodic; mesh cell i
 *      spans [i, i+1) l_c with its node at the centre; NGP takes the cell
 *      holding the halo, CIC and TSC the 2 and 3 nearest nodes per axis with
 *      the linear and quadratic weights; the second mesh gets the positions
 *      shifted by +l_c/2 on every axis;
 *   A2 the combined spectrum of Eq. (interlace) is formed on the full DFT grid
 *      with k_d = (2 pi / L) m~_d (m~ the signed frequency, +N/2 at the
 *      Nyquist index) and the field is the real part of its inverse transform
 *      (the Hermitian part of the spectrum); without interlacing it is the
 *      first mesh's spectrum over W_pm;
 *   G1 D(a) is the growing mode of a flat universe of matter and a
 *      cosmological constant, normalised to a at early times; its ratio
 *      G_j = D(z_j)/D(z_mid) is tabulated at the inversion-table nodes;
 *   G2 with growth, rank n solves m_n(z)/M(z) = x_i(z) with the growth-weighted
 *      masses m_n = n (1 - g) + g C_n (C_n the exact prefix of w = 1 + delta),
 *      evaluated at the nodes with g = G_j; the root's bracket ends at the
 *      first node, walking up from z = a_w, where the growth-weighted ionized
 *      fraction exceeds x_i, and z is interpolated linearly inside it.
 *
 * Parity pins for each routine live in tests/test_oracle_*.py.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_HISTORY (-3)
#define OR_E_DATA (-7)
#define OR_E_RANGE (-8)

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* Reionization history: Sec. 3.1.1 and Sec. 3.1.2                          */
/* ------------------------------------------------------------------------ */

/* Eqs. (duration), (asymmetry) solved for the early and late redshifts:
 * z_ear = z_mid + Delta_z A_z / (1 + A_z), z_lat = z_ear - Delta_z  (reading Z1). */
int oracle_history_points(double z_mid, double delta_z, double a_z,
                          double* z_ear, double* z_lat) {
    if (!(delta_z > 0.0) || !(a_z > 0.0) || !isfinite(z_mid)) return OR_E_ARG;
    *z_ear = z_mid + delta_z * a_z / (1.0 + a_z);
    *z_lat = *z_ear - delta_z;
    return OR_OK;
}

/* Eq. (weibull): x_i(z) = exp[-max((z - a_w)/b_w, 0)^c_w]. */
double oracle_weibull_x(double z, double a, double b, double c) {
    double u = (z - a) / b;
    if (u < 0.0) u = 0.0;
    return exp(-pow(u, c));
}

/* Inverse of Eq. (weibull): z = a_w + b_w |ln x|^(1/c_w). */
double oracle_weibull_z(double x, double a, double b, double c) {
    return a + b * pow(fabs(log(x)), 1.0 / c);
}

/* Appendix A: f(c_w) = (ln x_ear / ln x_mid)^(1/c_w) - (z_ear - a)/(z_mid - a),
 * a = (z_lat |ln x_mid|^(1/c) - z_mid |ln x_lat|^(1/c)) /
 *     (|ln x_mid|^(1/c) - |ln x_lat|^(1/c)). */
static double weibull_f(double c, double z_ear, double z_mid, double z_lat,
                        double x_ear, double x_mid, double x_lat) {
    double pm = pow(fabs(log(x_mid)), 1.0 / c);
    double pl = pow(fabs(log(x_lat)), 1.0 / c);
    double a = (z_lat * pm - z_mid * pl) / (pm - pl);
    return pow(log(x_ear) / log(x_mid), 1.0 / c) - (z_ear - a) / (z_mid - a);
}

/* Appendix A: root of f(c_w) by the secant method (Newton with a finite
 * difference), kept inside a sign-change bracket so that it always converges;
 * then the algebraic a_w and b_w.  Ionization points default to
 * (0.05, 0.5, 0.95) (Sec. 3.1.1) when passed as 0. */
int oracle_weibull_fit(double z_mid, double delta_z, double a_z,
                       double x_ear, double x_mid, double x_lat,
                       double* a_w, double* b_w, double* c_w) {
    double z_ear, z_lat;
    if (x_ear == 0.0) x_ear = 0.05;
    if (x_mid == 0.0) x_mid = 0.5;
    if (x_lat == 0.0) x_lat = 0.95;
    if (!(0.0 < x_ear && x_ear < x_mid && x_mid < x_lat && x_lat < 1.0)) return OR_E_ARG;
    if (oracle_history_points(z_mid, delta_z, a_z, &z_ear, &z_lat) != OR_OK) return OR_E_ARG;
    if (a_z > 15.0) return OR_E_HISTORY;

    /* f > 0 for small c_w and f < 0 for large c_w whenever a root exists; scan
     * powers of two for a sign change. */
    double lo = 0.0, hi = 0.0, flo = 0.0, fhi = 0.0;
    int found = 0;
    double cprev = ldexp(1.0, -6);
    double fprev = weibull_f(cprev, z_ear, z_mid, z_lat, x_ear, x_mid, x_lat);
    for (int k = -5; k <= 12; ++k) {
        double cc = ldexp(1.0, k);
        double fc = weibull_f(cc, z_ear, z_mid, z_lat, x_ear, x_mid, x_lat);
        if (isfinite(fprev) && isfinite(fc) && fprev > 0.0 && fc <= 0.0) {
            lo = cprev; hi = cc; flo = fprev; fhi = fc; found = 1;
            break;
        }
        cprev = cc; fprev = fc;
    }
    if (!found) return OR_E_HISTORY;
    if (fhi == 0.0) {
        lo = hi; flo = fhi;
    }
    /* Secant iterates (c0, c1); fall back to bisection when the secant step
     * leaves the bracket. */
    double c0 = lo, f0 = flo, c1 = hi, f1 = fhi, c = hi;
    for (int it = 0; it < 400 && lo != hi; ++it) {
        double cn;
        if (f1 != f0) cn = c1 - f1 * (c1 - c0) / (f1 - f0);
        else cn = 0.5 * (lo + hi);
        if (!(cn > lo && cn < hi)) cn = 0.5 * (lo + hi);
        double fn = weibull_f(cn, z_ear, z_mid, z_lat, x_ear, x_mid, x_lat);
        c = cn;
        if (fn == 0.0) break;
        if (fn > 0.0) { lo = cn; flo = fn; } else { hi = cn; fhi = fn; }
        if (fabs(cn - c1) <= 1e-15 * fabs(cn)) break;
        c0 = c1; f0 = f1; c1 = cn; f1 = fn;
    }
    double pe = pow(fabs(log(x_ear)), 1.0 / c);
    double pm = pow(fabs(log(x_mid)), 1.0 / c);
    double pl = pow(fabs(log(x_lat)), 1.0 / c);
    double a = (z_ear * pl - z_lat * pe) / (pl - pe);
    double b = (z_mid - a) / pm;
    if (!(a > 0.0) || !(b > 0.0) || !(c > 0.0) || !isfinite(a) || !isfinite(b))
        return OR_E_HISTORY;
    *a_w = a; *b_w = b; *c_w = c;
    return OR_OK;
}

/* Contract-mode inversion table geometry (reading Z6):
 *   z_top = a + b * (64 ln 2)^(1/c)      (x_i(z_top) = 2^-64)
 *   h     = the smallest power of two >= (z_top - a) / 2^22
 *   T     = ceil((z_top - a) / h)         (T <= 2^22)
 *   nodes z_j = a + j h, X_j = x_i(z_j), j = 0..T. */
int oracle_table_geometry(double a, double b, double c,
                          double* h, int64_t* T, double* z_top) {
    if (!(a > 0.0) || !(b > 0.0) || !(c > 0.0)) return OR_E_HISTORY;
    double top = a + b * pow(64.0 * 0.69314718055994530942, 1.0 / c);
    double span = top - a;
    double r = span / 4194304.0;
    int e;
    double f = frexp(r, &e);           /* r = f 2^e, f in [0.5, 1) */
    double hh = (f == 0.5) ? r : ldexp(1.0, e);
    *h = hh;
    *T = (int64_t)ceil(span / hh);
    *z_top = top;
    return OR_OK;
}

int oracle_table(double a, double b, double c, double h, int64_t T, double* X) {
    for (int64_t j = 0; j <= T; ++j) {
        double z = a + (double)j * h;
        X[j] = exp(-pow((z - a) / b, c));
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Radiation field: Sec. 3.4.1                                              */
/* ------------------------------------------------------------------------ */

/* Signed frequency of index m on an n-point periodic axis. */
static int signed_freq(int m, int n) { return (2 * m <= n) ? m : m - n; }

/* Fourier transform of exp(-r/l)/(4 pi r^2): (1/k) int_0^inf e^(-r/l) sin(kr)/r dr
 * = atan(k l)/k, and l at k = 0. */
double oracle_kernel_hat(double k, double l_mfp) {
    if (k == 0.0) return l_mfp;
    return atan(k * l_mfp) / k;
}

static void twiddles(int n, double* cs, double* sn) {
    for (int j = 0; j < n; ++j) {
        double t = 2.0 * M_PI * (double)j / (double)n;
        cs[j] = cos(t);
        sn[j] = sin(t);
    }
}

/* One axis of the 3D DFT of a complex n^3 array (row-major, z fastest):
 * out[.., k, ..] = sum_j in[.., j, ..] exp(sign * 2 pi i j k / n), with the
 * angle reduced by the exact integer (j k) mod n. */
static void dft_axis(int n, double* re, double* im, int axis, int sign,
                     const double* cs, const double* sn) {
    const int64_t n2 = (int64_t)n * n;
    const int64_t stride = (axis == 0) ? n2 : (axis == 1) ? n : 1;
#pragma omp parallel
    {
        double* lr = (double*)malloc(sizeof(double) * (size_t)n);
        double* li = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t line = 0; line < n2; ++line) {
            int64_t p = line / n, q = line % n, base;
            if (axis == 0) base = p * n + q;
            else if (axis == 1) base = p * n2 + q;
            else base = p * n2 + q * n;
            for (int j = 0; j < n; ++j) {
                lr[j] = re[base + j * stride];
                li[j] = im[base + j * stride];
            }
            for (int k = 0; k < n; ++k) {
                double sr = 0.0, si = 0.0;
                for (int j = 0; j < n; ++j) {
                    int t = (int)(((int64_t)j * k) % n);
                    double c = cs[t], s = sign * sn[t];
                    sr += lr[j] * c - li[j] * s;
                    si += lr[j] * s + li[j] * c;
                }
                re[base + k * stride] = sr;
                im[base + k * stride] = si;
            }
        }
        free(lr);
        free(li);
    }
}

/* Full 3D DFT (sign -1 forward, +1 inverse, unnormalised), in place. */
int oracle_dft3(int n, double* re, double* im, int sign) {
    if (n < 1 || (sign != 1 && sign != -1)) return OR_E_ARG;
    double* cs = (double*)malloc(sizeof(double) * (size_t)n);
    double* sn = (double*)malloc(sizeof(double) * (size_t)n);
    twiddles(n, cs, sn);
    for (int axis = 0; axis < 3; ++axis) dft_axis(n, re, im, axis, sign, cs, sn);
    free(cs);
    free(sn);
    return OR_OK;
}

/* J = IDFT[ DFT(S) * Khat(|k|; l_mfp) ] / n^3 (real part), Sec. 3.4.1 with
 * readings R1, R2.  imag_max receives max |Im J| (a self-check). */
int oracle_radiation(int n, double box_len, const double* src, double l_mfp,
                     double* J, double* imag_max) {
    if (n < 1 || !(box_len > 0.0) || !(l_mfp > 0.0)) return OR_E_ARG;
    const int64_t n3 = (int64_t)n * n * n;
    double* re = (double*)malloc(sizeof(double) * (size_t)n3);
    double* im = (double*)calloc((size_t)n3, sizeof(double));
    if (!re || !im) { free(re); free(im); return OR_E_ARG; }
    memcpy(re, src, sizeof(double) * (size_t)n3);
    oracle_dft3(n, re, im, -1);
    const double k0 = 2.0 * M_PI / box_len;
    for (int mx = 0; mx < n; ++mx)
        for (int my = 0; my < n; ++my)
            for (int mz = 0; mz < n; ++mz) {
                int sx = signed_freq(mx, n), sy = signed_freq(my, n), sz = signed_freq(mz, n);
                double k = k0 * sqrt((double)sx * sx + (double)sy * sy + (double)sz * sz);
                double g = oracle_kernel_hat(k, l_mfp);
                int64_t i = ((int64_t)mx * n + my) * n + mz;
                re[i] *= g;
                im[i] *= g;
            }
    oracle_dft3(n, re, im, +1);
    double mi = 0.0;
    for (int64_t i = 0; i < n3; ++i) {
        J[i] = re[i] / (double)n3;
        double a = fabs(im[i] / (double)n3);
        if (a > mi) mi = a;
    }
    if (imag_max) *imag_max = mi;
    free(re);
    free(im);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Two-point statistics: Sec. 2.3, Eqs. (deltaz), (Pk), (bias), (rcc)        */
/* ------------------------------------------------------------------------ */

/* The field as it enters the spectra (reading D1): kind 0 as given, kind 1
 * the overdensity f/mean - 1, kind 2 the normalised redshift of Eq. (deltaz),
 * (f - mean)/(1 + mean), with the volume-weighted mean. */
static int spectra_field(int64_t n3, const double* f, int kind, double* out) {
    double mean = 0.0;
    for (int64_t i = 0; i < n3; ++i) mean += f[i];
    mean /= (double)n3;
    for (int64_t i = 0; i < n3; ++i) {
        if (kind == 0) out[i] = f[i];
        else if (kind == 1) out[i] = f[i] / mean - 1.0;
        else if (kind == 2) out[i] = (f[i] - mean) / (1.0 + mean);
        else return OR_E_ARG;
    }
    return OR_OK;
}

/* Shell index of a mode with integer |m~|^2 = s2 (reading D2): the i with
 * (2i - 1)^2 <= 4 s2 < (2i + 1)^2, decided in integers. */
static int64_t shell_of(int64_t s2) {
    int64_t i = (int64_t)floor(sqrt((double)s2));
    while (i * i > s2) --i;
    while ((i + 1) * (i + 1) <= s2) ++i;
    if (4 * s2 >= (2 * i + 1) * (2 * i + 1)) ++i;
    return i;
}

/* Auto and cross power spectra of fields a and b (Eq. Pk) in n_bins shells:
 * k[i], modes[i] (number of DFT modes), p_aa, p_bb, p_ab (reading D2).
 * Modes beyond the last shell are left out.  Naive DFTs, O(n^4). */
int oracle_spectra(int n, double box_len, const double* a, int kind_a, const double* b, int kind_b, int n_bins,
                   double* k, double* modes, double* p_aa, double* p_bb, double* p_ab) {
    if (n < 1 || !(box_len > 0.0) || n_bins < 1 || !a || !b) return OR_E_ARG;
    const int64_t n3 = (int64_t)n * n * n;
    double* ar = (double*)malloc(sizeof(double) * (size_t)n3);
    double* ai = (double*)calloc((size_t)n3, sizeof(double));
    double* br = (double*)malloc(sizeof(double) * (size_t)n3);
    double* bi = (double*)calloc((size_t)n3, sizeof(double));
    int rc = OR_E_ARG;
    if (ar && ai && br && bi && spectra_field(n3, a, kind_a, ar) == OR_OK &&
        spectra_field(n3, b, kind_b, br) == OR_OK) {
        oracle_dft3(n, ar, ai, -1);
        oracle_dft3(n, br, bi, -1);
        for (int i = 0; i < n_bins; ++i) k[i] = modes[i] = p_aa[i] = p_bb[i] = p_ab[i] = 0.0;
        for (int mx = 0; mx < n; ++mx)
            for (int my = 0; my < n; ++my)
                for (int mz = 0; mz < n; ++mz) {
                    const int64_t sx = signed_freq(mx, n), sy = signed_freq(my, n), sz = signed_freq(mz, n);
                    const int64_t s2 = sx * sx + sy * sy + sz * sz;
                    const int64_t sh = shell_of(s2);
                    if (sh >= n_bins) continue;
                    const int64_t i = ((int64_t)mx * n + my) * n + mz;
                    modes[sh] += 1.0;
                    k[sh] += sqrt((double)s2);
                    p_aa[sh] += ar[i] * ar[i] + ai[i] * ai[i];
                    p_bb[sh] += br[i] * br[i] + bi[i] * bi[i];
                    p_ab[sh] += ar[i] * br[i] + ai[i] * bi[i];
                }
        const double vol = box_len * box_len * box_len / ((double)n3 * (double)n3);
        const double k0 = 2.0 * M_PI / box_len;
        for (int i = 0; i < n_bins; ++i) {
            if (modes[i] > 0.0) {
                k[i] = k0 * k[i] / modes[i];
                p_aa[i] = vol * p_aa[i] / modes[i];
                p_bb[i] = vol * p_bb[i] / modes[i];
                p_ab[i] = vol * p_ab[i] / modes[i];
            }
        }
        rc = OR_OK;
    }
    free(ar); free(ai); free(br); free(bi);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Halo source fields: Sec. 3.2.1, Eqs. (interlace), (Wofk)                  */
/* ------------------------------------------------------------------------ */

/* Mass assignment of one coordinate (in cell units, nodes at i + 1/2) with a
 * window of order p (reading A1): the first node index and up to 3 weights. */
static int assign_1d(double x, int p, int64_t* i0, double* wgt) {
    if (p == 1) {
        *i0 = (int64_t)floor(x);
        wgt[0] = 1.0;
        return 1;
    }
    if (p == 2) {
        const double d = x - 0.5;
        const double f = floor(d);
        *i0 = (int64_t)f;
        wgt[1] = d - f;
        wgt[0] = 1.0 - wgt[1];
        return 2;
    }
    /* TSC: nearest node c = floor(x), offset u = x - (c + 1/2) in [-1/2, 1/2) */
    const double c = floor(x);
    const double u = x - (c + 0.5);
    *i0 = (int64_t)c - 1;
    wgt[0] = 0.5 * (0.5 - u) * (0.5 - u);
    wgt[1] = 0.75 - u * u;
    wgt[2] = 0.5 * (0.5 + u) * (0.5 + u);
    return 3;
}

static int64_t wrap(int64_t i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

/* Deposit halos (positions pos[3h..3h+2] in [0, L), masses) onto an n^3 mesh
 * with window order p, positions shifted by `shift` cells on every axis. */
static void deposit(int n, double box_len, int64_t n_halo, const float* pos, const float* mass, int p,
                    double shift, double* mesh) {
    const int64_t n3 = (int64_t)n * n * n;
    for (int64_t i = 0; i < n3; ++i) mesh[i] = 0.0;
    const double to_cell = (double)n / box_len;
    for (int64_t h = 0; h < n_halo; ++h) {
        int64_t i0[3];
        double w[3][3];
        int cnt = 0;
        for (int d = 0; d < 3; ++d) cnt = assign_1d((double)pos[3 * h + d] * to_cell + shift, p, &i0[d], w[d]);
        for (int a = 0; a < cnt; ++a)
            for (int b = 0; b < cnt; ++b)
                for (int c = 0; c < cnt; ++c) {
                    const int64_t ix = wrap(i0[0] + a, n), iy = wrap(i0[1] + b, n), iz = wrap(i0[2] + c, n);
                    mesh[(ix * n + iy) * n + iz] += (double)mass[h] * w[0][a] * w[1][b] * w[2][c];
                }
    }
}

/* Radiation field of a halo catalogue (Sec. 3.2.1 and Sec. 3.4.1, readings A1,
 * A2, R1, R2): meshes rho_1 (positions as given) and rho_2 (shifted by +l_c/2),
 * rho(k) = [rho_1(k) + e^{i k.dx} rho_2(k)] / 2 / W_pm(k) (or rho_1(k)/W_pm(k)
 * without interlacing), then J = Re IDFT[rho(k) Khat(|k|)] / n^3.  Naive DFTs. */
int oracle_radiation_from_halos(int n, double box_len, int64_t n_halo, const float* pos, const float* mass, int p,
                                int interlace, double l_mfp, double* J) {
    if (n < 1 || !(box_len > 0.0) || !(l_mfp > 0.0) || p < 1 || p > 3 || n_halo < 0) return OR_E_ARG;
    const int64_t n3 = (int64_t)n * n * n;
    double* ar = (double*)malloc(sizeof(double) * (size_t)n3);
    double* ai = (double*)calloc((size_t)n3, sizeof(double));
    double* br = (double*)malloc(sizeof(double) * (size_t)n3);
    double* bi = (double*)calloc((size_t)n3, sizeof(double));
    if (!ar || !ai || !br || !bi) { free(ar); free(ai); free(br); free(bi); return OR_E_ARG; }
    deposit(n, box_len, n_halo, pos, mass, p, 0.0, ar);
    oracle_dft3(n, ar, ai, -1);
    if (interlace) {
        deposit(n, box_len, n_halo, pos, mass, p, 0.5, br);
        oracle_dft3(n, br, bi, -1);
    }
    const double k0 = 2.0 * M_PI / box_len;
    for (int mx = 0; mx < n; ++mx)
        for (int my = 0; my < n; ++my)
            for (int mz = 0; mz < n; ++mz) {
                const int s[3] = {signed_freq(mx, n), signed_freq(my, n), signed_freq(mz, n)};
                double W = 1.0, theta = 0.0;
                for (int d = 0; d < 3; ++d) {
                    const double arg = M_PI * (double)s[d] / (double)n;   /* k_d l_c / 2 */
                    const double sinc = (s[d] == 0) ? 1.0 : sin(arg) / arg;
                    W *= pow(sinc, (double)p);
                    theta += arg;                                           /* k_d dx_d, dx_d = l_c/2 */
                }
                const int64_t i = ((int64_t)mx * n + my) * n + mz;
                double xr = ar[i], xi = ai[i];
                if (interlace) {
                    const double c = cos(theta), sn = sin(theta);
                    xr = 0.5 * (ar[i] + c * br[i] - sn * bi[i]);
                    xi = 0.5 * (ai[i] + c * bi[i] + sn * br[i]);
                }
                const double k = k0 * sqrt((double)s[0] * s[0] + (double)s[1] * s[1] + (double)s[2] * s[2]);
                const double g = oracle_kernel_hat(k, l_mfp) / W;
                ar[i] = xr * g;
                ai[i] = xi * g;
            }
    oracle_dft3(n, ar, ai, +1);
    for (int64_t i = 0; i < n3; ++i) J[i] = ar[i] / (double)n3;
    free(ar); free(ai); free(br); free(bi);
    return OR_OK;
}

/* The mesh of one deposit (for the assignment pins). */
int oracle_deposit(int n, double box_len, int64_t n_halo, const float* pos, const float* mass, int p,
                   double shift, double* mesh) {
    if (n < 1 || !(box_len > 0.0) || p < 1 || p > 3) return OR_E_ARG;
    deposit(n, box_len, n_halo, pos, mass, p, shift, mesh);
    return OR_OK;
}

/* Real-space periodic kernel g(n) = (1/n^3) sum_m Khat(k_m) e^{+2 pi i m.n/n},
 * by the direct (non-separable) triple sum; O(n^6), tiny n only. */
int oracle_kernel_real(int n, double box_len, double l_mfp, double* g) {
    if (n < 1 || n > 24) return OR_E_ARG;
    const double k0 = 2.0 * M_PI / box_len;
    const int64_t n3 = (int64_t)n * n * n;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n3; ++p) {
        int px = (int)(p / ((int64_t)n * n)), py = (int)((p / n) % n), pz = (int)(p % n);
        double s = 0.0;
        for (int mx = 0; mx < n; ++mx)
            for (int my = 0; my < n; ++my)
                for (int mz = 0; mz < n; ++mz) {
                    int sx = signed_freq(mx, n), sy = signed_freq(my, n), sz = signed_freq(mz, n);
                    double k = k0 * sqrt((double)sx * sx + (double)sy * sy + (double)sz * sz);
                    double ph = 2.0 * M_PI * (double)(((int64_t)mx * px + (int64_t)my * py + (int64_t)mz * pz) % n) / n;
                    s += oracle_kernel_hat(k, l_mfp) * cos(ph);
                }
        g[p] = s / (double)n3;
    }
    return OR_OK;
}

/* Brute-force periodic convolution J(n) = sum_{n'} S(n') g(n - n'); O(n^6). */
int oracle_direct_convolution(int n, double box_len, const double* src, double l_mfp, double* J) {
    if (n < 1 || n > 24) return OR_E_ARG;
    const int64_t n3 = (int64_t)n * n * n;
    double* g = (double*)malloc(sizeof(double) * (size_t)n3);
    oracle_kernel_real(n, box_len, l_mfp, g);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n3; ++p) {
        int px = (int)(p / ((int64_t)n * n)), py = (int)((p / n) % n), pz = (int)(p % n);
        double s = 0.0;
        for (int64_t q = 0; q < n3; ++q) {
            int qx = (int)(q / ((int64_t)n * n)), qy = (int)((q / n) % n), qz = (int)(q % n);
            int dx = (px - qx + n) % n, dy = (py - qy + n) % n, dz = (pz - qz + n) % n;
            s += src[q] * g[((int64_t)dx * n + dy) * n + dz];
        }
        J[p] = s;
    }
    free(g);
    return OR_OK;
}

/* One DFT coefficient of a real FP32 field: sum_n f_n e^{-2 pi i m.n/N}.
 * O(N^3); used to check full-size GPU output at sampled wavevectors. */
int oracle_dft_coeff_f32(int n, const float* f, int mx, int my, int mz,
                         double* out_re, double* out_im) {
    double* cs = (double*)malloc(sizeof(double) * (size_t)n);
    double* sn = (double*)malloc(sizeof(double) * (size_t)n);
    twiddles(n, cs, sn);
    double sr = 0.0, si = 0.0;
#pragma omp parallel for reduction(+ : sr, si) schedule(static)
    for (int x = 0; x < n; ++x)
        for (int y = 0; y < n; ++y) {
            const float* row = f + ((int64_t)x * n + y) * n;
            int64_t base = (int64_t)mx * x + (int64_t)my * y;
            for (int z = 0; z < n; ++z) {
                int t = (int)((base + (int64_t)mz * z) % n);
                sr += (double)row[z] * cs[t];
                si -= (double)row[z] * sn[t];
            }
        }
    *out_re = sr;
    *out_im = si;
    free(cs);
    free(sn);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Abundance matching: Sec. 3.4.2                                           */
/* ------------------------------------------------------------------------ */

struct rank_ctx { const float* v32; const double* v64; };

/* Descending value, ties by ascending cell index (reading Z3). */
static int rank_cmp(const void* pa, const void* pb, void* pctx) {
    const struct rank_ctx* ctx = (const struct rank_ctx*)pctx;
    uint32_t i = *(const uint32_t*)pa, j = *(const uint32_t*)pb;
    double x = ctx->v32 ? (double)ctx->v32[i] : ctx->v64[i];
    double y = ctx->v32 ? (double)ctx->v32[j] : ctx->v64[j];
    if (x > y) return -1;
    if (x < y) return 1;
    return (i < j) ? -1 : (i > j) ? 1 : 0;
}

static int rank_any(int64_t n, const float* v32, const double* v64, uint32_t* perm) {
    if (n < 0 || n > ((int64_t)1 << 32)) return OR_E_ARG;
    for (int64_t i = 0; i < n; ++i) {
        double v = v32 ? (double)v32[i] : v64[i];
        if (isnan(v)) return OR_E_DATA;
        perm[i] = (uint32_t)i;
    }
    struct rank_ctx ctx = {v32, v64};
    qsort_r(perm, (size_t)n, sizeof(uint32_t), rank_cmp, &ctx);
    return OR_OK;
}

/* The cells ordered by intensity, highest first (Sec. 3.4.2). */
int oracle_rank_f32(int64_t n, const float* J, uint32_t* perm) { return rank_any(n, J, NULL, perm); }
int oracle_rank_f64(int64_t n, const double* J, uint32_t* perm) { return rank_any(n, NULL, J, perm); }

/* Exact fixed-point decomposition of a positive finite FP32 weight:
 * w = m 2^q with q the exponent of w's unit in the last place as an FP32
 * number (q = e - 24 from w = f 2^e, f in [0.5, 1), but at least -149 for
 * subnormals), so m < 2^24 is an integer. */
static int weight_parts(float wf, uint64_t* m, int* q) {
    double w = (double)wf;
    if (!isfinite(w) || !(w > 0.0)) return OR_E_DATA;
    int e;
    frexp(w, &e);
    int qq = e - 24;
    if (qq < -149) qq = -149;
    *m = (uint64_t)ldexp(w, -qq);
    *q = qq;
    return OR_OK;
}

static int bit_length64(uint64_t v) {
    int b = 0;
    while (v) { ++b; v >>= 1; }
    return b;
}

struct mass_scale { int qmin; u128 total; };

static int mass_scale_of(int64_t n, const float* w, struct mass_scale* ms) {
    int qmin = 1 << 30;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t m = 0; int q = 0;
        if (weight_parts(w[i], &m, &q) != OR_OK) return OR_E_DATA;
        if (q < qmin) qmin = q;
    }
    /* The exact total of w 2^-qmin must stay below 2^127 (else a range error). */
    u128 tot = 0;
    const u128 lim = (u128)1 << 127;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t m = 0; int q = 0;
        weight_parts(w[i], &m, &q);
        int sh = q - qmin;
        if (sh + bit_length64(m) > 127) return OR_E_RANGE;
        u128 t = (u128)m << sh;
        if (t >= lim - tot) return OR_E_RANGE;
        tot += t;
    }
    ms->qmin = qmin;
    ms->total = tot;
    return OR_OK;
}

static u128 scaled_weight(float wf, int qmin) {
    uint64_t m = 0; int q = qmin;
    weight_parts(wf, &m, &q);
    return (u128)m << (q - qmin);
}

/* Cumulative ionized-mass fraction in rank order, Sec. 3.4.2:
 * F_n = RN(sum_{k<=n} w_perm[k]) / RN(sum_k w_k), sums exact (reading Z4). */
int oracle_mass_fraction(int64_t n, const uint32_t* perm, const float* w, double* F) {
    struct mass_scale ms;
    int rc = mass_scale_of(n, w, &ms);
    if (rc != OR_OK) return rc;
    const double tot = (double)ms.total;
    u128 c = 0;
    for (int64_t k = 0; k < n; ++k) {
        c += scaled_weight(w[perm[k]], ms.qmin);
        F[k] = (double)c / tot;
    }
    return OR_OK;
}

/* z = x_i^{-1}(F) by the closed form (exact mode) or by table interpolation
 * (contract mode), clamped to z_top (readings Z5, Z6). */
static double invert_exact(double F, double a, double b, double c, double z_top) {
    double z = a + b * pow(-log(F), 1.0 / c);
    return (z < z_top) ? z : z_top;
}

static double invert_table(double F, double a, double h, int64_t T, double z_top, const double* X) {
    /* j = max{ j in [0, T] : X_j >= F }; X_0 = 1 >= F. */
    int64_t lo = 0, hi = T;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo + 1) / 2;
        if (X[mid] >= F) lo = mid; else hi = mid - 1;
    }
    int64_t j = (lo > T - 1) ? T - 1 : lo;
    double zj = a + (double)j * h;
    double zj1 = a + (double)(j + 1) * h;
    double den = X[j] - X[j + 1];
    double t = (den != 0.0) ? (X[j] - F) / den : 0.0;
    double dz = zj1 - zj;
    double z = zj + t * dz;
    return (z < z_top) ? z : z_top;
}

/* ------------------------------------------------------------------------ */
/* Growth-rescaled matching: Sec. 3.4.2 with delta_m(z) = D(z)/D(z_mid) delta_m */
/* ------------------------------------------------------------------------ */

/* Gauss-Legendre rule of order n on [-1, 1]: the nodes are the roots of the
 * Legendre polynomial P_n, found by Newton's method from the standard
 * asymptotic starting values, with P_n and P_n' from the three-term recurrence
 * (k + 1) P_{k+1} = (2k + 1) x P_k - k P_{k-1}; the weights are
 * 2 / ((1 - x^2) P_n'(x)^2).  A textbook construction, exact for polynomials
 * of degree up to 2n - 1. */
int oracle_gauss_legendre(int n, double* x, double* w) {
    if (n < 1 || n > 512) return OR_E_ARG;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double t = cos(3.14159265358979323846 * ((double)i + 0.75) / ((double)n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;  /* P_0, P_1; after the loop P_{n-1}, P_n */
            for (int k = 1; k < n; ++k) {
                const double p2 = ((2.0 * k + 1.0) * t * p1 - (double)k * p0) / ((double)k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = (double)n * (t * p1 - p0) / (t * t - 1.0);
            const double step = p1 / dp;
            t -= step;
            if (fabs(step) <= 1e-16 * (1.0 + fabs(t))) {
                /* P_n' at the updated node */
                p0 = 1.0;
                p1 = t;
                for (int k = 1; k < n; ++k) {
                    const double p2 = ((2.0 * k + 1.0) * t * p1 - (double)k * p0) / ((double)k + 1.0);
                    p0 = p1;
                    p1 = p2;
                }
                dp = (double)n * (t * p1 - p0) / (t * t - 1.0);
                break;
            }
        }
        x[i] = -t;
        x[n - 1 - i] = t;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
    return OR_OK;
}

/* Linear growth factor (reading G1): the growing mode of a flat universe of
 * matter density omega_m and a cosmological constant 1 - omega_m,
 *   D(a) = (5 omega_m / 2) E(a) int_0^a da' / (a' E(a'))^3,
 *   E(a) = sqrt(omega_m a^-3 + 1 - omega_m),
 * normalised so that D = a while matter dominates.  With a' = s^2 the
 * integrand becomes the smooth 2 s^4 / (omega_m + (1 - omega_m) s^6)^(3/2) on
 * [0, sqrt(a)], integrated by one 64-point Gauss-Legendre rule (gx, gw). */
#define GROWTH_GL 64
static double growth_quadrature(double z, double omega_m, const double* gx, const double* gw) {
    const double a = 1.0 / (1.0 + z);
    const double r = sqrt(a);
    const double lam = 1.0 - omega_m;
    double sum = 0.0;
    for (int i = 0; i < GROWTH_GL; ++i) {
        const double s = 0.5 * r * (gx[i] + 1.0);
        const double s2 = s * s;
        const double q = omega_m + lam * s2 * s2 * s2;
        sum += gw[i] * (2.0 * s2 * s2 / (q * sqrt(q)));
    }
    const double integral = 0.5 * r * sum;
    const double E = sqrt(omega_m / (a * a * a) + lam);
    return 2.5 * omega_m * E * integral;
}

double oracle_growth(double z, double omega_m) {
    double gx[GROWTH_GL], gw[GROWTH_GL];
    oracle_gauss_legendre(GROWTH_GL, gx, gw);
    return growth_quadrature(z, omega_m, gx, gw);
}

/* G_j = D(z_j)/D(z_mid) at the table nodes z_j = a + j h, j = 0..T. */
int oracle_growth_table(double a, double h, int64_t T, double z_mid, double omega_m, double* G) {
    if (!(h > 0.0) || T < 1 || !(omega_m > 0.0) || !(omega_m <= 1.0)) return OR_E_ARG;
    double gx[GROWTH_GL], gw[GROWTH_GL];
    oracle_gauss_legendre(GROWTH_GL, gx, gw);
    const double dmid = growth_quadrature(z_mid, omega_m, gx, gw);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j <= T; ++j) G[j] = growth_quadrature(a + (double)j * h, omega_m, gx, gw) / dmid;
    return OR_OK;
}

/* h_j = m_j / M_j - X_j for the rank with k cells ionized (reading G2):
 * m_j = (k s)(1 - G_j) + G_j cn, M_j = (N s)(1 - G_j) + G_j cN, where s = 2^-qmin
 * puts the cell count in the units of the exact mass sums cn = RN(C_k) and
 * cN = RN(C_N).  A fixed operation order, no fused multiply-add. */
static double growth_gap(double ks, double ns, double cn, double cN, double G, double X) {
    const double one_m = 1.0 - G;
    const double m = ks * one_m + G * cn;
    const double M = ns * one_m + G * cN;
    return m / M - X;
}

/* z of one rank (reading G2): walking up the nodes from z_0 = a_w, the first
 * node j with h_j > 0.  None: z = z_top.  j = 0: z = a_w.  Otherwise the
 * bracket is (j - 1, j) and z = z_lo + t (z_hi - z_lo), t = -h_lo / (h_hi - h_lo),
 * clamped to z_top. */
static double invert_growth(double ks, double ns, double cn, double cN, double a, double h, int64_t T,
                            double z_top, const double* X, const double* G) {
    int64_t j = 0;
    double hj = growth_gap(ks, ns, cn, cN, G[0], X[0]);
    if (hj > 0.0) return a;
    double hprev = hj;
    for (j = 1; j <= T; ++j) {
        hj = growth_gap(ks, ns, cn, cN, G[j], X[j]);
        if (hj > 0.0) break;
        hprev = hj;
    }
    if (j > T) return z_top;
    const double zl = a + (double)(j - 1) * h;
    const double zh = a + (double)j * h;
    const double t = -hprev / (hj - hprev);
    const double z = zl + t * (zh - zl);
    return (z < z_top) ? z : z_top;
}

/* Full growth-rescaled match (readings G1, G2): ranking as in oracle_zre_*,
 * exact prefix masses, then each rank's node walk (independent per rank).
 * With n_sel > 0 only the ranks listed in sel are matched: z_sel[i] receives
 * the z of rank sel[i] and cell_sel[i] its cell (zre and zre64 are unused). */
int oracle_zre_growth_f32(int64_t n, const float* J, const float* w, double a, double h, int64_t T,
                          double z_top, const double* X, const double* G, float* zre, double* zre64,
                          int64_t n_sel, const int64_t* sel, float* z_sel, uint32_t* cell_sel) {
    uint32_t* perm = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    double* cn = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    struct mass_scale ms;
    int rc = rank_any(n, J, NULL, perm);
    if (rc == OR_OK) rc = mass_scale_of(n, w, &ms);
    for (int64_t i = 0; rc == OR_OK && i < n_sel; ++i)
        if (sel[i] < 0 || sel[i] >= n) rc = OR_E_ARG;
    if (rc == OR_OK) {
        const double s = ldexp(1.0, -ms.qmin);
        const double cN = (double)ms.total;
        const double ns = (double)n * s;
        u128 c = 0;
        for (int64_t k = 0; k < n; ++k) {
            c += scaled_weight(w[perm[k]], ms.qmin);
            cn[k] = (double)c;
        }
        if (n_sel > 0) {
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t i = 0; i < n_sel; ++i) {
                const int64_t k = sel[i];
                z_sel[i] = (float)invert_growth((double)(k + 1) * s, ns, cn[k], cN, a, h, T, z_top, X, G);
                cell_sel[i] = perm[k];
            }
        } else {
#pragma omp parallel for schedule(dynamic, 64)
            for (int64_t k = 0; k < n; ++k) {
                const double z = invert_growth((double)(k + 1) * s, ns, cn[k], cN, a, h, T, z_top, X, G);
                if (zre) zre[perm[k]] = (float)z;
                if (zre64) zre64[perm[k]] = z;
            }
        }
    }
    free(cn);
    free(perm);
    return rc;
}

/* Inversion of an array of mass fractions (used by the inversion pins). */
int oracle_invert(int64_t n, const double* F, double a, double b, double c, double h,
                  int64_t T, double z_top, const double* X, int mode, double* z) {
    for (int64_t k = 0; k < n; ++k) {
        if (!(F[k] > 0.0 && F[k] <= 1.0)) return OR_E_ARG;
        z[k] = (mode == 0) ? invert_exact(F[k], a, b, c, z_top)
                           : invert_table(F[k], a, h, T, z_top, X);
    }
    return OR_OK;
}

/* Full abundance match: rank (FP32 or FP64 intensity), exact cumulative mass,
 * inversion, z_re[perm[n]] = z_n.  mode 0 = exact, 1 = contract (table X of
 * T+1 entries with the geometry of oracle_table_geometry). */
static int zre_any(int64_t n, const float* J32, const double* J64, const float* w,
                   double a, double b, double c, double h, int64_t T, double z_top,
                   const double* X, int mode, float* zre, double* zre64, uint32_t* perm_out) {
    uint32_t* perm = perm_out ? perm_out : (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    double* F = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int rc = rank_any(n, J32, J64, perm);
    if (rc == OR_OK) rc = oracle_mass_fraction(n, perm, w, F);
    if (rc == OR_OK) {
        for (int64_t k = 0; k < n; ++k) {
            double z = (mode == 0) ? invert_exact(F[k], a, b, c, z_top)
                                   : invert_table(F[k], a, h, T, z_top, X);
            if (zre) zre[perm[k]] = (float)z;
            if (zre64) zre64[perm[k]] = z;
        }
    }
    free(F);
    if (!perm_out) free(perm);
    return rc;
}

int oracle_zre_f32(int64_t n, const float* J, const float* w, double a, double b, double c,
                   double h, int64_t T, double z_top, const double* X, int mode,
                   float* zre, double* zre64, uint32_t* perm) {
    return zre_any(n, J, NULL, w, a, b, c, h, T, z_top, X, mode, zre, zre64, perm);
}

int oracle_zre_f64(int64_t n, const double* J, const float* w, double a, double b, double c,
                   double h, int64_t T, double z_top, const double* X, int mode,
                   float* zre, double* zre64, uint32_t* perm) {
    return zre_any(n, NULL, J, w, a, b, c, h, T, z_top, X, mode, zre, zre64, perm);
}

/* z_re of selected cells one by one, O(n) each: C(i) = sum of w_j over the
 * cells ranked at or before i (descending J, ties by index). */
int oracle_zre_cells_f32(int64_t n, const float* J, const float* w, int64_t n_cells,
                         const int64_t* cells, double a, double b, double c,
                         double h, int64_t T, double z_top, const double* X, int mode,
                         float* zre_out, double* F_out) {
    struct mass_scale ms;
    for (int64_t i = 0; i < n; ++i)
        if (isnan(J[i])) return OR_E_DATA;
    int rc = mass_scale_of(n, w, &ms);
    if (rc != OR_OK) return rc;
    const double tot = (double)ms.total;
    for (int64_t s = 0; s < n_cells; ++s) {
        int64_t i = cells[s];
        if (i < 0 || i >= n) return OR_E_ARG;
        const float ji = J[i];
        u128 cum = 0;
#pragma omp parallel
        {
            u128 part = 0;
#pragma omp for schedule(static)
            for (int64_t j = 0; j < n; ++j) {
                if (J[j] > ji || (J[j] == ji && j <= i)) part += scaled_weight(w[j], ms.qmin);
            }
#pragma omp critical
            cum += part;
        }
        double F = (double)cum / tot;
        double z = (mode == 0) ? invert_exact(F, a, b, c, z_top) : invert_table(F, a, h, T, z_top, X);
        zre_out[s] = (float)z;
        if (F_out) F_out[s] = F;
    }
    return OR_OK;
}

/* Exact u128 -> double helper exposed for the rounding pins. */
double oracle_u128_to_double(uint64_t hi, uint64_t lo) {
    u128 v = ((u128)hi << 64) | lo;
    return (double)v;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
