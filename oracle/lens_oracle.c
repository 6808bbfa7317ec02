/*
 * lens_oracle.c -- plain FP64 CPU oracle for the batched lens log-likelihood.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the GPU path is checked against.  It is called only from
 * tests/, from the smoke check and from the CPU-baseline leg of bench.py.
 * It shares no code, header, table or constant with the GPU library, and the
 * GPU library never calls it.
 *
 * What it computes (Cao et al. 2025, "CSST Strong Lensing Preparation: Fast
 * Modelling of Galaxy-Galaxy Strong Lenses in the Big Data Era"):
 *   - lens equation beta = theta - alpha(theta)               (Sec. 2.1, Eq. 1)
 *   - image = lens light at theta + source light at beta       (Sec. 2.1, Eq. 2)
 *   - s x s supersampling, binned by the pixel mean            (Sec. 2.1, text after Eq. 2)
 *   - PSF convolution of the binned image                       (Sec. 2.1, Eq. 3)
 *   - Gaussian pixel likelihood over the fitting region         (Sec. 2.2, Eq. 5; mask: App. A)
 *   - elliptical Sersic light                                   (Sec. 2.4, Eqs. 8-10)
 *   - SIE mass = elliptical power law at slope 2                (Sec. 2.4, Eq. 12 and text)
 *   - external shear                                            (Sec. 2.4, Eqs. 13-14)
 *   - light amplitudes by non-negative least squares            (Sec. 2.3)
 *   - light models with one or two components per galaxy, and lens-only /
 *     source-only fits                           (Sec. 3.1.2, Sec. 3.2 set-ups)
 *   - a sampler loop whose proposals never leave the device (the direction of
 *     Sec. 4.2, against the transfer overhead of Sec. 3.1.4): the ensemble
 *     stretch move of Goodman & Weare (2010, CAMCoS 5, 65), driven by the
 *     Philox4x32-10 counter-based generator of Salmon et al. (2011, SC'11),
 *     with the posterior of Sec. 2.2 under a uniform box prior
 *
 * Everything is FP64, scalar loops, libm only, on the full supersampled grid
 * (no skipping outside the mask), with a full-image direct convolution.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   R1  SIE convergence kappa = theta_E / (2 R_p) with the paper's elliptical
 *       radius R_p = sqrt(q x1^2 + x2^2/q) of Eq. 10; its deflection is the
 *       closed form of Kormann et al. (1994) rewritten for this normalisation.
 *   R2  q = 1 uses the circular form alpha = theta_E x/|x|; alpha = 0 at the
 *       mass centre.
 *   R3  shear follows the sign printed in Eq. 13,
 *       psi = -1/2 [g1 (x^2 - y^2) + 2 g2 x y], so
 *       alpha_sh = -(g1 x + g2 y, g2 x - g1 y), with origin at (0, 0).
 *   R5  position angles are counter-clockwise from +x1 (the rotation in
 *       Eq. 10); x1 grows with the column index, x2 with the row index.
 *   R6  the image centre is at pixel ((nx-1)/2, (ny-1)/2).
 *   R7  sub-pixels are the centres of an s x s equal split of each pixel; the
 *       binned value is their arithmetic mean; lens light is supersampled too.
 *   R8  lens light centre = mass centre (Table 1).
 *   R9  b_n is the exact root of Gamma(2n) = 2 gamma(2n, b_n) (Eq. 9).
 *   R11 the PSF is a true convolution (kernel flipped), k odd, centred at
 *       (k-1)/2, zero outside the image, output of the image's size.
 *   R12 supersample -> bin -> convolve.
 *   R13 lnL = -1/2 chi^2 - 1/2 sum_mask ln(2 pi sigma^2), sums over the mask.
 *   R14 the power-law convergence of Sec. 2.4 is made elliptical on the same
 *       elliptical radius R_p as the SIE, so gamma = 2 is exactly reading R1.
 *
 * Parameter vector of one proposal: 20 doubles:
 *   0 theta_E  1 q_m  2 phi_m  3 x_m  4 y_m  5 g1  6 g2
 *   7 I_l  8 R_l  9 n_l  10 q_l  11 phi_l
 *   12 I_s 13 R_s 14 n_s 15 q_s 16 phi_s 17 x_s 18 y_s
 *   19 mass slope: 0 for the SIE (its closed form), gamma in [1.05, 2.95]
 *      for the elliptical power law
 * Angles in radians, positions and radii in arcsec.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NP 20

/* ------------------------------------------------------------------------ */
/* Regularised lower incomplete gamma P(a, x) = gamma(a, x) / Gamma(a).      */
/* Series for x < a + 1, continued fraction for Q = 1 - P otherwise          */
/* (the standard pair of expansions, e.g. Numerical Recipes 3rd ed. 6.2).    */
/* ------------------------------------------------------------------------ */
static double orc_gser(double a, double x)
{
    /* P(a,x) = e^{-x} x^a / Gamma(a+1) * sum_{k>=0} x^k / ((a+1)...(a+k)) */
    double term = 1.0, sum = 1.0, ap = a;
    for (int k = 1; k < 100000; ++k) {
        ap += 1.0;
        term *= x / ap;
        sum += term;
        if (term < sum * 1e-17) break;
    }
    return sum * exp(a * log(x) - x - lgamma(a + 1.0));
}

static double orc_gcf(double a, double x)
{
    /* Q(a,x) by the modified Lentz evaluation of the Legendre continued fraction */
    const double tiny = 1e-300;
    double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 100000; ++i) {
        double an = -i * (i - a);
        b += 2.0;
        d = an * d + b;
        if (fabs(d) < tiny) d = tiny;
        c = b + an / c;
        if (fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        double del = d * c;
        h *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return exp(a * log(x) - x - lgamma(a)) * h;
}

double oracle_gammainc_lower_reg(double a, double x)
{
    if (!(a > 0.0) || !(x >= 0.0)) return NAN;
    if (x == 0.0) return 0.0;
    if (x < a + 1.0) return orc_gser(a, x);
    return 1.0 - orc_gcf(a, x);
}

/* b_n: root of P(2n, b) = 1/2 (Sec. 2.4, Eq. 9), by plain bisection to the
 * last bit.  P is increasing in b, P(2n, 0) = 0 and P(2n, 2n + 1) > 1/2. */
double oracle_bn(double n)
{
    if (!(n > 0.0) || !isfinite(n)) return NAN;
    double a = 2.0 * n, lo = 0.0, hi = a + 1.0;
    while (oracle_gammainc_lower_reg(a, hi) < 0.5) hi *= 2.0;
    for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (oracle_gammainc_lower_reg(a, mid) < 0.5) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------------ */
/* Light: elliptical Sersic (Sec. 2.4, Eqs. 8 and 10)                        */
/* ------------------------------------------------------------------------ */
double oracle_sersic(double I_e, double R_e, double n, double b_n, double q,
                     double phi, double xc, double yc, double x, double y)
{
    double dx = x - xc, dy = y - yc;
    double x1 = dx * cos(phi) + dy * sin(phi);       /* Eq. 10, first row  */
    double x2 = -dx * sin(phi) + dy * cos(phi);      /* Eq. 10, second row */
    double R = sqrt(x1 * x1 * q + x2 * x2 / q);      /* Eq. 10, third row  */
    return I_e * exp(-b_n * (pow(R / R_e, 1.0 / n) - 1.0));   /* Eq. 8 */
}

/* ------------------------------------------------------------------------ */
/* Mass: SIE (reading R1/R2) and external shear (reading R3)                 */
/* ------------------------------------------------------------------------ */
void oracle_sie_deflection(double theta_E, double q, double phi, double xm,
                           double ym, double x, double y, double *ax, double *ay)
{
    double dx = x - xm, dy = y - ym;
    double c = cos(phi), s = sin(phi);
    double x1 = c * dx + s * dy;          /* frame of the mass ellipse (Eq. 10) */
    double x2 = -s * dx + c * dy;
    double a1, a2;
    if (x1 == 0.0 && x2 == 0.0) { *ax = 0.0; *ay = 0.0; return; }
    if (q == 1.0) {
        double r = sqrt(x1 * x1 + x2 * x2);
        a1 = theta_E * x1 / r;
        a2 = theta_E * x2 / r;
    } else {
        double e = sqrt(1.0 - q * q);
        double psi = sqrt(q * q * x1 * x1 + x2 * x2);
        double b = theta_E * sqrt(q);
        a1 = b / e * atan(e * x1 / psi);
        a2 = b / e * atanh(e * x2 / psi);
    }
    *ax = c * a1 - s * a2;                /* rotate back to the image frame */
    *ay = s * a1 + c * a2;
}

/* Elliptical power law (EPL; Sec. 2.4, the power-law convergence made
 * elliptical, reading R14): in the frame of the mass ellipse,
 *   kappa = (3 - gamma)/2 (theta_E / R_p)^(gamma - 1),  R_p = sqrt(q x1^2 + x2^2/q),
 * which is the SIE's kappa = theta_E / (2 R_p) at gamma = 2.  With
 * xi^2 = x1^2 + x2^2/q^2 (so R_p = sqrt(q) xi) the deflection of any convergence
 * constant on the ellipses xi = const is the classical pair of integrals
 *   a1 = q x1 J0,  a2 = q x2 J1,
 *   Jn = int_0^1 kappa(xi(u)) / d(u)^(n + 1/2) du,  d(u) = 1 - (1 - q^2) u,
 *   xi(u)^2 = u A(u),  A(u) = x1^2 + x2^2 / d(u)
 * (Schramm 1990; Keeton 2001, "A catalog of mass models", Sec. 2).  kappa(xi(u))
 * carries the factor u^(-(gamma-1)/2), singular at u = 0; with u = v^m,
 * m = 2 / (3 - gamma), that factor times du/dv is the constant m, and
 *   Jn = int_0^1 (theta_E^2 / (q A(v^m)))^((gamma-1)/2) / d(v^m)^(n + 1/2) dv,
 * a smooth integrand, taken by tanh-sinh quadrature (Takahasi & Mori 1974):
 * v = 1/(1 + e^(-pi sinh tau)), tau = k h, h = 1/64, |tau| <= 4. */
void oracle_epl_deflection(double theta_E, double gamma, double q, double phi, double xm, double ym,
                           double x, double y, double *ax, double *ay)
{
    double dx = x - xm, dy = y - ym;
    double c = cos(phi), s = sin(phi);
    double x1 = c * dx + s * dy;          /* frame of the mass ellipse (Eq. 10) */
    double x2 = -s * dx + c * dy;
    if ((x1 == 0.0 && x2 == 0.0) || theta_E == 0.0) { *ax = 0.0; *ay = 0.0; return; }
    const double h = 1.0 / 64.0, e2 = 1.0 - q * q, m = 2.0 / (3.0 - gamma);
    const double b2 = theta_E * theta_E / q, p = 0.5 * (gamma - 1.0);
    double J0 = 0.0, J1 = 0.0;
    for (int k = -256; k <= 256; ++k) {
        const double tau = k * h, sh = sinh(tau), ch = cosh(tau);
        const double ex = exp(-M_PI * sh);
        const double v = 1.0 / (1.0 + ex);                              /* (1 + tanh(pi/2 sinh tau))/2 */
        const double w = h * M_PI * ch * ex / ((1.0 + ex) * (1.0 + ex));   /* dv/dtau */
        if (!(w > 0.0) || !isfinite(w)) continue;
        const double u = pow(v, m), d = 1.0 - e2 * u;
        const double A = x1 * x1 + x2 * x2 / d;
        const double f = w * pow(b2 / A, p) / sqrt(d);
        J0 += f;
        J1 += f / d;
    }
    const double a1 = q * x1 * J0, a2 = q * x2 * J1;
    *ax = c * a1 - s * a2;                /* rotate back to the image frame */
    *ay = s * a1 + c * a2;
}

void oracle_shear_deflection(double g1, double g2, double x, double y,
                             double *ax, double *ay)
{
    /* gradient of psi = -1/2 [g1 (x^2 - y^2) + 2 g2 x y]  (Eq. 13 with Eq. 14) */
    *ax = -(g1 * x + g2 * y);
    *ay = -(g2 * x - g1 * y);
}

/* Total deflection of one proposal at (x, y).  Slot 19 selects the mass:
 * 0 the SIE by its closed form, gamma in (1, 3) the EPL (reading R14). */
void oracle_deflection(const double *p, double x, double y, double *ax, double *ay)
{
    double sx, sy, hx, hy;
    if (p[19] == 0.0)
        oracle_sie_deflection(p[0], p[1], p[2], p[3], p[4], x, y, &sx, &sy);
    else
        oracle_epl_deflection(p[0], p[19], p[1], p[2], p[3], p[4], x, y, &sx, &sy);
    oracle_shear_deflection(p[5], p[6], x, y, &hx, &hy);
    *ax = sx + hx;
    *ay = sy + hy;
}

/* ------------------------------------------------------------------------ */
/* Proposal domain                                                           */
/* ------------------------------------------------------------------------ */
#define ORC_N_MIN 0.1
#define ORC_N_MAX 20.0

#define ORC_GAMMA_MIN 1.05
#define ORC_GAMMA_MAX 2.95

int oracle_params_valid(const double *p)
{
    for (int i = 0; i < 19; ++i)
        if (!isfinite(p[i])) return 0;
    if (p[19] != 0.0 && !(p[19] >= ORC_GAMMA_MIN && p[19] <= ORC_GAMMA_MAX)) return 0;
    if (p[0] < 0.0) return 0;
    const int qs[3] = {1, 10, 15};
    for (int i = 0; i < 3; ++i)
        if (!(p[qs[i]] > 0.0 && p[qs[i]] <= 1.0)) return 0;
    if (!(p[8] > 0.0) || !(p[13] > 0.0)) return 0;
    if (!(p[9] >= ORC_N_MIN && p[9] <= ORC_N_MAX)) return 0;
    if (!(p[14] >= ORC_N_MIN && p[14] <= ORC_N_MAX)) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Image grid (readings R6, R7)                                              */
/* ------------------------------------------------------------------------ */
void oracle_subpixel_xy(int ny, int nx, double dpix, int s, int i, int j,
                        int v, int u, double *x, double *y)
{
    *x = ((double)j - 0.5 * (nx - 1) + ((double)u + 0.5) / s - 0.5) * dpix;
    *y = ((double)i - 0.5 * (ny - 1) + ((double)v + 0.5) / s - 0.5) * dpix;
}

/* Surface brightness of the lensed scene at one image-plane point (Eq. 2). */
static double orc_scene(const double *p, double bl, double bs, double x, double y)
{
    double ax, ay;
    oracle_deflection(p, x, y, &ax, &ay);
    double bx = x - ax, by = y - ay;                                   /* Eq. 1 */
    double lens = oracle_sersic(p[7], p[8], p[9], bl, p[10], p[11], p[3], p[4], x, y);
    double src = oracle_sersic(p[12], p[13], p[14], bs, p[15], p[16], p[17], p[18], bx, by);
    return lens + src;
}

/* 'same'-size true convolution with zero padding (Eq. 3, reading R11):
 *   out[i][j] = sum_{a,b} K[a][b] * img[i + r - a][j + r - b],  r = (k-1)/2 */
void oracle_convolve_same(const double *img, int ny, int nx, const double *psf,
                          int k, double *out)
{
    int r = (k - 1) / 2;
    for (int i = 0; i < ny; ++i)
        for (int j = 0; j < nx; ++j) {
            double acc = 0.0;
            for (int a = 0; a < k; ++a) {
                int ii = i + r - a;
                if (ii < 0 || ii >= ny) continue;
                for (int b = 0; b < k; ++b) {
                    int jj = j + r - b;
                    if (jj < 0 || jj >= nx) continue;
                    acc += psf[a * k + b] * img[ii * nx + jj];
                }
            }
            out[i * nx + j] = acc;
        }
}

static int orc_geom_ok(int ny, int nx, double dpix, int s, int k)
{
    return ny > 0 && nx > 0 && s > 0 && k > 0 && (k & 1) && dpix > 0.0 && isfinite(dpix);
}

/* Model image of one proposal.
 *   stage 0: binned, unconvolved          [ny][nx]
 *   stage 1: binned and PSF-convolved     [ny][nx]
 *   stage 2: the supersampled grid        [ny*s][nx*s], fine row i*s+v, col j*s+u
 * Returns 0 on success, -1 on a bad argument, -2 for a proposal outside the
 * domain (out is then untouched). */
int oracle_model_image(int ny, int nx, double dpix, int s, int k, const double *psf,
                       const double *p, int stage, double *out)
{
    if (!orc_geom_ok(ny, nx, dpix, s, k) || !p || !out) return -1;
    if (stage == 1 && !psf) return -1;
    if (stage < 0 || stage > 2) return -1;
    if (!oracle_params_valid(p)) return -2;
    double bl = oracle_bn(p[9]), bs = oracle_bn(p[14]);
    if (stage == 2) {
        int fx = nx * s;
        for (int i = 0; i < ny; ++i)
            for (int v = 0; v < s; ++v)
                for (int j = 0; j < nx; ++j)
                    for (int u = 0; u < s; ++u) {
                        double x, y;
                        oracle_subpixel_xy(ny, nx, dpix, s, i, j, v, u, &x, &y);
                        out[(i * s + v) * fx + j * s + u] = orc_scene(p, bl, bs, x, y);
                    }
        return 0;
    }
    double *img = (double *)malloc(sizeof(double) * (size_t)ny * nx);
    if (!img) return -1;
    for (int i = 0; i < ny; ++i)
        for (int j = 0; j < nx; ++j) {
            double acc = 0.0;
            for (int v = 0; v < s; ++v)
                for (int u = 0; u < s; ++u) {
                    double x, y;
                    oracle_subpixel_xy(ny, nx, dpix, s, i, j, v, u, &x, &y);
                    acc += orc_scene(p, bl, bs, x, y);
                }
            img[i * nx + j] = acc / ((double)s * s);
        }
    if (stage == 0) memcpy(out, img, sizeof(double) * (size_t)ny * nx);
    else oracle_convolve_same(img, ny, nx, psf, k, out);
    free(img);
    return 0;
}

/* C = -1/2 sum_mask ln(2 pi sigma^2), the likelihood's normalisation (Eq. 5). */
double oracle_loglike_norm(int64_t npix, const double *sigma, const uint8_t *mask)
{
    double c = 0.0;
    for (int64_t i = 0; i < npix; ++i)
        if (mask[i]) c += -0.5 * log(2.0 * M_PI * sigma[i] * sigma[i]);
    return c;
}

/* lnL of n proposals (Eq. 5 over the fitting region).  out_chi2 may be NULL.
 * Proposals outside the domain give lnL = -inf and chi2 = +inf.
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 on a bad argument. */
int oracle_loglike(int ny, int nx, double dpix, int s, int k, const double *psf,
                   const double *data, const double *sigma, const uint8_t *mask,
                   const double *params, int64_t n, double *out, double *out_chi2,
                   int nthreads)
{
    if (!orc_geom_ok(ny, nx, dpix, s, k) || !psf || !data || !sigma || !mask ||
        (n > 0 && (!params || !out)) || n < 0)
        return -1;
    int64_t npix = (int64_t)ny * nx;
    for (int64_t i = 0; i < npix; ++i)
        if (mask[i] && !(sigma[i] > 0.0 && isfinite(sigma[i]) && isfinite(data[i]))) return -1;
    double C = oracle_loglike_norm(npix, sigma, mask);
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : bad)
#endif
    {
        double *m = (double *)malloc(sizeof(double) * (size_t)npix);
        if (!m) bad = 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t t = 0; t < n; ++t) {
            if (!m) continue;
            const double *p = params + t * ORC_NP;
            if (!oracle_params_valid(p)) {
                out[t] = -INFINITY;
                if (out_chi2) out_chi2[t] = INFINITY;
                continue;
            }
            oracle_model_image(ny, nx, dpix, s, k, psf, p, 1, m);
            double chi2 = 0.0;
            for (int64_t i = 0; i < npix; ++i)
                if (mask[i]) {
                    double r = (data[i] - m[i]) / sigma[i];
                    chi2 += r * r;
                }
            out[t] = C - 0.5 * chi2;
            if (out_chi2) out_chi2[t] = chi2;
        }
        free(m);
    }
    return bad ? -1 : 0;
}

/* lnL with the light amplitudes solved linearly (Sec. 2.3): the unit-amplitude
 * lens-light and source images, each binned and PSF-convolved, are the columns
 * a and b of M; the amplitudes (s_l, s_s) minimise chi^2 = sum_mask ((d - M s)/sigma)^2
 * subject to s >= 0 (non-negative least squares).  With two columns the
 * minimiser is found by plain enumeration: for every support S of {l, s}
 * (both, l only, s only, none) take the unconstrained least-squares solution on
 * S (normal equations on S, zero elsewhere); keep it if it is >= 0; the
 * feasible candidate with the smallest chi^2 -- computed by a direct pass over
 * the residuals -- is the NNLS solution (the optimum is the least-squares
 * solution on its own support).  A support whose normal matrix is singular
 * (a column that vanishes on the mask) is skipped; dropping that column gives
 * the same chi^2.  The proposal's amplitude slots 7 and 12 are ignored.
 * out_chi2 and out_amp ([n][2]: s_l, s_s) may be NULL; proposals outside the
 * domain give lnL = -inf, chi2 = +inf, amplitudes NaN.  Returns 0 or -1 on a
 * bad argument. */
int oracle_loglike_nnls(int ny, int nx, double dpix, int s, int k, const double *psf,
                        const double *data, const double *sigma, const uint8_t *mask,
                        const double *params, int64_t n, double *out, double *out_chi2,
                        double *out_amp, int nthreads)
{
    if (!orc_geom_ok(ny, nx, dpix, s, k) || !psf || !data || !sigma || !mask ||
        (n > 0 && (!params || !out)) || n < 0)
        return -1;
    int64_t npix = (int64_t)ny * nx;
    for (int64_t i = 0; i < npix; ++i)
        if (mask[i] && !(sigma[i] > 0.0 && isfinite(sigma[i]) && isfinite(data[i]))) return -1;
    double C = oracle_loglike_norm(npix, sigma, mask);
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : bad)
#endif
    {
        double *a = (double *)malloc(sizeof(double) * (size_t)npix);
        double *b = (double *)malloc(sizeof(double) * (size_t)npix);
        if (!a || !b) bad = 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t t = 0; t < n; ++t) {
            if (!a || !b) continue;
            double p[ORC_NP];
            memcpy(p, params + t * ORC_NP, sizeof(p));
            p[7] = 1.0;
            p[12] = 0.0;
            int ok = oracle_params_valid(p);
            if (ok) {
                oracle_model_image(ny, nx, dpix, s, k, psf, p, 1, a);   /* lens light, unit amplitude */
                p[7] = 0.0;
                p[12] = 1.0;
                oracle_model_image(ny, nx, dpix, s, k, psf, p, 1, b);   /* source, unit amplitude */
            }
            if (!ok) {
                out[t] = -INFINITY;
                if (out_chi2) out_chi2[t] = INFINITY;
                if (out_amp) out_amp[2 * t] = out_amp[2 * t + 1] = NAN;
                continue;
            }
            /* normal equations F s = g of the weighted problem */
            double F11 = 0.0, F12 = 0.0, F22 = 0.0, g1 = 0.0, g2 = 0.0;
            for (int64_t i = 0; i < npix; ++i)
                if (mask[i]) {
                    double w = 1.0 / (sigma[i] * sigma[i]);
                    F11 += w * a[i] * a[i];
                    F12 += w * a[i] * b[i];
                    F22 += w * b[i] * b[i];
                    g1 += w * a[i] * data[i];
                    g2 += w * b[i] * data[i];
                }
            double cand[4][2];
            int nc = 0;
            double det = F11 * F22 - F12 * F12;
            if (det > 0.0) {
                cand[nc][0] = (g1 * F22 - g2 * F12) / det;
                cand[nc][1] = (g2 * F11 - g1 * F12) / det;
                ++nc;
            }
            if (F11 > 0.0) {
                cand[nc][0] = g1 / F11;
                cand[nc][1] = 0.0;
                ++nc;
            }
            if (F22 > 0.0) {
                cand[nc][0] = 0.0;
                cand[nc][1] = g2 / F22;
                ++nc;
            }
            cand[nc][0] = 0.0;
            cand[nc][1] = 0.0;
            ++nc;
            double best = INFINITY, bl = 0.0, bs = 0.0;
            for (int c = 0; c < nc; ++c) {
                if (!(cand[c][0] >= 0.0 && cand[c][1] >= 0.0)) continue;
                double chi2 = 0.0;
                for (int64_t i = 0; i < npix; ++i)
                    if (mask[i]) {
                        double r = (data[i] - cand[c][0] * a[i] - cand[c][1] * b[i]) / sigma[i];
                        chi2 += r * r;
                    }
                if (chi2 < best) {
                    best = chi2;
                    bl = cand[c][0];
                    bs = cand[c][1];
                }
            }
            out[t] = C - 0.5 * best;
            if (out_chi2) out_chi2[t] = best;
            if (out_amp) {
                out_amp[2 * t] = bl;
                out_amp[2 * t + 1] = bs;
            }
        }
        free(a);
        free(b);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Light models with several components, amplitudes solved (Sec. 2.3, and   */
/* the fitting set-ups of Sec. 3.1.2 and Sec. 3.2)                           */
/* ------------------------------------------------------------------------ */
/* Components of the light models (amplitudes are never parameters here):
 *   model 0 (lens and source): lens Sersic  (R = p[8],  n = p[9],  q = p[10], phi = p[11], centre p[3], p[4])
 *                              source Sersic (R = p[13], n = p[14], q = p[15], phi = p[16], centre p[17], p[18])
 *   model 1 (lens light only, no lensing): the lens Sersic above
 *   model 2 (lensed source only, no lens light): the source Sersic above
 *   model 3 (two components per galaxy, shared centre and ellipticity, indices
 *            fixed): lens a (R = p[8], n = nfix[0]), lens b (R = p[9], n = nfix[1]),
 *            both with q = p[10], phi = p[11], centre p[3], p[4];
 *            source a (R = p[13], n = nfix[2]), source b (R = p[14], n = nfix[3]),
 *            both with q = p[15], phi = p[16], centre p[17], p[18].
 * The mass (slots 0-6) lenses the source components; model 1 ignores it. */
static int orc_light_count(int model)
{
    return model == 0 ? 2 : model == 1 || model == 2 ? 1 : model == 3 ? 4 : 0;
}

/* domain of the slots a light model reads */
static int orc_light_valid(const double *p, int model, const double *nfix)
{
    int mass = model != 1, lens = model != 2, src = model != 1;
    if (mass) {
        for (int i = 0; i < 7; ++i)
            if (!isfinite(p[i])) return 0;
        if (p[0] < 0.0 || !(p[1] > 0.0 && p[1] <= 1.0)) return 0;
        if (p[19] != 0.0 && !(p[19] >= ORC_GAMMA_MIN && p[19] <= ORC_GAMMA_MAX)) return 0;
    }
    if (lens) {
        for (int i = 8; i < 12; ++i)
            if (!isfinite(p[i])) return 0;
        if (!isfinite(p[3]) || !isfinite(p[4]) || !(p[10] > 0.0 && p[10] <= 1.0) || !(p[8] > 0.0)) return 0;
        if (model == 3 ? !(p[9] > 0.0) : !(p[9] >= ORC_N_MIN && p[9] <= ORC_N_MAX)) return 0;
    }
    if (src) {
        for (int i = 13; i < 19; ++i)
            if (!isfinite(p[i])) return 0;
        if (!(p[15] > 0.0 && p[15] <= 1.0) || !(p[13] > 0.0)) return 0;
        if (model == 3 ? !(p[14] > 0.0) : !(p[14] >= ORC_N_MIN && p[14] <= ORC_N_MAX)) return 0;
    }
    if (model == 3)
        for (int j = 0; j < 4; ++j)
            if (!(nfix[j] >= ORC_N_MIN && nfix[j] <= ORC_N_MAX)) return 0;
    return 1;
}

/* unit-amplitude surface brightness of component c of a light model at (x, y) */
static double orc_component(const double *p, int model, const double *nfix, const double *bn, int c,
                            double x, double y)
{
    int lens_side = model == 1 || (model == 0 && c == 0) || (model == 3 && c < 2);
    if (lens_side) {
        double R = (model == 3 && c == 1) ? p[9] : p[8];
        double n = model == 3 ? nfix[c] : p[9];
        return oracle_sersic(1.0, R, n, bn[c], p[10], p[11], p[3], p[4], x, y);
    }
    double ax, ay;
    oracle_deflection(p, x, y, &ax, &ay);
    double bx = x - ax, by = y - ay;                                       /* Eq. 1 */
    double R = (model == 3 && c == 3) ? p[14] : p[13];
    double n = model == 3 ? nfix[c] : p[14];
    return oracle_sersic(1.0, R, n, bn[c], p[15], p[16], p[17], p[18], bx, by);
}

/* Solve the m x m symmetric system A x = b (row-major, m <= 4) by Gaussian
 * elimination with partial pivoting; returns 0 if A is singular (a pivot
 * below 1e-13 of the largest diagonal entry). */
static int orc_solve(int m, double *A, double *b, double *x)
{
    double dmax = 0.0;
    for (int i = 0; i < m; ++i) dmax = fmax(dmax, fabs(A[i * m + i]));
    if (!(dmax > 0.0)) return 0;
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (fabs(A[r * m + col]) > fabs(A[piv * m + col])) piv = r;
        if (!(fabs(A[piv * m + col]) > 1e-13 * dmax)) return 0;
        if (piv != col) {
            for (int c = 0; c < m; ++c) {
                double t = A[col * m + c]; A[col * m + c] = A[piv * m + c]; A[piv * m + c] = t;
            }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < m; ++r) {
            double f = A[r * m + col] / A[col * m + col];
            for (int c = col; c < m; ++c) A[r * m + c] -= f * A[col * m + c];
            b[r] -= f * b[col];
        }
    }
    for (int r = m - 1; r >= 0; --r) {
        double acc = b[r];
        for (int c = r + 1; c < m; ++c) acc -= A[r * m + c] * x[c];
        x[r] = acc / A[r * m + r];
    }
    return 1;
}

/* lnL of a light model with its amplitudes solved by non-negative least
 * squares (Sec. 2.3), for any of the models above: the columns of M are the
 * components at unit amplitude, binned and PSF-convolved; the NNLS minimiser
 * is the least-squares solution, on one of the 2^N supports, that is >= 0
 * and has the smallest chi^2 (computed by a direct pass over the residuals).
 * nfix: the four fixed Sersic indices of model 3 (ignored otherwise).
 * out_amp: [n][N] amplitudes in component order (may be NULL).  Proposals
 * outside the model's domain give lnL = -inf and NaN amplitudes. */
int oracle_loglike_light(int ny, int nx, double dpix, int s, int k, const double *psf,
                         const double *data, const double *sigma, const uint8_t *mask,
                         const double *params, int64_t n, int model, const double *nfix,
                         double *out, double *out_chi2, double *out_amp, int nthreads)
{
    int N = orc_light_count(model);
    if (!orc_geom_ok(ny, nx, dpix, s, k) || !psf || !data || !sigma || !mask || N == 0 ||
        (model == 3 && !nfix) || (n > 0 && (!params || !out)) || n < 0)
        return -1;
    int64_t npix = (int64_t)ny * nx;
    for (int64_t i = 0; i < npix; ++i)
        if (mask[i] && !(sigma[i] > 0.0 && isfinite(sigma[i]) && isfinite(data[i]))) return -1;
    double C = oracle_loglike_norm(npix, sigma, mask);
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : bad)
#endif
    {
        double *col = (double *)malloc(sizeof(double) * (size_t)npix * 4);
        double *img = (double *)malloc(sizeof(double) * (size_t)npix);
        if (!col || !img) bad = 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t t = 0; t < n; ++t) {
            if (!col || !img) continue;
            const double *p = params + t * ORC_NP;
            if (!orc_light_valid(p, model, nfix)) {
                out[t] = -INFINITY;
                if (out_chi2) out_chi2[t] = INFINITY;
                if (out_amp)
                    for (int c = 0; c < N; ++c) out_amp[t * N + c] = NAN;
                continue;
            }
            double bn[4];
            for (int c = 0; c < N; ++c) {
                int lens_side = model == 1 || (model == 0 && c == 0) || (model == 3 && c < 2);
                bn[c] = oracle_bn(model == 3 ? nfix[c] : (lens_side ? p[9] : p[14]));
            }
            /* columns: each component binned (s x s mean) and convolved */
            for (int c = 0; c < N; ++c) {
                for (int i = 0; i < ny; ++i)
                    for (int j = 0; j < nx; ++j) {
                        double acc = 0.0;
                        for (int v = 0; v < s; ++v)
                            for (int u = 0; u < s; ++u) {
                                double x, y;
                                oracle_subpixel_xy(ny, nx, dpix, s, i, j, v, u, &x, &y);
                                acc += orc_component(p, model, nfix, bn, c, x, y);
                            }
                        img[i * nx + j] = acc / ((double)s * s);
                    }
                oracle_convolve_same(img, ny, nx, psf, k, col + (size_t)c * npix);
            }
            /* normal equations of the weighted problem */
            double F[16] = {0}, g[4] = {0};
            for (int64_t i = 0; i < npix; ++i)
                if (mask[i]) {
                    double w = 1.0 / (sigma[i] * sigma[i]);
                    for (int a = 0; a < N; ++a) {
                        g[a] += w * col[(size_t)a * npix + i] * data[i];
                        for (int b = 0; b < N; ++b) F[a * N + b] += w * col[(size_t)a * npix + i] * col[(size_t)b * npix + i];
                    }
                }
            double best = INFINITY, bs[4] = {0, 0, 0, 0};
            for (int S = 0; S < (1 << N); ++S) {
                int idx[4], m = 0;
                for (int c = 0; c < N; ++c)
                    if (S & (1 << c)) idx[m++] = c;
                double x[4] = {0, 0, 0, 0}, cand[4] = {0, 0, 0, 0};
                if (m > 0) {
                    double A[16], b[4];
                    for (int a = 0; a < m; ++a) {
                        b[a] = g[idx[a]];
                        for (int c = 0; c < m; ++c) A[a * m + c] = F[idx[a] * N + idx[c]];
                    }
                    if (!orc_solve(m, A, b, x)) continue;
                    int feasible = 1;
                    for (int a = 0; a < m; ++a) feasible = feasible && x[a] >= 0.0;
                    if (!feasible) continue;
                    for (int a = 0; a < m; ++a) cand[idx[a]] = x[a];
                }
                double chi2 = 0.0;
                for (int64_t i = 0; i < npix; ++i)
                    if (mask[i]) {
                        double mval = 0.0;
                        for (int c = 0; c < N; ++c) mval += cand[c] * col[(size_t)c * npix + i];
                        double r = (data[i] - mval) / sigma[i];
                        chi2 += r * r;
                    }
                if (chi2 < best) {
                    best = chi2;
                    for (int c = 0; c < N; ++c) bs[c] = cand[c];
                }
            }
            out[t] = C - 0.5 * best;
            if (out_chi2) out_chi2[t] = best;
            if (out_amp)
                for (int c = 0; c < N; ++c) out_amp[t * N + c] = bs[c];
        }
        free(col);
        free(img);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 3)             */
/* ------------------------------------------------------------------------ */
/* Ten rounds on a 4 x 32-bit counter under a 2 x 32-bit key.  One round
 * multiplies the counter's words 0 and 2 by the two Philox constants, takes
 * the 64-bit products apart, and recombines them with words 1 and 3 and the
 * round key; the key advances by the two Weyl increments between rounds. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;    /* multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;    /* key increments */
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Ensemble sampler: the stretch move (Goodman & Weare 2010, Sec. 3; its      */
/* parallel form splits the walkers in two halves that update in turn)       */
/* ------------------------------------------------------------------------ */
/* W walkers (W even), each a 20-slot parameter vector; half h holds walkers
 * [h W/2, (h+1) W/2).  In iteration t, half h moves; walker k of that half
 * draws the Philox words of counter (k, t mod 2^32, t div 2^32, 0) under key
 * (seed mod 2^32, seed div 2^32):
 *   word 0 -> partner j = (other half's first walker) + floor(word0 * (W/2) / 2^32)
 *   word 1 -> u1 = (word1 + 1/2) / 2^32,  z = ((a - 1) u1 + 1)^2 / a,
 *             distributed with density proportional to 1/sqrt(z) on [1/a, a]
 *   word 2 -> u2 = (word2 + 1/2) / 2^32
 * The proposal is Y = X_j + z (X_k - X_j); it replaces X_k when
 *   ln u2 < (d - 1) ln z + lnP(Y) - lnP(X_k),
 * d being the number of free slots.  Proposal of one half: */
void oracle_stretch_propose(int W, int half, int64_t t, uint64_t seed, double a, const double *walkers,
                            double *Y, double *z_out, double *logu_out, int32_t *partner_out)
{
    const int h = W / 2;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int i = 0; i < h; ++i) {
        const int k = half * h + i;
        const uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(uint64_t)t, (uint32_t)((uint64_t)t >> 32), 0u};
        uint32_t r[4];
        oracle_philox4x32_10(ctr, key, r);
        const int j = (1 - half) * h + (int)(((uint64_t)r[0] * (uint64_t)h) >> 32);
        const double u1 = ((double)r[1] + 0.5) / 4294967296.0;
        const double u2 = ((double)r[2] + 0.5) / 4294967296.0;
        const double w = (a - 1.0) * u1 + 1.0;
        const double z = w * w / a;
        for (int s = 0; s < ORC_NP; ++s)
            Y[(size_t)i * ORC_NP + s] = walkers[(size_t)j * ORC_NP + s] +
                z * (walkers[(size_t)k * ORC_NP + s] - walkers[(size_t)j * ORC_NP + s]);
        z_out[i] = z;
        logu_out[i] = log(u2);
        if (partner_out) partner_out[i] = j;
    }
}

/* Acceptance of one half: lnpY[i] is lnP of proposal i (-inf outside the
 * prior); accepted walkers take Y and lnpY, and their counters advance. */
void oracle_stretch_accept(int W, int half, int d, double *walkers, double *lnp, const double *Y,
                           const double *lnpY, const double *z, const double *logu, int64_t *accepted)
{
    const int h = W / 2;
    for (int i = 0; i < h; ++i) {
        const int k = half * h + i;
        const double lhs = logu[i], rhs = (d - 1) * log(z[i]) + lnpY[i] - lnp[k];
        if (lnpY[i] > -INFINITY && lhs < rhs) {
            memcpy(walkers + (size_t)k * ORC_NP, Y + (size_t)i * ORC_NP,
                   ORC_NP * sizeof(double));
            lnp[k] = lnpY[i];
            if (accepted) accepted[k] += 1;
        }
    }
}

/* ln of the uniform box prior up to its constant: 0 when lo[s] <= p[s] <=
 * hi[s] for every slot, else -inf (Sec. 2.2: posterior = likelihood x prior) */
double oracle_box_logprior(const double *p, const double *lo, const double *hi)
{
    for (int s = 0; s < ORC_NP; ++s)
        if (!(p[s] >= lo[s] && p[s] <= hi[s])) return -INFINITY;
    return 0.0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
