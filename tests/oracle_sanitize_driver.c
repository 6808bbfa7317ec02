/* Drives every entry point of the oracle on a small lens, for a build under
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py).
 * The sanitizers report any out-of-bounds access, use of freed memory, signed
 * overflow or invalid shift; the checks below only guard against a run that
 * silently computes nothing. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double oracle_gammainc_lower_reg(double a, double x);
double oracle_bn(double n);
void oracle_sie_deflection(double theta_E, double q, double phi, double xm, double ym, double x, double y,
                           double *ax, double *ay);
void oracle_epl_deflection(double theta_E, double gamma, double q, double phi, double xm, double ym, double x,
                           double y, double *ax, double *ay);
void oracle_deflection(const double *p, double x, double y, double *ax, double *ay);
int oracle_params_valid(const double *p);
void oracle_convolve_same(const double *img, int ny, int nx, const double *psf, int k, double *out);
int oracle_model_image(int ny, int nx, double dpix, int s, int k, const double *psf, const double *p, int stage,
                       double *out);
double oracle_loglike_norm(int64_t npix, const double *sigma, const uint8_t *mask);
int oracle_loglike(int ny, int nx, double dpix, int s, int k, const double *psf, const double *data,
                   const double *sigma, const uint8_t *mask, const double *params, int64_t n, double *out,
                   double *out_chi2, int nthreads);
int oracle_loglike_nnls(int ny, int nx, double dpix, int s, int k, const double *psf, const double *data,
                        const double *sigma, const uint8_t *mask, const double *params, int64_t n, double *out,
                        double *out_chi2, double *out_amp, int nthreads);
int oracle_loglike_light(int ny, int nx, double dpix, int s, int k, const double *psf, const double *data,
                         const double *sigma, const uint8_t *mask, const double *params, int64_t n, int model,
                         const double *nfix, double *out, double *out_chi2, double *out_amp, int nthreads);
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void oracle_stretch_propose(int W, int half, int64_t t, uint64_t seed, double a, const double *walkers, double *Y,
                            double *z_out, double *logu_out, int32_t *partner_out);
void oracle_stretch_accept(int W, int half, int d, double *walkers, double *lnp, const double *Y,
                           const double *lnpY, const double *z, const double *logu, int64_t *accepted);
double oracle_box_logprior(const double *p, const double *lo, const double *hi);

#define NY 14
#define NX 12
#define S 2
#define K 5
#define NP 4

static int fails = 0;
static void check(int ok, const char *what)
{
    if (!ok) {
        printf("FAIL: %s\n", what);
        fails++;
    }
}

int main(void)
{
    const double dpix = 0.12;
    double psf[K * K], sum = 0.0;
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            const double r2 = (a - K / 2) * (a - K / 2) + (b - K / 2) * (b - K / 2);
            psf[a * K + b] = exp(-0.5 * r2);
            sum += psf[a * K + b];
        }
    for (int i = 0; i < K * K; ++i) psf[i] /= sum;
    /* a valid proposal, one outside the domain (q_m > 1), one near a centre, an EPL one */
    double P[NP][20] = {
        {1.2, 0.7, 0.4, 0.02, -0.01, 0.03, -0.02, 0.3, 0.4, 2.5, 0.8, 1.1, 0.2, 0.3, 1.5, 0.7, 0.6, 0.1, -0.05, 0.0},
        {1.2, 1.5, 0.4, 0.02, -0.01, 0.03, -0.02, 0.3, 0.4, 2.5, 0.8, 1.1, 0.2, 0.3, 1.5, 0.7, 0.6, 0.1, -0.05, 0.0},
        {0.8, 0.55, 2.0, 0.0, 0.0, 0.0, 0.0, 0.2, 0.2, 4.0, 0.6, 0.3, 0.4, 0.1, 3.5, 0.9, 2.8, 0.0, 0.0, 0.0},
        {1.0, 0.6, 1.0, 0.01, 0.02, -0.04, 0.05, 0.25, 0.5, 1.5, 0.7, 2.0, 0.3, 0.2, 1.0, 0.6, 0.2, -0.2, 0.1, 2.3},
    };
    static double img[NY * NX], conv[NY * NX], data[NY * NX], sigma[NY * NX];
    static uint8_t mask[NY * NX];
    check(oracle_model_image(NY, NX, dpix, S, K, psf, P[0], 1, img) == 0, "model image");
    uint64_t st = 12345;
    for (int i = 0; i < NY * NX; ++i) {
        st = st * 6364136223846793005ULL + 1442695040888963407ULL;
        const double u = (double)(st >> 11) * 0x1p-53 - 0.5;
        sigma[i] = 0.02;
        data[i] = img[i] + 0.02 * u;
        mask[i] = (uint8_t)((i % 7) != 3);
    }
    oracle_convolve_same(img, NY, NX, psf, K, conv);
    check(oracle_model_image(NY, NX, dpix, S, K, psf, P[3], 0, img) == 0, "model image, EPL, unconvolved");
    check(isfinite(oracle_loglike_norm(NY * NX, sigma, mask)), "norm");

    double out[NP], chi2[NP], amp[NP * 4];
    check(oracle_loglike(NY, NX, dpix, S, K, psf, data, sigma, mask, &P[0][0], NP, out, chi2, 2) == 0, "loglike");
    check(isfinite(out[0]) && isinf(out[1]) && out[1] < 0 && isfinite(out[2]) && isfinite(out[3]), "loglike values");
    check(oracle_loglike_nnls(NY, NX, dpix, S, K, psf, data, sigma, mask, &P[0][0], NP, out, chi2, amp, 2) == 0,
          "nnls");
    check(isfinite(out[0]) && amp[0] >= 0.0 && amp[1] >= 0.0, "nnls values");
    const double nfix[4] = {1.0, 4.0, 1.0, 4.0};
    for (int model = 0; model < 4; ++model) {
        check(oracle_loglike_light(NY, NX, dpix, S, K, psf, data, sigma, mask, &P[0][0], NP, model, nfix, out, chi2,
                                   amp, 2) == 0,
              "light models");
        check(isfinite(out[0]), "light model value");
    }

    double ax, ay;
    oracle_sie_deflection(1.0, 0.6, 0.3, 0.0, 0.0, 0.4, -0.2, &ax, &ay);
    check(isfinite(ax) && isfinite(ay), "sie");
    oracle_sie_deflection(1.0, 0.6, 0.3, 0.0, 0.0, 0.0, 0.0, &ax, &ay);
    check(ax == 0.0 && ay == 0.0, "sie at the centre");
    for (double g = 1.05; g <= 2.95; g += 0.3) {
        oracle_epl_deflection(1.0, g, 0.4, 0.3, 0.0, 0.0, 0.4, -0.2, &ax, &ay);
        check(isfinite(ax) && isfinite(ay), "epl");
    }
    oracle_deflection(P[3], 0.3, 0.1, &ax, &ay);
    check(isfinite(ax), "deflection");
    check(oracle_params_valid(P[0]) && !oracle_params_valid(P[1]), "params_valid");
    check(fabs(oracle_bn(0.5) - log(2.0)) < 1e-12, "bn");
    check(oracle_gammainc_lower_reg(2.0, 1.0) > 0.0, "gammainc");

    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, word[4];
    oracle_philox4x32_10(ctr, key, word);
    enum { W = 8 };
    double walkers[W * 20], lnp[W], Y[W / 2 * 20], z[W / 2], logu[W / 2], lnpY[W / 2], lo[20], hi[20];
    int32_t partner[W / 2];
    int64_t accepted[W] = {0};
    for (int s = 0; s < 20; ++s) {
        lo[s] = -1.0;
        hi[s] = s == 19 ? -1.0 : 1.0;
    }
    for (int i = 0; i < W * 20; ++i) walkers[i] = (i % 20) == 19 ? -1.0 : 0.01 * (i % 37) - 0.18;
    for (int k = 0; k < W; ++k) lnp[k] = -1.0;
    for (int half = 0; half < 2; ++half) {
        oracle_stretch_propose(W, half, 3, 77, 2.0, walkers, Y, z, logu, partner);
        for (int i = 0; i < W / 2; ++i) lnpY[i] = oracle_box_logprior(&Y[i * 20], lo, hi) == 0.0 ? -0.5 : -INFINITY;
        oracle_stretch_accept(W, half, 19, walkers, lnp, Y, lnpY, z, logu, accepted);
    }
    check(conv[0] == conv[0], "convolution");
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
