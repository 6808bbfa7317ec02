// lens_device.h -- per-sub-pixel physics of the forward model, FP32, gfx950.
//
// Cao et al. (2025), Sec. 2.1 (Eqs. 1-2) and Sec. 2.4 (Eqs. 8-10, 12-14).
// Every function here is evaluated E times per proposal (E = sub-pixels in
// the mask's PSF-dilated footprint), so it is written for the vector ALU:
// no divisions, hardware exp2/log2/rsq/rcp, per-proposal constants folded in
// the prep kernel, branch-free except the two range splits of the SIE.
#pragma once

#include <hip/hip_runtime.h>

#include "lens_approx.h"
#include "lens_internal.h"

namespace lensk {

__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// 1/x refined by one Newton step (about half an ulp).
__device__ __forceinline__ float rcp_nr(float x)
{
    float r = hw_rcp(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

template <int N>
__device__ __forceinline__ float horner(const float (&c)[N], float w)
{
    float p = c[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) p = fmaf(p, w, c[i]);
    return p;
}

// atan(t)/t, even in t.  |t| <= 1: polynomial in t^2; |t| > 1: atan t = pi/2 - atan(1/t).
__device__ __forceinline__ float atan_over_t(float t)
{
    const float z = fabsf(t);
    const bool big = z > 1.0f;
    const float zi = big ? rcp_nr(z) : z;
    const float p = horner(kAtanOverT, zi * zi);
    return big ? fmaf(-zi, p, 1.57079632679f) * zi : p;
}

// atanh(t)/t, even in t, |t| < 1.  |t| <= 1/2: polynomial in t^2; otherwise
// (ln 2 / 2) log2((1+z)/(1-z)) / z with the rounding error of 1+z carried
// exactly (1-z is exact for z in [1/2, 1]).
__device__ __forceinline__ float atanh_over_t(float t)
{
    const float z = fabsf(t);
    if (z <= 0.5f) return horner(kAtanhOverT, z * z);
    const float num = 1.0f + z;
    const float err = z - (num - 1.0f);
    const float den = 1.0f - z;
    const float rd = hw_rcp(den);
    float q = num * rd;
    q = fmaf(fmaf(-q, den, num) + err, rd, q);
    return (0.346573590280f * hw_log2(q)) * rcp_nr(z);
}

// Derived constants of one proposal, uniform across the workgroup.
struct PropC {
    float xm, ym, cm, sm, q2m, ce, bsie, g1, g2;
    float Il, cl, sl, Al, Bl, el, BLh, BLl;
    float Is, xs, ys, cs, ss, As, Bs, es, BSh, BSl;
};

__device__ __forceinline__ PropC load_prop(const float *__restrict__ c)
{
    PropC P;
    P.xm = c[PC_XM]; P.ym = c[PC_YM]; P.cm = c[PC_CM]; P.sm = c[PC_SM];
    P.q2m = c[PC_Q2M]; P.ce = c[PC_CE]; P.bsie = c[PC_BSIE]; P.g1 = c[PC_G1]; P.g2 = c[PC_G2];
    P.Il = c[PC_IL]; P.cl = c[PC_CL]; P.sl = c[PC_SL]; P.Al = c[PC_AL]; P.Bl = c[PC_BL];
    P.el = c[PC_EL]; P.BLh = c[PC_BLH]; P.BLl = c[PC_BLL];
    P.Is = c[PC_IS]; P.xs = c[PC_XS]; P.ys = c[PC_YS]; P.cs = c[PC_CS]; P.ss = c[PC_SS];
    P.As = c[PC_AS]; P.Bs = c[PC_BS]; P.es = c[PC_ES]; P.BSh = c[PC_BSH]; P.BSl = c[PC_BSL];
    return P;
}

// Elliptical Sersic (Eqs. 8, 10) at offset (dx, dy) from its centre:
//   I exp(-b (R/R_e)^(1/n) + b) = I 2^(B (1 - t)),  t = ((R/R_e)^2)^(1/(2n)),  B = b log2 e.
// A = q/R_e^2 and Bq = 1/(q R_e^2) fold the axis ratio and radius; B is carried
// as hi + lo so that its FP32 rounding does not bias the central brightness.
__device__ __forceinline__ float sersic(float dx, float dy, float c, float s, float A, float Bq,
                                        float e, float Bh, float Bl, float I)
{
    const float x1 = fmaf(c, dx, s * dy);
    const float x2 = fmaf(c, dy, -(s * dx));
    const float r2 = fmaf(A, x1 * x1, Bq * (x2 * x2));
    const float t = hw_exp2(fminf(e * hw_log2(r2), 64.0f));
    const float omt = 1.0f - t;
    return I * hw_exp2(fmaf(Bh, omt, Bl * omt));
}

// Lens light at theta plus source light at beta = theta - alpha_SIE - alpha_shear (Eqs. 1-2).
// SIE (kappa = theta_E / (2 R_p)) in the frame of the mass ellipse:
//   alpha' = theta_E sqrt(q) (u1 F(c u1), u2 G(c u2)),  u = x'/psi,  psi = sqrt(q^2 x1'^2 + x2'^2),
//   c = sqrt(1 - q^2), F = atan(t)/t, G = atanh(t)/t  (smooth through q = 1, alpha = 0 at the centre).
// Shear: alpha = -(g1 x + g2 y, g2 x - g1 y).
__device__ __forceinline__ float scene(float x, float y, const PropC &P)
{
    const float dx = x - P.xm, dy = y - P.ym;
    const float x1 = fmaf(P.cm, dx, P.sm * dy);
    const float x2 = fmaf(P.cm, dy, -(P.sm * dx));
    const float psi2 = fmaf(P.q2m, x1 * x1, x2 * x2);
    const float ir = psi2 > 0.0f ? hw_rsq(psi2) : 0.0f;
    const float u1 = x1 * ir, u2 = x2 * ir;
    const float a1 = P.bsie * u1 * atan_over_t(P.ce * u1);
    const float a2 = P.bsie * u2 * atanh_over_t(P.ce * u2);
    const float bx = (x - fmaf(P.cm, a1, -(P.sm * a2))) + fmaf(P.g1, x, P.g2 * y);
    const float by = (y - fmaf(P.sm, a1, P.cm * a2)) + fmaf(P.g2, x, -(P.g1 * y));
    const float il = sersic(dx, dy, P.cl, P.sl, P.Al, P.Bl, P.el, P.BLh, P.BLl, P.Il);
    const float is = sersic(bx - P.xs, by - P.ys, P.cs, P.ss, P.As, P.Bs, P.es, P.BSh, P.BSl, P.Is);
    return il + is;
}

// Binned (mean) value of pixel (y, x): s x s sub-pixel centres (Sec. 2.1).
// Fine-grid index fx = x s + u maps to position (fx - (nx s - 1)/2) * pixel_scale / s.
__device__ __forceinline__ float binned_pixel(const LensGeom &g, const PropC &P, int y, int x)
{
    const int s = g.s;
    float acc = 0.0f;
    for (int v = 0; v < s; ++v) {
        const float yy = ((float)(y * s + v) - g.cfy) * g.sd;
        for (int u = 0; u < s; ++u) {
            const float xx = ((float)(x * s + u) - g.cfx) * g.sd;
            acc += scene(xx, yy, P);
        }
    }
    return acc * g.inv_s2;
}

// Sersic b_n: root of P(2n, b) = 1/2 (Eq. 9), FP64 Newton safeguarded by
// bisection on [0, 2n + 1].  P by its power series, which converges for every
// b in the bracket; the median of Gamma(2n) lies below 2n.
__device__ inline double bn_device(double n)
{
    const double a = 2.0 * n;
    const double lga1 = lgamma(a + 1.0);
    double lo = 0.0, hi = a + 1.0;
    double x = a - 1.0 / 3.0 + 4.0 / (405.0 * n);
    if (!(x > lo && x < hi)) x = 0.5 * a;
    for (int it = 0; it < 200; ++it) {
        double term = 1.0, sum = 1.0, ap = a;
        for (int k = 0; k < 4000; ++k) {
            ap += 1.0;
            term *= x / ap;
            sum += term;
            if (term < sum * 1e-17) break;
        }
        const double pref = exp(a * log(x) - x - lga1);
        const double f = pref * sum - 0.5;
        if (f < 0.0) lo = x; else hi = x;
        const double dens = pref * a / x;  // d/dx P(a, x) = x^(a-1) e^-x / Gamma(a)
        double xn = x - f / dens;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        const double dx = fabs(xn - x);
        x = xn;
        if (dx <= 4e-16 * x || hi - lo <= 4e-16 * x) break;
    }
    return x;
}

}  // namespace lensk
