// lens_device.h -- per-sub-pixel physics of the forward model, gfx950.
//
// Cao et al. (2025), Sec. 2.1 (Eqs. 1-2) and Sec. 2.4 (Eqs. 8-10, 12-14).
// Every function here runs E times per proposal (E = sub-pixels in the
// mask's PSF-dilated footprint).
//
// Precision.  beta = theta - alpha is a difference of arcsecond-sized
// numbers, and a Sersic profile with n > 1 has an infinitely steep cusp at
// its centre: an FP32 ray trace (absolute error ~4e-7 arcsec) gives 1e-5
// brightness errors next to a cusp.  Likewise b_n (R/R_e)^(1/n) amplifies the
// relative error of (R/R_e)^(1/n) by up to ~30.  So the ray trace and the
// profiles run in FP64 -- FP64 FMAs issue at the FP32 rate on CDNA4 -- with
// FP32 hardware only where its error is not amplified: the reciprocal and
// reciprocal-square-root seeds (refined by a Newton step) and log2 of the
// elliptical radius, whose error reaches the exponent scaled by
// b_n/(2n ln 2) ~ 1.  The binned pixel is rounded to FP32 once.
#pragma once

#include <hip/hip_runtime.h>

#include "lens_approx.h"
#include "lens_internal.h"

namespace lensk {

__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// 1/sqrt(x) and 1/x for x in the normal FP32 range: FP32 hardware seed and
// one FP64 Newton step (relative error ~1e-14).
__device__ __forceinline__ double rsq_nr(double x)
{
    const double r = (double)__builtin_amdgcn_rsqf((float)x);
    return fma(0.5 * r, fma(-(x * r), r, 1.0), r);
}

__device__ __forceinline__ double rcp_nr(double x)
{
    const double r = (double)__builtin_amdgcn_rcpf((float)x);
    return fma(r, fma(-x, r, 1.0), r);
}

// 1/sqrt(x) for any x > 0: FP64 hardware seed and two Newton steps.
__device__ __forceinline__ double rsq64(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    r = fma(0.5 * r, fma(-(x * r), r, 1.0), r);
    return fma(0.5 * r, fma(-(x * r), r, 1.0), r);
}

// 1/psi from psi2 = psi^2 >= 0, and 0 at psi = 0: rsq_nr where psi2 lies in
// FP32's normal range, else rsq64.  The test is wave-uniform and laid out
// for its usual outcome (no lane of the wave at the mass centre), which then
// runs without a taken branch; each lane's result is the same either way.
__device__ __forceinline__ double rsq_psi(double psi2)
{
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(!(psi2 >= 1e-30)) == 0, 1)) return rsq_nr(psi2);
    // a copy the compiler cannot see through, so that this path's per-lane
    // test stays inside it instead of being computed on the common path too
    double p = psi2;
    asm volatile("" : "+v"(p));
    return p >= 1e-30 ? rsq_nr(p) : p > 0.0 ? rsq64(p) : 0.0;
}

// a b + c as one VOP3 v_fma_f64 with c taken from an SGPR pair; c must be
// wave-uniform (here: a polynomial coefficient).  Written out because the
// compiler otherwise keeps FP64 coefficients in VGPRs and emits v_fmac_f64,
// whose tied addend costs a v_mov_b64 per step and ~40 VGPRs for the tables.
__device__ __forceinline__ double fma_c(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

// sum_i c[i] w^i; `lead` holds c[N - 1] (a caller may pass it in a VGPR
// loaded once outside its loop, which saves a v_mov_b64 per evaluation).
template <int N>
__device__ __forceinline__ double horner(const double (&c)[N], double w, double lead)
{
    double p = lead;
#pragma unroll
    for (int i = N - 2; i >= 0; --i) p = fma_c(p, w, c[i]);
    return p;
}

template <int N>
__device__ __forceinline__ double horner(const double (&c)[N], double w)
{
    return horner(c, w, c[N - 1]);
}

template <int N>
__device__ __forceinline__ constexpr double leading(const double (&c)[N])
{
    return c[N - 1];
}

// 2^y for y in [-1022, 1023]: 2^round(y) times a polynomial in the remainder.
template <int N>
__device__ __forceinline__ double exp2_64(const double (&c)[N], double y, double lead)
{
    const double k = rint(y);
    return ldexp(horner(c, y - k, lead), (int)k);
}

template <int N>
__device__ __forceinline__ double exp2_64(const double (&c)[N], double y)
{
    return exp2_64(c, y, c[N - 1]);
}

constexpr double kPi2 = 1.5707963267948966;
constexpr double kAtanh075 = 0.97295507452765665255;   // atanh(3/4)

// theta_E sqrt(q) atan(c u1)/c (the SIE deflection along the major axis).
// |c u1| <= 1: polynomial in (c u1)^2; else atan t = pi/2 - atan(1/t).
// |c u1| > 1 needs q < 1/sqrt(2) and a cone around the major axis, so most
// waves have no such lane: they skip the reduction on a wave-uniform branch
// (a divergent one would still issue it, with the lanes masked off).  Each
// lane's arithmetic is the same on either path.
__device__ __forceinline__ double sie_a1(double u1, double ce, double bsie, double bsc)
{
    const double t = ce * u1;
    const double z = fabs(t);
    const bool big = z > 1.0;
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(big) != 0, 0)) {
        const double zi = big ? rcp_nr(z) : z;
        const double p = horner(kAtanOverT64, zi * zi);
        return big ? copysign(bsc * fma(-zi, p, kPi2), t) : bsie * u1 * p;
    }
    return bsie * u1 * horner(kAtanOverT64, z * z);
}

// theta_E sqrt(q) atanh(c u2)/c (along the minor axis).  |t| <= 1/2:
// polynomial in t^2; 1/2 < |t| <= 0.9: atanh z = atanh(3/4) + atanh((z - 3/4)/(1 - 3z/4)),
// whose second argument lies in [-0.4, 0.47]; |t| > 0.9 (axis ratios below
// 0.44 only): the logarithm.
__device__ __forceinline__ double sie_a2(double u2, double ce, double bsie, double bsc)
{
    const double t = ce * u2;
    const double z = fabs(t);
    if (z <= 0.9) {
        const bool red = z > 0.5;
        // the reduction on a wave-uniform branch, as in sie_a1
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(red) != 0, 0)) {
            const double zr = red ? (z - 0.75) * rcp_nr(fma(-0.75, z, 1.0)) : z;
            const double p = horner(kAtanhOverT64, zr * zr);
            return red ? copysign(bsc * fma_c(zr, p, kAtanh075), t) : bsie * u2 * p;
        }
        return bsie * u2 * horner(kAtanhOverT64, z * z);
    }
    // atanh z = (ln 2 / 2) log2 y with y = (1 + z)/(1 - z) > 19:
    // FP32 log2 seed l0 (absolute error ~1e-6), then one Newton step on 2^l = y,
    // l1 = l0 + (y 2^-l0 - 1) log2 e: quadratic in the seed's error (~1e-13), plus the
    // 2^x polynomial's 1.9e-9, i.e. < 1e-9 relative in atanh z (log2 y > 4.2).
    const double y = (1.0 + z) * rcp_nr(1.0 - z);
    const double l0 = (double)hw_log2((float)y);
    const double l1 = fma(fma(y, exp2_64(kExp2_64, -l0), -1.0), 1.4426950408889634, l0);
    return copysign(bsc * 0.34657359027997264 * l1, t);
}

// Elliptical Sersic (Eqs. 8, 10) without its amplitude, from r2 = (R/R_e)^2:
//   exp(-b ((R/R_e)^(1/n) - 1)) = 2^(B (1 - t)),  t = r2^(1/(2n)),  B = b log2 e.
// log2 r2 = (binary exponent of r2) + log2(mantissa in [1/2, 1)), the FP32
// hardware log2 seeing only the mantissa and the sum taken in FP64: an absolute
// error of ~1e-7 at any magnitude.  (An FP32 log2 of r2 itself is good to one
// ulp of its result, ~1e-6 absolute once |log2 r2| nears 20, i.e. next to a
// steep Sersic centre, and the exponent carries that error into the
// brightness.)  The mantissa's log2 is clamped below at -2048, so the centre
// (r2 = 0) gives t = 2^-(2048 e) ~ 0 rather than NaN; a radius whose t
// overflows gives B (1 - t) = -inf, whose power of two exp2_hw makes 0.
// lead: the leading coefficient of kExp2_64 (see horner).
__device__ __forceinline__ double log2_r2(double r2)
{
    const float lm = __builtin_amdgcn_fmed3f(hw_log2((float)__builtin_amdgcn_frexp_mant(r2)), -2048.0f, 0.0f);
    return (double)__builtin_amdgcn_frexp_exp(r2) + (double)lm;
}

// log2 r2 for a Sersic exponent.  For a profile with n >= 1/2 (e <= 1),
// where every lane of the wave has log2 r2 >= -2 (R >= R_e / 2),
// it is the FP32 hardware log2 of r2 itself: an absolute error within an ulp
// of a result of that size (1.2e-7 for |l| < 2, 2.4e-7 for |l| < 4) plus
// 8.6e-8 from rounding r2 to FP32.  It reaches the brightness scaled by
// ln2^2 B e t (t = 2^(e l)): with one-ulp errors of this log2 and of exp2_hw
// aligned, at most 8.8e-7 of the local brightness wherever that is above 1/8
// of its value at R_e, against 1.1e-6 for the exponent split over the whole
// index domain (whose worst case is at n = 0.1, where this form would reach
// 1.7e-6: hence the gate on e).  A wave with a lane nearer a centre (where t
// is small and the cusp steep, and where r2 = 0 gives -inf) takes log2_r2.
// A radius whose FP32 value overflows gives l = +inf, t = NaN and, through
// exp2_hw, 0, as log2_r2's large finite value does.
// thr (uniform): -2 where the FP32 form is allowed, +inf where it is not (a
// threshold rather than a flag keeps the sub-pixel loop's code the same).
// The test is laid out for the FP32 form, which then runs without a taken
// branch (most waves take it; two taken branches per Sersic cost 2%).
__device__ __forceinline__ double log2_r2_sersic(double r2, float thr)
{
    const float l = hw_log2((float)r2);
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(!(l >= thr)) != 0, 0)) return log2_r2(r2);
    return (double)l;
}

// 2^y for y <= 1023, -inf and NaN included, for the brightness 2^(B (1 - t)), whose
// relative error is that of this function alone: nothing amplifies it.  The
// FP32 hardware 2^x is good to about one FP32 ulp of its result.
// - Where every lane of the wave has y <= 2, it is that 2^x of y rounded to
//   FP32.  The rounding adds at most ln2 2^-24 = 4.1e-8 relative for y in
//   [-2, 2], 8.3e-8 down to y = -4 (a sixteenth of the brightness at R_e),
//   and grows with |y| below, where the brightness shrinks faster.  Below
//   y = -126 the result is an FP32 subnormal or 0, under 1.2e-38 of the
//   brightness at R_e, and -inf gives 0.
// - Otherwise it is 2^round(y) times the 2^x of the remainder f in
//   [-1/2, 1/2] (f rounded to FP32: 1e-8 relative), as the centre of a steep
//   profile needs: there y reaches B, up to 57 at n = 20.  Here y is first
//   raised to -2000 (2^-2000 is 0 in FP64), which also maps NaN to 0: a NaN
//   lane fails the test above and lands here.
// The test is laid out for the first form, the common one.
__device__ __forceinline__ double exp2_hw(double y)
{
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(!(y <= 2.0)) == 0, 1)) return (double)__builtin_amdgcn_exp2f((float)y);
    y = fmax(y, -2000.0);
    const double k = rint(y);
    return ldexp((double)__builtin_amdgcn_exp2f((float)(y - k)), (int)k);
}

// 2^(B (1 - t)) with t = 2^(e lgd), lgd = log2 of (R/R_e)^2 (as above).  t's
// relative error is amplified by ln2 B t in the exponent, so it takes the FP64
// polynomial; the outer power's is not.
__device__ __forceinline__ double sersic_lg(double lgd, double e, double B, double lead)
{
    const double t = exp2_64(kExp2_64, e * lgd, lead);
    return exp2_hw(fma(-B, t, B));
}


// (R/R_e)^2 = P dx^2 + Q dy^2 + S dx dy at offset (dx, dy) from a light centre,
// the rotation and axis ratio of Eq. 10 folded into P, Q, S.
__device__ __forceinline__ double ellip_r2(double dx, double dy, const LightK &L)
{
    return fma(L.P, dx * dx, fma(L.Q, dy * dy, L.S * (dx * dy)));
}

// Source-plane position beta = theta - alpha_SIE - alpha_shear (Eqs. 1-2), given
// the sub-pixel's coordinates (x1, x2) in the frame of the mass ellipse and the
// part of beta linear in theta taken in that frame, (u1, u2) = R(-phi_m)
// (theta - alpha_shear - source centre).  Returns w = R(-phi_m) (beta - source
// centre) = u - alpha', the deflection alpha' staying in the mass frame (the
// source's quadratic form is rotated once per proposal instead).
// SIE (kappa = theta_E / (2 R_p)): psi = sqrt(q^2 x1^2 + x2^2), c = sqrt(1 - q^2),
// alpha' = theta_E sqrt(q) / c (atan(c x1/psi), atanh(c x2/psi)) in the mass
// frame; alpha' = 0 at the centre.  Shear (inside u): alpha = -(g1 x + g2 y, g2 x - g1 y).
__device__ __forceinline__ void ray_trace(double x1, double x2, double u1, double u2, const PropBlock &P,
                                          double &w1, double &w2)
{
    const double psi2 = fma(P.q2m, x1 * x1, x2 * x2);
    const double ir = rsq_psi(psi2);
    const double a1 = sie_a1(x1 * ir, P.ce, P.bsie, P.bsc);
    const double a2 = sie_a2(x2 * ir, P.ce, P.bsie, P.bsc);
    w1 = u1 - a1;
    w2 = u2 - a2;
}

// The SIE deflection from a per-proposal table.  With s = (x1, x2) / psi,
// q^2 s1^2 + s2^2 = 1, so alpha' = (s1 H1(u), s2 H2(u)) with u = q |s1| in
// [0, 1]: the deflection does not change along a ray from the mass centre,
// and both components are functions of u alone.  H1 and H2 are analytic
// except at u = +-i q / c; on each of kSieIntervals intervals of u the table
// holds the polynomial of degree kSieDeg through their values at the
// interval's Chebyshev nodes (from sie_a1 and sie_a2).  With 32 intervals
// and degree 5 that reproduces them to 1.3e-12 (q = 0.5) and 4e-11 (q = 0.3)
// relative, against 4e-10 and 1.3e-9 of the polynomials behind sie_a1 and
// sie_a2 (16 intervals at degree 6 are as accurate at two more FMAs per
// sub-pixel).  A sub-pixel then takes one interval lookup and two degree-5
// Horner sums instead of both deflection functions and, in most waves, a
// range reduction.  Below q = 0.3 the singularities come too close and the
// direct functions are used.
constexpr double kSieTabQ2 = 0.09;   // q^2 from which the table is used
static_assert(kSieEntry >= 2 * kSieDeg + 3, "SIE table entry");

__device__ __forceinline__ double *sie_table()
{
    __shared__ __attribute__((aligned(16))) double t[kSieIntervals * kSieEntry];
    return t;
}

__device__ __forceinline__ bool sie_use_table(const PropBlock &P) { return P.q2m >= kSieTabQ2; }

// Entry j of proposal P's table: [j + 1/2, H1 coefficients (t^0 .. t^6), H2
// coefficients, padding], t = u kSieIntervals - (j + 1/2) in [-1/2, 1/2];
// threads [0, 2 kSieIntervals) write one interval and one component each.
// The caller's next barrier publishes the table.
__device__ inline void sie_setup(const PropBlock &P)
{
    if (!sie_use_table(P) || threadIdx.x >= 2 * kSieIntervals) return;
    const int j = threadIdx.x >> 1, comp = threadIdx.x & 1;
    const double q = sqrt(P.q2m);
    double c[kSieDeg + 1] = {};
    // one node at a time (the kernels' register budget is set by their busiest
    // point, and all the nodes' deflections in flight would be it)
#pragma unroll 1
    for (int k = 0; k <= kSieDeg; ++k) {
        const double u = (j + 0.5 + kSieNode[k]) * (1.0 / kSieIntervals);
        double f;
        if (comp == 0) {
            const double s = u / q;
            f = sie_a1(s, P.ce, P.bsie, P.bsc) / s;
        } else {
            const double s = sqrt((1.0 - u) * (1.0 + u));
            f = sie_a2(s, P.ce, P.bsie, P.bsc) / s;
        }
#pragma unroll
        for (int i = 0; i <= kSieDeg; ++i) c[i] = fma(kSieInterp[i][k], f, c[i]);
    }
    double *e = sie_table() + j * kSieEntry;
    if (comp == 0) e[0] = j + 0.5;
#pragma unroll
    for (int i = 0; i <= kSieDeg; ++i) e[1 + comp * (kSieDeg + 1) + i] = c[i];
}

// ray_trace with the deflection from the table; qn = q kSieIntervals.
__device__ __forceinline__ void ray_trace_tab(double x1, double x2, double u1, double u2, const PropBlock &P,
                                              double qn, double &w1, double &w2)
{
    const double psi2 = fma(P.q2m, x1 * x1, x2 * x2);
    const double ir = rsq_psi(psi2);
    const double s1 = x1 * ir, s2 = x2 * ir;
    const double un = fabs(s1) * qn;   // u kSieIntervals
    // the entry's byte offset by a 24-bit multiply (full rate; j <= 31)
    const unsigned j = min((unsigned)un, (unsigned)(kSieIntervals - 1));
    const double *e = reinterpret_cast<const double *>(reinterpret_cast<const char *>(sie_table()) +
                                                       __umul24(j, (unsigned)(kSieEntry * sizeof(double))));
    const double t = un - e[0];
    double h1 = e[kSieDeg + 1];
#pragma unroll
    for (int i = kSieDeg - 1; i >= 0; --i) h1 = fma(h1, t, e[1 + i]);
    // the second set of coefficients is read after the first sum: 12 fewer
    // registers live at once (other waves hide the LDS latency)
    asm volatile("" ::: "memory");
    double h2 = e[2 * kSieDeg + 2];
#pragma unroll
    for (int i = kSieDeg - 1; i >= 0; --i) h2 = fma(h2, t, e[kSieDeg + 2 + i]);
    w1 = u1 - s1 * h1;
    w2 = u2 - s2 * h2;
}

// Elliptical power law (Sec. 2.4: kappa = (3 - gamma)/2 (theta_E / R_p)^(gamma - 1)
// on the SIE's elliptical radius R_p, so gamma = 2 is the SIE).  In the frame
// of the mass ellipse, with R e^(i phi) = q x1 + i x2, t = gamma - 1,
// b = theta_E sqrt(q) and f = (1 - q)/(1 + q), the deflection is (Tessore &
// Metcalf 2015, the hypergeometric function written as its series)
//   alpha1 + i alpha2 = 2 b^t / (1 + q) R^(1 - t) e^(i phi) sum_n a_n e^(2 i n phi),
//   a_0 = 1,  a_n = -f (2n - 2 + t) / (2n + 2 - t) a_(n-1),  |a_n| <= f^n.
// The sum is taken by Horner in w = e^(2 i phi) with the proposal's
// coefficients from LDS (epl_setup); R^(1 - t) = 2^((1 - t)/2 log2 R^2), with
// log2 R^2 refined by one Newton step on 2^l = R^2 and both powers of two at
// degree 11 (4e-16): the deflection is good to ~1e-14 relative.  alpha = 0 for
// R^2 < 1e-30 (a sub-pixel within 1e-15 arcsec of the mass centre).
__device__ __forceinline__ double *epl_coefs()
{
    __shared__ double c[kEplMaxTerms];
    return c;
}
__device__ __forceinline__ int *epl_nterms()
{
    __shared__ int n;
    return &n;
}

// The series coefficients of proposal P into LDS, by thread 0, with the number
// of terms that brings the tail f^N / (1 - f) below 1e-16 (at most
// kEplMaxTerms: axis ratios below 0.15 then keep a tail above 1e-16).  The
// caller's next barrier publishes them.
__device__ inline void epl_setup(const PropBlock &P)
{
    if (threadIdx.x != 0) return;
    const double f = -P.epl_mf, t = 1.0 - 2.0 * P.epl_h;
    int N = 1;
    if (f > 0.0) N = (int)ceil(log(1e-16 * (1.0 - f)) / log(f));
    N = N < 1 ? 1 : N > kEplMaxTerms ? kEplMaxTerms : N;
    double *c = epl_coefs();
    double a = 1.0;
    c[0] = 1.0;
    for (int n = 1; n < N; ++n) {
        a *= P.epl_mf * (2.0 * n - 2.0 + t) / (2.0 * n + 2.0 - t);
        c[n] = a;
    }
    *epl_nterms() = N;
}

__device__ __forceinline__ void ray_trace_epl(double x1, double x2, double u1, double u2, const PropBlock &P,
                                              double &w1, double &w2)
{
    const double psi2 = fma(P.q2m, x1 * x1, x2 * x2);   // R^2
    double a1 = 0.0, a2 = 0.0;
    if (psi2 >= 1e-30) {
        const double ir = rsq_nr(psi2);
        const double c1 = P.epl_q * x1 * ir, s1 = x2 * ir;                 // e^(i phi)
        const double wr = fma(c1, c1, -(s1 * s1)), wi = 2.0 * c1 * s1;     // e^(2 i phi)
        const double *c = epl_coefs();
        const int N = __builtin_amdgcn_readfirstlane(*epl_nterms());
        double sr = c[N - 1], si = 0.0;
        for (int n = N - 2; n >= 0; --n) {
            const double tr = fma(sr, wr, fma(-si, wi, c[n]));
            si = fma(sr, wi, si * wr);
            sr = tr;
        }
        const double l0 = log2_r2(psi2);
        const double l1 = fma(fma(psi2, exp2_64(kExp2Hi64, -l0), -1.0), 1.4426950408889634, l0);
        const double mag = P.epl_pref * exp2_64(kExp2Hi64, P.epl_h * l1);
        a1 = mag * fma(c1, sr, -(s1 * si));
        a2 = mag * fma(c1, si, s1 * sr);
    }
    w1 = u1 - a1;
    w2 = u2 - a2;
}

// Sub-pixel sums of pixel (y, x), whose binned value is their mean over the
// s x s sub-pixel centres (Sec. 2.1).  Fine-grid index fx = x s + u maps to position (fx - (nx s - 1)/2) * pixel_scale / s.
// Along a sub-pixel row the x offset dx from the mass centre steps by
// pixel_scale / s (at most 7 FP64 additions, ~1e-15 arcsec from the direct
// product), and everything else linear in x is one FMA in dx with per-row
// constants: the mass-frame coordinates, theta - alpha_shear - source centre
// (rotated into the mass frame), and the lens light's (R/R_e)^2 (a quadratic
// in dx).  Lens and source light
// are summed apart (al, as: sums over the sub-pixels at unit amplitude).
template <int LM>
struct LightChannels {
    static constexpr int N = LM == LIGHT_BOTH ? 2 : LM == LIGHT_DOUBLE ? 4 : 1;
};

// Sub-pixel sums of pixel (y, x) of every light component at unit amplitude,
// in the order: lens (a, b), source (a, b).  Lens light only skips the ray
// trace; two components per galaxy share the elliptical radius of their side,
// whose second component differs only in R_e: log2 (R/R_b)^2 = log2 (R/R_a)^2
// + 2 log2(R_a/R_b).
template <int LM, bool EPL = false, bool TAB = false>
__device__ __forceinline__ void binned_channels(const LensGeom &g, const PropBlock &P, int y, int x,
                                                double (&acc)[LightChannels<LM>::N])
{
    constexpr bool LENS = LM != LIGHT_SRC, SRC = LM != LIGHT_LENS, DBL = LM == LIGHT_DOUBLE;
    constexpr int IS = DBL ? 2 : LENS ? 1 : 0;   // index of the (first) source channel
    constexpr int N = LightChannels<LM>::N;
    const int s = g.s;
    const double x0 = ((double)(x * s) - g.cfx) * g.sd;
    const double dx0 = x0 - P.xm;
    // the step and the 2^x table's leading coefficient live in VGPRs: as SGPR
    // pairs they are spilled or rematerialised on every sub-pixel
    double h = g.sd, lead = leading(kExp2_64);
    asm("" : "+v"(h), "+v"(lead));
    const double qn = TAB ? sqrt(P.q2m) * kSieIntervals : 0.0;
#pragma unroll
    for (int c = 0; c < N; ++c) acc[c] = 0.0;
    const double el = DBL ? g.fix_e[0] : P.lens.e, Bl = DBL ? g.fix_B[0] : P.lens.B;
    const double es = DBL ? g.fix_e[2] : P.src.e, Bs = DBL ? g.fix_B[2] : P.src.B;
    // the FP32 log2 of the Sersic radii only for indices >= 1/2
    // (log2_r2_sersic), and not for two components per galaxy: the second
    // one's exponent takes the first one's log2 shifted by 2 log2(R_a/R_b),
    // so an ulp of a large first log2 can land where the second profile is
    // still bright
    float thr_l = !DBL && el <= 1.0 ? -2.0f : __builtin_inff();
    float thr_s = !DBL && es <= 1.0 ? -2.0f : __builtin_inff();
    // in VGPRs too: the kernels have no scalar registers to spare
    asm("" : "+v"(thr_l), "+v"(thr_s));
    for (int v = 0; v < s; ++v) {
        const double yy = ((double)(y * s + v) - g.cfy) * g.sd;
        const double dy = yy - P.ym;
        // values at dx = 0 of: x1 = cm dx + sm dy, x2 = cm dy - sm dx and of
        // u = R(-phi_m) (theta - alpha_shear - source centre)
        const double c1 = P.sm * dy, c2 = P.cm * dy;
        const double cu1 = fma(P.bu1, yy, P.au1), cu2 = fma(P.bu2, yy, P.au2);
        const double rs = P.lens.S * dy, rq = P.lens.Q * (dy * dy);
        // the channel values of the sub-pixel at offset dx
        auto sub = [&](double dx, double (&val)[N]) {
            if constexpr (SRC) {
                double w1, w2;
                if constexpr (EPL)
                    ray_trace_epl(fma(P.cm, dx, c1), fma(-P.sm, dx, c2), fma(P.ku1, dx, cu1), fma(P.ku2, dx, cu2), P,
                                  w1, w2);
                else if constexpr (TAB)
                    ray_trace_tab(fma(P.cm, dx, c1), fma(-P.sm, dx, c2), fma(P.ku1, dx, cu1), fma(P.ku2, dx, cu2), P,
                                  qn, w1, w2);
                else
                    ray_trace(fma(P.cm, dx, c1), fma(-P.sm, dx, c2), fma(P.ku1, dx, cu1), fma(P.ku2, dx, cu2), P, w1,
                              w2);
                if constexpr (LENS && !DBL) {
                    val[0] = sersic_lg(log2_r2_sersic(fma(fma(P.lens.P, dx, rs), dx, rq), thr_l), el, Bl, lead);
                    val[1] = sersic_lg(log2_r2_sersic(ellip_r2(w1, w2, P.src), thr_s), es, Bs, lead);
                } else {
                    const double lgs = log2_r2_sersic(ellip_r2(w1, w2, P.src), thr_s);
                    val[IS] = sersic_lg(lgs, es, Bs, lead);
                    if constexpr (DBL) val[IS + 1] = sersic_lg(lgs + P.dlg_s, g.fix_e[3], g.fix_B[3], lead);
                }
            }
            if constexpr (LENS && (DBL || !SRC)) {
                const double lgl = log2_r2_sersic(fma(fma(P.lens.P, dx, rs), dx, rq), thr_l);
                val[0] = sersic_lg(lgl, el, Bl, lead);
                if constexpr (DBL) val[1] = sersic_lg(lgl + P.dlg_l, g.fix_e[1], g.fix_B[1], lead);
            }
        };
        double dx = dx0;
        int u = 0;
        // two sub-pixels per step (one-component and two-channel models, direct
        // deflection), with the positions and the order of the additions of one
        // at a time: measured +2% on the survey-scale lens (four channels would
        // spill; with the deflection table it measured 1.6% and 4% slower on the
        // batched and survey-scale lenses)
        for (; !DBL && !TAB && u + 2 <= s; u += 2) {
            const double dxb = dx + h;
            double va[N], vb[N];
            sub(dx, va);
            sub(dxb, vb);
#pragma unroll
            for (int c = 0; c < N; ++c) acc[c] += va[c];
#pragma unroll
            for (int c = 0; c < N; ++c) acc[c] += vb[c];
            dx = dxb + h;
        }
        for (; u < s; ++u) {
            double va[N];
            sub(dx, va);
#pragma unroll
            for (int c = 0; c < N; ++c) acc[c] += va[c];
            dx += h;
        }
    }
}

template <bool EPL = false, bool TAB = false>
__device__ __forceinline__ void binned_sums(const LensGeom &g, const PropBlock &P, int y, int x, double &al_out,
                                            double &as_out)
{
    double acc[2];
    binned_channels<LIGHT_BOTH, EPL, TAB>(g, P, y, x, acc);
    al_out = acc[0];
    as_out = acc[1];
}

template <bool EPL = false, bool TAB = false>
__device__ __forceinline__ float binned_pixel(const LensGeom &g, const PropBlock &P, int y, int x)
{
    double al, as;
    binned_sums<EPL, TAB>(g, P, y, x, al, as);
    return (float)(fma(P.lens.I, al, P.src.I * as) * g.inv_s2);
}

// The unit-amplitude channels of pixel (y, x) (binned values, FP32), for
// amplitudes solved by non-negative least squares (Sec. 2.3).
template <int LM, bool EPL = false, bool TAB = false>
__device__ __forceinline__ void binned_pixel_channels(const LensGeom &g, const PropBlock &P, int y, int x,
                                                      float (&ch)[LightChannels<LM>::N])
{
    double acc[LightChannels<LM>::N];
    binned_channels<LM, EPL, TAB>(g, P, y, x, acc);
#pragma unroll
    for (int c = 0; c < LightChannels<LM>::N; ++c) ch[c] = (float)(acc[c] * g.inv_s2);
}

// Sersic b_n: root of P(2n, b) = 1/2 (Eq. 9), FP64 Newton safeguarded by
// bisection on [0, 2n + 1].  P by its power series, which converges for every
// b in the bracket; the median of Gamma(2n) lies below 2n.  Host only (the
// fixed indices of two-component light); the device uses sersic_bn_fit.
__host__ inline double sersic_bn(double n)
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
        // Newton converges quadratically: after a step below 1e-9 relative the new
        // iterate is exact to rounding (~1e-15 from the series and exp); waiting for
        // a step below 4e-16 instead runs up to 11 iterations bouncing at the last ulp
        if (dx <= 1e-9 * x || hi - lo <= 4e-16 * x) break;
    }
    return x;
}

// b_n of Eq. 9 from the piecewise fit (lens_approx.h): the quarter-octave
// interval of n from an FP32 log2 (each interval's fit covers a rounding across
// its edges), then one degree-10 Horner pass in FP64; within 5e-15 relative of
// the root for n in [kNMin, kNMax], where the iteration above needs an
// incomplete-gamma series with a division per term at every Newton step.
__device__ __forceinline__ double sersic_bn_fit(double n)
{
    int j = (int)__builtin_floorf((float)kBnPerOctave * hw_log2((float)(n * (1.0 / kBnLo))));
    j = j < 0 ? 0 : j > kBnIntervals - 1 ? kBnIntervals - 1 : j;
    const double u = (n - kBnMid[j]) * kBnInvHalf[j];
    const double *c = kBnCoef[j];
    double r = c[kBnDeg];
#pragma unroll
    for (int i = kBnDeg - 1; i >= 0; --i) r = fma(r, u, c[i]);
    return r;
}

}  // namespace lensk
