"""Writes lens_approx.h: polynomial coefficients for the device math.

Functions of the FP64 part of the forward model:
  F(t) = atan(t) / t   on |t| <= 1  (|t| > 1 is reduced by atan t = pi/2 - atan(1/t))
  G(t) = atanh(t) / t  on |t| <= 1/2 (|t| > 1/2 is reduced by the addition formula)
  2^f                  on |f| <= 1/2 (2^y = 2^round(y) 2^(y - round(y))), at two degrees
  b_n                  the Sersic constant of Eq. 9, the root b of P(2n, b) = 1/2
                       (P: regularized lower incomplete gamma), piecewise on n
and the interpolation matrix that turns values at the Chebyshev nodes of
[-1/2, 1/2] into the coefficients of the interpolating polynomial (the
per-proposal deflection tables of the SIE).
F and G are fitted as polynomials in w = t^2, 2^f in f, b_n in the interval's
own variable u, by least squares in *relative* error on Chebyshev-distributed
nodes (a near-minimax fit), with the function values taken at 40 significant
digits (mpmath).  Run from this directory:
    python gen_approx.py > lens_approx.h
"""
import sys

import mpmath as mp
import numpy as np

mp.mp.dps = 40


def f_atan(w):
    w = mp.mpf(w)
    if w == 0:
        return mp.mpf(1)
    s = mp.sqrt(w)
    return mp.atan(s) / s


def f_atanh(w):
    w = mp.mpf(w)
    if w == 0:
        return mp.mpf(1)
    s = mp.sqrt(w)
    return mp.atanh(s) / s


def f_exp2(x):
    return mp.power(2, mp.mpf(x))


def sersic_bn(n):
    """b_n: the root b of P(2n, b) = 1/2.  Start: the large-n expansion
    2n - 1/3 + 4/(405 n); for small n, the leading term of the series of P,
    b^(2n) / Gamma(2n + 1) = 1/2."""
    n = mp.mpf(n)
    a = 2 * n
    x0 = a - mp.mpf(1) / 3 + mp.mpf(4) / (405 * n) if n > 0.35 else (mp.gamma(a + 1) / 2) ** (1 / a)
    return mp.findroot(lambda b: mp.gammainc(a, 0, b, regularized=True) - mp.mpf(1) / 2, x0)


# b_n table: quarter-octave intervals in n from BN_LO, fitted on the interval
# widened by 2.5% of its half-width either side (the device picks the interval
# from an FP32 log2, which may round across an edge)
BN_LO, BN_PER_OCT, BN_INTERVALS, BN_DEG, BN_WIDEN = 0.1, 4, 31, 10, 1.025


def fit_bn():
    mids, invh, coefs, worst = [], [], [], 0.0
    npts = 60
    k = np.arange(npts)
    u = BN_WIDEN * np.cos(np.pi * (k + 0.5) / npts)
    uv = np.linspace(-BN_WIDEN, BN_WIDEN, 201)
    for j in range(BN_INTERVALS):
        lo = mp.mpf(BN_LO) * mp.power(2, mp.mpf(j) / BN_PER_OCT)
        hi = mp.mpf(BN_LO) * mp.power(2, mp.mpf(j + 1) / BN_PER_OCT)
        m, h = (lo + hi) / 2, (hi - lo) / 2
        y = np.array([float(sersic_bn(m + h * mp.mpf(float(v)))) for v in u])
        V = np.vander(u, BN_DEG + 1, increasing=True) / y[:, None]
        c, *_ = np.linalg.lstsq(V, np.ones_like(y), rcond=None)
        yv = np.array([float(sersic_bn(m + h * mp.mpf(float(v)))) for v in uv])
        worst = max(worst, float(np.abs(np.polyval(c[::-1], uv) / yv - 1).max()))
        mids.append(float(m))
        invh.append(float(1 / h))
        coefs.append(c)
    return mids, invh, coefs, worst


def emit_bn(mids, invh, coefs, err):
    out = ["// b_n of Eq. 9 (Sersic): %d intervals of a quarter octave in n from %.1f (to %.4g);"
           % (BN_INTERVALS, BN_LO, BN_LO * 2 ** (BN_INTERVALS / BN_PER_OCT)),
           "// on interval j, b_n = sum_i kBnCoef[j][i] u^i, u = (n - kBnMid[j]) kBnInvHalf[j];",
           "// max relative fit error %.2e for |u| <= %.3f" % (err, BN_WIDEN),
           "constexpr int kBnIntervals = %d, kBnPerOctave = %d, kBnDeg = %d;" % (BN_INTERVALS, BN_PER_OCT, BN_DEG),
           "constexpr double kBnLo = %.17e;" % BN_LO,
           "__device__ static constexpr double kBnMid[%d] = {" % BN_INTERVALS]
    out += ["    %.17e," % v for v in mids]
    out += ["};", "__device__ static constexpr double kBnInvHalf[%d] = {" % BN_INTERVALS]
    out += ["    %.17e," % v for v in invh]
    out += ["};", "__device__ static constexpr double kBnCoef[%d][%d] = {" % (BN_INTERVALS, BN_DEG + 1)]
    for c in coefs:
        out += ["    {" + ", ".join("%.17e" % v for v in c) + "},"]
    out += ["};"]
    return "\n".join(out)


# degree of the per-interval polynomials of the SIE deflection tables
SIE_DEG = 5


def emit_sie_interp():
    """Nodes t_k = cos((2k + 1) pi / (2 N)) / 2, k < N = SIE_DEG + 1, and the
    inverse of the Vandermonde matrix V[k][i] = t_k^i, at 40 digits."""
    n = SIE_DEG + 1
    nodes = [mp.cos((2 * k + 1) * mp.pi / (2 * n)) / 2 for k in range(n)]
    V = mp.matrix(n, n)
    for k in range(n):
        for i in range(n):
            V[k, i] = nodes[k] ** i
    M = V ** -1
    snap = lambda v: 0.0 if abs(v) < 1e-30 else float(v)   # the middle node is 0: exact zeros
    out = ["// Interpolation at the %d Chebyshev nodes of [-1/2, 1/2]: the polynomial of" % n,
           "// degree %d through (kSieNode[k], f_k) is sum_i c_i t^i, c_i = sum_k kSieInterp[i][k] f_k" % SIE_DEG,
           "constexpr int kSieDeg = %d;" % SIE_DEG,
           "__device__ static constexpr double kSieNode[%d] = {" % n]
    out += ["    %.17e," % snap(v) for v in nodes]
    out += ["};", "__device__ static constexpr double kSieInterp[%d][%d] = {" % (n, n)]
    for i in range(n):
        out += ["    {" + ", ".join("%.17e" % snap(M[i, k]) for k in range(n)) + "},"]
    out += ["};"]
    return "\n".join(out)


def fit(f, a, b, deg, npts=4000):
    k = np.arange(npts)
    x = 0.5 * (a + b) + 0.5 * (b - a) * np.cos(np.pi * (k + 0.5) / npts)
    y = np.array([float(f(v)) for v in x])
    V = np.vander(x, deg + 1, increasing=True) / y[:, None]
    c, *_ = np.linalg.lstsq(V, np.ones_like(y), rcond=None)
    xs = np.linspace(a, b, 20001)
    ys = np.array([float(f(v)) for v in xs])
    err = np.abs(np.polyval(c[::-1], xs) / ys - 1).max()
    return c, err


def emit(name, c, err, dom, ctype="float"):
    out = ["// %s: max relative fit error %.2e on w in %s" % (name, err, dom),
           "__device__ static constexpr %s %s[%d] = {" % (ctype, name, len(c))]
    if ctype == "float":
        out += ["    %.9ef," % v for v in c]
    else:
        out += ["    %.17e," % v for v in c]
    out += ["};"]
    return "\n".join(out)


def main():
    # Degrees from what each use needs, measured as the worst shift of the
    # parity metric |dlnL| / (chi2/2 + |C|) when an FP64 forward model of the
    # survey-scale lens swaps the exact function for the fitted polynomial, over
    # prior-box proposals, Sersic indices up to 20 and mass axis ratios down to
    # 0.05 (sources with n ~ 20 are the most sensitive):
    #   atan   degree 9: 1.0e-7, 10: below that           -> 10
    #   atanh  degree 5: 1.3e-6, 6: 3.5e-8                  -> 6
    #   2^x for t = (R/R_e)^(1/n)  degree 5: 2.7e-6, 6: 4.1e-8  -> 6
    #   2^x for the final 2^(B (1 - t))  degree 4: 1.2e-6, 5: 3.7e-8, 6: 3.9e-10
    #   -> 6, one table for both (degree 5 there raised the worst Sersic-index
    #   sweep error on the device from 5.2e-7 to 5.9e-7 and saved no time)
    ca64, ea64 = fit(f_atan, 0.0, 1.0, 10)
    ch64, eh64 = fit(f_atanh, 0.0, 0.25, 6)
    ce64, ee64 = fit(f_exp2, -0.5, 0.5, 6)
    # 2^x at the FP64 rounding level, for the power-law mass: the deflection
    # (b/R)^(gamma - 2) enters the ray trace directly, where ~1e-9 relative
    # already moves lnL next to a steep source centre
    cx64, ex64 = fit(f_exp2, -0.5, 0.5, 11)
    print("// Generated by gen_approx.py; do not edit.  Coefficients c[0..N-1] of")
    print("// sum_i c[i] w^i, lowest order first.")
    print("#pragma once")
    print(emit("kAtanOverT64", ca64, ea64, "[0, 1]", "double"))
    print(emit("kAtanhOverT64", ch64, eh64, "[0, 1/4]", "double"))
    print(emit("kExp2_64", ce64, ee64, "[-1/2, 1/2] (2^f, f = w)", "double"))
    print(emit("kExp2Hi64", cx64, ex64, "[-1/2, 1/2] (2^f, f = w)", "double"))
    # b_n: degree 10 on quarter octaves reaches the FP64 least-squares floor
    # (~2e-15; degree 8 leaves 3e-13 on the first intervals)
    print(emit_bn(*fit_bn()))
    print(emit_sie_interp())


if __name__ == "__main__":
    sys.exit(main())
