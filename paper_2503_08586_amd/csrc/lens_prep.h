// lens_prep.h -- derived constants of one proposal (the prep step of the
// likelihood), shared by the prep kernel and the sampler's fused propose step.
//
// Cao et al. (2025), Sec. 2.4: SIE and shear constants (Eqs. 12-14), Sersic
// constants with b_n from Eq. 9 and the rotation of Eq. 10 folded in.
#pragma once

#include <hip/hip_runtime.h>

#include "lens_device.h"
#include "lens_internal.h"

namespace lensk {

__device__ inline LightK light_constants(double I, double R, double n, double q, double phi)
{
    // x1 = c dx + s dy, x2 = -s dx + c dy, (R_p/R_e)^2 = (q x1^2 + x2^2/q) / R_e^2
    double s, c;
    sincos(phi, &s, &c);
    const double A = q / (R * R), Bq = 1.0 / (q * R * R);
    LightK L;
    L.P = A * c * c + Bq * s * s;
    L.Q = A * s * s + Bq * c * c;
    L.S = 2.0 * (A - Bq) * c * s;
    L.e = 0.5 / n;
    L.B = sersic_bn_fit(n) * 1.4426950408889634;
    L.I = I;
    return L;
}

// Derived constants of the proposal with slots v[0..19] under model code
// (light model | mass << kMassShift).  The light model decides which slots are
// read and validated: lens light only ignores the mass, shear and source
// slots; source only ignores the lens light; two components per galaxy read
// slots n_l and n_s as the second components' R_e (their indices are fixed per
// lens and taken from the lens descriptor by the likelihood kernel).  The
// elliptical power law reads its slope gamma from slot 19 (the SIE ignores it).
__device__ inline PropBlock prep_proposal(const double *v, int code)
{
    PropBlock b{};
    const int lm = code & ((1 << kMassShift) - 1);
    const bool epl = (code >> kMassShift) & 1;
    const bool mass = lm != LIGHT_LENS, lens = lm != LIGHT_SRC, src = lm != LIGHT_LENS, dbl = lm == LIGHT_DOUBLE;
    bool ok = isfinite(v[3]) && isfinite(v[4]);
    if (mass) {
#pragma unroll
        for (int j = 0; j < 7; ++j) ok = ok && isfinite(v[j]);
        ok = ok && v[0] >= 0.0 && v[1] > 0.0 && v[1] <= 1.0;
        if (epl) ok = ok && v[19] >= kGammaMin && v[19] <= kGammaMax;
    }
    if (lens) {
        ok = ok && isfinite(v[8]) && isfinite(v[9]) && isfinite(v[10]) && isfinite(v[11]);
        ok = ok && v[10] > 0.0 && v[10] <= 1.0 && v[8] > 0.0;
        ok = ok && (dbl ? v[9] > 0.0 : v[9] >= kNMin && v[9] <= kNMax);
    }
    if (src) {
#pragma unroll
        for (int j = 13; j < 19; ++j) ok = ok && isfinite(v[j]);
        ok = ok && v[15] > 0.0 && v[15] <= 1.0 && v[13] > 0.0;
        ok = ok && (dbl ? v[14] > 0.0 : v[14] >= kNMin && v[14] <= kNMax);
    }
    const bool amps_ok = isfinite(v[7]) && isfinite(v[12]);
    if (ok) {
        b.valid = (lm == LIGHT_BOTH && amps_ok) ? 1.0 : 2.0;
        b.xm = v[3];
        b.ym = v[4];
        if (mass) {
            const double q = v[1];
            sincos(v[2], &b.sm, &b.cm);
            b.q2m = q * q;
            b.ce = sqrt((1.0 - q) * (1.0 + q));
            b.bsie = v[0] * sqrt(q);
            b.bsc = b.ce > 0.0 ? b.bsie / b.ce : 0.0;
            // theta - alpha_shear - source centre = (lx, ly) with (x = xm + dx)
            //   lx = (1 + g1) x + g2 y - xs,  ly = g2 x + (1 - g1) y - ys,
            // rotated into the mass frame: u1 = cm lx + sm ly, u2 = cm ly - sm lx
            const double g1 = v[5], g2 = v[6], xs = v[17], ys = v[18];
            const double X0 = fma(1.0 + g1, v[3], -xs), Y0 = fma(g2, v[3], -ys);   // lx, ly at x = xm, y = 0
            b.ku1 = fma(b.cm, 1.0 + g1, b.sm * g2);
            b.ku2 = fma(b.cm, g2, -(b.sm * (1.0 + g1)));
            b.au1 = fma(b.cm, X0, b.sm * Y0);
            b.bu1 = fma(b.cm, g2, b.sm * (1.0 - g1));
            b.au2 = fma(b.cm, Y0, -(b.sm * X0));
            b.bu2 = fma(b.cm, 1.0 - g1, -(b.sm * g2));
            if (epl) {
                const double t = v[19] - 1.0;
                b.epl_q = q;
                b.epl_pref = 2.0 * pow(v[0] * sqrt(q), t) / (1.0 + q);
                b.epl_h = 0.5 * (1.0 - t);
                b.epl_mf = -(1.0 - q) / (1.0 + q);
            }
        }
        // two-component light: e and B of the fixed indices come from the lens descriptor
        if (lens) b.lens = light_constants(v[7], v[8], dbl ? 1.0 : v[9], v[10], v[11]);
        if (src) {
            b.src = light_constants(v[12], v[13], dbl ? 1.0 : v[14], v[15], v[16]);
            // the source's quadratic form in the mass frame: beta - centre = R(phi_m) w, so
            // P' w1^2 + Q' w2^2 + S' w1 w2 with [P' S'/2; S'/2 Q'] = R^T [P S/2; S/2 Q] R
            const double c = b.cm, s = b.sm, P = b.src.P, Q = b.src.Q, S = b.src.S;
            b.src.P = fma(P, c * c, fma(Q, s * s, S * (c * s)));
            b.src.Q = fma(P, s * s, fma(Q, c * c, -(S * (c * s))));
            b.src.S = fma(2.0 * (Q - P), c * s, S * ((c - s) * (c + s)));
        }
        if (dbl) {
            b.dlg_l = 2.0 * log2(v[8] / v[9]);
            b.dlg_s = 2.0 * log2(v[13] / v[14]);
        }
    }
    return b;
}

}  // namespace lensk
