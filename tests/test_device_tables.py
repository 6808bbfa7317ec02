"""The polynomial tables the device math is built from (lens_approx.h), read
as text and evaluated in FP64 numpy the way the kernels evaluate them, against
the oracle and numpy's own functions: the Sersic constant b_n of Eq. 9 from its
piecewise fit against the oracle's root of P(2n, b) = 1/2, and atan, atanh and
2^x within the fit errors the header states."""
import math
import os
import re

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2503_08586_amd", "csrc", "lens_approx.h")


def _text():
    with open(HDR) as f:
        return f.read()


def _array(name):
    m = re.search(r"\b%s\[[^=]*=\s*\{(.*?)\};" % name, _text(), re.S)
    assert m, name
    return np.array([float(v) for v in re.findall(r"[-+0-9.eE]+(?=\s*[,}])", m.group(1) + ",")])


def _const(name):
    m = re.search(r"\b%s\s*=\s*([-+0-9.eE]+)" % name, _text())
    assert m, name
    return float(m.group(1))


def _stated_error(name):
    m = re.search(r"// %s: max relative fit error ([0-9.e+-]+)" % name, _text())
    assert m, name
    return float(m.group(1))


def _horner(c, x):
    r = np.full_like(x, c[-1])
    for v in c[-2::-1]:
        r = r * x + v
    return r


class BnTable:
    def __init__(self):
        self.J = int(_const("kBnIntervals"))
        self.per = int(_const("kBnPerOctave"))
        self.deg = int(_const("kBnDeg"))
        self.lo = _const("kBnLo")
        self.mid = _array("kBnMid")
        self.invh = _array("kBnInvHalf")
        self.coef = _array("kBnCoef").reshape(self.J, self.deg + 1)

    def interval(self, n):
        """The device's choice: floor(per * log2(n / lo)) in FP32, clamped."""
        l2 = np.log2((np.asarray(n) * (1.0 / self.lo)).astype(np.float32)).astype(np.float32)
        j = np.floor(np.float32(self.per) * l2).astype(np.int64)
        return np.clip(j, 0, self.J - 1)

    def eval(self, n, j):
        n = np.asarray(n, dtype=np.float64)
        u = (n - self.mid[j]) * self.invh[j]
        out = np.empty_like(n)
        for jj in np.unique(j):
            sel = j == jj
            out[sel] = _horner(self.coef[jj], u[sel])
        return out


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle.default()


def test_bn_table_matches_oracle_root(orc):
    t = BnTable()
    assert t.J == len(t.mid) == len(t.invh)
    # the table covers the model's index range [0.1, 20]
    assert t.lo <= 0.1 and t.lo * 2 ** (t.J / t.per) >= 20.0
    rng = np.random.default_rng(9)
    n = np.concatenate([np.geomspace(0.1, 20.0, 3001), rng.uniform(0.1, 20.0, 2000), [0.1, 0.5, 1.0, 4.0, 20.0]])
    ref = np.array([orc.bn(v) for v in n])
    got = t.eval(n, t.interval(n))
    rel = np.abs(got / ref - 1)
    assert rel.max() < 1e-14, (rel.max(), n[np.argmax(rel)])
    # closed forms: b_(1/2) = ln 2 (P(1, b) = 1 - e^-b); b_1 solves (1 + b) e^-b = 1/2
    half = t.eval(np.array([0.5]), t.interval(np.array([0.5])))[0]
    assert abs(half / math.log(2.0) - 1) < 1e-14
    one = t.eval(np.array([1.0]), t.interval(np.array([1.0])))[0]
    assert abs((1 + one) * math.exp(-one) - 0.5) < 1e-14


def test_bn_table_neighbour_intervals_agree(orc):
    """Near each interval edge the FP32 log2 may round either way: both
    neighbouring fits must hold there."""
    t = BnTable()
    for j in range(1, t.J):
        edge = t.lo * 2 ** (j / t.per)
        if edge > 20.0:
            break
        n = edge * (1 + np.linspace(-1e-4, 1e-4, 9))
        ref = np.array([orc.bn(v) for v in n])
        for jj in (j - 1, j):
            got = t.eval(n, np.full(n.shape, jj))
            assert np.abs(got / ref - 1).max() < 1e-14, (j, jj)


@pytest.mark.parametrize("name,fn,lo,hi,var", [
    ("kAtanOverT64", lambda t: np.arctan(t) / t, 1e-6, 1.0, "t2"),
    ("kAtanhOverT64", lambda t: np.arctanh(t) / t, 1e-6, 0.5, "t2"),
    ("kExp2_64", np.exp2, -0.5, 0.5, "f"),
    ("kExp2Hi64", np.exp2, -0.5, 0.5, "f"),
])
def test_polynomial_tables_within_stated_error(name, fn, lo, hi, var):
    c = _array(name)
    t = np.linspace(lo, hi, 20001)
    w = t * t if var == "t2" else t
    rel = np.abs(_horner(c, w) / fn(t) - 1)
    stated = _stated_error(name)
    # the stated error was measured at 40 digits; FP64 evaluation adds a few ulp
    assert rel.max() <= stated * 1.05 + 4e-16, (name, rel.max(), stated)


# --- the per-proposal SIE deflection table (lens_device.h: sie_setup, ray_trace_tab)

def _src_const(fname, name):
    path = os.path.join(os.path.dirname(HDR), fname)
    with open(path) as f:
        m = re.search(r"\b%s\s*=\s*([-+0-9.eE]+)" % name, f.read())
    assert m, (fname, name)
    return float(m.group(1))


def test_sie_interpolation_matrix():
    """kSieInterp inverts the Vandermonde matrix of the Chebyshev nodes of
    [-1/2, 1/2]: it maps the values of any polynomial of degree <= kSieDeg at
    the nodes to that polynomial's coefficients."""
    deg = int(_const("kSieDeg"))
    nodes = _array("kSieNode")
    M = _array("kSieInterp").reshape(deg + 1, deg + 1)
    k = np.arange(deg + 1)
    assert np.allclose(nodes, 0.5 * np.cos((2 * k + 1) * np.pi / (2 * (deg + 1))), rtol=0, atol=4e-16)
    V = np.vander(nodes, deg + 1, increasing=True)
    assert np.abs(M @ V - np.eye(deg + 1)).max() < 1e-12
    rng = np.random.default_rng(3)
    c = rng.normal(size=deg + 1)
    assert np.abs(M @ (V @ c) - c).max() < 1e-12


class SieTable:
    """The device's table, built the way sie_setup builds it but from the
    oracle's SIE deflection (phi = 0, centre 0: the mass frame), and evaluated
    the way ray_trace_tab evaluates it."""

    def __init__(self, orc, q, theta_e=1.3):
        self.q, self.te, self.orc = q, theta_e, orc
        self.NI = int(_src_const("lens_internal.h", "kSieIntervals"))
        self.deg = int(_const("kSieDeg"))
        nodes = _array("kSieNode")
        M = _array("kSieInterp").reshape(self.deg + 1, self.deg + 1)
        self.c1 = np.zeros((self.NI, self.deg + 1))
        self.c2 = np.zeros((self.NI, self.deg + 1))
        for j in range(self.NI):
            u = (j + 0.5 + nodes) / self.NI
            f1, f2 = [], []
            for uk in u:
                s1, s2 = uk / q, math.sqrt((1 - uk) * (1 + uk))   # on the ellipse q^2 s1^2 + s2^2 = 1
                a1, a2 = orc.sie_deflection(theta_e, q, 0.0, 0.0, 0.0, s1, s2)
                f1.append(a1 / s1)
                f2.append(a2 / s2)
            self.c1[j] = M @ np.array(f1)
            self.c2[j] = M @ np.array(f2)

    def deflection(self, x1, x2):
        ir = 1.0 / math.sqrt(self.q * self.q * x1 * x1 + x2 * x2)
        s1, s2 = x1 * ir, x2 * ir
        un = abs(s1) * (math.sqrt(self.q * self.q) * self.NI)
        j = min(int(un), self.NI - 1)
        t = un - (j + 0.5)
        return s1 * _horner(self.c1[j], np.array([t]))[0], s2 * _horner(self.c2[j], np.array([t]))[0]


@pytest.mark.parametrize("q,tol", [(0.3, 6e-11), (0.4, 1e-11), (0.5, 2e-12), (0.7, 2e-13), (0.95, 1e-13),
                                   (1.0 - 1e-9, 1e-13)])
def test_sie_table_reproduces_the_deflection(orc, q, tol):
    """The table's deflection at points all around the mass centre, radii
    1e-3 .. 10 arcsec, against the oracle's closed-form SIE: the deflection
    depends on the direction alone, so intervals of u = q |x1| / psi cover
    every point.  The tolerance is the interpolation error for this q."""
    assert q * q >= _src_const("lens_device.h", "kSieTabQ2") - 1e-12
    tab = SieTable(orc, q)
    rng = np.random.default_rng(int(q * 1000))
    ang = np.concatenate([rng.uniform(0, 2 * np.pi, 400), np.arange(8) * np.pi / 4])
    rad = np.exp(rng.uniform(np.log(1e-3), np.log(10.0), ang.size))
    worst = 0.0
    for a, r in zip(ang, rad):
        x1, x2 = r * math.cos(a), r * math.sin(a)
        ref = np.array(orc.sie_deflection(tab.te, q, 0.0, 0.0, 0.0, x1, x2))
        got = np.array(tab.deflection(x1, x2))
        worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
    assert worst < tol, worst


def _sersic_exact(B, e, l):
    """exp(-b ((R/R_e)^(1/n) - 1)) = 2^(B (1 - t)), t = 2^(e l), l = log2 (R/R_e)^2."""
    return 2.0 ** (B * (1.0 - 2.0 ** (e * l)))


def _exp2_hw_worst(g, exact):
    """Largest error of exp2_hw(g) against `exact` over either sign of a
    one-ulp error of the FP32 hardware 2^x: 2^round(g) times the 2^x of the
    FP32-rounded remainder and, where g <= 2 (every lane of a wave that takes
    it has g <= 2, but a lane with g <= 2 can sit in a wave that does not),
    also the 2^x of g itself rounded to FP32."""
    k = np.rint(g)
    f = (g - k).astype(np.float32).astype(np.float64)
    g32 = g.astype(np.float32).astype(np.float64)
    worst = np.zeros_like(g)
    for se in (-1.0, 1.0):
        split = np.abs(np.ldexp(2.0 ** f * (1.0 + se * 2.0 ** -23), k.astype(int)) - exact)
        direct = np.abs(2.0 ** g32 * (1.0 + se * 2.0 ** -23) - exact)
        worst = np.maximum(worst, np.where(g <= 2.0, np.maximum(split, direct), split))
    return worst


def _sersic_fp32_log2(B, e, l):
    """Worst case of log2_r2_sersic's fast path: r2 rounded to FP32, its log2
    one FP32 ulp off either way, t in FP64, then exp2_hw."""
    r2 = (2.0 ** l).astype(np.float32)
    l32 = np.log2(r2.astype(np.float64)).astype(np.float32)
    ulp = np.spacing(np.abs(l32)).astype(np.float64)
    exact = _sersic_exact(B, e, l)
    worst = np.zeros_like(l)
    for sl in (-1.0, 1.0):
        t = 2.0 ** (e * (l32.astype(np.float64) + sl * ulp))
        worst = np.maximum(worst, _exp2_hw_worst(np.maximum(B * (1.0 - t), -2000.0), exact))
    return worst


def _sersic_split_log2(B, e, l):
    """Worst case of the exponent-split form (log2_r2): the binary exponent
    exact, the FP32 log2 of the mantissa one ulp off either way, t at the
    FP64 polynomial's 1.9e-9, then exp2_hw."""
    m, E = np.frexp(2.0 ** l)
    lm = np.log2(m.astype(np.float32).astype(np.float64)).astype(np.float32)
    ulp = np.spacing(np.abs(lm)).astype(np.float64)
    exact = _sersic_exact(B, e, l)
    worst = np.zeros_like(l)
    for sl in (-1.0, 1.0):
        t = 2.0 ** (e * (E + lm.astype(np.float64) + sl * ulp)) * (1.0 + sl * 1.9e-9)
        worst = np.maximum(worst, _exp2_hw_worst(np.maximum(B * (1.0 - t), -2000.0), exact))
    return worst


def _worst_relative(orc, form, n_lo, l_lo, l_hi=16.0):
    """Largest error of a Sersic form relative to max(local value, 1/8 of the
    value at R_e), over indices n in [n_lo, 20] and l in [l_lo, l_hi]."""
    w = 0.0
    for n in np.geomspace(n_lo, 20.0, 30):
        B, e = orc.bn(n) / math.log(2.0), 1.0 / (2.0 * n)
        l = np.linspace(l_lo, l_hi, 4001)
        err = form(B, e, l)
        w = max(w, float(np.max(err / np.maximum(_sersic_exact(B, e, l), 0.125))))
    return w


def test_sersic_hardware_log2_error_model(orc):
    """Why log2_r2_sersic takes the FP32 log2 of r2 only for n >= 1/2 and
    log2 r2 >= -2: with every one-ulp error aligned (exp2_hw's included), that
    form stays below 9e-7 of the local brightness (wherever it is above 1/8 of
    its value at R_e), inside the exponent split's own worst case over the
    whole index domain (1.1e-6, at n = 0.1); at n = 0.1 the FP32 form would
    reach ~1.7e-6."""
    fast = _worst_relative(orc, _sersic_fp32_log2, 0.5, -2.0)
    split = _worst_relative(orc, _sersic_split_log2, 0.1, -40.0)
    assert fast < 9e-7, fast
    assert split < 1.15e-6, split
    assert fast < split
    assert _worst_relative(orc, _sersic_fp32_log2, 0.1, -2.0) > 1.2e-6
