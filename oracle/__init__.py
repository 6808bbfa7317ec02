"""FP64 CPU oracle for the batched lens log-likelihood (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of ``bench.py`` use
this package.  The GPU library never imports it; the two share no code.  The
arithmetic lives in ``lens_oracle.c`` (plain C, FP64, libm, OpenMP across
proposals); this module only marshals numpy arrays through ctypes.

``Oracle(path)`` binds one compiled copy of the C file, so that tests can also
load deliberately broken copies (planted mistakes) and check that the pins
catch them.  The module-level functions use the default build.

Sections and equations cited refer to Cao et al. (2025), "CSST Strong Lensing
Preparation: Fast Modelling of Galaxy-Galaxy Strong Lenses in the Big Data Era".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "lens_oracle.c")
LIB_PATH = os.path.join(_HERE, "liblens_oracle.so")
NPARAM_STRIDE = 20

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def compile_oracle(src: str, out: str) -> str:
    """gcc the oracle source ``src`` into the shared library ``out``."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off",
           "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile lens_oracle.c into liblens_oracle.so next to it."""
    if force or not os.path.exists(LIB_PATH):
        compile_oracle(SRC, LIB_PATH)
    return LIB_PATH


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


class Oracle:
    """ctypes view of one compiled oracle library."""

    def __init__(self, path: str = LIB_PATH):
        if path == LIB_PATH and not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        d, i, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
        sig = {
            "oracle_gammainc_lower_reg": ([d, d], d),
            "oracle_bn": ([d], d),
            "oracle_sersic": ([d] * 10, d),
            "oracle_sie_deflection": ([d] * 7 + [_dp, _dp], None),
            "oracle_shear_deflection": ([d, d, d, d, _dp, _dp], None),
            "oracle_epl_deflection": ([d] * 8 + [_dp, _dp], None),
            "oracle_deflection": ([_dp, d, d, _dp, _dp], None),
            "oracle_params_valid": ([_dp], i),
            "oracle_subpixel_xy": ([i, i, d, i, i, i, i, i, _dp, _dp], None),
            "oracle_convolve_same": ([_dp, i, i, _dp, i, _dp], None),
            "oracle_model_image": ([i, i, d, i, i, _dp, _dp, i, _dp], i),
            "oracle_loglike_norm": ([i64, _dp, _u8p], d),
            "oracle_loglike": ([i, i, d, i, i, _dp, _dp, _dp, _u8p, _dp, i64, _dp, _dp, i], i),
            "oracle_loglike_nnls": ([i, i, d, i, i, _dp, _dp, _dp, _u8p, _dp, i64, _dp, _dp, _dp, i], i),
            "oracle_loglike_light": ([i, i, d, i, i, _dp, _dp, _dp, _u8p, _dp, i64, i, _dp, _dp, _dp, _dp, i], i),
            "oracle_num_threads": ([], i),
            "oracle_philox4x32_10": ([_u32p, _u32p, _u32p], None),
            "oracle_stretch_propose": ([i, i, i64, ctypes.c_uint64, d, _dp, _dp, _dp, _dp, _i32p], None),
            "oracle_stretch_accept": ([i, i, i, _dp, _dp, _dp, _dp, _dp, _dp, _i64p], None),
            "oracle_box_logprior": ([_dp, _dp, _dp], d),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        self.lib = lib
        self.path = path

    # -- scalar pieces -------------------------------------------------------
    def gammainc_lower_reg(self, a: float, x: float) -> float:
        """Regularised lower incomplete gamma P(a, x) (enters Sec. 2.4, Eq. 9)."""
        return self.lib.oracle_gammainc_lower_reg(float(a), float(x))

    def bn(self, n: float) -> float:
        """Sersic b_n: the root of Gamma(2n) = 2 gamma(2n, b_n) (Sec. 2.4, Eq. 9)."""
        return self.lib.oracle_bn(float(n))

    def sersic(self, I_e, R_e, n, b_n, q, phi, xc, yc, x, y) -> float:
        """Elliptical Sersic surface brightness at (x, y) (Sec. 2.4, Eqs. 8, 10)."""
        return self.lib.oracle_sersic(*[float(v) for v in (I_e, R_e, n, b_n, q, phi, xc, yc, x, y)])

    def sie_deflection(self, theta_E, q, phi, xm, ym, x, y):
        """SIE deflection (Sec. 2.4: elliptical power law at slope 2) at one point."""
        ax, ay = ctypes.c_double(), ctypes.c_double()
        self.lib.oracle_sie_deflection(float(theta_E), float(q), float(phi), float(xm), float(ym),
                                       float(x), float(y), ctypes.byref(ax), ctypes.byref(ay))
        return ax.value, ay.value

    def epl_deflection(self, theta_E, gamma, q, phi, xm, ym, x, y):
        """Elliptical power-law deflection (Sec. 2.4; gamma = 2 is the SIE) at one point,
        by quadrature of the elliptical-mass integrals."""
        ax, ay = ctypes.c_double(), ctypes.c_double()
        self.lib.oracle_epl_deflection(float(theta_E), float(gamma), float(q), float(phi), float(xm), float(ym),
                                       float(x), float(y), ctypes.byref(ax), ctypes.byref(ay))
        return ax.value, ay.value

    def shear_deflection(self, g1, g2, x, y):
        """External-shear deflection (Sec. 2.4, Eqs. 13-14) at one point."""
        ax, ay = ctypes.c_double(), ctypes.c_double()
        self.lib.oracle_shear_deflection(float(g1), float(g2), float(x), float(y),
                                         ctypes.byref(ax), ctypes.byref(ay))
        return ax.value, ay.value

    def deflection(self, params, x, y):
        """SIE + shear deflection of one proposal at one point."""
        p = _f64(params)
        assert p.size >= 19
        ax, ay = ctypes.c_double(), ctypes.c_double()
        self.lib.oracle_deflection(_ptr(p), float(x), float(y), ctypes.byref(ax), ctypes.byref(ay))
        return ax.value, ay.value

    def params_valid(self, params) -> bool:
        p = _f64(params)
        return bool(self.lib.oracle_params_valid(_ptr(p)))

    def subpixel_xy(self, ny, nx, dpix, s, i, j, v, u):
        """Image-plane position of sub-pixel (v, u) of pixel (i, j)."""
        x, y = ctypes.c_double(), ctypes.c_double()
        self.lib.oracle_subpixel_xy(ny, nx, float(dpix), s, i, j, v, u, ctypes.byref(x), ctypes.byref(y))
        return x.value, y.value

    # -- images ----------------------------------------------------------------
    def convolve_same(self, img, psf):
        """Zero-padded 'same' true convolution (Sec. 2.1, Eq. 3)."""
        img = _f64(img)
        psf = _f64(psf)
        ny, nx = img.shape
        k = psf.shape[0]
        assert psf.shape == (k, k) and k % 2 == 1
        out = np.empty_like(img)
        self.lib.oracle_convolve_same(_ptr(img), ny, nx, _ptr(psf), k, _ptr(out))
        return out

    def model_image(self, ny, nx, dpix, s, psf, params, stage=1):
        """Model image of one proposal: stage 0 binned, 1 convolved, 2 supersampled."""
        psf = _f64(psf)
        k = psf.shape[0]
        p = _f64(params).reshape(-1)
        if p.size == 19:
            p = np.concatenate([p, [0.0]])
        shape = (ny * s, nx * s) if stage == 2 else (ny, nx)
        out = np.empty(shape, dtype=np.float64)
        rc = self.lib.oracle_model_image(ny, nx, float(dpix), s, k, _ptr(psf), _ptr(p), stage, _ptr(out))
        if rc == -2:
            raise ValueError("proposal outside the parameter domain")
        if rc != 0:
            raise ValueError("bad argument to oracle_model_image")
        return out

    # -- likelihood --------------------------------------------------------------
    def loglike_norm(self, sigma, mask) -> float:
        """C = -1/2 sum over the mask of ln(2 pi sigma^2) (Sec. 2.2, Eq. 5)."""
        sigma = _f64(sigma).reshape(-1)
        mask = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        return self.lib.oracle_loglike_norm(sigma.size, _ptr(sigma), _ptr(mask, _u8p))

    def loglike(self, geom, psf, data, sigma, mask, params, nthreads=0, return_chi2=False):
        """lnL of every proposal row of ``params`` ([n, 20] float64), Sec. 2.2, Eq. 5.

        ``geom`` is (ny, nx, pixel_scale, supersample)."""
        ny, nx, dpix, s = geom
        psf = _f64(psf)
        k = psf.shape[0]
        data = _f64(data)
        sigma = _f64(sigma)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert data.shape == (ny, nx) and sigma.shape == (ny, nx) and mask.shape == (ny, nx)
        p = _f64(params).reshape(-1, NPARAM_STRIDE)
        n = p.shape[0]
        out = np.empty(n, dtype=np.float64)
        chi2 = np.empty(n, dtype=np.float64)
        rc = self.lib.oracle_loglike(ny, nx, float(dpix), s, k, _ptr(psf), _ptr(data), _ptr(sigma),
                                     _ptr(mask, _u8p), _ptr(p), n, _ptr(out), _ptr(chi2), int(nthreads))
        if rc != 0:
            raise ValueError("bad argument to oracle_loglike")
        return (out, chi2) if return_chi2 else out

    def loglike_nnls(self, geom, psf, data, sigma, mask, params, nthreads=0, return_chi2=False,
                     return_amps=False):
        """lnL with the two light amplitudes solved by non-negative least squares
        (Sec. 2.3); the amplitude slots of ``params`` are ignored.  Returns lnL,
        plus chi2 and/or the amplitudes [n, 2] (s_l, s_s) when asked."""
        ny, nx, dpix, s = geom
        psf = _f64(psf)
        k = psf.shape[0]
        data = _f64(data)
        sigma = _f64(sigma)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert data.shape == (ny, nx) and sigma.shape == (ny, nx) and mask.shape == (ny, nx)
        p = _f64(params).reshape(-1, NPARAM_STRIDE)
        n = p.shape[0]
        out = np.empty(n, dtype=np.float64)
        chi2 = np.empty(n, dtype=np.float64)
        amps = np.empty((n, 2), dtype=np.float64)
        rc = self.lib.oracle_loglike_nnls(ny, nx, float(dpix), s, k, _ptr(psf), _ptr(data), _ptr(sigma),
                                          _ptr(mask, _u8p), _ptr(p), n, _ptr(out), _ptr(chi2), _ptr(amps),
                                          int(nthreads))
        if rc != 0:
            raise ValueError("bad argument to oracle_loglike_nnls")
        res = (out,)
        if return_chi2:
            res += (chi2,)
        if return_amps:
            res += (amps,)
        return res if len(res) > 1 else out

    LIGHT_COMPONENTS = {0: 2, 1: 1, 2: 1, 3: 4}

    def loglike_light(self, geom, psf, data, sigma, mask, params, model, nfix=None, nthreads=0,
                      return_chi2=False, return_amps=False):
        """lnL of light model ``model`` (0 lens + source, 1 lens only, 2 lensed source only,
        3 two components per galaxy with fixed indices ``nfix``) with all amplitudes
        solved by non-negative least squares (Sec. 2.3).  Amplitudes [n, N] in component order."""
        ny, nx, dpix, s = geom
        psf = _f64(psf)
        k = psf.shape[0]
        data = _f64(data)
        sigma = _f64(sigma)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        p = _f64(params).reshape(-1, NPARAM_STRIDE)
        n = p.shape[0]
        N = self.LIGHT_COMPONENTS[model]
        nf = _f64(nfix if nfix is not None else [1.0, 1.0, 1.0, 1.0]).reshape(4)
        out = np.empty(n, dtype=np.float64)
        chi2 = np.empty(n, dtype=np.float64)
        amps = np.empty((n, N), dtype=np.float64)
        rc = self.lib.oracle_loglike_light(ny, nx, float(dpix), s, k, _ptr(psf), _ptr(data), _ptr(sigma),
                                           _ptr(mask, _u8p), _ptr(p), n, int(model), _ptr(nf), _ptr(out),
                                           _ptr(chi2), _ptr(amps), int(nthreads))
        if rc != 0:
            raise ValueError("bad argument to oracle_loglike_light")
        res = (out,)
        if return_chi2:
            res += (chi2,)
        if return_amps:
            res += (amps,)
        return res if len(res) > 1 else out

    def num_threads(self) -> int:
        return self.lib.oracle_num_threads()

    # -- sampler loop: the stretch move (Goodman & Weare 2010) driven by
    #    Philox4x32-10 (Salmon et al. 2011), posterior of Sec. 2.2 -----------
    def philox(self, ctr, key):
        """The four Philox4x32-10 words of counter ``ctr`` (4 words) under ``key`` (2 words)."""
        c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(4)
        k = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
        out = np.empty(4, dtype=np.uint32)
        self.lib.oracle_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
        return out

    def stretch_propose(self, walkers, half, t, seed, a):
        """Proposals of half ``half`` in iteration ``t``: (Y [W/2, 20], z, ln u, partner index)."""
        w = _f64(walkers).reshape(-1, NPARAM_STRIDE)
        W = w.shape[0]
        assert W % 2 == 0 and half in (0, 1)
        h = W // 2
        Y = np.empty((h, NPARAM_STRIDE))
        z = np.empty(h)
        logu = np.empty(h)
        j = np.empty(h, dtype=np.int32)
        self.lib.oracle_stretch_propose(W, int(half), int(t), int(seed), float(a), _ptr(w), _ptr(Y), _ptr(z),
                                        _ptr(logu), _ptr(j, _i32p))
        return Y, z, logu, j

    def stretch_accept(self, walkers, lnp, half, d, Y, lnpY, z, logu, accepted=None):
        """Acceptance of half ``half`` in place on ``walkers`` [W, 20] and ``lnp`` [W]."""
        assert walkers.dtype == np.float64 and walkers.flags.c_contiguous
        assert lnp.dtype == np.float64 and lnp.flags.c_contiguous
        W = walkers.shape[0]
        Y, lnpY, z, logu = _f64(Y), _f64(lnpY), _f64(z), _f64(logu)
        acc = None
        if accepted is not None:
            assert accepted.dtype == np.int64 and accepted.flags.c_contiguous
            acc = _ptr(accepted, _i64p)
        self.lib.oracle_stretch_accept(W, int(half), int(d), _ptr(walkers), _ptr(lnp), _ptr(Y), _ptr(lnpY),
                                       _ptr(z), _ptr(logu), acc)

    def box_logprior(self, p, lo, hi) -> float:
        """0 inside the uniform box [lo, hi] (every slot), -inf outside."""
        return self.lib.oracle_box_logprior(_ptr(_f64(p)), _ptr(_f64(lo)), _ptr(_f64(hi)))

    def ensemble_iteration(self, walkers, lnp, t, seed, a, lo, hi, loglike, accepted=None, trace=None):
        """One iteration of the ensemble (half 0, then half 1) in place.  ``loglike(P)``
        gives lnL of proposals [m, 20]; those outside the box get lnP = -inf and are
        not evaluated.  ``trace`` (a list) receives (Y, z, ln u, partner, lnP(Y)) per half."""
        d = int(np.count_nonzero(np.asarray(hi) > np.asarray(lo)))
        for half in (0, 1):
            Y, z, logu, j = self.stretch_propose(walkers, half, t, seed, a)
            inside = np.array([self.box_logprior(y, lo, hi) == 0.0 for y in Y])
            lnpY = np.full(len(Y), -np.inf)
            if inside.any():
                lnpY[inside] = loglike(Y[inside])
            self.stretch_accept(walkers, lnp, half, d, Y, lnpY, z, logu, accepted)
            if trace is not None:
                trace.append((Y, z, logu, j, lnpY))


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(LIB_PATH)
    return _default


def __getattr__(name):
    # module-level access to the default oracle's methods: oracle.bn(...), oracle.loglike(...)
    if name.startswith("_"):
        raise AttributeError(name)
    return getattr(default(), name)
