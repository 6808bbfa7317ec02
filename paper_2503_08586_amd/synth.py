"""Seeded synthetic workloads for the lens likelihood (inputs only).

This module draws what the likelihood is evaluated on: proposal vectors inside
a prior box, PSF kernels, fitting-region masks, noise maps and the five
benchmark workloads.  It holds none of the likelihood's own arithmetic (no ray
tracing, no light profile, no convolution, no chi-square): the noise-free data
image of a workload is produced by a ``model_fn`` that the caller passes in.

The prior box follows the paper's parameterisation (Cao et al. 2025, Sec. 2.4
and Table 1) with the ranges of the workloads: SIE theta_E in [0.5, 2] arcsec,
axis ratios in [0.5, 1], angles in [0, pi], mass centre within 0.1 arcsec
(Table 1 gives a 0.1 arcsec Gaussian), shear components in [-0.1, 0.1], Sersic
radii in [0.1, 1] arcsec and indices in [0.5, 4], source centre within 1 arcsec
(Table 1 gives a 1 arcsec Gaussian).  The amplitudes, which the paper solves
linearly (Sec. 2.3), are explicit parameters here, drawn in [0.05, 0.5].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

NPARAM = 19
STRIDE = 20
SEED_BASE = 250308586

# slot -> (name, lo, hi)
PRIOR_BOX = [
    ("theta_E", 0.5, 2.0),
    ("q_m", 0.5, 1.0),
    ("phi_m", 0.0, math.pi),
    ("x_m", -0.1, 0.1),
    ("y_m", -0.1, 0.1),
    ("g1", -0.1, 0.1),
    ("g2", -0.1, 0.1),
    ("I_l", 0.05, 0.5),
    ("R_l", 0.1, 1.0),
    ("n_l", 0.5, 4.0),
    ("q_l", 0.5, 1.0),
    ("phi_l", 0.0, math.pi),
    ("I_s", 0.05, 0.5),
    ("R_s", 0.1, 1.0),
    ("n_s", 0.5, 4.0),
    ("q_s", 0.5, 1.0),
    ("phi_s", 0.0, math.pi),
    ("x_s", -1.0, 1.0),
    ("y_s", -1.0, 1.0),
]
PARAM_NAMES = [p[0] for p in PRIOR_BOX]
SLOT = {name: i for i, name in enumerate(PARAM_NAMES)}


def rng_for_config(c: int) -> np.random.Generator:
    """The root generator of workload ``c`` (1-based)."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + c))


def draw_params(rng: np.random.Generator, n: int) -> np.ndarray:
    """n proposals, iid uniform in the prior box, as a [n, 20] float64 array."""
    lo = np.array([b[1] for b in PRIOR_BOX])
    hi = np.array([b[2] for b in PRIOR_BOX])
    out = np.zeros((n, STRIDE), dtype=np.float64)
    out[:, :NPARAM] = lo + (hi - lo) * rng.random((n, NPARAM))
    return out


# the fixed Sersic indices of the two-component light model (Sec. 3.2): an
# exponential disc and a de Vaucouleurs bulge per galaxy
DOUBLE_SERSIC_N = (1.0, 4.0, 1.0, 4.0)


def double_component_params(rng: np.random.Generator, params: np.ndarray) -> np.ndarray:
    """Proposals of the two-component light model: a copy of ``params`` whose
    n_l and n_s slots hold the second components' R_e, R_a x U[0.3, 3]."""
    out = np.array(params, dtype=np.float64, copy=True)
    n = out.shape[0]
    out[:, SLOT["n_l"]] = out[:, SLOT["R_l"]] * rng.uniform(0.3, 3.0, n)
    out[:, SLOT["n_s"]] = out[:, SLOT["R_s"]] * rng.uniform(0.3, 3.0, n)
    return out


def gaussian_psf(k: int, fwhm: float, dpix: float) -> np.ndarray:
    """k x k Gaussian, point-sampled at pixel centres, normalised to unit sum."""
    assert k % 2 == 1
    sig = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0))) / dpix
    r = (k - 1) // 2
    yy, xx = np.mgrid[-r:r + 1, -r:r + 1].astype(np.float64)
    psf = np.exp(-0.5 * (xx * xx + yy * yy) / (sig * sig))
    return psf / psf.sum()


def moffat_psf(k: int, fwhm: float, beta: float, dpix: float) -> np.ndarray:
    """k x k Moffat [1 + (r/alpha)^2]^-beta, alpha from the FWHM, unit sum."""
    assert k % 2 == 1
    alpha = fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0)) / dpix
    r = (k - 1) // 2
    yy, xx = np.mgrid[-r:r + 1, -r:r + 1].astype(np.float64)
    psf = (1.0 + (xx * xx + yy * yy) / (alpha * alpha)) ** (-beta)
    return psf / psf.sum()


def circular_mask(ny: int, nx: int, dpix: float, radius: float = 3.0) -> np.ndarray:
    """uint8 mask: 1 where the pixel centre lies within ``radius`` arcsec of the centre."""
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    x = (xx - 0.5 * (nx - 1)) * dpix
    y = (yy - 0.5 * (ny - 1)) * dpix
    return (x * x + y * y <= radius * radius).astype(np.uint8)


@dataclasses.dataclass
class LensSpec:
    """One lens: geometry, PSF, noise, mask, truth and the proposals to evaluate."""
    ny: int
    nx: int
    dpix: float
    s: int
    psf: np.ndarray
    sigma: np.ndarray
    mask: np.ndarray
    truth: np.ndarray            # [20]
    proposals: np.ndarray        # [B, 20]
    noise: np.ndarray            # [ny, nx] unit-free noise realisation (already scaled by sigma)
    data: Optional[np.ndarray] = None

    @property
    def k(self) -> int:
        return int(self.psf.shape[0])

    @property
    def geom(self):
        return (self.ny, self.nx, self.dpix, self.s)

    def make_data(self, model_fn: Callable[["LensSpec", np.ndarray], np.ndarray]) -> np.ndarray:
        """data = model_fn(self, truth) + noise; model_fn supplies the noise-free image."""
        m = np.asarray(model_fn(self, self.truth), dtype=np.float64)
        assert m.shape == (self.ny, self.nx)
        self.data = m + self.noise
        return self.data


def _lens(rng, ny, nx, dpix, s, psf, nprop, sigma=0.01, radius=3.0) -> LensSpec:
    truth = draw_params(rng, 1)[0]
    props = draw_params(rng, nprop)
    sig = np.full((ny, nx), sigma, dtype=np.float64)
    noise = rng.normal(0.0, 1.0, (ny, nx)) * sig
    return LensSpec(ny, nx, dpix, s, psf, sig, circular_mask(ny, nx, dpix, radius), truth, props, noise)


def config1(nprop: int = 1000) -> List[LensSpec]:
    """Plain, small: 64x64 at 0.074"/px, s = 1, 11x11 Gaussian FWHM 0.15", 1,000 proposals."""
    rng = rng_for_config(1)
    return [_lens(rng, 64, 64, 0.074, 1, gaussian_psf(11, 0.15, 0.074), nprop)]


def config2(nprop: int = 65536) -> List[LensSpec]:
    """Plain, survey scale: 128x128 at 0.05"/px, s = 4, 21x21 Gaussian FWHM 0.1", 65,536 proposals."""
    rng = rng_for_config(2)
    return [_lens(rng, 128, 128, 0.05, 4, gaussian_psf(21, 0.10, 0.05), nprop)]


def config3(nlens: int = 256, scale_props: float = 1.0) -> List[LensSpec]:
    """Batching: 256 lenses, N ~ U{48..160}, 0.05-0.074"/px, s in {2, 4}, k in {11..31} odd,
    Gaussian FWHM ~ U[0.10, 0.15]", proposals per lens ~ U{128..4096}."""
    root = rng_for_config(3)
    out = []
    for sub in root.spawn(nlens):
        n = int(sub.integers(48, 161))
        dpix = float(sub.uniform(0.05, 0.074))
        s = int(sub.choice([2, 4]))
        k = int(sub.choice(np.arange(11, 32, 2)))
        fwhm = float(sub.uniform(0.10, 0.15))
        b = int(sub.integers(128, 4097))
        b = max(1, int(round(b * scale_props)))
        out.append(_lens(sub, n, n, dpix, s, gaussian_psf(k, fwhm, dpix), b))
    return out


def config4(nlens: int = 64, nprop: int = 16384) -> List[LensSpec]:
    """Precision: 64 lenses, 200x200 at 0.05"/px, s = 4, 41x41 Moffat (beta 3, FWHM 0.15"),
    16,384 proposals each."""
    root = rng_for_config(4)
    psf = moffat_psf(41, 0.15, 3.0, 0.05)
    return [_lens(sub, 200, 200, 0.05, 4, psf, nprop) for sub in root.spawn(nlens)]


def config5_lenses(nlens: int = 1000) -> List[LensSpec]:
    """Serving: resident lenses with N ~ U{48..200}, k ~ U{11..41} odd, Gaussian or Moffat
    (50/50) with FWHM ~ U[0.10, 0.15]", 0.05-0.074"/px, s = 4.  No proposals attached."""
    root = rng_for_config(5)
    out = []
    for sub in root.spawn(nlens):
        n = int(sub.integers(48, 201))
        dpix = float(sub.uniform(0.05, 0.074))
        k = int(sub.choice(np.arange(11, 42, 2)))
        fwhm = float(sub.uniform(0.10, 0.15))
        psf = gaussian_psf(k, fwhm, dpix) if sub.random() < 0.5 else moffat_psf(k, fwhm, 3.0, dpix)
        out.append(_lens(sub, n, n, dpix, 4, psf, 0))
    return out


def poisson_arrivals(rng: np.random.Generator, rate_per_s: float, n: int) -> np.ndarray:
    """Open-loop arrival times (seconds) of n requests at the given mean rate."""
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))


def e12_to_qphi(e1: float, e2: float):
    """Ellipticity components (Sec. 2.4, Eq. 11) -> (q, phi)."""
    e = math.hypot(e1, e2)
    q = (1.0 - e) / (1.0 + e)
    phi = 0.5 * math.atan2(e2, e1)
    return q, phi


def qphi_to_e12(q: float, phi: float):
    """(q, phi) -> ellipticity components (Sec. 2.4, Eq. 11)."""
    f = (1.0 - q) / (1.0 + q)
    return f * math.cos(2.0 * phi), f * math.sin(2.0 * phi)


def gamma_to_g12(gamma: float, phi_ext: float):
    """Shear magnitude/angle -> Cartesian components (Sec. 2.4, Eq. 14; g1 = g cos 2phi)."""
    return gamma * math.cos(2.0 * phi_ext), gamma * math.sin(2.0 * phi_ext)
