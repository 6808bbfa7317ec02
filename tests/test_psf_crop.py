"""The PSF tail crop of lens_load_data (host logic, no GPU): lens_psf_crop against
a brute-force restatement of its rule, and the bound it guarantees."""
import math

import numpy as np
import pytest

from paper_2503_08586_amd import binding, synth


def brute(psf, tail):
    """Smallest centred odd square whose outside taps carry <= tail * sum|K| (tail 0 -> 2^-48)."""
    k = psf.shape[0]
    if tail < 0:
        return k
    tol = tail if tail > 0 else 2.0 ** -48
    r = k // 2
    tot = np.abs(psf).sum()
    for R in range(r):
        inside = np.zeros_like(psf, dtype=bool)
        inside[r - R:r + R + 1, r - R:r + R + 1] = True
        if np.abs(psf[~inside]).sum() <= tol * tot:
            return 2 * R + 1
    return k


@pytest.fixture(scope="module")
def lib():
    try:
        return binding.load()
    except RuntimeError as e:
        pytest.skip(str(e))


def test_survey_psf_crops_to_13(lib):
    psf = synth.config2(nprop=1)[0].psf                      # 21x21 Gaussian, FWHM 2 px
    assert binding.lens_psf_crop(psf) == brute(psf, 0.0) == 13
    assert binding.lens_psf_crop(psf, -1.0) == 21           # negative: full kernel
    # the discarded weight is within the stated bound
    r, R = 10, 6
    out = np.abs(psf).sum() - np.abs(psf[r - R:r + R + 1, r - R:r + R + 1]).sum()
    assert out <= 2.0 ** -48 * np.abs(psf).sum()


def test_heavy_tails_are_kept(lib):
    psf = synth.config4(nlens=1, nprop=1)[0].psf             # 41x41 Moffat beta = 3
    assert binding.lens_psf_crop(psf) == 41


@pytest.mark.parametrize("seed", range(12))
def test_random_kernels_match_brute_force(lib, seed):
    rng = np.random.default_rng(seed)
    k = int(rng.choice([1, 3, 5, 9, 15, 21, 33]))
    y, x = np.mgrid[:k, :k] - k // 2
    width = rng.uniform(0.3, 4.0)
    psf = np.exp(-0.5 * (x * x + y * y) / width ** 2) * rng.uniform(0.5, 1.5, (k, k))
    psf *= np.where(rng.random((k, k)) < 0.1, -1.0, 1.0)   # a few negative taps: |weight| counts
    for tail in (0.0, 1e-3, 1e-8, 2.0 ** -60, -1.0):
        assert binding.lens_psf_crop(psf, tail) == brute(psf, tail), (k, tail)


def test_edge_kernels(lib):
    assert binding.lens_psf_crop(np.ones((1, 1))) == 1
    assert binding.lens_psf_crop(np.zeros((7, 7))) == 1      # nothing outside the centre
    delta = np.zeros((9, 9)); delta[4, 4] = 1.0
    assert binding.lens_psf_crop(delta) == 1
    corner = np.zeros((9, 9)); corner[0, 0] = 1e-300; corner[4, 4] = 1.0
    assert binding.lens_psf_crop(corner) == 1                # 1e-300 of the weight: dropped
    corner[0, 0] = 1e-10
    assert binding.lens_psf_crop(corner) == 9                # 1e-10: kept


def test_bad_arguments(lib):
    import ctypes
    out = ctypes.c_int32()
    psf = np.ones((3, 3))
    dp = psf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.lens_psf_crop(dp, 2, 0.0, ctypes.byref(out)) == binding.LENS_EINVAL
    assert lib.lens_psf_crop(dp, 3, math.nan, ctypes.byref(out)) == binding.LENS_EINVAL
    assert lib.lens_psf_crop(None, 3, 0.0, ctypes.byref(out)) == binding.LENS_EINVAL
