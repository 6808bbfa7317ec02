"""The seeded input generators: deterministic, inside the prior box, normalised PSFs."""
import math

import numpy as np

from paper_2503_08586_amd import synth


def test_params_in_box_and_deterministic():
    a = synth.draw_params(synth.rng_for_config(1), 500)
    b = synth.draw_params(synth.rng_for_config(1), 500)
    assert np.array_equal(a, b)
    assert a.shape == (500, 20) and np.all(a[:, 19] == 0)
    for i, (_, lo, hi) in enumerate(synth.PRIOR_BOX):
        assert a[:, i].min() >= lo and a[:, i].max() <= hi


def test_psfs():
    g = synth.gaussian_psf(21, 0.1, 0.05)
    assert g.shape == (21, 21) and abs(g.sum() - 1) < 1e-14
    assert np.argmax(g) == 10 * 21 + 10 and np.allclose(g, g.T) and np.allclose(g, g[::-1, ::-1])
    m = synth.moffat_psf(41, 0.15, 3.0, 0.05)
    assert abs(m.sum() - 1) < 1e-14
    # FWHM: along a row, the half-maximum crossing sits at FWHM/2 = 1.5 px for the profile
    alpha = 0.15 / (2 * math.sqrt(2 ** (1 / 3) - 1)) / 0.05
    assert abs((1 + 1.5 ** 2 / alpha ** 2) ** -3 - 0.5) < 1e-12


def test_mask_radius():
    m = synth.circular_mask(128, 128, 0.05, 3.0)
    assert m.dtype == np.uint8
    assert abs(int(m.sum()) - math.pi * 60 ** 2) < 200


def test_configs_shapes():
    c1 = synth.config1(nprop=10)[0]
    assert (c1.ny, c1.nx, c1.s, c1.k) == (64, 64, 1, 11) and c1.proposals.shape == (10, 20)
    c3 = synth.config3(nlens=8, scale_props=0.01)
    for L in c3:
        assert 48 <= L.ny <= 160 and L.s in (2, 4) and 11 <= L.k <= 31 and L.k % 2 == 1
    c5 = synth.config5_lenses(6)
    assert all(48 <= L.ny <= 200 and 11 <= L.k <= 41 for L in c5)


def test_ellipticity_roundtrip():
    for q, phi in ((0.6, 0.3), (0.9, 2.5)):
        e1, e2 = synth.qphi_to_e12(q, phi)
        q2, phi2 = synth.e12_to_qphi(e1, e2)
        assert abs(q2 - q) < 1e-14 and abs((phi2 - phi) % math.pi) < 1e-12
