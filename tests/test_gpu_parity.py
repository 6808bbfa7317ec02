"""GPU path (through the C ABI) against the FP64 oracle, element by element.

Gate: |lnL_gpu - lnL_oracle| / (chi2/2 + |C|) <= 1e-6 for the FP32 path and
the two splits and 2e-3 for plain BF16
(the reasons are at MODE_TOL and TOL_BF16), with C = -1/2 sum_mask
ln(2 pi sigma^2).  Out-of-domain proposals must be -inf on both sides.
"""
import math

import numpy as np
import pytest

from gpu_cases import TOL_BF16, TOL_FP32, custom_spec, fp32_floor, oracle_data, oracle_loglike, rel_err, say
from paper_2503_08586_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2503_08586_amd import binding
    c = binding.LensContext(0)
    yield c
    c.close()


# storage unit of each convolution mode: FP32, hi+lo FP16 (two planes of 11
# significant bits at each ring row's own scale: 2^-22 relative), plain BF16,
# hi+mid+lo BF16
UNIT = {0: 2.0 ** -24, 1: 2.0 ** -22, 2: 2.0 ** -8, 3: 2.0 ** -24}
MODE_TOL = {0: TOL_FP32, 1: TOL_FP32, 2: TOL_BF16, 3: TOL_FP32}
MODES = [("fp32", 0), ("split", 1), ("bf16", 2), ("split3", 3)]


def _check(spec, got, params, tol=TOL_FP32, label="", storage_floor=False, unit=2.0 ** -24):
    """Element-wise gate.  storage_floor=True (tiny edge-case images only) raises
    each proposal's tolerance to the storage floor of its model image in the
    mode's unit when that exceeds tol; the benchmark configs never use it."""
    ref, chi2, C = oracle_loglike(spec, params)
    assert np.array_equal(np.isneginf(got), np.isneginf(ref)), label
    e = rel_err(got, ref, chi2, C)
    tols = np.full(len(e), tol)
    if storage_floor:
        tols = np.maximum(tols, fp32_floor(spec, params, chi2, C) * unit / 2.0 ** -24)
    say("%s: n=%d max err %.3e p99 %.3e (max tol %.3e)" % (label, len(got), e.max(), np.quantile(e, 0.99), tols.max()))
    assert np.all(e <= tols), (label, e.max(), int(np.argmax(e / tols)))
    return e


def test_c1_all_proposals(ctx):
    say("case: 64x64 s=1 k=11, 1000 proposals")
    spec = synth.config1()[0]
    oracle_data(spec)
    lid = ctx.load(spec)
    got = ctx.loglike(lid, spec.proposals)
    _check(spec, got, spec.proposals, label="c1")
    ctx.unload(lid)


def test_c2_full_call_sampled(ctx):
    say("case: 128x128 s=4 k=21, 65536 proposals in one call, 1024 sampled")
    spec = synth.config2()[0]
    oracle_data(spec)
    lid = ctx.load(spec)
    got = ctx.loglike(lid, spec.proposals)
    assert got.shape == (65536,) and np.all(np.isfinite(got))
    idx = np.random.default_rng(0).choice(np.arange(1, 65535), 1022, replace=False)
    idx = np.concatenate([idx, [0, 65535]])
    _check(spec, got[idx], spec.proposals[idx], label="c2 sampled")
    # the truth itself: chi2 ~ M
    t = ctx.loglike(lid, spec.truth[None, :])
    _check(spec, t, spec.truth[None, :], label="c2 truth")
    ctx.unload(lid)


def test_model_image_stages(ctx):
    say("case: model images, 128x128 s=4 k=21")
    import oracle
    orc = oracle.default()
    spec = synth.config2(nprop=4)[0]
    oracle_data(spec)
    lid = ctx.load(spec)
    for t in range(4):
        p = spec.proposals[t]
        for stage in (0, 1):
            g = ctx.model_image(lid, p, stage)
            r = orc.model_image(spec.ny, spec.nx, spec.dpix, spec.s, spec.psf, p, stage=stage)
            scale = np.abs(r).max()
            err = np.abs(g - r).max() / scale
            say("stage %d proposal %d: max |diff|/max|img| = %.3e" % (stage, t, err))
            assert err < 3e-6
    ctx.unload(lid)


GEOMS = [
    # (name, ny, nx, dpix, s, k, mask)
    ("psf_larger_than_image", 5, 7, 0.2, 1, 11, "full"),
    ("odd_sizes_s3", 17, 23, 0.1, 3, 5, "circle"),
    ("delta_psf", 33, 30, 0.08, 2, 1, "full"),
    ("ring_mask_s4", 40, 37, 0.07, 4, 9, "ring"),
    ("max_psf_63", 64, 64, 0.05, 1, 63, "circle"),
    ("wide_sparse_mask", 9, 130, 0.05, 2, 7, "random"),
    ("single_pixel", 1, 1, 0.1, 2, 3, "full"),
    ("tall_s2_k13", 150, 41, 0.06, 2, 13, "circle"),
    ("s5_k41", 48, 52, 0.05, 5, 41, "circle"),
    ("max_width_4096", 6, 4096, 0.05, 1, 3, "random"),
    ("max_height_4096", 4096, 5, 0.05, 1, 5, "random"),
]


def _mask(kind, ny, nx, dpix, rng):
    if kind == "full":
        return np.ones((ny, nx), np.uint8)
    if kind == "circle":
        return synth.circular_mask(ny, nx, dpix, 0.45 * min(ny, nx) * dpix)
    if kind == "ring":
        a = synth.circular_mask(ny, nx, dpix, 0.45 * min(ny, nx) * dpix)
        b = synth.circular_mask(ny, nx, dpix, 0.2 * min(ny, nx) * dpix)
        return (a - b).astype(np.uint8)
    return (rng.random((ny, nx)) < 0.3).astype(np.uint8)


_geom_cache = {}


def _geom_spec(geom):
    name, ny, nx, dpix, s, k, mk = geom
    if name not in _geom_cache:
        rng = np.random.default_rng(sum(map(ord, name)))
        psf = synth.gaussian_psf(k, 3.0 * dpix, dpix) if k > 1 else np.ones((1, 1))
        psf = psf * (1.0 + 0.3 * rng.random(psf.shape))      # asymmetric, not normalised
        _geom_cache[name] = custom_spec(7, ny, nx, dpix, s, psf, _mask(mk, ny, nx, dpix, rng), 37)
    return _geom_cache[name]


@pytest.mark.parametrize("mode", MODES, ids=[m[0] for m in MODES])
@pytest.mark.parametrize("geom", GEOMS, ids=[g[0] for g in GEOMS])
def test_geometries(ctx, geom, mode):
    name, ny, nx = geom[0], geom[1], geom[2]
    mname, m = mode
    say("case: geometry %s, mode %s" % (name, mname))
    spec = _geom_spec(geom)
    lid = ctx.load(spec, precision=m)
    got = ctx.loglike(lid, spec.proposals)
    # The benchmark workloads keep the plain gates.  These edge images (delta
    # PSF, tiny images, s = 1..5) average little, so a mode's per-pixel storage
    # unit shows through: masks of fewer than 64 pixels in every mode (chi2
    # averages the rounding over the masked pixels only), and every edge image
    # in the two reduced-precision modes, are gated at the mode's storage floor
    # (a worst-case bound) when that exceeds the plain gate.
    _check(spec, got, spec.proposals, tol=MODE_TOL[m], label="%s/%s" % (name, mname),
           storage_floor=int(spec.mask.sum()) < 64 or m in (1, 2), unit=UNIT[m])
    ctx.unload(lid)


def test_mfma_operand_layout(ctx):
    say("case: matrix-core operand layout self-test, BF16 and FP16")
    assert ctx.selftest(0) == 0.0
    assert ctx.selftest(1) == 0.0
    from paper_2503_08586_amd import binding
    with pytest.raises(binding.LensError):
        ctx.selftest(2)


@pytest.mark.parametrize("mode", MODES, ids=[m[0] for m in MODES])
def test_precision_workload(ctx, mode):
    """200x200 px, s = 4, 41x41 Moffat PSF: the precision workload's lens shape."""
    mname, m = mode
    say("case: 200x200 s=4 Moffat k=41, mode %s, 24 proposals" % mname)
    spec = synth.config4(nlens=1, nprop=24)[0]
    oracle_data(spec)
    lid = ctx.load(spec, precision=m)
    got = ctx.loglike(lid, spec.proposals)
    _check(spec, got, spec.proposals, tol=MODE_TOL[m], label="precision/%s" % mname)
    t = ctx.loglike(lid, spec.truth[None, :])
    _check(spec, t, spec.truth[None, :], tol=MODE_TOL[m], label="precision truth/%s" % mname)
    ctx.unload(lid)


def test_mfma_batch_composition_bitwise(ctx):
    say("case: batch composition, split mode")
    spec = synth.config1(nprop=500)[0]
    oracle_data(spec)
    lid = ctx.load(spec, precision=1)
    full = ctx.loglike(lid, spec.proposals)
    perm = np.random.default_rng(2).permutation(500)
    assert np.array_equal(full[perm], ctx.loglike(lid, spec.proposals[perm]))
    assert np.array_equal(full[100:133], ctx.loglike(lid, spec.proposals[100:133]))
    ctx.unload(lid)


def test_empty_mask_and_empty_batch(ctx):
    say("case: empty mask, empty batch")
    spec = custom_spec(3, 20, 20, 0.1, 2, synth.gaussian_psf(5, 0.2, 0.1), np.zeros((20, 20)), 5)
    lid = ctx.load(spec)
    got = ctx.loglike(lid, spec.proposals)
    assert np.all(got == 0.0)
    assert ctx.loglike(lid, np.zeros((0, 20))).shape == (0,)
    ctx.unload(lid)


def test_special_proposals(ctx):
    say("case: special and out-of-domain proposals")
    spec = synth.config1(nprop=1)[0]
    oracle_data(spec)
    lid = ctx.load(spec)
    base = spec.truth.copy()
    S = synth.SLOT

    def mod(**kw):
        p = base.copy()
        for k_, v in kw.items():
            p[S[k_]] = v
        return p

    good = [mod(q_m=1.0), mod(q_l=1.0, q_s=1.0), mod(theta_E=0.0), mod(g1=0.0, g2=0.0),
            mod(I_l=0.0), mod(I_s=0.0), mod(n_l=0.1, n_s=20.0), mod(n_l=20.0, n_s=0.1),
            mod(q_m=0.999999), mod(q_m=0.05), mod(x_m=0.0, y_m=0.0), mod(x_s=0.0, y_s=0.0, q_s=1.0),
            mod(R_s=1e-3), mod(R_l=30.0), mod(theta_E=3.0, q_m=0.3), mod(g1=0.3, g2=-0.3),
            # (R/R_e)^2 beyond FP32's range: an infinite FP32 log2, a NaN
            # exponent, and a brightness of 0 (the oracle's FP64 gives 0 too)
            mod(R_s=1e-20), mod(R_l=1e-20)]
    bad = [mod(theta_E=-1e-9), mod(q_m=0.0), mod(q_l=1.0000001), mod(q_s=-0.2), mod(R_l=0.0),
           mod(R_s=-1.0), mod(n_l=0.0999), mod(n_s=20.01), mod(x_s=math.nan), mod(g2=math.inf),
           mod(I_l=-math.inf)]
    P = np.stack(good + bad)
    got = ctx.loglike(lid, P)
    assert np.all(np.isneginf(got[len(good):]))
    _check(spec, got, P, label="special")
    ctx.unload(lid)


def test_low_axis_ratio_mass(ctx):
    """Mass axis ratios below 0.44 send the minor-axis deflection through its
    logarithm branch (|c u2| > 0.9) on part of the grid; sweep q down to 0.05
    with the rest of each proposal from the prior."""
    say("case: low mass axis ratios (atanh logarithm branch)")
    spec = synth.config1(nprop=96)[0]
    oracle_data(spec)
    lid = ctx.load(spec)
    P = spec.proposals.copy()
    P[:, synth.SLOT["q_m"]] = np.linspace(0.05, 0.45, len(P))
    got = ctx.loglike(lid, P)
    _check(spec, got, P, label="low q_m")
    ctx.unload(lid)


def test_sersic_index_sweep(ctx):
    """Sersic indices over the whole domain [0.1, 20] (log-uniform, both
    components): b_n (R/R_e)^(1/n) grows to ~60 at n = 20 and amplifies any
    error in (R/R_e)^(1/n), so the prior box alone (n <= 4) would not show it."""
    say("case: Sersic index sweep over [0.1, 20]")
    spec = synth.config2(nprop=48)[0]
    spec.s = 2                                   # survey geometry, fewer sub-pixels for the oracle
    oracle_data(spec)
    lid = ctx.load(spec)
    P = spec.proposals.copy()
    rng = np.random.default_rng(20)
    P[:, synth.SLOT["n_l"]] = np.exp(rng.uniform(np.log(0.1), np.log(20.0), len(P)))
    P[:, synth.SLOT["n_s"]] = np.exp(rng.uniform(np.log(0.1), np.log(20.0), len(P)))
    got = ctx.loglike(lid, P)
    _check(spec, got, P, label="n sweep")
    ctx.unload(lid)


def test_psf_tail_crop(ctx):
    """The survey PSF (21x21 Gaussian, FWHM 2 px) is convolved at its 2^-48 tail
    crop (13x13); with psf_tail < 0 the full kernel is used.  Both match the
    oracle, which always convolves with the full kernel, and each other to far
    below the gate."""
    say("case: PSF tail crop, default and full kernel")
    spec = synth.config2(nprop=64)[0]
    spec.s = 2
    oracle_data(spec)
    lc = ctx.load(spec)
    lf = ctx.load(spec, psf_tail=-1.0)
    ic, i_f = ctx.info(lc), ctx.info(lf)
    assert (ic["psf_size"], ic["psf_used"]) == (21, 13)
    assert (i_f["psf_size"], i_f["psf_used"]) == (21, 21)
    assert ic["needed_pixels"] < i_f["needed_pixels"]
    gc, gf = ctx.loglike(lc, spec.proposals), ctx.loglike(lf, spec.proposals)
    _check(spec, gc, spec.proposals, label="psf cropped")
    _check(spec, gf, spec.proposals, label="psf full")
    ref, chi2, C = oracle_loglike(spec, spec.proposals)
    d = rel_err(gc, gf, chi2, C)
    say("cropped vs full kernel: max %.3e" % d.max())
    assert d.max() <= 1e-7
    ctx.unload(lc)
    ctx.unload(lf)


def test_batch_composition_bitwise(ctx):
    say("case: batch composition and order")
    spec = synth.config2(nprop=3000)[0]
    oracle_data(spec)
    lid = ctx.load(spec)
    full = ctx.loglike(lid, spec.proposals)
    perm = np.random.default_rng(1).permutation(3000)
    shuf = ctx.loglike(lid, spec.proposals[perm])
    assert np.array_equal(full[perm], shuf)
    part = ctx.loglike(lid, spec.proposals[1234:1301])
    assert np.array_equal(full[1234:1301], part)
    ctx.unload(lid)


def test_device_entry_point_matches_host(ctx):
    say("case: device-buffer entry point")
    import torch
    spec = synth.config1(nprop=777)[0]
    oracle_data(spec)
    lid = ctx.load(spec)
    host = ctx.loglike(lid, spec.proposals)
    dp = torch.from_numpy(spec.proposals).cuda()
    do = torch.empty(777, dtype=torch.float64, device="cuda")
    ctx.loglike_device(lid, dp, do)
    torch.cuda.synchronize()
    assert np.array_equal(do.cpu().numpy(), host)
    s2 = torch.cuda.Stream()
    do2 = torch.empty(777, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s2):
        ctx.loglike_device(lid, dp, do2, stream=s2)
    s2.synchronize()
    assert np.array_equal(do2.cpu().numpy(), host)
    ctx.unload(lid)


def test_multi_matches_single(ctx):
    say("case: multi-lens call")
    specs = synth.config3(nlens=6, scale_props=0.05)
    lids = []
    for sp in specs:
        oracle_data(sp)
        lids.append(ctx.load(sp))
    outs = ctx.loglike_multi(lids, [sp.proposals for sp in specs])
    for sp, lid, o in zip(specs, lids, outs):
        assert np.array_equal(o, ctx.loglike(lid, sp.proposals))
    _check(specs[0], outs[0][:16], specs[0].proposals[:16], label="multi lens0")
    for lid in lids:
        ctx.unload(lid)


def test_serving_mixed_equals_alone(ctx):
    say("case: serving, mixed vs alone")
    specs = synth.config5_lenses(5)
    lids = []
    for sp in specs:
        oracle_data(sp)
        lids.append(ctx.load(sp))
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(24):
        j = int(rng.integers(0, len(lids)))
        n = int(rng.integers(100, 10001)) if i % 6 else 9000
        P = synth.draw_params(rng, n)
        reqs.append((j, P, ctx.submit(lids[j], P)))
    for j, P, rq in reqs:
        assert ctx.wait(rq) == 0
        alone = ctx.loglike(lids[j], P)
        assert np.array_equal(rq.out, alone)
    st = ctx.stats()
    assert st["requests_done"] >= 24
    _check(specs[reqs[0][0]], reqs[0][2].out[:8], reqs[0][1][:8], label="served")
    for lid in lids:
        ctx.unload(lid)


@pytest.mark.parametrize("mode", [("fp32", 0), ("split", 1)], ids=["fp32", "split"])
def test_multi_graph_replays(ctx, mode):
    """The multi-lens call is a captured graph: replay it several times with eager
    single-lens calls in between; every replay equals the single-lens results."""
    mname, m = mode
    say("case: multi-lens graph replays, mode %s" % mname)
    specs = synth.config3(nlens=10, scale_props=0.04)
    lids = []
    for sp in specs:
        oracle_data(sp)
        lids.append(ctx.load(sp, precision=m))
    singles = [ctx.loglike(lid, sp.proposals) for sp, lid in zip(specs, lids)]
    for rep in range(4):
        outs = ctx.loglike_multi(lids, [sp.proposals for sp in specs])
        for o, ref in zip(outs, singles):
            assert np.array_equal(o, ref), rep
        j = rep % len(specs)
        assert np.array_equal(ctx.loglike(lids[j], specs[j].proposals), singles[j])
    _check(specs[1], outs[1][:12], specs[1].proposals[:12], tol=MODE_TOL[m], label="multi/%s" % mname)
    # a different call shape (subset, other counts) builds its own plan
    outs2 = ctx.loglike_multi(lids[2:5], [sp.proposals[:7] for sp in specs[2:5]])
    for o, ref in zip(outs2, singles[2:5]):
        assert np.array_equal(o, ref[:7])
    for lid in lids:
        ctx.unload(lid)


def test_autotuned_context():
    say("case: autotuned context")
    from paper_2503_08586_amd import binding
    with binding.LensContext(0, autotune=True) as c2:
        for sp in (synth.config2(nprop=64)[0], synth.config4(nlens=1, nprop=8)[0]):
            oracle_data(sp)
            lid = c2.load(sp)
            got = c2.loglike(lid, sp.proposals)
            _check(sp, got, sp.proposals, label="autotuned %dx%d" % (sp.ny, sp.nx))
            c2.unload(lid)


def test_sampler_path_proposals(ctx):
    """Proposals an ensemble sampler makes near a steep (n ~ 3.5) source centre
    with large residuals at the brightest pixels: a regime a uniform draw from
    the prior box rarely reaches, where the Sersic exponent amplifies any
    absolute error in log2 (R/R_e)^2."""
    import oracle
    say("case: 64x64 s=1 k=11, 240 proposals from 5 seeded stretch-move iterations")
    orc = oracle.default()
    spec = synth.config1(nprop=1)[0]
    oracle_data(spec)
    lo = np.array([b[1] for b in synth.PRIOR_BOX] + [0.0])
    hi = np.array([b[2] for b in synth.PRIOR_BOX] + [0.0])
    rng = np.random.default_rng(2)
    w = np.clip(np.clip(spec.truth, lo, hi)[None, :] + 0.02 * (hi - lo)[None, :] * rng.normal(size=(48, 20)), lo, hi)
    lnp = orc.loglike(spec.geom, spec.psf, spec.data, spec.sigma, spec.mask, w)
    props = []
    for t in range(5):
        trace = []
        orc.ensemble_iteration(w, lnp, t, 1234567, 2.0, lo, hi,
                               lambda P: orc.loglike(spec.geom, spec.psf, spec.data, spec.sigma, spec.mask, P),
                               trace=trace)
        props += [Y for Y, _, _, _, _ in trace]
    P = np.concatenate(props)
    lid = ctx.load(spec)
    _check(spec, ctx.loglike(lid, P), P, label="sampler path")
    ctx.unload(lid)


def _random_geoms(n=10, seed=2503):
    """Seeded random geometries: sizes 1-71 px, supersampling 1-8 (6-8 not in
    GEOMS), odd PSF sides 1-63, all four mask kinds."""
    rng = np.random.default_rng(seed)
    out = []
    for i, s in enumerate((6, 7, 8, 1, 2, 3, 4, 5, 6, 8)[:n]):
        ny, nx = int(rng.integers(1, 72)), int(rng.integers(1, 72))
        k = int(rng.choice(np.arange(1, 64, 2)))
        dpix = float(rng.uniform(0.03, 0.12))
        out.append(("rand%d_%dx%d_s%d_k%d" % (i, ny, nx, s, k), ny, nx, dpix, s, k, ("full", "circle", "ring",
                                                                                    "random")[i % 4]))
    return out


RAND_GEOMS = _random_geoms()


def _random_spec(geom, epl):
    name, ny, nx, dpix, s, k, mk = geom
    rng = np.random.default_rng(sum(map(ord, name)) + (7 if epl else 0))
    psf = synth.gaussian_psf(k, 3.0 * dpix, dpix) if k > 1 else np.ones((1, 1))
    psf = psf * (1.0 + 0.3 * rng.random(psf.shape))
    mask = _mask(mk, ny, nx, dpix, rng)
    if mask.sum() == 0:
        mask[ny // 2, nx // 2] = 1
    spec = custom_spec(11 + epl, ny, nx, dpix, s, psf, mask, 24)
    if epl:
        spec.truth = spec.truth.copy()
        spec.truth[19] = 2.1
        spec.proposals = np.array(spec.proposals, copy=True)
        spec.proposals[:, 19] = rng.uniform(1.2, 2.8, len(spec.proposals))
        oracle_data(spec)
    return spec


@pytest.mark.parametrize("geom", RAND_GEOMS, ids=[g[0] for g in RAND_GEOMS])
def test_random_geometries(ctx, geom):
    """fp32 and both splits on every random geometry (PSF windows of one,
    two and three K-chunks per row for the FP16 split), and the elliptical
    power law (fp32) on three of them, against the oracle."""
    name = geom[0]
    say("case: random geometry %s" % name)
    spec = _random_spec(geom, False)
    for mname, m in (("fp32", 0), ("split", 1), ("split3", 3)):
        lid = ctx.load(spec, precision=m)
        _check(spec, ctx.loglike(lid, spec.proposals), spec.proposals, tol=MODE_TOL[m],
               label="%s/%s" % (name, mname), storage_floor=int(spec.mask.sum()) < 64, unit=UNIT[m])
        ctx.unload(lid)
    if RAND_GEOMS.index(geom) % 3 == 0:
        spec = _random_spec(geom, True)
        lid = ctx.load(spec, mass_model=1)
        _check(spec, ctx.loglike(lid, spec.proposals), spec.proposals, label="%s/epl" % name,
               storage_floor=int(spec.mask.sum()) < 64)
        ctx.unload(lid)
