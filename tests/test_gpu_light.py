"""GPU parity of the light models with solved amplitudes (Sec. 2.3, the set-ups
of Sec. 3.1.2 and 3.2): lens and source, lens light only, lensed source only,
and two components per galaxy with fixed indices, each against the oracle's
support-enumeration NNLS over the same columns."""
import numpy as np
import pytest

from gpu_cases import TOL_FP32, oracle_data, rel_err, say
from paper_2503_08586_amd import synth

pytestmark = pytest.mark.gpu

NNLS = 1
NFIX = synth.DOUBLE_SERSIC_N
N_AMP = {0: 2, 1: 1, 2: 1, 3: 4}
S = synth.SLOT


@pytest.fixture(scope="module")
def ctx():
    from paper_2503_08586_amd import binding
    c = binding.LensContext(0)
    yield c
    c.close()


def _C(spec):
    sel = spec.mask == 1
    return -0.5 * np.sum(np.log(2 * np.pi * spec.sigma[sel] ** 2))


def _props(spec, model, n=None):
    P = spec.proposals if n is None else spec.proposals[:n]
    if model == 3:
        P = synth.double_component_params(np.random.default_rng(7), P)
    return P


def _oracle(spec, P, model):
    import oracle
    return oracle.default().loglike_light(spec.geom, spec.psf, spec.data, spec.sigma, spec.mask, P, model,
                                          nfix=NFIX, return_chi2=True, return_amps=True)


def _columns(spec, p, model):
    """Unit-amplitude columns of a light model, rendered one component at a
    time through the oracle's one-component model image."""
    import oracle
    orc = oracle.default()

    def img(**kw):
        q = p.copy()
        for k, v in kw.items():
            q[S[k]] = v
        return orc.model_image(spec.ny, spec.nx, spec.dpix, spec.s, spec.psf, q, stage=1)
    lens0 = dict(I_l=1.0, I_s=0.0)
    src0 = dict(I_l=0.0, I_s=1.0)
    if model == 0:
        return [img(**lens0), img(**src0)]
    if model == 1:
        return [img(theta_E=0.0, g1=0.0, g2=0.0, **lens0)]
    if model == 2:
        return [img(**src0)]
    return [img(n_l=NFIX[0], n_s=1.0, **lens0), img(R_l=p[S["n_l"]], n_l=NFIX[1], n_s=1.0, **lens0),
            img(n_s=NFIX[2], n_l=1.0, **src0), img(R_s=p[S["n_s"]], n_s=NFIX[3], n_l=1.0, **src0)]


def _check(spec, lid, ctx, P, model, label, n_amp):
    got, amp = ctx.loglike_amps(lid, P)
    assert amp.shape == (len(P), N_AMP[model])
    ref, chi2, ramp = _oracle(spec, P, model)
    assert np.array_equal(np.isneginf(got), np.isneginf(ref)), label
    e = rel_err(got, ref, chi2, C=_C(spec))
    say("%s: n=%d max lnL err %.3e" % (label, len(got), e.max()))
    assert np.all(e <= TOL_FP32), (label, e.max(), int(np.argmax(e)))
    # amplitudes in the metric of the normal matrix: the chi^2 excess of the
    # device amplitudes over the optimum stays within the lnL gate
    sel = spec.mask == 1
    w = 1.0 / spec.sigma[sel] ** 2
    worst = 0.0
    idx = [i for i in range(len(P)) if np.isfinite(ref[i])][:n_amp]
    for i in idx:
        A = np.stack([c[sel] for c in _columns(spec, P[i], model)], axis=1)
        F = A.T @ (w[:, None] * A)
        ds = amp[i] - ramp[i]
        worst = max(worst, float(ds @ F @ ds) / (0.5 * chi2[i] + abs(_C(spec))))
        assert np.all(amp[i] >= 0.0)
    say("%s: max amplitude chi2 excess %.3e over %d proposals" % (label, worst, len(idx)))
    assert worst <= TOL_FP32
    return got, amp


@pytest.mark.parametrize("model", [0, 1, 2, 3])
def test_light_model_small(ctx, model):
    say("case: light model %d, 64x64 s=1 k=11, 200 proposals" % model)
    spec = synth.config1(nprop=200)[0]
    oracle_data(spec)
    lid = ctx.load(spec, amplitudes=NNLS, light_model=model, sersic_n=NFIX)
    info = ctx.info(lid)
    assert info["light_model"] == model and info["n_amplitudes"] == N_AMP[model]
    _check(spec, lid, ctx, _props(spec, model), model, "light %d c1" % model, n_amp=12)
    ctx.unload(lid)


@pytest.mark.parametrize("model", [1, 2, 3])
def test_light_model_survey_sampled(ctx, model):
    say("case: light model %d, 128x128 s=4, 21x21 PSF, 12 proposals" % model)
    spec = synth.config2(nprop=12)[0]
    oracle_data(spec)
    lid = ctx.load(spec, amplitudes=NNLS, light_model=model, sersic_n=NFIX)
    _check(spec, lid, ctx, _props(spec, model), model, "light %d c2" % model, n_amp=3)
    ctx.unload(lid)


def test_light_model0_equals_two_channel_nnls(ctx):
    spec = synth.config1(nprop=64)[0]
    oracle_data(spec)
    a = ctx.load(spec, amplitudes=NNLS)
    b = ctx.load(spec, amplitudes=NNLS, light_model=0)
    ga, aa = ctx.loglike_amps(a, spec.proposals)
    gb, ab = ctx.loglike_amps(b, spec.proposals)
    assert np.array_equal(ga, gb) and np.array_equal(aa, ab)
    ctx.unload(a)
    ctx.unload(b)


def test_double_recovers_four_amplitudes(ctx):
    say("case: two components per galaxy on noise-free data")
    spec = synth.config1(nprop=1)[0]
    p = _props(spec, 3, 1)[0]
    p[S["theta_E"]] = 1.2
    cols = _columns(spec, p, 3)
    truth = np.array([0.3, 0.12, 0.25, 0.08])
    spec.data = sum(a * c for a, c in zip(truth, cols))
    lid = ctx.load(spec, amplitudes=NNLS, light_model=3, sersic_n=NFIX)
    got, amp = ctx.loglike_amps(lid, p[None])
    say("recovered %s vs %s" % (amp[0], truth))
    assert np.allclose(amp[0], truth, rtol=1e-4, atol=0)
    ctx.unload(lid)


def test_light_models_ignore_unused_slots(ctx):
    spec = synth.config1(nprop=8)[0]
    oracle_data(spec)
    P = spec.proposals
    l1 = ctx.load(spec, amplitudes=NNLS, light_model=1)
    l2 = ctx.load(spec, amplitudes=NNLS, light_model=2)
    base1 = ctx.loglike(l1, P)
    Q = P.copy()
    Q[:, S["theta_E"]] = -3.0
    Q[:, S["q_m"]] = 0.0
    Q[:, S["g1"]] = np.nan
    Q[:, S["R_s"]] = -1.0
    Q[:, S["I_l"]] = np.inf
    assert np.array_equal(ctx.loglike(l1, Q), base1)
    base2 = ctx.loglike(l2, P)
    Q = P.copy()
    Q[:, S["R_l"]] = -1.0
    Q[:, S["n_l"]] = 99.0
    Q[:, S["phi_l"]] = np.nan
    assert np.array_equal(ctx.loglike(l2, Q), base2)
    Q = P.copy()
    Q[:, S["theta_E"]] = 0.0
    assert not np.array_equal(ctx.loglike(l2, Q), base2)
    # the slots a model does read are checked
    Q = P.copy()
    Q[0, S["R_l"]] = 0.0
    Q[1, S["q_s"]] = 1.5
    assert ctx.loglike(l1, Q)[0] == -np.inf and np.isfinite(ctx.loglike(l1, Q)[1])
    assert ctx.loglike(l2, Q)[1] == -np.inf and np.isfinite(ctx.loglike(l2, Q)[0])
    ctx.unload(l1)
    ctx.unload(l2)


def test_light_model_load_rules(ctx):
    from paper_2503_08586_amd import binding
    spec = synth.config1(nprop=1)[0]
    oracle_data(spec)
    for kw in (dict(light_model=1),                                    # needs NNLS
               dict(amplitudes=NNLS, light_model=4),
               dict(amplitudes=NNLS, light_model=3, sersic_n=(1.0, 4.0, 1.0, 25.0)),
               dict(amplitudes=NNLS, light_model=3, sersic_n=(0.0, 4.0, 1.0, 4.0))):
        with pytest.raises(binding.LensError) as ei:
            ctx.load(spec, **kw)
        assert ei.value.status == binding.LENS_EINVAL, kw


def test_mixed_light_models_in_multi_call(ctx):
    say("case: lenses of every light model in one multi-lens call")
    specs = synth.config3(nlens=6, scale_props=0.03)
    models = [0, 1, 2, 3, 3, 1]
    lids, props = [], []
    for sp, m in zip(specs, models):
        oracle_data(sp)
        lids.append(ctx.load(sp, amplitudes=NNLS, light_model=m, sersic_n=NFIX))
        props.append(_props(sp, m))
    outs = ctx.loglike_multi(lids, props)
    for lid, P, o in zip(lids, props, outs):
        assert np.array_equal(o, ctx.loglike(lid, P))
    for j in (1, 3):
        sp, P = specs[j], props[j][:8]
        ref, chi2, _ = _oracle(sp, P, models[j])
        e = rel_err(outs[j][:8], ref, chi2, C=_C(sp))
        say("multi light %d: max %.3e" % (models[j], e.max()))
        assert np.all(e <= TOL_FP32)
    for lid in lids:
        ctx.unload(lid)


def _random_light_cases(seed=3582):
    """Seeded geometries for the solved-amplitude kernels: supersampling 1-8,
    odd PSF sides up to 63, sizes 12-60 px, masks of at least 64 pixels;
    each with one light model, one of them with the power-law mass."""
    rng = np.random.default_rng(seed)
    out = []
    for i, (s, model) in enumerate(((7, 0), (3, 1), (8, 2), (5, 3), (2, 0), (6, 3))):
        ny, nx = int(rng.integers(12, 61)), int(rng.integers(12, 61))
        k = int(rng.choice(np.arange(1, 64, 2)))
        dpix = float(rng.uniform(0.04, 0.1))
        out.append(("rl%d_%dx%d_s%d_k%d_m%d" % (i, ny, nx, s, k, model), ny, nx, dpix, s, k, model, i == 4))
    return out


RAND_LIGHT = _random_light_cases()


@pytest.mark.parametrize("case", RAND_LIGHT, ids=[c[0] for c in RAND_LIGHT])
def test_light_models_random_geometries(ctx, case):
    from gpu_cases import custom_spec
    name, ny, nx, dpix, s, k, model, epl = case
    say("case: %s%s" % (name, " (power-law mass)" if epl else ""))
    rng = np.random.default_rng(sum(map(ord, name)))
    psf = synth.gaussian_psf(k, 3.0 * dpix, dpix) if k > 1 else np.ones((1, 1))
    psf = psf * (1.0 + 0.3 * rng.random(psf.shape))
    mask = synth.circular_mask(ny, nx, dpix, 0.45 * min(ny, nx) * dpix)
    if mask.sum() < 64:
        mask = np.ones((ny, nx), np.uint8)
    spec = custom_spec(29 + model, ny, nx, dpix, s, psf, mask, 16)
    P = _props(spec, model)
    if epl:
        P = np.array(P, copy=True)
        P[:, 19] = rng.uniform(1.3, 2.7, len(P))
    lid = ctx.load(spec, amplitudes=NNLS, light_model=model, sersic_n=NFIX, mass_model=1 if epl else 0)
    _check(spec, lid, ctx, P, model, name, n_amp=4)
    ctx.unload(lid)
