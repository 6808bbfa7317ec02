"""GPU parity of the device-resident sampler loop: the Philox4x32-10 stream bit
for bit against the oracle and the published known answers, and every
stretch-move half-step of a device run checked against the oracle's proposal,
lnL and acceptance rule (Goodman & Weare 2010; posterior of Sec. 2.2 under a
box prior)."""
import numpy as np
import pytest

from gpu_cases import TOL_FP32, oracle_data, say
from paper_2503_08586_amd import synth

pytestmark = pytest.mark.gpu

S = synth.SLOT


@pytest.fixture(scope="module")
def ctx():
    from paper_2503_08586_amd import binding
    c = binding.LensContext(0)
    yield c
    c.close()


def _box(fixed=()):
    lo = np.array([b[1] for b in synth.PRIOR_BOX] + [0.0])
    hi = np.array([b[2] for b in synth.PRIOR_BOX] + [0.0])
    for name, v in fixed:
        lo[S[name]] = hi[S[name]] = v
    return lo, hi


def _init(rng, W, lo, hi, around=None, scale=0.05):
    """W walkers inside the box: a small ball around ``around`` (or uniform)."""
    if around is None:
        return lo + (hi - lo) * rng.random((W, 20))
    w = around[None, :] + scale * (hi - lo)[None, :] * rng.normal(size=(W, 20))
    return np.clip(w, lo, hi)


def _C(spec):
    sel = spec.mask == 1
    return -0.5 * np.sum(np.log(2 * np.pi * spec.sigma[sel] ** 2))


def test_philox_matches_oracle_and_known_answers(ctx):
    import oracle
    import oracle_pins
    orc = oracle.default()
    for c, k, want in oracle_pins.philox_kat():
        got = ctx.philox(c, k, 1)[0]
        assert [int(v) for v in got] == want
    rng = np.random.default_rng(1)
    for base, key in (([0xFFFFFFF0, 7, 1, 0], [3, 9]), (list(rng.integers(0, 2 ** 32, 4)), list(rng.integers(0, 2 ** 32, 2)))):
        n = 3000
        got = ctx.philox(base, key, n)
        for i in range(0, n, 7):
            c = [(int(base[0]) + i) % 2 ** 32, base[1], base[2], base[3]]
            assert np.array_equal(got[i], orc.philox(c, key)), (base, i)


def _lnl_oracle(spec, P, nnls):
    import oracle
    orc = oracle.default()
    fn = orc.loglike_nnls if nnls else orc.loglike
    lnl, chi2 = fn(spec.geom, spec.psf, spec.data, spec.sigma, spec.mask, P, return_chi2=True)
    return lnl, chi2


def _check_iteration(spec, before, lnp_before, after, lnp_after, t, seed, a, lo, hi, nnls, stats):
    """One device iteration (half 0, then half 1) against the oracle."""
    import oracle
    orc = oracle.default()
    W = before.shape[0]
    h = W // 2
    d = int(np.count_nonzero(hi > lo))
    C = abs(_C(spec))
    state = before.copy()
    lnp = lnp_before.copy()
    for half in (0, 1):
        moving = slice(half * h, (half + 1) * h)
        Y, z, logu, j = orc.stretch_propose(state, half, t, seed, a)
        inside = np.array([orc.box_logprior(y, lo, hi) == 0.0 for y in Y])
        lnY = np.full(h, -np.inf)
        chi2Y = np.full(h, np.inf)
        if inside.any():
            lnY[inside], chi2Y[inside] = _lnl_oracle(spec, Y[inside], nnls)
        new, new_lnp = after[moving], lnp_after[moving]
        moved = np.any(new != state[moving], axis=1)
        for i in range(h):
            k = half * h + i
            # the oracle's decision and its margin, taken with the device's lnP
            # of the current walker; the lnL gate bounds how far the device's
            # lnL of the proposal may be from the oracle's
            band = TOL_FP32 * ((0.5 * chi2Y[i] if np.isfinite(chi2Y[i]) else 0.0) + C) + 1e-12 * (abs(lnp[k]) + C)
            margin = (d - 1) * np.log(z[i]) + lnY[i] - lnp[k] - logu[i]
            if moved[i]:
                stats["acc"] += 1
                assert inside[i], (t, half, k)
                assert np.allclose(new[i], Y[i], rtol=1e-13, atol=1e-15), (t, half, k, new[i] - Y[i])
                assert abs(new_lnp[i] - lnY[i]) <= TOL_FP32 * (0.5 * chi2Y[i] + C), (t, half, k)
                assert margin > -band, (t, half, k, margin, band)
                # the device's own rule, in FP64 from its own lnP values
                assert logu[i] < (d - 1) * np.log(z[i]) + new_lnp[i] - lnp[k] + 1e-9 * C
            else:
                stats["rej"] += 1
                assert np.array_equal(new[i], state[k]) and new_lnp[i] == lnp[k], (t, half, k)
                assert not inside[i] or margin < band, (t, half, k, margin, band)
        state[moving] = new
        lnp[moving] = new_lnp
    # the half that did not move kept its walkers: the state is exactly the device's
    assert np.array_equal(state, after) and np.array_equal(lnp, lnp_after)


@pytest.mark.parametrize("nnls", [False, True])
def test_ensemble_iterations_match_oracle(ctx, nnls):
    say("case: stretch-move ensemble, 64x64 s=1 k=11 lens, W=48, 6 iterations, nnls=%s" % nnls)
    spec = synth.config1(nprop=1)[0]
    oracle_data(spec)
    fixed = [("I_l", 0.0), ("I_s", 0.0)] if nnls else []
    lo, hi = _box(fixed)
    rng = np.random.default_rng(2 + nnls)
    init = _init(rng, 48, lo, hi, around=np.clip(spec.truth, lo, hi), scale=0.02)
    lid = ctx.load(spec, amplitudes=1 if nnls else 0)
    seed, a = 1234567 + nnls, 2.0
    ens = ctx.ensemble(lid, init, lo, hi, stretch=a, seed=seed)
    w0, lnp0, acc0, it0 = ctx.ensemble_get(ens)
    assert it0 == 0 and np.array_equal(w0, init) and np.all(acc0 == 0)
    ref0, chi0 = _lnl_oracle(spec, init, nnls)
    assert np.all(np.abs(lnp0 - ref0) <= TOL_FP32 * (0.5 * chi0 + abs(_C(spec))))
    T = 6
    chain, chain_lnp = ctx.ensemble_run(ens, T, thin=1, chain=True)
    stats = {"acc": 0, "rej": 0}
    before, lb = init, lnp0
    for t in range(T):
        _check_iteration(spec, before, lb, chain[t], chain_lnp[t], t, seed, a, lo, hi, nnls, stats)
        before, lb = chain[t], chain_lnp[t]
    w1, lnp1, acc1, it1 = ctx.ensemble_get(ens)
    assert it1 == T and np.array_equal(w1, chain[-1]) and np.array_equal(lnp1, chain_lnp[-1])
    assert acc1.sum() == stats["acc"]
    say("accepted %d, rejected %d" % (stats["acc"], stats["rej"]))
    assert stats["acc"] > 10 and stats["rej"] > 10
    ctx.ensemble_destroy(ens)
    ctx.unload(lid)


def test_ensemble_split_runs_equal_one_run(ctx):
    spec = synth.config1(nprop=1)[0]
    oracle_data(spec)
    lo, hi = _box()
    init = _init(np.random.default_rng(4), 64, lo, hi, around=np.clip(spec.truth, lo, hi), scale=0.03)
    lid = ctx.load(spec)
    e1 = ctx.ensemble(lid, init, lo, hi, seed=99)
    e2 = ctx.ensemble(lid, init, lo, hi, seed=99)
    c1, l1 = ctx.ensemble_run(e1, 9, thin=3, chain=True)
    ctx.ensemble_run(e2, 3)
    c2, l2 = ctx.ensemble_run(e2, 6, thin=3, chain=True)
    a, b = ctx.ensemble_get(e1), ctx.ensemble_get(e2)
    assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3])) and a[3] == b[3] == 9
    assert np.array_equal(c1[1:], c2) and np.array_equal(l1[1:], l2)
    # another seed gives another run
    e3 = ctx.ensemble(lid, init, lo, hi, seed=100)
    ctx.ensemble_run(e3, 9)
    assert not np.array_equal(ctx.ensemble_get(e3)[0], a[0])
    for e in (e1, e2, e3):
        ctx.ensemble_destroy(e)
    ctx.unload(lid)


def test_ensemble_box_and_fixed_slots(ctx):
    spec = synth.config1(nprop=1)[0]
    oracle_data(spec)
    lo, hi = _box([("g1", 0.01), ("g2", -0.02)])
    lo[S["x_s"]], hi[S["x_s"]] = -0.2, 0.2       # a tight box that proposals leave often
    init = _init(np.random.default_rng(6), 32, lo, hi)
    lid = ctx.load(spec)
    ens = ctx.ensemble(lid, init, lo, hi, seed=5, stretch=3.0)
    chain, _ = ctx.ensemble_run(ens, 20, thin=1, chain=True)
    assert np.all((chain >= lo) & (chain <= hi))
    assert np.all(chain[..., S["g1"]] == 0.01) and np.all(chain[..., S["g2"]] == -0.02)
    assert np.all(chain[..., 19] == 0.0)
    ctx.ensemble_destroy(ens)
    ctx.unload(lid)


def test_ensemble_errors(ctx):
    from paper_2503_08586_amd import binding
    spec = synth.config1(nprop=1)[0]
    oracle_data(spec)
    lid = ctx.load(spec)
    lo, hi = _box()
    good = _init(np.random.default_rng(7), 8, lo, hi)

    def einval(**kw):
        args = dict(init=good, lo=lo, hi=hi, stretch=2.0, seed=0)
        args.update(kw)
        with pytest.raises(binding.LensError) as ei:
            ctx.ensemble(lid, **args)
        assert ei.value.status == binding.LENS_EINVAL, kw
    einval(init=good[:7])                       # odd walker count
    einval(init=good[:2])                       # too few
    einval(stretch=1.0)
    einval(stretch=np.nan)
    bad = good.copy()
    bad[3, S["q_m"]] = 1.5                      # outside the box
    einval(init=bad)
    lo2, hi2 = lo.copy(), hi.copy()
    lo2[S["n_l"]] = 0.05                        # inside this box, outside the model's domain
    bad = good.copy()
    bad[2, S["n_l"]] = 0.05
    einval(init=bad, lo=lo2, hi=hi2)
    einval(lo=hi, hi=lo)                        # lo > hi
    ens = ctx.ensemble(lid, good, lo, hi)
    with pytest.raises(binding.LensError) as ei:
        ctx.unload(lid)
    assert ei.value.status == binding.LENS_EBUSY
    ctx.ensemble_destroy(ens)
    with pytest.raises(binding.LensError) as ei:
        ctx.ensemble_destroy(ens)
    assert ei.value.status == binding.LENS_ENOENT
    ctx.unload(lid)


def _many_cases():
    """Lenses of several kinds and sizes, each with an ensemble size and a
    box: (label, spec, load kwargs, W, lo, hi)."""
    out = []
    lo, hi = _box()
    s1 = synth.config1(nprop=1)[0]
    oracle_data(s1)
    out.append(("c1 sie", s1, {}, 32, lo, hi))
    out.append(("c1 sie W=4", s1, {}, 4, lo, hi))
    lo_n, hi_n = _box([("I_l", 0.0), ("I_s", 0.0)])
    out.append(("c1 nnls", s1, {"amplitudes": 1}, 48, lo_n, hi_n))
    se = synth.config1(nprop=1)[0]
    se.truth = se.truth.copy()
    se.truth[19] = 2.2
    oracle_data(se)
    lo_e, hi_e = lo.copy(), hi.copy()
    lo_e[19], hi_e[19] = 1.5, 2.5
    out.append(("c1 epl", se, {"mass_model": 1}, 20, lo_e, hi_e))
    for i, spec in enumerate(synth.config3(nlens=3, scale_props=0.0)):
        oracle_data(spec)
        out.append(("c3 lens %d (%dpx s=%d k=%d)" % (i, spec.ny, spec.s, spec.psf.shape[0]), spec,
                    {"precision": 3} if i == 1 else {}, 64 + 32 * i, lo, hi))
    return out


def test_ensemble_run_many_equals_separate_runs(ctx):
    """Pooled half-steps over many ensembles move each exactly as its own run,
    bit for bit, from its own iteration count; one pooled iteration of a
    member is checked against the oracle directly."""
    cases = _many_cases()
    say("case: %d ensembles on %d lenses, pooled vs separate runs" % (len(cases), len(cases)))
    rng = np.random.default_rng(11)
    lids, pooled, single = [], [], []
    for n, (label, spec, kw, W, lo, hi) in enumerate(cases):
        lid = ctx.load(spec, **kw)
        lids.append(lid)
        around = np.clip(spec.truth, lo, hi)
        init = _init(rng, W, lo, hi, around=around, scale=0.02)
        pooled.append(ctx.ensemble(lid, init, lo, hi, seed=500 + n))
        single.append(ctx.ensemble(lid, init, lo, hi, seed=500 + n))
    # members start from different iteration counts
    ctx.ensemble_run(pooled[2], 2)
    ctx.ensemble_run(single[2], 2)
    for calls in (1, 3, 2):
        ctx.ensemble_run_many(pooled, calls)
        for e in single:
            ctx.ensemble_run(e, calls)
        for (label, *_), p, s in zip(cases, pooled, single):
            a, b = ctx.ensemble_get(p), ctx.ensemble_get(s)
            assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3])) and a[3] == b[3], label
    assert sum(int(ctx.ensemble_get(p)[2].sum()) for p in pooled) > 50
    # chains: every second iteration of a 4-iteration call, per ensemble
    pc = ctx.ensemble_run_many(pooled, 4, thin=2, chain=True)
    for (label, *_), (cw, cl), s_ in zip(cases, pc, single):
        sw, sl = ctx.ensemble_run(s_, 4, thin=2, chain=True)
        assert cw.shape == sw.shape and np.array_equal(cw, sw) and np.array_equal(cl, sl), label
    # one pooled iteration of the first member against the oracle
    label, spec, kw, W, lo, hi = cases[0]
    before, lb, _, t = ctx.ensemble_get(pooled[0])
    ctx.ensemble_run_many(pooled, 1)
    after, la, _, _ = ctx.ensemble_get(pooled[0])
    stats = {"acc": 0, "rej": 0}
    _check_iteration(spec, before, lb, after, la, t, 500, 2.0, lo, hi, False, stats)
    for e in pooled + single:
        ctx.ensemble_destroy(e)
    for lid in lids:
        ctx.unload(lid)


def test_ensemble_run_many_errors(ctx):
    from paper_2503_08586_amd import binding
    spec = synth.config1(nprop=1)[0]
    oracle_data(spec)
    lid = ctx.load(spec)
    lo, hi = _box()
    init = _init(np.random.default_rng(8), 8, lo, hi, around=np.clip(spec.truth, lo, hi), scale=0.02)
    e1 = ctx.ensemble(lid, init, lo, hi, seed=1)
    e2 = ctx.ensemble(lid, init, lo, hi, seed=2)
    ctx.ensemble_run_many([], 5)
    ctx.ensemble_run_many([e1, e2], 0)
    for ids, status in (([e1, e1], binding.LENS_EINVAL), ([e1, e2 + 1000], binding.LENS_ENOENT)):
        with pytest.raises(binding.LensError) as ei:
            ctx.ensemble_run_many(ids, 1)
        assert ei.value.status == status, ids
    with pytest.raises(binding.LensError) as ei:
        ctx.ensemble_run_many([e1], -1)
    assert ei.value.status == binding.LENS_EINVAL
    # a chain with thin < 1
    import ctypes
    dp = ctypes.POINTER(ctypes.c_double)
    buf = np.empty((2, 8, 20))
    arr = (dp * 1)(buf.ctypes.data_as(dp))
    ids = np.array([e1], dtype=np.int64)
    st = binding.load().lens_ensemble_run_many(ctx.ctx, 1, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 2, 0,
                                                arr, None)
    assert st == binding.LENS_EINVAL
    # nothing moved
    assert ctx.ensemble_get(e1)[3] == 0 and np.array_equal(ctx.ensemble_get(e1)[0], init)
    ctx.ensemble_run_many([e2, e1], 2)
    assert ctx.ensemble_get(e1)[3] == 2 and ctx.ensemble_get(e2)[3] == 2
    for e in (e1, e2):
        ctx.ensemble_destroy(e)
    ctx.unload(lid)


def test_ensemble_concurrent_with_multi_plan_builds(ctx):
    """A multi-lens call shape is captured into a graph the first time it is
    seen; the capture uses a stream of its own, so an ensemble advancing on
    another thread meanwhile is neither captured nor disturbed."""
    import threading
    say("case: ensemble run on one thread while multi-lens plans are captured on another")
    specs = synth.config3(nlens=4, scale_props=0.01)
    lids = []
    for sp in specs:
        oracle_data(sp)
        lids.append(ctx.load(sp))
    singles = [ctx.loglike(lid, sp.proposals) for sp, lid in zip(specs, lids)]
    s1 = synth.config1(nprop=1)[0]
    oracle_data(s1)
    lo, hi = _box()
    init = _init(np.random.default_rng(21), 32, lo, hi, around=np.clip(s1.truth, lo, hi), scale=0.02)
    lid1 = ctx.load(s1)
    e_conc = ctx.ensemble(lid1, init, lo, hi, seed=77)
    e_ref = ctx.ensemble(lid1, init, lo, hi, seed=77)
    errors = []

    def sampler():
        try:
            for _ in range(30):
                ctx.ensemble_run(e_conc, 1)
        except Exception as ex:   # reported by the main thread
            errors.append(ex)

    th = threading.Thread(target=sampler)
    th.start()
    try:
        # new call shapes (other counts each time) build and capture new plans
        for m in range(1, 9):
            outs = ctx.loglike_multi(lids, [sp.proposals[:m + j] for j, sp in enumerate(specs)])
            for j, (o, ref) in enumerate(zip(outs, singles)):
                assert np.array_equal(o, ref[:m + j]), (m, j)
    finally:
        th.join()
    assert not errors, errors
    ctx.ensemble_run(e_ref, 30)
    a, b = ctx.ensemble_get(e_conc), ctx.ensemble_get(e_ref)
    assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3])) and a[3] == b[3] == 30
    for e in (e_conc, e_ref):
        ctx.ensemble_destroy(e)
    for lid in lids + [lid1]:
        ctx.unload(lid)


def test_device_sampler_settles_in_the_posterior(ctx):
    """End to end: 600 iterations of a 48-walker ensemble from a ball around
    the truth on the 64x64 lens.  The walkers' lnP settles within a few
    posterior units of lnL at the truth (samples of a d-dimensional posterior
    sit about d/2 below its maximum, here d = 19), never worse than the start;
    the Einstein radius stays at its true value; a sane acceptance rate."""
    say("case: device sampler, 600 iterations, 48 walkers, 64x64 lens")
    spec = synth.config1(nprop=1)[0]
    oracle_data(spec)
    lo, hi = _box()
    init = _init(np.random.default_rng(31), 48, lo, hi, around=np.clip(spec.truth, lo, hi), scale=0.01)
    lid = ctx.load(spec)
    truth_lnl = ctx.loglike(lid, spec.truth[None, :])[0]
    ens = ctx.ensemble(lid, init, lo, hi, seed=2026)
    lnp0 = ctx.ensemble_get(ens)[1]
    chain, chain_lnp = ctx.ensemble_run(ens, 600, thin=10, chain=True)
    w, lnp, acc, it = ctx.ensemble_get(ens)
    tail = chain_lnp[-20:].ravel()
    d = int(np.count_nonzero(hi > lo))
    say("lnL(truth) %.2f, median lnP start %.2f, last 200 iterations %.2f (d = %d), acceptance %.3f" %
        (truth_lnl, np.median(lnp0), np.median(tail), d, acc.sum() / (48 * it)))
    assert it == 600 and 0.05 < acc.sum() / (48 * it) < 0.8
    assert np.median(tail) >= np.median(lnp0) - 1.0
    assert truth_lnl - np.median(tail) < d / 2 + 6 * np.sqrt(d / 2)
    te = chain[-20:, :, S["theta_E"]].ravel()
    assert abs(np.median(te) - spec.truth[S["theta_E"]]) < 0.02
    ctx.ensemble_destroy(ens)
    ctx.unload(lid)
