"""Error conventions and request life cycle of the C ABI, on the device."""
import numpy as np
import pytest

from gpu_cases import oracle_data, say
from paper_2503_08586_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def b():
    from paper_2503_08586_amd import binding
    return binding


@pytest.fixture(scope="module")
def ctx(b):
    c = b.LensContext(0, max_inflight=4)
    yield c
    c.close()


def _spec(nprop=50):
    sp = synth.config1(nprop=nprop)[0]
    oracle_data(sp)
    return sp


def test_bad_descriptors(ctx, b):
    say("case: bad descriptors")
    sp = _spec(1)
    good = dict(ny=sp.ny, nx=sp.nx, dpix=sp.dpix, s=sp.s, psf=sp.psf, data=sp.data, sigma=sp.sigma, mask=sp.mask)
    bad = [
        dict(s=0), dict(s=9), dict(dpix=0.0), dict(dpix=-1.0), dict(dpix=float("nan")),
        dict(psf=np.ones((4, 4))), dict(sigma=np.where(sp.mask == 1, 0.0, 1.0)),
        dict(sigma=np.where(sp.mask == 1, np.nan, 1.0)), dict(data=np.where(sp.mask == 1, np.inf, 0.0)),
        dict(psf=np.full((3, 3), np.nan)),
    ]
    for kw in bad:
        a = dict(good)
        a.update(kw)
        with pytest.raises(b.LensError) as ei:
            ctx.load_raw(a["ny"], a["nx"], a["dpix"], a["s"], a["psf"], a["data"], a["sigma"], a["mask"])
        assert ei.value.status == b.LENS_EINVAL, kw
    with pytest.raises(b.LensError) as ei:
        ctx.load_raw(sp.ny, sp.nx, sp.dpix, sp.s, sp.psf, sp.data, sp.sigma, sp.mask, precision=7)
    assert ei.value.status == b.LENS_EINVAL
    # dimensions past 4096, and an image too wide for the LDS line buffer at its PSF size
    z = np.zeros((2, 4097))
    with pytest.raises(b.LensError) as ei:
        ctx.load_raw(2, 4097, 0.05, 1, np.ones((1, 1)), z, z + 1.0, np.ones((2, 4097), np.uint8))
    assert ei.value.status == b.LENS_EINVAL
    wide = np.zeros((70, 4096))
    psf63 = np.zeros((63, 63))
    psf63[31, 31] = 1.0
    psf63[0, 0] = psf63[62, 62] = 0.25       # keeps the 63x63 footprint through the tail crop
    with pytest.raises(b.LensError) as ei:
        ctx.load_raw(70, 4096, 0.05, 1, psf63, wide, wide + 1.0, np.ones((70, 4096), np.uint8))
    assert ei.value.status == b.LENS_EINVAL
    # sigma and data may be anything outside the mask
    lid = ctx.load_raw(sp.ny, sp.nx, sp.dpix, sp.s, sp.psf, np.where(sp.mask == 1, sp.data, np.nan),
                       np.where(sp.mask == 1, sp.sigma, 0.0), sp.mask)
    assert np.array_equal(ctx.loglike(lid, sp.proposals), ctx.loglike(lid, sp.proposals))
    ctx.unload(lid)


def test_unknown_ids(ctx, b):
    say("case: unknown lens and request ids")
    for fn in (lambda: ctx.loglike(987654, np.zeros((1, 20))), lambda: ctx.unload(987654),
               lambda: ctx.info(987654), lambda: ctx.submit(987654, np.zeros((1, 20)))):
        with pytest.raises(b.LensError) as ei:
            fn()
        assert ei.value.status == b.LENS_ENOENT
    fake = b.Request(ctx.ctx, 123456789, np.zeros(1))
    with pytest.raises(b.LensError):
        ctx.poll(fake)


def test_info_and_norm(ctx):
    say("case: lens info")
    sp = _spec(1)
    lid = ctx.load(sp)
    info = ctx.info(lid)
    assert info["masked_pixels"] == int(sp.mask.sum())
    C = -0.5 * np.sum(np.log(2 * np.pi * sp.sigma[sp.mask == 1] ** 2))
    assert abs(info["norm"] - C) < 1e-9 * abs(C)
    assert info["needed_pixels"] >= info["masked_pixels"]
    assert info["threads"] in (256, 512) and 1 <= info["strip_rows"] <= 32
    assert 0 < info["lds_bytes"] <= 160 * 1024 and info["blocks_per_cu"] >= 1
    say("tile: %d rows x %d threads, %d B LDS, %d workgroups/CU" % (
        info["strip_rows"], info["threads"], info["lds_bytes"], info["blocks_per_cu"]))
    ctx.unload(lid)


def _slow_spec():
    """200x200 px, s = 4, 41x41 PSF: ~30 ms per 16,384 proposals, so requests stay in flight."""
    sp = synth.config4(nlens=1, nprop=16384)[0]
    oracle_data(sp)
    return sp


def test_request_life_cycle(ctx, b):
    say("case: submit / poll / wait / cancel")
    sp = _spec(3000)
    lid = ctx.load(sp)
    ref = ctx.loglike(lid, sp.proposals)
    r = ctx.submit(lid, sp.proposals)
    assert ctx.wait(r) == b.LENS_OK
    assert np.array_equal(r.out, ref)
    with pytest.raises(b.LensError) as ei:       # the id is forgotten after its final answer
        ctx.poll(r)
    assert ei.value.status == b.LENS_ENOENT
    r2 = ctx.submit(lid, sp.proposals[:100])
    while ctx.poll(r2) == b.LENS_PENDING:
        pass
    assert np.array_equal(r2.out, ref[:100])
    r0 = ctx.submit(lid, np.zeros((0, 20)))      # zero-proposal request
    assert ctx.wait(r0) == b.LENS_OK
    ctx.unload(lid)
    # a slow lens keeps requests in flight: unload is refused, the last queued
    # request can be cancelled before it runs and its output is never written
    slow = _slow_spec()
    sl = ctx.load(slow)
    reqs = [ctx.submit(sl, slow.proposals) for _ in range(6)]
    with pytest.raises(b.LensError) as ei:
        ctx.unload(sl)
    assert ei.value.status == b.LENS_EBUSY
    reqs[-1].out[:] = 12345.0
    ctx.cancel(reqs[-1])
    for rq in reqs[:-1]:
        assert ctx.wait(rq) == b.LENS_OK
    assert np.all(reqs[-1].out == 12345.0)
    assert np.array_equal(reqs[0].out, reqs[1].out)
    st = ctx.stats()
    assert st["requests_canceled"] >= 1 and st["requests_done"] >= 7
    ctx.unload(sl)


def test_wait_timeout(ctx, b):
    say("case: wait timeout")
    sp = _spec(2000)
    lid = ctx.load(sp)
    big = np.tile(sp.proposals, (40, 1))
    r = ctx.submit(lid, big)
    st = ctx.wait(r, timeout_us=1)
    assert st in (b.LENS_ETIMEDOUT, b.LENS_OK)
    if st == b.LENS_ETIMEDOUT:
        assert ctx.wait(r) == b.LENS_OK
    ctx.unload(lid)


def test_hbm_budget(b):
    say("case: HBM budget")
    sp = _spec(10)
    with b.LensContext(0, hbm_budget_bytes=200_000) as c:
        with pytest.raises(b.LensError) as ei:
            for _ in range(10):
                c.load(sp)
        assert ei.value.status == b.LENS_ENOMEM
        assert c.stats()["hbm_used_bytes"] <= 200_000


def test_nonblocking_submit(b):
    say("case: non-blocking submit")
    slow = _slow_spec()
    with b.LensContext(0, max_inflight=1, nonblocking_submit=True) as c:
        lid = c.load(slow)
        reqs, again = [], 0
        for _ in range(12):
            try:
                reqs.append(c.submit(lid, slow.proposals[:8192]))
            except b.LensError as e:
                assert e.status == b.LENS_EAGAIN
                again += 1
            if reqs and again == 0:
                import time
                time.sleep(0.002)   # let the scheduler occupy the single slot
        for r in reqs:
            assert c.wait(r) == b.LENS_OK
        assert again > 0 and len(reqs) > 0
        c.unload(lid)


def test_model_image_rejects_bad_proposal(ctx, b):
    say("case: model image domain")
    sp = _spec(1)
    lid = ctx.load(sp)
    p = sp.truth.copy()
    p[synth.SLOT["q_m"]] = 1.5
    with pytest.raises(b.LensError) as ei:
        ctx.model_image(lid, p, 1)
    assert ei.value.status == b.LENS_EINVAL
    ctx.unload(lid)


def test_latency_statistics(b):
    """The context's request-latency window against the client's own clock:
    each request's latency (submit to result written) lies inside the client's
    submit-to-wait bracket, so every order statistic is bounded by the
    client's."""
    import time
    say("case: serving latency statistics")
    with b.LensContext(0, max_inflight=2) as c:
        sp = _spec(2000)
        lid = c.load(sp)
        st0 = c.stats()
        assert st0["latency_count"] == 0 and st0["latency_p50_us"] == 0.0 and st0["latency_max_us"] == 0.0
        walls = []
        for i in range(12):
            t0 = time.perf_counter()
            r = c.submit(lid, sp.proposals[:100 + 150 * i])
            assert c.wait(r) == b.LENS_OK
            walls.append((time.perf_counter() - t0) * 1e6)
        st = c.stats()
        walls.sort()
        assert st["latency_count"] == 12
        assert 0.0 < st["latency_p50_us"] <= st["latency_p99_us"] <= st["latency_max_us"]
        assert st["latency_p99_us"] == st["latency_max_us"]          # nearest rank of 12: the largest
        assert st["latency_p50_us"] <= walls[5] and st["latency_max_us"] <= walls[-1]
        # a reset starts a new interval: counters and the window empty, then only new requests
        c.reset_stats()
        st = c.stats()
        assert st["latency_count"] == 0 and st["requests_done"] == 0 and st["launches"] == 0
        assert st["latency_max_us"] == 0.0 and st["hbm_used_bytes"] > 0
        for n in (300, 900, 1500):
            assert c.wait(c.submit(lid, sp.proposals[:n])) == b.LENS_OK
        st = c.stats()
        assert st["latency_count"] == 3 and st["requests_done"] == 3 and st["proposals_done"] == 2700
        assert st["launches"] >= 3 and st["batch_pieces"] >= 3
        c.unload(lid)


def test_env_gated_log(tmp_path):
    """LENS_LOG=1 at lens_init: one stderr line per event, errors with their
    message; without it the library writes nothing."""
    import os
    import subprocess
    import sys
    say("case: LENS_LOG in a child process")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = "\n".join([
        "import numpy as np",
        "from paper_2503_08586_amd import binding, synth",
        "sp = synth.config1(nprop=8)[0]",
        "sp.make_data(lambda s, t: np.zeros((s.ny, s.nx)))",
        "with binding.LensContext(0) as c:",
        "    lid = c.load(sp)",
        "    c.loglike(lid, sp.proposals)",
        "    try:",
        "        c.unload(lid + 1000)",
        "    except binding.LensError:",
        "        pass",
        "    c.unload(lid)",
        "print('child done')",
    ])
    for log in ("1", "0"):
        env = dict(os.environ, LENS_LOG=log, PYTHONPATH=root)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=180,
                           cwd=root)
        assert r.returncode == 0 and "child done" in r.stdout, r.stderr[-2000:]
        lines = [x for x in r.stderr.splitlines() if x.startswith("[lens ")]
        if log == "1":
            text = "\n".join(lines)
            for want in ("init: device 0", "load lens", "error -3 (", "unknown lens id", "unload lens", "shutdown"):
                assert want in text, (want, text)
        else:
            assert lines == [], lines


def test_serving_every_lens_kind(ctx, b):
    """Serving with lenses of every kind at once (FP32, FP16-split and split3
    convolution, amplitudes solved for two light models, the power-law mass
    with explicit and solved amplitudes): each request's results equal the same
    proposals evaluated alone, bit for bit."""
    say("case: serving across lens kinds")
    specs = synth.config3(nlens=7, scale_props=0.0)
    kinds = [dict(), dict(precision=3), dict(amplitudes=1), dict(amplitudes=1, light_model=3, sersic_n=(1, 4, 1, 4)),
             dict(mass_model=1), dict(mass_model=1, amplitudes=1), dict(precision=1)]
    rng = np.random.default_rng(41)
    lids = []
    for sp, kw in zip(specs, kinds):
        oracle_data(sp)
        lids.append(ctx.load(sp, **kw))
    reqs = []
    for i in range(18):
        j = i % len(lids)
        P = synth.draw_params(rng, int(rng.integers(50, 3000)))
        if kinds[j].get("mass_model") == 1:
            P[:, 19] = rng.uniform(1.4, 2.6, len(P))
        reqs.append((j, P, ctx.submit(lids[j], P)))
    for j, P, r in reqs:
        assert ctx.wait(r) == b.LENS_OK
        assert np.array_equal(r.out, ctx.loglike(lids[j], P)), (j, kinds[j])
        assert np.isfinite(r.out).sum() > 0
    for lid in lids:
        ctx.unload(lid)


def test_concurrent_calls_from_threads(b):
    """Four threads on one context, each repeating a different kind of call
    (blocking batch, multi-lens graph, serving, sampler ensemble): every
    result equals the one computed alone beforehand."""
    import threading
    say("case: concurrent calls from four threads")
    with b.LensContext(0, max_inflight=4) as c:
        specs = synth.config3(nlens=3, scale_props=0.02)
        lids = []
        for sp in specs:
            oracle_data(sp)
            lids.append(c.load(sp))
        P = [sp.proposals for sp in specs]
        ref_single = [c.loglike(lid, p) for lid, p in zip(lids, P)]
        ref_multi = c.loglike_multi(lids, P)
        lo = np.array([x[1] for x in synth.PRIOR_BOX] + [0.0])
        hi = np.array([x[2] for x in synth.PRIOR_BOX] + [0.0])
        init = np.clip(specs[0].truth + 0.02 * (hi - lo) * np.random.default_rng(3).normal(size=(16, 20)), lo, hi)
        e_ref = c.ensemble(lids[0], init, lo, hi, seed=5)
        e_run = c.ensemble(lids[0], init, lo, hi, seed=5)
        errors = []
        reps = 12

        def guard(fn):
            def run():
                try:
                    fn()
                except Exception as ex:   # reported by the main thread
                    errors.append(ex)
            return run

        def blocking():
            for r in range(reps):
                j = r % 3
                assert np.array_equal(c.loglike(lids[j], P[j]), ref_single[j])

        def multi():
            for _ in range(reps):
                out = c.loglike_multi(lids, P)
                assert all(np.array_equal(o, x) for o, x in zip(out, ref_multi))

        def serving():
            for r in range(reps):
                j = r % 3
                q = c.submit(lids[j], P[j])
                assert c.wait(q) == b.LENS_OK and np.array_equal(q.out, ref_single[j])

        def sampler():
            for _ in range(reps):
                c.ensemble_run(e_run, 1)

        th = [threading.Thread(target=guard(f)) for f in (blocking, multi, serving, sampler)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert not errors, errors
        c.ensemble_run(e_ref, reps)
        a, r = c.ensemble_get(e_run), c.ensemble_get(e_ref)
        assert all(np.array_equal(x, y) for x, y in zip(a[:3], r[:3])) and a[3] == r[3] == reps
        for e in (e_ref, e_run):
            c.ensemble_destroy(e)
        for lid in lids:
            c.unload(lid)
