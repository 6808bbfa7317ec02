"""Device-buffer entry points through the C ABI: the multi-lens call on device
buffers against the host-buffer multi-lens call and the oracle, and calls from
several threads sharing one stream (and so one scratch buffer)."""
import threading

import numpy as np
import pytest

from gpu_cases import TOL_FP32, oracle_data, oracle_loglike, rel_err, say
from paper_2503_08586_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2503_08586_amd import binding
    c = binding.LensContext(0)
    yield c
    c.close()


def _lenses(ctx, n=9):
    """A mix of lens kinds: FP32, split3 and NNLS-solved amplitudes."""
    specs = synth.config3(nlens=n, scale_props=0.03)
    lids = []
    for i, sp in enumerate(specs):
        oracle_data(sp)
        kind = i % 3
        lids.append(ctx.load(sp, precision=3 if kind == 1 else 0, amplitudes=1 if kind == 2 else 0))
    return specs, lids


def test_multi_device_equals_multi(ctx):
    import torch
    say("case: multi-lens call on device buffers, 9 lenses of three kinds")
    specs, lids = _lenses(ctx)
    plist = [sp.proposals for sp in specs]
    ref = ctx.loglike_multi(lids, plist)
    dev = torch.device("cuda", 0)
    st = torch.cuda.Stream()
    for rep, sel in enumerate([list(range(9)), [4, 1, 7], list(range(9))]):
        counts = [plist[j].shape[0] - (rep % 2) for j in sel]
        P = np.concatenate([plist[j][:c] for j, c in zip(sel, counts)])
        pd = torch.from_numpy(P).to(dev)
        od = torch.full((P.shape[0],), np.nan, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        ctx.loglike_multi_device([lids[j] for j in sel], counts, pd, od, st)
        st.synchronize()
        got = np.split(od.cpu().numpy(), np.cumsum(counts)[:-1])
        for j, c, g in zip(sel, counts, got):
            assert np.array_equal(g, ref[j][:c]), (rep, j)
    # the FP32 and split3 lenses against the oracle (the solved ones have their own tests)
    for j in (0, 1):
        r, chi2, C = oracle_loglike(specs[j], specs[j].proposals[:6])
        e = rel_err(ref[j][:6], r, chi2, C)
        say("lens %d: max err %.3e" % (j, e.max()))
        assert e.max() <= TOL_FP32
    for lid in lids:
        ctx.unload(lid)


def test_threads_share_one_stream(ctx):
    """Two threads enqueue device-buffer calls of different sizes on the same
    stream, over and over: each result equals its solo run bit for bit (the
    stream's scratch is held by one call from take to last launch)."""
    import torch
    say("case: two threads, one stream, single- and multi-lens device calls")
    specs, lids = _lenses(ctx, 6)
    dev = torch.device("cuda", 0)
    st = torch.cuda.Stream()
    big = synth.draw_params(np.random.default_rng(1), 3000)
    small = synth.draw_params(np.random.default_rng(2), 700)
    counts = [sp.proposals.shape[0] for sp in specs]
    allp = np.concatenate([sp.proposals for sp in specs])
    solo_a = ctx.loglike(lids[0], big)
    solo_b = ctx.loglike(lids[1], small)
    solo_m = np.concatenate(ctx.loglike_multi(lids, [sp.proposals for sp in specs]))
    pa, pb, pm = (torch.from_numpy(x).to(dev) for x in (big, small, allp))
    reps = 12
    oa = [torch.empty(len(big), dtype=torch.float64, device=dev) for _ in range(reps)]
    ob = [torch.empty(len(small), dtype=torch.float64, device=dev) for _ in range(reps)]
    om = [torch.empty(len(allp), dtype=torch.float64, device=dev) for _ in range(reps)]
    torch.cuda.synchronize()
    errors = []

    def run(fn):
        def body():
            try:
                fn()
            except Exception as ex:   # reported by the main thread
                errors.append(ex)
        return body

    def t1():
        for i in range(reps):
            ctx.loglike_device(lids[0], pa, oa[i], st)
            ctx.loglike_multi_device(lids, counts, pm, om[i], st)

    def t2():
        for i in range(reps):
            ctx.loglike_device(lids[1], pb, ob[i], st)

    th = [threading.Thread(target=run(f)) for f in (t1, t2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    st.synchronize()
    assert not errors, errors
    for i in range(reps):
        assert np.array_equal(oa[i].cpu().numpy(), solo_a), i
        assert np.array_equal(ob[i].cpu().numpy(), solo_b), i
        assert np.array_equal(om[i].cpu().numpy(), solo_m), i
    for lid in lids:
        ctx.unload(lid)
