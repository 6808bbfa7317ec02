"""Parity at the workloads' full sizes, in the launch configurations bench.py
times, on sampled outputs the oracle computes one by one:

- the 64 precision-workload lenses (200x200 px, s = 4, 41x41 Moffat PSF,
  16,384 proposals each) in one device-buffer multi-lens call in the FP16
  split (the default bench line): 64 outputs on each of two lenses and two on
  every other lens, then the other convolution modes on the same two lenses,
  64 outputs each;
- the 256 uneven lenses of the batching workload in one multi-lens call: 8
  outputs per lens.
Every output against the FP64 oracle at the mode's gate."""
import numpy as np
import pytest

from gpu_cases import TOL_BF16, TOL_FP32, oracle_data, oracle_loglike, rel_err, say
from paper_2503_08586_amd import synth

pytestmark = pytest.mark.gpu

MODE_TOL = {0: TOL_FP32, 1: TOL_FP32, 2: TOL_BF16, 3: TOL_FP32}


def _errors(spec, got, idx):
    ref, chi2, C = oracle_loglike(spec, spec.proposals[idx])
    assert np.array_equal(np.isneginf(got), np.isneginf(ref))
    return rel_err(got, ref, chi2, C)


def test_precision_workload_full_call():
    import torch

    from paper_2503_08586_amd import binding
    say("case: 64 lenses 200x200 s=4 k=41 Moffat, 16384 proposals each, one multi-lens device call, FP16 split")
    specs = synth.config4()
    for sp in specs:
        oracle_data(sp)
    dev = torch.device("cuda", 0)
    st = torch.cuda.Stream()
    rng = np.random.default_rng(4040)
    dense = (0, 37)                         # lenses sampled 64 times
    picks = [np.sort(rng.choice(16384, 64 if j in dense else 2, replace=False)) for j in range(64)]
    with binding.LensContext(0) as ctx:
        lids = [ctx.load(sp, precision=1) for sp in specs]
        counts = [16384] * 64
        P = torch.from_numpy(np.ascontiguousarray(np.concatenate([sp.proposals for sp in specs]))).to(dev)
        out = torch.full((P.shape[0],), np.nan, dtype=torch.float64, device=dev)
        ctx.loglike_multi_device(lids, counts, P, out, st)
        st.synchronize()
        got = out.cpu().numpy().reshape(64, 16384)
        assert np.all(np.isfinite(got))
        errs = np.concatenate([_errors(specs[j], got[j, picks[j]], picks[j]) for j in range(64)])
        say("split full call: %d outputs, max err %.3e, p99 %.3e" % (errs.size, errs.max(), np.quantile(errs, 0.99)))
        assert errs.max() <= TOL_FP32
        for lid in lids:
            ctx.unload(lid)
        # the other modes on the two densely sampled lenses, one lens per call
        for m, name in ((0, "fp32"), (3, "split3"), (2, "bf16")):
            for j in dense:
                lid = ctx.load(specs[j], precision=m)
                g = ctx.loglike(lid, specs[j].proposals[picks[j]])
                e = _errors(specs[j], g, picks[j])
                say("%s lens %d: 64 outputs, max err %.3e" % (name, j, e.max()))
                assert e.max() <= MODE_TOL[m]
                ctx.unload(lid)


def test_batching_workload_full_call():
    from paper_2503_08586_amd import binding
    say("case: 256 uneven lenses, one multi-lens call, 8 outputs per lens")
    specs = synth.config3()
    for sp in specs:
        oracle_data(sp)
    rng = np.random.default_rng(3030)
    with binding.LensContext(0) as ctx:
        lids = [ctx.load(sp) for sp in specs]
        outs = ctx.loglike_multi(lids, [sp.proposals for sp in specs])
        errs = []
        for sp, o in zip(specs, outs):
            idx = np.sort(rng.choice(sp.proposals.shape[0], 8, replace=False))
            errs.append(_errors(sp, o[idx], idx))
        errs = np.concatenate(errs)
        say("batching full call: %d outputs, max err %.3e, p99 %.3e" % (errs.size, errs.max(),
                                                                        np.quantile(errs, 0.99)))
        assert errs.max() <= TOL_FP32
        for lid in lids:
            ctx.unload(lid)
