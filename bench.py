#!/usr/bin/env python3
"""Throughput of the batched lens log-likelihood on one MI355X.

Default workload (batched, the largest single-GPU configuration): one step =
one multi-lens call of the whole hot path over 64 lenses of 200x200 px at
0.05"/px with 4x4 supersampling and a 41x41 Moffat PSF (beta 3, FWHM 0.15"),
16,384 proposals per lens (1,048,576 per step) already resident in HBM: the
prep step, then one persistent launch in which workgroups pull (lens,
proposal) items, with the PSF convolution on the BF16 matrix cores in the
three-plane split that meets the 1e-6 lnL gate and an FP64 chi-square.
Beside it, in the same JSON line:
- the plain path: the FP32 one-lens-per-call kernels over the same lenses
  and proposals, device buffers;
- the lnL error of both against the FP64 oracle on a seeded sample (max and
  p99), and the oracle's own rate on that sample (all host cores and one);
- a short serving leg: Poisson requests over 1,000 resident lenses of mixed
  shape in the same precision, with p50/p99 latency at 80% of peak and a
  sampled error;
- the roofline of the persistent kernel with its vector-ALU and matrix-core
  terms.

--workload plain|batch|precision|serving|sampler|sampler_many runs the
other measurements (one survey-scale lens with 65,536 proposals per call;
256 uneven lenses in one persistent graph-captured launch vs one lens at a
time; the 64 precision lenses in every convolution mode; the serving sweep
over offered loads; a stretch-move ensemble on the device vs driven from the
host; many pooled ensembles).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "loglike evals/s at ≤1e-6 rel err, batched vs plain; p50/p99 req latency"
PEAK_SLOT_PER_S = 256 * 4 * 16 * 2.4e9        # FP32 VALU lane-slots/s (non-packed)
PEAK_BF16_FLOP_S = 2.5e15                       # dense BF16 / FP16 matrix-core peak
TRANS_SLOTS = 2                                 # full-rate slots per FP32 transcendental (measured: 1.9)
SLOTS_PER_EVAL = 60 + TRANS_SLOTS * 10          # 60 FMA-class ops + 10 half-rate transcendentals
PRODUCTS = {1: 3, 2: 1, 3: 6}                   # matrix-core products per PSF tap: split (FP16), bf16, split3
DOUBLE_N = (1.0, 4.0, 1.0, 4.0)                 # fixed indices of the two-component model: disc and bulge


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nprop", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="batched: skip the serving leg")
    ap.add_argument("--no-plain", action="store_true", help="batched: skip the plain one-lens-per-call leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target wall time of the oracle sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (for HBM counter calibration)")
    ap.add_argument("--workload", default="batched", choices=["batched", "plain", "batch", "precision", "serving", "peaks",
                                                               "sampler", "sampler_many"])
    ap.add_argument("--sample-per-lens", type=int, default=96,
                    help="batched: proposals per sampled lens checked against the oracle (and timing its CPU "
                         "rate: about 10 s of oracle work on 16 host threads at the default)")
    ap.add_argument("--sample-lenses", type=int, default=16,
                    help="batched: lenses sampled (evenly spaced) for the oracle check")
    ap.add_argument("--serve-requests", type=int, default=240, help="batched: requests of the serving leg")
    ap.add_argument("--walkers", type=int, default=16384, help="sampler: ensemble size")
    ap.add_argument("--lenses", type=int, default=256, help="sampler_many: lenses, one ensemble each")
    ap.add_argument("--walkers-per-lens", type=int, default=64, help="sampler_many: walkers per ensemble")
    ap.add_argument("--precision", default=None, choices=["fp32", "split", "bf16", "split3"])
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--amplitudes", default="explicit", choices=["explicit", "nnls"],
                    help="light amplitudes as parameters, or solved by NNLS (Sec. 2.3; FP32 convolution)")
    ap.add_argument("--light-model", default="both", choices=list(LIGHT),
                    help="light model (solved amplitudes): lens and source, lens light only, lensed source "
                         "only, or two components per galaxy with indices 1 and 4 (implies --amplitudes nnls)")
    ap.add_argument("--mass", default="sie", choices=["sie", "epl"],
                    help="mass model: the SIE, or the elliptical power law with slope gamma ~ U[1.5, 2.5] "
                         "in slot 19")
    ap.add_argument("--requests", type=int, default=300, help="serving: requests per offered load")
    return ap.parse_args()


PREC = {"fp32": 0, "split": 1, "bf16": 2, "split3": 3}
LIGHT = {"both": 0, "lens": 1, "source": 2, "double": 3}
# credited lane-slots per sub-pixel evaluation of each light model: the ray trace
# (grid, SIE, shear, lens equation: ~34 FMA-class ops + 4 transcendentals), a
# Sersic component (~13 FMA + 3 transcendentals with its elliptical radius), and
# a second component sharing that radius (~5 FMA + 2 transcendentals); model 0
# adds up to SLOTS_PER_EVAL
RAY_SLOTS = 34 + 4 * TRANS_SLOTS
SERSIC_SLOTS = 13 + 3 * TRANS_SLOTS
SECOND_SLOTS = 5 + 2 * TRANS_SLOTS
SLOTS_BY_MODEL = {0: RAY_SLOTS + 2 * SERSIC_SLOTS, 1: SERSIC_SLOTS, 2: RAY_SLOTS + SERSIC_SLOTS,
                  3: RAY_SLOTS + 2 * (SERSIC_SLOTS + SECOND_SLOTS)}
CHANNELS = {0: 2, 1: 1, 2: 1, 3: 4}


def gpu_data(ctx, spec):
    """Noise-free image from the library's forward model at the truth, plus the seeded noise."""
    tmp = ctx.load(spec, data=np.zeros((spec.ny, spec.nx)))
    model = ctx.model_image(tmp, spec.truth, stage=1)
    ctx.unload(tmp)
    spec.data = model + spec.noise


def path_dtype(prec):
    """Arithmetic types of the path: FP64 ray trace, light and chi2; FP32, FP16-MFMA or BF16-MFMA convolution."""
    return "f64+f32" if prec in (None, "fp32") else "f64+f16" if prec == "split" else "f64+bf16"


def credited_slots(spec, info, nnls=False, model=0, prec=0):
    """Credited VALU work of one proposal (60 FMA-class + 10 transcendentals per sub-pixel
    evaluation, one FMA per PSF tap at each masked pixel, one FP64 FMA per masked pixel).
    The PSF is the kernel the library convolves with after its tail crop (info["psf_used"]),
    and the sub-pixels are those of the mask dilated by that kernel (info["needed_pixels"]).
    Solved amplitudes (nnls) convolve one channel per light component (N) and take
    N(N+1)/2 + N FP64 moments per masked pixel; the per-evaluation credit follows the
    light model (SLOTS_BY_MODEL).  In the matrix-core precisions (prec 1-3) the PSF taps
    run on the BF16 MFMA and are credited there (conv_flops), not to the vector ALU."""
    M, k = info["masked_pixels"], info["psf_used"]
    E = info["needed_pixels"] * spec.s * spec.s
    if nnls:
        N = CHANNELS[model]
        return E * SLOTS_BY_MODEL[model] + N * M * k * k + (N * (N + 1) // 2 + N) * M, E
    if prec in PRODUCTS:
        return E * SLOTS_PER_EVAL + M, E
    return E * SLOTS_PER_EVAL + M * k * k + M, E


def conv_flops(info):
    """Algorithmic PSF-convolution flops of one proposal: 2 M k^2 (the band padding of
    the Toeplitz operand is not credited)."""
    return 2.0 * info["masked_pixels"] * info["psf_used"] ** 2


def roofline_terms(slots, flops, prec, seconds):
    """T_valu = credited slots / VALU peak; T_mfma = credited convolution flops times the
    products per tap / dense BF16 peak (matrix-core precisions only); the fraction is
    max(T_valu, T_mfma) / measured time."""
    t_valu = slots / PEAK_SLOT_PER_S
    t_mfma = flops * PRODUCTS[prec] / PEAK_BF16_FLOP_S if prec in PRODUCTS else 0.0
    return {"t_valu_s": t_valu, "t_mfma_s": t_mfma, "t_measured_s": seconds,
            "frac": max(t_valu, t_mfma) / seconds,
            "bound": "alu" if t_valu >= t_mfma else "mfma"}


def epl_terms(P):
    """Mean length of the power-law deflection series over proposals P: the terms that
    bring the tail f^N/(1 - f) below 1e-16, f = (1 - q_m)/(1 + q_m), at most 128."""
    q = P[:, 1]
    f = (1.0 - q) / (1.0 + q)
    with np.errstate(divide="ignore"):
        n = np.where(f > 0, np.ceil(np.log(1e-16 * (1.0 - f)) / np.log(np.where(f > 0, f, 0.5))), 1.0)
    return float(np.clip(n, 1, 128).mean())


def oracle_fn(nnls=False, model=0):
    """The oracle's lnL of the chosen amplitude mode and light model, as
    f(geom, psf, data, sigma, mask, P, nthreads=0, return_chi2=False)."""
    import oracle
    orc = oracle.default()
    if not nnls:
        return orc.loglike
    if model == 0:
        return orc.loglike_nnls

    def f(geom, psf, data, sigma, mask, P, nthreads=0, return_chi2=False):
        return orc.loglike_light(geom, psf, data, sigma, mask, P, model, nfix=DOUBLE_N, nthreads=nthreads,
                                 return_chi2=return_chi2)
    return f


def oracle_sample(specs_props, nthreads=0, nnls=False, model=0):
    """Times the oracle over (spec, proposals) pairs; returns (lnL list, chi2 list, C list, seconds)."""
    import oracle
    orc = oracle.default()
    fn = oracle_fn(nnls, model)
    out = []
    t0 = time.perf_counter()
    for spec, P in specs_props:
        ref, chi2 = fn(spec.geom, spec.psf, spec.data, spec.sigma, spec.mask, P, nthreads=nthreads,
                       return_chi2=True)
        out.append((ref, chi2, orc.loglike_norm(spec.sigma, spec.mask)))
    return out, time.perf_counter() - t0, orc.num_threads()


def rel_errors(gpu, ref, chi2, C):
    return np.abs(gpu - ref) / (0.5 * chi2 + abs(C))


def measured_traffic(workload):
    """HBM bytes per launch of the workload's dominant kernel from its committed rocprofv3
    FETCH_SIZE/WRITE_SIZE record, or None when there is none or the kernel sources have
    changed since it was taken."""
    from paper_2503_08586_amd import profiling
    if workload not in profiling.RECORDS:
        return None
    try:
        with open(profiling.record_path(workload)) as f:
            rec = json.load(f)
        if rec.get("kernel_src_sha256") != profiling.kernel_hash():
            return None
        return rec["traffic_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2503_08586_amd import binding, synth

    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "copies": 3}))
        return
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "precision":
        return run_precision(args)
    if args.workload == "serving":
        return run_serving(args)
    if args.workload == "sampler":
        return run_sampler(args)
    if args.workload == "sampler_many":
        return run_sampler_many(args)
    if args.workload == "peaks":
        return run_peaks(args)

    spec = synth.config2(nprop=args.nprop)[0]
    n = spec.proposals.shape[0]
    ctx = binding.LensContext(0, autotune=args.autotune)
    gpu_data(ctx, spec)
    prec = PREC[args.precision or "fp32"]
    model = LIGHT[args.light_model]
    nnls = args.amplitudes == "nnls" or model != 0
    if model == 3:
        spec.proposals = synth.double_component_params(synth.rng_for_config(2), spec.proposals)
    epl = args.mass == "epl"
    if epl:
        spec.proposals[:, 19] = synth.rng_for_config(2).uniform(1.5, 2.5, n)
        spec.truth = spec.truth.copy()
        spec.truth[19] = 2.0
    lid = ctx.load(spec, precision=prec, amplitudes=1 if nnls else 0, light_model=model, sersic_n=DOUBLE_N,
                   mass_model=1 if epl else 0)
    info = ctx.info(lid)

    dev = torch.device("cuda", 0)
    params = torch.from_numpy(spec.proposals).to(dev)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        ctx.loglike_device(lid, params, out, stream)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        ctx.loglike_device(lid, params, out, stream)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    value = n / step_s
    gpu_out = out.cpu().numpy()

    # PCIe-inclusive rate through the host-buffer entry point (reported beside, never as value):
    # one call to size the pinned staging, then the mean of three
    host_out = ctx.loglike(lid, spec.proposals)
    t2 = time.perf_counter()
    for _ in range(3):
        host_out = ctx.loglike(lid, spec.proposals)
    t3 = time.perf_counter()
    host_rate = 3 * n / (t3 - t2)
    assert np.array_equal(host_out, gpu_out)

    # roofline: credited algorithmic VALU work of one launch
    slots_per_prop, E = credited_slots(spec, info, nnls, model, prec)
    if epl:   # the series' extra complex Horner steps, 4 FMAs each, per sub-pixel
        slots_per_prop += E * 4 * (epl_terms(spec.proposals) - 1.0)
    achieved = slots_per_prop * n / (kern_ms * 1e-3)
    terms = roofline_terms(slots_per_prop * n, conv_flops(info) * n, prec, kern_ms * 1e-3)
    kname = ("k_loglike_rt<8,%d>" % info["threads"] if epl and not nnls and prec == 0 else
             "k_loglike_nnls<%d,%d>" % (4 + model + (8 if epl else 0), info["threads"]) if nnls else
             "k_loglike_fp32<%d,%d>" % (info["psf_used"], info["threads"]) if prec == 0 else
             "k_loglike_mfma<%d,%d>" % (prec, info["threads"]))
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOT_PER_S / 1e12,
                "unit": "Tslot/s", "frac": terms["frac"], "terms": terms, "traffic": measured_traffic("plain") if prec == 0 and not nnls and not epl else None,
                "kernel": kname + " (+ k_prep)", "kernel_ms": kern_ms,
                "slots_per_proposal": slots_per_prop, "subpixel_evals_per_proposal": E,
                "psf_used": info["psf_used"], "psf_given": info["psf_size"]}

    cpu = None
    max_err = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.default()
        threads = orc.num_threads()
        # calibrate on a few proposals, then size the sample for ~cpu_seconds
        probe = spec.proposals[:threads]
        ofn = oracle_fn(nnls, model)
        tc0 = time.perf_counter()
        ofn(spec.geom, spec.psf, spec.data, spec.sigma, spec.mask, probe)
        per = (time.perf_counter() - tc0) / len(probe)
        ns = int(max(threads, min(n, round(args.cpu_seconds / max(per, 1e-9)))))
        sample = spec.proposals[:ns]
        tc0 = time.perf_counter()
        ref, chi2 = ofn(spec.geom, spec.psf, spec.data, spec.sigma, spec.mask, sample, return_chi2=True)
        tc = time.perf_counter() - tc0
        C = orc.loglike_norm(spec.sigma, spec.mask)
        err = np.abs(gpu_out[:ns] - ref) / (0.5 * chi2 + abs(C))
        max_err = float(err.max())
        cpu = {"value": ns / tc, "unit": "loglike evals/s", "cores": threads, "kind": "oracle",
               "sample": "first %d of the %d proposals (same lens and data), %.1f s" % (ns, n, tc)}

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "loglike evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": path_dtype(args.precision),
        "data": "synthetic",
        "config": {"workload": "plain survey scale: 1 lens, 128x128 px at 0.05\"/px, 4x4 supersampling, "
                               "21x21 Gaussian PSF FWHM 0.1\", r=3\" mask, %d proposals per call, "
                               "FP64 ray trace, %s PSF convolution, FP64 chi2, %s amplitudes%s%s"
                               % (n, args.precision or "fp32", "NNLS-solved" if nnls else "explicit",
                                  "" if model == 0 else ", light model: " + args.light_model,
                                  ", elliptical power-law mass, gamma ~ U[1.5, 2.5]" if epl else ""),
                   "path": "lens_loglike_batch_device", "proposals_per_call": n,
                   "subpixel_evals_per_s": value * E},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": max_err,
        "pcie_inclusive_evals_per_s": host_rate,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


def _stream_ctx(binding, torch, **kw):
    """A context whose blocking calls run on a torch stream (so HIP events see them)."""
    st = torch.cuda.Stream()
    return binding.LensContext(0, stream=st.cuda_stream, **kw), st


def cpu_model():
    """The host CPU's model name and logical core count (from /proc/cpuinfo)."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


def _timed_steps(fn, stream, steps, warmup):
    """warmup untimed calls, then steps timed calls bracketed by synchronisations; returns
    (wall seconds per step, mean HIP-event milliseconds per step on `stream`)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    return wall, float(np.mean([a.elapsed_time(b) for a, b in ev]))


def run_batched(args):
    """The default line: 64 precision-workload lenses in one device-buffer multi-lens call
    per step, batched mixed precision vs the plain FP32 one-lens-per-call path."""
    import torch

    from paper_2503_08586_amd import binding, synth
    mode = args.precision or "split"
    prec = PREC[mode]
    specs = synth.config4()
    dev = torch.device("cuda", 0)
    st = torch.cuda.Stream()
    ctx = binding.LensContext(0, stream=st.cuda_stream, autotune=args.autotune)
    for sp in specs:
        gpu_data(ctx, sp)
    lids = [ctx.load(sp, precision=prec) for sp in specs]
    counts = [sp.proposals.shape[0] for sp in specs]
    n = int(sum(counts))
    P = np.ascontiguousarray(np.concatenate([sp.proposals for sp in specs]))
    pd = torch.from_numpy(P).to(dev)
    od = torch.empty(n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    step_s, kern_ms = _timed_steps(lambda: ctx.loglike_multi_device(lids, counts, pd, od, st), st, args.steps,
                                   args.warmup)
    got = od.cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(counts)])
    infos = [ctx.info(l) for l in lids]
    slots = sum(credited_slots(sp, inf, prec=prec)[0] * c for sp, inf, c in zip(specs, infos, counts))
    flops = sum(conv_flops(inf) * c for inf, c in zip(infos, counts))
    evals = sum(credited_slots(sp, inf, prec=prec)[1] * c for sp, inf, c in zip(specs, infos, counts))
    terms = roofline_terms(slots, flops, prec, kern_ms * 1e-3)
    roofline = {"bound": terms["bound"], "achieved": slots / (kern_ms * 1e-3) / 1e12,
                "peak": PEAK_SLOT_PER_S / 1e12, "unit": "Tslot/s", "frac": terms["frac"],
                "traffic": measured_traffic("batched") if mode == "split" else None,
                "mfma": {"achieved": flops * PRODUCTS.get(prec, 0) / (kern_ms * 1e-3) / 1e12,
                         "peak": PEAK_BF16_FLOP_S / 1e12, "unit": "TFLOP/s",
                         "frac": terms["t_mfma_s"] / (kern_ms * 1e-3),
                         "note": "2 M k^2 flops per proposal times %d %s products per tap"
                                 % (PRODUCTS.get(prec, 0), "FP16" if prec == 1 else "BF16")},
                "terms": terms,
                "kernel": "k_loglike_batch<%d,%d> (+ k_prep, counter reset)" % (prec, infos[0]["threads"]),
                "kernel_ms": kern_ms, "slots_per_step": slots, "conv_flops_per_step": flops,
                "tile": [infos[0]["strip_rows"], infos[0]["threads"], infos[0]["blocks_per_cu"],
                         infos[0]["lds_bytes"]]}

    # the FP64 FMA issue rate measured on this device, beside the nominal peak
    fma = ctx.peak_rate("fma_f64")
    roofline["peak_measured"] = {"fma_f64": fma / 1e12, "unit": "Tslot/s",
                                 "frac": roofline["achieved"] * 1e12 / fma,
                                 "note": "lens_peak_rate(LENS_PEAK_FMA_F64) after the timed steps"}

    # the plain path: FP32, one lens per call, same proposals, device buffers
    plain = None
    got32 = None
    if not args.no_plain:
        lids32 = [ctx.load(sp, precision=0) for sp in specs]
        o32 = torch.empty(n, dtype=torch.float64, device=dev)

        def plain_pass():
            for j, l in enumerate(lids32):
                ctx.loglike_device(l, pd[offs[j]:offs[j + 1]], o32[offs[j]:offs[j + 1]], st)
        pstep, pms = _timed_steps(plain_pass, st, 1, 1)
        got32 = o32.cpu().numpy()
        plain = {"evals_per_s": n / pstep, "ms_per_pass": pstep * 1e3, "event_ms": pms,
                 "path": "lens_loglike_batch_device per lens, FP32 PSF convolution (k_loglike_fp32<41,256>)"}
        for l in lids32:
            ctx.unload(l)

    # error of both paths on a seeded sample, and the oracle's own rate on it
    errs = {}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.default()
        rng = np.random.default_rng(synth.SEED_BASE + 40)
        k = args.sample_per_lens
        sel = np.unique(np.linspace(0, len(specs) - 1, args.sample_lenses).round().astype(int))
        picks = {int(j): np.sort(rng.choice(counts[j], k, replace=False)) for j in sel}
        sample = [(specs[j], specs[j].proposals[picks[j]]) for j in picks]
        res, tc, threads = oracle_sample(sample)
        e_b = np.concatenate([rel_errors(got[offs[j] + picks[j]], r[0], r[1], r[2]) for j, r in zip(picks, res)])
        errs["batched"] = {"max": float(e_b.max()), "p99": float(np.quantile(e_b, 0.99)), "n": int(e_b.size)}
        if got32 is not None:
            e_p = np.concatenate([rel_errors(got32[offs[j] + picks[j]], r[0], r[1], r[2])
                                  for j, r in zip(picks, res)])
            errs["plain"] = {"max": float(e_p.max()), "p99": float(np.quantile(e_p, 0.99)), "n": int(e_p.size)}
        # one thread, four proposals of the first sampled lens
        j0 = int(sel[0])
        t1 = time.perf_counter()
        orc.loglike(specs[j0].geom, specs[j0].psf, specs[j0].data, specs[j0].sigma, specs[j0].mask,
                    specs[j0].proposals[picks[j0][:4]], nthreads=1)
        t1 = time.perf_counter() - t1
        model, ncpu = cpu_model()
        cpu = {"value": k * len(picks) / tc, "unit": "loglike evals/s", "cores": min(threads, k), "kind": "oracle",
               "sample": "%d seeded proposals of each of %d evenly spaced lenses (%d; one oracle call per lens), "
                         "%.1f s" % (k, len(picks), k * len(picks), tc),
               "single_thread": {"value": 4 / t1, "sample": "4 proposals of lens %d, %.1f s" % (j0, t1)},
               "cpu_model": model, "logical_cpus": ncpu}
    for l in lids:
        ctx.unload(l)
    ctx.close()

    serving = None if args.no_serving else serving_leg(args, mode)
    rec = {
        "metric": METRIC, "value": n / step_s, "unit": "loglike evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": path_dtype(mode), "data": "synthetic",
        "config": {"workload": "batched precision workload: 64 lenses 200x200 px at 0.05\"/px, 4x4 supersampling, "
                               "41x41 Moffat PSF beta 3 FWHM 0.15\", r=3\" mask, 16,384 proposals per lens per step, "
                               "one device-buffer multi-lens call (persistent launch), FP64 ray trace, %s "
                               "matrix-core PSF convolution, FP64 chi2"
                               % {"split": "FP16 hi+lo split", "split3": "BF16 hi+mid+lo split",
                                  "bf16": "BF16"}.get(mode, mode),
                   "path": "lens_loglike_multi_device", "proposals_per_step": n, "precision": mode,
                   "subpixel_evals_per_s": evals / step_s},
        "plain": plain,
        "batched_over_plain": (n / step_s) / plain["evals_per_s"] if plain else None,
        "rel_err_vs_oracle": errs,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(rec), flush=True)


def serve_stream(ctx, lids, reqs, rate, rng):
    """Open-loop Poisson arrivals of reqs [(lens index, proposals)] at `rate` requests/s
    (None: all at once), then a wait for every request.  Returns (served evals/s over
    the makespan, the handles, the library's latency statistics of exactly these requests:
    submit to result written, exact nearest-rank p50/p99)."""
    arr = np.zeros(len(reqs)) if rate is None else synth_mod().poisson_arrivals(rng, rate, len(reqs))
    ctx.reset_stats()
    handles = []
    t0 = time.perf_counter()
    for i, (j, P) in enumerate(reqs):
        while time.perf_counter() - t0 < arr[i]:
            time.sleep(20e-6)
        handles.append(ctx.submit(lids[j], P))
    for h in handles:
        assert ctx.wait(h) == 0
    t_end = time.perf_counter()
    st = ctx.stats()
    assert st["latency_count"] == len(reqs)
    props = sum(P.shape[0] for _, P in reqs)
    return props / (t_end - t0), handles, st


def synth_mod():
    from paper_2503_08586_amd import synth
    return synth


def serving_leg(args, mode, loads=(0.8,), nreq=None, sample_err=True):
    """C5 serving: 1,000 resident lenses of mixed shape in precision `mode`, Poisson requests
    of U{100..10000} proposals on random lenses; the saturated peak from a backlog, then
    each offered load as a fraction of that peak with p50/p99 latency; a few requests'
    results against the oracle."""
    from paper_2503_08586_amd import binding
    synth = synth_mod()
    nreq = nreq or args.serve_requests
    prec = PREC[mode]
    lenses = synth.config5_lenses()
    ctx = binding.LensContext(0, autotune=args.autotune)
    t_load = time.perf_counter()
    lids = []
    for sp in lenses:
        gpu_data(ctx, sp)
        lids.append(ctx.load(sp, precision=prec))
    t_load = time.perf_counter() - t_load
    rng = synth.rng_for_config(5)
    mean_b = 5050.0

    def make_requests(count):
        out = []
        for _ in range(count):
            j = int(rng.integers(0, len(lids)))
            b = int(rng.integers(100, 10001))
            out.append((j, synth.draw_params(rng, b)))
        return out

    peak_reqs = make_requests(max(40, nreq // 3))
    peak, _, _ = serve_stream(ctx, lids, peak_reqs, None, rng)
    # the same requests as one batched call on host buffers (the graph-captured multi-lens call,
    # copies included, as serving's are) and on device buffers
    # the same requests as one batched call on device buffers (no serving): the rate serving is held to
    import torch
    dev = torch.device("cuda", 0)
    st = torch.cuda.Stream()
    ids = [lids[j] for j, _ in peak_reqs]
    cnt = [P.shape[0] for _, P in peak_reqs]
    pd = torch.from_numpy(np.ascontiguousarray(np.concatenate([P for _, P in peak_reqs]))).to(dev)
    od = torch.empty(int(sum(cnt)), dtype=torch.float64, device=dev)
    bstep, _ = _timed_steps(lambda: ctx.loglike_multi_device(ids, cnt, pd, od, st), st, 2, 1)
    batched = sum(cnt) / bstep
    plist = [P for _, P in peak_reqs]
    ctx.loglike_multi(ids, plist)
    th0 = time.perf_counter()
    for _ in range(2):
        ctx.loglike_multi(ids, plist)
    batched_host = 2 * sum(cnt) / (time.perf_counter() - th0)
    out = {"peak_evals_per_s": peak, "batched_same_requests_evals_per_s": batched,
           "batched_same_requests_host_buffers_evals_per_s": batched_host,
           "peak_over_batched": peak / batched, "peak_over_batched_host_buffers": peak / batched_host,
           "precision": mode, "lenses": len(lids), "load_s": t_load, "loads": {}}
    last = None
    for rho in loads:
        reqs = make_requests(nreq)
        thr, hs, stt = serve_stream(ctx, lids, reqs, rho * peak / mean_b, rng)
        out["loads"][str(rho)] = {"offered_evals_per_s": rho * peak, "evals_per_s": thr, "requests": len(reqs),
                                  "p50_ms": stt["latency_p50_us"] * 1e-3, "p99_ms": stt["latency_p99_us"] * 1e-3,
                                  "max_ms": stt["latency_max_us"] * 1e-3, "batches": stt["launches"],
                                  "request_pieces_per_batch": stt["batch_pieces"] / max(1, stt["launches"])}
        last = (reqs, hs)
    out["latency"] = "lens_get_stats: lens_submit to the result written, exact nearest-rank quantiles per load"
    if sample_err and last is not None:
        reqs, hs = last
        sample = []
        for (j, P), h in list(zip(reqs, hs))[:8]:
            sample.append((lenses[j], P[:2], h.out[:2]))
        res, _, _ = oracle_sample([(sp, P) for sp, P, _ in sample])
        e = np.concatenate([rel_errors(g, r[0], r[1], r[2]) for (_, _, g), r in zip(sample, res)])
        out["rel_err_vs_oracle"] = {"max": float(e.max()), "n": int(e.size),
                                    "sample": "2 proposals of each of the last load's first 8 requests"}
    ctx.close()
    return out


def run_batch(args):
    import torch

    from paper_2503_08586_amd import binding, synth
    prec = PREC[args.precision or "fp32"]
    model = LIGHT[args.light_model]
    nnls = args.amplitudes == "nnls" or model != 0
    specs = synth.config3()
    ctx, st = _stream_ctx(binding, torch, autotune=args.autotune)
    lids, slots, evs, flops = [], 0.0, 0, 0.0
    drng = synth.rng_for_config(3)
    for sp in specs:
        gpu_data(ctx, sp)
        if model == 3:
            sp.proposals = synth.double_component_params(drng, sp.proposals)
        lid = ctx.load(sp, precision=prec, amplitudes=1 if nnls else 0, light_model=model, sersic_n=DOUBLE_N)
        lids.append(lid)
        sl, E = credited_slots(sp, ctx.info(lid), nnls, model, prec)
        slots += sl * sp.proposals.shape[0]
        flops += conv_flops(ctx.info(lid)) * sp.proposals.shape[0]
        evs += E * sp.proposals.shape[0]
    plist = [sp.proposals for sp in specs]
    n = int(sum(p.shape[0] for p in plist))
    for _ in range(args.warmup):
        outs = ctx.loglike_multi(lids, plist)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(st)
        outs = ctx.loglike_multi(lids, plist)
        ev[i][1].record(st)
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / args.steps
    gpu_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    # plain: the same proposals one lens at a time, no graph, no persistent kernel
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    singles = [ctx.loglike(lid, p) for lid, p in zip(lids, plist)]
    plain_s = time.perf_counter() - t0
    same = all(np.array_equal(a, b) for a, b in zip(outs, singles))
    sample = [(specs[j], specs[j].proposals[:2]) for j in range(0, len(specs), 8)]
    res, tc, threads = oracle_sample(sample, nnls=nnls, model=model)
    errs = [rel_errors(outs[j][:2], r[0], r[1], r[2]).max() for (j, r) in zip(range(0, len(specs), 8), res)]
    rec = {
        "metric": METRIC, "value": n / step_s, "unit": "loglike evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": path_dtype(args.precision), "data": "synthetic",
        "config": {"workload": "batching: 256 lenses, N~U{48..160}, 0.05-0.074\"/px, s in {2,4}, k in 11..31, "
                               "%d proposals (U{128..4096} per lens), one persistent launch in a hipGraph, "
                               "host buffers, %s PSF convolution, %s amplitudes%s"
                               % (n, args.precision or "fp32", "NNLS-solved" if nnls else "explicit",
                                  "" if model == 0 else ", light model: " + args.light_model),
                   "proposals_per_call": n, "autotune": bool(args.autotune)},
        "plain_one_lens_at_a_time_evals_per_s": n / plain_s,
        "batched_over_plain": plain_s / step_s,
        "batched_equals_plain_bitwise": bool(same),
        "roofline": {"bound": "alu", "achieved": slots / (gpu_ms * 1e-3) / 1e12, "peak": PEAK_SLOT_PER_S / 1e12,
                     "unit": "Tslot/s", "frac": roofline_terms(slots, flops, prec, gpu_ms * 1e-3)["frac"],
                     "terms": roofline_terms(slots, flops, prec, gpu_ms * 1e-3), "traffic": None,
                     "kernel": "k_loglike_batch (graph: H2D, prep, persistent kernel, D2H)", "call_ms": gpu_ms},
        "cpu_baseline": {"value": sum(len(P) for _, P in sample) / tc, "unit": "loglike evals/s", "cores": threads,
                         "kind": "oracle", "sample": "2 proposals of each of 32 lenses (every 8th)"},
        "max_rel_err_vs_oracle": float(max(errs)),
        "subpixel_evals_per_s": evs / step_s,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


def _host_stretch(binding, ctx, lid, w, lnp, lo, hi, a, iters, rng):
    """The stretch move driven from the host (numpy draws, host-buffer lnL calls):
    the transfer pattern of a host-side sampler, for comparison with the device loop."""
    W = w.shape[0]
    h = W // 2
    d = int(np.count_nonzero(hi > lo))
    for _ in range(iters):
        for half in (0, 1):
            k = np.arange(half * h, (half + 1) * h)
            j = (1 - half) * h + rng.integers(0, h, h)
            z = ((a - 1.0) * rng.random(h) + 1.0) ** 2 / a
            Y = w[j] + z[:, None] * (w[k] - w[j])
            inside = np.all((Y >= lo) & (Y <= hi), axis=1)
            lnY = np.full(h, -np.inf)
            lnY[inside] = ctx.loglike(lid, Y[inside])
            take = np.log(rng.random(h)) < (d - 1) * np.log(z) + lnY - lnp[k]
            w[k[take]] = Y[take]
            lnp[k[take]] = lnY[take]


def run_sampler(args):
    """Device-resident sampler loop on the plain survey-scale lens: an ensemble of
    --walkers walkers moved by the stretch move, each half-step's proposals made,
    evaluated and accepted on the device; one step = one iteration (W proposals)."""
    import torch

    from paper_2503_08586_amd import binding, synth
    spec = synth.config2(nprop=1)[0]
    ctx, st = _stream_ctx(binding, torch)
    gpu_data(ctx, spec)
    lid = ctx.load(spec)
    info = ctx.info(lid)
    lo = np.array([b[1] for b in synth.PRIOR_BOX] + [0.0])
    hi = np.array([b[2] for b in synth.PRIOR_BOX] + [0.0])
    W = args.walkers
    rng = np.random.default_rng(synth.SEED_BASE + 6)
    init = np.clip(spec.truth[None, :] + 0.02 * (hi - lo)[None, :] * rng.normal(size=(W, 20)), lo, hi)
    ens = ctx.ensemble(lid, init, lo, hi, stretch=2.0, seed=synth.SEED_BASE)
    ctx.ensemble_run(ens, args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(st)
    ctx.ensemble_run(ens, args.steps)
    ev1.record(st)
    torch.cuda.synchronize()
    loop_s = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    n = W * args.steps
    w, lnp, acc, it = ctx.ensemble_get(ens)
    # the same moves from the host: numpy draws, proposals and results over PCIe
    hw, hl = init.copy(), ctx.loglike(lid, init)
    hsteps = max(1, args.steps // 4)
    t2 = time.perf_counter()
    _host_stretch(binding, ctx, lid, hw, hl, lo, hi, 2.0, hsteps, rng)
    host_s = time.perf_counter() - t2
    host_rate = W * hsteps / host_s
    slots_per_prop, E = credited_slots(spec, info)
    cpu = None
    max_err = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.default()
        threads = orc.num_threads()
        tc0 = time.perf_counter()
        orc.loglike(spec.geom, spec.psf, spec.data, spec.sigma, spec.mask, w[:threads])
        per = (time.perf_counter() - tc0) / threads
        ns = int(max(threads, min(W, round(args.cpu_seconds / max(per, 1e-9)))))
        tc0 = time.perf_counter()
        ref, chi2 = orc.loglike(spec.geom, spec.psf, spec.data, spec.sigma, spec.mask, w[:ns], return_chi2=True)
        tc = time.perf_counter() - tc0
        C = orc.loglike_norm(spec.sigma, spec.mask)
        max_err = float((np.abs(lnp[:ns] - ref) / (0.5 * chi2 + abs(C))).max())
        cpu = {"value": ns / tc, "unit": "loglike evals/s", "cores": threads, "kind": "oracle",
               "sample": "lnL of the first %d final walkers, %.1f s" % (ns, tc)}
    rec = {
        "metric": METRIC, "value": n / loop_s, "unit": "loglike evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": loop_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": path_dtype(None),
        "data": "synthetic",
        "config": {"workload": "sampler loop on the device: %d-walker stretch-move ensemble on the plain "
                               "survey-scale lens (128x128 px, s=4, 21x21 PSF), one step = one iteration "
                               "(%d proposals made, evaluated and accepted on the device)" % (W, W),
                   "walkers": W, "acceptance": float(acc.sum()) / max(1, W * it)},
        "host_driven_loop_evals_per_s": host_rate,
        "device_over_host_loop": (n / loop_s) / host_rate,
        "roofline": {"bound": "alu", "achieved": slots_per_prop * n / (gpu_ms * 1e-3) / 1e12,
                     "peak": PEAK_SLOT_PER_S / 1e12, "unit": "Tslot/s",
                     "frac": slots_per_prop * n / (gpu_ms * 1e-3) / PEAK_SLOT_PER_S, "traffic": None,
                     "kernel": "k_stretch_propose + k_loglike_fp32 + k_stretch_accept per half-step",
                     "loop_ms": gpu_ms},
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": max_err,
    }
    print(json.dumps(rec), flush=True)
    ctx.ensemble_destroy(ens)
    ctx.close()


def run_sampler_many(args):
    """Survey fitting: --lenses heterogeneous lenses of the batching mix, each
    with its own --walkers-per-lens ensemble, advanced together (pooled
    proposals per half-step); one step = one iteration of every ensemble.
    Beside it, the same ensembles advanced one after another."""
    import torch

    from paper_2503_08586_amd import binding, synth
    specs = synth.config3(nlens=args.lenses, scale_props=0.0)
    ctx, st = _stream_ctx(binding, torch)
    lo = np.array([b[1] for b in synth.PRIOR_BOX] + [0.0])
    hi = np.array([b[2] for b in synth.PRIOR_BOX] + [0.0])
    W = args.walkers_per_lens
    rng = np.random.default_rng(synth.SEED_BASE + 7)
    lids, pooled, single, slots = [], [], [], 0.0
    for i, sp in enumerate(specs):
        gpu_data(ctx, sp)
        lid = ctx.load(sp)
        lids.append(lid)
        sl, _ = credited_slots(sp, ctx.info(lid))
        slots += sl * W
        init = np.clip(sp.truth[None, :] + 0.02 * (hi - lo)[None, :] * rng.normal(size=(W, 20)), lo, hi)
        pooled.append(ctx.ensemble(lid, init, lo, hi, stretch=2.0, seed=synth.SEED_BASE + i))
        single.append(ctx.ensemble(lid, init, lo, hi, stretch=2.0, seed=synth.SEED_BASE + i))
    ctx.ensemble_run_many(pooled, args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(st)
    ctx.ensemble_run_many(pooled, args.steps)
    ev1.record(st)
    torch.cuda.synchronize()
    loop_s = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    n = W * len(specs) * args.steps
    # the same ensembles one after another (after the same warm-up)
    for e in single:
        ctx.ensemble_run(e, args.warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for e in single:
        ctx.ensemble_run(e, args.steps)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t1
    same = all(all(np.array_equal(x, y) for x, y in zip(ctx.ensemble_get(p)[:3], ctx.ensemble_get(q)[:3]))
               for p, q in zip(pooled, single))
    acc = sum(float(ctx.ensemble_get(p)[2].sum()) for p in pooled)
    cpu = None
    if not args.no_cpu_baseline:
        # the final walkers of the first lenses, lens by lens, until about --cpu-seconds
        tc, ns, nl = 0.0, 0, 0
        for j in range(len(specs)):
            w, _, _, _ = ctx.ensemble_get(pooled[j])
            _, dt, threads = oracle_sample([(specs[j], w)])
            tc, ns, nl = tc + dt, ns + len(w), nl + 1
            if tc >= args.cpu_seconds:
                break
        cpu = {"value": ns / tc, "unit": "loglike evals/s", "cores": min(threads, W), "kind": "oracle",
               "sample": "lnL of the %d final walkers of each of the first %d lenses, %.1f s" % (W, nl, tc)}
    rec = {
        "metric": METRIC, "value": n / loop_s, "unit": "loglike evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": loop_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": path_dtype(None),
        "data": "synthetic",
        "config": {"workload": "survey sampling on the device: %d lenses of the batching mix (N 48-160 px, "
                               "s 2|4, k 11-31), one %d-walker stretch-move ensemble each, advanced together; "
                               "one step = one iteration of every ensemble (%d proposals)"
                               % (len(specs), W, W * len(specs)),
                   "lenses": len(specs), "walkers_per_lens": W,
                   "acceptance": acc / max(1, W * len(specs) * (args.steps + args.warmup))},
        "separate_runs_evals_per_s": n / seq_s,
        "pooled_over_separate": seq_s / loop_s,
        "pooled_equals_separate_bitwise": same,
        "roofline": {"bound": "alu", "achieved": slots * args.steps / (gpu_ms * 1e-3) / 1e12,
                     "peak": PEAK_SLOT_PER_S / 1e12, "unit": "Tslot/s",
                     "frac": slots * args.steps / (gpu_ms * 1e-3) / PEAK_SLOT_PER_S, "traffic": None,
                     "kernel": "k_stretch_propose_many + k_loglike_batch + k_stretch_accept_many per half-step",
                     "loop_ms": gpu_ms},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    for e in pooled + single:
        ctx.ensemble_destroy(e)
    ctx.close()


def run_precision(args):
    import torch

    from paper_2503_08586_amd import binding, synth
    specs = synth.config4()
    ctx, st = _stream_ctx(binding, torch, autotune=args.autotune)
    for sp in specs:
        gpu_data(ctx, sp)
    modes = [args.precision] if args.precision else ["fp32", "split", "split3", "bf16"]
    sample_idx = list(range(0, len(specs), 4))
    ns = 8   # proposals per sampled lens (one oracle call each)
    res, tc, threads = oracle_sample([(specs[j], specs[j].proposals[:ns]) for j in sample_idx])
    per = {}
    for m in modes:
        lids = [ctx.load(sp, precision=PREC[m]) for sp in specs]
        plist = [sp.proposals for sp in specs]
        n = int(sum(p.shape[0] for p in plist))
        slots = sum(credited_slots(sp, ctx.info(l), prec=PREC[m])[0] * sp.proposals.shape[0]
                    for sp, l in zip(specs, lids))
        flops = sum(conv_flops(ctx.info(l)) * sp.proposals.shape[0] for sp, l in zip(specs, lids))
        for _ in range(max(1, args.warmup)):
            outs = ctx.loglike_multi(lids, plist)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a.record(st)
        for _ in range(args.steps):
            outs = ctx.loglike_multi(lids, plist)
        b.record(st)
        torch.cuda.synchronize()
        step_s = (time.perf_counter() - t0) / args.steps
        gpu_ms = a.elapsed_time(b) / args.steps
        errs = np.concatenate([rel_errors(outs[j][:ns], r[0], r[1], r[2]) for j, r in zip(sample_idx, res)])
        inf = ctx.info(lids[0])
        per[m] = {"tile": [inf["strip_rows"], inf["threads"], inf["blocks_per_cu"], inf["lds_bytes"]],
                  "evals_per_s": n / step_s, "ms_per_step": step_s * 1e3, "max_rel_err": float(errs.max()),
                  "p99_rel_err": float(np.quantile(errs, 0.99)),
                  "roofline": roofline_terms(slots, flops, PREC[m], gpu_ms * 1e-3)}
        for l in lids:
            ctx.unload(l)
    # value: the fastest mode gated at 1e-6 (fp32, split, split3); plain BF16 (~1e-3) is
    # reported beside it in "modes" but never as value
    ok = [m for m in per if m in ("fp32", "split", "split3")] or list(per)
    best = max(ok, key=lambda m: per[m]["evals_per_s"])
    rec = {"metric": METRIC, "value": per[best]["evals_per_s"], "unit": "loglike evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": per[best]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": path_dtype(best), "data": "synthetic",
           "config": {"workload": "precision: 64 lenses 200x200 px at 0.05\"/px, s=4, 41x41 Moffat beta=3 FWHM 0.15\", "
                                  "16,384 proposals each, one multi-lens call per step", "value_mode": best},
           "modes": per,
           "cpu_baseline": {"value": ns * len(sample_idx) / tc, "unit": "loglike evals/s", "cores": min(threads, ns),
                            "kind": "oracle", "sample": "%d proposals of each of 16 lenses" % ns}}
    print(json.dumps(rec), flush=True)
    ctx.close()


def run_serving(args):
    """The serving sweep: offered loads of 50-100% of the saturated peak."""
    mode = args.precision or "split"
    out = serving_leg(args, mode, loads=(0.5, 0.6, 0.7, 0.8, 0.9, 1.0), nreq=args.requests)
    rec = {"metric": METRIC, "value": out["peak_evals_per_s"], "unit": "loglike evals/s", "n_gpus": 1,
           "steps": args.requests, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": path_dtype(mode), "data": "synthetic",
           "config": {"workload": "serving: 1,000 resident lenses N~U{48..200}, k~U{11..41}, s=4, Gaussian/Moffat "
                                  "PSFs; Poisson requests of U{100..10000} proposals on random lenses; %s convolution"
                                  % mode, "requests_per_load": args.requests},
           "serving": out}
    print(json.dumps(rec), flush=True)


def run_peaks(args):
    """Issue rates of the instruction kinds the likelihood kernels are built from
    (lens_peak_rate), in lane operations/s (vector ALU) or FLOP/s (matrix cores),
    with each one's cost in full-rate slots at the nominal peak (PEAK_SLOT_PER_S /
    rate): the credit behind the roofline counts a transcendental as TRANS_SLOTS slots."""
    from paper_2503_08586_amd import binding
    ctx = binding.LensContext(0)
    rates = {}
    for name in binding.PEAK_OPS:
        r = ctx.peak_rate(name)
        if name in ("mfma_f16", "mfma_bf16"):
            rates[name] = {"tflop_s": r / 1e12, "frac_of_nominal": r / PEAK_BF16_FLOP_S}
        else:
            rates[name] = {"t_lane_ops_s": r / 1e12, "slots_per_op": PEAK_SLOT_PER_S / r}
        print("peak %s: %.4g" % (name, r), file=sys.stderr, flush=True)
    print(json.dumps({"metric": "instruction issue rates", "n_gpus": 1, "data": "synthetic",
                      "nominal": {"valu_lane_slots_s": PEAK_SLOT_PER_S, "mfma_flop_s": PEAK_BF16_FLOP_S},
                      "launch": "8 waves per SIMD, 8 independent chains per lane, best of 3 launches of ~25 ms",
                      "rates": rates}))


if __name__ == "__main__":
    main()
