"""Host-side logic of bench.py, on the CPU: the one-GPU refusal, the credited
work behind the roofline fraction, and the gate that keeps a stale HBM-traffic
record out of the bench line."""
import json
import os
import subprocess
import sys
import types

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr and r.stdout == ""


def test_peak_from_unit_counts():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    assert bench.PEAK_SLOT_PER_S == pytest.approx(256 * 4 * 16 * 2.4e9)


def test_credited_slots_of_the_survey_workload():
    """E = 225,024 sub-pixels (the mask dilated by the 13x13 cropped PSF, at
    s = 4), M = 11,304 masked pixels: E (60 + 2 x 10) + M k^2 + M, a
    transcendental costing two full-rate slots (half rate on CDNA4)."""
    assert bench.TRANS_SLOTS == 2
    spec = types.SimpleNamespace(s=4)
    info = {"masked_pixels": 11304, "psf_used": 13, "needed_pixels": 225024 // 16}
    slots, E = bench.credited_slots(spec, info)
    assert E == 225024
    assert slots == 225024 * 80 + 11304 * 169 + 11304 == 19923600


@pytest.mark.parametrize("model,per_eval,n", [(0, 80, 2), (1, 19, 1), (2, 61, 1), (3, 98, 4)])
def test_credited_slots_of_the_solved_amplitude_models(model, per_eval, n):
    """Per sub-pixel: ray trace 34 + 4 x 2, a Sersic with its radius 13 + 3 x 2,
    a second component on the same radius 5 + 2 x 2; per masked pixel N k^2
    taps and N(N+1)/2 + N FP64 moments for N components."""
    spec = types.SimpleNamespace(s=2)
    info = {"masked_pixels": 1000, "psf_used": 11, "needed_pixels": 1500}
    slots, E = bench.credited_slots(spec, info, nnls=True, model=model)
    assert E == 6000
    assert slots == 6000 * per_eval + n * 1000 * 121 + (n * (n + 1) // 2 + n) * 1000


def test_stale_traffic_record_is_ignored(tmp_path, monkeypatch):
    from paper_2503_08586_amd import profiling
    rec = tmp_path / "traffic.txt"
    rec.write_text(json.dumps({"kernel_src_sha256": profiling.kernel_hash(), "traffic_bytes_per_launch": 123.0}))
    monkeypatch.setattr(profiling, "record_path", lambda w: str(rec))
    assert bench.measured_traffic("batched") == 123.0
    assert bench.measured_traffic("precision") is None   # no record for that workload
    rec.write_text(json.dumps({"kernel_src_sha256": "0" * 64, "traffic_bytes_per_launch": 123.0}))
    assert bench.measured_traffic("batched") is None
    rec.write_text("not json")
    assert bench.measured_traffic("batched") is None


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_matrix_core_modes_credit_the_convolution_to_the_mfma(prec):
    """In the BF16 matrix-core precisions the PSF taps are not vector-ALU work:
    E (60 + 2 x 10) + M slots, and 2 M k^2 flops times the products per tap
    against the dense BF16 peak."""
    spec = types.SimpleNamespace(s=4)
    info = {"masked_pixels": 11304, "psf_used": 41, "needed_pixels": 22504}
    slots, E = bench.credited_slots(spec, info, prec=prec)
    assert E == 360064
    assert slots == 360064 * 80 + 11304
    fl = bench.conv_flops(info)
    assert fl == 2 * 11304 * 41 * 41
    t = bench.roofline_terms(slots, fl, prec, 2.0e-6)
    assert t["t_valu_s"] == pytest.approx(slots / (256 * 4 * 16 * 2.4e9))
    assert t["t_mfma_s"] == pytest.approx(fl * {1: 3, 2: 1, 3: 6}[prec] / 2.5e15)
    assert t["frac"] == pytest.approx(max(t["t_valu_s"], t["t_mfma_s"]) / 2.0e-6)
    assert t["bound"] == "alu"
    # the FP32 convolution stays on the vector ALU, with no matrix-core term
    s32, _ = bench.credited_slots(spec, info, prec=0)
    assert s32 == slots + 11304 * 41 * 41
    assert bench.roofline_terms(s32, fl, 0, 1.0)["t_mfma_s"] == 0.0


def test_epl_series_length():
    """The tail f^N/(1 - f) < 1e-16 with f = (1 - q)/(1 + q): one term at q = 1."""
    import numpy as np
    P = np.zeros((3, 20))
    P[:, 1] = [1.0, 0.5, 0.05]
    f = (1 - P[:, 1]) / (1 + P[:, 1])
    want = [1.0]
    for x in f[1:]:
        n = 1
        while x ** n / (1 - x) >= 1e-16:
            n += 1
        want.append(min(n, 128))
    assert bench.epl_terms(P) == pytest.approx(np.mean(want))
