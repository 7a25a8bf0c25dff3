"""The benchmark's measurement arithmetic, on the CPU: the roofline objects
(the step kernel's VALU-issue figure from the committed counters, the HBM
view, the fallback when the counters belong to other kernel sources), the
replay roofline, and the paired mixed-vs-FP64 deviation split into its
systematic part and its noise."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _stats(launches=16, esteps=1.0e9, ms_estep=46.0):
    return dict(timed_iterations=launches, ms_estep=ms_estep, esteps=esteps, evisits=1.9e7, ewrites=2.1e7,
                inserts=1.1e8)


def _counters():
    with open(bench.COUNTERS) as fh:
        return json.load(fh)


def test_issue_peak_is_the_chip_wave_issue_rate():
    # 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD every 4 cycles, 2.4 GHz
    assert bench.VALU_ISSUE_PEAK == pytest.approx(256 * 4 * 2.4e9 / 4 / 1e9)
    # the FP32 vector peak is that rate x 64 lanes x 2 (FMA) x 2 (packed)
    assert bench.VALU_ISSUE_PEAK * 64 * 2 * 2 / 1e3 == pytest.approx(157.3, rel=1e-3)


def test_algorithmic_bytes_per_unit():
    st = dict(evisits=1.0, ewrites=2.0, esteps=10.0, inserts=3.0)
    # mixed record: 3 x 8 + 4 x 4 + 8 + 4 x 4 = 64 B; FP64: 80 B
    assert bench.estep_algorithmic_bytes(st, fp64=False) == 64 * 3 + 4 * 10 + 32 * 3
    assert bench.estep_algorithmic_bytes(st, fp64=True) == 80 * 3 + 8 * 10 + 32 * 3


def test_roofline_from_the_committed_counters():
    prof = _counters()
    if prof["kernel_source_digest"] != bench.kernel_source_digest():
        pytest.skip("the committed counters belong to other kernel sources (the benchmark reports the HBM view)")
    st = _stats()
    r = bench.roofline(st)
    per_launch = st["esteps"] / st["timed_iterations"]
    avg_s = st["ms_estep"] / st["timed_iterations"] * 1e-3
    want = prof["valu_wave_instr_per_estep"] * per_launch / avg_s / 1e9
    assert r["bound"] == "alu" and r["unit"] == "G VALU wave-instr/s"
    assert r["achieved"] == pytest.approx(want)
    assert r["frac"] == pytest.approx(want / bench.VALU_ISSUE_PEAK)
    assert r["traffic"] == pytest.approx(prof["hbm_bytes_per_estep"] * per_launch)
    alg = bench.estep_algorithmic_bytes(st, fp64=False) / st["timed_iterations"]
    assert r["hbm"]["achieved"] == pytest.approx(alg / avg_s / 1e9)
    r64 = bench.roofline(st, fp64=True)
    assert r64["achieved"] == pytest.approx(prof["fp64_k_estep"]["valu_wave_instr_per_estep"] * per_launch / avg_s / 1e9)
    assert bench.roofline(dict(st, timed_iterations=0)) is None


def test_roofline_falls_back_to_hbm_for_other_kernel_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0000000000000000")
    r = bench.roofline(_stats())
    assert r["bound"] == "hbm" and r["traffic"] is None and r["unit"] == "GB/s"
    assert bench.replay_roofline(400.0, 40, 1e9) is None


def test_replay_roofline():
    prof = _counters()
    if prof["kernel_source_digest"] != bench.kernel_source_digest():
        pytest.skip("the committed counters belong to other kernel sources")
    per = sum(v["valu_wave_instr_per_forward_step"] for k, v in prof["gradient_replays"].items()
              if k.startswith("replay"))
    r = bench.replay_roofline(450.0, 40, 1.0e9)
    assert r["valu_wave_instr_per_forward_step"] == pytest.approx(per)
    assert r["achieved"] == pytest.approx(per * 1.0e9 / 0.45 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.VALU_ISSUE_PEAK)


def test_paired_deviation_separates_a_systematic_shift_from_noise():
    rng = np.random.default_rng(3)
    shape = (8, 16, 16)
    base = 1.0 + rng.random(shape)
    k = 20
    d64 = [base * (1.0 + 0.02 * rng.standard_normal(shape)) for _ in range(k)]
    # pure noise between the paths: no systematic part
    noisy = [d * (1.0 + 0.01 * rng.standard_normal(shape)) for d in d64]
    p = bench.paired_deviation(noisy, d64)
    assert abs(p["mean_shift"]) < 4 * p["mean_shift_se"]
    assert p["systematic_rms"] < 0.3 * p["rms_noise"]
    # the same noise plus a 1% shift: found, with its size
    shifted = [d * 1.01 for d in noisy]
    q = bench.paired_deviation(shifted, d64)
    assert q["mean_shift"] == pytest.approx(0.01, abs=5 * q["mean_shift_se"])
    assert q["systematic_rms"] == pytest.approx(0.01, rel=0.15)
    assert q["depth_systematic_rms"] == pytest.approx(0.01, rel=0.15)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
