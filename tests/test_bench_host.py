"""Host logic of bench.py, on the CPU: the one-GPU refusal, the per-sample
work the rooflines divide by, the choice of bound, the parse of the counter
summary (and its refusal when the kernel sources changed), and the per-step
distribution."""
import hashlib
import os

import numpy as np
import pytest

import bench
import workloads as W


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU only" in capsys.readouterr().err


def test_per_sample_work_of_the_paper_scale_net():
    # 32 -> 64 -> 16 density net, (16 + 16) -> 64 -> 64 -> 3 colour net: the
    # forward takes 2048 + 1024 + 2048 + 4096 + 192 multiply-adds; the input
    # gradient skips the 16 SH inputs of the first colour layer (16 x 64)
    fwd, dx, dw = bench.mlp_macs(W.C2_FIELD)
    assert (fwd, dx, dw) == (9408, 8384, 9408)
    work = bench.kernel_work(W.C2_FIELD, 2)
    assert work["encode"] == dict(flops=0, bytes=8 * 16 * 2 * 2)       # 8 corners, 16 levels, 2 FP16 features
    assert work["table_grad"] == dict(flops=0, bytes=8 * 16 * 2 * 4)   # the same as FP32 gradient adds
    assert work["field_bwd"]["flops"] == 2 * (9408 + 8384 + 9408)
    assert bench.kernel_work(W.C2_FIELD, 4)["encode"]["bytes"] == 1024


def test_roofline_bound_and_fraction():
    # byte-bound: 1024 B a sample, 2^18 samples in 0.1 ms -> 2.68 TB/s
    r = bench.roofline_of("table_grad", dict(flops=0, bytes=1024), 1 << 18, 0.1, bench.PEAK_BF16)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(1024 * (1 << 18) / 1e-4 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    # FLOP-bound at the FP32 peak: 54 kFLOP a sample against no bytes
    r = bench.roofline_of("field_bwd", dict(flops=54400, bytes=0), 1 << 18, 0.2, bench.PEAK_FP32)
    assert r["bound"] == "mfma" and r["peak"] == pytest.approx(157.3)
    assert r["frac"] == pytest.approx(54400 * (1 << 18) / 2e-4 / 157.3e12)


def _summary(path, digest, rows):
    lines = ["# counters", "", f"kernel sources sha256: {digest}", "",
             "| kernel | dispatches | fetch MB / launch | write MB / launch |", "|---|---:|---:|---:|"]
    lines += [f"| `{k}` | 18 | {f} | {w} |" for k, (f, w) in rows.items()]
    path.write_text("\n".join(lines) + "\n")


def _sources_digest():
    h = hashlib.sha256()
    for name in bench.PMC_SOURCES:
        with open(os.path.join(bench.ROOT, "paper_2210_13641_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def test_counter_summary_parse_and_source_check(tmp_path, monkeypatch):
    p = tmp_path / "pmc.md"
    rows = {bench.BIN_KERNELS[0]: (57.0, 114.9), bench.BIN_KERNELS[1]: (114.7, 51.4),
            "mixed_bwd8_kernel<NetFull>": (22.9, 26.4)}
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(p))
    _summary(p, _sources_digest(), rows)
    assert bench.measured_traffic("table_grad", 2) == pytest.approx((57.0 + 114.9 + 114.7 + 51.4) * 1e6)
    assert bench.measured_traffic("field_bwd", 2) == pytest.approx((22.9 + 26.4) * 1e6)
    assert bench.measured_traffic("field_fwd", 2) is None          # a kernel the summary lacks
    assert bench.measured_traffic("table_grad", 4) is None         # counters are of the mixed step only
    _summary(p, "0" * 64, rows)                                   # taken on other kernel sources
    assert bench.measured_traffic("table_grad", 2) is None
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("table_grad", 2) is None


def test_step_time_distribution():
    ms = np.arange(1, 102, dtype=np.float64)      # 1 .. 101
    d = bench.distribution(ms)
    assert d == dict(median=51.0, p10=11.0, p90=91.0, min=1.0, max=101.0, n=101)
