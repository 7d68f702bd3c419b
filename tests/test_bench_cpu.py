"""Host logic of bench.py: the algorithmic byte model of the slice pass, the
roofline fraction, the workload- and source-scoped HBM traffic records, and
the single-GPU guard.  No GPU is used."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _res(batch=1 << 18):
    # a plan of the 256^3 workload's encoding: levels 0-5 privatized, 6-15 partitioned
    ent = [min(int(16 * (16.0 ** (1 / 15)) ** l + 1e-6) ** 3, 1 << 19) for l in range(16)]
    return {"batch": batch, "priv_levels": 6, "part_levels": 6, "level_entries": ent, "n_blocks": 1,
            "n_params": sum(ent) * 2 + 6208, "phase_ms": {"part_accum": 0.1, "part_bucket": 0.05, "mlp": 0.06}}


def test_slice_pass_bytes_and_fraction():
    """10 partitioned levels x 8 records of 8 B per sample, plus 26 B of Adam
    traffic per partitioned table parameter; achieved = bytes / launch time."""
    res = _res()
    npar = sum(res["level_entries"][6:]) * 2
    assert bench.part_params(res) == npar
    want = 10 * 8 * 8 * (1 << 18) + 26 * npar
    assert bench.phase_bytes("mixed", "part_accum", res) == want
    r = bench.roofline_for("mixed", res, "c9")
    assert r["kernel"] == "k_part_accum" and r["bound"] == "hbm" and r["traffic"] is None
    assert r["achieved"] == pytest.approx(want / 1e-4 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)


def test_traffic_record_scoped_to_workload_and_sources(tmp_path, monkeypatch):
    dig = bench.sources_digest("k_part_accum")
    rec = {"kernel": "k_part_accum", "workload": "c2", "read_bytes": 3, "write_bytes": 4, "sources_sha256": dig}
    stale = dict(rec, kernel="k_part_bucket", sources_sha256="0" * 64)
    f = tmp_path / "counters.md"
    f.write_text("# counters\n\ntraffic-record: " + json.dumps(rec) + "\ntraffic-record: " + json.dumps(stale) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILES", [str(tmp_path / "missing.md"), str(f)])
    assert bench.measured_traffic("part_accum", "c2") == 7
    assert bench.measured_traffic("part_accum", "c3") is None  # taken on another workload
    assert bench.measured_traffic("part_bucket", "c2") is None  # sources changed since
    assert bench.measured_traffic("mlp", "c2") is None  # no record


def test_committed_traffic_records_name_their_workload():
    for path in bench.TRAFFIC_FILES:
        with open(path) as fh:
            recs = [json.loads(l.split(":", 1)[1]) for l in fh if l.startswith("traffic-record:")]
        assert recs and all(r.get("workload") in ("c2", "c3", "c5") and r["kernel"] in bench.KERNEL_SOURCES
                            for r in recs)


def test_step_payload_of_the_batched_and_256cube_workloads():
    """The step payload: 1568 B per sample (gathers, ground truth, scatter adds)
    plus 34 B of Adam traffic per parameter -- 7.35 GB for the 64-block step
    (167.9 M parameters, 2^20 samples), 0.715 GB for the 256^3 step."""
    c3 = {"batch": 1 << 20, "n_params": 64 * (1308419 * 2 + 6208)}
    c2 = {"batch": 1 << 18, "n_params": 4461462 * 2 + 6208}
    assert bench.step_payload_bytes(c3) == pytest.approx(7.35e9, rel=2e-3)
    assert bench.step_payload_bytes(c2) == pytest.approx(0.715e9, rel=2e-3)


def test_leg_records_and_equal_psnr():
    legs = {"mixed": dict(samples_per_s=4e8, psnr=37.0), "fp32_plain": dict(samples_per_s=1e8, psnr=36.8),
            "fp32_same_plan": dict(samples_per_s=2e8, psnr=36.5)}
    base = dict(ms_per_step=1.0, decode_voxels_per_s=1.0, quality_ms_per_step=1.0, phase_ms={}, bins_per_axis=2,
                priv_levels=5, part_levels=5)
    for r in legs.values():
        r.update(base)
    rec = {leg: bench.leg_record(r) for leg, r in legs.items()}
    assert rec["mixed"]["plan"] == {"bins_per_axis": 2, "priv_levels": 5, "part_from_level": 5}
    out = bench.speedups(legs)
    assert out["speedup_vs_fp32_plain"] == pytest.approx(4.0) and out["speedup_vs_fp32_same_plan"] == pytest.approx(2.0)
    assert out["equal_psnr_vs_fp32_plain"] and not out["equal_psnr_vs_fp32_same_plan"]


def test_cpu_baseline_pool_runs_the_oracle():
    """The CPU baseline's worker pool (spawned processes, one block per task) on
    a tiny two-block configuration: samples of the blocks processed, cores and
    host recorded."""
    import numpy as np
    import torch

    from paper_2304_10516_amd.dvnr import EncodingCfg, MlpCfg, OptimCfg
    cfg = dict(enc=EncodingCfg(4, 2, 12, 4, 2.0), mlp=MlpCfg(1, 16), optim=OptimCfg(lr=1e-2), batch=1024)
    blocks = [((12, 10, 9), 1), ((9, 11, 14), 1)]
    rng = np.random.default_rng(0)
    vols = [torch.tensor(rng.random((d[2] + 2, d[1] + 2, d[0] + 2), dtype=np.float32)) for d, _ in blocks]
    r = bench.cpu_baseline(cfg, blocks, vols, max_workers=2)
    assert r["kind"] == "oracle" and r["unit"] == "samples/s" and r["value"] > 0
    assert r["cores"] == 2 and r["nproc"] >= 1 and r["cpu_model"]
    assert "1024 samples" in r["sample"]


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""


def test_phases_against_the_measured_rates_of_their_access_patterns():
    """Encode lookups against random gathers at the smallest measured footprint
    that holds the tables (the 64 MB point for the 17.8 MB fp16 tables of the
    256^3 workload), the MLP against the measured MFMA rate, streaming phases
    against the non-temporal copy."""
    res = _res()
    res["phase_ms"] = {"encode": 0.08, "mlp": 0.064, "part_accum": 0.1, "part_bucket": 0.07, "scatter": 0.0,
                       "sample": 0.04, "adam": 0.01}
    pts = {f"{mb}MB": float(mb) for mb in bench.MICRO_FOOTPRINTS_MB}
    micro = {"copy_nontemporal_gbs": 5000.0, "copy_gbs": 4000.0, "gather_4byte_g_per_s": pts,
             "atomic_fp32_g_per_s": pts, "atomic_fp32_groups_of_4_g_per_s": pts, "mfma_bf16_tflops": 2000.0}
    r = bench.phases_vs_micro("mixed", res, micro)
    table = sum(res["level_entries"]) * 4
    assert r["table_footprint_bytes"] == table and 16 << 20 < table <= 64 << 20 and r["footprint_point"] == "64MB"
    lookups = (1 << 18) * 16 * 8 / 0.08e-3 / 1e9
    assert r["encode"]["g_lookups_per_s"] == pytest.approx(lookups)
    assert r["encode"]["frac"] == pytest.approx(lookups / 64.0)
    assert r["mlp"]["frac"] == pytest.approx(37248.0 * (1 << 18) / 0.064e-3 / 1e12 / 2000.0)
    gbs = bench.phase_bytes("mixed", "part_accum", res) / 0.1e-3 / 1e9
    assert r["part_accum"]["frac"] == pytest.approx(gbs / 5000.0)
    assert "scatter" not in r  # no direct-atomic levels in this plan
    assert bench._footprint_key(1) == "4MB" and bench._footprint_key(1 << 40) == "1024MB"
