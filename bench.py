"""Benchmark of the DVNR hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): one 256^3
block of a seeded turbulence-like field (random-phase Fourier modes, shell
energy ~ k^-5/3), multiresolution hash grid L=16, T=2^19, F=2, base 16,
finest 256, MLP 2 hidden layers of 64, L2 loss, Adam lr 1e-2, 2^18 samples per
step.  A step is one pass of the whole training path: coordinate sampling and
ground-truth fetch, encoding, MLP forward / loss / backward, encoding
backward, weight-gradient reduction and Adam.

Two runs of K steps each: mixed precision (fp16 tables, bf16 MFMA MLP, fp32
masters) -- the headline `value` -- and the plain fp32 path.  Each run is then
decoded to the full grid (voxels/s) and scored by PSNR with an fp64
reduction.  The float64 CPU oracle is timed on one full training step of the
same workload as the CPU baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BATCH = 1 << 18
N = 256
PEAK_HBM_GBS = 8000.0

# Algorithmic bytes per training sample of each phase (mixed precision; fp32 in brackets):
#   sample : 3 coords written (12) + 8 voxel reads (32) + target written (4)            = 48
#   encode : coords read (12) + 16 levels x 8 corners x F=2 x 2 B [4 B] + 32 feats x 2 B [4 B] written
#   scatter: coords (12) + 32 dX x 4 B read (128) + 16 x 8 x 2 fp32 atomic adds (1024)
PHASE_BYTES = {
    "mixed": {"sample": 48, "encode": 12 + 512 + 64, "scatter": 12 + 128 + 1024},
    "fp32": {"sample": 48, "encode": 12 + 1024 + 128, "scatter": 12 + 128 + 1024},
}
ADAM_BYTES_PER_PARAM = {"mixed": 34, "fp32": 32}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_precision(torch, DVNR, cfg, vol_dev, precision, steps, warmup, seed=3):
    from paper_2304_10516_amd.dvnr import EncodingCfg, MlpCfg, OptimCfg  # noqa: F401
    enc, mlp, optim = cfg["enc"], cfg["mlp"], cfg["optim"]
    model = DVNR(enc, mlp, [((N, N, N), 0)], optim, precision=precision, max_batch=BATCH, seed=seed)
    model.bind_volumes([vol_dev])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        model.init_params(1, stream=stream)
        if warmup:
            model.train(warmup, BATCH, stream=stream)
        model.init_params(1, stream=stream)  # the timed run starts from the initial state
        model.set_option("profile_phases", 1)
        model.phase_times()
        stream.synchronize()
        log(f"[bench] {precision}: timing {steps} steps")
        t0 = time.perf_counter()
        loss = model.train(steps, BATCH, want_loss=True, stream=stream)
        stream.synchronize()
        t1 = time.perf_counter()
        phases, nsteps = model.phase_times()
        model.set_option("profile_phases", 0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        out = torch.empty((N, N, N), dtype=torch.float32, device="cuda")
        model.decode(0, out=out, stream=stream)  # warm
        e0.record(stream)
        model.decode(0, out=out, stream=stream)
        e1.record(stream)
        stream.synchronize()
        dec_ms = e0.elapsed_time(e1)
        sse, cnt = model.squared_error(0, out, stream=stream)
        model.sync(stream=stream)
    ms = (t1 - t0) * 1e3 / steps
    lossv = loss[:, 0].float().cpu().numpy()
    res = dict(ms_per_step=ms, samples_per_s=BATCH / (ms * 1e-3), decode_ms=dec_ms,
               decode_voxels_per_s=N ** 3 / (dec_ms * 1e-3), psnr=float(10 * np.log10(cnt / sse)),
               loss_first=float(lossv[0]), loss_last=float(lossv[-1]),
               phase_ms={k: v / max(nsteps, 1) for k, v in phases.items()}, n_params=model.sizes.n_params)
    log(f"[bench] {precision}: {ms:.3f} ms/step, {res['samples_per_s'] / 1e6:.1f} M samples/s, "
        f"psnr {res['psnr']:.2f} dB, decode {dec_ms:.2f} ms, phases " +
        ", ".join(f"{k} {v:.3f}" for k, v in res["phase_ms"].items()))
    del model
    return res


def roofline_for(precision, res):
    ph = res["phase_ms"]
    dom = max(ph, key=lambda k: ph[k])
    if dom == "adam":
        per_launch = ADAM_BYTES_PER_PARAM[precision] * res["n_params"]
    elif dom in PHASE_BYTES[precision]:
        per_launch = PHASE_BYTES[precision][dom] * BATCH
    else:  # mlp: MFMA-bound reading, 37,248 flop per sample
        flops = 37248.0 * BATCH
        tf = flops / (ph[dom] * 1e-3) / 1e12
        peak = 2500.0 if precision == "mixed" else 157.3
        return {"kernel": dom, "bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s",
                "frac": tf / peak, "traffic": None}
    gbs = per_launch / (ph[dom] * 1e-3) / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs / PEAK_HBM_GBS, "traffic": None, "algorithmic_bytes_per_launch": per_launch,
            "avg_launch_ms": ph[dom]}


def cpu_baseline(cfg, vol):
    """The float64 oracle, untuned, on one full training step of the workload (single thread)."""
    from threadpoolctl import threadpool_limits

    from fixtures import init_param_draws
    from oracle import dvnr_oracle as o
    enc, mlp = cfg["enc"], cfg["mlp"]
    lay = o.layout(o.Encoding(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution,
                              enc.per_level_scale, enc.finest_resolution), o.MLP(mlp.n_hidden_layers, mlp.width))
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=1).astype(np.float64)
    st = o.adam_init(lay.n_params)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        x = o.training_coords(3, 0, 0, BATCH)
        tgt = o.normalized_targets(vol, (N, N, N), 0, x)
        o.train_step(lay, p, st, o.Optim(lr=1e-2), x, tgt)
        dt = time.perf_counter() - t0
    return {"value": BATCH / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"one full training step (2^18 samples, dense Adam over {lay.n_params} params) "
                      f"of the same workload, float64 numpy, 1 thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precisions", default="mixed,fp32")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB elementwise copy kernel (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the DVNR hot path trains independent per-block models with no "
              "inter-GPU exchange, and this build targets a single MI355X; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from fixtures import kolmogorov_field
    from paper_2304_10516_amd import presets
    from paper_2304_10516_amd.dvnr import DVNR
    cfg = presets.get("c2")
    log("[bench] generating the 256^3 k^-5/3 field")
    vol = kolmogorov_field(N, seed=2)
    vol_dev = torch.tensor(vol, device="cuda")
    if args.calibrate_copy:
        a = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)  # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del a, b
    results = {}
    for prec in args.precisions.split(","):
        results[prec] = run_precision(torch, DVNR, cfg, vol_dev, prec, args.steps, args.warmup)
    head = results.get("mixed") or next(iter(results.values()))
    head_prec = "mixed" if "mixed" in results else next(iter(results))
    out = {
        "metric": "train samples/s & decode voxels/s at fixed PSNR; BF16 batched vs FP32 plain",
        "value": head["samples_per_s"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if head_prec == "mixed" else "f32",
        "data": "synthetic",
        "config": {"workload": "single 256^3 block of a seeded k^-5/3 field; hash grid L=16, T=2^19, F=2, "
                               "base 16, finest 256; MLP 2x64 ReLU; L2 loss; Adam lr 1e-2",
                   "batch": BATCH, "steps": args.steps, "precision": head_prec},
        "decode_voxels_per_s": head["decode_voxels_per_s"],
        "psnr_db": head["psnr"],
        "phase_ms": head["phase_ms"],
        "roofline": roofline_for(head_prec, head),
    }
    if "fp32" in results and "mixed" in results:
        f = results["fp32"]
        out["fp32_plain"] = {"samples_per_s": f["samples_per_s"], "ms_per_step": f["ms_per_step"],
                             "decode_voxels_per_s": f["decode_voxels_per_s"], "psnr_db": f["psnr"],
                             "phase_ms": f["phase_ms"]}
        out["speedup_vs_fp32_plain"] = head["samples_per_s"] / f["samples_per_s"]
        out["psnr_gap_db"] = head["psnr"] - f["psnr"]
    if not args.no_cpu_baseline:
        log("[bench] timing the float64 CPU oracle on one full step")
        out["cpu_baseline"] = cpu_baseline(cfg, vol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
