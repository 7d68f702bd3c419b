"""Benchmark of the DVNR hot path on one MI355X.

Default workload (the batched configuration the headline metric names): 64
blocks cut from one seeded periodic k^-5/3 field with per-axis extents
U{96..160} and a 1-voxel periodic ghost layer, one INR per block (hash grid
L=16, T=2^17, F=2, base 16, finest 160; MLP 2 hidden layers of 64), L2 loss,
Adam lr 1e-2, 2^20 samples per step apportioned by owned voxel count.
`--workload c2`: one 256^3 block (T=2^19, finest 256, 2^18 samples per step);
`c4`: the warm-started 40-timestep series; `c5`: 512 blocks of 128^3 (2^21
samples per step).

A step is one pass of the whole training path: coordinate sampling and
ground-truth fetch, encoding, MLP forward / loss / backward, encoding
backward, weight-gradient reduction and Adam.  Three legs per workload:

* mixed: fp16 tables, bf16 MFMA MLP, fp32 masters, the default plan (ordered
  sampling, bin-privatized coarse levels, destination-partitioned fine
  levels) -- the headline `value`;
* fp32_plain: the fp32 path with its own defaults (unordered samples,
  one thread per sample and level, plain atomics);
* fp32_same_plan: the fp32 path on the mixed leg's plan (same ordered
  sampling, grouped and privatized scatter, same partitioned levels), so that
  the ratio to it isolates precision.

Per leg: K timed steps (hipGraph replays; inputs resident in HBM), per-phase
device times from a short eager run with HIP events between the phases, and a
quality run: Q steps from the initial parameters with the learning rate
decaying exponentially to 0.1x over the Q steps, then a decode of every block
(voxels/s) and the fp64 PSNR over all owned voxels.  The speedups are quoted
with the PSNR gap of the quality runs ("equal PSNR": within 0.3 dB).  With
the default workload the 256^3 workload is measured as a secondary record.
The float64 CPU oracle is timed on one training step of a subset of the
blocks, over a pool of worker processes (blocks are independent).

Before the workload, the measurement kernels of include/dvnr_micro.h give
the attainable rate of each phase's access pattern (streaming copy, random
gathers and fp32 atomics at several table footprints, bf16 MFMA); the line
reports them under "micro" and each phase's fraction of its own pattern's
rate under roofline.phases_vs_micro (`--no-micro` skips them).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c4|c5]
                       [--quality-steps Q] [--no-secondary] [--no-cpu-baseline] [--no-micro]
                       [--legs mixed,fp32_plain,fp32_same_plan]
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

PEAK_HBM_GBS = 8000.0
L_LEVELS, F_FEAT = 16, 2
ADAM_BYTES_PER_PARAM = {"mixed": 34, "fp32": 32}
# algorithmic payload of one training sample (fp16 tables): 16 levels x 8 corners
# x 4 B gathered, 32 B of ground-truth voxels, 256 fp32 gradient adds of 4 B
PAYLOAD_BYTES_PER_SAMPLE = 512 + 32 + 1024
METRIC = "train samples/s & decode voxels/s at fixed PSNR; BF16 batched vs FP32 plain"
LEGS = ("mixed", "fp32_plain", "fp32_same_plan")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def part_params(res):
    """Table parameters of the destination-partitioned levels (updated by the slice pass)."""
    lf = res["part_levels"]
    return sum(res["level_entries"][lf:]) * F_FEAT * res["n_blocks"] if lf < L_LEVELS else 0


def phase_bytes(precision, phase, res):
    """Algorithmic bytes of one launch of a phase's kernel (None: not a byte-bound phase).

    Per sample (x samples per step), with lp the bin-privatized levels [0, lp),
    lf the first destination-partitioned level and nd = lf - lp direct levels:
    sample       : 3 coords written (12) + 8 voxel reads (32) + target written (4) = 48
    encode       : coords (12) + L levels x 8 corners x F x table element (2 B fp16, 4 B fp32)
                   + L x F features written (2 B bf16, 4 B fp32)
    scatter_priv : coords (12) + lp x F dL/dy reads (4 B) + lp x 8 corners x F fp32 gradient adds (4 B)
    scatter      : the same for the nd direct levels
    part_bucket  : coords (12) + np x F dL/dy reads (4 B) + np x 8 records written, np = L - lf
                   partitioned levels; a record is 8 B for F = 2 (packed), (1 + F) x 4 B otherwise
    part_accum   : np x 8 records read, plus per launch the Adam update of every partitioned
                   table parameter, which the slice pass applies itself: theta, m, v read and
                   written (24 B) and the fp16 working copy written (2 B, mixed precision)
    adam         : the remaining parameters (34 B each mixed, 32 B fp32)
    """
    rec = 8 if F_FEAT == 2 else (1 + F_FEAT) * 4
    te = 2 if precision == "mixed" else 4
    batch = res["batch"]
    lp, lf = res["priv_levels"], res["part_levels"]
    npart = L_LEVELS - lf
    if phase == "sample":
        return 48 * batch
    if phase == "encode":
        return (12 + L_LEVELS * 8 * F_FEAT * te + L_LEVELS * F_FEAT * te) * batch
    if phase in ("scatter_priv", "scatter"):
        nl = lp if phase == "scatter_priv" else lf - lp
        return (12 + nl * F_FEAT * 4 + nl * 8 * F_FEAT * 4) * batch if nl > 0 else 0
    if phase == "part_bucket":
        return (12 + npart * F_FEAT * 4 + npart * 8 * rec) * batch if npart > 0 else 0
    if phase == "part_accum":
        if npart <= 0:
            return 0
        return npart * 8 * rec * batch + part_params(res) * (26 if precision == "mixed" else 24)
    if phase == "adam":
        return ADAM_BYTES_PER_PARAM[precision] * (res["n_params"] - part_params(res))
    return None


def make_workload(name, torch):
    """(config, blocks [(dims, ghost)], device volumes, description)."""
    from paper_2304_10516_amd import presets
    cfg = presets.get(name)
    if name == "c2":
        from fixtures import kolmogorov_field
        log("[bench] generating the 256^3 k^-5/3 field")
        vol = kolmogorov_field(256, seed=2)
        desc = ("single 256^3 block of a seeded k^-5/3 field; hash grid L=16, T=2^19, F=2, base 16, finest 256; "
                "MLP 2x64 ReLU; L2 loss; 2^18 samples per step")
        return cfg, [((256, 256, 256), 0)], [torch.tensor(vol, device="cuda")], desc
    from fixtures import kolmogorov_field_torch, uneven_block_sizes
    if name == "c3":
        sx, sy, sz = uneven_block_sizes(4, 96, 160, seed=3)
        seed = 3
    else:
        sx = sy = sz = np.full(8, 128)
        seed = 5
    nb_axis = len(sx)
    shape = (int(sz.sum()), int(sy.sum()), int(sx.sum()))
    log(f"[bench] generating the {shape} periodic k^-5/3 field on the GPU and cutting {nb_axis ** 3} blocks")
    f = kolmogorov_field_torch(shape, seed=seed)
    fp = torch.nn.functional.pad(f[None, None], (1, 1, 1, 1, 1, 1), mode="circular")[0, 0]
    del f
    ox, oy, oz = [np.concatenate([[0], np.cumsum(s)[:-1]]) for s in (sx, sy, sz)]
    blocks, vols = [], []
    for iz in range(nb_axis):
        for iy in range(nb_axis):
            for ix in range(nb_axis):
                d = (int(sx[ix]), int(sy[iy]), int(sz[iz]))
                z0, y0, x0 = int(oz[iz]), int(oy[iy]), int(ox[ix])
                vols.append(fp[z0:z0 + d[2] + 2, y0:y0 + d[1] + 2, x0:x0 + d[0] + 2].contiguous())
                blocks.append((d, 1))
    del fp
    torch.cuda.empty_cache()
    if name == "c3":
        desc = ("64 blocks, extents U{96..160} per axis, 1-voxel periodic ghost layer, cut from one seeded "
                f"k^-5/3 field of {shape[2]}x{shape[1]}x{shape[0]}; one INR per block: L=16, T=2^17, F=2, base 16, "
                "finest 160, MLP 2x64 ReLU; L2 loss; 2^20 samples per step apportioned by voxel count")
    else:
        desc = ("one GPU's share at scale: 1024^3 seeded k^-5/3 field cut into 512 blocks of 128^3 with a "
                "1-voxel periodic ghost layer; one INR per block: L=16, T=2^19, F=2, base 16, finest 128, MLP 2x64; "
                "2^21 samples per step (4096 per block)")
    return cfg, blocks, vols, desc


def _optim_over(cfg, n_steps):
    """The workload's Adam with the learning rate decaying exponentially to 0.1x
    over n_steps (Sec. III-F names an exponential decay)."""
    import dataclasses
    return dataclasses.replace(cfg["optim"], lr_decay_base=0.1, lr_decay_start=0, lr_decay_interval=max(n_steps, 1))


def run_leg(torch, DVNR, cfg, blocks, vols, leg, steps, warmup, quality_steps, plan=None, seed=3):
    """One leg: timed steps, per-phase times, quality run, decode and PSNR."""
    precision = "mixed" if leg == "mixed" else "fp32"
    batch = cfg["batch"]
    model = DVNR(cfg["enc"], cfg["mlp"], blocks, _optim_over(cfg, quality_steps), precision=precision,
                 max_batch=batch, seed=seed)
    model.bind_volumes(vols)
    if leg == "fp32_same_plan":
        model.set_option("spatial_sort", 1)
        model.set_option("scatter_grouped", 1)
        model.set_option("scatter_part", plan["part_levels"])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        model.init_params(1, stream=stream)
        if warmup:
            model.train(warmup, batch, stream=stream)  # plan, graph capture, clocks
        model.init_params(1, stream=stream)
        stream.synchronize()
        log(f"[bench] {leg}: timing {steps} steps of {batch} samples over {len(blocks)} block(s)")
        t0 = time.perf_counter()
        model.train(steps, batch, stream=stream)  # hipGraph replays
        stream.synchronize()
        t1 = time.perf_counter()
        bins, priv = model.plan_info()
        part = model.partitioned_levels()
        # per-phase device times: a short eager run with HIP events between the
        # phases, the concurrent branches run one after the other (each phase is
        # then one kernel's time)
        model.set_option("profile_phases", 1)
        model.set_option("part_concurrent", 0)
        model.set_option("encode_concurrent", 0)
        model.phase_times()
        model.train(min(max(steps, 10), 50), batch, stream=stream)
        stream.synchronize()
        phases, nsteps = model.phase_times()
        model.set_option("profile_phases", 0)
        model.set_option("part_concurrent", 1)
        model.set_option("encode_concurrent", 1)
        # quality run from the initial parameters
        model.init_params(1, stream=stream)
        stream.synchronize()
        q0 = time.perf_counter()
        loss = model.train(quality_steps, batch, want_loss=True, stream=stream)
        stream.synchronize()
        q_ms = (time.perf_counter() - q0) * 1e3 / max(quality_steps, 1)
        outs = [torch.empty((d[2], d[1], d[0]), dtype=torch.float32, device="cuda") for d, _ in blocks]
        for b in range(len(blocks)):  # warm
            model.decode(b, out=outs[b], stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for b in range(len(blocks)):
            model.decode(b, out=outs[b], stream=stream)
        e1.record(stream)
        stream.synchronize()
        dec_ms = e0.elapsed_time(e1)
        sse, cnt = 0.0, 0
        for b in range(len(blocks)):
            s, c = model.squared_error(b, outs[b], stream=stream)
            sse += s
            cnt += c
        del outs
        render = None
        if len(blocks) == 1 and leg == "mixed":
            # sample-streaming direct volume rendering of the trained block, 1024^2 rays
            lo, hi = model.ranges()
            tf = torch.tensor([[0.05, 0.1, 0.6, 0.0], [0.1, 0.6, 0.7, 0.05], [0.9, 0.8, 0.2, 0.3],
                               [1.0, 0.3, 0.1, 0.8]], dtype=torch.float32)
            kw = dict(eye=(1.6, 1.3, 2.1), center=(0.5, 0.5, 0.5), up=(0.0, 1.0, 0.0), fovy_deg=45.0, tf=tf,
                      tf_range=(lo[0], hi[0]), step=1.0 / 512, ref_step=1.0 / 256, samples_per_round=64,
                      stream=stream)
            model.render(0, width=256, height=256, **kw)  # warm
            r0 = time.perf_counter()
            model.render(0, width=1024, height=1024, **kw)
            r_ms = (time.perf_counter() - r0) * 1e3
            render = {"width": 1024, "height": 1024, "step": 1.0 / 512, "ms": r_ms,
                      "samples": model.last_render_samples,
                      "samples_per_s": model.last_render_samples / (r_ms * 1e-3)}
        model.sync(stream=stream)
    ms = (t1 - t0) * 1e3 / steps
    lossv = loss.float().mean(dim=1).cpu().numpy()
    res = dict(ms_per_step=ms, samples_per_s=batch / (ms * 1e-3), decode_ms=dec_ms,
               decode_voxels_per_s=cnt / (dec_ms * 1e-3), psnr=float(10 * np.log10(cnt / sse)),
               quality_ms_per_step=q_ms, loss_first=float(lossv[0]), loss_last=float(lossv[-1]),
               phase_ms={k: v / max(nsteps, 1) for k, v in phases.items()}, n_params=model.sizes.n_params,
               bins_per_axis=bins, priv_levels=priv, part_levels=part, batch=batch, render=render,
               level_entries=model.level_info()[3], n_blocks=len(blocks))
    log(f"[bench] {leg}: {ms:.3f} ms/step, {res['samples_per_s'] / 1e6:.1f} M samples/s, quality run "
        f"{q_ms:.3f} ms/step, psnr {res['psnr']:.2f} dB after {quality_steps} steps, decode {dec_ms:.2f} ms, "
        f"bins {bins}^3, privatized levels {priv}, partitioned from level {part}, phases " +
        ", ".join(f"{k} {v:.3f}" for k, v in res["phase_ms"].items()))
    del model
    torch.cuda.empty_cache()
    return res


def leg_record(r):
    return {"samples_per_s": r["samples_per_s"], "ms_per_step": r["ms_per_step"],
            "decode_voxels_per_s": r["decode_voxels_per_s"], "psnr_db": r["psnr"],
            "quality_ms_per_step": r["quality_ms_per_step"], "phase_ms": r["phase_ms"],
            "plan": {"bins_per_axis": r["bins_per_axis"], "priv_levels": r["priv_levels"],
                     "part_from_level": r["part_levels"]}}


def run_workload(torch, DVNR, name, legs, steps, warmup, quality_steps):
    cfg, blocks, vols, desc = make_workload(name, torch)
    results = {}
    for leg in legs:
        plan = results.get("mixed")
        if leg == "fp32_same_plan" and plan is None:
            raise ValueError("fp32_same_plan needs the mixed leg first")
        results[leg] = run_leg(torch, DVNR, cfg, blocks, vols, leg, steps, warmup, quality_steps, plan=plan)
    rec = {leg: leg_record(results[leg]) for leg in legs}
    rec.update(speedups(results))
    return cfg, blocks, vols, desc, results, rec


def speedups(results):
    """Mixed-leg throughput over each fp32 leg's, with the PSNR gap of the
    quality runs and whether it is within 0.3 dB (equal PSNR)."""
    out = {}
    if "mixed" in results:
        for leg in ("fp32_plain", "fp32_same_plan"):
            if leg in results:
                gap = results["mixed"]["psnr"] - results[leg]["psnr"]
                out[f"speedup_vs_{leg}"] = results["mixed"]["samples_per_s"] / results[leg]["samples_per_s"]
                out[f"psnr_gap_vs_{leg}_db"] = gap
                out[f"equal_psnr_vs_{leg}"] = bool(abs(gap) <= 0.3)
    return out


PHASE_KERNEL = {"scatter_priv": "k_scatter_priv", "scatter": "k_scatter", "adam": "k_adam", "encode": "k_encode",
                "mlp": "k_mlp_train", "sample": "k_sort_place", "reduce": "k_reduce_slots",
                "part_bucket": "k_part_bucket", "part_accum": "k_part_accum"}
TRAFFIC_FILES = [os.path.join(ROOT, "profiles", f"train_step_{n}_hbm_counters.md") for n in ("64blocks", "256cube")]


KERNEL_SOURCES = {"k_scatter_priv": ["k_sort.hip", "dvnr_device.h", "dvnr_internal.h"],
                  "k_part_bucket": ["k_scatter_part.hip", "dvnr_device.h", "dvnr_internal.h"],
                  "k_part_accum": ["k_scatter_part.hip", "dvnr_device.h", "dvnr_internal.h"],
                  "k_adam": ["k_core.hip", "dvnr_device.h", "dvnr_internal.h"],
                  "k_encode": ["k_core.hip", "dvnr_device.h", "dvnr_internal.h"],
                  "k_mlp_train": ["k_mlp.hip", "dvnr_device.h", "dvnr_internal.h"],
                  "k_sort_place": ["k_sort.hip", "dvnr_device.h", "dvnr_internal.h"]}


def sources_digest(kernel):
    """sha256 over the source files that define `kernel` (names and contents)."""
    import hashlib
    d = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2304_10516_amd", "csrc")
    for name in KERNEL_SOURCES[kernel]:
        d.update(name.encode())
        with open(os.path.join(src, name), "rb") as f:
            d.update(f.read())
    return d.hexdigest()


def measured_traffic(phase, workload):
    """HBM bytes per launch of the phase's kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the summary does not cover it,
    was taken on another workload, or the kernel sources changed since the
    counters were taken."""
    for path in TRAFFIC_FILES:
        try:
            with open(path) as f:
                for line in f:
                    if line.startswith("traffic-record:"):
                        rec = json.loads(line.split(":", 1)[1])
                        if (rec["kernel"] == PHASE_KERNEL.get(phase) and rec["kernel"] in KERNEL_SOURCES
                                and rec.get("workload") == workload
                                and rec["sources_sha256"] == sources_digest(rec["kernel"])):
                            return rec["read_bytes"] + rec["write_bytes"]
        except (OSError, ValueError, KeyError):
            continue
    return None


def roofline_for(precision, res, workload):
    ph = res["phase_ms"]
    dom = max(ph, key=lambda k: ph[k])
    batch = res["batch"]
    if phase_bytes(precision, dom, res) is not None:
        per_launch = phase_bytes(precision, dom, res)
    else:  # mlp: MFMA-bound reading, 37,248 flop per sample
        flops = 37248.0 * batch
        tf = flops / (ph[dom] * 1e-3) / 1e12
        peak = 2500.0 if precision == "mixed" else 157.3
        return {"kernel": PHASE_KERNEL.get(dom, dom), "phase": dom, "bound": "mfma", "achieved": tf, "peak": peak,
                "unit": "TFLOP/s", "frac": tf / peak, "traffic": None}
    gbs = per_launch / (ph[dom] * 1e-3) / 1e9
    # the other byte-bound phases against the same peak
    others = {}
    for k, v in ph.items():
        b = phase_bytes(precision, k, res)
        if k != dom and b and v > 0:
            others[k] = round(b / (v * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    return {"kernel": PHASE_KERNEL.get(dom, dom), "phase": dom, "bound": "hbm", "achieved": gbs,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "traffic": measured_traffic(dom, workload) if precision == "mixed" else None,
            "algorithmic_bytes_per_launch": per_launch, "avg_launch_ms": ph[dom], "other_phases_frac": others}


def run_timeseries(torch, DVNR, cfg, precision, n_timesteps, steps_per_t, seed=3):
    """In situ time series: every timestep of the advected-blob field is compressed by
    training the previous timestep's model for `steps_per_t` steps (weights kept,
    Adam moments and step reset: warm start); reports per-timestep latency."""
    from fixtures import advected_blobs_series_torch
    n = 256
    batch = cfg["batch"]
    series = advected_blobs_series_torch(n, n_timesteps, 16, seed=4)
    vol = next(series).contiguous()
    model = DVNR(cfg["enc"], cfg["mlp"], [((n, n, n), 0)], cfg["optim"], precision=precision, max_batch=batch,
                 seed=seed)
    model.bind_volumes([vol])
    vol_bound = model._vols[0]
    stream = torch.cuda.Stream()
    lat, psnr = [], []
    out = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    with torch.cuda.stream(stream):
        model.init_params(1, stream=stream)
        model.train(5, batch, stream=stream)  # build the plan and the graph
        model.init_params(1, stream=stream)
        stream.synchronize()
        for t in range(n_timesteps):
            if t > 0:
                vol_bound.copy_(next(series))
            stream.synchronize()
            t0 = time.perf_counter()
            model.prepare(stream=stream)
            model.reset_optimizer(stream=stream)
            model.train(steps_per_t, batch, stream=stream)
            stream.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
            model.decode(0, out=out, stream=stream)
            sse, cnt = model.squared_error(0, out, stream=stream)
            psnr.append(float(10 * np.log10(cnt / sse)))
            log(f"[bench] c4 {precision} timestep {t}: {lat[-1]:.1f} ms, psnr {psnr[-1]:.2f} dB")
        model.sync(stream=stream)
    del model
    ms = float(np.mean(lat)) / steps_per_t
    return dict(ms_per_step=ms, samples_per_s=batch / (ms * 1e-3), latency_ms=lat, psnr_per_t=psnr,
                psnr=float(np.mean(psnr)), batch=batch)


MICRO_FOOTPRINTS_MB = (4, 16, 64, 256, 1024)


def micro_rates(torch):
    """Attainable rates of the step's access patterns (include/dvnr_micro.h),
    timed with HIP events on the stream the kernels run on: streaming copy
    (plain and non-temporal), random 4-byte gathers and random fp32 atomic adds
    (scattered and in groups of 4 consecutive lanes) at several table
    footprints, and the dense bf16 MFMA rate."""
    import ctypes as C

    from paper_2304_10516_amd import _lib as L
    lib = L.lib()
    st = torch.cuda.Stream()
    sp = C.c_void_p(st.cuda_stream)

    def timed(launch, reps=5):
        with torch.cuda.stream(st):
            launch()  # warm
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(reps):
                launch()
            e1.record(st)
        st.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    def ok(code):
        if code != 0:
            raise RuntimeError(f"micro kernel returned {code}")

    out = {}
    nbytes = 1 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for nt in (0, 1):
        t = timed(lambda: ok(lib.dvnr_micro_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                                 C.c_int64(nbytes), nt, sp)))
        out["copy_nontemporal_gbs" if nt else "copy_gbs"] = 2 * nbytes / t / 1e9
    del a, b
    n_threads, per = 1 << 21, 64
    res = torch.empty(n_threads, dtype=torch.int32, device="cuda")
    gather, atomic, atomic4 = {}, {}, {}
    for mb in MICRO_FOOTPRINTS_MB:
        n = (mb << 20) // 4
        tab = torch.zeros(n, dtype=torch.float32, device="cuda")
        t = timed(lambda: ok(lib.dvnr_micro_gather(C.c_void_p(tab.data_ptr()), C.c_int64(n), C.c_int64(n_threads),
                                                   per, 12345, C.c_void_p(res.data_ptr()), sp)))
        gather[f"{mb}MB"] = n_threads * per / t / 1e9
        for grp, dst in ((1, atomic), (4, atomic4)):
            t = timed(lambda: ok(lib.dvnr_micro_atomic(C.c_void_p(tab.data_ptr()), C.c_int64(n),
                                                       C.c_int64(n_threads), 16, grp, 777, sp)), reps=3)
            dst[f"{mb}MB"] = n_threads * 16 / t / 1e9
        del tab
    out["gather_4byte_g_per_s"] = gather
    out["atomic_fp32_g_per_s"] = atomic
    out["atomic_fp32_groups_of_4_g_per_s"] = atomic4
    nwg, iters = 4096, 2000
    o = torch.empty(nwg * 256, dtype=torch.float32, device="cuda")
    t = timed(lambda: ok(lib.dvnr_micro_mfma_bf16(C.c_int64(nwg), iters, C.c_void_p(o.data_ptr()), sp)), reps=3)
    out["mfma_bf16_tflops"] = nwg * 4 * iters * 8 * 16384 / t / 1e12
    torch.cuda.empty_cache()
    log("[bench] micro: copy {:.0f} GB/s (non-temporal {:.0f}), gather {} G/s, atomics {} G/s, groups of 4 {} G/s, "
        "bf16 MFMA {:.0f} TFLOP/s".format(out["copy_gbs"], out["copy_nontemporal_gbs"],
                                          {k: round(v, 1) for k, v in gather.items()},
                                          {k: round(v, 1) for k, v in atomic.items()},
                                          {k: round(v, 1) for k, v in atomic4.items()}, out["mfma_bf16_tflops"]))
    return out


def _footprint_key(nbytes):
    """The smallest measured footprint at least as large as nbytes (the largest otherwise)."""
    for mb in MICRO_FOOTPRINTS_MB:
        if nbytes <= mb << 20:
            return f"{mb}MB"
    return f"{MICRO_FOOTPRINTS_MB[-1]}MB"


def phases_vs_micro(precision, res, micro):
    """Each phase's rate against the attainable rate of its own access pattern:
    encode (table lookups, one per corner, level and sample) against random
    4-byte gathers at the step's table footprint; the direct-atomic backward
    (scatter) against random fp32 atomics at that footprint; the MLP against
    the measured bf16 MFMA rate; the streaming phases (sampling, bucketing,
    slice pass, Adam) against the non-temporal copy."""
    ph, batch = res["phase_ms"], res["batch"]
    te = 4 if precision == "mixed" else 8  # bytes per table entry: F = 2 fp16 or fp32 values
    table_bytes = sum(res["level_entries"]) * te * res["n_blocks"]
    key = _footprint_key(table_bytes)
    out = {"table_footprint_bytes": table_bytes, "footprint_point": key}
    if ph.get("encode", 0) > 0:
        rate = batch * L_LEVELS * 8 / (ph["encode"] * 1e-3) / 1e9
        out["encode"] = {"g_lookups_per_s": rate, "micro": micro["gather_4byte_g_per_s"][key],
                         "frac": rate / micro["gather_4byte_g_per_s"][key]}
    nd = res["part_levels"] - res["priv_levels"]
    if ph.get("scatter", 0) > 0.01 and nd > 0:
        rate = batch * nd * 8 * F_FEAT / (ph["scatter"] * 1e-3) / 1e9
        out["scatter"] = {"g_atomics_per_s": rate, "micro": micro["atomic_fp32_g_per_s"][key],
                          "frac": rate / micro["atomic_fp32_g_per_s"][key]}
    if ph.get("mlp", 0) > 0 and precision == "mixed":
        tf = 37248.0 * batch / (ph["mlp"] * 1e-3) / 1e12
        out["mlp"] = {"tflops": tf, "micro": micro["mfma_bf16_tflops"], "frac": tf / micro["mfma_bf16_tflops"]}
    for k in ("sample", "part_bucket", "part_accum", "adam"):
        bts = phase_bytes(precision, k, res)
        if bts and ph.get(k, 0) > 0:
            gbs = bts / (ph[k] * 1e-3) / 1e9
            out[k] = {"gbs": gbs, "micro": micro["copy_nontemporal_gbs"], "frac": gbs / micro["copy_nontemporal_gbs"]}
    return out


def step_payload_bytes(res):
    """Algorithmic HBM payload of one mixed-precision step: the per-sample gather,
    ground-truth and scatter bytes of every sample plus 34 B of Adam traffic per
    parameter."""
    return PAYLOAD_BYTES_PER_SAMPLE * res["batch"] + ADAM_BYTES_PER_PARAM["mixed"] * res["n_params"]


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_block_step(task):
    """One float64 oracle training step of one block (a pool worker, one thread)."""
    path, dims, ghost, n, seed, block, enc, mlp = task
    from threadpoolctl import threadpool_limits

    from fixtures import init_param_draws
    from oracle import dvnr_oracle as o
    vol = np.array(np.load(path, mmap_mode="r"))
    lay = o.layout(o.Encoding(*enc), o.MLP(*mlp))
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=1).astype(np.float64)
    st = o.adam_init(lay.n_params)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        x = o.training_coords(seed, block, 0, n)
        tgt = o.normalized_targets(vol, dims, ghost, x)
        o.train_step(lay, p, st, o.Optim(lr=1e-2), x, tgt)
        return time.perf_counter() - t0


def cpu_baseline(cfg, blocks, vols, max_workers=16):
    """The float64 oracle, untuned, on one training step of the workload's first
    blocks (each with its own apportioned sample count; up to four per worker,
    so the whole 64-block step with 16 workers: about 13 s of compute), one
    block per task over a pool of single-threaded worker processes (at most
    16: the machine's CPU share of one GPU)."""
    import multiprocessing as mp
    import shutil
    import tempfile

    from oracle import dvnr_oracle as o
    nproc = os.cpu_count() or 1
    workers = max(1, min(max_workers, nproc))
    nb = len(blocks)
    n = [cfg["batch"]] if nb == 1 else [int(v) for v in o.apportion([d[0] * d[1] * d[2] for d, _ in blocks],
                                                                       cfg["batch"])]
    k = nb if nb <= 4 * workers else 4 * workers
    enc, mlp = cfg["enc"], cfg["mlp"]
    e = (enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution, enc.per_level_scale,
         enc.finest_resolution)
    tmp = tempfile.mkdtemp(prefix="dvnr_cpu_", dir=os.environ.get("TMPDIR", "/tmp"))
    try:
        tasks = []
        for b in range(k):
            path = os.path.join(tmp, f"b{b}.npy")
            np.save(path, vols[b].cpu().numpy())
            tasks.append((path, blocks[b][0], blocks[b][1], n[b], 3, b, e, (mlp.n_hidden_layers, mlp.width)))
        used = min(workers, k)
        with mp.get_context("spawn").Pool(used) as pool:
            pool.map(_cpu_block_step, tasks[:1])  # workers started and modules imported
            t0 = time.perf_counter()
            per = pool.map(_cpu_block_step, tasks, chunksize=1)
            wall = time.perf_counter() - t0
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    samples = sum(n[:k])
    return {"value": samples / wall, "unit": "samples/s", "cores": used, "kind": "oracle",
            "sample": f"one float64 training step (dense Adam) of {k} of the workload's {nb} block(s), "
                      f"{samples} samples, one block per task over {used} single-threaded worker processes: "
                      f"{wall:.1f} s wall, {sum(per):.1f} s of worker compute",
            "nproc": nproc, "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: 500 for c3, 2000 for c2)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--quality-steps", type=int, default=None,
                    help="steps of each leg's quality run (default: 1000 for c3, 2000 for c2, 300 for c5)")
    ap.add_argument("--timesteps", type=int, default=40, help="c4: timesteps of the series")
    ap.add_argument("--legs", default=",".join(LEGS))
    ap.add_argument("--no-secondary", action="store_true", help="c3: skip the secondary 256^3 record")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-micro", action="store_true", help="skip the measurement kernels (roofline denominators)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB elementwise copy kernel (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the DVNR hot path trains independent per-block models with no "
              "inter-GPU exchange, and this build targets a single MI355X; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    wl = args.workload
    steps = args.steps if args.steps is not None else {"c2": 2000, "c3": 500, "c4": 500, "c5": 50}[wl]
    qsteps = args.quality_steps if args.quality_steps is not None else {"c2": 2000, "c3": 1000, "c5": 300}.get(wl, 0)
    legs = [l for l in args.legs.split(",") if l]
    import torch

    from paper_2304_10516_amd.dvnr import DVNR
    if wl == "c4":
        from paper_2304_10516_amd import presets
        cfg = presets.get("c4")
        precs = ["mixed" if l == "mixed" else "fp32" for l in legs if l in ("mixed", "fp32_plain")]
        res = {p: run_timeseries(torch, DVNR, cfg, p, args.timesteps, steps) for p in precs}
        head_prec = "mixed" if "mixed" in res else next(iter(res))
        head = res[head_prec]
        out = {"metric": METRIC, "value": head["samples_per_s"], "unit": "samples/s", "n_gpus": 1,
               "steps": steps * args.timesteps, "warmup": 5, "ms_per_step": head["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "bf16" if head_prec == "mixed" else "f32", "data": "synthetic",
               "config": {"workload": f"in situ time series: {args.timesteps} timesteps of a 256^3 field of 16 "
                                      "Gaussian blobs advected by a seeded divergence-free flow; per timestep "
                                      f"{steps} warm-started steps of 2^18 samples; 256^3 model",
                          "name": "c4", "timesteps": args.timesteps, "steps_per_timestep": steps},
               "timestep_latency_ms": {p: r["latency_ms"] for p, r in res.items()},
               "psnr_per_timestep_db": {p: r["psnr_per_t"] for p, r in res.items()}}
        print(json.dumps(out), flush=True)
        return
    if args.calibrate_copy:
        a = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)  # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del a, b
    micro = None if args.no_micro else micro_rates(torch)
    cfg, blocks, vols, desc, results, rec = run_workload(torch, DVNR, wl, legs, steps, args.warmup, qsteps)
    head_leg = "mixed" if "mixed" in results else legs[0]
    head = results[head_leg]
    head_prec = "mixed" if head_leg == "mixed" else "fp32"
    roof = roofline_for(head_prec, head, wl)
    if micro:
        roof["phases_vs_micro"] = phases_vs_micro(head_prec, head, micro)
    if head_prec == "mixed":
        pay = step_payload_bytes(head)
        roof["step_payload_bytes"] = pay
        roof["step_frac"] = pay / (head["ms_per_step"] * 1e-3) / 1e9 / PEAK_HBM_GBS
    out = {
        "metric": METRIC,
        "value": head["samples_per_s"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if head_prec == "mixed" else "f32",
        "data": "synthetic",
        "config": {"workload": desc, "name": wl, "blocks": len(blocks), "batch": cfg["batch"], "steps": steps,
                   "precision": head_prec, "quality_steps": qsteps},
        "decode_voxels_per_s": head["decode_voxels_per_s"],
        "psnr_db": head["psnr"],
        "phase_ms": head["phase_ms"],
        "roofline": roof,
    }
    if micro:
        out["micro"] = micro
    if head.get("render"):
        out["render"] = head["render"]
    for leg in legs:
        if leg != head_leg:
            out[leg] = rec[leg]
    for k, v in rec.items():
        if k.startswith(("speedup_", "psnr_gap_", "equal_psnr_")):
            out[k] = v
    if not args.no_cpu_baseline:
        log("[bench] timing the float64 CPU oracle on one training step of a subset of the blocks")
        out["cpu_baseline"] = cpu_baseline(cfg, blocks, vols)
    del vols
    torch.cuda.empty_cache()
    if wl == "c3" and not args.no_secondary:
        log("[bench] secondary record: the 256^3 workload")
        q2 = 2000 if args.quality_steps is None else args.quality_steps
        _, _, v2, d2, r2, rec2 = run_workload(torch, DVNR, "c2", legs, steps, args.warmup, q2)
        sec = {"workload": d2, "quality_steps": q2}
        sec.update(rec2)
        if "mixed" in r2:
            sec["roofline"] = roofline_for("mixed", r2["mixed"], "c2")
            pay = step_payload_bytes(r2["mixed"])
            sec["roofline"]["step_payload_bytes"] = pay
            sec["roofline"]["step_frac"] = pay / (r2["mixed"]["ms_per_step"] * 1e-3) / 1e9 / PEAK_HBM_GBS
            if micro:
                sec["roofline"]["phases_vs_micro"] = phases_vs_micro("mixed", r2["mixed"], micro)
            if r2["mixed"].get("render"):
                sec["render"] = r2["mixed"]["render"]
        out["secondary"] = {"c2": sec}
        del v2
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
