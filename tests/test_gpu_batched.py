"""GPU parity of the batched training plan at the shapes of the batched
workloads (one INR per partition, trained independently: Sec. III-A).

* 64-block workload's shape: 8 uneven blocks (extents U{96..160} per axis, a
  2x2x2 rectilinear cut of one periodic k^-5/3 field, 1-voxel periodic ghost
  layer), per block L=16, T=2^17, F=2, base 16, finest 160, MLP 2x64; 2^17
  samples per step apportioned by voxel count (about 2^14 per block, as in the
  2^20-sample, 64-block step).  One step through dvnr_train_steps with the
  default plan: ordered sampling, levels 0-4 bin-privatized, levels 5-15
  (the ones with at least 2^15 entries that receive a contribution per entry
  per step) destination-partitioned.  Per block, loss and gradient against the
  oracle on the block's own Philox draws: fp32 within 1e-5 (positive
  parameters, so that no ReLU unit sits at its kink), mixed precision with the
  bf16 bars (random signs).  Isolation: a block trained alone, on the same
  coordinates, gets the gradient it gets inside the batch.
* 512-block workload's shape, a subset: 8 blocks of 128^3 with a 1-voxel
  periodic ghost layer (a 2x2x2 cut of a 256^3 periodic k^-5/3 field), per
  block L=16, T=2^19, F=2, base 16, finest 128; 4096 samples per block (2^21
  over 512 blocks); one step of the default plan against the oracle.
"""
import sys

import numpy as np
import pytest
import torch

from fixtures import cut_blocks, init_param_draws, kolmogorov_field, uneven_block_sizes
from oracle import dvnr_oracle as o
from tests import precision_model as pm

pytestmark = pytest.mark.gpu

C3 = (o.Encoding(16, 2, 17, 16, 0.0, 160), o.MLP(2, 64))
C5 = (o.Encoding(16, 2, 19, 16, 0.0, 128), o.MLP(2, 64))


def say(msg):
    print(f"[gpu-batched] {msg}", flush=True)
    sys.stdout.flush()


def normwise(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _model(cfg, blocks, precision, max_batch, seed):
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    enc, mlp = cfg
    e = EncodingCfg(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution, enc.per_level_scale,
                    enc.finest_resolution)
    return DVNR(e, MlpCfg(mlp.n_hidden_layers, mlp.width), blocks, OptimCfg(lr=1e-2), precision=precision,
                max_batch=max_batch, seed=seed)


@pytest.fixture(scope="module")
def c3_blocks():
    sx, sy, sz = uneven_block_sizes(2, 96, 160, seed=3)
    field = kolmogorov_field(seed=3, shape=(int(sz.sum()), int(sy.sum()), int(sx.sum())))
    return cut_blocks(field, (sx, sy, sz), ghost=1, periodic=True)


@pytest.fixture(scope="module")
def c5_blocks():
    field = kolmogorov_field(256, seed=5)
    return cut_blocks(field, ([128, 128], [128, 128], [128, 128]), ghost=1, periodic=True)


def _params(lay, nb, seed, positive):
    ps = []
    for b in range(nb):
        p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=seed + b).astype(np.float64)
        p[:lay.n_table_params] *= 1e3  # table values O(0.1): the encoding matters
        ps.append(np.abs(p) if positive else p)
    return ps


def _check_blocks(lay, model, ps, loss, blks, precision, total, seed, label):
    n = o.apportion([int(np.prod(b["dims"])) for b in blks], total)
    worst = 0.0
    for b, blk in enumerate(blks):
        x = o.training_coords(seed, b, 0, int(n[b]))
        tgt = o.normalized_targets(blk["data"], blk["dims"], blk["ghost"], x)
        gg = model.block_grads(b).cpu().numpy()
        if precision == "mixed":
            r = pm.check_mixed_gradient(gg, lay, pm.working_copy(lay, ps[b]), x, tgt)
            fol = max(f / e for f, e in zip(r["follow"], r["intrinsic"]))
            say(f"{label} block {b} ({n[b]} samples): largest follow/intrinsic {fol:.3f}, "
                f"{r['near_kink']} units near the kink, loss {loss[b]:.7g} vs model {r['loss_model']:.7g}")
            assert abs(loss[b] - r["loss_model"]) <= 1e-5 * r["loss_model"], b
            continue
        L, g, _ = o.loss_and_grad(lay, model.block_params(b).cpu().numpy().astype(np.float64), x, tgt)
        assert abs(loss[b] - L) <= 1e-5 * L, b
        errs = [normwise(gg[a:c], g[a:c]) for a, c in pm.level_spans(lay)]
        werr = normwise(gg[lay.n_table_params:], g[lay.n_table_params:])
        worst = max(worst, max(errs), werr)
        assert max(errs) <= 1e-5 and werr <= 1e-5, (b, errs, werr)
    if precision == "fp32":
        say(f"{label}: largest per-level normwise error over blocks {worst:.2e}")
    return n


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_batched_default_plan_64_block_shape(c3_blocks, precision):
    total, seed = 8 * 16384, 31
    lay = o.layout(*C3)
    blocks = [(b["dims"], b["ghost"]) for b in c3_blocks]
    say(f"8 uneven blocks {[b[0] for b in blocks]}, {total} samples, {precision}")
    model = _model(C3, blocks, precision, total, seed)
    model.bind_volumes([torch.as_tensor(b["data"], device="cuda") for b in c3_blocks])
    ps = _params(lay, len(blocks), 40, positive=precision == "fp32")
    model.load_params(ps)
    if precision == "fp32":  # the fp32 path on the mixed path's plan (its own defaults differ)
        model.set_option("spatial_sort", 1)
        model.set_option("scatter_grouped", 1)
        model.set_option("scatter_part", 5)
    model.set_option("apply_update", 0)
    loss = model.train(1, total, want_loss=True)
    torch.cuda.synchronize()
    bins, priv = model.plan_info()
    lf = model.partitioned_levels()
    say(f"plan: {bins}^3 bins, privatized levels [0, {priv}), partitioned [{lf}, 16)")
    assert lf == 5 and priv == 5 and bins >= 2
    _check_blocks(lay, model, ps, loss.cpu().numpy()[0], c3_blocks, precision, total, seed, "c3 shape")


def test_block_alone_matches_block_in_batch(c3_blocks):
    """Isolation (Sec. III-A: no block sees another's data or parameters): block
    5 trained alone on the coordinates it drew inside the batch gets the same
    loss and gradient (fp32; different plans sum in different orders)."""
    total, seed, k = 8 * 16384, 31, 5
    lay = o.layout(*C3)
    blocks = [(b["dims"], b["ghost"]) for b in c3_blocks]
    ps = _params(lay, len(c3_blocks), 40, True)
    batched = _model(C3, blocks, "fp32", total, seed)
    batched.bind_volumes([torch.as_tensor(b["data"], device="cuda") for b in c3_blocks])
    batched.load_params(ps)
    batched.set_option("spatial_sort", 1)
    batched.set_option("scatter_part", 5)
    batched.set_option("apply_update", 0)
    lb = batched.train(1, total, want_loss=True)[0, k].item()
    n = o.apportion([int(np.prod(b["dims"])) for b in c3_blocks], total)
    x = o.training_coords(seed, k, 0, int(n[k]))
    alone = _model(C3, [blocks[k]], "fp32", int(n[k]), 7)
    alone.bind_volumes([torch.as_tensor(c3_blocks[k]["data"], device="cuda")])
    alone.load_params([ps[k]])
    alone.set_option("scatter_part", 5)
    alone.set_option("apply_update", 0)
    la = alone.train_step_coords(torch.as_tensor(x, device="cuda"), [int(n[k])])[0].item()
    torch.cuda.synchronize()
    assert alone.partitioned_levels() == 5
    ga = alone.block_grads(0).cpu().numpy()
    gb = batched.block_grads(k).cpu().numpy()
    say(f"block {k} alone vs in batch: loss {la:.7g} / {lb:.7g}, gradient normwise {normwise(ga, gb):.2e}")
    assert abs(la - lb) <= 1e-5 * lb
    for a, c in pm.level_spans(lay):
        assert normwise(ga[a:c], gb[a:c]) <= 1e-5
    assert normwise(ga[lay.n_table_params:], gb[lay.n_table_params:]) <= 1e-5
    # and the other blocks' gradients are their own (none is zero, none equals block k's)
    for b in range(len(blocks)):
        if b != k:
            assert float(batched.block_grads(b).abs().max()) > 0.0


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_batched_default_plan_512_block_subset(c5_blocks, precision):
    total, seed = 8 * 4096, 17
    say(f"8 blocks of 128^3, {total} samples, {precision}")
    lay = o.layout(*C5)
    blocks = [(b["dims"], b["ghost"]) for b in c5_blocks]
    model = _model(C5, blocks, precision, total, seed)
    model.bind_volumes([torch.as_tensor(b["data"], device="cuda") for b in c5_blocks])
    ps = _params(lay, len(c5_blocks), 60, precision == "fp32")
    model.load_params(ps)
    if precision == "fp32":
        model.set_option("spatial_sort", 1)
        model.set_option("scatter_grouped", 1)
    model.set_option("apply_update", 0)
    loss = model.train(1, total, want_loss=True)
    torch.cuda.synchronize()
    bins, priv = model.plan_info()
    say(f"plan: {bins}^3 bins, privatized levels [0, {priv}), partitioned from {model.partitioned_levels()}")
    _check_blocks(lay, model, ps, loss.cpu().numpy()[0], c5_blocks, precision, total, seed, "c5 subset")


def test_working_copy_is_rounded_master(c3_blocks):
    """Mixed precision keeps a 16-bit working copy of every parameter: after
    training steps (default plan: Adam in the slice pass for levels 5-15, the
    Adam kernel for the rest) each table entry of the copy is the fp16
    rounding (to nearest even) of the stored fp32 parameter and each MLP
    weight its bf16 rounding, bit for bit, also where the fp32 value is a tie
    between two 16-bit neighbours."""
    total, seed = 8 * 16384, 35
    lay = o.layout(*C3)
    blocks = [(b["dims"], b["ghost"]) for b in c3_blocks]
    model = _model(C3, blocks, "mixed", total, seed)
    model.bind_volumes([torch.as_tensor(b["data"], device="cuda") for b in c3_blocks])
    model.load_params(_params(lay, len(blocks), 70, positive=False))
    model.train(3, total)
    torch.cuda.synchronize()
    assert model.partitioned_levels() == 5
    S, nt = model.block_stride, lay.n_table_params
    nm = lay.n_params - nt
    bad = 0
    for b in range(len(blocks)):
        p = model.params[b * S:b * S + nt + nm]
        w = model.work16[b * S:b * S + nt + nm]
        bad += int((w[:nt] != p[:nt].half().view(torch.int16)).sum())
        bad += int((w[nt:] != p[nt:].bfloat16().view(torch.int16)).sum())
    say(f"working copy against the rounded master parameters: {bad} mismatches")
    assert bad == 0
