"""GPU parity of the HIP path (through the C ABI) against the float64 oracle.

Bars: integer corner indices bit-exact; fp32 results within 1e-5 normwise
(max |gpu - oracle| / max |oracle|); bf16 MLP outputs within 1e-2 normwise;
fp64 building blocks within 1e-10; end-to-end reconstruction PSNR within
0.3 dB of the oracle-trained model on the small 64^3 configuration.
"""
import sys

import numpy as np
import pytest
import torch

from fixtures import adversarial_coords, gaussian_sum_field, init_param_draws, uniform_coords
from oracle import dvnr_oracle as o
from tests import precision_model as pm
from tests.adam_bound import adam_bound, excess_report

pytestmark = pytest.mark.gpu

C1 = (o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16))
C2 = (o.Encoding(16, 2, 19, 16, 0.0, 256), o.MLP(2, 64))
GC = (o.Encoding(3, 2, 6, 2, 2.0), o.MLP(1, 16))


def say(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


def normwise(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def make(cfg, blocks, precision="fp32", max_batch=1 << 14, seed=0):
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    enc, mlp = cfg
    e = EncodingCfg(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution,
                    enc.per_level_scale, enc.finest_resolution)
    return DVNR(e, MlpCfg(mlp.n_hidden_layers, mlp.width), blocks, OptimCfg(lr=1e-2), precision=precision,
                max_batch=max_batch, seed=seed)


def set_waves(model, waves):
    """MLP training kernel variant: 1 or 2 waves per SIMD of the 4-wave kernel,
    or 8, the 8-wave workgroup (the default)."""
    if waves == 8:
        model.set_option("mlp_wg_waves", 8)
    else:
        model.set_option("mlp_wg_waves", 4)
        model.set_option("mlp_waves", waves)


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def check_mixed(gg, gpu_loss, lay, p, x, tgt, label, loss="l2"):
    """Bars of a mixed-precision step (the bf16 tolerance reading of the design
    notes): the oracle evaluates the fp16 / bf16 working copy of `p`; per level
    the GPU gradient stays within 0.1 x the level's intrinsic bf16 error of the
    rounding model and within 1.25 x of the exact gradient; the loss is float32
    arithmetic on the model's values (the fp32 bar, 1e-5)."""
    r = pm.check_mixed_gradient(gg, lay, pm.working_copy(lay, p), x, tgt, loss)
    Lm = r["loss_model"]
    say(f"{label}: following the rounding model per level (x intrinsic): " +
        " ".join(f"{f / max(e, 1e-300):.3f}" for f, e in zip(r["follow"], r["intrinsic"])) +
        f"; weights {r['weights_follow']:.2e} (intrinsic {r['weights_intrinsic']:.2e}); loss {gpu_loss:.7g} vs {Lm:.7g}")
    assert abs(gpu_loss - Lm) <= 1e-5 * Lm, "loss"


# ---------------------------------------------------------------------------
def test_corner_indices_bit_exact_c2():
    say("corner indices C2, 2^20 random + adversarial coordinates")
    lay = o.layout(*C2)
    model = make(C2, [((8, 8, 8), 0)])
    x = np.concatenate([uniform_coords(1 << 20, seed=11), adversarial_coords([l.R for l in lay.levels])])
    xd = dev(x)
    for l, lvl in enumerate(lay.levels):
        idx, w = model.debug_indices(l, xd)
        torch.cuda.synchronize()
        ri, rw = o.corner_indices_and_weights(x, lvl, lay.T)
        gi = idx.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        assert np.array_equal(gi, ri), f"level {l}: {np.sum(gi != ri)} index mismatches"
        assert np.max(np.abs(w.cpu().numpy() - rw)) <= 2e-7, f"level {l} weights"


@pytest.mark.parametrize("cfg_name", ["c1", "c2"])
def test_encode_forward_fp32_and_fp64(cfg_name):
    cfg = {"c1": C1, "c2": C2}[cfg_name]
    say(f"encode forward {cfg_name}")
    lay = o.layout(*cfg)
    rng = np.random.default_rng(3)
    table = rng.normal(size=lay.n_table_params)
    x = np.concatenate([uniform_coords(5000, seed=4), adversarial_coords([l.R for l in lay.levels])])
    ref = o.encode(lay, np.concatenate([table, np.zeros(lay.n_params - lay.n_table_params)]), x)
    for prec, tol in (("fp32", 1e-5), ("fp64", 1e-12)):
        model = make(cfg, [((8, 8, 8), 0)], precision=prec)
        dt = torch.float64 if prec == "fp64" else torch.float32
        y = model.encode_forward(dev(x), dev(table, dt))
        torch.cuda.synchronize()
        assert normwise(y.cpu().numpy(), ref) <= tol, prec


def test_encode_backward_fp64_and_fp32():
    say("encode backward c1")
    lay = o.layout(*C1)
    rng = np.random.default_rng(5)
    x = np.concatenate([uniform_coords(3000, seed=6), adversarial_coords([l.R for l in lay.levels])])
    dy = rng.normal(size=(x.shape[0], lay.in_dim))
    ref = o.encode_backward(lay, x, dy)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-5)):
        model = make(C1, [((8, 8, 8), 0)], precision=prec)
        dt = torch.float64 if prec == "fp64" else torch.float32
        g = torch.zeros(lay.n_table_params, dtype=dt, device="cuda")
        model.encode_backward(dev(x), dev(dy, dt), g)
        torch.cuda.synchronize()
        assert normwise(g.cpu().numpy(), ref) <= tol, prec


def test_empty_and_ragged_inputs():
    say("empty / ragged inputs")
    lay = o.layout(*C1)
    model = make(C1, [((8, 8, 8), 0)])
    table = dev(np.random.default_rng(0).normal(size=lay.n_table_params))
    y = model.encode_forward(torch.empty((0, 3), device="cuda"), table)
    assert y.shape == (0, lay.in_dim)
    for n in (1, 255, 257, 1000):
        x = uniform_coords(n, seed=n)
        y = model.encode_forward(dev(x), table)
        torch.cuda.synchronize()
        ref = o.encode(lay, np.concatenate([table.cpu().numpy(), np.zeros(lay.n_params - lay.n_table_params)]), x)
        assert normwise(y.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("nh,width", [(1, 16), (2, 64), (3, 32)])
def test_mlp_building_blocks_fp64(nh, width):
    say(f"mlp building blocks fp64 nh={nh} w={width}")
    cfg = (o.Encoding(4, 2, 12, 4, 2.0), o.MLP(nh, width))
    lay = o.layout(*cfg)
    rng = np.random.default_rng(nh)
    Ws = [rng.normal(size=s) * 0.5 for s in lay.mlp_shapes]
    wv = np.concatenate([W.ravel() for W in Ws])
    y = rng.normal(size=(777, lay.in_dim))
    do = rng.normal(size=777)
    ref_o, acts = o.mlp_forward(Ws, y)
    ref_dy, ref_dW = o.mlp_backward(Ws, acts, do[:, None])
    model = make(cfg, [((8, 8, 8), 0)], precision="fp64")
    out = model.mlp_forward(dev(y, torch.float64), dev(wv, torch.float64))
    dw = torch.zeros(wv.size, dtype=torch.float64, device="cuda")
    dy = model.mlp_backward(dev(y, torch.float64), dev(wv, torch.float64), dev(do, torch.float64), dw)
    torch.cuda.synchronize()
    assert normwise(out.cpu().numpy(), ref_o[:, 0]) <= 1e-12
    assert normwise(dy.cpu().numpy(), ref_dy) <= 1e-12
    assert normwise(dw.cpu().numpy(), np.concatenate([d.ravel() for d in ref_dW])) <= 1e-12


@pytest.mark.parametrize("dims,ghost", [((16, 16, 16), 0), ((13, 9, 11), 1), ((20, 7, 5), 2)])
def test_training_samples_match_oracle(dims, ghost):
    say(f"training samples dims={dims} ghost={ghost}")
    rng = np.random.default_rng(sum(dims))
    vol = rng.random((dims[2] + 2 * ghost, dims[1] + 2 * ghost, dims[0] + 2 * ghost)).astype(np.float32)
    model = make(C1, [(dims, ghost)], seed=1234)
    model.bind_volumes([dev(vol)])
    for step in (0, 7):
        c, t = model.draw_training_samples(0, step, 3000)
        torch.cuda.synchronize()
        rc = o.training_coords(1234, 0, step, 3000)
        assert np.array_equal(c.cpu().numpy(), rc)
        rt = o.normalized_targets(vol, dims, ghost, rc)
        assert np.max(np.abs(t.cpu().numpy() - rt)) <= 2e-6
    lo, hi = model.ranges()
    assert lo[0] == float(vol.min()) and hi[0] == float(vol.max())


def _setup_c1_block(precision, n=64, seed=0, blocks=None):
    vol = gaussian_sum_field(n, seed=1)
    lay = o.layout(*C1)
    p0 = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=seed)
    model = make(C1, blocks or [((n, n, n), 0)], precision=precision, max_batch=1 << 14, seed=77)
    return vol, lay, p0, model


@pytest.mark.parametrize("precision,grouped,waves", [("fp32", 0, 1), ("fp32", 1, 1), ("mixed", 1, 1),
                                                     ("mixed", 1, 2), ("mixed", 1, 8)])
def test_one_step_gradient_parity_c1(precision, grouped, waves):
    say(f"one-step gradient c1 {precision} grouped={grouped} mlp_waves={waves}")
    vol, lay, p0, model = _setup_c1_block(precision)
    set_waves(model, waves)
    model.bind_volumes([dev(vol)])
    p = p0.astype(np.float64).copy()
    p[:lay.n_table_params] *= 1e3  # table values O(0.1) so that the encoding matters
    model.load_params([p])
    model.set_option("scatter_grouped", grouped)
    model.set_option("apply_update", 0)
    x = o.training_coords(77, 0, 0, 4096)
    loss = model.train_step_coords(dev(x), [4096])
    torch.cuda.synchronize()
    tgt = o.normalized_targets(vol, (64, 64, 64), 0, x)
    gg = model.block_grads(0).cpu().numpy()
    if precision == "mixed":
        check_mixed(gg, loss.item(), lay, p, x, tgt, "c1 one step")
        return
    pref = model.block_params(0).cpu().numpy().astype(np.float64)
    L, g, _ = o.loss_and_grad(lay, pref, x, tgt)
    nt = lay.n_table_params
    assert abs(loss.item() - L) <= 1e-5 * L
    assert normwise(gg[:nt], g[:nt]) <= 1e-5, "table gradient"
    assert normwise(gg[nt:], g[nt:]) <= 1e-5, "weight gradient"


@pytest.mark.parametrize("nh,width", [(1, 16), (3, 32), (2, 64), (3, 64)])
def test_mlp_workgroup_waves_parity(nh, width):
    """The 8-wave MLP training kernel (taken where its LDS fits; the 3 x 64
    network falls back to 4 waves) against the oracle under the bf16 rounding
    model, and against the 4-wave kernel on the same draws: the two differ only
    in the order of the fp32 weight-gradient sums."""
    say(f"mlp 8-wave workgroup parity {nh}x{width}")
    cfg = (C1[0], o.MLP(nh, width))
    vol = gaussian_sum_field(64, seed=1)
    lay = o.layout(*cfg)
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=4).astype(np.float64)
    p[:lay.n_table_params] *= 1e3
    x = o.training_coords(78, 0, 0, 4096)
    grads = {}
    for wg in (4, 8):
        model = make(cfg, [((64, 64, 64), 0)], precision="mixed", max_batch=1 << 14, seed=77)
        model.set_option("mlp_wg_waves", wg)
        model.bind_volumes([dev(vol)])
        model.load_params([p])
        model.set_option("apply_update", 0)
        loss = model.train_step_coords(dev(x), [4096])
        torch.cuda.synchronize()
        grads[wg] = (model.block_grads(0).cpu().numpy().astype(np.float64), loss.item())
        del model
    tgt = o.normalized_targets(vol, (64, 64, 64), 0, x)
    gg, L8 = grads[8]
    check_mixed(gg.astype(np.float32), L8, lay, p, x, tgt, f"mlp {nh}x{width} 8 waves")
    g4, L4 = grads[4]
    assert abs(L8 - L4) <= 1e-6 * abs(L4)
    nt = lay.n_table_params
    assert normwise(gg[:nt], g4[:nt]) <= 1e-5, "table gradient, 8 against 4 waves"
    assert normwise(gg[nt:], g4[nt:]) <= 1e-5, "weight gradient, 8 against 4 waves"


@pytest.mark.parametrize("precision,priv,classes,binned", [("fp32", -1, 0, 1), ("fp32", -1, 1, 1), ("fp32", 0, 0, 0),
                                                           ("mixed", -1, 0, 1), ("mixed", -1, 1, 0),
                                                           ("mixed", 2, 0, 1)])
def test_sorted_sampling_gradient_parity(precision, priv, classes, binned):
    """Spatially ordered sampling stores the same Philox draws grouped by bin; the
    gradient (a sum over samples) must match the oracle's on the unordered draws."""
    say(f"ordered sampling + privatized scatter {precision} priv_levels={priv} LDS classes {classes}")
    vol, lay, p0, model = _setup_c1_block(precision)
    model.bind_volumes([dev(vol)])
    p = p0.astype(np.float64).copy()
    p[:lay.n_table_params] *= 1e3
    model.load_params([p])
    model.set_option("spatial_sort", 1)
    model.set_option("priv_levels", priv)
    model.set_option("priv_classes", classes)
    model.set_option("encode_binned", binned)
    model.set_option("apply_update", 0)
    model.set_option("use_graph", 0)
    loss = model.train(1, 4096, want_loss=True)
    torch.cuda.synchronize()
    x = o.training_coords(77, 0, 0, 4096)
    tgt = o.normalized_targets(vol, (64, 64, 64), 0, x)
    gg = model.block_grads(0).cpu().numpy()
    if precision == "mixed":
        check_mixed(gg, loss[0, 0].item(), lay, p, x, tgt, "c1 ordered")
        return
    pref = model.block_params(0).cpu().numpy().astype(np.float64)
    L, g, _ = o.loss_and_grad(lay, pref, x, tgt)
    nt = lay.n_table_params
    assert abs(loss[0, 0].item() - L) <= 1e-5 * L
    assert normwise(gg[:nt], g[:nt]) <= 1e-5, "table gradient"
    assert normwise(gg[nt:], g[nt:]) <= 1e-5, "weight gradient"


# (precision, LDS classes, MLP waves, concurrent, ordered, scatter_part, bucket cap, slice floats,
#  first partitioned level expected: scatter_part = 0 asks for every level, and every level of this
#  encoding has at least the 2^12 entries a partitioned table needs)
FINE_CASES = [("fp32", 0, 1, 0, 1, -1, 0, 8192, 16), ("fp32", 1, 1, 0, 1, -1, 0, 8192, 16),
              ("fp32", 0, 1, 1, 1, -1, 0, 8192, 16),
              # mixed, automatic: with Adam in the slice pass every level with at
              # least 2^15 entries is partitioned (levels 4..15), however sparse
              ("mixed", 0, 1, 0, 1, -1, 0, 8192, 4), ("mixed", 0, 8, 0, 1, -1, 0, 8192, 4),
              # mixed with every level privatized (the in-kernel direct atomics of
              # the fine levels), two MLP waves per SIMD, LDS classes
              ("mixed", 0, 2, 0, 1, 16, 0, 8192, 16), ("mixed", 1, 1, 1, 1, 16, 0, 8192, 16),
              # destination-partitioned levels: fine only, every eligible one (ordered and not),
              # tiny buckets (most records overflow into direct atomics), other slice sizes
              ("fp32", 0, 1, 0, 1, 9, 0, 8192, 9), ("fp32", 0, 1, 0, 1, 0, 0, 8192, 0),
              ("fp32", 0, 1, 0, 0, 6, 0, 16384, 6), ("fp32", 0, 1, 0, 1, 9, 8, 8192, 9),
              ("fp32", 0, 1, 0, 0, 12, 0, 4096, 12), ("mixed", 0, 1, 0, 1, 9, 0, 8192, 9),
              # 16384 samples, 64 slices per level: 4 sub-buckets per bucket
              ("fp32", 0, 1, 0, 1, 9, 0, 16384, 9, 16384),
              # ragged sample counts: a partial last tile and uneven bins
              ("fp32", 0, 1, 0, 1, 9, 0, 8192, 9, 10000), ("mixed", 0, 1, 0, 1, 4, 0, 8192, 4, 9999),
              ("mixed", 0, 8, 0, 1, 4, 0, 8192, 4, 9999)]
FINE_CASES = [c if len(c) == 10 else c + (8192,) for c in FINE_CASES]


@pytest.mark.parametrize("precision,classes,waves,conc,sort,part,cap,slice_,lf,n", FINE_CASES)
def test_sorted_sampling_gradient_parity_fine_levels(precision, classes, waves, conc, sort, part, cap, slice_, lf, n):
    """16 levels up to R = 256 with 8192 samples (2^3 bins of ~1024): coarse
    levels accumulate in LDS, levels whose bin box exceeds the LDS budget take
    the in-kernel direct-atomic path; bins above 1024 samples take two chunks.
    With lf < 16 the levels [lf, 16) take the destination-partitioned
    backward instead (slice buckets summed in LDS); cap > 0 shrinks its
    buckets to cap records so that most records take the overflow atomics."""
    say(f"c2 levels {precision}: ordered {sort}, LDS classes {classes}, partitioned from level {part}, "
        f"bucket cap {cap}")
    vol = gaussian_sum_field(64, seed=3)
    lay = o.layout(*C2)
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=2).astype(np.float64)
    p[:lay.n_table_params] *= 1e3
    if n > 8192:
        # all parameters positive, so every ReLU unit is active: with random signs and
        # this many samples, some sample's hidden pre-activation lies within fp32
        # rounding of zero, its unit switches between fp32 and fp64 and all its
        # corner entries move by a macroscopic amount
        p = np.abs(p)
    model = make(C2, [((64, 64, 64), 0)], precision=precision, max_batch=1 << 14, seed=91)
    model.bind_volumes([dev(vol)])
    model.load_params([p])
    model.set_option("spatial_sort", sort)
    model.set_option("priv_levels", -1)
    model.set_option("priv_classes", classes)
    set_waves(model, waves)
    model.set_option("scatter_concurrent", conc)
    model.set_option("scatter_part", part)
    model.set_option("part_capacity", cap)
    model.set_option("part_slice", slice_)
    model.set_option("apply_update", 0)
    model.set_option("use_graph", 0)
    loss = model.train(1, n, want_loss=True)
    torch.cuda.synchronize()
    bins = max(B for B in range(1, 9) if B ** 3 * 192 <= n)  # at least 192 samples per bin
    assert model.plan_info() == ((bins, lf) if sort else (0, 0))
    assert model.partitioned_levels() == lf
    x = o.training_coords(91, 0, 0, n)
    tgt = o.normalized_targets(vol, (64, 64, 64), 0, x)
    gg = model.block_grads(0).cpu().numpy()
    if precision == "mixed":
        check_mixed(gg, loss[0, 0].item(), lay, p, x, tgt, f"c2 levels, partitioned from {lf}")
        return
    pref = model.block_params(0).cpu().numpy().astype(np.float64)
    L, g, _ = o.loss_and_grad(lay, pref, x, tgt)
    nt = lay.n_table_params
    assert abs(loss[0, 0].item() - L) <= 1e-5 * L
    for l, lvl in enumerate(lay.levels):
        a, b_ = lvl.off * 2, (lvl.off + lvl.E) * 2
        assert normwise(gg[a:b_], g[a:b_]) <= 1e-5, f"level {l} table gradient"
    assert normwise(gg[nt:], g[nt:]) <= 1e-5, "weight gradient"


# (features, precision, ordered sampling, scatter_part, first partitioned level expected)
WIDTH_CASES = [(1, "fp32", 1, 2, 2), (4, "fp32", 1, 2, 2), (8, "fp32", 1, 2, 2), (4, "fp32", 0, 2, 2),
               (8, "fp32", 1, -1, 4), (1, "mixed", 1, 2, 2), (4, "mixed", 1, 2, 2), (8, "mixed", 1, 2, 2),
               (4, "fp32", 1, 3, 3), (4, "fp32", 1, 0, 0), (1, "mixed", 1, 0, 0)]


@pytest.mark.parametrize("F,precision,sort,part,lf", WIDTH_CASES)
def test_feature_width_gradient_parity(F, precision, sort, part, lf):
    """Feature widths other than 2 (L F <= 32: 8 levels of 1 or 4 features, 4
    levels of 8), base 16, scale 1.5, T = 2^17: levels 0-2 dense (level 2:
    36^3 entries, the first with at least 2^15), 3 and up hashed with 2^17
    entries, so with scatter_part 2 levels 2 and up take the
    destination-partitioned backward (unpacked (1 + F)-word records for
    F != 2), the coarse ones the bin-privatized or plain scatter; scatter_part
    0 partitions every level (each has at least the 2^12 entries a
    partitioned table needs).  One step of 8192 samples against the oracle's
    float64 gradient."""
    L = 4 if F == 8 else 8
    cfg = (o.Encoding(L, F, 17, 16, 1.5), o.MLP(2, 32))
    say(f"feature width {F} ({L} levels) {precision}: ordered {sort}, partitioned from level {part}")
    vol = gaussian_sum_field(64, seed=5)
    lay = o.layout(*cfg)
    assert [lv.E for lv in lay.levels][2:4] == [36 ** 3, 1 << 17]
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=6).astype(np.float64)
    p[:lay.n_table_params] *= 1e3
    model = make(cfg, [((64, 64, 64), 0)], precision=precision, max_batch=1 << 14, seed=17)
    model.bind_volumes([dev(vol)])
    model.load_params([p])
    model.set_option("spatial_sort", sort)
    model.set_option("priv_levels", -1)
    model.set_option("scatter_part", part)
    model.set_option("apply_update", 0)
    model.set_option("use_graph", 0)
    n = 8192
    loss = model.train(1, n, want_loss=True)
    torch.cuda.synchronize()
    assert model.partitioned_levels() == (lf if part >= 0 else L)
    x = o.training_coords(17, 0, 0, n)
    tgt = o.normalized_targets(vol, (64, 64, 64), 0, x)
    gg = model.block_grads(0).cpu().numpy()
    if precision == "mixed":
        check_mixed(gg, loss[0, 0].item(), lay, p, x, tgt, f"F={F}")
        return
    pref = model.block_params(0).cpu().numpy().astype(np.float64)
    Lo, g, _ = o.loss_and_grad(lay, pref, x, tgt)
    nt = lay.n_table_params
    assert abs(loss[0, 0].item() - Lo) <= 1e-5 * Lo
    for l, (a, b_) in enumerate(pm.level_spans(lay)):
        assert normwise(gg[a:b_], g[a:b_]) <= 1e-5, f"level {l} table gradient"
    assert normwise(gg[nt:], g[nt:]) <= 1e-5, "weight gradient"


@pytest.mark.parametrize("empty", [0, 1])
def test_block_without_samples_partitioned_c2(empty):
    """Two c2 blocks, levels 9-15 partitioned with Adam in the slice pass, one
    step on explicit coordinates where one block draws no sample: that block's
    parameters stay bit-identical (neither pass nor the Adam kernel touches
    it), the other takes the oracle's Adam step (bars of the fused-Adam test),
    and every gradient is left at zero."""
    say(f"c2, two blocks, block {empty} without samples, partitioned levels with fused Adam")
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    enc, mlp = C2
    lay = o.layout(*C2)
    vols = [gaussian_sum_field(64, seed=3), gaussian_sum_field(64, seed=4)]
    ps = []
    for seed in (2, 8):
        q = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=seed).astype(np.float64)
        q[:lay.n_table_params] *= 1e3
        ps.append(q)
    model = DVNR(EncodingCfg(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution,
                             enc.per_level_scale, enc.finest_resolution), MlpCfg(mlp.n_hidden_layers, mlp.width),
                 [((64, 64, 64), 0), ((64, 64, 64), 0)], OptimCfg(lr=1e-2), precision="fp32", max_batch=1 << 14,
                 seed=91)
    model.bind_volumes([dev(v) for v in vols])
    model.load_params(ps)
    model.set_option("scatter_part", 9)
    before = [model.block_params(b).clone() for b in range(2)]
    full = 1 - empty
    x = o.training_coords(91, full, 0, 8192)
    counts = [0, 0]
    counts[full] = 8192
    model.train_step_coords(dev(x), counts)
    torch.cuda.synchronize()
    assert model.partitioned_levels() == 9
    assert torch.equal(model.block_params(empty), before[empty])
    pr = before[full].cpu().numpy().astype(np.float64)
    st, opt = o.adam_init(lay.n_params), o.Optim(lr=1e-2)
    _, g, _ = o.loss_and_grad(lay, pr, x, o.normalized_targets(vols[full], (64, 64, 64), 0, x))
    ref, bar = adam_bound(pr, [g], opt)
    got = model.block_params(full).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= bar), excess_report(got, ref, bar, [g])
    assert float(model.grads.abs().max()) == 0.0


def test_phase_times_cover_the_step():
    """dvnr_phase_times: with profile_phases on, every phase of the 16-level
    step (levels 9-15 partitioned) is timed, the sums cover no more than the
    steps' elapsed device time, and a second call finds the sums reset."""
    say("per-phase device times")
    vol = gaussian_sum_field(64, seed=3)
    model = make(C2, [((64, 64, 64), 0)], precision="mixed", max_batch=1 << 14, seed=5)
    model.bind_volumes([dev(vol)])
    model.init_params(1)
    model.set_option("scatter_part", 9)
    model.train(3, 1 << 14)
    model.set_option("profile_phases", 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    model.train(10, 1 << 14)
    e1.record()
    torch.cuda.synchronize()
    ph, n = model.phase_times()
    assert n == 10 and list(ph) == list(model.PHASES)
    assert model.partitioned_levels() == 9
    assert all(v >= 0.0 for v in ph.values())
    for k in ("sample", "encode", "mlp", "scatter_priv", "part_bucket", "part_accum", "reduce", "adam"):
        assert ph[k] > 0.0, k
    assert sum(ph.values()) <= e0.elapsed_time(e1) * 1.05
    ph2, n2 = model.phase_times()
    assert n2 == 0 and all(v == 0.0 for v in ph2.values())


@pytest.mark.parametrize("decay", [False, True])
def test_adam_update_parity_c1(decay):
    say(f"adam update c1 fp32, learning-rate decay {decay}")
    vol, lay, p0, model = _setup_c1_block("fp32")
    if decay:  # exponential decay: lr 1e-2 * 0.5^((t - 1) / 1) from the second update on
        from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
        enc, mlp = C1
        model = DVNR(EncodingCfg(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution,
                                 enc.per_level_scale, enc.finest_resolution),
                     MlpCfg(mlp.n_hidden_layers, mlp.width), [((64, 64, 64), 0)],
                     OptimCfg(lr=1e-2, lr_decay_base=0.5, lr_decay_start=1, lr_decay_interval=1),
                     precision="fp32", max_batch=1 << 14, seed=77)
    model.bind_volumes([dev(vol)])
    p = p0.astype(np.float64)
    model.load_params([p])
    st = o.adam_init(lay.n_params)
    opt = o.Optim(lr=1e-2, lr_decay_base=0.5, lr_decay_start=1, lr_decay_interval=1) if decay else o.Optim(lr=1e-2)
    pr = model.block_params(0).cpu().numpy().astype(np.float64)
    p_start, grads = pr.copy(), []
    for step in range(3):
        x = o.training_coords(77, 0, step, 4096)
        model.train_step_coords(dev(x), [4096])
        tgt = o.normalized_targets(vol, (64, 64, 64), 0, x)
        L, g, _ = o.loss_and_grad(lay, pr, x, tgt)
        grads.append(g)
        pr = o.adam(pr, g, st, opt)
    torch.cuda.synchronize()
    ref, bar = adam_bound(p_start, grads, opt)
    assert np.array_equal(ref, pr)
    got = model.block_params(0).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= bar), excess_report(got, ref, bar, grads)


@pytest.mark.parametrize("decay", [False, True])
def test_adam_fused_in_slice_pass_c2(decay):
    """Levels 9..15 destination-partitioned with the Adam update applied by the
    slice pass (part_adam): three fp32 steps on explicit coordinates against the
    oracle's Adam (same bars as the plain update test), and on the partitioned
    levels after the first step against the separate Adam kernel (the same
    arithmetic on the same fixed-point sums: within 1e-7)."""
    say(f"adam fused into the slice pass, c2 levels fp32, learning-rate decay {decay}")
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    vol = gaussian_sum_field(64, seed=3)
    lay = o.layout(*C2)
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=2).astype(np.float64)
    p[:lay.n_table_params] *= 1e3
    kw = dict(lr=1e-2, lr_decay_base=0.5, lr_decay_start=1, lr_decay_interval=1) if decay else dict(lr=1e-2)
    enc, mlp = C2
    out, first = {}, {}
    for fused in (1, 0):
        model = DVNR(EncodingCfg(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution,
                                 enc.per_level_scale, enc.finest_resolution), MlpCfg(mlp.n_hidden_layers, mlp.width),
                     [((64, 64, 64), 0)], OptimCfg(**kw), precision="fp32", max_batch=1 << 14, seed=91)
        model.bind_volumes([dev(vol)])
        model.load_params([p])
        model.set_option("scatter_part", 9)
        model.set_option("part_adam", fused)
        pr = model.block_params(0).cpu().numpy().astype(np.float64)
        st, opt = o.adam_init(lay.n_params), o.Optim(**kw)
        p_start, grads = pr.copy(), []
        for step in range(3):
            x = o.training_coords(91, 0, step, 8192)
            model.train_step_coords(dev(x), [8192])
            assert model.partitioned_levels() == 9
            if step == 0:
                first[fused] = model.block_params(0).cpu().numpy().astype(np.float64)
            L, g, _ = o.loss_and_grad(lay, pr, x, o.normalized_targets(vol, (64, 64, 64), 0, x))
            grads.append(g)
            pr = o.adam(pr, g, st, opt)
        torch.cuda.synchronize()
        out[fused] = model.block_params(0).cpu().numpy().astype(np.float64)
        ref, bar = adam_bound(p_start, grads, opt)
        assert np.all(np.abs(out[fused] - ref) <= bar), excess_report(out[fused], ref, bar, grads)
        assert float(model.grads.abs().max()) == 0.0  # every gradient is left at zero for the next step
    # after the first step: the partitioned levels' sums are fixed point (order
    # independent), so both ways apply Adam to the same gradient there (later
    # steps differ through the other levels' float atomics, taken in any order)
    a0 = lay.levels[9].off * 2
    assert np.max(np.abs(first[1][a0:lay.n_table_params] - first[0][a0:lay.n_table_params])) <= 1e-7


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("mixed", 1e-2)])
@pytest.mark.parametrize("fused,dims,cfg_name", [(1, (24, 20, 16), "c2"), (0, (24, 20, 16), "c2"),
                                                 (1, (37, 9, 21), "c1")])
def test_decode_and_sample_parity(precision, tol, fused, dims, cfg_name):
    say(f"decode / sample parity {precision} fused={fused} dims={dims} {cfg_name}")
    ghost = 1
    rng = np.random.default_rng(9)
    vol = rng.random((dims[2] + 2, dims[1] + 2, dims[0] + 2)).astype(np.float32)
    cfg = {"c1": C1, "c2": C2}[cfg_name]
    lay = o.layout(*cfg)
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=5).astype(np.float64)
    p[:lay.n_table_params] = rng.normal(size=lay.n_table_params) * 0.5
    model = make(cfg, [(dims, ghost)], precision=precision, max_batch=4096)
    model.bind_volumes([dev(vol)])
    model.load_params([p])
    model.set_option("decode_fused", fused)
    if precision == "mixed":  # the oracle evaluates the rounded working copy
        tab = p[:lay.n_table_params].astype(np.float16).astype(np.float64)
        w = torch.tensor(p[lay.n_table_params:]).to(torch.bfloat16).to(torch.float64).numpy()
        pe = np.concatenate([tab, w])
    else:
        pe = model.block_params(0).cpu().numpy().astype(np.float64)
    vmin, vmax = float(vol.min()), float(vol.max())
    dec = model.decode(0)
    torch.cuda.synchronize()
    ref = o.decode(lay, pe, dims, vmin, vmax)
    assert normwise(dec.cpu().numpy() - vmin, ref - vmin) <= tol
    x = np.concatenate([uniform_coords(3001, seed=2), adversarial_coords([16, 256])])
    s = model.sample(0, dev(x))
    torch.cuda.synchronize()
    rs = o.infer(lay, pe, x) * (vmax - vmin)
    assert normwise(s.cpu().numpy() - vmin, rs) <= tol
    sse, cnt = model.squared_error(0, dec)
    rsse, rcnt = o.squared_error(dec.cpu().numpy(), vol[1:-1, 1:-1, 1:-1])
    assert cnt == rcnt and abs(sse - rsse) <= 1e-9 * rsse


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_c1_end_to_end_psnr_within_03db(precision):
    say(f"c1 end-to-end training {precision}")
    vol, lay, p0, model = _setup_c1_block(precision)
    model.bind_volumes([dev(vol)])
    model.load_params([p0.astype(np.float64)])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        loss = model.train(200, 4096, want_loss=True, stream=s)
        dec = model.decode(0, stream=s)
        sse, cnt = model.squared_error(0, dec, stream=s)
    s.synchronize()
    gpu_psnr = o.psnr(sse, cnt)
    params, losses, _ = o.train(lay, p0, vol, (64, 64, 64), 0, n_steps=200, batch=4096, seed=77, opt=o.Optim(lr=1e-2))
    vmin, vmax = o.block_value_range(vol)
    ref = o.decode(lay, params, (64, 64, 64), vmin, vmax)
    ref_psnr = o.psnr(*o.squared_error(ref, vol))
    say(f"psnr gpu {gpu_psnr:.3f} oracle {ref_psnr:.3f}")
    assert abs(gpu_psnr - ref_psnr) <= 0.3
    lg = loss.cpu().numpy()[:, 0]
    assert np.all(np.isfinite(lg)) and lg[-10:].mean() < lg[:10].mean()
    model.sync(stream=s)


def test_multi_block_isolation():
    say("three uneven blocks: per-block gradients")
    rng = np.random.default_rng(3)
    blocks = [((12, 10, 9), 1), ((7, 15, 8), 1), ((9, 9, 16), 0)]
    vols = [rng.random((d[2] + 2 * g, d[1] + 2 * g, d[0] + 2 * g)).astype(np.float32) for d, g in blocks]
    lay = o.layout(*C1)
    ps = [init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=10 + b).astype(np.float64) * 1.0 for b in range(3)]
    for p in ps:
        p[:lay.n_table_params] *= 1e3
    model = make(C1, blocks, precision="fp32", max_batch=4096, seed=5)
    model.bind_volumes([dev(v) for v in vols])
    model.load_params(ps)
    model.set_option("apply_update", 0)
    n = [300, 700, 257]
    xs = [o.training_coords(5, b, 0, n[b]) for b in range(3)]
    model.train_step_coords(dev(np.concatenate(xs)), n)
    torch.cuda.synchronize()
    for b, ((d, g), v) in enumerate(zip(blocks, vols)):
        tgt = o.normalized_targets(v, d, g, xs[b])
        L, gr, _ = o.loss_and_grad(lay, model.block_params(b).cpu().numpy().astype(np.float64), xs[b], tgt)
        assert normwise(model.block_grads(b).cpu().numpy(), gr) <= 1e-5, b


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_batched_ordered_training_gradients(precision):
    """Several uneven blocks trained in one step through dvnr_train_steps: samples
    apportioned by voxel count, Philox draws per block, ordered sampling with a
    mix of bin-privatized and direct levels; per-block gradients vs the oracle."""
    say(f"batched ordered training gradients {precision}")
    rng = np.random.default_rng(8)
    blocks = [((12, 10, 9), 1), ((7, 15, 8), 1), ((9, 9, 16), 0), ((20, 6, 11), 1)]
    vols = [rng.random((d[2] + 2 * g, d[1] + 2 * g, d[0] + 2 * g)).astype(np.float32) for d, g in blocks]
    lay = o.layout(*C1)
    ps = [init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=20 + b).astype(np.float64) for b in range(4)]
    for p in ps:
        p[:lay.n_table_params] *= 1e3
    model = make(C1, blocks, precision=precision, max_batch=8192, seed=31)
    model.bind_volumes([dev(v) for v in vols])
    model.load_params(ps)
    model.set_option("apply_update", 0)
    model.set_option("spatial_sort", 1)
    model.set_option("priv_levels", 2)
    total = 4096
    loss = model.train(1, total, want_loss=True)
    torch.cuda.synchronize()
    bins, priv = model.plan_info()
    assert bins >= 1 and priv == 2  # both scatter paths are exercised
    n = o.apportion([d[0] * d[1] * d[2] for d, _ in blocks], total)
    for b, ((d, g), v) in enumerate(zip(blocks, vols)):
        x = o.training_coords(31, b, 0, int(n[b]))
        tgt = o.normalized_targets(v, d, g, x)
        if precision == "mixed":
            check_mixed(model.block_grads(b).cpu().numpy(), loss[0, b].item(), lay, ps[b], x, tgt, f"block {b}")
            continue
        L, gr, _ = o.loss_and_grad(lay, model.block_params(b).cpu().numpy().astype(np.float64), x, tgt)
        assert abs(loss[0, b].item() - L) <= 1e-5 * L, b
        assert normwise(model.block_grads(b).cpu().numpy(), gr) <= 1e-5, b


def test_autotune_leaves_state_and_results_unchanged():
    say("autotune: state untouched, gradients still match the oracle")
    vol, lay, p0, model = _setup_c1_block("mixed")
    model.bind_volumes([dev(vol)])
    p = p0.astype(np.float64).copy()
    p[:lay.n_table_params] *= 1e3
    model.load_params([p])
    before = model.params.clone()
    ms = model.autotune(4096, 3)
    torch.cuda.synchronize()
    assert ms > 0
    assert torch.equal(model.params, before)
    assert float(model.grads.abs().max()) == 0.0
    model.set_option("apply_update", 0)
    loss = model.train(1, 4096, want_loss=True)
    torch.cuda.synchronize()
    x = o.training_coords(77, 0, 0, 4096)  # step 0: the tuner restored the step counter
    check_mixed(model.block_grads(0).cpu().numpy(), loss[0, 0].item(), lay, p, x,
                o.normalized_targets(vol, (64, 64, 64), 0, x), "after autotune")


@pytest.mark.parametrize("precision,conc,part", [("fp32", 0, -1), ("mixed", 1, -1), ("mixed", 0, 9)])
def test_graph_replay_matches_eager_steps(precision, conc, part):
    """Steps replayed from the captured hipGraph (with eager work and host syncs
    between replays) follow the same trajectory as eagerly launched steps; with
    conc, the captured step forks part of the backward onto a second stream;
    with part >= 0 (c2 levels), levels [part, 16) take the partitioned
    backward, whose bucket cursors each step leaves at zero for the next."""
    say(f"graph replay vs eager steps {precision} concurrent={conc} partitioned from level {part}")
    vol, lay, p0, _ = _setup_c1_block("fp32")
    cfg = C1
    if part >= 0:
        cfg = C2
        p0 = init_param_draws(o.layout(*C2).n_table_params, o.layout(*C2).mlp_shapes, seed=4)
    losses = {}
    for use_graph in (0, 1):
        model = make(cfg, [((64, 64, 64), 0)], precision=precision, max_batch=1 << 14, seed=77)
        model.bind_volumes([dev(vol)])
        model.load_params([p0.astype(np.float64)])
        model.set_option("scatter_part", part)
        model.set_option("use_graph", use_graph)
        model.set_option("scatter_concurrent", conc)
        s = torch.cuda.Stream()
        out = []
        with torch.cuda.stream(s):
            for _ in range(4):
                out.append(model.train(3, 4096, want_loss=True, stream=s)[:, 0].clone())
                torch.mul(model.params, 1.0)  # unrelated eager work on the stream
                s.synchronize()
        losses[use_graph] = torch.cat(out).cpu().numpy()
        model.sync(stream=s)
        if part >= 0:
            assert model.partitioned_levels() == part
    np.testing.assert_allclose(losses[1], losses[0], rtol=2e-4 if precision == "fp32" else 1e-3, atol=0)


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_sampler_lookahead_draws_the_same_samples(precision):
    """With ordered sampling, replayed steps draw step i + 1's samples on a
    third stream while step i trains (the other of two sample sets).  The
    draws are those of the inline sampler: with explicit per-step sample
    counts of two blocks, the first step's gradient (no update) is the
    oracle's on the Philox draws of that step, and 6 steps in one call, in 6
    calls of one step, and without look-ahead follow the same loss
    trajectory (float atomics' order aside)."""
    say(f"sampler look-ahead {precision}")
    vol = gaussian_sum_field(32, seed=9)
    lay = o.layout(*C1)
    p0 = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=12).astype(np.float64)
    p0[:lay.n_table_params] *= 1e3
    blocks = [((32, 32, 32), 0), ((32, 32, 32), 0)]
    runs = {}
    for name, ahead, calls in (("ahead", 2, 1), ("ahead, one step per call", 2, 6), ("ahead at step start", 1, 1),
                               ("ahead after the MLP", 3, 1), ("inline", 0, 1)):
        model = make(C1, blocks, precision=precision, max_batch=4096, seed=5)
        model.bind_volumes([dev(vol), dev(vol[::-1].copy())])
        model.load_params([p0, p0])
        model.set_option("spatial_sort", 1)
        model.set_option("sample_ahead", ahead)
        s = torch.cuda.Stream()
        out = []
        with torch.cuda.stream(s):
            for _ in range(calls):
                out.append(model.train(6 // calls, 2048, want_loss=True, stream=s).clone())
        s.synchronize()
        runs[name] = torch.cat(out).cpu().numpy()
        model.sync(stream=s)
    tol = 1e-5 if precision == "fp32" else 1e-3
    np.testing.assert_allclose(runs["ahead"], runs["inline"], rtol=tol, atol=0)
    np.testing.assert_allclose(runs["ahead, one step per call"], runs["inline"], rtol=tol, atol=0)
    np.testing.assert_allclose(runs["ahead at step start"], runs["inline"], rtol=tol, atol=0)
    np.testing.assert_allclose(runs["ahead after the MLP"], runs["inline"], rtol=tol, atol=0)
    # the first step's draws are the oracle's (step 0, block b)
    model = make(C1, blocks, precision="fp32", max_batch=4096, seed=5)
    model.bind_volumes([dev(vol), dev(vol)])
    model.load_params([p0, p0])
    model.set_option("spatial_sort", 1)
    model.set_option("apply_update", 0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        loss = model.train(1, 2048, want_loss=True, stream=s)
    s.synchronize()
    n = o.apportion([32 ** 3, 32 ** 3], 2048)
    for b in range(2):
        x = o.training_coords(5, b, 0, int(n[b]))
        L, g, _ = o.loss_and_grad(lay, model.block_params(b).cpu().numpy().astype(np.float64), x,
                                  o.normalized_targets(vol, (32, 32, 32), 0, x))
        assert abs(loss[0, b].item() - L) <= 1e-5 * L
        assert normwise(model.block_grads(b).cpu().numpy(), g) <= 1e-5
    model.sync(stream=s)


def test_nonfinite_loss_is_reported_at_sync():
    """A NaN voxel in the input makes the loss non-finite; the library reports it
    at dvnr_sync (every kernel still runs to completion)."""
    say("non-finite loss reporting")
    from paper_2304_10516_amd._lib import DVNR_E_NONFINITE, DvnrError
    vol = gaussian_sum_field(16, seed=2)
    vol[3] = np.nan  # a NaN plane: many samples interpolate it
    model = make(C1, [((16, 16, 16), 0)], precision="fp32", max_batch=1024, seed=3)
    model.bind_volumes([dev(vol)])
    model.init_params(0)
    model.train(2, 1024)
    with pytest.raises(DvnrError) as ei:
        model.sync()
    assert ei.value.code == DVNR_E_NONFINITE
    model.sync()  # the flag is cleared once reported


def test_gradcheck_fp64_autograd():
    say("fp64 gradcheck of the autograd function on an 8^3 block")
    from paper_2304_10516_amd.autograd import inr
    lay = o.layout(*GC)
    model = make(GC, [((8, 8, 8), 0)], precision="fp64", max_batch=256)
    rng = np.random.default_rng(0)
    x = dev((0.1 + 0.8 * rng.random((32, 3))).astype(np.float32))
    table = torch.tensor(rng.normal(size=lay.n_table_params) * 0.5, dtype=torch.float64, device="cuda",
                         requires_grad=True)
    w = torch.tensor(np.concatenate([rng.normal(size=s).ravel() * 0.5 for s in lay.mlp_shapes]),
                     dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda t, ww: inr(x, t, ww, model), (table, w), eps=1e-6, atol=1e-7, rtol=1e-6)
    # and against the oracle's gradient of sum(out * c)
    cvec = rng.normal(size=32)
    out = inr(x, table, w, model)
    (out * dev(cvec, torch.float64)).sum().backward()
    pv = np.concatenate([table.detach().cpu().numpy(), w.detach().cpu().numpy()])
    xn = x.cpu().numpy()
    y = o.encode(lay, pv, xn)
    Ws = o.mlp_weights(lay, pv)
    oo, acts = o.mlp_forward(Ws, y)
    dy, dWs = o.mlp_backward(Ws, acts, cvec[:, None])
    gt = o.encode_backward(lay, xn, dy)
    assert normwise(table.grad.cpu().numpy(), gt) <= 1e-10
    assert normwise(w.grad.cpu().numpy(), np.concatenate([d.ravel() for d in dWs])) <= 1e-10
    assert normwise(out.detach().cpu().numpy(), oo[:, 0]) <= 1e-12


def test_autograd_training_with_the_fused_adam_step():
    """Training through the autograd function of block 1 of a two-block fp32
    handle, with the library's Adam (dvnr_adam_step) applying the gradients
    copied into the handle's gradient buffer: two steps against the oracle's
    gradient and Adam; block 0, which got no gradient, takes the oracle's
    zero-gradient (weight-decay only) update; the NULL-pointer forms of the
    building blocks address block 1's bound buffers."""
    say("autograd training of block 1 with dvnr_adam_step")
    from paper_2304_10516_amd.autograd import inr
    lay = o.layout(*C1)
    vol = gaussian_sum_field(32, seed=6)
    model = make(C1, [((32, 32, 32), 0), ((32, 32, 32), 0)], precision="fp32", max_batch=4096, seed=3)
    model.bind_volumes([dev(vol), dev(vol)])
    ps = [init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=30 + b).astype(np.float64) for b in range(2)]
    for p in ps:
        p[:lay.n_table_params] *= 1e3
    model.load_params(ps)
    nt = lay.n_table_params
    ref = [model.block_params(b).cpu().numpy().astype(np.float64) for b in range(2)]
    states = [o.adam_init(lay.n_params) for _ in range(2)]
    opt = o.Optim(lr=1e-2)
    p_start, grads = ref[1].copy(), []
    for step in range(2):
        x = o.training_coords(3, 1, step, 2048)
        tgt = o.normalized_targets(vol, (32, 32, 32), 0, x)
        # leaves sharing storage with block 1's parameters
        t = model.block_params(1)[:nt].detach().requires_grad_()
        w = model.block_params(1)[nt:].detach().requires_grad_()
        out = inr(dev(x), t, w, model, 1)
        loss = ((out - dev(tgt)) ** 2).mean()
        loss.backward()
        model.block_grads(1)[:nt].copy_(t.grad)
        model.block_grads(1)[nt:].copy_(w.grad)
        model.adam_step()
        L, g, _ = o.loss_and_grad(lay, ref[1], x, tgt)
        assert abs(loss.item() - L) <= 1e-5 * L
        grads.append(g)
        ref[1] = o.adam(ref[1], g, states[1], opt)
        ref[0] = o.adam(ref[0], np.zeros(lay.n_params), states[0], opt)
    torch.cuda.synchronize()
    exact, bar = adam_bound(p_start, grads, opt)
    assert np.array_equal(exact, ref[1])
    got = model.block_params(1).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref[1]) <= bar), excess_report(got, ref[1], bar, grads)
    d0 = np.abs(model.block_params(0).cpu().numpy().astype(np.float64) - ref[0])
    assert np.max(d0) <= 1e-7
    assert float(model.grads.abs().max()) == 0.0  # the Adam step leaves the gradient at zero
    # NULL-pointer forms: block 1's bound parameters and gradient
    x = dev(o.training_coords(3, 1, 9, 1000))
    tb = model.block_params(1)[:nt].contiguous()
    wb = model.block_params(1)[nt:].contiguous()
    f_explicit = model.encode_forward(x, tb)
    f_bound = model.encode_forward(x, None, block=1)
    assert torch.equal(f_explicit, f_bound)
    assert torch.equal(model.mlp_forward(f_bound, wb), model.mlp_forward(f_bound, None, block=1))
    dfe = torch.ones_like(f_bound)
    g_explicit = torch.zeros(nt, dtype=torch.float32, device="cuda")
    model.encode_backward(x, dfe, g_explicit)
    model.encode_backward(x, dfe, None, block=1)
    torch.cuda.synchronize()
    assert float(model.block_grads(0).abs().max()) == 0.0
    np.testing.assert_allclose(model.block_grads(1)[:nt].cpu().numpy(), g_explicit.cpu().numpy(), rtol=1e-6,
                               atol=1e-6 * float(g_explicit.abs().max()))


def test_adam_step_refreshes_the_working_copy():
    """Mixed precision: after dvnr_adam_step the fp16 table / bf16 weight working
    copy is the round-to-nearest copy of the updated fp32 masters."""
    say("dvnr_adam_step on a mixed handle: working copy refreshed")
    lay = o.layout(*C1)
    vol = gaussian_sum_field(16, seed=2)
    model = make(C1, [((16, 16, 16), 0)], precision="mixed", max_batch=1024, seed=3)
    model.bind_volumes([dev(vol)])
    model.init_params(5)
    rng = np.random.default_rng(2)
    model.block_grads(0).copy_(dev(rng.normal(size=lay.n_params)))
    model.adam_step()
    torch.cuda.synchronize()
    p = model.block_params(0)
    nt = lay.n_table_params
    w16 = model.work16[:lay.n_params]
    assert torch.equal(w16[:nt], p[:nt].to(torch.float16).view(torch.int16))
    assert torch.equal(w16[nt:], p[nt:].to(torch.bfloat16).view(torch.int16))
    assert float(model.grads.abs().max()) == 0.0
