"""GPU parity of warm-started training against the oracle (weight caching,
Sec. III-E: the next timestep's network starts from the previous one's
weights; temporal caching, Sec. IV-B).

The reading of a warm start: the parameters are kept, the Adam moments and
the step counter are reset (so the next update is t = 1 with fresh bias
corrections, and the Philox draws restart at step 0).  A 64^3 block of the
advected-blob time series is trained for 60 steps on timestep 0; the volume
is then replaced by timestep 1 in place, the value range recomputed and the
optimizer reset.  Checked against the oracle started from the GPU's
parameters with a fresh Adam state: the first step's gradient (fp32, 1e-5),
the first update (the bars of the plain Adam test) and, after 100
warm-started steps, the reconstruction PSNR (0.3 dB; mixed precision on a
field that keeps the model away from its bf16 floor).
"""
import sys

import numpy as np
import pytest
import torch

from fixtures import advected_blobs_field, init_param_draws, kolmogorov_field
from oracle import dvnr_oracle as o
from tests import precision_model as pm
from tests.adam_bound import adam_bound, excess_report

pytestmark = pytest.mark.gpu

C1 = (o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16))
N, BATCH, SEED = 64, 4096, 23


def say(msg):
    print(f"[gpu-warmstart] {msg}", flush=True)
    sys.stdout.flush()


def normwise(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def series():
    return [advected_blobs_field(N, n_steps=2, n_blobs=6, seed=4, step=t) for t in range(2)]


def _trained_on_t0(precision, series):
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    enc, mlp = C1
    model = DVNR(EncodingCfg(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution,
                             enc.per_level_scale), MlpCfg(mlp.n_hidden_layers, mlp.width), [((N, N, N), 0)],
                 OptimCfg(lr=1e-2), precision=precision, max_batch=BATCH, seed=SEED)
    model.bind_volumes([torch.as_tensor(series[0], device="cuda")])
    lay = o.layout(*C1)
    model.load_params([init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=3).astype(np.float64)])
    model.train(60, BATCH)
    # timestep 1 replaces the voxels in place; ranges recomputed; optimizer reset
    model._vols[0].copy_(torch.as_tensor(series[1], device="cuda"))
    model.prepare()
    model.reset_optimizer()
    torch.cuda.synchronize()
    return model, lay


def test_warm_start_first_gradient_and_update(series):
    say("warm start fp32: first gradient and first update after the reset")
    model, lay = _trained_on_t0("fp32", series)
    p1 = model.block_params(0).cpu().numpy().astype(np.float64)
    vol1 = series[1]
    x = o.training_coords(SEED, 0, 0, BATCH)  # the Philox step restarts at 0
    tgt = o.normalized_targets(vol1, (N, N, N), 0, x)
    lo, hi = model.ranges()
    assert (lo[0], hi[0]) == (float(vol1.min()), float(vol1.max()))
    model.set_option("apply_update", 0)
    loss = model.train(1, BATCH, want_loss=True)
    torch.cuda.synchronize()
    L, g, _ = o.loss_and_grad(lay, p1, x, tgt)
    assert abs(loss[0, 0].item() - L) <= 1e-5 * L
    assert normwise(model.block_grads(0).cpu().numpy(), g) <= 1e-5
    # the first update after the reset: fresh moments, t = 1
    model.set_option("apply_update", 1)
    model.reset_optimizer()
    model.train(1, BATCH)
    torch.cuda.synchronize()
    ref, bar = adam_bound(p1, [g], o.Optim(lr=1e-2))
    got = model.block_params(0).cpu().numpy().astype(np.float64)
    say(f"first warm update: largest distance {np.abs(got - ref).max():.2e}")
    assert np.all(np.abs(got - ref) <= bar), excess_report(got, ref, bar, [g])
    small = np.abs(g) < 1e-5 * np.abs(g).max()
    # the t = 1 update moves every well-conditioned entry by about lr (Adam's first step)
    assert np.median(np.abs(ref - p1)[~small]) > 0.5e-2


def test_warm_started_psnr_within_03db_fp32(series):
    say("warm-started training fp32: 100 steps on timestep 1")
    model, lay = _trained_on_t0("fp32", series)
    p1 = model.block_params(0).cpu().numpy().astype(np.float64)
    gpu_psnr = _warm_psnr(model)
    vol1 = series[1]
    params, losses, _ = o.train(lay, p1, vol1, (N, N, N), 0, n_steps=100, batch=BATCH, seed=SEED,
                                opt=o.Optim(lr=1e-2))
    vmin, vmax = o.block_value_range(vol1)
    ref_psnr = o.psnr(*o.squared_error(o.decode(lay, params, (N, N, N), vmin, vmax), vol1))
    cold = o.psnr(*o.squared_error(o.decode(lay, p1, (N, N, N), vmin, vmax), vol1))
    say(f"psnr gpu {gpu_psnr:.3f} oracle {ref_psnr:.3f} (timestep-0 model on timestep 1: {cold:.3f})")
    assert abs(gpu_psnr - ref_psnr) <= 0.3
    assert ref_psnr > cold  # the warm-started run improved on the cached weights
    model.sync()


def _warm_psnr(model):
    model.train(100, BATCH)
    dec = model.decode(0)
    sse, cnt = model.squared_error(0, dec)
    torch.cuda.synchronize()
    return o.psnr(sse, cnt)


def test_warm_started_psnr_within_03db_mixed():
    """Mixed precision on the blob series ends near 61 dB, at the bf16 floor of
    this small model: there the final error is set by rounding noise, and
    trajectories that differ by float32 rounding end up to 0.4 dB apart, in
    the oracle run under the mixed path's rounding model
    (tests/precision_model.py) as on the GPU.  The mixed check therefore uses a
    field the model cannot fit to that floor: a 64^3 k^-5/3 field and the same
    field advected by one voxel along x (periodic), where warm-started
    training goes from about 24 to 26 dB and both the fp64 oracle and the
    rounding model end within 0.001 dB of themselves under such
    perturbations.  The GPU's PSNR after 100 warm-started steps must lie within
    0.3 dB of the fp64 oracle's and of the rounding model's from the same start."""
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    say("warm-started training mixed: k^-5/3 field advected by one voxel")
    f = kolmogorov_field(N, seed=7)
    pair = [f, np.roll(f, 1, axis=2)]
    enc, mlp = C1
    lay = o.layout(*C1)
    model = DVNR(EncodingCfg(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution,
                             enc.per_level_scale), MlpCfg(mlp.n_hidden_layers, mlp.width), [((N, N, N), 0)],
                 OptimCfg(lr=1e-2), precision="mixed", max_batch=BATCH, seed=SEED)
    model.bind_volumes([torch.as_tensor(pair[0], device="cuda")])
    model.load_params([init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=3).astype(np.float64)])
    model.train(60, BATCH)
    model._vols[0].copy_(torch.as_tensor(pair[1], device="cuda"))
    model.prepare()
    model.reset_optimizer()
    p1 = model.block_params(0).cpu().numpy().astype(np.float64)
    gpu_psnr = _warm_psnr(model)
    model.sync()
    vol1 = pair[1]
    vmin, vmax = o.block_value_range(vol1)
    params, _, _ = o.train(lay, p1, vol1, (N, N, N), 0, n_steps=100, batch=BATCH, seed=SEED, opt=o.Optim(lr=1e-2))
    ref = o.psnr(*o.squared_error(o.decode(lay, params, (N, N, N), vmin, vmax), vol1))
    pmix = pm.train(lay, p1, vol1, (N, N, N), 0, 100, BATCH, SEED, o.Optim(lr=1e-2))
    ref_mixed = o.psnr(*o.squared_error(pm.decode(lay, pmix, (N, N, N), vmin, vmax), vol1))
    cold = o.psnr(*o.squared_error(pm.decode(lay, p1, (N, N, N), vmin, vmax), vol1))
    say(f"psnr gpu {gpu_psnr:.3f} oracle {ref:.3f} rounding model {ref_mixed:.3f} (start on the new field: {cold:.3f})")
    assert abs(gpu_psnr - ref) <= 0.3 and abs(gpu_psnr - ref_mixed) <= 0.3
    assert gpu_psnr > cold + 1.0
