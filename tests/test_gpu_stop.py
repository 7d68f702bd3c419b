"""GPU parity of the training-length policy (Sec. III-B) against the oracle.

Three uneven blocks train in one batched call; each stops on its own, either
at its step budget max(N_min, ceil(N_vox / n_b) * N_epoch) or when the moving
average of its loss crosses the threshold at a check.  The oracle trains each
block alone with the same per-block sample count; the stop steps must be
identical and every block's reconstruction within 0.3 dB of the oracle's.
"""
import sys

import numpy as np
import pytest
import torch

from fixtures import gaussian_sum_field, init_param_draws
from oracle import dvnr_oracle as o

pytestmark = pytest.mark.gpu

ENC, MLP = o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16)
SEED, BATCH = 31, 4096


def say(msg):
    print(f"[gpu-stop] {msg}", flush=True)
    sys.stdout.flush()


def _blocks():
    f1 = gaussian_sum_field(48, n_gauss=8, seed=4)
    f2 = gaussian_sum_field(48, n_gauss=24, seed=5)
    vols = [f1[:24, :32, :40], f2[:24, :24, :24], f1[8:20, 10:30, 20:36]]
    dims = [(v.shape[2], v.shape[1], v.shape[0]) for v in vols]
    return [np.ascontiguousarray(v, dtype=np.float32) for v in vols], dims


def _model(dims):
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    e = EncodingCfg(ENC.n_levels, ENC.n_features, ENC.log2_table_size, ENC.base_resolution,
                    ENC.per_level_scale, ENC.finest_resolution)
    return DVNR(e, MlpCfg(MLP.n_hidden_layers, MLP.width), [(d, 0) for d in dims], OptimCfg(lr=1e-2),
                precision="fp32", max_batch=BATCH, seed=SEED)


def _oracle(vols, dims, n, pol, lay, p0):
    out = []
    for b, (v, d) in enumerate(zip(vols, dims)):
        params, losses, steps = o.train_until(lay, p0, v, d, 0, batch=int(n[b]), seed=SEED, opt=o.Optim(lr=1e-2),
                                              pol=pol, block=b)
        vmin, vmax = o.block_value_range(v)
        psnr = o.psnr(*o.squared_error(o.decode(lay, params, d, vmin, vmax), v))
        out.append((steps, losses, psnr))
    return out


def _run_gpu(vols, dims, p0, pol):
    model = _model(dims)
    model.bind_volumes([torch.as_tensor(v, device="cuda") for v in vols])
    model.load_params([p0] * len(vols))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        steps, avg = model.train_until(BATCH, min_steps=pol.min_steps, epochs=pol.epochs,
                                       loss_threshold=pol.loss_threshold, window=pol.window,
                                       check_every=pol.check_every, stream=s)
        psnr = []
        for b in range(len(vols)):
            dec = model.decode(b, stream=s)
            psnr.append(o.psnr(*model.squared_error(b, dec, stream=s)))
    s.synchronize()
    model.sync(stream=s)
    return steps, avg, psnr


def test_step_budget_per_block():
    vols, dims = _blocks()
    lay = o.layout(ENC, MLP)
    p0 = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=1).astype(np.float64)
    n = o.apportion([int(np.prod(d)) for d in dims], BATCH)
    pol = o.StopPolicy(min_steps=0, epochs=20, loss_threshold=0.0)
    want = [o.max_train_steps(int(np.prod(d)), int(n[b]), pol) for b, d in enumerate(dims)]
    say(f"samples per block {list(n)}, budgets {want}")
    assert len(set(want)) > 1  # the blocks stop at different steps
    steps, _, psnr = _run_gpu(vols, dims, p0, pol)
    assert steps == want
    ref = _oracle(vols, dims, n, pol, lay, p0)
    for b in range(3):
        say(f"block {b}: steps {steps[b]}, psnr gpu {psnr[b]:.3f} oracle {ref[b][2]:.3f}")
        assert ref[b][0] == want[b]
        assert abs(psnr[b] - ref[b][2]) <= 0.3


def test_moving_average_early_stop_per_block():
    vols, dims = _blocks()
    lay = o.layout(ENC, MLP)
    p0 = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=1).astype(np.float64)
    n = o.apportion([int(np.prod(d)) for d in dims], BATCH)
    base = o.StopPolicy(min_steps=300, epochs=1, loss_threshold=0.0, window=10, check_every=20)
    full = _oracle(vols, dims, n, base, lay, p0)
    # choose a threshold whose crossings differ per block and whose moving
    # averages at every check stay at least 3 % away from it (a float32 loss
    # cannot flip a decision)
    checks = range(base.check_every, base.min_steps + 1, base.check_every)
    mas = [[o.moving_average(r[1][:k], base.window) for k in checks] for r in full]
    chosen = None
    for thr in np.geomspace(max(m[-1] for m in mas) * 1.05, min(m[0] for m in mas) * 0.95, 60):
        margin = min(abs(v / thr - 1.0) for m in mas for v in m)
        stops = [next((k for k, v in zip(checks, m) if v < thr), base.min_steps) for m in mas]
        if margin > 0.03 and len(set(stops)) >= 2:
            chosen = (thr, stops)
            break
    assert chosen is not None
    thr, stops = chosen
    pol = o.StopPolicy(min_steps=300, epochs=1, loss_threshold=float(thr), window=10, check_every=20)
    say(f"threshold {thr:.4e}: oracle stop steps {stops}")
    steps, avg, psnr = _run_gpu(vols, dims, p0, pol)
    assert steps == stops
    ref = _oracle(vols, dims, n, pol, lay, p0)
    for b in range(3):
        say(f"block {b}: steps {steps[b]}, moving average {avg[b]:.4e}, psnr gpu {psnr[b]:.3f} oracle {ref[b][2]:.3f}")
        assert ref[b][0] == stops[b]
        assert abs(psnr[b] - ref[b][2]) <= 0.3
