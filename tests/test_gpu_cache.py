"""GPU checks of the sliding-window model cache (temporal caching, Sec. IV;
weight caching, Sec. III-E).

Three timesteps of a two-block model are trained with warm starts and pushed
into a cache of capacity 2.  The cache must drop the oldest timestep, and
decoding or sampling a cached timestep must reproduce, bit for bit, what the
live model returned at that timestep (same parameters, same ranges, same
kernels), also after the live model has moved on.  Live decoding itself is
checked against the oracle in test_gpu_parity.py.
"""
import sys

import numpy as np
import pytest
import torch

from fixtures import gaussian_sum_field, uniform_coords
from oracle import dvnr_oracle as o

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-cache] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision,fused", [("mixed", 1), ("fp32", 0)])
def test_cache_window_and_bit_exact_replay(precision, fused):
    from paper_2304_10516_amd._lib import DvnrError
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    say(f"model cache {precision} decode_fused={fused}")
    blocks = [((24, 20, 16), 1), ((16, 20, 12), 1)]
    model = DVNR(EncodingCfg(6, 2, 14, 4, 1.6), MlpCfg(2, 32), blocks, OptimCfg(lr=1e-2), precision=precision,
                 max_batch=8192, seed=5)
    model.set_option("decode_fused", fused)

    def volumes(t):
        f = gaussian_sum_field(48, n_gauss=10, seed=100 + t)
        return [f[:18, :22, :26], f[20:34, 10:32, 30:48]]

    vols = [torch.as_tensor(np.ascontiguousarray(v), device="cuda") for v in volumes(0)]
    model.bind_volumes(vols)
    bound = model._vols
    model.cache_bind(2)
    x = torch.as_tensor(uniform_coords(3000, seed=3), device="cuda")
    live_dec, live_smp = {}, {}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        model.init_params(2, stream=s)
        for t in range(3):
            if t:
                for dst, v in zip(bound, volumes(t)):
                    dst.copy_(torch.as_tensor(np.ascontiguousarray(v), device="cuda"))
                model.prepare(stream=s)
                model.reset_optimizer(stream=s)
            model.train(40, 4096, stream=s)
            live_dec[t] = [model.decode(b, stream=s).clone() for b in range(2)]
            live_smp[t] = [model.sample(b, x, stream=s).clone() for b in range(2)]
            model.cache_push(t, stream=s)
        model.train(25, 4096, stream=s)  # the live model moves on
    s.synchronize()
    assert model.cache_keys() == [1, 2]
    with torch.cuda.stream(s):
        for t in (1, 2):
            for b in range(2):
                dec = model.cache_decode(t, b, stream=s)
                smp = model.cache_sample(t, b, x, stream=s)
                s.synchronize()
                assert torch.equal(dec, live_dec[t][b]), (t, b)
                assert torch.equal(smp, live_smp[t][b]), (t, b)
        # the snapshots hold different models, and timestep 0 was dropped
        assert not torch.equal(model.cache_decode(1, 0, stream=s), model.cache_decode(2, 0, stream=s))
    with pytest.raises(DvnrError):
        model.cache_decode(0, 0)
    with pytest.raises(DvnrError):
        model.cache_push(2)  # already cached
    # a cached timestep's reconstruction is that of its own field
    vs = volumes(1)
    for b, (d, g) in enumerate(blocks):
        dec = model.cache_decode(1, b).cpu().numpy()
        own = o.psnr(*o.squared_error(dec, vs[b][g:-g, g:-g, g:-g]))
        other = o.psnr(*o.squared_error(dec, volumes(2)[b][g:-g, g:-g, g:-g]))
        say(f"block {b}: cached t=1 vs field t=1 {own:.2f} dB, vs field t=2 {other:.2f} dB")
        assert own > other + 3.0
    model.sync()


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("mixed", 1e-2)])
def test_cached_decode_matches_oracle(precision, tol):
    """A cached timestep decodes as the oracle decodes the parameters that were
    pushed, de-normalized with the value range at push time (the working copy
    for mixed precision: the bf16 MLP output bar), also after the live model
    trained on and its voxels and range changed."""
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    say(f"cached decode vs oracle {precision}")
    enc, mlp = o.Encoding(6, 2, 14, 4, 1.6), o.MLP(2, 32)
    lay = o.layout(enc, mlp)
    dims, g = (24, 20, 16), 1
    model = DVNR(EncodingCfg(6, 2, 14, 4, 1.6), MlpCfg(2, 32), [(dims, g)], OptimCfg(lr=1e-2),
                 precision=precision, max_batch=8192, seed=5)
    f0 = gaussian_sum_field(48, n_gauss=10, seed=200)
    vol = np.ascontiguousarray(f0[:dims[2] + 2 * g, :dims[1] + 2 * g, :dims[0] + 2 * g]) * 3.0 - 1.0
    model.bind_volumes([torch.as_tensor(vol, device="cuda")])
    model.cache_bind(2)
    model.init_params(4)
    model.train(30, 4096)
    model.cache_push(7)
    pushed = model.block_params(0).cpu().numpy().astype(np.float64)
    lo, hi = model.ranges()
    # the live model moves on, on other voxels with another range
    model._vols[0].copy_(torch.as_tensor(vol * 0.5 + 2.0, device="cuda"))
    model.prepare()
    model.train(20, 4096)
    dec = model.cache_decode(7, 0).cpu().numpy()
    pe = pushed
    if precision == "mixed":
        from tests import precision_model as pm
        pe = pm.working_copy(lay, pushed)
    ref = o.decode(lay, pe, dims, lo[0], hi[0])
    err = float(np.max(np.abs(dec - ref)) / np.max(np.abs(ref - lo[0])))
    say(f"cached decode vs oracle: normwise {err:.2e} (range [{lo[0]:.3f}, {hi[0]:.3f}])")
    assert lo[0] < 0.0 < hi[0]
    assert err <= tol
    model.sync()
