"""dvnr_render_static (rendering with the library's static per-GPU scratch
instead of a caller workspace) against dvnr_render on the same model: the
same kernels on the same inputs, so the images must be identical, on two calls
in a row (the second with a smaller image, so that it runs over the state the
first one left in the shared array)."""
import sys

import numpy as np
import pytest
import torch

from fixtures import gaussian_sum_field, init_param_draws
from oracle import dvnr_oracle as o

pytestmark = pytest.mark.gpu

ENC, MLP = o.Encoding(5, 2, 12, 4, 2.0), o.MLP(2, 32)
TF = np.array([[0.1, 0.2, 0.9, 0.0], [0.2, 0.8, 0.3, 0.2], [0.9, 0.7, 0.1, 0.5], [1.0, 0.2, 0.1, 0.9]])


def say(msg):
    print(f"[gpu-no-alloc] {msg}", flush=True)
    sys.stdout.flush()


def _model(precision):
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    e = EncodingCfg(ENC.n_levels, ENC.n_features, ENC.log2_table_size, ENC.base_resolution,
                    ENC.per_level_scale, ENC.finest_resolution)
    vol = gaussian_sum_field(24, seed=8)
    model = DVNR(e, MlpCfg(MLP.n_hidden_layers, MLP.width), [((24, 24, 24), 0)], OptimCfg(lr=1e-2),
                 precision=precision, max_batch=1 << 13, seed=1)
    model.bind_volumes([torch.as_tensor(vol, device="cuda")])
    lay = o.layout(ENC, MLP)
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=6).astype(np.float64)
    p[:lay.n_table_params] = np.random.default_rng(6).normal(size=lay.n_table_params) * 0.4
    model.load_params([p])
    return model, float(vol.min()), float(vol.max())


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_render_static_matches_render(precision):
    model, vmin, vmax = _model(precision)
    tf = torch.tensor(TF, dtype=torch.float32, device="cuda")
    lo, hi = vmin - 0.1 * (vmax - vmin), vmax
    calls = [((1.9, 1.4, 2.3), 96, 80, 1.0, 64), ((-0.9, 1.6, 1.7), 40, 30, 0.8, 16)]
    for eye, w, hgt, stop, spr in calls:
        say(f"{precision}: eye {eye}, {w}x{hgt}, alpha_stop {stop}, {spr} samples per round")
        args = (0, eye, (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 50.0, w, hgt, tf, (lo, hi), 1.0 / 40, 1.0 / 64)
        img_ws = model.render(*args, alpha_stop=stop, samples_per_round=spr)
        n_ws = model.last_render_samples
        out = torch.full((hgt, w, 4), float("nan"), dtype=torch.float32, device="cuda")
        img_st = model.render(*args, alpha_stop=stop, samples_per_round=spr, static_scratch=True, out=out)
        n_st = model.last_render_samples
        torch.cuda.synchronize()
        assert img_st.data_ptr() == out.data_ptr()
        assert n_st == n_ws > 0
        assert float((img_ws[..., 3] > 0).float().mean()) > 0.2
        assert torch.equal(img_st, img_ws)
    model.sync()


def test_render_static_rejects_images_above_its_limit():
    from paper_2304_10516_amd import _lib as L
    model, vmin, vmax = _model("fp32")
    tf = torch.tensor(TF, dtype=torch.float32, device="cuda")
    limit = 1 << 20
    with pytest.raises(L.DvnrError, match="DVNR_RENDER_STATIC_MAX_RAYS"):
        model.render(0, (1.9, 1.4, 2.3), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 50.0, limit + 1, 1, tf, (vmin, vmax),
                     1.0 / 40, static_scratch=True)
    model.sync()
