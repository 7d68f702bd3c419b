"""GPU parity at the full size of the 256^3 training workload, in the launch
configuration the benchmark times: one 256^3 block of the seeded k^-5/3
field, hash grid L=16, T=2^19, F=2, base 16, finest 256, MLP 2x64, 2^18
samples per step.  The float64 oracle computes the whole step at this size
(about 10 s on one core), so the gradient is compared element by element.

* fp32 with the mixed path's kernel structure (ordered samples, bin-privatized
  coarse levels, destination-partitioned levels 9..15 with 16 sub-buckets per
  bucket): loss and every level's table gradient within 1e-5 normwise.  The
  table entries and weights are made positive for this case, so that every
  ReLU unit is active for every sample: with random signs, about 1000 of the
  2^18 samples have a hidden pre-activation within 1e-5 of its magnitude
  scale of zero, a few of them switch their unit between fp32 and fp64, and a
  switched sample moves all its 128 corner entries by a macroscopic amount
  (the small-size tests cover inactive units);
* mixed precision with its default options (those of the benchmark: levels
  4..15 partitioned), positive parameters as above: the bars of the bf16
  tolerance reading -- per level within 0.1 x the level's intrinsic bf16
  error of the rounding model (tests/precision_model.py) and within 1.25 x of
  the exact gradient; the loss within 1e-5 of the model's.  (With random
  signs, a few hundred of the 2^18 x 128 hidden units sit within float32
  rounding of the kink; the bars allow each to switch, which at this size
  adds up to several percent; the smaller tests cover that case.)
"""
import sys

import numpy as np
import pytest
import torch

from fixtures import init_param_draws, kolmogorov_field
from oracle import dvnr_oracle as o
from tests import precision_model as pm

pytestmark = pytest.mark.gpu

C2 = (o.Encoding(16, 2, 19, 16, 0.0, 256), o.MLP(2, 64))
N = 1 << 18


def say(msg):
    print(f"[gpu-fullsize] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def field():
    return kolmogorov_field(256, seed=2)


def _model(precision):
    from paper_2304_10516_amd.dvnr import DVNR, EncodingCfg, MlpCfg, OptimCfg
    enc, mlp = C2
    e = EncodingCfg(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution,
                    enc.per_level_scale, enc.finest_resolution)
    return DVNR(e, MlpCfg(mlp.n_hidden_layers, mlp.width), [((256, 256, 256), 0)], OptimCfg(lr=1e-2),
                precision=precision, max_batch=N, seed=3)


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_full_size_step_gradient(field, precision):
    say(f"256^3 block, 2^18 samples, {precision}")
    lay = o.layout(*C2)
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=2).astype(np.float64)
    p[:lay.n_table_params] *= 1e3
    p = np.abs(p)  # every ReLU unit active: no unit near its kink (see above)
    model = _model(precision)
    model.bind_volumes([torch.as_tensor(field, device="cuda")])
    model.load_params([p])
    if precision == "fp32":
        model.set_option("spatial_sort", 1)
        model.set_option("scatter_part", 9)
    model.set_option("apply_update", 0)
    loss = model.train(1, N, want_loss=True)
    torch.cuda.synchronize()
    lf = model.partitioned_levels()
    say(f"partitioned levels from {lf}; plan {model.plan_info()}")
    assert lf == (9 if precision == "fp32" else 4)  # mixed default: every level with 2^15 entries or more
    x = o.training_coords(3, 0, 0, N)
    tgt = o.normalized_targets(field, (256, 256, 256), 0, x)
    gg = model.block_grads(0).cpu().numpy().astype(np.float64)
    nt = lay.n_table_params
    if precision == "mixed":
        r = pm.check_mixed_gradient(gg, lay, pm.working_copy(lay, p), x, tgt)
        say("following the rounding model per level (x intrinsic): " +
            " ".join(f"{f / e:.3f}" for f, e in zip(r["follow"], r["intrinsic"])) +
            "; intrinsic " + " ".join(f"{e:.3f}" for e in r["intrinsic"]) +
            f"; weights {r['weights_follow']:.2e} (intrinsic {r['weights_intrinsic']:.2e})")
        rel = abs(loss[0, 0].item() - r["loss_model"]) / r["loss_model"]
        say(f"loss {loss[0, 0].item():.6g} vs model {r['loss_model']:.6g} (rel {rel:.2e})")
        assert rel <= 1e-5
        return
    pref = model.block_params(0).cpu().numpy().astype(np.float64)
    L, g, _ = o.loss_and_grad(lay, pref, x, tgt)
    rel = abs(loss[0, 0].item() - L) / L
    say(f"loss {loss[0, 0].item():.6g} vs oracle {L:.6g} (rel {rel:.2e})")
    assert rel <= 1e-5
    errs = []
    for lvl in lay.levels:
        a, b = lvl.off * 2, (lvl.off + lvl.E) * 2
        errs.append(float(np.max(np.abs(gg[a:b] - g[a:b])) / np.max(np.abs(g[a:b]))))
    say("per-level normwise error: " + " ".join(f"{e:.1e}" for e in errs))
    assert max(errs) <= 1e-5
    assert float(np.max(np.abs(gg[nt:] - g[nt:])) / np.max(np.abs(g[nt:]))) <= 1e-5
