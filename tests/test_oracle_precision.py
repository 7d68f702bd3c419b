"""The bfloat16 tolerance of the mixed-precision gradient, derived on the CPU.

The mixed path feeds the MLP's matrix-core products 16-bit operands (encoding
features, hidden activations, backward deltas; float32 accumulation).  The
rounding model in tests/precision_model.py applies exactly those roundings
around the oracle's layer functions.  Its distance from the oracle's exact
gradient is the intrinsic error of bf16 operands; the GPU bars of the mixed
gradient are stated multiples of it (see precision_model.check_mixed_gradient).
"""
import numpy as np
import pytest

from fixtures import gaussian_sum_field, init_param_draws
from oracle import dvnr_oracle as o
from tests import precision_model as pm

C1 = (o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16))
C2 = (o.Encoding(16, 2, 19, 16, 0.0, 256), o.MLP(2, 64))


def test_bf16_rounding_is_round_to_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7  # bfloat16 keeps 7 explicit mantissa bits
    cases = {one + ulp / 2: one,                      # tie, even neighbour below
             one + 1.5 * ulp: one + 2 * ulp,           # tie, even neighbour above
             one + ulp / 2 + 2.0 ** -20: one + ulp,    # just above the tie
             one + ulp / 2 - 2.0 ** -20: one,          # just below the tie
             -(one + 1.5 * ulp): -(one + 2 * ulp),
             3.4e38: np.inf,                           # above the midpoint past the largest finite bf16
             0.0: 0.0}
    for v, want in cases.items():
        assert pm.round_bf16(np.array([v]))[0] == want, v


@pytest.mark.parametrize("cfg", [C1, (o.Encoding(3, 4, 10, 4, 2.0), o.MLP(3, 32))])
@pytest.mark.parametrize("loss", ["l2", "l1"])
def test_model_without_rounding_is_the_oracle(cfg, loss):
    """The layer-by-layer composition of oracle calls, with no rounding, is the
    oracle's own loss and gradient."""
    lay = o.layout(*cfg)
    rng = np.random.default_rng(4)
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=3).astype(np.float64)
    p[:lay.n_table_params] = rng.normal(size=lay.n_table_params) * 0.3
    x = o.training_coords(5, 0, 0, 700)
    tgt = rng.random(700)
    L, g, _ = o.loss_and_grad(lay, p, x, tgt, loss)
    Lm, gm = pm.loss_and_grad(lay, p, x, tgt, loss, rounded=False)
    assert abs(L - Lm) <= 1e-13 * L
    assert np.max(np.abs(g - gm)) <= 1e-12 * np.max(np.abs(g))


def _c2_case(n=8192):
    """The 16-level 256^3 configuration's encoding on a 64^3 field, 8192 samples:
    the case of the GPU's fine-level gradient tests."""
    lay = o.layout(*C2)
    vol = gaussian_sum_field(64, seed=3)
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=2).astype(np.float64)
    p[:lay.n_table_params] *= 1e3
    pw = pm.working_copy(lay, p)
    x = o.training_coords(91, 0, 0, n)
    return lay, pw, x, o.normalized_targets(vol, (64, 64, 64), 0, x)


def test_intrinsic_bf16_gradient_error_on_the_16_level_encoding():
    """bf16 operands alone move each level's table gradient by a few percent in
    2-norm (recorded in the design notes), the weight gradient by ~1e-3 and the
    loss by ~1e-5: the error a correct mixed kernel cannot avoid."""
    lay, pw, x, tgt = _c2_case()
    errs, werr, _, _, Le, Lm = pm.intrinsic_errors(lay, pw, x, tgt)
    print("intrinsic per-level 2-norm error: " + " ".join(f"{e:.4f}" for e in errs) + f"; weights {werr:.2e}")
    assert all(5e-3 <= e <= 8e-2 for e in errs)
    assert max(errs) >= 3e-2
    assert werr <= 3e-3
    assert abs(Le - Lm) <= 1e-4 * Le
    # the feature rounding alone (the encoding output fed to the first product)
    # already accounts for most of it: it moves the output, hence dL/do of every sample
    ge = pm.o.loss_and_grad(lay, pw, x, tgt)[1]
    only_feat = _only_feature_rounding(lay, pw, x, tgt)
    ef = [pm.rel2(only_feat[a:b], ge[a:b]) for a, b in pm.level_spans(lay)]
    assert max(ef) >= 0.5 * max(errs)


def _only_feature_rounding(lay, pw, x, tgt):
    y = pm.round_bf16(pm.round_f32(o.encode(lay, pw, x)))
    W = o.mlp_weights(lay, pw)
    out, acts = o.mlp_forward(W, y)
    do = 2.0 * (out[:, 0] - tgt) / out.shape[0]
    dy, _ = o.mlp_backward(W, acts, do[:, None])
    return o.encode_backward(lay, x, dy)


def test_mixed_gradient_bars_catch_a_level_error():
    """The GPU bars: the rounding model itself passes; a 3 % error planted on
    one level (a fraction of that level's intrinsic error added as a systematic
    bias) fails the bar of following the model."""
    lay, pw, x, tgt = _c2_case(4096)
    _, gm = pm.loss_and_grad(lay, pw, x, tgt)
    pm.check_mixed_gradient(gm, lay, pw, x, tgt)
    # a unit within float32 rounding of its ReLU kink that lands on the other
    # side (as a float32 sum may put it) is within the bars
    _, _, near = pm.loss_and_grad(lay, pw, x, tgt, kink=pm.KINK)
    assert near, "the case has near-kink units"
    pm.check_mixed_gradient(gm + pm.kink_toggles(lay, pw, x, tgt, near[:1])[0], lay, pw, x, tgt)
    a, b = pm.level_spans(lay)[12]
    bad = gm.copy()
    bad[a:b] *= 1.03
    with pytest.raises(AssertionError, match="level 12"):
        pm.check_mixed_gradient(bad, lay, pw, x, tgt)
    bad = gm.copy()
    nt = lay.n_table_params
    bad[nt:nt + 100] *= 1.05
    with pytest.raises(AssertionError, match="weights"):
        pm.check_mixed_gradient(bad, lay, pw, x, tgt)


def test_mixed_forward_is_the_oracle_when_every_rounding_is_exact():
    """pm.infer rounds features and hidden-layer inputs to bf16 and activations
    to fp32: with tables, weights and coordinates chosen so that every one of
    those values is already a bf16 number, it equals the oracle's forward
    exactly; a non-representable weight makes them differ.  Levels R = 3, 5:
    coordinates k/4 are vertices of the fine level and cell midpoints (weights
    1/2) of the coarse one; tables in quarters and first-layer weights of
    +-1/2 keep features and hidden values within 8 significant bits."""
    enc, mlp = o.Encoding(2, 2, 10, 3, 5.0 / 3.0), o.MLP(2, 16)
    lay = o.layout(enc, mlp)
    assert [lv.R for lv in lay.levels] == [3, 5]
    rng = np.random.default_rng(3)
    p = np.empty(lay.n_params)
    nt = lay.n_table_params
    (o1, o2, o3) = lay.mlp_offsets
    p[:nt] = rng.integers(-4, 5, nt) / 4.0
    p[o1:o2] = rng.integers(-1, 2, o2 - o1) / 2.0
    p[o2:o3] = rng.integers(-1, 2, o3 - o2) / 4.0
    p[o3:] = rng.integers(-8, 9, lay.n_params - o3) / 16.0
    assert np.array_equal(pm.working_copy(lay, p), p)
    x = (rng.integers(0, 5, (300, 3)) / 4.0).astype(np.float32)
    ref = o.infer(lay, p, x)
    assert np.array_equal(pm.infer(lay, p, x), ref) and np.abs(ref).max() > 0
    q = p.copy()
    q[o1:o2] += rng.uniform(-1, 1, o2 - o1) * 2.0 ** -10  # first-layer weights off the bf16 grid
    assert not np.array_equal(pm.infer(lay, pm.working_copy(lay, q), x), o.infer(lay, q, x))


def test_mixed_training_loop_takes_the_rounded_gradient_and_the_oracle_adam():
    enc, mlp = C1
    lay = o.layout(enc, mlp)
    vol = gaussian_sum_field(16, seed=1)
    p0 = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=0).astype(np.float64)
    assert np.array_equal(pm.train(lay, p0, vol, (16, 16, 16), 0, 0, 256, 5, o.Optim()), p0)
    p = pm.train(lay, p0, vol, (16, 16, 16), 0, 2, 256, 5, o.Optim())
    st, q = o.adam_init(lay.n_params), p0.copy()
    for step in range(2):
        x = o.training_coords(5, 0, step, 256)
        _, g = pm.loss_and_grad(lay, pm.working_copy(lay, q), x, o.normalized_targets(vol, (16, 16, 16), 0, x))
        q = o.adam(q, g, st, o.Optim())
    assert np.array_equal(p, q)
