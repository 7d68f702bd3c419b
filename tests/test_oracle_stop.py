"""Pins of the oracle's training-length policy (Sec. III-B).

* N_train^max = max(N_train^min, ceil(N_vox / N_batch) * N_epoch) on
  hand-computed cases;
* the moving-average stop rule on a loss sequence 1/k whose stop step is
  worked out by hand;
* train_until: without a loss criterion it runs exactly N_train^max steps and
  equals plain training for that many steps; with a threshold above every
  loss it stops at the first check that has a full window.
"""
import numpy as np

from fixtures import gaussian_sum_field, init_param_draws
from oracle import dvnr_oracle as o


def test_max_train_steps_formula():
    P = o.StopPolicy
    assert o.max_train_steps(64 ** 3, 4096, P(min_steps=0, epochs=2)) == 128      # 64 * 2
    assert o.max_train_steps(64 ** 3, 4096, P(min_steps=500, epochs=2)) == 500    # floor N_min wins
    assert o.max_train_steps(1000, 300, P(min_steps=0, epochs=3)) == 12           # ceil(3.33) = 4, * 3
    assert o.max_train_steps(1000, 0, P(min_steps=50, epochs=3)) == 0             # no samples, no steps
    assert o.max_train_steps(100, 4096, P(min_steps=0, epochs=5)) == 5            # ceil(0.02) = 1


def test_moving_average_stop_step_by_hand():
    # losses 1/k, window 4, checks every 5 steps, threshold 0.1:
    #   k = 5 : mean(1/2, 1/3, 1/4, 1/5)    = 0.3208 -> continue
    #   k = 10: mean(1/7, 1/8, 1/9, 1/10)   = 0.1197 -> continue
    #   k = 15: mean(1/12, 1/13, 1/14, 1/15) = 0.0746 -> stop
    pol = o.StopPolicy(loss_threshold=0.1, window=4, check_every=5)
    losses = []
    stop = None
    for k in range(1, 40):
        losses.append(1.0 / k)
        if o.should_stop(losses, pol):
            stop = k
            break
    assert stop == 15
    assert abs(o.moving_average(losses, 4) - (1 / 12 + 1 / 13 + 1 / 14 + 1 / 15) / 4) < 1e-15
    # no decision between checks, nor before a full window exists
    assert not o.should_stop([1e-9] * 3, o.StopPolicy(loss_threshold=1.0, window=4, check_every=3))
    assert not o.should_stop([1e-9] * 7, o.StopPolicy(loss_threshold=1.0, window=4, check_every=5))
    assert o.should_stop([1e-9] * 5, o.StopPolicy(loss_threshold=1.0, window=4, check_every=5))
    assert not o.should_stop([1e-9] * 5, o.StopPolicy(loss_threshold=0.0, window=4, check_every=5))


def _small():
    vol = gaussian_sum_field(16, seed=1)
    lay = o.layout(o.Encoding(3, 2, 10, 4, 2.0), o.MLP(1, 16))
    p0 = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=0)
    return vol, lay, p0


def test_train_until_budget_and_early_stop():
    vol, lay, p0 = _small()
    opt = o.Optim(lr=1e-2)
    pol = o.StopPolicy(min_steps=0, epochs=3, loss_threshold=0.0)
    params, losses, steps = o.train_until(lay, p0, vol, (16, 16, 16), 0, batch=1024, seed=5, opt=opt, pol=pol)
    assert steps == 12 and len(losses) == 12  # ceil(4096 / 1024) * 3
    ref, ref_losses, _ = o.train(lay, p0, vol, (16, 16, 16), 0, n_steps=12, batch=1024, seed=5, opt=opt)
    np.testing.assert_array_equal(params, ref)
    np.testing.assert_array_equal(losses, ref_losses)
    pol = o.StopPolicy(min_steps=40, epochs=1, loss_threshold=1e9, window=6, check_every=4)
    _, losses, steps = o.train_until(lay, p0, vol, (16, 16, 16), 0, batch=1024, seed=5, opt=opt, pol=pol)
    assert steps == 8  # first multiple of 4 with 6 losses available
