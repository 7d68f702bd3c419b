"""CPU checks of the derived Adam bars (tests/adam_bound.py)."""
import numpy as np

from oracle import dvnr_oracle as o
from tests.adam_bound import adam_bound, update_ratio_bound


def _grads(rng, n, steps):
    # gradients of mixed sign and magnitudes over 3.5 decades, changing sign between steps
    return [rng.standard_normal(n) * np.exp(rng.uniform(-8, 0, n)) for _ in range(steps)]


def _adam(p0, grads, opt):
    st, p = o.adam_init(p0.size), p0.copy()
    for g in grads:
        p = o.adam(p, g, st, opt)
    return p


def test_perturbations_inside_the_gradient_bar_stay_inside_the_bar():
    rng = np.random.default_rng(0)
    n, tol = 50000, 1e-5
    for opt in (o.Optim(lr=1e-2), o.Optim(lr=1e-2, lr_decay_base=0.5, lr_decay_start=1, lr_decay_interval=1)):
        p0 = rng.uniform(-1e-1, 1e-1, n)
        grads = _grads(rng, n, 3)
        exact, bar = adam_bound(p0, grads, opt, tol)
        for _ in range(6):  # interior points and corners of the box
            pert = [g + rng.choice([-1.0, rng.uniform(-1, 1), 1.0], n) * tol * np.abs(g).max() for g in grads]
            assert np.all(np.abs(_adam(p0, pert, opt) - exact) <= bar)


def test_bar_is_tight_where_adam_is_well_conditioned_and_catches_larger_errors():
    rng = np.random.default_rng(1)
    n, tol = 50000, 1e-5
    opt = o.Optim(lr=1e-2)
    p0 = rng.uniform(-1e-1, 1e-1, n)
    grads = _grads(rng, n, 3)
    exact, bar = adam_bound(p0, grads, opt, tol)
    # elements whose gradients keep their sign and stay within a decade of the largest:
    # far below 1e-4 lr per step
    big = np.all([np.abs(g) > 0.1 * np.abs(g).max() for g in grads], axis=0)
    big &= np.all([np.sign(g) == np.sign(grads[0]) for g in grads], axis=0)
    assert big.sum() >= 5 and np.max(bar[big]) < 1e-4 * opt.lr
    # gradients off by 30 times the gradient bar: some parameter leaves its bar
    pert = [g + 30 * tol * np.abs(g).max() for g in grads]
    assert np.any(np.abs(_adam(p0, pert, opt) - exact) > bar)
    # a wrong first-moment rate is caught on most elements
    wrong = _adam(p0, grads, o.Optim(lr=1e-2, beta1=0.89))
    assert np.mean(np.abs(wrong - exact) > bar) > 0.5


def test_update_ratio_bound_is_attained_and_not_exceeded():
    opt = o.Optim()
    assert update_ratio_bound(opt, 1) == 1.0
    rng = np.random.default_rng(2)
    for t in (2, 3, 5):
        g = rng.standard_normal((t, 200000))
        st = o.adam_init(g.shape[1])
        p = np.zeros(g.shape[1])
        for k in range(t):
            p = o.adam(p, g[k], st, o.Optim(lr=0.0, weight_decay=0.0))
        ratio = np.abs(st.m / (1 - opt.beta1 ** t)) / np.sqrt(st.v / (1 - opt.beta2 ** t))
        rb = update_ratio_bound(opt, t)
        assert ratio.max() <= rb * (1 + 1e-12)
        # attained by the gradients g_k proportional to a_k / b_k
        a = np.array([(1 - opt.beta1) * opt.beta1 ** (t - k) / (1 - opt.beta1 ** t) for k in range(1, t + 1)])
        b = np.array([(1 - opt.beta2) * opt.beta2 ** (t - k) / (1 - opt.beta2 ** t) for k in range(1, t + 1)])
        gk = a / b
        assert abs(np.dot(a, gk) / np.sqrt(np.dot(b, gk * gk)) - rb) <= 1e-12 * rb
