"""Elementwise bars for parameters after fp32 Adam steps, derived from the
gradient bar (test helper; Adam as in Sec. III-F).

The fp32 path's gradients are held to 1e-5 of the largest gradient magnitude
(normwise), so each gradient element may differ from the oracle's by up to
tol * max|g_s| at step s.  Adam acts element by element, and its update
m_hat / (sqrt(v_hat) + eps) is ill-conditioned where the moments nearly
cancel, so a fixed bar per step (say 1e-4 lr) is either loose where the update
is stable or too tight where it is not.  The bar here propagates the gradient
bar through the oracle's own Adam instead: the trajectory is re-run from the
same start with every step's gradient moved by +-tol * max|g_s| in each of the
2^S sign patterns (S steps; one pattern per run, applied to every element, so
that each element sees every corner of its perturbation box), and the bar of
an element is the largest distance of those runs from the exact one.  The
corners bound the box where the update is close to linear in the gradients.
Where a corner already moves the parameter by a tenth of a step or more, the
update direction itself is uncertain (moments near cancellation), and the bar
there is the largest distance any two trajectories can have: each update is
at most rho_t lr_t in magnitude, rho_t = sqrt(sum_k a_k^2 / b_k) by
Cauchy-Schwarz over the moment weights a_k (first moment) and b_k (second)
of the gradients of steps k <= t.  Added to the bar: the rounding of the fp32
update, lr_t 2^-20 per step (a few roundings of the moment ratio), and of the
stored parameter, 2^-23 |theta| per step.
"""
from __future__ import annotations

import itertools

import numpy as np

from oracle import dvnr_oracle as o


def _run(p0: np.ndarray, grads, opt: o.Optim) -> np.ndarray:
    st = o.adam_init(p0.size)
    p = np.asarray(p0, np.float64)
    for g in grads:
        p = o.adam(p, g, st, opt)
    return p


def adam_bound(p0: np.ndarray, grads, opt: o.Optim, tol: float = 1e-5):
    """(oracle parameters after the steps, elementwise bar) for Adam from fresh
    moments over the gradient sequence `grads`, starting at p0."""
    grads = [np.asarray(g, np.float64) for g in grads]
    exact = _run(p0, grads, opt)
    dev = np.zeros_like(exact)
    scale = [tol * float(np.abs(g).max()) for g in grads]
    for signs in itertools.product((-1.0, 1.0), repeat=len(grads)):
        pert = [g + s * d for g, s, d in zip(grads, signs, scale)]
        np.maximum(dev, np.abs(_run(p0, pert, opt) - exact), out=dev)
    lrs = [o.learning_rate(opt, t) for t in range(1, len(grads) + 1)]
    reach = 2.0 * sum(lr * update_ratio_bound(opt, t) for t, lr in enumerate(lrs, 1))
    dev = np.where(dev >= 0.1 * min(lrs), reach, dev)
    return exact, dev + sum(lrs) * 2.0 ** -20 + len(grads) * 2.0 ** -23 * np.abs(exact)


def update_ratio_bound(opt: o.Optim, t: int) -> float:
    """Largest |m_hat / sqrt(v_hat)| of Adam update t over all gradient
    sequences (fresh moments): m_hat = sum_k a_k g_k, v_hat = sum_k b_k g_k^2."""
    b1, b2 = opt.beta1, opt.beta2
    a = [(1 - b1) * b1 ** (t - k) / (1 - b1 ** t) for k in range(1, t + 1)]
    b = [(1 - b2) * b2 ** (t - k) / (1 - b2 ** t) for k in range(1, t + 1)]
    return float(np.sqrt(sum(ak * ak / bk for ak, bk in zip(a, b))))


def excess_report(got: np.ndarray, exact: np.ndarray, bar: np.ndarray, grads) -> str:
    """Where `got` leaves the bar furthest: index, distance, bar, and that element's gradients."""
    d = np.abs(np.asarray(got, np.float64) - exact)
    i = int(np.argmax(d - bar))
    gs = ", ".join(f"{float(g[i]):.3e} (max {float(np.abs(g).max()):.3e})" for g in grads)
    return f"element {i}: distance {d[i]:.3e}, bar {bar[i]:.3e}, oracle {exact[i]:.6e}, gradients {gs}"
