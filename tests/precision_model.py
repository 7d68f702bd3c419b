"""Rounding model of the mixed-precision training step, built around oracle calls.

TEST INFRASTRUCTURE ONLY.  The oracle computes the loss gradient exactly (float64).
The mixed-precision path rounds some intermediate values to bfloat16 because
the MLP's matrix-core products take 16-bit operands: the encoding features, the
hidden activations that feed the next layer, and the backward deltas that feed
the weight-gradient and input-gradient products.  Accumulation is float32;
the output layer, the loss and its derivative stay float32.  This module
evaluates the oracle's own layer functions (`mlp_forward`, `mlp_backward`,
`encode`, `encode_backward`) one layer at a time and applies those roundings
between the calls, so that

* its distance from the exact gradient is the error that bfloat16 operands
  cause in ANY correct implementation (the intrinsic error; its size on the
  256^3 configuration is recorded in the design notes), and
* a correct GPU kernel follows it far more closely than that (only the float32
  summation order differs).

It adds no arithmetic of the method: every product and sum is an oracle call;
only roundings and ReLU masks are applied here.  With rounding switched off it
reproduces `oracle.loss_and_grad` exactly (pinned in test_oracle_precision.py).
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import dvnr_oracle as o


def round_bf16(a):
    """Nearest bfloat16 value (ties to even) of float32(a), returned as float64."""
    t = torch.as_tensor(np.asarray(a, dtype=np.float64)).to(torch.float32)
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def round_f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def working_copy(lay, params):
    """The parameters the mixed path computes with: fp16 tables, bf16 weights."""
    nt = lay.n_table_params
    p = np.asarray(params, dtype=np.float64)
    tab = p[:nt].astype(np.float32).astype(np.float16).astype(np.float64)
    return np.concatenate([tab, round_bf16(p[nt:])])


def loss_and_grad(lay, params, x, target, loss="l2", rounded=True, kink=None, force=None, n_scale=None):
    """(loss, gradient vector) of one block with the mixed path's roundings.

    `params` must already be the working copy (see `working_copy`).  With
    rounded=False no rounding is applied and the result equals
    oracle.loss_and_grad up to float64 summation order.

    kink=tau: also return the hidden units that lie within float32 rounding of
    the ReLU kink, as (sample, layer, unit) triples: pre-activation z with
    |z| <= tau * sum_i |W_ji a_i|, so that a float32 sum may land on either
    side of zero.  force={(layer, unit): active}: take that unit's ReLU
    derivative as given for every sample (its forward value max(z, 0) is ~0
    either way).  n_scale: the sample count of the mean (default: len(x))."""
    bf = round_bf16 if rounded else (lambda a: np.asarray(a, np.float64))
    f32 = round_f32 if rounded else (lambda a: np.asarray(a, np.float64))
    W = o.mlp_weights(lay, params)
    nh = len(W) - 1
    y = o.encode(lay, params, x)
    a = [bf(f32(y))]                 # inputs of the hidden layers' products
    h, masks = [], []                # float32 hidden activations, ReLU derivatives
    near = []
    for k in range(nh):
        z, _ = o.mlp_forward([W[k]], a[k])
        m = z > 0.0
        for (kk, j), v in (force or {}).items():
            if kk == k:
                m[:, j] = v
        if kink is not None:
            mag, _ = o.mlp_forward([np.abs(W[k])], np.abs(a[k]))
            near.extend((int(i), k, int(j)) for i, j in zip(*np.nonzero(np.abs(z) <= kink * mag)))
        h.append(f32(np.maximum(z, 0.0)))
        masks.append(m)
        if k + 1 < nh:
            a.append(bf(h[k]))
    out, _ = o.mlp_forward([W[nh]], h[nh - 1])
    out = out[:, 0]
    n = out.shape[0] if n_scale is None else n_scale
    r = out - np.asarray(target, dtype=np.float64)
    if loss == "l2":
        L = float(np.sum(r * r) / n)
        do = (2.0 / n) * r
    elif loss == "l1":
        L = float(np.sum(np.abs(r)) / n)
        do = np.sign(r) / n
    else:
        raise ValueError(loss)
    dh, (dWo,) = o.mlp_backward([W[nh]], [h[nh - 1]], do[:, None])
    dWs = [None] * nh
    for k in range(nh - 1, -1, -1):
        dz = bf(f32(dh * masks[k]))
        dh, (dWs[k],) = o.mlp_backward([W[k]], [a[k]], dz)
    g = np.empty(lay.n_params, dtype=np.float64)
    g[:lay.n_table_params] = o.encode_backward(lay, x, dh)
    for dW, off in zip(dWs + [dWo], lay.mlp_offsets):
        g[off:off + dW.size] = dW.reshape(-1)
    if kink is not None:
        return L, g, near
    return L, g


def kink_toggles(lay, params, x, target, near, loss="l2"):
    """Gradient change of every near-kink unit switched to the other side:
    for (sample i, layer k, unit j), sample i's contribution (1/n scaling of
    the whole batch) with unit j's ReLU derivative forced on minus forced off.
    Returns a list of gradient vectors."""
    n = len(x)
    x = np.asarray(x)
    target = np.asarray(target)
    out = []
    for i, k, j in near:
        _, g_on = loss_and_grad(lay, params, x[i:i + 1], target[i:i + 1], loss, force={(k, j): True}, n_scale=n)
        _, g_off = loss_and_grad(lay, params, x[i:i + 1], target[i:i + 1], loss, force={(k, j): False}, n_scale=n)
        out.append(g_on - g_off)
    return out


def level_spans(lay):
    F = lay.enc.n_features
    return [(lv.off * F, (lv.off + lv.E) * F) for lv in lay.levels]


def rel2(a, b):
    """||a - b||_2 / ||b||_2 (float64)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def intrinsic_errors(lay, params, x, target, loss="l2"):
    """Per-level and weight 2-norm distances of the rounding model from the exact
    gradient, and both gradients: (level_errs, weight_err, exact, model, L_exact, L_model)."""
    Le, ge, _ = o.loss_and_grad(lay, params, x, target, loss)
    Lm, gm = loss_and_grad(lay, params, x, target, loss)
    nt = lay.n_table_params
    errs = [rel2(gm[a:b], ge[a:b]) for a, b in level_spans(lay)]
    return errs, rel2(gm[nt:], ge[nt:]), ge, gm, Le, Lm


# a float32 sum of at most 64 exact products errs by less than 64 half-ulps
# (2^-24 * 32 = 1.9e-6) of sum |W a|
KINK = 2e-6


def check_mixed_gradient(gpu_grad, lay, params, x, target, loss="l2", follow=0.1, excess=1.25, floor=1e-4,
                         weight_follow=0.1):
    """Bars of a mixed-precision gradient (design notes: the bf16 tolerance reading).

    Per table level l, with e_l the rounding model's own distance from the exact
    gradient (the intrinsic bf16 error of that level) and k_l the sum, over the
    hidden units within float32 rounding of the ReLU kink (`KINK`), of the
    level-l norm of the gradient change if that unit switched sides (the GPU's
    float32 sum may put it on either side):
      ||gpu - model||_2 <= (follow * e_l + floor) * ||exact||_2 + k_l
      ||gpu - exact||_2 <= (excess * e_l + floor) * ||exact||_2 + k_l
    and for the weights the same with `weight_follow`.  Returns a dict of the
    measured ratios and both losses (for the test log); raises AssertionError
    on a failed bar."""
    errs, werr, ge, gm, Le, Lm = intrinsic_errors(lay, params, x, target, loss)
    _, _, near = loss_and_grad(lay, params, x, target, loss, kink=KINK)
    toggles = kink_toggles(lay, params, x, target, near, loss)
    gg = np.asarray(gpu_grad, dtype=np.float64)
    out = {"intrinsic": errs, "weights_intrinsic": werr, "follow": [], "excess": [], "loss_exact": Le,
           "loss_model": Lm, "near_kink": len(near)}

    def kslack(a, b):
        return sum(float(np.linalg.norm(t[a:b])) for t in toggles)

    for l, (a, b) in enumerate(level_spans(lay)):
        ref = np.linalg.norm(ge[a:b])
        if ref == 0.0:
            assert np.max(np.abs(gg[a:b])) == 0.0, f"level {l}: gradient where the oracle has none"
            continue
        slack = kslack(a, b) / ref
        fol = np.linalg.norm(gg[a:b] - gm[a:b]) / ref
        exc = np.linalg.norm(gg[a:b] - ge[a:b]) / ref
        out["follow"].append(fol)
        out["excess"].append(exc)
        assert fol <= follow * errs[l] + floor + slack, \
            f"level {l}: {fol:.2e} from the rounding model (intrinsic {errs[l]:.2e}, kink slack {slack:.1e})"
        assert exc <= excess * errs[l] + floor + slack, \
            f"level {l}: {exc:.2e} from the exact gradient (intrinsic {errs[l]:.2e}, kink slack {slack:.1e})"
    nt = lay.n_table_params
    ref = np.linalg.norm(ge[nt:])
    slack = kslack(nt, lay.n_params) / ref
    wf = rel2(gg[nt:], gm[nt:])
    we = rel2(gg[nt:], ge[nt:])
    out["weights_follow"], out["weights_excess"] = wf, we
    assert wf <= weight_follow * werr + floor + slack, \
        f"weights: {wf:.2e} from the rounding model (intrinsic {werr:.2e}, kink slack {slack:.1e})"
    assert we <= excess * werr + floor + slack, \
        f"weights: {we:.2e} from the exact gradient (intrinsic {werr:.2e}, kink slack {slack:.1e})"
    return out


def infer(lay, params, x):
    """Normalized INR output with the mixed path's roundings of the forward
    (features and hidden-layer inputs in bfloat16, float32 activations);
    `params` is the working copy."""
    W = o.mlp_weights(lay, params)
    a = round_bf16(round_f32(o.encode(lay, params, x)))
    for k in range(len(W) - 1):
        z, _ = o.mlp_forward([W[k]], a)
        h = round_f32(np.maximum(z, 0.0))
        a = round_bf16(h) if k + 2 < len(W) else h
    out, _ = o.mlp_forward([W[-1]], a)
    return out[:, 0]


def decode(lay, params, dims, vmin, vmax, chunk=1 << 16):
    """oracle.decode with the mixed path's forward (`infer`) on the working
    copy of the float64 masters `params`."""
    wc = working_copy(lay, params)
    x = o.voxel_center_coords(dims)
    out = np.concatenate([infer(lay, wc, x[i:i + chunk]) for i in range(0, len(x), chunk)])
    return (out * (vmax - vmin) + vmin).reshape(dims[2], dims[1], dims[0])


def train(lay, params0, vol, dims, ghost, n_steps, batch, seed, opt, block=0):
    """oracle.train's loop (uniform samples, L2) with the mixed path's
    roundings: each step's gradient is `loss_and_grad` on the working copy of
    the float64 masters, and the oracle's Adam updates the masters."""
    p = np.asarray(params0, np.float64).copy()
    st = o.adam_init(p.size)
    for step in range(n_steps):
        x = o.training_coords(seed, block, step, batch)
        _, g = loss_and_grad(lay, working_copy(lay, p), x, o.normalized_targets(vol, dims, ghost, x))
        p = o.adam(p, g, st, opt)
    return p
