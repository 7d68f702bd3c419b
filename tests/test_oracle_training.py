"""Pins of the oracle's sampler, network, loss, optimizer and metrics.

* Philox4x32-10 against published known-answer vectors;
* the cell-centered sampler against torch grid_sample (align_corners=False,
  border padding) and an affine volume with a ghost layer (closed form);
* the MLP against torch.nn.functional.linear, its backward against autograd;
* the full loss gradient against central finite differences;
* Adam against torch.optim.Adam;
* PSNR against its closed form; the apportionment against its invariants.
"""
import json
import os

import numpy as np
import pytest
import torch

from fixtures import gaussian_sum_field, init_param_draws, uniform_coords
from oracle import dvnr_oracle as o

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLD, "philox4x32_10_kat.json")) as f:
        kat = json.load(f)["vectors"]
    for v in kat:
        ctr = np.array([[int(w, 16) for w in v["ctr"]]], dtype=np.uint64)
        out = o.philox4x32_10(ctr, [int(w, 16) for w in v["key"]])[0]
        assert [int(w) for w in out] == [int(w, 16) for w in v["out"]]


def test_training_coords_are_uniform_float32_grid():
    x = o.training_coords(seed=7, block=3, step=11, n=1 << 16)
    assert x.dtype == np.float32 and x.shape == (1 << 16, 3)
    assert x.min() >= 0.0 and x.max() < 1.0
    scaled = x.astype(np.float64) * 2.0 ** 24
    assert np.array_equal(scaled, np.floor(scaled))
    # chi-square over 16^3 bins (4096 dof): mean 4095, sd ~ 90.5
    b = np.floor(x * 16).astype(int)
    counts = np.bincount(b[:, 0] + 16 * b[:, 1] + 256 * b[:, 2], minlength=4096)
    e = x.shape[0] / 4096
    chi2 = np.sum((counts - e) ** 2 / e)
    assert abs(chi2 - 4095) < 6 * 90.5
    # different steps / blocks give different streams; same arguments repeat
    assert not np.array_equal(x, o.training_coords(7, 3, 12, 1 << 16))
    assert not np.array_equal(x, o.training_coords(7, 4, 11, 1 << 16))
    assert np.array_equal(x[100:200], o.training_coords(7, 3, 11, 100, first=100))


def _grid_sample_ref(vol, x):
    t = torch.tensor(vol, dtype=torch.float64)[None, None]
    g = torch.tensor(2.0 * x.astype(np.float64) - 1.0).view(1, -1, 1, 1, 3)
    return torch.nn.functional.grid_sample(t, g, mode="bilinear", padding_mode="border",
                                           align_corners=False).view(-1).numpy()


@pytest.mark.parametrize("dims", [(5, 7, 6), (16, 16, 16), (3, 2, 9)])
def test_sampler_matches_grid_sample_without_ghosts(dims):
    rng = np.random.default_rng(sum(dims))
    vol = rng.normal(size=dims[::-1])
    x = np.concatenate([uniform_coords(2000, seed=1),
                        np.array([[0, 0, 0], [1, 1, 1], [0.5, 0, 1], [1e-3, 0.999, 0.25]], np.float32)])
    np.testing.assert_allclose(o.sample_volume(vol, dims, 0, x), _grid_sample_ref(vol, x), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("ghost", [1, 2])
def test_sampler_affine_with_ghost_is_exact(ghost):
    dims = (6, 9, 5)
    a = np.array([0.7, -0.2, 1.3])
    sz = [d + 2 * ghost for d in dims]
    Z, Y, X = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in sz[::-1]], indexing="ij")
    vol = a[0] * X + a[1] * Y + a[2] * Z + 0.5  # value at stored index (i, j, k)
    x = np.concatenate([uniform_coords(3000, seed=4), np.array([[0, 0, 0], [1, 1, 1]], np.float32)]).astype(np.float64)
    p = x * np.array(dims) - 0.5 + ghost  # stored-index position
    np.testing.assert_allclose(o.sample_volume(vol, dims, ghost, x), p @ a + 0.5, rtol=1e-12, atol=1e-12)


def test_normalized_targets_in_unit_interval():
    vol = gaussian_sum_field(16, seed=3)
    x = uniform_coords(4000, seed=2)
    t = o.normalized_targets(vol, (16, 16, 16), 0, x)
    assert t.min() >= -1e-12 and t.max() <= 1 + 1e-12
    const = np.full((4, 4, 4), 0.3, np.float32)
    assert np.allclose(o.normalized_targets(const, (4, 4, 4), 0, x[:10]), 0.0)


def _mlp_setup(nh=2, w=16, din=8, n=37, seed=0):
    rng = np.random.default_rng(seed)
    shapes = [(w, din)] + [(w, w)] * (nh - 1) + [(1, w)]
    Ws = [rng.normal(size=s) for s in shapes]
    y = rng.normal(size=(n, din))
    return Ws, y


@pytest.mark.parametrize("nh", [1, 2, 4])
def test_mlp_forward_matches_torch_linear(nh):
    Ws, y = _mlp_setup(nh=nh)
    o_, _ = o.mlp_forward(Ws, y)
    h = torch.tensor(y)
    for W in Ws[:-1]:
        h = torch.relu(torch.nn.functional.linear(h, torch.tensor(W)))
    ref = torch.nn.functional.linear(h, torch.tensor(Ws[-1])).numpy()
    np.testing.assert_allclose(o_, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("nh", [1, 3])
def test_mlp_backward_matches_autograd(nh):
    Ws, y = _mlp_setup(nh=nh, seed=4)
    rng = np.random.default_rng(1)
    do = rng.normal(size=(y.shape[0], 1))
    _, acts = o.mlp_forward(Ws, y)
    dy, dWs = o.mlp_backward(Ws, acts, do)
    ty = torch.tensor(y, requires_grad=True)
    tW = [torch.tensor(W, requires_grad=True) for W in Ws]
    h = ty
    for W in tW[:-1]:
        h = torch.relu(h @ W.T)
    (h @ tW[-1].T).backward(torch.tensor(do))
    np.testing.assert_allclose(dy, ty.grad.numpy(), rtol=1e-12, atol=1e-12)
    for a, b in zip(dWs, tW):
        np.testing.assert_allclose(a, b.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_loss_gradient_matches_finite_differences():
    enc, mlp = o.Encoding(3, 2, 6, 2, 2.0), o.MLP(1, 16)
    lay = o.layout(enc, mlp)
    params = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=3).astype(np.float64)
    params[:lay.n_table_params] *= 3e3  # O(0.3) table values so every term matters
    rng = np.random.default_rng(2)
    # keep coordinates away from cell faces so that the encoding is smooth in x
    x = (0.1 + 0.8 * rng.random((32, 3))).astype(np.float32)
    tgt = rng.random(32)
    L, g, _ = o.loss_and_grad(lay, params, x, tgt)
    h = 1e-6
    pick = np.concatenate([rng.choice(lay.n_table_params, 12, replace=False),
                           lay.n_table_params + rng.choice(lay.n_params - lay.n_table_params, 12, replace=False)])
    for j in pick:
        e = np.zeros_like(params)
        e[j] = h
        fd = (o.loss_and_grad(lay, params + e, x, tgt)[0] - o.loss_and_grad(lay, params - e, x, tgt)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1e-3, abs(g[j])), (j, fd, g[j])


def test_adam_matches_torch():
    rng = np.random.default_rng(0)
    n = 50
    p0 = rng.normal(size=n)
    grads = [rng.normal(size=n) * 10 ** rng.uniform(-6, 0) for _ in range(7)]
    opt = o.Optim(lr=1e-2)
    st = o.adam_init(n)
    p = p0.copy()
    for g in grads:
        p = o.adam(p, g, st, opt)
    tp = torch.tensor(p0, requires_grad=True)
    topt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-9)
    for g in grads:
        topt.zero_grad()
        tp.grad = torch.tensor(g)
        topt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_learning_rate_decay_closed_form():
    # under a constant gradient g, Adam's bias-corrected moments are exactly g
    # and g^2, so update t moves theta by lr_t * |g| / (|g| + eps): the schedule
    opt = o.Optim(lr=1e-2, weight_decay=0.0, lr_decay_base=0.1, lr_decay_start=3, lr_decay_interval=8)
    st = o.adam_init(1)
    g = np.array([0.5])
    th = np.zeros(1)
    for t in range(1, 30):
        new = o.adam(th, g, st, opt)
        want = 1e-2 * (0.1 ** (max(0, t - 3) / 8)) * 0.5 / (0.5 + 1e-8)
        assert abs((th - new)[0] - want) <= 1e-15 + 1e-12 * want, t
        th = new
    assert o.learning_rate(opt, 11) == 1e-3 and o.learning_rate(o.Optim(lr=2e-2), 500) == 2e-2


def test_psnr_closed_form():
    truth = np.random.default_rng(1).random((8, 8, 8))
    for e in (1e-1, 1e-2, 3e-4):
        sse, cnt = o.squared_error(truth + e, truth)
        assert abs(o.psnr(sse, cnt) - (-20 * np.log10(e))) < 1e-9


def test_apportion_invariants():
    rng = np.random.default_rng(3)
    vox = rng.integers(96, 161, size=(64, 3)).prod(axis=1)
    n = o.apportion(vox, 1 << 20)
    assert n.sum() == 1 << 20 and (n % 256 == 0).all()
    quota = (1 << 20) * vox / vox.sum()
    assert np.abs(n - quota).max() <= 256
    assert list(o.apportion([1, 1, 1], 768 * 3)) == [768, 768, 768]
    assert list(o.apportion([1, 1, 1], 1024)) == [512, 256, 256]  # tie goes to the lower id


def test_decode_coordinates_are_voxel_centers():
    x = o.voxel_center_coords((4, 2, 3))
    assert x.shape == (24, 3)
    np.testing.assert_array_equal(x[:4, 0], np.float32([0.125, 0.375, 0.625, 0.875]))
    np.testing.assert_array_equal(x[[0, 4], 1], np.float32([0.25, 0.75]))
    np.testing.assert_array_equal(x[[0, 8, 16], 2], np.float32([1 / 6, 0.5, 5 / 6]))


@pytest.mark.parametrize("vmin,vmax", [(-2.5, 4.0), (3.0, 3.0), (0.25, 0.5)])
def test_decode_denormalizes_with_the_block_range(vmin, vmax):
    """A model whose output is a known constant c decodes to vmin + c (vmax - vmin)
    (scale 1 for a constant block, vmax = vmin).  Construction: every table
    entry a (the trilinear weights sum to 1, so every feature is a), first
    layer 1/(L F) everywhere (each hidden unit sees a > 0, ReLU passes it),
    output layer 1/width: c = a."""
    enc, mlp = o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16)
    lay = o.layout(enc, mlp)
    a = 0.3
    p = np.empty(lay.n_params)
    p[:lay.n_table_params] = a
    (w1o, w1i), (woo, woi) = lay.mlp_shapes
    off1, off2 = lay.mlp_offsets
    p[off1:off1 + w1o * w1i] = 1.0 / w1i
    p[off2:off2 + woo * woi] = 1.0 / woi
    dims = (5, 3, 4)
    dec = o.decode(lay, p, dims, vmin, vmax)
    assert dec.shape == (4, 3, 5)
    want = vmin + a * ((vmax - vmin) if vmax > vmin else 1.0)
    np.testing.assert_allclose(dec, want, rtol=0, atol=1e-14)


def test_small_training_run_reduces_loss():
    n = 16
    vol = gaussian_sum_field(n, seed=1)
    lay = o.layout(o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16))
    p0 = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=0)
    params, losses, _ = o.train(lay, p0, vol, (n, n, n), 0, n_steps=40, batch=512, seed=1, opt=o.Optim(lr=1e-2))
    assert losses[-5:].mean() < 0.5 * losses[:5].mean()
    vmin, vmax = o.block_value_range(vol)
    dec = o.decode(lay, params, (n, n, n), vmin, vmax)
    sse, cnt = o.squared_error(dec, vol)
    assert o.psnr(sse, cnt) > 15.0
