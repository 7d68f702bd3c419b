"""Pins of the oracle's encoding against things other than itself.

* resolution tables, entry counts and hash values: hand-computed golden values;
* dense level == torch grid_sample(align_corners=True) (a library routine);
* affine tables are reproduced exactly (closed form);
* vertex invariant on hashed levels;
* trilinear weights form a partition of unity;
* the backward is the exact adjoint of the forward.
"""
import json
import os

import numpy as np
import pytest
import torch

from fixtures import adversarial_coords, uniform_coords
from oracle import dvnr_oracle as o

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


CFG = {
    "c1_L4_base4_scale2_T12": (o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16)),
    "c2_L16_base16_finest256_T19": (o.Encoding(16, 2, 19, 16, 0.0, 256), o.MLP(2, 64)),
    "c3_L16_base16_finest160_T17": (o.Encoding(16, 2, 17, 16, 0.0, 160), o.MLP(2, 64)),
    "c5_L16_base16_finest128_T19": (o.Encoding(16, 2, 19, 16, 0.0, 128), o.MLP(2, 64)),
    "gradcheck_L3_base2_scale2_T6": (o.Encoding(3, 2, 6, 2, 2.0), o.MLP(1, 16)),
}


@pytest.mark.parametrize("name", list(CFG))
def test_resolution_tables_and_entries(name):
    g = _gold("encoding_tables.json")["resolutions"][name]
    lay = o.layout(*CFG[name])
    assert [l.R for l in lay.levels] == g["R"]
    assert lay.n_entries == g["entries"]
    assert sum(l.dense for l in lay.levels) == g["dense_levels"]
    # offsets are the running sums of level sizes
    assert [l.off for l in lay.levels] == list(np.cumsum([0] + [l.E for l in lay.levels])[:-1])


def test_param_count_c1():
    lay = o.layout(*CFG["c1_L4_base4_scale2_T12"])
    # 8768 entries x 2 features + 16x8 + 1x16 weights
    assert lay.n_params == 8768 * 2 + 16 * 8 + 16


def test_hash_golden():
    g = _gold("encoding_tables.json")["hash"]
    for case in g["cases"]:
        for k, h in zip(g["log2_T"], case["h"]):
            assert int(o.spatial_hash(np.array(case["v"]), 1 << k)) == h


def test_hash_x_prime_is_one():
    v = np.stack([np.arange(4096), np.zeros(4096, int), np.zeros(4096, int)], axis=1)
    assert np.array_equal(o.spatial_hash(v, 1 << 12), np.arange(4096))


def test_grid_position_edges():
    for R in (2, 3, 16, 19, 256):
        i0, t = o.grid_position(np.array([0.0, 1.0, np.nextafter(np.float32(1), np.float32(0))], np.float32), R)
        assert i0[0] == 0 and t[0] == 0.0
        assert i0[1] == R - 2 and t[1] == 1.0
        assert 0 <= i0[2] <= R - 2 and 0.0 <= t[2] <= 1.0
    # out-of-range inputs clamp
    i0, t = o.grid_position(np.array([-0.5, 1.5], np.float32), 8)
    assert (i0[0], t[0]) == (0, 0.0) and (i0[1], t[1]) == (6, 1.0)


def _dense_single(R, F=2, T_log2=None):
    T_log2 = T_log2 if T_log2 is not None else int(np.ceil(np.log2(R ** 3)))
    return o.layout(o.Encoding(1, F, T_log2, R, 1.0), o.MLP(1, 16))


@pytest.mark.parametrize("R", [2, 4, 7, 16])
def test_dense_level_matches_grid_sample(R):
    lay = _dense_single(R)
    assert lay.levels[0].dense
    rng = np.random.default_rng(R)
    params = rng.normal(size=lay.n_params)
    x = np.concatenate([uniform_coords(500, seed=R), adversarial_coords([R])])
    y = o.encode(lay, params, x)
    # table viewed as (z, y, x, F) because entry = x + R y + R^2 z, x fastest
    vol = torch.tensor(params[:lay.n_table_params].reshape(R, R, R, 2)).permute(3, 0, 1, 2)[None]
    # the oracle's position is the float32 product p = x * (R - 1); hand grid_sample that p
    p = (np.clip(x, 0, 1).astype(np.float32) * np.float32(R - 1)).astype(np.float64)
    grid = torch.tensor(2.0 * p / (R - 1) - 1.0).view(1, -1, 1, 1, 3)
    ref = torch.nn.functional.grid_sample(vol, grid, mode="bilinear", align_corners=True)
    ref = ref.view(2, -1).T.numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("R", [3, 9, 33])
def test_affine_table_is_reproduced(R):
    lay = _dense_single(R, F=1)
    a = np.array([0.3, -1.7, 2.2])
    c = np.arange(R, dtype=np.float64)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    table = a[0] * X + a[1] * Y + a[2] * Z + 0.25  # storage order z, y, x (x fastest)
    params = np.concatenate([table.ravel(), np.zeros(lay.n_params - lay.n_table_params)])
    x = np.concatenate([uniform_coords(1000, seed=3), adversarial_coords([R])])
    y = o.encode(lay, params, x)[:, 0]
    p = (np.clip(x, 0, 1).astype(np.float32) * np.float32(R - 1)).astype(np.float64)
    np.testing.assert_allclose(y, p @ a + 0.25, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("R,log2T", [(5, 6), (17, 10), (65, 12)])
def test_vertex_invariant_hashed(R, log2T):
    lay = o.layout(o.Encoding(1, 2, log2T, R, 1.0), o.MLP(1, 16))
    assert not lay.levels[0].dense
    rng = np.random.default_rng(R)
    params = rng.normal(size=lay.n_params)
    theta = params[:lay.n_table_params].reshape(-1, 2)
    v = rng.integers(0, R, size=(300, 3))
    x = (v / (R - 1)).astype(np.float32)  # exact: R - 1 is a power of two
    y = o.encode(lay, params, x)
    np.testing.assert_array_equal(y, theta[o.spatial_hash(v, 1 << log2T)])


def test_weights_partition_of_unity():
    lay = o.layout(*CFG["c2_L16_base16_finest256_T19"])
    x = uniform_coords(2000, seed=9)
    for lvl in lay.levels:
        idx, w = o.corner_indices_and_weights(x, lvl, lay.T)
        np.testing.assert_allclose(w.sum(axis=1), 1.0, rtol=0, atol=1e-14)
        assert (w >= 0).all() and idx.min() >= 0 and idx.max() < lvl.E


def test_multilevel_is_concatenation_of_levels():
    enc, mlp = CFG["c1_L4_base4_scale2_T12"]
    lay = o.layout(enc, mlp)
    rng = np.random.default_rng(0)
    params = rng.normal(size=lay.n_params)
    x = uniform_coords(300, seed=1)
    y = o.encode(lay, params, x)
    theta = params[:lay.n_table_params].reshape(-1, 2)
    for l, lvl in enumerate(lay.levels):
        single = o.layout(o.Encoding(1, 2, 12, lvl.R, 1.0), mlp)
        sub = np.concatenate([theta[lvl.off:lvl.off + lvl.E].ravel(), np.zeros(single.n_params - single.n_table_params)])
        np.testing.assert_allclose(y[:, 2 * l:2 * l + 2], o.encode(single, sub, x), rtol=0, atol=0)


def test_encode_backward_is_adjoint():
    enc, mlp = CFG["c1_L4_base4_scale2_T12"]
    lay = o.layout(enc, mlp)
    rng = np.random.default_rng(5)
    params = rng.normal(size=lay.n_params)
    x = np.concatenate([uniform_coords(700, seed=2), adversarial_coords([l.R for l in lay.levels])])
    dy = rng.normal(size=(x.shape[0], lay.in_dim))
    lhs = np.sum(o.encode(lay, params, x) * dy)
    g = o.encode_backward(lay, x, dy)
    rhs = np.dot(params[:lay.n_table_params], g)
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
    # and a few entries by central differences (the map is linear: exact up to rounding)
    for j in rng.choice(lay.n_table_params, size=10, replace=False):
        e = np.zeros(lay.n_params)
        e[j] = 1e-3
        fd = (np.sum(o.encode(lay, params + e, x) * dy) - np.sum(o.encode(lay, params - e, x) * dy)) / 2e-3
        assert abs(fd - g[j]) <= 1e-8 * max(1.0, abs(g[j]))
