"""Pins of the oracle's boundary-centered sampler and L1 loss (Sec. III-C, Eqs. (2)-(3)).

* the distance of a boundary sample to the nearest face against its closed-form
  distribution (half-normal distance to the chosen face, two uniform
  tangential coordinates), by a Kolmogorov-Smirnov test;
* the nearest-face label uniform over the six faces (chi-square), the
  tangential coordinates uniform (KS);
* the first (1 - lambda) n samples of a step identical to the uniform draws;
* the rounding of lambda * n;
* the L1 loss gradient against central finite differences.
"""
import numpy as np
import pytest
from scipy import special, stats

from fixtures import init_param_draws
from oracle import dvnr_oracle as o


def _nearest_face(x):
    dist = np.concatenate([x, 1.0 - x], axis=1).astype(np.float64)  # faces: low x,y,z then high x,y,z
    face = np.argmin(dist, axis=1)
    return face, dist[np.arange(len(x)), face]


@pytest.mark.parametrize("sigma", [0.005, 0.05])
def test_boundary_distance_distribution(sigma):
    x = o.boundary_coords(seed=11, block=3, step=5, n=200_000, first=0, sigma=sigma)
    assert x.dtype == np.float32 and x.min() >= 0.0 and x.max() <= 1.0
    _, s = _nearest_face(x)

    # nearest-face distance m = min(d, t1, 1 - t1, t2, 1 - t2): d half-normal,
    # t uniform, so P(m > s) = (1 - erf(s / (sigma sqrt 2))) (1 - 2 s)^2
    def cdf(s):
        s = np.asarray(s, dtype=np.float64)
        return 1.0 - (1.0 - special.erf(s / (sigma * np.sqrt(2.0)))) * (1.0 - 2.0 * s) ** 2

    assert stats.kstest(s, cdf).pvalue > 1e-3


def test_boundary_faces_and_tangents_uniform():
    n = 120_000
    x = o.boundary_coords(seed=5, block=0, step=1, n=n, first=1000, sigma=0.005)
    face, _ = _nearest_face(x)
    counts = np.bincount(face, minlength=6)
    assert stats.chisquare(counts).pvalue > 1e-3
    axis = face % 3
    for a in range(3):
        rows = x[axis == a]
        for t in [b for b in range(3) if b != a]:
            assert stats.kstest(rows[:, t], "uniform").pvalue > 1e-3


def test_step_coords_prefix_is_uniform_draw():
    n, nb = 4096, o.boundary_count(4096, 0.15)
    x = o.step_coords(9, 2, 7, n, nb, 0.005)
    np.testing.assert_array_equal(x[:n - nb], o.training_coords(9, 2, 7, n - nb))
    np.testing.assert_array_equal(x[n - nb:], o.boundary_coords(9, 2, 7, nb, n - nb, 0.005))
    np.testing.assert_array_equal(o.step_coords(9, 2, 7, n, 0), o.training_coords(9, 2, 7, n))


def test_boundary_count_rounds_half_up():
    assert o.boundary_count(4096, 0.15) == 614       # 614.4
    assert o.boundary_count(1 << 18, 0.15) == 39322  # 39321.6
    assert o.boundary_count(10, 0.25) == 3           # 2.5
    assert o.boundary_count(1000, 0.0) == 0


def test_l1_loss_gradient_matches_finite_differences():
    enc, mlp = o.Encoding(3, 2, 6, 2, 2.0), o.MLP(1, 16)
    lay = o.layout(enc, mlp)
    params = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=4).astype(np.float64)
    params[:lay.n_table_params] *= 3e3
    rng = np.random.default_rng(6)
    x = (0.1 + 0.8 * rng.random((32, 3))).astype(np.float32)
    out = o.infer(lay, params, x)
    # residuals bounded away from 0 so that no finite-difference step crosses the kink
    tgt = out + rng.choice([-1.0, 1.0], 32) * rng.uniform(0.05, 0.3, 32)
    L, g, _ = o.loss_and_grad(lay, params, x, tgt, "l1")
    assert abs(L - np.mean(np.abs(out - tgt))) < 1e-14
    h = 1e-6
    pick = np.concatenate([rng.choice(lay.n_table_params, 12, replace=False),
                           lay.n_table_params + rng.choice(lay.n_params - lay.n_table_params, 12, replace=False)])
    for j in pick:
        e = np.zeros_like(params)
        e[j] = h
        fd = (o.loss_and_grad(lay, params + e, x, tgt, "l1")[0]
              - o.loss_and_grad(lay, params - e, x, tgt, "l1")[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1e-3, abs(g[j])), (j, fd, g[j])
