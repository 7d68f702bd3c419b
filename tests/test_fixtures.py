"""The seeded input generators are deterministic and produce what they promise."""
import numpy as np

from fixtures import (adversarial_coords, cut_blocks, gaussian_sum_field, init_param_draws, kolmogorov_field,
                      uniform_coords, uneven_block_sizes)


def test_fields_are_seeded_and_normalized():
    a = gaussian_sum_field(16, seed=1)
    assert a.dtype == np.float32 and a.shape == (16, 16, 16)
    assert a.min() == 0.0 and a.max() == 1.0
    assert np.array_equal(a, gaussian_sum_field(16, seed=1))
    assert not np.array_equal(a, gaussian_sum_field(16, seed=2))
    k = kolmogorov_field(32, seed=2)
    assert k.shape == (32, 32, 32) and k.min() == 0.0 and k.max() == 1.0
    assert np.array_equal(k, kolmogorov_field(32, seed=2))


def test_kolmogorov_spectrum_slope():
    f = kolmogorov_field(64, seed=5).astype(np.float64)
    F = np.abs(np.fft.fftn(f - f.mean())) ** 2
    k = np.fft.fftfreq(64) * 64
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    shells = np.arange(4, 24)
    E = np.array([F[(kk >= s - 0.5) & (kk < s + 0.5)].sum() for s in shells])
    slope = np.polyfit(np.log(shells), np.log(E), 1)[0]
    assert abs(slope - (-5.0 / 3.0)) < 0.25


def test_cut_blocks_ghosts_are_periodic_neighbours():
    f = kolmogorov_field(24, seed=3)
    sizes = [np.array([10, 14]), np.array([12, 12]), np.array([8, 16])]
    blocks = cut_blocks(f, sizes, ghost=1)
    assert len(blocks) == 8
    b = blocks[0]
    assert b["dims"] == (10, 12, 8) and b["data"].shape == (10, 14, 12)
    np.testing.assert_array_equal(b["data"][1:-1, 1:-1, 1:-1], f[0:8, 0:12, 0:10])
    np.testing.assert_array_equal(b["data"][0, 1:-1, 1:-1], f[-1, 0:12, 0:10])  # periodic halo
    sx, sy, sz = uneven_block_sizes(4, 96, 160, seed=3)
    assert all(((s >= 96) & (s <= 160)).all() for s in (sx, sy, sz))


def test_param_and_coordinate_draws():
    p = init_param_draws(100, [(16, 8), (1, 16)], seed=0)
    assert p.shape == (100 + 128 + 16,) and p.dtype == np.float32
    assert np.abs(p[:100]).max() <= 1e-4
    assert np.abs(p[100:228]).max() <= np.sqrt(6 / 24) + 1e-7
    x = uniform_coords(1000, seed=1)
    assert x.dtype == np.float32 and (x >= 0).all() and (x < 1).all()
    a = adversarial_coords([4, 8])
    assert a.dtype == np.float32 and a.min() == 0.0 and a.max() == 1.0
