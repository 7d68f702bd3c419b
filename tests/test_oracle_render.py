"""Pins of the oracle's volume renderer (Sec. IV, direct volume rendering).

* camera rays: unit length; the center pixel looks at the target; the
  top-center and right-center pixels sit at the closed-form angles
  atan((1 - 1/H) tan(fovy/2)) and atan((1 - 1/W) tan(fovy/2) W/H);
* ray/cube intersection against a brute-force inside test along each ray;
* the transfer function against numpy.interp per channel;
* a constant field: every pixel equals the closed form A = 1 - (1 - alpha)^n,
  C = rgb A with n the number of samples in the chord;
* front-to-back compositing against the back-to-front "over" recursion on the
  same samples; early termination stops at the first sample reaching the limit.
"""
import numpy as np
import pytest

from fixtures import init_param_draws
from oracle import dvnr_oracle as o

CAM = o.Camera(eye=(1.9, 1.4, 2.3), center=(0.5, 0.45, 0.55), up=(0.0, 1.0, 0.0), fovy_deg=38.0, width=21, height=15)


def test_camera_rays_geometry():
    eye, d = o.camera_rays(CAM)
    assert d.dtype == np.float32
    np.testing.assert_allclose(np.linalg.norm(d.astype(np.float64), axis=1), 1.0, atol=2e-7)
    fw = np.subtract(CAM.center, CAM.eye)
    fw = fw / np.linalg.norm(fw)
    W, H = CAM.width, CAM.height
    center = d[(H // 2) * W + W // 2].astype(np.float64)
    np.testing.assert_allclose(center, fw, atol=2e-7)
    t = np.tan(np.radians(CAM.fovy_deg) / 2)
    top = d[0 * W + W // 2].astype(np.float64)
    right = d[(H // 2) * W + W - 1].astype(np.float64)
    assert abs(np.arccos(np.clip(top @ fw, -1, 1)) - np.arctan((1 - 1 / H) * t)) < 1e-6
    assert abs(np.arccos(np.clip(right @ fw, -1, 1)) - np.arctan((1 - 1 / W) * t * W / H)) < 1e-6
    # row 0 is the top: its rays lean towards +up
    assert top[1] > center[1] and right @ np.cross(fw, [0, 1, 0]) > 0


def test_ray_box_against_brute_force():
    eye, d = o.camera_rays(CAM)
    t0, t1 = o.ray_box(eye, d)
    ts = np.arange(0.0, 6.0, 2e-4)
    for r in range(0, d.shape[0], 7):
        x = eye[None, :].astype(np.float64) + ts[:, None] * d[r].astype(np.float64)[None, :]
        inside = np.all((x >= 0) & (x <= 1), axis=1)
        if not inside.any():
            assert not t1[r] > t0[r]
            continue
        assert t1[r] > t0[r]
        assert abs(ts[inside][0] - t0[r]) <= 3e-4 and abs(ts[inside][-1] - t1[r]) <= 3e-4


def test_transfer_matches_interp():
    rng = np.random.default_rng(4)
    tf = rng.random((7, 4))
    v = rng.uniform(-0.5, 2.5, 500)
    got = o.transfer(tf, 0.2, 1.7, v)
    xs = np.linspace(0.2, 1.7, 7)
    for c in range(4):
        np.testing.assert_allclose(got[:, c], np.interp(v, xs, tf[:, c]), atol=1e-12)


def _const_layout():
    lay = o.layout(o.Encoding(3, 2, 8, 4, 2.0), o.MLP(1, 16))
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=3).astype(np.float64)
    p[:lay.n_table_params] = 0.37  # every entry equal: the encoding, hence the INR, is constant
    return lay, p


def test_constant_field_closed_form():
    lay, p = _const_layout()
    v = 0.2 + 0.5 * o.infer(lay, p, np.array([[0.3, 0.3, 0.3]], np.float32))[0]
    tf = np.array([[0.9, 0.1, 0.2, 0.0], [0.2, 0.6, 0.8, 0.7]])
    dt, ref = 1.0 / 37, 1.0 / 100
    img = o.render(lay, p, 0.2, 0.7, CAM, tf, -1.0, 1.0, dt, ref)
    c = o.transfer(tf, -1.0, 1.0, np.array([v]))[0]
    alpha = 1 - (1 - c[3]) ** (dt / ref)
    eye, d = o.camera_rays(CAM)
    t0, t1 = o.ray_box(eye, d)
    chord = np.where(t1 > t0, t1.astype(np.float64) - t0, 0.0)
    n = np.maximum(np.ceil(chord / dt - 0.5), 0)  # samples k with (k + 1/2) dt < chord
    away = np.abs(chord / dt - 0.5 - np.round(chord / dt - 0.5)) > 1e-4
    A = 1 - (1 - alpha) ** n
    got = img.reshape(-1, 4)
    np.testing.assert_allclose(got[away, 3], A[away], atol=1e-12)
    np.testing.assert_allclose(got[away, :3], c[None, :3] * A[away, None], atol=1e-12)
    assert (n[away] > 0).sum() > 20


def test_front_to_back_equals_over_recursion_and_early_stop():
    lay = o.layout(o.Encoding(3, 2, 8, 4, 2.0), o.MLP(1, 16))
    p = init_param_draws(lay.n_table_params, lay.mlp_shapes, seed=5).astype(np.float64)
    p[:lay.n_table_params] *= 4e3
    tf = np.random.default_rng(2).random((6, 4)) * [1, 1, 1, 0.6]
    lo, hi, dt, ref = -0.2, 1.2, 1.0 / 29, 1.0 / 50
    img = o.render(lay, p, 0.0, 1.0, CAM, tf, lo, hi, dt, ref)
    stop = o.render(lay, p, 0.0, 1.0, CAM, tf, lo, hi, dt, ref, alpha_stop=0.6)
    eye, d = o.camera_rays(CAM)
    t0, t1 = o.ray_box(eye, d)
    checked = 0
    for r in range(0, d.shape[0], 5):
        if not t1[r] > t0[r]:
            assert np.all(img.reshape(-1, 4)[r] == 0)
            continue
        ks = []
        k = 0
        while True:
            tk, ok = o.sample_params(t0[r:r + 1], t1[r:r + 1], dt, k)
            if not ok[0]:
                break
            ks.append(tk[0])
            k += 1
        x = (eye[None, :] + (np.array(ks, np.float32)[:, None] * d[r][None, :]).astype(np.float32)).astype(np.float32)
        c = o.transfer(tf, lo, hi, o.infer(lay, p, x))
        a = 1 - (1 - c[:, 3]) ** (dt / ref)
        C, A = np.zeros(3), 0.0
        for i in reversed(range(len(ks))):  # back to front: C = a c + (1 - a) C_behind
            C = a[i] * c[i, :3] + (1 - a[i]) * C
            A = a[i] + (1 - a[i]) * A
        np.testing.assert_allclose(img.reshape(-1, 4)[r], np.r_[C, A], atol=1e-12)
        # early termination: the front-to-back prefix up to the first sample with A >= 0.6
        Cf, Af = np.zeros(3), 0.0
        for i in range(len(ks)):
            Cf += (1 - Af) * a[i] * c[i, :3]
            Af += (1 - Af) * a[i]
            if Af >= 0.6:
                break
        np.testing.assert_allclose(stop.reshape(-1, 4)[r], np.r_[Cf, Af], atol=1e-12)
        checked += 1
    assert checked > 10
