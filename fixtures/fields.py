"""Seeded synthetic scalar fields and other inputs for the DVNR hot path.

The paper trains on simulation output and eight public volume datasets that are
not available here; these generators stand in for them with fields of the same
kind (smooth blobs plus oscillation, and turbulence-like fields with a
Kolmogorov k^-5/3 energy spectrum), normalized to [0, 1] globally as the paper
does before every compressor runs (Sec. V-B, pre-normalization).

Arrays are numpy, indexed [z, y, x] (x fastest in memory).
"""
from __future__ import annotations

import numpy as np


def _normalize01(f: np.ndarray) -> np.ndarray:
    lo, hi = float(f.min()), float(f.max())
    scale = 1.0 / (hi - lo) if hi > lo else 1.0
    return ((f - lo) * scale).astype(np.float32)


def gaussian_sum_field(n: int = 64, n_gauss: int = 8, seed: int = 1) -> np.ndarray:
    """Sum of random 3D Gaussians plus a 0.1-amplitude plane wave, in [0, 1].

    Draw order (PCG64, `seed`): centers U[0, n)^3 voxels, sigma U[4, 12] voxels,
    amplitudes U[0.5, 1], wave vector k U[1, 4]^3 (continuous).  The wave is
    0.1*sin(2*pi*k.x) with x = (i + 1/2)/n.  Computed in float64, min/max
    normalized, returned as float32 of shape (n, n, n).
    """
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, n, size=(n_gauss, 3))
    sigma = rng.uniform(4.0, 12.0, size=n_gauss)
    amp = rng.uniform(0.5, 1.0, size=n_gauss)
    k = rng.uniform(1.0, 4.0, size=3)
    c = np.arange(n, dtype=np.float64)  # voxel index; Gaussians live in voxel units
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    f = np.zeros((n, n, n), dtype=np.float64)
    for g in range(n_gauss):
        d2 = (x - centers[g, 0]) ** 2 + (y - centers[g, 1]) ** 2 + (z - centers[g, 2]) ** 2
        f += amp[g] * np.exp(-d2 / (2.0 * sigma[g] ** 2))
    u = (c + 0.5) / n
    uz, uy, ux = np.meshgrid(u, u, u, indexing="ij")
    f += 0.1 * np.sin(2.0 * np.pi * (k[0] * ux + k[1] * uy + k[2] * uz))
    return _normalize01(f)


def kolmogorov_field(n: int = 256, seed: int = 2, shape=None) -> np.ndarray:
    """Periodic turbulence-like field with shell energy E(k) ~ k^-5/3, in [0, 1].

    Random-phase Fourier modes with amplitude |k|^(-11/6) (so that the energy
    per spherical shell, |k|^2 * amplitude^2, falls as k^-5/3), the DC mode and
    modes beyond |k| = n/2 zeroed, synthesized with an inverse real FFT in
    float64.  `shape` (nz, ny, nx) overrides the cubic size; the cutoff then uses
    the smallest axis.
    """
    if shape is None:
        shape = (n, n, n)
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.rfftfreq(nx) * nx
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    kk = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    kmax = min(shape) / 2.0
    amp = np.zeros_like(kk)
    m = (kk > 0) & (kk <= kmax)
    amp[m] = kk[m] ** (-11.0 / 6.0)
    del KZ, KY, KX, kk
    phase = rng.uniform(0.0, 2.0 * np.pi, size=amp.shape)
    spec = amp * np.exp(1j * phase)
    del amp, phase
    f = np.fft.irfftn(spec, s=(nz, ny, nx))
    return _normalize01(f)


def kolmogorov_field_torch(shape, seed: int = 2, device="cuda"):
    """`kolmogorov_field` synthesized with torch.fft in float32 on `device`.

    Same recipe (random phases, amplitude |k|^(-11/6), DC and |k| > min(shape)/2
    zeroed, min/max normalized), for fields too large for a host FFT; the phases
    come from a torch generator, so the values differ from the numpy version.
    Returns a float32 tensor (nz, ny, nx) on `device`.
    """
    import torch
    nz, ny, nx = shape
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    kz = torch.fft.fftfreq(nz, device=device) * nz
    ky = torch.fft.fftfreq(ny, device=device) * ny
    kx = torch.fft.rfftfreq(nx, device=device) * nx
    kk = torch.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    kmax = min(shape) / 2.0
    amp = torch.where((kk > 0) & (kk <= kmax), kk.clamp_min(1e-12) ** (-11.0 / 6.0), torch.zeros_like(kk))
    del kk
    phase = torch.rand(amp.shape, generator=g, device=device) * (2.0 * np.pi)
    spec = torch.polar(amp, phase)
    del amp, phase
    f = torch.fft.irfftn(spec, s=(nz, ny, nx))
    del spec
    lo, hi = f.min(), f.max()
    return ((f - lo) / (hi - lo)).contiguous()


def advected_blobs_series_torch(n: int = 256, n_steps: int = 40, n_blobs: int = 16, seed: int = 4, device="cuda"):
    """Generator of the `advected_blobs_field` time series synthesized with torch on `device`.

    Blob parameters and trajectories are the numpy ones (same seed and draw
    order); each timestep's field is built with separable Gaussians in float32
    on the device.  Yields float32 tensors (n, n, n), clipped to [0, 1] after
    dividing by the sum of amplitudes.
    """
    import torch
    traj, sigma, amp = advected_blob_trajectories(n, n_steps, n_blobs, seed)
    c = torch.arange(n, device=device, dtype=torch.float32)
    for t in range(n_steps):
        f = torch.zeros((n, n, n), device=device, dtype=torch.float32)
        for g in range(n_blobs):
            cx, cy, cz = [float(v) for v in traj[t, g]]
            s2 = float(2.0 * sigma[g] ** 2)
            ds = []
            for cc in (cz, cy, cx):
                d = torch.abs(c - cc)
                d = torch.minimum(d, n - d)
                ds.append(torch.exp(-d * d / s2))
            f += float(amp[g]) * ds[0][:, None, None] * ds[1][None, :, None] * ds[2][None, None, :]
        yield torch.clamp(f / float(amp.sum()), 0.0, 1.0)


def advected_blob_trajectories(n: int = 256, n_steps: int = 40, n_blobs: int = 16, seed: int = 4):
    """Blob centers of every timestep [n_steps, n_blobs, 3] (voxels), sigma and amplitude.

    Same draws and RK4 advection as `advected_blobs_field`."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, n, size=(n_blobs, 3))
    sigma = rng.uniform(8.0, 16.0, size=n_blobs)
    amp = rng.uniform(0.5, 1.0, size=n_blobs)
    modes = []
    while len(modes) < 4:
        kv = rng.integers(-3, 4, size=3)
        if 0 < np.linalg.norm(kv) <= 3:
            modes.append(kv.astype(np.float64))
    avec = rng.normal(size=(4, 3))
    phs = rng.uniform(0.0, 2.0 * np.pi, size=4)

    def vel(p):
        u = np.zeros_like(p)
        for kv, a, ph in zip(modes, avec, phs):
            arg = 2.0 * np.pi * (p @ kv) / n + ph
            grad = (2.0 * np.pi / n) * np.cos(arg)[:, None] * kv[None, :]
            u += np.cross(grad, a[None, :])
        return u

    probe = rng.uniform(0.0, n, size=(4096, 3))
    umax = np.abs(vel(probe)).max()
    scale = 2.0 / umax if umax > 0 else 1.0
    traj = np.empty((n_steps, n_blobs, 3))
    for t in range(n_steps):
        traj[t] = centers
        k1 = scale * vel(centers)
        k2 = scale * vel(centers + 0.5 * k1)
        k3 = scale * vel(centers + 0.5 * k2)
        k4 = scale * vel(centers + k3)
        centers = np.mod(centers + (k1 + 2 * k2 + 2 * k3 + k4) / 6.0, n)
    return traj, sigma, amp


def advected_blobs_field(n: int = 256, n_steps: int = 40, n_blobs: int = 16, seed: int = 4, step: int = 0) -> np.ndarray:
    """One timestep of Gaussian blobs advected by a seeded divergence-free flow.

    Blob centers (voxels) U[0, n)^3, sigma U[8, 16], amplitude U[0.5, 1].  The
    velocity is the curl of a vector potential made of 4 random Fourier modes
    with |k| <= 3, scaled so that max|u| is about 2 voxels per timestep; centers
    move by classical RK4 with periodic wrap, distances use the minimum image.
    Returns the field at timestep `step` (0 <= step < n_steps), normalized to
    [0, 1] with the global range of step 0 so that a time series stays
    comparable.
    """
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, n, size=(n_blobs, 3))
    sigma = rng.uniform(8.0, 16.0, size=n_blobs)
    amp = rng.uniform(0.5, 1.0, size=n_blobs)
    modes = []
    while len(modes) < 4:
        kv = rng.integers(-3, 4, size=3)
        if 0 < np.linalg.norm(kv) <= 3:
            modes.append(kv.astype(np.float64))
    avec = rng.normal(size=(4, 3))
    phs = rng.uniform(0.0, 2.0 * np.pi, size=4)

    def vel(p):  # p [m, 3] in voxels (x, y, z); u = curl A, A = sum a_j sin(2 pi k_j.p/n + phi_j)
        u = np.zeros_like(p)
        for kv, a, ph in zip(modes, avec, phs):
            arg = 2.0 * np.pi * (p @ kv) / n + ph
            grad = (2.0 * np.pi / n) * np.cos(arg)[:, None] * kv[None, :]  # d/dp of sin(arg)
            u += np.cross(grad, a[None, :])
        return u

    probe = rng.uniform(0.0, n, size=(4096, 3))
    umax = np.abs(vel(probe)).max()
    scale = 2.0 / umax if umax > 0 else 1.0
    for _ in range(step):
        k1 = scale * vel(centers)
        k2 = scale * vel(centers + 0.5 * k1)
        k3 = scale * vel(centers + 0.5 * k2)
        k4 = scale * vel(centers + k3)
        centers = np.mod(centers + (k1 + 2 * k2 + 2 * k3 + k4) / 6.0, n)
    c = np.arange(n, dtype=np.float64)
    f = np.zeros((n, n, n), dtype=np.float64)
    for g in range(n_blobs):
        dx = np.abs(c - centers[g, 0]); dx = np.minimum(dx, n - dx)
        dy = np.abs(c - centers[g, 1]); dy = np.minimum(dy, n - dy)
        dz = np.abs(c - centers[g, 2]); dz = np.minimum(dz, n - dz)
        s2 = 2.0 * sigma[g] ** 2
        f += amp[g] * (np.exp(-dz * dz / s2)[:, None, None] * np.exp(-dy * dy / s2)[None, :, None]
                       * np.exp(-dx * dx / s2)[None, None, :])
    return np.clip(f / amp.sum(), 0.0, 1.0).astype(np.float32)


def uneven_block_sizes(n_per_axis: int = 4, lo: int = 96, hi: int = 160, seed: int = 3):
    """Per-axis block extents U{lo..hi} for a rectilinear n x n x n cut.

    Returns three integer arrays (x, y, z extents), drawn in that order.
    """
    rng = np.random.default_rng(seed)
    return [rng.integers(lo, hi + 1, size=n_per_axis) for _ in range(3)]


def cut_blocks(field: np.ndarray, sizes_xyz, ghost: int = 1, periodic: bool = True):
    """Cut a rectilinear partition of `field` into blocks with a ghost layer.

    `sizes_xyz` holds the owned extents along x, y and z (they must sum to the
    field's extent along that axis).  Each block is returned as a dict with
    `dims` (owned nx, ny, nz), `ghost`, `origin` (owned x0, y0, z0) and `data`,
    a float32 array of shape (nz + 2g, ny + 2g, nx + 2g) whose halo is taken
    from the neighbouring voxels (periodic wrap at the domain faces, or edge
    replication when `periodic` is False).  Blocks are ordered x fastest.
    """
    sx, sy, sz = [np.asarray(s, dtype=np.int64) for s in sizes_xyz]
    nz, ny, nx = field.shape
    assert sx.sum() == nx and sy.sum() == ny and sz.sum() == nz
    ox = np.concatenate([[0], np.cumsum(sx)[:-1]])
    oy = np.concatenate([[0], np.cumsum(sy)[:-1]])
    oz = np.concatenate([[0], np.cumsum(sz)[:-1]])
    mode = "wrap" if periodic else "edge"
    padded = np.pad(field, ghost, mode=mode) if ghost > 0 else field
    blocks = []
    for iz in range(len(sz)):
        for iy in range(len(sy)):
            for ix in range(len(sx)):
                x0, y0, z0 = int(ox[ix]), int(oy[iy]), int(oz[iz])
                bx, by, bz = int(sx[ix]), int(sy[iy]), int(sz[iz])
                data = padded[z0:z0 + bz + 2 * ghost, y0:y0 + by + 2 * ghost, x0:x0 + bx + 2 * ghost]
                blocks.append(dict(dims=(bx, by, bz), ghost=ghost, origin=(x0, y0, z0),
                                   data=np.ascontiguousarray(data, dtype=np.float32)))
    return blocks


def init_param_draws(n_table_params: int, mlp_shapes, seed: int = 0, table_scale: float = 1e-4) -> np.ndarray:
    """Initial parameter vector of one block, float32.

    Table parameters are U(-table_scale, table_scale); each weight matrix of
    shape (fan_out, fan_in) is Glorot-uniform, U(-a, a) with
    a = sqrt(6 / (fan_in + fan_out)).  Draws come from PCG64(`seed`) in storage
    order: the tables first, then the matrices in layer order, row-major.
    """
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-table_scale, table_scale, size=n_table_params)]
    for fan_out, fan_in in mlp_shapes:
        a = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-a, a, size=fan_out * fan_in))
    return np.concatenate(parts).astype(np.float32)


def uniform_coords(n: int, seed: int = 0) -> np.ndarray:
    """n coordinates uniform in [0, 1)^3 as float32 multiples of 2^-24, shape [n, 3] (x, y, z)."""
    rng = np.random.default_rng(seed)
    u = rng.integers(0, 1 << 24, size=(n, 3), dtype=np.int64)
    return (u.astype(np.float64) * 2.0 ** -24).astype(np.float32)


def adversarial_coords(resolutions) -> np.ndarray:
    """Coordinates on the faces, at 1, just below 1 and on lattice vertices of every level.

    For each resolution R the set contains v/(R-1) for a few vertices v, and the
    float32 neighbours of those values; plus 0, 1 and nextafter(1, 0) on every
    axis.  Returned as float32 [m, 3].
    """
    vals = {0.0, 1.0, float(np.nextafter(np.float32(1.0), np.float32(0.0)))}
    for R in resolutions:
        for v in (0, 1, R // 2, R - 2, R - 1):
            x = np.float32(v / (R - 1))
            vals.add(float(x))
            vals.add(float(np.nextafter(x, np.float32(0.0))))
            vals.add(float(np.nextafter(x, np.float32(2.0))))
    v = np.array(sorted(x for x in vals if 0.0 <= x <= 1.0), dtype=np.float32)
    rng = np.random.default_rng(12345)
    m = len(v)
    idx = np.stack([np.arange(m), rng.permutation(m), rng.permutation(m)], axis=1)
    return np.ascontiguousarray(v[idx], dtype=np.float32)
