"""Plain float64 CPU oracle of the DVNR training and decoding hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module; only the tests, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code with the HIP library: it is written from the
paper (Sec. III, Eq. (1)-(3)) and from the instant neural graphics primitives
encoding that the paper builds on (Muller et al. 2022, the multiresolution hash
encoding the paper cites in Sec. III), step by step, without blocking, fusion or
reordering.

What it computes, per partition block (one implicit neural representation,
"INR", per block; Sec. III-A):

* resolution table and storage of the multiresolution grid (`layout`);
* the spatial hash / dense index of every cell corner and the trilinear corner
  weights (`corner_indices_and_weights`);
* the encoding y = concat_l sum_c w_c * theta_l[idx_c] (`encode`);
* the bias-free ReLU MLP and its backward (`mlp_forward`, `mlp_backward`);
* uniform sampling with a counter-based generator (Philox4x32-10, Salmon et
  al., SC'11) and trilinear ground-truth fetch in cell-centered convention with
  per-block min/max normalization (`training_coords`, `sample_volume`);
* boundary-centered half-normal samples (Sec. III-C, Eq. (2)) mixed into a
  step's batch (`boundary_coords`, `step_coords`);
* the step budget and the moving-average early termination (Sec. III-B)
  (`max_train_steps`, `should_stop`, `train_until`);
* the L2 or L1 loss (Sec. III-C, Eq. (3)), the encoding backward
  (scatter-add), Adam with L2 weight decay (Sec. III-F) (`train_step`, `adam`);
* decoding at voxel centers and PSNR over owned voxels (`decode`, `psnr`);
* the sliding-window cache needs no oracle of its own (a snapshot must decode
  exactly as the live model did);
* direct volume rendering of a block's INR by front-to-back ray marching
  (`camera_rays`, `ray_box`, `transfer`, `render`; Sec. IV).

Readings of points the paper leaves open are listed in the design notes and
restated at each function.  Floating point: float64 throughout, except the
index path (position p = x * (R - 1) is one float32 multiply, so that integer
corner indices are defined exactly as the GPU computes them) and the decode
coordinates (float32 voxel centers).

Parity status: every function here is pinned by a test in tests/test_oracle_*.py
against something other than itself (closed forms, invariants, torch library
routines, finite differences, published Philox known-answer vectors).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Spatial-hash primes of the multiresolution hash encoding (x gets 1).
PRIME_X = 1
PRIME_Y = 2654435761
PRIME_Z = 805459861
MASK32 = 0xFFFFFFFF


# --------------------------------------------------------------------------
# Configuration and storage layout (Sec. III; multiresolution grid of the cited
# encoding; storage as R x R x R x F dense arrays or T x F hash tables, Sec. III-D)
# --------------------------------------------------------------------------
@dataclass
class Encoding:
    n_levels: int
    n_features: int
    log2_table_size: int
    base_resolution: int
    per_level_scale: float = 0.0  # 0 -> derived from finest_resolution
    finest_resolution: int = 0


@dataclass
class MLP:
    n_hidden_layers: int
    width: int
    out_dim: int = 1


@dataclass
class Level:
    R: int
    dense: bool
    E: int
    off: int


@dataclass
class Layout:
    enc: Encoding
    mlp: MLP
    levels: list = field(default_factory=list)
    n_entries: int = 0
    n_table_params: int = 0
    mlp_shapes: list = field(default_factory=list)  # (fan_out, fan_in) per layer
    mlp_offsets: list = field(default_factory=list)
    n_params: int = 0

    @property
    def T(self) -> int:
        return 1 << self.enc.log2_table_size

    @property
    def in_dim(self) -> int:
        return self.enc.n_levels * self.enc.n_features


def resolutions(enc: Encoding) -> list:
    """Per-level vertex resolution R_l = floor(R_0 * b^l + 1e-6).

    b is the per-level scale when given, else exp(ln(R_finest / R_0) / (L - 1)),
    the geometric growth of the cited multiresolution encoding.  R counts grid
    vertices per axis (the paper stores a dense level as an R x R x R x F
    array, Sec. III-D); the 1e-6 guards against b^l landing just below an
    integer.  Every level needs R >= 2.
    """
    L = enc.n_levels
    if enc.per_level_scale and enc.per_level_scale > 0:
        b = float(enc.per_level_scale)
    elif L == 1:
        b = 1.0
    else:
        b = float(np.exp(np.log(enc.finest_resolution / enc.base_resolution) / (L - 1)))
    R = [int(np.floor(enc.base_resolution * b ** l + 1e-6)) for l in range(L)]
    if min(R) < 2:
        raise ValueError("every level needs at least 2 vertices per axis")
    return R


def layout(enc: Encoding, mlp: MLP) -> Layout:
    """Storage layout of one block's parameter vector.

    A level is dense when its R^3 vertices fit the table size T (R^3 <= T) and
    then holds E = R^3 entries indexed x + R*y + R^2*z; otherwise it is a hash
    table of E = T entries.  Levels are concatenated (entry offsets off_l), each
    entry holds F features (feature-minor), then the weight matrices follow in
    layer order, each row-major [fan_out][fan_in]: W_1 [width][L*F], the hidden
    [width][width] matrices, W_out [out_dim][width].
    """
    T = 1 << enc.log2_table_size
    lay = Layout(enc=enc, mlp=mlp)
    off = 0
    for R in resolutions(enc):
        dense = R ** 3 <= T
        E = R ** 3 if dense else T
        lay.levels.append(Level(R=R, dense=dense, E=E, off=off))
        off += E
    lay.n_entries = off
    lay.n_table_params = off * enc.n_features
    shapes = [(mlp.width, enc.n_levels * enc.n_features)]
    shapes += [(mlp.width, mlp.width)] * (mlp.n_hidden_layers - 1)
    shapes += [(mlp.out_dim, mlp.width)]
    lay.mlp_shapes = shapes
    pos = lay.n_table_params
    for fo, fi in shapes:
        lay.mlp_offsets.append(pos)
        pos += fo * fi
    lay.n_params = pos
    return lay


def mlp_weights(lay: Layout, params: np.ndarray) -> list:
    """Views of the weight matrices inside a block parameter vector (float64 copies)."""
    out = []
    for (fo, fi), off in zip(lay.mlp_shapes, lay.mlp_offsets):
        out.append(np.asarray(params[off:off + fo * fi], dtype=np.float64).reshape(fo, fi))
    return out


# --------------------------------------------------------------------------
# Encoding (Sec. III: multiresolution hash encoding, "latent grids")
# --------------------------------------------------------------------------
def grid_position(x: np.ndarray, R: int):
    """Cell origin and fraction on a level of R vertices per axis.

    x is clamped to [0, 1]; p = x * (R - 1) is ONE float32 multiply (round to
    nearest, no fused multiply-add), i0 = min(floor(p), R - 2) so that x = 1
    falls in the last cell with fraction 1, and t = p - i0 (exact in float32).
    Returns i0 (int64, shape like x) and t (float64).
    """
    x32 = np.clip(np.asarray(x, dtype=np.float32), np.float32(0.0), np.float32(1.0))
    s = np.float32(R - 1)
    p = (x32 * s).astype(np.float32)
    i0 = np.minimum(np.floor(p).astype(np.int64), R - 2)
    t = (p - i0.astype(np.float32)).astype(np.float32)
    return i0, t.astype(np.float64)


def spatial_hash(v: np.ndarray, T: int) -> np.ndarray:
    """XOR of coordinate-times-prime, modulo 2^32, masked to the table size T (a power of 2)."""
    v = np.asarray(v, dtype=np.uint64)
    h = (v[..., 0] * np.uint64(PRIME_X)) & np.uint64(MASK32)
    h ^= (v[..., 1] * np.uint64(PRIME_Y)) & np.uint64(MASK32)
    h ^= (v[..., 2] * np.uint64(PRIME_Z)) & np.uint64(MASK32)
    return (h & np.uint64(T - 1)).astype(np.int64)


def corner_indices_and_weights(x: np.ndarray, lvl: Level, T: int):
    """Entry indices (within the level) and trilinear weights of the 8 cell corners.

    Corner c = cx + 2 cy + 4 cz sits at vertex v = i0 + (cx, cy, cz).  Dense
    level: index vx + R vy + R^2 vz.  Hashed level: spatial_hash(v).  Weight
    w_c = prod over axes of (t if the corner bit is set else 1 - t).
    Returns idx [n, 8] int64, w [n, 8] float64.
    """
    x = np.asarray(x, dtype=np.float32).reshape(-1, 3)
    i0, t = grid_position(x, lvl.R)  # [n, 3]
    n = x.shape[0]
    idx = np.empty((n, 8), dtype=np.int64)
    w = np.empty((n, 8), dtype=np.float64)
    for c in range(8):
        bits = np.array([(c >> a) & 1 for a in range(3)], dtype=np.int64)
        v = i0 + bits[None, :]
        if lvl.dense:
            idx[:, c] = v[:, 0] + lvl.R * v[:, 1] + lvl.R * lvl.R * v[:, 2]
        else:
            idx[:, c] = spatial_hash(v, T)
        wc = np.ones(n, dtype=np.float64)
        for a in range(3):
            wc *= t[:, a] if bits[a] else (1.0 - t[:, a])
        w[:, c] = wc
    return idx, w


def encode(lay: Layout, params: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Encoding y[n, L*F]: y[l*F + f] = sum_c w_c * theta[(off_l + idx_c) * F + f]."""
    F = lay.enc.n_features
    theta = np.asarray(params[:lay.n_table_params], dtype=np.float64).reshape(lay.n_entries, F)
    x = np.asarray(x, dtype=np.float32).reshape(-1, 3)
    y = np.zeros((x.shape[0], lay.in_dim), dtype=np.float64)
    for l, lvl in enumerate(lay.levels):
        idx, w = corner_indices_and_weights(x, lvl, lay.T)
        for c in range(8):
            y[:, l * F:(l + 1) * F] += w[:, c:c + 1] * theta[lvl.off + idx[:, c]]
    return y


def encode_backward(lay: Layout, x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """Gradient of the table parameters: scatter-add of w_c * dy into every corner entry.

    Colliding corners (two samples, or two corners of one sample, landing on the
    same hash entry) accumulate.  Returns a vector of length n_table_params.
    """
    F = lay.enc.n_features
    g = np.zeros((lay.n_entries, F), dtype=np.float64)
    x = np.asarray(x, dtype=np.float32).reshape(-1, 3)
    dy = np.asarray(dy, dtype=np.float64).reshape(x.shape[0], lay.in_dim)
    for l, lvl in enumerate(lay.levels):
        idx, w = corner_indices_and_weights(x, lvl, lay.T)
        for c in range(8):
            np.add.at(g, lvl.off + idx[:, c], w[:, c:c + 1] * dy[:, l * F:(l + 1) * F])
    return g.reshape(-1)


# --------------------------------------------------------------------------
# MLP (Sec. III: small MLP with ReLU between layers; no biases)
# --------------------------------------------------------------------------
def mlp_forward(weights: list, y: np.ndarray):
    """o = W_out relu(W_K ... relu(W_1 y)).  Returns o [n, out_dim] and the list
    of layer inputs [y, h_1, ..., h_K] needed by the backward."""
    h = np.asarray(y, dtype=np.float64)
    acts = [h]
    for W in weights[:-1]:
        h = np.maximum(h @ W.T, 0.0)
        acts.append(h)
    o = h @ weights[-1].T
    return o, acts


def mlp_backward(weights: list, acts: list, do: np.ndarray):
    """Backward of `mlp_forward`.  ReLU'(0) = 0 (a unit is active iff its output > 0).

    Returns (dy [n, in_dim], [dW_1, ..., dW_out])."""
    do = np.asarray(do, dtype=np.float64).reshape(acts[-1].shape[0], -1)
    dWs = [None] * len(weights)
    dWs[-1] = do.T @ acts[-1]
    dh = do @ weights[-1]
    for k in range(len(weights) - 2, -1, -1):
        dz = dh * (acts[k + 1] > 0.0)
        dWs[k] = dz.T @ acts[k]
        dh = dz @ weights[k]
    return dh, dWs


# --------------------------------------------------------------------------
# Sampling (Sec. III-B: uniform stochastic sampling + trilinear interpolation of
# the reference volume; Fig. 2 / Sec. III-C: cell-centered voxels, ghost layer)
# --------------------------------------------------------------------------
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).

    Each round: two 32x32->64 multiplies of counter words 0 and 2 by the
    multipliers M0, M1; the new counter is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
    the key is bumped by the Weyl constants (W0, W1) between rounds.
    ctr: [n, 4] uint32-valued; key: (k0, k1).  Returns [n, 4] uint32.
    """
    c = np.asarray(ctr, dtype=np.uint64).reshape(-1, 4).copy()
    k0 = np.uint64(int(key[0]) & MASK32)
    k1 = np.uint64(int(key[1]) & MASK32)
    m32 = np.uint64(MASK32)
    for r in range(10):
        if r > 0:
            k0 = np.uint64((int(k0) + PHILOX_W0) & MASK32)
            k1 = np.uint64((int(k1) + PHILOX_W1) & MASK32)
        p0 = c[:, 0] * np.uint64(PHILOX_M0)
        p1 = c[:, 2] * np.uint64(PHILOX_M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & m32
        hi1, lo1 = p1 >> np.uint64(32), p1 & m32
        c = np.stack([hi1 ^ c[:, 1] ^ k0, lo1, hi0 ^ c[:, 3] ^ k1, lo0], axis=1)
    return c.astype(np.uint32)


COORD_TAG = 0x44564E52  # fourth counter word of training-coordinate draws


def training_coords(seed: int, block: int, step: int, n: int, first: int = 0) -> np.ndarray:
    """Uniform training coordinates of one block at one optimizer step.

    Sample i (i = first .. first + n - 1) draws Philox4x32-10 with counter
    (i, step, block, COORD_TAG) and key (seed low word, seed high word); its
    first three output words u give x = (u >> 8) * 2^-24 in [0, 1), exactly
    representable in float32.  Returns float32 [n, 3] (x, y, z).
    """
    i = np.arange(first, first + n, dtype=np.uint64)
    ctr = np.stack([i & np.uint64(MASK32), np.full_like(i, step & MASK32),
                    np.full_like(i, block & MASK32), np.full_like(i, COORD_TAG)], axis=1)
    u = philox4x32_10(ctr, (seed & MASK32, (seed >> 32) & MASK32))
    return ((u[:, :3] >> 8).astype(np.float64) * 2.0 ** -24).astype(np.float32)


BOUND_TAG = 0x44564E42  # fourth counter word of boundary-sample draws


def boundary_count(n: int, frac: float) -> int:
    """Boundary samples among a block's n samples of one step: lambda * n
    rounded half up (Sec. III-C draws (1 - lambda) N uniform and lambda N
    boundary samples, so that the step always trains on N samples)."""
    return int(np.floor(frac * n + 0.5))


def boundary_coords(seed: int, block: int, step: int, n: int, first: int, sigma: float) -> np.ndarray:
    """Boundary-centered training coordinates (Sec. III-C, Eq. (2)).

    Reading of the density: an equal-weight mixture over the six faces of the
    unit cube; a sample picks a face, sits at a half-normal distance
    abs(N(0, sigma^2)) from it along the face normal, and is uniform in the
    two tangential coordinates.
    Sample i (i = first .. first + n - 1) draws Philox4x32-10 with counter
    (i, step, block, BOUND_TAG) and the seed as key.  Output words u0..u3:
      face  = floor(u3 * 6 / 2^32)  (axis = face // 2, side = face % 2);
      tangential coordinates, in increasing axis order: (u0 >> 8) 2^-24, (u1 >> 8) 2^-24;
      distance d = sigma * sqrt(2) * erfinv(v), v = (u2 >> 8) 2^-24 (the half-normal
      quantile of v), clipped to [0, 1];
      normal coordinate d on the low face, 1 - d on the high face.
    Returns float32 [n, 3]; the distance is evaluated in float64 and the
    coordinate rounded to float32 once.
    """
    from scipy.special import erfinv

    i = np.arange(first, first + n, dtype=np.uint64)
    ctr = np.stack([i & np.uint64(MASK32), np.full_like(i, step & MASK32),
                    np.full_like(i, block & MASK32), np.full_like(i, BOUND_TAG)], axis=1)
    u = philox4x32_10(ctr, (seed & MASK32, (seed >> 32) & MASK32)).astype(np.uint64)
    face = (u[:, 3] * np.uint64(6)) >> np.uint64(32)
    axis, side = (face // 2).astype(np.int64), (face % 2).astype(np.int64)
    tang = (u[:, :2] >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    v = (u[:, 2] >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    d = np.clip(sigma * np.sqrt(2.0) * erfinv(v), 0.0, 1.0)
    x = np.empty((n, 3), dtype=np.float64)
    rows = np.arange(n)
    x[rows, axis] = np.where(side == 1, 1.0 - d, d)
    t0 = np.where(axis == 0, 1, 0)          # first tangential axis
    t1 = np.where(axis == 2, 1, 2)          # second tangential axis
    x[rows, t0] = tang[:, 0]
    x[rows, t1] = tang[:, 1]
    return x.astype(np.float32)


def step_coords(seed: int, block: int, step: int, n: int, n_boundary: int = 0, sigma: float = 0.005) -> np.ndarray:
    """All n coordinates of one block at one step: samples 0 .. n - n_boundary - 1
    uniform (`training_coords`), the remaining n_boundary boundary-centered
    (`boundary_coords`).  Returns float32 [n, 3]."""
    nu = n - n_boundary
    x = training_coords(seed, block, step, nu)
    if n_boundary == 0:
        return x
    return np.concatenate([x, boundary_coords(seed, block, step, n_boundary, nu, sigma)], axis=0)


def block_value_range(vol: np.ndarray):
    """(vmin, vmax) over every stored voxel of a block, ghost layer included."""
    return float(np.min(vol)), float(np.max(vol))


def sample_volume(vol: np.ndarray, dims, ghost: int, x: np.ndarray) -> np.ndarray:
    """Trilinear value of a cell-centered block volume at normalized coordinates.

    vol has shape (nz + 2g, ny + 2g, nx + 2g) (x fastest); dims = owned (nx, ny, nz).
    Owned voxel j along an axis of n owned voxels sits at x = (j + 1/2) / n, so
    the stored index position is p = x * n - 1/2 + g; the cell origin is
    i0 = clamp(floor(p), 0, N - 2) with N = n + 2g stored voxels and the
    fraction t = clamp(p - i0, 0, 1) (which clamps to the border voxel where
    no ghost layer exists).  Returns float64 [n].
    """
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    v = np.asarray(vol, dtype=np.float64)
    i0s, ts = [], []
    for a in range(3):
        n = int(dims[a])
        N = n + 2 * ghost
        p = x[:, a] * n - 0.5 + ghost
        i0 = np.clip(np.floor(p), 0, N - 2).astype(np.int64)
        t = np.clip(p - i0, 0.0, 1.0)
        i0s.append(i0)
        ts.append(t)
    (ix, iy, iz), (tx, ty, tz) = i0s, ts
    out = np.zeros(x.shape[0], dtype=np.float64)
    for c in range(8):
        bx, by, bz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        wc = (tx if bx else 1 - tx) * (ty if by else 1 - ty) * (tz if bz else 1 - tz)
        out += wc * v[iz + bz, iy + by, ix + bx]
    return out


def normalized_targets(vol, dims, ghost, x) -> np.ndarray:
    """Targets in [0, 1]: (v - vmin) / (vmax - vmin) with the block's own range
    (Sec. III-A); a constant block uses scale 1."""
    vmin, vmax = block_value_range(vol)
    scale = 1.0 / (vmax - vmin) if vmax > vmin else 1.0
    return (sample_volume(vol, dims, ghost, x) - vmin) * scale


# --------------------------------------------------------------------------
# Optimization (Sec. III-B; Adam with L2 weight decay, Sec. III-F)
# --------------------------------------------------------------------------
@dataclass
class Optim:
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    weight_decay: float = 1e-9
    lr_decay_base: float = 1.0
    lr_decay_start: int = 0
    lr_decay_interval: int = 0   # 0: constant learning rate


def learning_rate(opt: Optim, t: int) -> float:
    """Learning rate of Adam update t (1, 2, ...): exponential decay
    lr * base^(max(0, t - start) / interval) (Sec. III-F names the decay; its
    form is this reading); constant when the interval is 0."""
    if opt.lr_decay_interval <= 0 or t <= opt.lr_decay_start:
        return opt.lr
    return opt.lr * opt.lr_decay_base ** ((t - opt.lr_decay_start) / opt.lr_decay_interval)


@dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    t: int = 0


def adam_init(n: int) -> AdamState:
    return AdamState(m=np.zeros(n), v=np.zeros(n), t=0)


def adam(params: np.ndarray, grad: np.ndarray, st: AdamState, opt: Optim) -> np.ndarray:
    """One Adam step on every parameter (dense: untouched entries still decay).

    g <- g + wd * theta; m <- b1 m + (1 - b1) g; v <- b2 v + (1 - b2) g^2;
    theta <- theta - lr_t * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
    lr_t = learning_rate(opt, t).
    Returns the new parameters (float64); st is updated in place.
    """
    th = np.asarray(params, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64) + opt.weight_decay * th
    st.t += 1
    st.m = opt.beta1 * st.m + (1.0 - opt.beta1) * g
    st.v = opt.beta2 * st.v + (1.0 - opt.beta2) * g * g
    mhat = st.m / (1.0 - opt.beta1 ** st.t)
    vhat = st.v / (1.0 - opt.beta2 ** st.t)
    return th - learning_rate(opt, st.t) * mhat / (np.sqrt(vhat) + opt.eps)


def loss_and_grad(lay: Layout, params: np.ndarray, x: np.ndarray, target: np.ndarray, loss: str = "l2"):
    """Loss of one block, mean over its samples, and its gradient.

    loss "l2": L = (1/n) sum (o - y)^2, dL/do = 2 (o - y) / n.
    loss "l1" (the unweighted L1 of Sec. III-C, Eq. (3)): L = (1/n) sum abs(o - y),
    dL/do = sign(o - y) / n with sign(0) = 0.
    Returns (L, grad vector, o).
    """
    y = encode(lay, params, x)
    W = mlp_weights(lay, params)
    o, acts = mlp_forward(W, y)
    o = o[:, 0]
    n = o.shape[0]
    r = o - np.asarray(target, dtype=np.float64)
    if loss == "l2":
        L = float(np.mean(r * r))
        do = (2.0 / n) * r
    elif loss == "l1":
        L = float(np.mean(np.abs(r)))
        do = np.sign(r) / n
    else:
        raise ValueError(loss)
    dy, dWs = mlp_backward(W, acts, do[:, None])
    g = np.empty(lay.n_params, dtype=np.float64)
    g[:lay.n_table_params] = encode_backward(lay, x, dy)
    for dW, off in zip(dWs, lay.mlp_offsets):
        g[off:off + dW.size] = dW.reshape(-1)
    return L, g, o


def train_step(lay: Layout, params, st: AdamState, opt: Optim, x, target, loss: str = "l2"):
    """One iteration: forward, loss, backward, Adam.  Returns (new params, loss)."""
    L, g, _ = loss_and_grad(lay, params, x, target, loss)
    return adam(params, g, st, opt), L


def train(lay: Layout, params0, vol, dims, ghost, n_steps: int, batch: int, seed: int,
          opt: Optim, block: int = 0, coords_fn=None, loss: str = "l2", boundary_frac: float = 0.0,
          sigma: float = 0.005):
    """Train one block's INR for n_steps from params0.

    Coordinates of step s are step_coords(seed, block, s, batch,
    boundary_count(batch, boundary_frac), sigma) unless `coords_fn(s)` supplies
    them.  Returns (params, losses, adam state).
    """
    params = np.asarray(params0, dtype=np.float64).copy()
    st = adam_init(lay.n_params)
    losses = []
    nbd = boundary_count(batch, boundary_frac)
    for s in range(n_steps):
        x = coords_fn(s) if coords_fn is not None else step_coords(seed, block, s, batch, nbd, sigma)
        tgt = normalized_targets(vol, dims, ghost, x)
        params, L = train_step(lay, params, st, opt, x, tgt, loss)
        losses.append(L)
    return params, np.array(losses), st


# --------------------------------------------------------------------------
# Training length and early termination (Sec. III-B)
# --------------------------------------------------------------------------
@dataclass
class StopPolicy:
    min_steps: int = 0            # N_train^min
    epochs: int = 1               # N_epoch
    loss_threshold: float = 0.0   # stop when the moving average falls below it; <= 0 disables
    window: int = 16              # moving-average window, in steps
    check_every: int = 16         # steps between two checks of the moving average


def max_train_steps(n_vox: int, batch: int, pol: StopPolicy) -> int:
    """N_train^max = max(N_train^min, ceil(N_vox / N_batch) * N_epoch) (Sec. III-B);
    0 when the block draws no samples."""
    if batch <= 0:
        return 0
    return max(int(pol.min_steps), -(-int(n_vox) // int(batch)) * int(pol.epochs))


def moving_average(losses, window: int) -> float:
    """Plain mean of the last `window` losses."""
    w = np.asarray(losses[-window:], dtype=np.float64)
    return float(np.mean(w))


def should_stop(losses, pol: StopPolicy) -> bool:
    """Loss criterion after len(losses) steps: checked only at multiples of
    check_every steps and once a full window exists; N_train^min bounds only
    the step budget (the formula above), not this test."""
    k = len(losses)
    if pol.loss_threshold <= 0 or k == 0 or k % pol.check_every or k < pol.window:
        return False
    return moving_average(losses, pol.window) < pol.loss_threshold


def train_until(lay: Layout, params0, vol, dims, ghost, batch: int, seed: int, opt: Optim, pol: StopPolicy,
                block: int = 0, n_vox: int | None = None, loss: str = "l2", boundary_frac: float = 0.0,
                sigma: float = 0.005):
    """Train one block until the loss criterion holds or N_train^max steps are
    done.  n_vox defaults to the block's owned voxel count.
    Returns (params, losses, steps done)."""
    if n_vox is None:
        n_vox = int(np.prod(dims))
    n_max = max_train_steps(n_vox, batch, pol)
    params = np.asarray(params0, dtype=np.float64).copy()
    st = adam_init(lay.n_params)
    nbd = boundary_count(batch, boundary_frac)
    losses = []
    while len(losses) < n_max:
        s = len(losses)
        x = step_coords(seed, block, s, batch, nbd, sigma)
        tgt = normalized_targets(vol, dims, ghost, x)
        params, L = train_step(lay, params, st, opt, x, tgt, loss)
        losses.append(L)
        if should_stop(losses, pol):
            break
    return params, np.array(losses), len(losses)


# --------------------------------------------------------------------------
# Access (Sec. III: on-demand inference and decoding back to the grid)
# --------------------------------------------------------------------------
def infer(lay: Layout, params, x) -> np.ndarray:
    """Normalized INR output at coordinates x (float64 [n])."""
    o, _ = mlp_forward(mlp_weights(lay, params), encode(lay, params, x))
    return o[:, 0]


def voxel_center_coords(dims) -> np.ndarray:
    """Float32 coordinates (i + 1/2) / n of every owned voxel, x fastest, [nz*ny*nx, 3]."""
    nx, ny, nz = [int(d) for d in dims]
    cx = ((np.arange(nx) + 0.5) / nx).astype(np.float32)
    cy = ((np.arange(ny) + 0.5) / ny).astype(np.float32)
    cz = ((np.arange(nz) + 0.5) / nz).astype(np.float32)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float32)


def decode(lay: Layout, params, dims, vmin: float, vmax: float, chunk: int = 1 << 16) -> np.ndarray:
    """Decoded owned voxels, de-normalized with the block range: o * (vmax - vmin) + vmin.

    Returns float64 of shape (nz, ny, nx)."""
    x = voxel_center_coords(dims)
    out = np.empty(x.shape[0], dtype=np.float64)
    for s in range(0, x.shape[0], chunk):
        out[s:s + chunk] = infer(lay, params, x[s:s + chunk])
    rng = (vmax - vmin) if vmax > vmin else 1.0
    nx, ny, nz = [int(d) for d in dims]
    return (out * rng + vmin).reshape(nz, ny, nx)


def squared_error(decoded: np.ndarray, truth: np.ndarray):
    """(sum of squared differences, voxel count) in float64."""
    d = np.asarray(decoded, dtype=np.float64) - np.asarray(truth, dtype=np.float64)
    return float(np.sum(d * d)), int(d.size)


def psnr(sse: float, count: int, peak: float = 1.0) -> float:
    """PSNR = 10 log10(peak^2 / MSE) with MSE = sse / count (data pre-normalized to [0, 1], Sec. V-B)."""
    mse = sse / count
    return float(10.0 * np.log10(peak * peak / mse))


# --------------------------------------------------------------------------
# Batching: per-block sample counts proportional to voxel count
# --------------------------------------------------------------------------
def apportion(voxels, total: int, unit: int = 256) -> np.ndarray:
    """Split `total` samples over blocks in proportion to their voxel counts.

    Largest-remainder method in units of `unit` samples: each block first gets
    floor(quota) units, the remaining units go to the largest fractional
    remainders, ties to the lower block id.  Requires total % unit == 0.
    """
    voxels = np.asarray(voxels, dtype=np.float64)
    if total % unit:
        raise ValueError("total must be a multiple of unit")
    units = total // unit
    quota = units * voxels / voxels.sum()
    base = np.floor(quota).astype(np.int64)
    rem = units - int(base.sum())
    frac = quota - base
    order = sorted(range(len(voxels)), key=lambda b: (-frac[b], b))
    for b in order[:rem]:
        base[b] += 1
    return base * unit


# --------------------------------------------------------------------------
# Direct volume rendering of one block's INR (Sec. IV, sample streaming)
# --------------------------------------------------------------------------
@dataclass
class Camera:
    eye: tuple
    center: tuple
    up: tuple
    fovy_deg: float
    width: int
    height: int


def camera_rays(cam: Camera):
    """Pinhole camera rays through pixel centers, in the block's unit-cube
    coordinates.  Row 0 is the top of the image.  Evaluated in float32 with the
    operation order below (the sample count of a ray is an integer decided by
    these values, so the renderer computes them identically):
      f = normalize(center - eye), r = normalize(f x up), u = r x f,
      s = tan(fovy / 2) (float64, then rounded), a = width / height,
      px = ((2 (i + 1/2) / width) - 1) * s * a, py = (1 - 2 (j + 1/2) / height) * s,
      d = normalize(f + px r + py u)  (left to right, no fused multiply-add).
    Returns (origin float32 [3], directions float32 [height * width, 3])."""
    f32 = np.float32

    def norm(v):
        n = np.sqrt(f32(v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]).astype(f32)
        return (v / n).astype(f32)

    def cross(a, b):
        return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]], f32)

    eye, ctr, up = (np.asarray(v, f32) for v in (cam.eye, cam.center, cam.up))
    fw = norm((ctr - eye).astype(f32))
    rt = norm(cross(fw, up))
    uu = cross(rt, fw)
    tan_h = f32(np.tan(np.radians(cam.fovy_deg) / 2.0))
    aspect = f32(f32(cam.width) / f32(cam.height))
    i = np.arange(cam.width, dtype=f32)
    j = np.arange(cam.height, dtype=f32)
    px = ((f32(2) * (i + f32(0.5)) / f32(cam.width) - f32(1)) * tan_h * aspect).astype(f32)
    py = ((f32(1) - f32(2) * (j + f32(0.5)) / f32(cam.height)) * tan_h).astype(f32)
    PX, PY = np.meshgrid(px, py)
    d = np.empty((cam.height * cam.width, 3), f32)
    for a in range(3):
        d[:, a] = ((fw[a] + PX.ravel() * rt[a]).astype(f32) + PY.ravel() * uu[a]).astype(f32)
    n = np.sqrt(((d[:, 0] * d[:, 0]).astype(f32) + d[:, 1] * d[:, 1]).astype(f32) + d[:, 2] * d[:, 2]).astype(f32)
    return eye, (d / n[:, None]).astype(f32)


def ray_box(origin, dirs):
    """Entry and exit parameters of rays with the unit cube (slab method,
    float32): per axis t = (0 - o) / d and (1 - o) / d; t0 = max(0, max of the
    near values), t1 = min of the far values.  A ray misses when t1 <= t0."""
    f32 = np.float32
    o = np.asarray(origin, f32)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = (f32(1) / dirs).astype(f32)
        ta = ((f32(0) - o) * inv).astype(f32)
        tb = ((f32(1) - o) * inv).astype(f32)
    near = np.minimum(ta, tb)
    far = np.maximum(ta, tb)
    t0 = np.maximum(np.max(near, axis=1), f32(0))
    t1 = np.min(far, axis=1)
    return t0.astype(f32), t1.astype(f32)


def sample_params(t0, t1, dt: float, k):
    """t_k = t0 + (k + 1/2) dt in float32; the sample exists iff t_k < t1."""
    f32 = np.float32
    tk = (t0 + (f32(k) + f32(0.5)) * f32(dt)).astype(f32)
    return tk, tk < t1


def transfer(tf: np.ndarray, lo: float, hi: float, v):
    """Piecewise-linear transfer function: tf [n][4] RGBA at n equally spaced
    values over [lo, hi]; v is clamped to the range."""
    n = tf.shape[0]
    s = np.clip((np.asarray(v, np.float64) - lo) / (hi - lo), 0.0, 1.0) * (n - 1)
    i = np.minimum(np.floor(s).astype(np.int64), n - 2)
    w = (s - i)[:, None]
    return (1.0 - w) * tf[i] + w * tf[i + 1]


def render(lay: Layout, params, vmin: float, vmax: float, cam: Camera, tf: np.ndarray, lo: float, hi: float,
           dt: float, ref_dt: float, alpha_stop: float = 1.0):
    """Front-to-back emission-absorption ray marching through the block's INR.

    Sample k of a ray sits at x = o + t_k d; its value is the de-normalized
    INR output; the transfer function gives (r, g, b, a) with a the opacity
    over a reference length ref_dt, corrected to the step: alpha = 1 - (1 - a)^(dt / ref_dt).
    C += (1 - A) alpha rgb, A += (1 - A) alpha, in sample order; a ray stops
    after the sample that brings A to alpha_stop or above.  Returns a float64
    image [height][width][4] of premultiplied (C, A)."""
    f32 = np.float32
    o, d = camera_rays(cam)
    t0, t1 = ray_box(o, d)
    n_rays = d.shape[0]
    out = np.zeros((n_rays, 4))
    done = ~(t1 > t0)
    k = 0
    while not done.all():
        live = np.nonzero(~done)[0]
        tk, ok = sample_params(t0[live], t1[live], dt, k)
        done[live[~ok]] = True
        live, tk = live[ok], tk[ok]
        if live.size:
            x = (o[None, :] + (tk[:, None] * d[live]).astype(f32)).astype(f32)
            v = vmin + infer(lay, params, x) * (vmax - vmin)
            c = transfer(tf, lo, hi, v)
            alpha = 1.0 - (1.0 - np.clip(c[:, 3], 0.0, 1.0)) ** (dt / ref_dt)
            A = out[live, 3]
            out[live, :3] += ((1.0 - A) * alpha)[:, None] * c[:, :3]
            out[live, 3] = A + (1.0 - A) * alpha
            done[live[out[live, 3] >= alpha_stop]] = True
        k += 1
    return out.reshape(cam.height, cam.width, 4)
