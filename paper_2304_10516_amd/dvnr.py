"""Python handle over the DVNR C ABI.  torch provides device memory and streams;
every step of the hot path runs in the HIP library."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L


@dataclass
class EncodingCfg:
    n_levels: int
    n_features: int
    log2_table_size: int
    base_resolution: int
    per_level_scale: float = 0.0
    finest_resolution: int = 0


@dataclass
class MlpCfg:
    n_hidden_layers: int
    width: int
    out_dim: int = 1


@dataclass
class OptimCfg:
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    weight_decay: float = 1e-9
    lr_decay_base: float = 1.0      # exponential decay: lr * base^(max(0, t - start) / interval)
    lr_decay_start: int = 0
    lr_decay_interval: int = 0      # 0: constant learning rate


PRECISIONS = {"fp32": L.DVNR_FP32, "mixed": L.DVNR_MIXED_BF16, "bf16": L.DVNR_MIXED_BF16, "fp64": L.DVNR_FP64}


def _aligned_empty(nbytes: int, device, align: int = 256) -> tuple[torch.Tensor, int]:
    """A byte tensor with a 256-byte aligned region of nbytes; returns (tensor, offset)."""
    t = torch.empty(max(nbytes, 1) + align, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % align
    return t, off


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class DVNR:
    """One configuration of INRs over `blocks` (list of (dims_xyz, ghost)) on one GPU.

    Allocates the parameter, gradient, Adam and workspace buffers with torch and
    binds them; `bind_volumes` hands over each block's voxels (float32 device
    tensors of shape (nz+2g, ny+2g, nx+2g)).
    """

    def __init__(self, enc: EncodingCfg, mlp: MlpCfg, blocks, optim: OptimCfg | None = None, precision="mixed",
                 max_batch: int = 1 << 18, seed: int = 0, device="cuda"):
        self.lib = L.lib()
        self.enc, self.mlp, self.optim = enc, mlp, optim or OptimCfg()
        self.precision = precision
        self.device = torch.device(device)
        self.blocks = [(tuple(int(v) for v in d), int(g)) for d, g in blocks]
        nb = len(self.blocks)
        barr = (L.Block * nb)()
        for i, (d, g) in enumerate(self.blocks):
            barr[i].dims[0], barr[i].dims[1], barr[i].dims[2] = d
            barr[i].ghost = g
        e = L.Encoding(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution,
                       float(enc.per_level_scale), enc.finest_resolution)
        m = L.Mlp(mlp.n_hidden_layers, mlp.width, mlp.out_dim)
        o = L.Optim(self.optim.lr, self.optim.beta1, self.optim.beta2, self.optim.eps, self.optim.weight_decay,
                    self.optim.lr_decay_base, self.optim.lr_decay_start, self.optim.lr_decay_interval)
        h = C.c_void_p()
        L.check(self.lib.dvnr_create(C.byref(e), C.byref(m), C.byref(o), PRECISIONS[precision], nb, barr,
                                     int(max_batch), int(seed), C.byref(h)))
        self.h = h
        self.max_batch = int(max_batch)
        sz = L.Sizes()
        L.check(self.lib.dvnr_get_sizes(self.h, C.byref(sz)))
        self.sizes = sz
        self.n_blocks = nb
        self.block_stride = sz.block_stride
        self.n_table = sz.n_table_params
        self.n_mlp = sz.n_mlp_params
        self.pdtype = torch.float64 if precision == "fp64" else torch.float32
        self._bufs = None
        self._vols = None

    # -- layout -----------------------------------------------------------
    def level_info(self):
        nl = self.enc.n_levels
        R, D = (C.c_int32 * nl)(), (C.c_int32 * nl)()
        off, E = (C.c_int64 * nl)(), (C.c_int64 * nl)()
        L.check(self.lib.dvnr_level_info(self.h, R, D, off, E))
        return list(R), [bool(v) for v in D], list(off), list(E)

    # -- buffers ------------------------------------------------------------
    def _alloc(self):
        dev = self.device
        n = self.sizes.n_params
        self.params = torch.zeros(n, dtype=self.pdtype, device=dev)
        self.grads = torch.zeros(n, dtype=self.pdtype, device=dev)
        self.adam_m = torch.zeros(n, dtype=self.pdtype, device=dev)
        self.adam_v = torch.zeros(n, dtype=self.pdtype, device=dev)
        self.work16 = torch.zeros(max(n, 1), dtype=torch.int16, device=dev) if self.sizes.work16_bytes else None
        self._ws, self._ws_off = _aligned_empty(self.sizes.workspace_bytes, dev)
        for t in (self.params, self.grads, self.adam_m, self.adam_v) + ((self.work16,) if self.work16 is not None else ()):
            if t.data_ptr() % 256:
                raise RuntimeError("torch allocation is not 256-byte aligned")

    def bind_volumes(self, volumes, stream=None):
        if len(volumes) != self.n_blocks:
            raise ValueError("one volume per block")
        vols = []
        for (d, g), v in zip(self.blocks, volumes):
            v = v.to(device=self.device, dtype=torch.float32).contiguous()
            want = (d[2] + 2 * g, d[1] + 2 * g, d[0] + 2 * g)
            if tuple(v.shape) != want:
                raise ValueError(f"volume shape {tuple(v.shape)} != {want}")
            vols.append(v)
        if self._bufs is None:
            self._alloc()
        self._vols = vols
        ptrs = (C.c_void_p * self.n_blocks)(*[v.data_ptr() for v in vols])
        self._vol_ptrs = ptrs
        b = L.Buffers(self.params.data_ptr(), self.grads.data_ptr(), self.adam_m.data_ptr(), self.adam_v.data_ptr(),
                      self.work16.data_ptr() if self.work16 is not None else None,
                      self._ws.data_ptr() + self._ws_off, ptrs)
        self._bufs = b
        L.check(self.lib.dvnr_bind(self.h, C.byref(b)))
        L.check(self.lib.dvnr_prepare(self.h, _stream_ptr(stream)))

    def prepare(self, stream=None):
        """Recompute the per-block value ranges (after the bound voxels changed in place)."""
        L.check(self.lib.dvnr_prepare(self.h, _stream_ptr(stream)))

    def ranges(self, stream=None):
        lo = (C.c_float * self.n_blocks)()
        hi = (C.c_float * self.n_blocks)()
        L.check(self.lib.dvnr_get_ranges(self.h, lo, hi, _stream_ptr(stream)))
        return list(lo), list(hi)

    def set_option(self, name: str, value: int):
        L.check(self.lib.dvnr_set_option(self.h, name.encode(), int(value)))

    LOSSES = {"l2": 0, "l1": 1}

    def set_loss(self, loss: str = "l2", boundary_frac: float = 0.0, sigma: float = 0.005):
        """Training loss ("l2" or "l1") and the share / spread of
        boundary-centered samples (Sec. III-C, Eqs. (2)-(3); the paper uses l1, 0.15, 0.005)."""
        if loss not in self.LOSSES:
            raise ValueError(f"unknown loss {loss!r}")
        L.check(self.lib.dvnr_set_loss(self.h, self.LOSSES[loss], float(boundary_frac), float(sigma)))

    # -- parameters ---------------------------------------------------------------
    def block_params(self, b: int) -> torch.Tensor:
        """View of block b's parameters (tables then weights, canonical layout)."""
        s = b * self.block_stride
        return self.params[s:s + self.n_table + self.n_mlp]

    def block_grads(self, b: int) -> torch.Tensor:
        s = b * self.block_stride
        return self.grads[s:s + self.n_table + self.n_mlp]

    def init_params(self, seed: int = 0, stream=None):
        L.check(self.lib.dvnr_init_params(self.h, int(seed), _stream_ptr(stream)))

    def load_params(self, per_block, stream=None):
        """Overwrite every block's parameters (list of 1-D tensors/arrays of n_table + n_mlp)."""
        for b, p in enumerate(per_block):
            self.block_params(b).copy_(torch.as_tensor(p, dtype=self.pdtype))
        L.check(self.lib.dvnr_params_updated(self.h, _stream_ptr(stream)))
        L.check(self.lib.dvnr_reset_optimizer(self.h, _stream_ptr(stream)))

    def reset_optimizer(self, stream=None):
        L.check(self.lib.dvnr_reset_optimizer(self.h, _stream_ptr(stream)))

    # -- training -----------------------------------------------------------------
    def train(self, n_steps: int, samples_per_step: int, want_loss: bool = False, stream=None):
        loss = torch.empty((n_steps, self.n_blocks), dtype=torch.float32, device=self.device) if want_loss else None
        L.check(self.lib.dvnr_train_steps(self.h, int(n_steps), int(samples_per_step),
                                          loss.data_ptr() if loss is not None else None, _stream_ptr(stream)))
        return loss

    def train_until(self, samples_per_step: int, min_steps: int = 0, epochs: int = 1, loss_threshold: float = 0.0,
                    window: int = 16, check_every: int = 16, stream=None):
        """Train every block up to max(min_steps, ceil(N_vox / n_b) * epochs)
        steps, stopping a block early when the mean of its last `window`
        losses, checked every `check_every` steps, is below loss_threshold
        (Sec. III-B).  Returns (steps per block, last moving average per block)."""
        pol = L.StopPolicy(int(min_steps), int(epochs), float(loss_threshold), int(window), int(check_every))
        steps = (C.c_int64 * self.n_blocks)()
        avg = (C.c_double * self.n_blocks)()
        L.check(self.lib.dvnr_train_until(self.h, C.byref(pol), int(samples_per_step), steps, avg,
                                          _stream_ptr(stream)))
        return list(steps), list(avg)

    def train_step_coords(self, coords: torch.Tensor, n_per_block, stream=None):
        coords = coords.to(device=self.device, dtype=torch.float32).contiguous()
        n = (C.c_int64 * self.n_blocks)(*[int(v) for v in n_per_block])
        loss = torch.empty(self.n_blocks, dtype=torch.float32, device=self.device)
        L.check(self.lib.dvnr_train_step_coords(self.h, coords.data_ptr(), n, loss.data_ptr(), _stream_ptr(stream)))
        return loss

    def draw_training_samples(self, block: int, step: int, n: int, stream=None):
        coords = torch.empty((n, 3), dtype=torch.float32, device=self.device)
        target = torch.empty(n, dtype=torch.float32, device=self.device)
        L.check(self.lib.dvnr_draw_training_samples(self.h, block, step, n, coords.data_ptr(), target.data_ptr(),
                                                    _stream_ptr(stream)))
        return coords, target

    PHASES = ("sample", "encode", "mlp", "scatter_priv", "scatter", "part_bucket", "part_accum", "reduce", "adam")

    def phase_times(self):
        """{phase: total ms} and the step count since the previous call (needs option profile_phases=1)."""
        ms = (C.c_double * len(self.PHASES))()
        n = C.c_int64()
        L.check(self.lib.dvnr_phase_times(self.h, ms, C.byref(n)))
        return dict(zip(self.PHASES, list(ms))), n.value

    def autotune(self, samples_per_step: int, n_trial_steps: int = 5, stream=None) -> float:
        """Pick the fastest step configuration for this sample count; returns its ms per step (no update)."""
        ms = C.c_double()
        L.check(self.lib.dvnr_autotune(self.h, int(samples_per_step), int(n_trial_steps), C.byref(ms),
                                       _stream_ptr(stream)))
        return ms.value

    def plan_info(self):
        """(spatial bins per axis, number of bin-privatized coarse levels) of the current training plan."""
        bpa, pl = C.c_int32(), C.c_int32()
        L.check(self.lib.dvnr_plan_info(self.h, C.byref(bpa), C.byref(pl)))
        return bpa.value, pl.value

    def partitioned_levels(self):
        """First level whose encoding backward is destination-partitioned in the current plan (n_levels: none)."""
        lf = C.c_int32()
        L.check(self.lib.dvnr_plan_partition(self.h, C.byref(lf)))
        return lf.value

    def sync(self, stream=None):
        L.check(self.lib.dvnr_sync(self.h, _stream_ptr(stream)))

    # -- access -------------------------------------------------------------------
    def sample(self, block: int, coords: torch.Tensor, stream=None) -> torch.Tensor:
        coords = coords.to(device=self.device, dtype=torch.float32).contiguous()
        out = torch.empty(coords.shape[0], dtype=torch.float32, device=self.device)
        L.check(self.lib.dvnr_sample(self.h, block, coords.shape[0], coords.data_ptr(), out.data_ptr(),
                                     _stream_ptr(stream)))
        return out

    def decode(self, block: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        d, _ = self.blocks[block]
        if out is None:
            out = torch.empty((d[2], d[1], d[0]), dtype=torch.float32, device=self.device)
        L.check(self.lib.dvnr_decode(self.h, block, out.data_ptr(), _stream_ptr(stream)))
        return out

    # -- direct volume rendering ----------------------------------------------------
    def render(self, block: int, eye, center, up, fovy_deg: float, width: int, height: int, tf: torch.Tensor,
               tf_range, step: float, ref_step: float | None = None, alpha_stop: float = 1.0,
               samples_per_round: int = 64, stream=None, static_scratch: bool = False,
               out: torch.Tensor | None = None) -> torch.Tensor:
        """Front-to-back ray marching of block `block`'s INR through a pinhole
        camera (unit-cube coordinates of the block); tf: [n][4] RGBA over
        tf_range (float32, on the device).  Returns the premultiplied RGBA image
        [height][width][4] (written into `out` when given).  static_scratch:
        call dvnr_render_static, which keeps the ray state in the library's
        static device array instead of a workspace allocated here."""
        cam = L.Camera((C.c_float * 3)(*eye), (C.c_float * 3)(*center), (C.c_float * 3)(*up), float(fovy_deg),
                       int(width), int(height))
        tf = tf.to(device=self.device, dtype=torch.float32).contiguous()
        rp = L.RenderParams(float(step), float(ref_step if ref_step is not None else step), float(alpha_stop),
                            float(tf_range[0]), float(tf_range[1]), int(tf.shape[0]), int(samples_per_round))
        if out is not None and (tuple(out.shape) != (height, width, 4) or out.dtype != torch.float32
                                or not out.is_contiguous() or out.device.type != "cuda"):
            raise ValueError("out must be a contiguous float32 device tensor of shape (height, width, 4)")
        img = out if out is not None else torch.empty((height, width, 4), dtype=torch.float32, device=self.device)
        n = C.c_int64()
        if static_scratch:
            L.check(self.lib.dvnr_render_static(self.h, block, C.byref(cam), C.byref(rp), tf.data_ptr(),
                                                img.data_ptr(), C.byref(n), _stream_ptr(stream)))
        else:
            nb = C.c_int64()
            L.check(self.lib.dvnr_render_workspace_bytes(self.h, int(width), int(height), C.byref(nb)))
            ws, off = _aligned_empty(nb.value, self.device)
            L.check(self.lib.dvnr_render(self.h, block, C.byref(cam), C.byref(rp), tf.data_ptr(),
                                         ws.data_ptr() + off, img.data_ptr(), C.byref(n), _stream_ptr(stream)))
        self.last_render_samples = n.value
        return img

    # -- sliding-window model cache -------------------------------------------------
    def cache_bind(self, capacity: int):
        """Device buffer for `capacity` model snapshots (clears the cache)."""
        nb = C.c_int64()
        L.check(self.lib.dvnr_cache_snapshot_bytes(self.h, C.byref(nb)))
        self._cache, off = _aligned_empty(int(capacity) * nb.value, self.device)
        L.check(self.lib.dvnr_cache_bind(self.h, int(capacity), self._cache.data_ptr() + off if capacity else None))
        return nb.value

    def cache_push(self, key: int, stream=None):
        L.check(self.lib.dvnr_cache_push(self.h, int(key), _stream_ptr(stream)))

    def cache_keys(self):
        """Cached keys, oldest first."""
        n = C.c_int32()
        L.check(self.lib.dvnr_cache_keys(self.h, None, C.byref(n)))
        keys = (C.c_int64 * max(n.value, 1))()
        L.check(self.lib.dvnr_cache_keys(self.h, keys, C.byref(n)))
        return list(keys)[:n.value]

    def cache_decode(self, key: int, block: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        d, _ = self.blocks[block]
        if out is None:
            out = torch.empty((d[2], d[1], d[0]), dtype=torch.float32, device=self.device)
        L.check(self.lib.dvnr_cache_decode(self.h, int(key), block, out.data_ptr(), _stream_ptr(stream)))
        return out

    def cache_sample(self, key: int, block: int, coords: torch.Tensor, stream=None) -> torch.Tensor:
        coords = coords.to(device=self.device, dtype=torch.float32).contiguous()
        out = torch.empty(coords.shape[0], dtype=torch.float32, device=self.device)
        L.check(self.lib.dvnr_cache_sample(self.h, int(key), block, coords.shape[0], coords.data_ptr(),
                                           out.data_ptr(), _stream_ptr(stream)))
        return out

    def squared_error(self, block: int, decoded: torch.Tensor, stream=None):
        sse, cnt = C.c_double(), C.c_int64()
        L.check(self.lib.dvnr_mse_fp64(self.h, block, decoded.data_ptr(), C.byref(sse), C.byref(cnt),
                                       _stream_ptr(stream)))
        return sse.value, cnt.value

    # -- autograd building blocks ------------------------------------------------
    # A tensor argument of None stands for block `block`'s bound parameters
    # (table, weights) or gradients (dtable, dweights).
    @staticmethod
    def _ptr(t):
        return t.data_ptr() if t is not None else None

    def encode_forward(self, coords, table=None, block: int = 0, stream=None):
        n = coords.shape[0]
        dt = table.dtype if table is not None else self.pdtype
        feats = torch.empty((n, self.enc.n_levels * self.enc.n_features), dtype=dt, device=self.device)
        L.check(self.lib.dvnr_encode_forward(self.h, int(block), n, coords.data_ptr(), self._ptr(table),
                                             feats.data_ptr(), _stream_ptr(stream)))
        return feats

    def encode_backward(self, coords, dfeats, dtable=None, block: int = 0, stream=None):
        L.check(self.lib.dvnr_encode_backward(self.h, int(block), coords.shape[0], coords.data_ptr(),
                                              dfeats.data_ptr(), self._ptr(dtable), _stream_ptr(stream)))
        return dtable

    def mlp_forward(self, feats, weights=None, block: int = 0, stream=None):
        out = torch.empty(feats.shape[0], dtype=feats.dtype, device=self.device)
        L.check(self.lib.dvnr_mlp_forward(self.h, int(block), feats.shape[0], feats.data_ptr(), self._ptr(weights),
                                          out.data_ptr(), _stream_ptr(stream)))
        return out

    def mlp_backward(self, feats, weights, dout, dweights=None, block: int = 0, stream=None):
        dfeats = torch.empty_like(feats)
        L.check(self.lib.dvnr_mlp_backward(self.h, int(block), feats.shape[0], feats.data_ptr(),
                                           self._ptr(weights), dout.data_ptr(), dfeats.data_ptr(),
                                           self._ptr(dweights), _stream_ptr(stream)))
        return dfeats

    def adam_step(self, stream=None):
        """One fused Adam update of every block from the gradient buffer (`grads`);
        leaves the gradient at zero and advances the shared step counter."""
        L.check(self.lib.dvnr_adam_step(self.h, _stream_ptr(stream)))

    def debug_indices(self, level: int, coords, stream=None):
        n = coords.shape[0]
        idx = torch.empty((n, 8), dtype=torch.int32, device=self.device)
        w = torch.empty((n, 8), dtype=torch.float32, device=self.device)
        L.check(self.lib.dvnr_debug_indices(self.h, level, n, coords.data_ptr(), idx.data_ptr(), w.data_ptr(),
                                            _stream_ptr(stream)))
        return idx, w

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.dvnr_destroy(self.h)
                self.h = None
        except Exception:
            pass
