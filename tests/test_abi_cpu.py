"""Host-side checks of the C ABI that need no GPU: every declared symbol is
exported, configuration validation, and the host layout logic (resolution
table, dense/hash split, offsets, sizes) against the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import dvnr_oracle as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dvnr.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
LIB = os.path.join(ROOT, "paper_2304_10516_amd", "libdvnr.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdvnr.so not built")


def _declared(headers=(HEADER,)):
    names = set()
    for h in headers:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(dvnr_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    for must in ("dvnr_create", "dvnr_train_steps", "dvnr_sample", "dvnr_decode", "dvnr_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    names = _declared(HEADERS)
    assert "dvnr_micro_gather" in names and "dvnr_render_static" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _make(enc, mlp, blocks=(((8, 8, 8), 0),), precision="fp32", max_batch=1024):
    from paper_2304_10516_amd import _lib as L
    lib = L.lib()
    nb = len(blocks)
    barr = (L.Block * nb)()
    for i, (d, g) in enumerate(blocks):
        barr[i].dims[0], barr[i].dims[1], barr[i].dims[2] = d
        barr[i].ghost = g
    e = L.Encoding(enc.n_levels, enc.n_features, enc.log2_table_size, enc.base_resolution,
                   float(enc.per_level_scale), enc.finest_resolution)
    m = L.Mlp(mlp.n_hidden_layers, mlp.width, 1)
    opt = L.Optim(1e-2, 0.9, 0.999, 1e-8, 1e-9)
    h = C.c_void_p()
    prec = {"fp32": 0, "mixed": 1, "fp64": 2}[precision]
    code = lib.dvnr_create(C.byref(e), C.byref(m), C.byref(opt), prec, nb, barr, max_batch, 0, C.byref(h))
    return lib, code, h


CONFIGS = [
    (o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16)),
    (o.Encoding(16, 2, 19, 16, 0.0, 256), o.MLP(2, 64)),
    (o.Encoding(16, 2, 17, 16, 0.0, 160), o.MLP(2, 64)),
    (o.Encoding(16, 2, 19, 16, 0.0, 128), o.MLP(2, 64)),
    (o.Encoding(3, 2, 6, 2, 2.0), o.MLP(1, 16)),
    (o.Encoding(5, 4, 12, 16, 2.0), o.MLP(3, 16)),
    (o.Encoding(8, 4, 16, 8, 1.5), o.MLP(2, 32)),
]


@pytest.mark.parametrize("enc,mlp", CONFIGS)
def test_layout_matches_oracle(enc, mlp):
    from paper_2304_10516_amd import _lib as L
    lib, code, h = _make(enc, mlp)
    assert code == 0, lib.dvnr_last_error()
    try:
        lay = o.layout(enc, mlp)
        nl = enc.n_levels
        R, D = (C.c_int32 * nl)(), (C.c_int32 * nl)()
        off, E = (C.c_int64 * nl)(), (C.c_int64 * nl)()
        assert lib.dvnr_level_info(h, R, D, off, E) == 0
        assert list(R) == [l.R for l in lay.levels]
        assert [bool(v) for v in D] == [l.dense for l in lay.levels]
        assert list(off) == [l.off for l in lay.levels]
        assert list(E) == [l.E for l in lay.levels]
        sz = L.Sizes()
        assert lib.dvnr_get_sizes(h, C.byref(sz)) == 0
        assert sz.n_entries == lay.n_entries
        assert sz.n_table_params == lay.n_table_params
        assert sz.n_mlp_params == lay.n_params - lay.n_table_params
        assert sz.block_stride % 64 == 0 and sz.block_stride >= lay.n_params
    finally:
        lib.dvnr_destroy(h)


@pytest.mark.parametrize("bad", [
    dict(n_levels=0), dict(n_levels=17), dict(n_features=3), dict(log2_table_size=25), dict(base_resolution=1),
    dict(width=48), dict(n_hidden_layers=0), dict(n_levels=16, n_features=4),
])
def test_invalid_configurations_are_rejected(bad):
    e = dict(n_levels=4, n_features=2, log2_table_size=12, base_resolution=4, per_level_scale=2.0)
    m = dict(n_hidden_layers=1, width=16)
    for k, v in bad.items():
        (m if k in m else e)[k] = v
    lib, code, h = _make(o.Encoding(**e), o.MLP(**m))
    assert code == 1 and not h.value
    assert lib.dvnr_last_error()


def test_calls_in_wrong_order_report_state_errors():
    lib, code, h = _make(o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16))
    assert code == 0
    try:
        assert lib.dvnr_prepare(h, None) == 4
        assert lib.dvnr_train_steps(h, 1, 256, None, None) == 4
        assert lib.dvnr_set_option(h, b"no_such_option", 1) == 1
        assert lib.dvnr_set_option(h, b"scatter_grouped", 1) == 0
    finally:
        lib.dvnr_destroy(h)


def test_fp64_handle_rejects_training():
    lib, code, h = _make(o.Encoding(3, 2, 6, 2, 2.0), o.MLP(1, 16), precision="fp64")
    assert code == 0
    lib.dvnr_destroy(h)


def test_set_loss_validates_arguments():
    lib, code, h = _make(o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16))
    assert code == 0
    lib.dvnr_set_loss.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double]
    try:
        assert lib.dvnr_set_loss(h, 1, 0.15, 0.005) == 0
        assert lib.dvnr_set_loss(h, 0, 0.0, 0.005) == 0
        assert lib.dvnr_set_loss(h, 2, 0.15, 0.005) == 1       # unknown loss
        assert lib.dvnr_set_loss(h, 1, -0.1, 0.005) == 1       # fraction out of [0, 1]
        assert lib.dvnr_set_loss(h, 1, 1.5, 0.005) == 1
        assert lib.dvnr_set_loss(h, 1, float("nan"), 0.005) == 1
        assert lib.dvnr_set_loss(h, 1, 0.15, 0.0) == 1         # sigma must be positive
        assert lib.dvnr_set_loss(h, 1, 0.15, 2.0) == 1
    finally:
        lib.dvnr_destroy(h)


def test_model_cache_host_logic():
    from paper_2304_10516_amd import _lib as L
    for prec, elem in (("fp32", 4), ("mixed", 2)):
        lib, code, h = _make(o.Encoding(4, 2, 12, 4, 2.0), o.MLP(1, 16),
                             blocks=(((8, 8, 8), 0), ((5, 6, 7), 1)), precision=prec)
        assert code == 0
        try:
            lib.dvnr_cache_snapshot_bytes.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
            lib.dvnr_cache_bind.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
            lib.dvnr_cache_push.argtypes = [C.c_void_p, C.c_int64, C.c_void_p]
            lib.dvnr_cache_keys.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
            sz = L.Sizes()
            assert lib.dvnr_get_sizes(h, C.byref(sz)) == 0
            nb = C.c_int64()
            assert lib.dvnr_cache_snapshot_bytes(h, C.byref(nb)) == 0
            align = lambda v: (v + 255) // 256 * 256
            assert nb.value == align(sz.n_params * elem) + align(16 * 2)
            assert lib.dvnr_cache_bind(h, 3, None) == 1          # buffer required
            assert lib.dvnr_cache_bind(h, 3, 4096 + 8) == 1      # 256-byte alignment
            assert lib.dvnr_cache_bind(h, -1, 4096) == 1
            assert lib.dvnr_cache_bind(h, 3, 4096) == 0          # the pointer is only stored here
            assert lib.dvnr_cache_push(h, 0, None) == 4          # not prepared: state error
            n = C.c_int32(-1)
            assert lib.dvnr_cache_keys(h, None, C.byref(n)) == 0 and n.value == 0
            assert lib.dvnr_cache_bind(h, 0, None) == 0
        finally:
            lib.dvnr_destroy(h)
    lib, code, h = _make(o.Encoding(3, 2, 6, 2, 2.0), o.MLP(1, 16), precision="fp64")
    nb = C.c_int64()
    assert lib.dvnr_cache_snapshot_bytes(h, C.byref(nb)) == 2
    lib.dvnr_destroy(h)


def test_partitioned_backward_options():
    """Option validation of the destination-partitioned backward; no level is
    partitioned before a training plan exists."""
    lib, code, h = _make(o.Encoding(16, 2, 19, 16, 0.0, 256), o.MLP(2, 64), precision="mixed")
    assert code == 0
    try:
        lib.dvnr_plan_partition.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
        lf = C.c_int32(-7)
        assert lib.dvnr_plan_partition(h, C.byref(lf)) == 0 and lf.value == 16
        assert lib.dvnr_plan_partition(h, None) == 1
        for v, ok in ((4096, 0), (8192, 0), (16384, 0), (1000, 1), (32768, 1), (0, 1)):
            assert lib.dvnr_set_option(h, b"part_slice", v) == ok, v
        assert lib.dvnr_set_option(h, b"scatter_part", 9) == 0
        assert lib.dvnr_set_option(h, b"scatter_part", -1) == 0
        assert lib.dvnr_set_option(h, b"part_capacity", 8) == 0
        for v in (-1, 0, 1):
            assert lib.dvnr_set_option(h, b"priv_classes", v) == 0
    finally:
        lib.dvnr_destroy(h)


def test_mlp_and_sampler_options():
    """Option validation of the MLP kernel variants (waves per workgroup 4 or
    8; register budget of the 4-wave kernel) and of the sampler look-ahead's
    fork point (0 .. 3)."""
    lib, code, h = _make(o.Encoding(16, 2, 19, 16, 0.0, 256), o.MLP(2, 64), precision="mixed")
    assert code == 0
    try:
        for v, ok in ((4, 0), (8, 0), (0, 1), (2, 1), (6, 1), (16, 1)):
            assert lib.dvnr_set_option(h, b"mlp_wg_waves", v) == ok, v
        for v in (1, 2):
            assert lib.dvnr_set_option(h, b"mlp_waves", v) == 0
        for v, ok in ((0, 0), (1, 0), (2, 0), (3, 0), (4, 1), (-1, 1)):
            assert lib.dvnr_set_option(h, b"sample_ahead", v) == ok, v
    finally:
        lib.dvnr_destroy(h)
