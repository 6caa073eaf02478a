"""The C ABI of libnpm.so, checked without a GPU: the library loads, exports
every entry point include/npm.h declares, validates its arguments before
touching a device, and lays out a configuration exactly as the oracle does
(grid resolutions, dense/hashed levels, offsets, flat parameter layout)."""
import ctypes as C
import os
import re

import pytest

from paper_2504_04315_amd import npm as B
from paper_2504_04315_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")):
        text = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"^\s*(?:npm_status|const char \*)\s*(npm_\w+)\s*\(", text, re.M))
    return names


def test_every_declared_symbol_is_exported():
    lib = B.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(B.SIGNATURES) <= names
    from paper_2504_04315_amd import serve as S
    assert set(S.SIGNATURES) <= names
    assert {"npm_server_create", "npm_submit_train", "npm_server_hold",
            "npm_backward_static", "npm_query_select", "npm_backward_select",
            "npm_train_step_select", "npm_measure_peaks"} <= names


def test_peak_probe_validates_before_touching_a_device():
    lib = B.lib()
    out = (C.c_double * 4)(-1.0, -1.0, -1.0, -1.0)
    assert lib.npm_measure_peaks(None, 1) == -1
    assert lib.npm_measure_peaks(out, 0) == -1
    assert b"reps" in lib.npm_last_error()
    assert list(out) == [-1.0] * 4            # written only on success


def test_version_and_last_error():
    lib = B.lib()
    assert b"gfx950" in lib.npm_version()
    assert lib.npm_create(None, None) == -1
    assert b"null" in lib.npm_last_error()


@pytest.mark.parametrize("net", [W.CFG1, W.CFG2, W.CFG5, W.TINY], ids=["cfg1", "cfg2", "cfg5", "tiny"])
def test_layout_matches_oracle(O, net):
    cfg = B.make_config(net)
    L = B.layout_of(cfg)
    on = O.Net(net.n_levels, net.feat, net.base_res, net.max_res, net.log2_table, net.dense_only,
               net.n_hidden, net.width, net.n_lobes)
    assert L.n_params == on.n_params and L.grid_params == on.grid_params
    assert L.grid_entries == on.grid_entries
    for l in range(net.n_levels):
        assert L.resolution[l] == on.res[l]
        assert L.hashed[l] == on.hashed[l]
        assert L.level_size[l] == on.level_size[l]
        assert L.level_offset[l] == on.level_offset[l]
    assert L.n_layers == len(on.layer_offset)
    for i in range(L.n_layers):
        assert L.layer_offset[i] == on.layer_offset[i]
        assert (L.layer_out[i], L.layer_in[i]) == on.layer_shape[i]


@pytest.mark.parametrize("net", ["CFG2P", "TINYP", "PAPERP"])
def test_product_layout_matches_oracle(O, net):
    """NPM-product (Sec. 4.3): G(x) then 2 * sh_degree^2 + 1 extra inputs;
    the flat layout of the library equals the oracle's."""
    cfg = getattr(W, net)
    L = B.layout_of(B.make_config(cfg, exec_mode=B.EXEC_FUSED))
    on = O.Net(cfg.n_levels, cfg.feat, cfg.base_res, cfg.max_res, cfg.log2_table, cfg.dense_only,
               cfg.n_hidden, cfg.width, cfg.n_lobes, sh_degree=cfg.sh_degree)
    assert L.n_in == on.n_in == cfg.n_levels * cfg.feat + 2 * cfg.sh_degree ** 2 + 1
    assert L.n_params == on.n_params and L.grid_params == on.grid_params
    for i in range(L.n_layers):
        assert L.layer_offset[i] == on.layer_offset[i]
        assert (L.layer_out[i], L.layer_in[i]) == on.layer_shape[i]


def test_product_shapes():
    lib = B.lib()
    out = B.npm_layout()
    c = B.make_config(W.CFG1, exec_mode=B.EXEC_FUSED, sh_degree=4)   # 16 grid features
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == -1        # no fused kernels
    c = B.make_config(W.CFG1, exec_mode=B.EXEC_STAGED, sh_degree=4)
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == 0 and out.n_in == 16 + 33
    c = B.make_config(W.CFG2, sh_degree=5)
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == -1


def test_invalid_configs_rejected_without_device():
    lib = B.lib()
    base = B.make_config(W.CFG2)
    out = B.npm_layout()
    for field, value in [("n_levels", 0), ("n_levels", 33), ("feat_per_level", 3),
                         ("n_lobes", 4), ("mlp_width", 65), ("mlp_hidden_layers", 0),
                         ("log2_table_size", 40), ("precision", 7), ("lr", -1.0),
                         ("beta1", 1.0), ("max_resolution", 8), ("batch_order", 3),
                         ("ema_decay", 1.0), ("ema_decay", -0.5), ("scatter_mode", 3),
                         ("scatter_mode", -1)]:
        c = B.npm_config.from_buffer_copy(base)
        setattr(c, field, value)
        assert lib.npm_get_layout(C.byref(c), C.byref(out)) == -1, field
        ctx = C.c_void_p()
        assert lib.npm_create(C.byref(c), C.byref(ctx)) == -1, field
        assert not ctx
    c = B.npm_config.from_buffer_copy(base)
    c.precision = B.PREC_BF16
    c.exec_mode = B.EXEC_STAGED
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == -1
    # a fused context needs kernels for its shape: 16 inputs into three
    # 32-wide hidden layers have none (the staged path takes it)
    c = B.npm_config.from_buffer_copy(base)
    c.n_levels, c.mlp_width, c.exec_mode = 8, 32, B.EXEC_FUSED
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == -1
    assert b"no fused kernels" in lib.npm_last_error()
    c.exec_mode = B.EXEC_STAGED
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == 0


def test_explicit_resolution_table_matches_oracle(O):
    """npm_config.resolution: an explicit integer table (Sec. 5.1 leaves the
    growth rule open) gives the oracle's layout for the same table; invalid
    tables are rejected."""
    from dataclasses import replace
    table = (5, 7, 13, 13, 40, 97)
    net = replace(W.TINY, n_levels=6, log2_table=12, width=64, resolution=table)
    L = B.layout_of(B.make_config(net, exec_mode=B.EXEC_FUSED))
    on = O.Net(net.n_levels, net.feat, net.base_res, net.max_res, net.log2_table, net.dense_only,
               net.n_hidden, net.width, net.n_lobes, resolution=table)
    assert [L.resolution[l] for l in range(6)] == list(table) == on.res
    assert [L.hashed[l] for l in range(6)] == on.hashed
    assert [L.level_offset[l] for l in range(6)] == on.level_offset
    assert L.n_params == on.n_params
    lib = B.lib()
    out = B.npm_layout()
    for bad in ((5, 4, 13, 13, 40, 97), (0, 7, 13, 13, 40, 97), (5, 7, 13, 13, 40, 70000)):
        c = B.make_config(replace(net, resolution=bad))
        assert lib.npm_get_layout(C.byref(c), C.byref(out)) == -1, bad
    c = B.make_config(net)
    c.resolution[6] = 9                         # an entry past n_levels
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == -1


@pytest.mark.parametrize("net", ["TINYS", "CFG1S", "PAPERS"])
def test_selection_layout_matches_oracle(O, net):
    """learn_selection (the Sec. 6.3 extension): the last layer gets one more
    row, 4K + 1 outputs, as in the oracle."""
    net = getattr(W, net)
    L = B.layout_of(B.make_config(net))
    on = O.Net(net.n_levels, net.feat, net.base_res, net.max_res, net.log2_table, net.dense_only,
               net.n_hidden, net.width, net.n_lobes, select=True)
    plain = B.layout_of(B.make_config(net, learn_selection=False))
    assert L.n_out == on.n_out == 4 * net.n_lobes + 1 and plain.n_out == 4 * net.n_lobes
    assert L.n_params == on.n_params == plain.n_params + net.width
    for i in range(L.n_layers):
        assert L.layer_offset[i] == on.layer_offset[i]
        assert (L.layer_out[i], L.layer_in[i]) == on.layer_shape[i]


def test_selection_config_rules():
    """The selection output runs on the staged path for any shape and fused
    for the shapes with kernels for it; the flag is 0 or 1; the selection
    calls refuse a null context."""
    from dataclasses import replace
    lib = B.lib()
    out = B.npm_layout()
    for net in (W.TINYS, W.CFG1S, W.PAPERS, replace(W.CFG2, select=True)):
        for mode in (B.EXEC_STAGED, B.EXEC_FUSED):
            c = B.make_config(net, exec_mode=mode)
            assert lib.npm_get_layout(C.byref(c), C.byref(out)) == 0, (net, mode)
    c = B.make_config(replace(W.TINYS, n_hidden=3), exec_mode=B.EXEC_FUSED)
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == -1
    assert b"selection output" in lib.npm_last_error()
    c = B.make_config(replace(W.TINYS, sh_degree=2), exec_mode=B.EXEC_FUSED)
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == -1
    c.exec_mode = B.EXEC_STAGED
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == 0
    c = B.make_config(W.TINYS)
    c.learn_selection = 2
    assert lib.npm_get_layout(C.byref(c), C.byref(out)) == -1
    assert lib.npm_query_select(None, 4, None, None, None, 0, 0, None, None, None, None, None,
                                None) == -1
    assert lib.npm_backward_select(None, 4, None, None, None, None, None, None, None, None,
                                   None) == -1
    assert lib.npm_train_step_select(None, 4, None, None, None, None, None, None, None,
                                     None) == -1


def test_moving_average_adds_its_buffers_to_the_layout():
    """A kept moving average (Sec. 5.3's inference weights) costs an FP32
    copy of the parameters, its packed images and, in the precision form,
    its FP16 grid."""
    for net in (W.CFG2, W.CFG3):
        off, on = (B.layout_of(B.make_config(net, exec_mode=B.EXEC_FUSED, ema_decay=d))
                   for d in (0.0, 0.99))
        extra = on.device_bytes - off.device_bytes
        lowp = 2 * off.grid_params if net.precision == "bf16" else 0
        assert extra > 4 * off.n_params + lowp
        assert extra < 4 * off.n_params + lowp + 6 * 64 * 1024


def test_null_context_calls_fail_cleanly():
    lib = B.lib()
    assert lib.npm_destroy(None) == 0
    assert lib.npm_query(None, 10, None, None, 0, 0, None, None, None, None, None) == -1
    assert lib.npm_train_step(None, 10, None, None, None, None, None, None) == -1
    assert lib.npm_optimizer_step(None, None, None, None) == -1
    assert lib.npm_get_state(None, 0, None, 0) == -1


def test_create_without_gpu_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cfg = B.make_config(W.CFG1)
    ctx = C.c_void_p()
    assert B.lib().npm_create(C.byref(cfg), C.byref(ctx)) == -2
