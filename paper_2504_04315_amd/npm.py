"""Thin Python binding of libnpm.so (include/npm.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  PyTorch provides device memory and the current HIP stream; batch
tensors must be float32 CUDA (HIP) tensors in the SoA layout the C ABI
documents.  The module fails loudly if the library has not been built.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnpm.so")

NPM_OK = 0
STATUS = {0: "NPM_OK", -1: "NPM_ERR_INVALID_ARG", -2: "NPM_ERR_NO_DEVICE", -3: "NPM_ERR_OOM",
          -4: "NPM_ERR_BUDGET", -5: "NPM_ERR_HIP", -6: "NPM_ERR_STATE", -7: "NPM_ERR_TIMEOUT"}
GRID_DENSE, GRID_HASH = 0, 1
PREC_FP32, PREC_BF16 = 0, 1
EXEC_STAGED, EXEC_FUSED = 0, 1
ORDER_AUTO, ORDER_NONE, ORDER_SPATIAL = 0, 1, 2
SCATTER_AUTO, SCATTER_ATOMIC, SCATTER_BINNED = 0, 1, 2
INIT_NORMAL, INIT_UNIFORM = 0, 1
STATE_PARAMS, STATE_GRADS, STATE_ADAM_M, STATE_ADAM_V, STATE_EMA = 0, 1, 2, 3, 4
MAX_LEVELS, MAX_LAYERS = 32, 5


class npm_config(C.Structure):
    _fields_ = [
        ("grid_kind", C.c_int32), ("n_levels", C.c_int32), ("feat_per_level", C.c_int32),
        ("log2_table_size", C.c_int32), ("base_resolution", C.c_int32),
        ("max_resolution", C.c_int32), ("mlp_width", C.c_int32),
        ("mlp_hidden_layers", C.c_int32), ("n_lobes", C.c_int32), ("precision", C.c_int32),
        ("exec_mode", C.c_int32), ("grid_init", C.c_int32), ("grid_init_scale", C.c_float),
        ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
        ("batch_order", C.c_int32), ("ema_decay", C.c_float), ("sh_degree", C.c_int32),
        ("scatter_mode", C.c_int32), ("resolution", C.c_int32 * MAX_LEVELS),
        ("learn_selection", C.c_int32), ("seed", C.c_uint64),
    ]


class npm_layout(C.Structure):
    _fields_ = [
        ("n_params", C.c_int64), ("grid_entries", C.c_int64), ("grid_params", C.c_int64),
        ("level_offset", C.c_int64 * MAX_LEVELS), ("level_size", C.c_int64 * MAX_LEVELS),
        ("layer_offset", C.c_int64 * MAX_LAYERS), ("resolution", C.c_int32 * MAX_LEVELS),
        ("hashed", C.c_int32 * MAX_LEVELS), ("layer_in", C.c_int32 * MAX_LAYERS),
        ("layer_out", C.c_int32 * MAX_LAYERS), ("n_layers", C.c_int32), ("n_in", C.c_int32),
        ("n_out", C.c_int32), ("reserved", C.c_int32), ("device_bytes", C.c_int64),
    ]


class npm_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double)]


# C ABI entry points and their argument types (the names of include/npm.h).
_P, _i64, _u64, _u32, _i32 = C.c_void_p, C.c_int64, C.c_uint64, C.c_uint32, C.c_int
SIGNATURES = {
    "npm_config_default": [_P],
    "npm_get_layout": [_P, _P],
    "npm_create": [_P, _P],
    "npm_destroy": [_P],
    "npm_query": [_P, _i64, _P, _P, _u64, _u32, _P, _P, _P, _P, _P],
    "npm_backward": [_P, _i64, _P, _P, _P, _P, _P, _P, _P],
    "npm_loss": [_P, _i64, _P, _P, _P, _P, _P, _P],
    "npm_optimizer_step": [_P, _P, _P, _P],
    "npm_train_step": [_P, _i64, _P, _P, _P, _P, _P, _P],
    "npm_corner_index": [_P, _i64, _P, _P, _P],
    "npm_encode": [_P, _i64, _P, _P, _P],
    "npm_forward_raw": [_P, _i64, _P, _P, _P],
    "npm_get_state": [_P, _i32, _P, _i64],
    "npm_set_state": [_P, _i32, _P, _i64],
    "npm_get_step": [_P, _P],
    "npm_set_step": [_P, _i64],
    "npm_state_device_ptr": [_P, _i32, _P],
    "npm_set_timing": [_P, _i32],
    "npm_kernel_times": [_P, _P, C.c_int32, _P],
    "npm_reset_timing": [_P],
    "npm_query_aux": [_P, _i64, _P, _P, _P, _u64, _u32, _P, _P, _P, _P, _P],
    "npm_backward_aux": [_P, _i64, _P, _P, _P, _P, _P, _P, _P, _P],
    "npm_loss_aux": [_P, _i64, _P, _P, _P, _P, _P, _P, _P],
    "npm_train_step_aux": [_P, _i64, _P, _P, _P, _P, _P, _P, _P],
    "npm_encode_aux": [_P, _i64, _P, _P, _P, _P],
    "npm_forward_raw_aux": [_P, _i64, _P, _P, _P, _P],
    "npm_backward_static": [_P, _i64, _P, _P, _P, _P, _P, _P, _P, _P],
    "npm_query_select": [_P, _i64, _P, _P, _P, _u64, _u32, _P, _P, _P, _P, _P, _P],
    "npm_backward_select": [_P, _i64, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "npm_train_step_select": [_P, _i64, _P, _P, _P, _P, _P, _P, _P, _P],
    "npm_measure_peaks": [_P, _i32],
}
STATIC_MAX_N = 32768

_lib = None


class NPMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded libnpm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2504_04315_amd/build.py "
                              "(python -m paper_2504_04315_amd.build); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.npm_last_error.restype = C.c_char_p
        L.npm_last_error.argtypes = []
        L.npm_version.restype = C.c_char_p
        L.npm_version.argtypes = []
        _lib = L
    return _lib


def check(status):
    if status != NPM_OK:
        raise NPMError(status, lib().npm_last_error().decode())
    return status


def make_config(net, exec_mode=EXEC_STAGED, precision=None, lr=None, seed=None,
                batch_order=ORDER_AUTO, ema_decay=0.0, sh_degree=None, scatter_mode=SCATTER_AUTO,
                learn_selection=None):
    """npm_config from a workload.NetConfig (sizes of a workload)."""
    c = npm_config()
    check(lib().npm_config_default(C.byref(c)))
    c.grid_kind = GRID_DENSE if net.dense_only else GRID_HASH
    c.n_levels, c.feat_per_level = net.n_levels, net.feat
    c.log2_table_size = net.log2_table
    c.base_resolution, c.max_resolution = net.base_res, net.max_res
    c.mlp_width, c.mlp_hidden_layers, c.n_lobes = net.width, net.n_hidden, net.n_lobes
    prec = net.precision if precision is None else precision
    c.precision = PREC_BF16 if prec in ("bf16", PREC_BF16) else PREC_FP32
    c.exec_mode = EXEC_FUSED if c.precision == PREC_BF16 else exec_mode
    c.grid_init = INIT_NORMAL if net.grid_init == "normal" else INIT_UNIFORM
    c.grid_init_scale = net.grid_init_scale
    c.lr = net.lr if lr is None else lr
    c.beta1, c.beta2, c.eps = net.beta1, net.beta2, net.eps
    c.seed = net.seed if seed is None else seed
    c.batch_order = batch_order
    c.scatter_mode = scatter_mode
    c.ema_decay = ema_decay
    c.sh_degree = getattr(net, "sh_degree", 0) if sh_degree is None else sh_degree
    for l, d in enumerate(getattr(net, "resolution", None) or ()):
        c.resolution[l] = d
    sel = getattr(net, "select", False) if learn_selection is None else learn_selection
    c.learn_selection = int(bool(sel))
    return c


def layout_of(cfg):
    out = npm_layout()
    check(lib().npm_get_layout(C.byref(cfg), C.byref(out)))
    return out


def _ptr(t):
    if t is None:
        return None
    import torch
    assert t.is_cuda, "device tensor expected"
    assert t.dtype in (torch.float32, torch.int32, torch.float64), t.dtype
    assert t.is_contiguous(), "contiguous tensor expected"
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class NPM:
    """One guiding network (a libnpm context) on the current device."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.layout = layout_of(cfg)
        self._ctx = C.c_void_p()
        check(lib().npm_create(C.byref(cfg), C.byref(self._ctx)))

    # -- lifetime
    def close(self):
        if self._ctx:
            check(lib().npm_destroy(self._ctx))
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._ctx

    @property
    def n_params(self):
        return self.layout.n_params

    # -- hot path
    def query(self, pos, dir=None, seed=0, stream_id=0, lobes=True, pdf=None, sample=True,
              stream=None, aux=None):
        """Returns dict with lobes [4][8][n], pdf [n], sample_dir [3][n], sample_pdf [n].
        aux: the NPM-product inputs [7][n] (omega_o, normal, roughness)."""
        import torch
        n = pos.shape[1]
        dev = pos.device
        out = {}
        out["lobes"] = torch.empty((4, 8, n), device=dev) if lobes else None
        want_pdf = (dir is not None) if pdf is None else pdf
        out["pdf"] = torch.empty(n, device=dev) if want_pdf else None
        out["sample_dir"] = torch.empty((3, n), device=dev) if sample else None
        out["sample_pdf"] = torch.empty(n, device=dev) if sample else None
        check(lib().npm_query_aux(self._ctx, n, _ptr(pos), _ptr(aux), _ptr(dir), seed, stream_id,
                                  _ptr(out["lobes"]), _ptr(out["pdf"]), _ptr(out["sample_dir"]),
                                  _ptr(out["sample_pdf"]), _stream(stream)))
        return out

    def backward(self, pos, dir, radiance, pdf, grad=None, loss=None, stream=None, aux=None):
        check(lib().npm_backward_aux(self._ctx, pos.shape[1], _ptr(pos), _ptr(aux), _ptr(dir),
                                     _ptr(radiance), _ptr(pdf), _ptr(grad), _ptr(loss),
                                     _stream(stream)))

    def backward_static(self, pos, dir, radiance, pdf, grad=None, loss=None, stream=None,
                        aux=None):
        """npm_backward_static: npm_backward with no allocation (fixed scratch)."""
        check(lib().npm_backward_static(self._ctx, pos.shape[1], _ptr(pos), _ptr(aux), _ptr(dir),
                                        _ptr(radiance), _ptr(pdf), _ptr(grad), _ptr(loss),
                                        _stream(stream)))

    def loss(self, pos, dir, radiance, pdf, out=None, stream=None, aux=None):
        import torch
        out = torch.zeros(1, dtype=torch.float64, device=pos.device) if out is None else out
        check(lib().npm_loss_aux(self._ctx, pos.shape[1], _ptr(pos), _ptr(aux), _ptr(dir),
                                 _ptr(radiance), _ptr(pdf), _ptr(out), _stream(stream)))
        return out

    def optimizer_step(self, grad=None, gradnorm=None, stream=None):
        check(lib().npm_optimizer_step(self._ctx, _ptr(grad), _ptr(gradnorm), _stream(stream)))

    def train_step(self, pos, dir, radiance, pdf, stats=None, stream=None, aux=None):
        check(lib().npm_train_step_aux(self._ctx, pos.shape[1], _ptr(pos), _ptr(aux), _ptr(dir),
                                       _ptr(radiance), _ptr(pdf), _ptr(stats), _stream(stream)))

    # -- learned BSDF-selection probability (learn_selection networks)
    def query_select(self, pos, dir=None, seed=0, stream_id=0, lobes=True, pdf=None, sample=True,
                     stream=None, aux=None):
        """query() plus "select_prob" [n], the probability of sampling the BSDF."""
        import torch
        n = pos.shape[1]
        dev = pos.device
        out = {}
        out["lobes"] = torch.empty((4, 8, n), device=dev) if lobes else None
        want_pdf = (dir is not None) if pdf is None else pdf
        out["pdf"] = torch.empty(n, device=dev) if want_pdf else None
        out["sample_dir"] = torch.empty((3, n), device=dev) if sample else None
        out["sample_pdf"] = torch.empty(n, device=dev) if sample else None
        out["select_prob"] = torch.empty(n, device=dev)
        check(lib().npm_query_select(self._ctx, n, _ptr(pos), _ptr(aux), _ptr(dir), seed,
                                     stream_id, _ptr(out["lobes"]), _ptr(out["pdf"]),
                                     _ptr(out["sample_dir"]), _ptr(out["sample_pdf"]),
                                     _ptr(out["select_prob"]), _stream(stream)))
        return out

    def backward_select(self, pos, dir, radiance, pdf, bsdf_pdf, grad=None, loss=None,
                        stream=None, aux=None):
        """npm_backward_select; loss: two doubles (mixture, selection) or None."""
        check(lib().npm_backward_select(self._ctx, pos.shape[1], _ptr(pos), _ptr(aux), _ptr(dir),
                                        _ptr(radiance), _ptr(pdf), _ptr(bsdf_pdf), _ptr(grad),
                                        _ptr(loss), _stream(stream)))

    def train_step_select(self, pos, dir, radiance, pdf, bsdf_pdf, stats=None, stream=None,
                          aux=None):
        """npm_train_step_select; stats: three doubles (loss, loss_sel, |g|^2) or None."""
        check(lib().npm_train_step_select(self._ctx, pos.shape[1], _ptr(pos), _ptr(aux),
                                          _ptr(dir), _ptr(radiance), _ptr(pdf), _ptr(bsdf_pdf),
                                          _ptr(stats), _stream(stream)))

    # -- stage outputs
    def corner_index(self, pos, stream=None):
        import torch
        n = pos.shape[1]
        idx = torch.empty((self.cfg.n_levels, 8, n), dtype=torch.int32, device=pos.device)
        check(lib().npm_corner_index(self._ctx, n, _ptr(pos), _ptr(idx), _stream(stream)))
        return idx

    def encode(self, pos, stream=None, aux=None):
        import torch
        n = pos.shape[1]
        G = torch.empty((self.layout.n_in, n), device=pos.device)
        check(lib().npm_encode_aux(self._ctx, n, _ptr(pos), _ptr(aux), _ptr(G), _stream(stream)))
        return G

    def forward_raw(self, pos, stream=None, aux=None):
        import torch
        n = pos.shape[1]
        raw = torch.empty((self.layout.n_out, n), device=pos.device)
        check(lib().npm_forward_raw_aux(self._ctx, n, _ptr(pos), _ptr(aux), _ptr(raw),
                                        _stream(stream)))
        return raw

    # -- state
    def get_state(self, which=STATE_PARAMS):
        a = np.empty(self.n_params, dtype=np.float32)
        check(lib().npm_get_state(self._ctx, which, a.ctypes.data_as(C.c_void_p), a.size))
        return a

    def set_state(self, a, which=STATE_PARAMS):
        a = np.ascontiguousarray(a, dtype=np.float32)
        check(lib().npm_set_state(self._ctx, which, a.ctypes.data_as(C.c_void_p), a.size))

    @property
    def step(self):
        v = C.c_int64()
        check(lib().npm_get_step(self._ctx, C.byref(v)))
        return v.value

    @step.setter
    def step(self, v):
        check(lib().npm_set_step(self._ctx, int(v)))

    def device_ptr(self, which=STATE_PARAMS):
        p = C.c_void_p()
        check(lib().npm_state_device_ptr(self._ctx, which, C.byref(p)))
        return p.value

    def state_tensor(self, which=STATE_PARAMS):
        """A torch tensor aliasing a state buffer of the context (no copy)."""
        import torch
        ptr = self.device_ptr(which)

        class _Buf:
            __cuda_array_interface__ = {"shape": (self.n_params,), "typestr": "<f4",
                                        "data": (ptr, False), "version": 2, "strides": None}
        return torch.as_tensor(_Buf(), device="cuda")

    # -- timing
    def set_timing(self, enabled=True):
        check(lib().npm_set_timing(self._ctx, int(enabled)))

    def reset_timing(self):
        check(lib().npm_reset_timing(self._ctx))

    def kernel_times(self):
        arr = (npm_kernel_time * 64)()
        cnt = C.c_int32()
        check(lib().npm_kernel_times(self._ctx, arr, 64, C.byref(cnt)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms)
                for i in range(min(cnt.value, 64))}


def measure_peaks(reps=3):
    """Achievable rates of the current device (include/npm_probe.h): FP32 and
    BF16 matrix TFLOP/s, HBM read and copy GB/s, each the best of `reps`."""
    out = (C.c_double * 4)()
    check(lib().npm_measure_peaks(out, int(reps)))
    return {"mfma_f32_tflops": out[0], "mfma_bf16_tflops": out[1], "hbm_read_gbs": out[2],
            "hbm_copy_gbs": out[3]}
