"""ctypes wrapper of the FP64 CPU oracle (oracle/npm_oracle.c).

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It never imports the HIP library
and the library never imports it.

All arrays are numpy.  Positions and directions are float32 SoA [3][n], as the
library takes them; parameters are the flat FP32 parameter vector promoted to
float64 (exactly).  Per-vertex outputs are row-major [n][...] float64.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

MAX_LEVELS = 32
MAX_LAYERS = 8


class NpmoNet(C.Structure):
    _fields_ = [
        ("size", C.c_int64 * MAX_LEVELS),
        ("offset", C.c_int64 * MAX_LEVELS),
        ("layer_offset", C.c_int64 * MAX_LAYERS),
        ("grid_entries", C.c_int64),
        ("grid_params", C.c_int64),
        ("n_params", C.c_int64),
        ("res", C.c_int32 * MAX_LEVELS),
        ("hashed", C.c_int32 * MAX_LEVELS),
        ("layer_in", C.c_int32 * MAX_LAYERS),
        ("layer_out", C.c_int32 * MAX_LAYERS),
        ("n_levels", C.c_int32), ("feat", C.c_int32), ("log2_table", C.c_int32),
        ("dense_only", C.c_int32), ("base_res", C.c_int32), ("max_res", C.c_int32),
        ("n_in", C.c_int32), ("width", C.c_int32), ("n_hidden", C.c_int32),
        ("n_lobes", C.c_int32), ("n_layers", C.c_int32), ("n_out", C.c_int32),
        ("sh_degree", C.c_int32), ("n_aux", C.c_int32), ("select", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        P = C.c_void_p
        i64, u64, u32, i32 = C.c_int64, C.c_uint64, C.c_uint32, C.c_int
        L.npmo_net_init.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, i32, i32]
        L.npmo_net_init.restype = i32
        L.npmo_philox.argtypes = [P, P, P]
        L.npmo_uniforms.argtypes = [i64, P, u64, u32, u32, P]
        L.npmo_corners.argtypes = [P, i64, P, P, P]
        L.npmo_net_set_resolution.argtypes = [P, P]
        L.npmo_net_set_resolution.restype = i32
        L.npmo_net_set_inputs.argtypes = [P, i32]
        L.npmo_net_set_inputs.restype = i32
        L.npmo_net_set_selection.argtypes = [P, i32]
        L.npmo_net_set_selection.restype = i32
        L.npmo_sh.argtypes = [i32, C.c_double, C.c_double, C.c_double, P, P]
        L.npmo_encode.argtypes = [P, i64, P, P, P, P, P]
        L.npmo_mlp_forward.argtypes = [P, i64, P, P, P, P]
        L.npmo_head.argtypes = [P, i64, P, P]
        L.npmo_logpdf.argtypes = [P, i64, P, P, P]
        L.npmo_query.argtypes = [P, i64, P, P, P, P, u64, u32, P, P, P, P, P, P, P, P, P, P]
        L.npmo_sample_raw.argtypes = [P, i64, P, P, P, P]
        L.npmo_loss_grad.argtypes = [P, i64, i64, P, P, P, P, P, P, P]
        L.npmo_loss_grad.restype = C.c_double
        L.npmo_backward.argtypes = [P, i64, i64, P, P, P, P, P, P, P, P, P, P, P, P]
        L.npmo_backward.restype = C.c_double
        L.npmo_backward_cond.argtypes = [P, i64, i64, P, P, P, P, P, P, P, P]
        L.npmo_adam.argtypes = [i64, P, P, P, P, i64, C.c_double, C.c_double, C.c_double,
                                C.c_double]
        L.npmo_ema.argtypes = [i64, P, P, C.c_double]
        L.npmo_backward_threads.argtypes = [P, i64, i32]
        L.npmo_backward_threads.restype = i32
        L.npmo_set_threads.argtypes = [C.c_int]
        L.npmo_set_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32soa(a, n):
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.shape == (3, n), a.shape
    return a


def _aux(net, aux, n):
    """The NPM-product inputs [7][n] float32 (omega_o, normal, roughness)."""
    if not net.n_aux:
        return None
    assert aux is not None, "this network takes omega_o, normal and roughness"
    a = np.ascontiguousarray(aux, dtype=np.float32)
    assert a.shape == (7, n), a.shape
    return a


def sh(degree, v):
    """Real orthonormal spherical harmonics of `degree` bands at the vectors
    v [m][3]: values [m][degree^2] and their condition scales."""
    v = np.asarray(v, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((v.shape[0], degree * degree))
    sc = np.zeros_like(out)
    for i in range(v.shape[0]):
        o = np.zeros(degree * degree)
        c = np.zeros(degree * degree)
        lib().npmo_sh(degree, v[i, 0], v[i, 1], v[i, 2], _p(o), _p(c))
        out[i], sc[i] = o, c
    return out, sc


class Net:
    """Network shape and grid layout, computed by the oracle from the paper's
    rules (Sec. 5.1 level resolutions; Sec. 5.3 MLP)."""

    def __init__(self, n_levels, feat, base_res, max_res, log2_table, dense_only,
                 n_hidden, width, n_lobes=8, sh_degree=0, resolution=None, select=False):
        self.s = NpmoNet()
        rc = lib().npmo_net_init(C.byref(self.s), n_levels, feat, base_res, max_res,
                                 log2_table, int(dense_only), n_hidden, width, n_lobes)
        if rc == 0 and resolution:
            if len(resolution) != n_levels:
                raise ValueError("oracle: one resolution per level")
            r = np.ascontiguousarray(resolution, dtype=np.int32)
            rc = lib().npmo_net_set_resolution(C.byref(self.s), _p(r))
        if rc == 0 and sh_degree:
            rc = lib().npmo_net_set_inputs(C.byref(self.s), sh_degree)
        if rc == 0 and select:
            rc = lib().npmo_net_set_selection(C.byref(self.s), 1)
        if rc != 0:
            raise ValueError("oracle: invalid network shape")
        self.sh_degree, self.n_aux = self.s.sh_degree, self.s.n_aux
        self.select = bool(self.s.select)
        s = self.s
        self.n_levels, self.feat, self.n_in = s.n_levels, s.feat, s.n_in
        self.n_out, self.n_lobes, self.n_params = s.n_out, s.n_lobes, s.n_params
        self.grid_params, self.grid_entries = s.grid_params, s.grid_entries
        self.res = [s.res[i] for i in range(s.n_levels)]
        self.hashed = [s.hashed[i] for i in range(s.n_levels)]
        self.level_size = [s.size[i] for i in range(s.n_levels)]
        self.level_offset = [s.offset[i] for i in range(s.n_levels)]
        self.layer_offset = [s.layer_offset[i] for i in range(s.n_layers)]
        self.layer_shape = [(s.layer_out[i], s.layer_in[i]) for i in range(s.n_layers)]

    @property
    def ref(self):
        return C.byref(self.s)

    def weights(self, params, i):
        o, k = self.layer_shape[i]
        off = self.layer_offset[i]
        return params[off:off + o * k].reshape(o, k)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().npmo_philox(_p(c), _p(k), _p(out))
    return out


def uniforms(n, seed, stream, sample=0, vid=None):
    u = np.zeros((n, 3))
    v = None if vid is None else np.ascontiguousarray(vid, dtype=np.int64)
    lib().npmo_uniforms(n, _p(v), seed, stream, sample, _p(u))
    return u


def corners(net, pos):
    n = pos.shape[1]
    pos = _f32soa(pos, n)
    idx = np.zeros((n, net.n_levels, 8), dtype=np.int64)
    w = np.zeros((n, net.n_levels, 8))
    lib().npmo_corners(net.ref, n, _p(pos), _p(idx), _p(w))
    return idx, w


def encode(net, pos, params, with_scale=False, aux=None):
    n = pos.shape[1]
    pos = _f32soa(pos, n)
    ax = _aux(net, aux, n)
    params = np.ascontiguousarray(params, dtype=np.float64)
    G = np.zeros((n, net.n_in))
    S = np.zeros((n, net.n_in)) if with_scale else None
    lib().npmo_encode(net.ref, n, _p(pos), _p(ax), _p(params), _p(G), _p(S))
    return (G, S) if with_scale else G


def mlp_forward(net, G, params, with_scale=False):
    G = np.ascontiguousarray(G, dtype=np.float64)
    n = G.shape[0]
    params = np.ascontiguousarray(params, dtype=np.float64)
    raw = np.zeros((n, net.n_out))
    S = np.zeros((n, net.n_out)) if with_scale else None
    lib().npmo_mlp_forward(net.ref, n, _p(G), _p(params), _p(raw), _p(S))
    return (raw, S) if with_scale else raw


def head(net, raw):
    raw = np.ascontiguousarray(raw, dtype=np.float64)
    n = raw.shape[0]
    lobes = np.zeros((n, net.n_lobes, 4))
    lib().npmo_head(net.ref, n, _p(raw), _p(lobes))
    return lobes


def logpdf(net, raw, dirs):
    """dirs: [n][3] float64 (any unit vectors)."""
    raw = np.ascontiguousarray(raw, dtype=np.float64)
    dirs = np.ascontiguousarray(dirs, dtype=np.float64)
    n = raw.shape[0]
    out = np.zeros(n)
    lib().npmo_logpdf(net.ref, n, _p(raw), _p(dirs), _p(out))
    return out


def sample_raw(net, raw, u):
    raw = np.ascontiguousarray(raw, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = raw.shape[0]
    d = np.zeros((n, 3))
    lobe = np.zeros(n, dtype=np.int32)
    lib().npmo_sample_raw(net.ref, n, _p(raw), _p(u), _p(d), _p(lobe))
    return d, lobe


def query(net, pos, params, dirs=None, seed=0, stream=0, vid=None, aux=None):
    """Full query: returns a dict of G, raw, lobes [n][K][4], logpdf (if dirs),
    sample dir [n][3], sample logpdf, sampled lobe, CDF margin and, on a
    network with the selection output, the selection probability sel [n]."""
    n = pos.shape[1]
    pos = _f32soa(pos, n)
    ax = _aux(net, aux, n)
    d = None if dirs is None else _f32soa(dirs, n)
    params = np.ascontiguousarray(params, dtype=np.float64)
    v = None if vid is None else np.ascontiguousarray(vid, dtype=np.int64)
    out = dict(G=np.zeros((n, net.n_in)), raw=np.zeros((n, net.n_out)),
               lobes=np.zeros((n, net.n_lobes, 4)),
               logpdf=np.zeros(n) if d is not None else None,
               sdir=np.zeros((n, 3)), slogpdf=np.zeros(n), slobe=np.zeros(n, dtype=np.int32),
               margin=np.zeros(n), sel=np.zeros(n) if net.select else None)
    lib().npmo_query(net.ref, n, _p(pos), _p(ax), _p(d), _p(v), seed, stream, _p(params),
                     _p(out["G"]), _p(out["raw"]), _p(out["lobes"]), _p(out["logpdf"]),
                     _p(out["sdir"]), _p(out["slogpdf"]), _p(out["slobe"]), _p(out["margin"]),
                     _p(out["sel"]))
    return out


def _bsdf(bsdf, n):
    if bsdf is None:
        return None
    b = np.ascontiguousarray(bsdf, dtype=np.float32)
    assert b.shape == (n,), b.shape
    return b


def loss_grad(net, raw, dirs, rad, spdf, n_total=None):
    """Mixture loss and d loss / d raw [n][n_out] from raw outputs."""
    loss, _, draw = loss_grad_select(net, raw, dirs, rad, spdf, None, n_total)
    return loss, draw


def loss_grad_select(net, raw, dirs, rad, spdf, bsdf, n_total=None):
    """The mixture's loss, the selection term's loss and d loss / d raw
    [n][n_out] (the selection logit's column last) from raw outputs; bsdf
    [n] is the BSDF density of each sample's direction (None: no selection
    term)."""
    raw = np.ascontiguousarray(raw, dtype=np.float64)
    n = raw.shape[0]
    dirs = _f32soa(dirs, n)
    rad = np.ascontiguousarray(rad, dtype=np.float32)
    spdf = np.ascontiguousarray(spdf, dtype=np.float32)
    b = _bsdf(bsdf, n)
    draw = np.zeros((n, net.n_out))
    lsel = C.c_double(0.0)
    loss = lib().npmo_loss_grad(net.ref, n, n if n_total is None else n_total, _p(raw), _p(dirs),
                                _p(rad), _p(spdf), _p(b), _p(draw), C.byref(lsel))
    return loss, lsel.value, draw


def backward(net, pos, dirs, rad, spdf, params, n_total=None, with_abs=True, with_vertex=False,
             aux=None, bsdf=None):
    """Gradient of the surrogate loss w.r.t. the flat parameters (float64),
    the sum of |contributions| per parameter, and the loss value (loss: the
    mixture's term; loss_sel: the selection term, with bsdf [n] the BSDF
    density of each sample's direction on a network with the selection
    output)."""
    n = pos.shape[1]
    pos = _f32soa(pos, n)
    ax = _aux(net, aux, n)
    dirs = _f32soa(dirs, n)
    rad = np.ascontiguousarray(rad, dtype=np.float32)
    spdf = np.ascontiguousarray(spdf, dtype=np.float32)
    params = np.ascontiguousarray(params, dtype=np.float64)
    grad = np.zeros(net.n_params)
    gabs = np.zeros(net.n_params) if with_abs else None
    draw = np.zeros((n, net.n_out)) if with_vertex else None
    dG = np.zeros((n, net.n_in)) if with_vertex else None
    b = _bsdf(bsdf, n)
    lsel = C.c_double(0.0)
    loss = lib().npmo_backward(net.ref, n, n if n_total is None else n_total, _p(pos), _p(ax),
                               _p(dirs), _p(rad), _p(spdf), _p(b), _p(params), _p(grad), _p(gabs),
                               _p(draw), _p(dG), C.byref(lsel))
    out = dict(grad=grad, gabs=gabs, loss=loss, loss_sel=lsel.value)
    if with_vertex:
        out.update(draw=draw, dG=dG)
    return out


def backward_cond(net, pos, dirs, rad, spdf, params, n_total=None, aux=None, bsdf=None):
    """Condition scale of every gradient entry (float64): the sum of the
    absolute sizes of the terms an FP32 evaluation of the backward rounds,
    propagated from the KL-gradient head through the MLP and the scatter.
    Parity tolerances are relative to it."""
    n = pos.shape[1]
    pos = _f32soa(pos, n)
    ax = _aux(net, aux, n)
    dirs = _f32soa(dirs, n)
    rad = np.ascontiguousarray(rad, dtype=np.float32)
    spdf = np.ascontiguousarray(spdf, dtype=np.float32)
    params = np.ascontiguousarray(params, dtype=np.float64)
    b = _bsdf(bsdf, n)
    out = np.zeros(net.n_params)
    lib().npmo_backward_cond(net.ref, n, n if n_total is None else n_total, _p(pos), _p(ax),
                             _p(dirs), _p(rad), _p(spdf), _p(b), _p(params), _p(out))
    return out


def adam(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays; t is the 1-based step."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().npmo_adam(params.size, _p(params), _p(grad), _p(m), _p(v), t, lr, beta1, beta2, eps)


def ema(avg, params, decay):
    """In-place moving average of float64 arrays, after an optimizer step:
    avg <- decay * avg + (1 - decay) * params."""
    for a in (avg, params):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().npmo_ema(avg.size, _p(avg), _p(params), decay)


def backward_threads(net, n, with_abs=True):
    """Threads the oracle's backward runs a batch of n vertices on."""
    return lib().npmo_backward_threads(net.ref, n, int(with_abs))


def set_threads(n):
    """Sets the oracle's OpenMP thread count; returns the previous maximum."""
    return lib().npmo_set_threads(n)
