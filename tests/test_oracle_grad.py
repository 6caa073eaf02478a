"""Pins of the oracle's training gradient (Sec. 4.2, eq. mcgradients) and Adam.

- The head gradient d loss / d Theta' is checked against central finite
  differences of the oracle's own loss value (whose log-density is pinned in
  test_oracle_vmf) and against torch.autograd in float64 on an independent
  torch transcription that uses kappa / (4 pi sinh kappa) directly.
- Softmax invariance: sum_k d loss / d lambda'_k = 0.
- The full backward (MLP + grid scatter) of a tiny net is checked against
  central finite differences of the loss in every parameter.
- Adam against closed forms of Kingma and Ba's update.
"""
import math

import numpy as np
import pytest
import torch

from paper_2504_04315_amd import workload as W


def _head_case(rng, n=40):
    raw = rng.normal(size=(n, 32))
    raw[:, 2::4] = rng.uniform(-1.0, 3.0, (n, 8))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    dirs = d.T.astype(np.float32)
    rad = rng.exponential(size=n).astype(np.float32)
    pdf = rng.uniform(0.05, 1.0, n).astype(np.float32)
    rad[3] = 0.0          # zero radiance: no contribution
    pdf[5] = 0.0          # invalid pdf: weight 0
    rad[7] = np.inf       # non-finite: weight 0
    return raw, dirs, rad, pdf


@pytest.fixture(scope="module")
def net8(O):
    return O.Net(1, 1, 1, 1, 8, True, 1, 1, n_lobes=8)


def test_head_gradient_vs_finite_differences(O, net8):
    rng = np.random.default_rng(1)
    raw, dirs, rad, pdf = _head_case(rng)
    loss, draw = O.loss_grad(net8, raw, dirs, rad, pdf)
    h = 1e-6
    fd = np.zeros_like(raw)
    for j in range(32):
        rp = raw.copy(); rp[:, j] += h
        rm = raw.copy(); rm[:, j] -= h
        # per-vertex losses: evaluate one vertex at a time
        for i in range(raw.shape[0]):
            lp, _ = O.loss_grad(net8, rp[i:i + 1], dirs[:, i:i + 1], rad[i:i + 1], pdf[i:i + 1],
                                n_total=raw.shape[0])
            lm, _ = O.loss_grad(net8, rm[i:i + 1], dirs[:, i:i + 1], rad[i:i + 1], pdf[i:i + 1],
                                n_total=raw.shape[0])
            fd[i, j] = (lp - lm) / (2 * h)
    scale = np.abs(draw).max()
    np.testing.assert_allclose(draw, fd, rtol=0, atol=1e-7 * scale)
    assert np.all(draw[[3, 5, 7]] == 0.0)


def test_head_gradient_vs_torch_autograd(O, net8):
    rng = np.random.default_rng(2)
    raw, dirs, rad, pdf = _head_case(rng, n=64)
    loss, draw = O.loss_grad(net8, raw, dirs, rad, pdf)
    r = torch.tensor(raw, dtype=torch.float64, requires_grad=True)
    th = torch.sigmoid(r[:, 0::4]); ph = torch.sigmoid(r[:, 1::4])
    ka = torch.exp(r[:, 2::4]); lam = torch.softmax(r[:, 3::4], dim=1)
    T, P = math.pi * th, 2 * math.pi * ph
    mu = torch.stack([torch.sin(T) * torch.cos(P), torch.sin(T) * torch.sin(P), torch.cos(T)], -1)
    w = torch.tensor(dirs.T.astype(np.float64))
    cosv = (mu * w[:, None, :]).sum(-1)
    v = ka / (4 * math.pi * torch.sinh(ka)) * torch.exp(ka * cosv)
    V = (lam * v).sum(1)
    radd = rad.astype(np.float64); pdd = pdf.astype(np.float64)
    ok = np.isfinite(radd) & np.isfinite(pdd) & (pdd > 0) & (radd > 0)
    wt = torch.tensor(np.where(ok, radd / np.where(ok, pdd, 1.0), 0.0))
    L = -(wt * torch.log(V)).sum() / raw.shape[0]
    L.backward()
    assert float(L.detach()) == pytest.approx(loss, rel=1e-12)
    np.testing.assert_allclose(draw, r.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_softmax_gradient_sums_to_zero(O, net8):
    rng = np.random.default_rng(3)
    raw, dirs, rad, pdf = _head_case(rng, n=100)
    _, draw = O.loss_grad(net8, raw, dirs, rad, pdf)
    np.testing.assert_allclose(draw[:, 3::4].sum(axis=1), 0.0, atol=1e-15)


def _tiny(O):
    # 2-level hash grid (T = 2^8), F = 2, MLP 4 -> 8 -> 8 -> 32
    return O.Net(2, 2, 4, 16, 8, False, 2, 8)


def _tiny_batch(rng, n):
    pos = rng.random((3, n)).astype(np.float32)
    d = rng.normal(size=(n, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    return pos, d.T.astype(np.float32), rng.exponential(size=n).astype(np.float32), \
        np.full(n, 1 / (4 * math.pi), dtype=np.float32)


def test_full_backward_vs_finite_differences(O):
    net = _tiny(O)
    assert net.hashed == [0, 1]
    rng = np.random.default_rng(4)
    params = rng.normal(scale=0.6, size=net.n_params)
    n = 48
    pos, dirs, rad, pdf = _tiny_batch(rng, n)
    out = O.backward(net, pos, dirs, rad, pdf, params)
    g = out["grad"]
    h = 1e-6
    fd = np.zeros(net.n_params)
    touched = np.nonzero(out["gabs"])[0]
    for j in touched:
        p = params.copy(); p[j] += h
        lp = O.backward(net, pos, dirs, rad, pdf, p, with_abs=False)["loss"]
        p[j] -= 2 * h
        lm = O.backward(net, pos, dirs, rad, pdf, p, with_abs=False)["loss"]
        fd[j] = (lp - lm) / (2 * h)
    # untouched grid entries have exactly zero gradient
    assert np.all(g[out["gabs"] == 0] == 0)
    np.testing.assert_allclose(g, fd, rtol=0, atol=2e-7 * np.abs(g).max())
    # the loss is the mean over all samples of -w log V
    q = O.query(net, pos, params, dirs=dirs)
    w = rad.astype(np.float64) / pdf.astype(np.float64)
    assert out["loss"] == pytest.approx(-np.mean(w * q["logpdf"]), rel=1e-12)


def test_grid_gradient_sums_to_dG(O):
    # partition of unity: per level and feature, the scattered grid gradient
    # sums to the sum over vertices of dG
    net = O.Net(3, 2, 4, 32, 9, False, 1, 16)
    rng = np.random.default_rng(5)
    params = rng.normal(scale=0.4, size=net.n_params)
    pos, dirs, rad, pdf = _tiny_batch(rng, 200)
    out = O.backward(net, pos, dirs, rad, pdf, params, with_vertex=True)
    F = net.feat
    for l in range(3):
        a, b = net.level_offset[l] * F, (net.level_offset[l] + net.level_size[l]) * F
        for f in range(F):
            assert out["grad"][a + f:b:F].sum() == pytest.approx(out["dG"][:, l * F + f].sum(),
                                                                 rel=1e-12, abs=1e-15)


def test_adam_first_step_closed_form(O):
    rng = np.random.default_rng(6)
    g = rng.normal(size=1000) * np.logspace(-12, 2, 1000)
    p = np.zeros(1000); p0 = p.copy()   # from 0: the step is read off exactly
    m = np.zeros(1000); v = np.zeros(1000)
    O.adam(p, g, m, v, 1, lr=5e-3)
    # bias-corrected first step: m_hat = g, v_hat = g^2
    np.testing.assert_allclose(p0 - p, 5e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-20)


def test_adam_constant_gradient(O):
    g = np.array([3.0, -0.02, 1e-9, 0.0])
    p = np.zeros(4); m = np.zeros(4); v = np.zeros(4)
    for t in range(1, 11):
        O.adam(p, g.copy(), m, v, t, lr=1e-2)
    # with a constant gradient every bias-corrected step is lr g / (|g| + eps)
    np.testing.assert_allclose(p, -10 * 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-18)


def test_adam_alternating_gradient(O):
    b1, b2, lr, eps = 0.9, 0.999, 1e-2, 1e-8
    p = np.zeros(1); m = np.zeros(1); v = np.zeros(1)
    O.adam(p, np.array([1.0]), m, v, 1, lr)
    O.adam(p, np.array([-1.0]), m, v, 2, lr)
    # after +1, -1: m_hat = -(1 - b1)/(1 + b1), v_hat = 1
    mh = -(1 - b1) / (1 + b1)
    assert p[0] == pytest.approx(-lr * 1 / (1 + eps) - lr * mh / (1 + eps), rel=1e-12)


def test_condition_scale_dominates_contributions(O):
    # the propagated condition scale of every gradient entry is at least the
    # sum of |contributions| (each seed and propagation step bounds |value|)
    net = _tiny(O)
    rng = np.random.default_rng(11)
    params = rng.normal(scale=0.6, size=net.n_params)
    pos, dirs, rad, pdf = _tiny_batch(rng, 64)
    out = O.backward(net, pos, dirs, rad, pdf, params)
    cond = O.backward_cond(net, pos, dirs, rad, pdf, params)
    assert np.all(cond >= out["gabs"] * (1 - 1e-12))
    assert np.all((cond > 0) == (out["gabs"] > 0))


def test_ema_closed_forms(O):
    """Moving average of the weights (Sec. 5.3): with the parameters held at p
    after every step, ema_t = p + d^t (ema_0 - p); d = 0 follows the
    parameters; a ramp p_t = t gives the weighted sum in closed form."""
    rng = np.random.default_rng(4)
    e0, p = rng.normal(size=64), rng.normal(size=64)
    e = e0.copy()
    for t in range(1, 11):
        O.ema(e, p, 0.9)
        np.testing.assert_allclose(e, p + 0.9 ** t * (e0 - p), rtol=1e-13, atol=1e-14)
    e = e0.copy()
    O.ema(e, p, 0.0)
    assert np.array_equal(e, p)
    d, T = 0.75, 12
    e = np.zeros(3)
    for t in range(1, T + 1):
        O.ema(e, np.full(3, float(t)), d)
    ref = sum((1 - d) * d ** (T - t) * t for t in range(1, T + 1))
    np.testing.assert_allclose(e, ref, rtol=1e-13)


@pytest.mark.parametrize("with_abs", [False, True])
def test_parallel_backward_equals_serial(O, with_abs):
    """The backward and its condition scales on several threads (contiguous
    vertex ranges, per-thread sums added in thread order) equal the serial
    loop up to the order of FP64 additions."""
    net = W.TINY
    on = O.Net(net.n_levels, net.feat, net.base_res, net.max_res, net.log2_table,
               net.dense_only, net.n_hidden, net.width, net.n_lobes)
    rng = np.random.default_rng(17)
    params = rng.normal(0, 0.3, on.n_params)
    b = W.make_batch("cube", 4000, seed=17)
    old = O.set_threads(1)
    try:
        s = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, params, with_abs=with_abs)
        sc = O.backward_cond(on, b.pos, b.dir, b.radiance, b.pdf, params)
        O.set_threads(4)
        assert O.backward_threads(on, b.n, with_abs) == 4
        p = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, params, with_abs=with_abs)
        pc = O.backward_cond(on, b.pos, b.dir, b.radiance, b.pdf, params)
    finally:
        O.set_threads(old)
    scale = s["gabs"] if with_abs else np.abs(s["grad"]).max()
    np.testing.assert_allclose(p["grad"], s["grad"], rtol=0, atol=1e-12 * np.max(scale))
    if with_abs:
        np.testing.assert_allclose(p["gabs"], s["gabs"], rtol=1e-12)
    np.testing.assert_allclose(pc, sc, rtol=1e-12)
    assert p["loss"] == pytest.approx(s["loss"], rel=1e-13)
