"""Size of the gradient condition scale (the parity tolerance's unit), pinned
against an independent FP32 evaluation of the backward (CPU).

The gradient tolerance is 1e-5 * cond, cond being the oracle's first-order
bound on an FP32 evaluation's error in units of the unit roundoff
(npmo_backward_cond).  A bound can fail two ways: too small (an honest FP32
evaluation falls outside it) or too large (the tolerance hides real errors).
This test runs a plain FP32 transcription of the backward written here in
numpy -- float32 corner weights and interpolation, float32 MLP, head and
delta chain, float32 scatter -- and compares it with the FP64 oracle:

* every entry's error is within 1e-5 * cond (the bar can be met);
* the largest errors reach a stated fraction of 2^-24 * cond, so cond is at
  most that factor above what FP32 rounding actually does: 1/25 with the
  networks' initial-scale parameters, 1/250 with spread parameters (kappa
  over several e-folds, wide weights), where cancellation through three
  64-wide layers and sums over ~100 vertices per grid entry keep the
  first-order worst case above the errors' random walk.

The same holds with the learned selection output (one more row of the last
layer, its head derivative in the t = log p_bsdf - log V form an FP32
implementation takes), for the whole gradient and for that row alone.

Before the head's condition factor was derived as a sum of independent
first-order sources (it multiplied them), the spread case reached only
1/2,500 of the bound.
"""
import math

import numpy as np
import pytest

from paper_2504_04315_amd import workload as W

f32 = np.float32
U = 2.0 ** -24


def oracle_net(O, net):
    return O.Net(net.n_levels, net.feat, net.base_res, net.max_res, net.log2_table,
                 net.dense_only, net.n_hidden, net.width, net.n_lobes)


def corner_entries(on, pos):
    """Global table entry [n][L][8] and float32 trilinear weight of every corner."""
    n = pos.shape[1]
    L = on.n_levels
    idx = np.zeros((n, L, 8), np.int64)
    wts = np.zeros((n, L, 8), f32)
    T = None
    for l in range(L):
        D = on.res[l]
        c, fr = [], []
        for a in range(3):
            x = np.clip(pos[a].astype(f32), f32(0), f32(1))
            p = (x * f32(D)).astype(f32)
            ci = np.minimum(np.floor(p), f32(D - 1)).astype(f32)
            c.append(ci.astype(np.int64))
            fr.append((p - ci).astype(f32))
        if on.hashed[l]:
            T = on.level_size[l]
        for b in range(8):
            X, Y, Z = c[0] + (b & 1), c[1] + ((b >> 1) & 1), c[2] + ((b >> 2) & 1)
            if on.hashed[l]:
                h = (X.astype(np.uint64) ^ (Y.astype(np.uint64) * np.uint64(2654435761))
                     ^ (Z.astype(np.uint64) * np.uint64(805459861))) & np.uint64(0xFFFFFFFF)
                e = (h % np.uint64(T)).astype(np.int64)
            else:
                e = X + (D + 1) * (Y + (D + 1) * Z)
            idx[:, l, b] = on.level_offset[l] + e
            w = ((fr[0] if b & 1 else f32(1) - fr[0]) * (fr[1] if b & 2 else f32(1) - fr[1]))
            wts[:, l, b] = (w.astype(f32) * (fr[2] if b & 4 else f32(1) - fr[2])).astype(f32)
    return idx, wts


def fp32_backward(on, pos, dirs, rad, spdf, params, bsdf=None):
    """The gradient of the surrogate loss, every step in float32 (with the
    selection output's term when the network has one and bsdf is given)."""
    n = pos.shape[1]
    P = params.astype(f32)
    L, F, K = on.n_levels, on.feat, on.n_lobes
    idx, wts = corner_entries(on, pos)
    table = P[:on.grid_params].reshape(-1, F)
    G = np.zeros((n, L * F), f32)
    for l in range(L):
        for b in range(8):
            G[:, l * F:(l + 1) * F] += (wts[:, l, b, None] * table[idx[:, l, b]]).astype(f32)
    acts, h = [G], G
    nl = len(on.layer_shape)
    for i in range(nl):
        z = (h @ on.weights(P, i).T).astype(f32)
        if i < nl - 1:
            z = np.maximum(z, f32(0))
            acts.append(z)
        h = z
    r4 = h[:, :4 * K].reshape(n, K, 4)
    th = f32(1) / (f32(1) + np.exp(-r4[..., 0]))
    ph = f32(1) / (f32(1) + np.exp(-r4[..., 1]))
    kap = np.exp(np.clip(r4[..., 2], f32(-80), f32(80))).astype(f32)
    mx = r4[..., 3].max(axis=1, keepdims=True)
    loglam = (r4[..., 3] - (mx + np.log(np.exp(r4[..., 3] - mx).sum(1, keepdims=True)))).astype(f32)
    T_, P_ = (f32(np.pi) * th).astype(f32), (f32(2 * np.pi) * ph).astype(f32)
    sT, cT, sP, cP = np.sin(T_), np.cos(T_), np.sin(P_), np.cos(P_)
    mu = np.stack([sT * cP, sT * sP, cT], -1).astype(f32)
    t1 = np.stack([cT * cP, cT * sP, -sT], -1).astype(f32)
    t2 = np.stack([-sP, cP, np.zeros_like(sP)], -1).astype(f32)
    w3 = dirs.T.astype(f32)[:, None, :]
    d = (mu * w3).sum(-1).astype(f32)
    with np.errstate(over="ignore"):
        lnorm = (np.log(kap / (-np.expm1(f32(-2) * kap))) - f32(math.log(2 * math.pi))).astype(f32)
        lt = (loglam + lnorm + kap * (d - f32(1))).astype(f32)
        m = lt.max(axis=1, keepdims=True)
        lv = (m + np.log(np.exp(lt - m).sum(axis=1, keepdims=True))).astype(f32)
        r = np.exp(lt - lv).astype(f32)
        lam = np.exp(loglam).astype(f32)
        ok = np.isfinite(rad) & np.isfinite(spdf) & (spdf > 0) & (rad > 0)
        wgt = np.where(ok, rad.astype(f32) / np.where(ok, spdf, 1).astype(f32), 0).astype(f32)
        g = (-wgt / f32(n)).astype(f32)[:, None]
        dt1 = (t1 * w3).sum(-1).astype(f32)
        dt2 = (t2 * w3).sum(-1).astype(f32)
        th1 = f32(1) / (f32(1) + np.exp(r4[..., 0]))
        ph1 = f32(1) / (f32(1) + np.exp(r4[..., 1]))
        dth = kap * dt1 * f32(np.pi) * th * th1
        dph = kap * sT * dt2 * f32(2 * np.pi) * ph * ph1
        dka = f32(1) - f32(2) * kap / np.expm1(f32(2) * kap) + kap * (d - f32(1))
    delta = np.stack([g * r * dth, g * r * dph, g * r * dka, g * (r - lam)],
                     -1).reshape(n, 4 * K).astype(f32)
    if on.select:
        dsel = np.zeros((n, 1), f32)
        if bsdf is not None:
            with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
                cp = h[:, 4 * K]
                c = f32(1) / (f32(1) + np.exp(-cp))
                c1 = f32(1) / (f32(1) + np.exp(cp))
                b32 = bsdf.astype(f32)
                t = (np.log(b32) - lv[:, 0]).astype(f32)
                x = np.expm1(np.minimum(t, f32(0)))
                y = -np.expm1(-np.maximum(t, f32(0)))
                E = np.where(t <= 0, x / (f32(1) + c * x), y / (np.exp(-t) + c * y)).astype(f32)
                use = ok & np.isfinite(b32) & (b32 >= 0)
                dsel[:, 0] = np.where(use, (g[:, 0] * c * c1 * E).astype(f32), f32(0))
        delta = np.concatenate([delta, dsel], 1)
    grad = np.zeros(on.n_params, f32)
    for i in range(nl - 1, -1, -1):
        if i < nl - 1:
            delta = np.where(acts[i + 1] > 0, delta, f32(0)).astype(f32)
        o, k = on.layer_shape[i]
        off = on.layer_offset[i]
        grad[off:off + o * k] = (delta.T @ acts[i]).astype(f32).ravel()
        delta = (delta @ on.weights(P, i)).astype(f32)
    gg = np.zeros(on.grid_params, f32)
    for l in range(L):
        for b in range(8):
            for f in range(F):
                np.add.at(gg, idx[:, l, b] * F + f, (wts[:, l, b] * delta[:, l * F + f]).astype(f32))
    grad[:on.grid_params] = gg
    return grad


def spread_params(on, rng, grid_sd=1.0, mlp_gain=2.0):
    p = np.zeros(on.n_params)
    p[:on.grid_params] = rng.normal(0, grid_sd, on.grid_params)
    for i, (o, k) in enumerate(on.layer_shape):
        a = mlp_gain * math.sqrt(6.0 / (o + k)) / math.sqrt(k / 8.0)
        off = on.layer_offset[i]
        p[off:off + o * k] = rng.uniform(-a, a, o * k)
    return p.astype(f32).astype(np.float64)


def init_params(on, rng):
    """Initial scale: grid N(0, 0.01^2), Xavier-uniform weights."""
    p = np.zeros(on.n_params)
    p[:on.grid_params] = rng.normal(0, 0.01, on.grid_params)
    for i, (o, k) in enumerate(on.layer_shape):
        a = math.sqrt(6.0 / (o + k))
        off = on.layer_offset[i]
        p[off:off + o * k] = rng.uniform(-a, a, o * k)
    return p.astype(f32).astype(np.float64)


FLOOR = {"init": 1.0 / 25.0, "spread": 1.0 / 250.0}


@pytest.mark.parametrize("kind", ["init", "spread"])
@pytest.mark.parametrize("case", ["tiny", "cfg1"])
def test_condition_scale_is_sized_to_fp32_error(O, case, kind):
    net, n = (W.TINY, 4000) if case == "tiny" else (W.CFG1, 16384)
    on = oracle_net(O, net)
    rng = np.random.default_rng(3)
    p = init_params(on, rng) if kind == "init" else spread_params(on, rng)
    b = W.make_batch("cube", n, seed=5)
    ref = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, p)
    cond = O.backward_cond(on, b.pos, b.dir, b.radiance, b.pdf, p)
    g32 = fp32_backward(on, b.pos, b.dir, b.radiance, b.pdf, p).astype(np.float64)
    err = np.abs(g32 - ref["grad"])
    gp = on.grid_params
    for part, sl in (("grid", slice(0, gp)), ("mlp", slice(gp, None))):
        c, e = cond[sl], err[sl]
        assert np.all(e <= 1e-5 * c + 1e-30), part
        nz = c > 0
        ratio = e[nz] / (U * c[nz])
        q = np.quantile(ratio, [0.5, 0.99, 0.999])
        print(f"{case} {kind} {part}: err / (2^-24 cond) median {q[0]:.4f}, p99 {q[1]:.4f}, "
              f"p99.9 {q[2]:.4f}, max {ratio.max():.4f}; max err / (1e-5 cond) "
              f"{(e[nz] / (1e-5 * c[nz])).max():.2e}")
        assert ratio.max() >= FLOOR[kind], (part, ratio.max())


SEL_FLOOR = {"init": 1.0 / 25.0, "spread": 1.0 / 250.0}


@pytest.mark.parametrize("kind", ["init", "spread"])
@pytest.mark.parametrize("case", ["tiny", "cfg1"])
def test_selection_condition_scale(O, case, kind):
    """The same bound with the learned selection output (Sec. 6.3): the
    condition of its head derivative and of the extra row, through the
    network; BSDF densities from the diffuse / glossy mix, zeros included."""
    net, n = (W.TINY, 4000) if case == "tiny" else (W.CFG1, 16384)
    on = O.Net(net.n_levels, net.feat, net.base_res, net.max_res, net.log2_table,
               net.dense_only, net.n_hidden, net.width, net.n_lobes, select=True)
    rng = np.random.default_rng(13)
    p = init_params(on, rng) if kind == "init" else spread_params(on, rng)
    b = W.make_batch("cube", n, seed=15)
    bsdf = W.make_bsdf(b, 15)
    ref = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, p, bsdf=bsdf)
    cond = O.backward_cond(on, b.pos, b.dir, b.radiance, b.pdf, p, bsdf=bsdf)
    g32 = fp32_backward(on, b.pos, b.dir, b.radiance, b.pdf, p, bsdf=bsdf).astype(np.float64)
    err = np.abs(g32 - ref["grad"])
    last = on.layer_offset[-1]
    width = on.layer_shape[-1][1]
    row = slice(last + 4 * on.n_lobes * width, last + (4 * on.n_lobes + 1) * width)
    for part, sl in (("all", slice(0, on.n_params)), ("selection row", row)):
        c, e = cond[sl], err[sl]
        assert np.all(e <= 1e-5 * c + 1e-30), part
        nz = c > 0
        ratio = e[nz] / (U * c[nz])
        print(f"{case} {kind} {part}: err / (2^-24 cond) median {np.median(ratio):.4f}, "
              f"max {ratio.max():.4f}")
        assert ratio.max() >= SEL_FLOOR[kind], (part, ratio.max())


def test_condition_scale_covers_relu_kinks(O):
    """A hidden pre-activation within 2^-20 of its condition scale has a sign
    FP32 does not determine, and an FP32 evaluation may take either side of
    the ReLU: the backward's condition scale covers both (the unit's
    derivative may move by its whole size).  The case: the paper's network
    with the selection output, 2^18 surface samples, widely spread
    parameters, where vertex 82,506 has a second-layer pre-activation at
    2e-8 of its scale and the FP32 transcription takes the other side; every
    entry of its gradient stays within 1e-5 of the condition scale."""
    net = W.PAPERS
    on = O.Net(net.n_levels, net.feat, net.base_res, net.max_res, net.log2_table,
               net.dense_only, net.n_hidden, net.width, net.n_lobes, select=True)
    rng = np.random.default_rng(25)
    p = np.zeros(on.n_params, dtype=np.float32)
    p[:on.grid_params] = rng.normal(0, 0.5, on.grid_params)
    for i, (o, k) in enumerate(on.layer_shape):
        a = 2.0 * math.sqrt(6.0 / (o + k)) / math.sqrt(k / 8.0)
        off = on.layer_offset[i]
        p[off:off + o * k] = rng.uniform(-a, a, o * k)
    p = p.astype(np.float64)
    b = W.make_batch("surface", W.N_PAPER_TRAIN, seed=26)
    bsdf = W.make_bsdf(b, 26)
    # the kink: FP64 and FP32 disagree on the sign of one pre-activation
    v = 82506
    h64 = O.encode(on, b.pos[:, v:v + 1], p)[0]
    h32 = h64.astype(f32)
    for i in range(2):
        Wm = on.weights(p, i)
        z64, z32 = Wm @ h64, (Wm.astype(f32) @ h32).astype(f32)
        scale = np.abs(Wm) @ np.abs(h64)
        h64, h32 = np.maximum(z64, 0), np.maximum(z32, f32(0))
    j = int(np.argmin(np.abs(z64) / scale))
    assert abs(z64[j]) <= 2.0 ** -20 * scale[j]
    ref = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, p, bsdf=bsdf, with_abs=False)
    cond = O.backward_cond(on, b.pos, b.dir, b.radiance, b.pdf, p, bsdf=bsdf)
    g32 = fp32_backward(on, b.pos, b.dir, b.radiance, b.pdf, p, bsdf=bsdf).astype(np.float64)
    err = np.abs(g32 - ref["grad"])
    assert np.all(err <= 1e-5 * cond + 1e-30)
