"""NPM-product (Sec. 4.3, Full Integrand Learning) on the GPU, through the C
ABI's *_aux calls, against the FP64 oracle.

The MLP input is G(x), then the spherical harmonics of the outgoing
direction and of the normal, then the roughness.  Checked at the production
shape (16-level hash grid, 4 SH bands: 65 inputs in a 96-wide first layer)
and on the 2-level finite-difference net (2 bands, 13 inputs): every stage,
the query, the gradient (staged, fused in the caller's order and in spatial
order), a full train step, order-invariance of the query, and the precision
form's pdf error.  Same tolerance policy as the radiance-based network
(tests/parity.py).
"""
import numpy as np
import pytest

import parity as P
from paper_2504_04315_amd import npm as B
from paper_2504_04315_amd import workload as W
from test_gpu_parity import (adam_hp, check_backward, check_query, check_stages, dev, oracle_net,
                             randomize)

pytestmark = pytest.mark.gpu

MODES = {"staged": (B.EXEC_STAGED, B.ORDER_AUTO, B.SCATTER_AUTO),
         "fused": (B.EXEC_FUSED, B.ORDER_NONE, B.SCATTER_ATOMIC),
         "fused-spatial": (B.EXEC_FUSED, B.ORDER_SPATIAL, B.SCATTER_ATOMIC),
         # every hashed level through the binned pass (the 2-level net's one
         # hashed level is a single bin)
         "fused-binned": (B.EXEC_FUSED, B.ORDER_NONE, B.SCATTER_BINNED)}


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


def model_of(net, mode, **kw):
    ex, order, scatter = MODES[mode]
    return B.NPM(B.make_config(net, exec_mode=ex, batch_order=order, scatter_mode=scatter, **kw))


@pytest.mark.parametrize("mode", ["staged", "fused", "fused-spatial", "fused-binned"])
@pytest.mark.parametrize("name,n", [("TINYP", 3001), ("CFG2P", 8192 + 45)])
def test_product_stages_query_and_gradient(O, torch, mode, name, n):
    net = getattr(W, name)
    model = model_of(net, mode)
    on = oracle_net(O, net)
    rng = np.random.default_rng(21)
    params = randomize(model, on, rng, grid_sd=0.5)
    kind = "cube" if name == "TINYP" else "surface"
    batch = W.make_batch(kind, n, seed=31)
    aux = W.make_aux(batch, 31)
    msgs = check_stages(O, torch, model, on, params, batch.pos, aux=aux)
    m2, _ = check_query(O, torch, model, on, params, batch, aux=aux)
    tb = W.make_batch(kind, n // 2 + 7, seed=32)
    m3, g, ref = check_backward(O, torch, model, on, params, tb, f"{name} {mode}",
                                aux=W.make_aux(tb, 32))
    # the first layer's columns of the extra inputs receive gradient
    w0 = on.layer_offset[0]
    gf = net.n_levels * net.feat
    cols = np.array([w0 + o * on.n_in + k for o in range(net.width) for k in range(gf, on.n_in)])
    assert np.abs(ref["grad"][cols]).max() > 0
    print("\n".join(msgs + m2 + m3))
    model.close()


@pytest.mark.parametrize("mode", ["staged", "fused", "fused-binned"])
def test_product_train_step(O, torch, mode):
    """npm_train_step_aux = backward + Adam, one step from the GPU's state,
    within the Adam spread of the gradient's tolerance."""
    net = W.TINYP
    model = model_of(net, mode)
    on = oracle_net(O, net)
    hp = adam_hp(net)
    p0 = model.get_state().astype(np.float64)
    b = W.make_batch("cube", 997, seed=41)
    aux = W.make_aux(b, 41)
    stats = torch.zeros(2, dtype=torch.float64, device="cuda")
    model.train_step(dev(torch, b.pos), dev(torch, b.dir), dev(torch, b.radiance),
                     dev(torch, b.pdf), stats=stats, aux=dev(torch, aux))
    torch.cuda.synchronize()
    ref = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, p0, aux=aux)
    cond = O.backward_cond(on, b.pos, b.dir, b.radiance, b.pdf, p0, aux=aux)
    outs = []
    for dg in (0.0, 1e-5, -1e-5):
        p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
        O.adam(p, ref["grad"] + dg * cond, m, v, 1, **hp)
        outs.append(p)
    assert float(stats[0]) == pytest.approx(ref["loss"], rel=1e-5)
    bound = 1e-5 * np.abs(outs[0]) + np.abs(outs[1] - outs[2]) + 1e-9 * hp["lr"]
    print(P.assert_within("product train step", model.get_state().astype(np.float64), outs[0],
                          bound))
    model.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_product_query_order_is_invisible(torch, prec):
    net = W.CFG2P
    a = B.NPM(B.make_config(net, exec_mode=B.EXEC_FUSED, precision=prec,
                            batch_order=B.ORDER_NONE))
    b = B.NPM(B.make_config(net, exec_mode=B.EXEC_FUSED, precision=prec,
                            batch_order=B.ORDER_SPATIAL))
    batch = W.make_batch("surface", 40001, seed=51)
    aux = dev(torch, W.make_aux(batch, 51))
    pos, d = dev(torch, batch.pos), dev(torch, batch.dir)
    qa = a.query(pos, d, seed=2, aux=aux)
    qb = b.query(pos, d, seed=2, aux=aux)
    torch.cuda.synchronize()
    for k, v in qa.items():
        assert torch.equal(v, qb[k]), k
    a.close()
    b.close()


def test_product_precision_form(O, torch):
    """BF16 MLP + FP16 grid on the product network: pdf relative error
    against the FP64 oracle at the same parameters (target p99 <= 1e-2)."""
    net = W.CFG2P
    model = B.NPM(B.make_config(net, exec_mode=B.EXEC_FUSED, precision="bf16"))
    on = oracle_net(O, net)
    params = randomize(model, on, np.random.default_rng(61), grid_sd=0.5)
    batch = W.make_batch("surface", 1 << 16, seed=62)
    aux = W.make_aux(batch, 62)
    out = model.query(dev(torch, batch.pos), dev(torch, batch.dir), seed=1,
                      aux=dev(torch, aux))
    torch.cuda.synchronize()
    m = 4096
    sub = batch.subset(np.arange(m))
    q = O.query(on, sub.pos, params, dirs=sub.dir, aux=aux[:, :m])
    rel = np.abs(out["pdf"].cpu().numpy()[:m].astype(np.float64) / np.exp(q["logpdf"]) - 1)
    print(f"product BF16 pdf rel err: median {np.median(rel):.3e}, p99 "
          f"{np.percentile(rel, 99):.3e}, max {rel.max():.3e}")
    assert np.percentile(rel, 99) <= 1e-2
    model.close()


def test_product_calls_need_the_extra_inputs(torch):
    model = model_of(W.TINYP, "fused")
    b = W.make_batch("cube", 64, seed=1)
    with pytest.raises(B.NPMError):
        model.query(dev(torch, b.pos), dev(torch, b.dir))
    plain = model_of(W.TINY, "fused")
    with pytest.raises(B.NPMError):
        plain.query(dev(torch, b.pos), dev(torch, b.dir), aux=dev(torch, W.make_aux(b, 1)))
    model.close()
    plain.close()


def test_product_autograd_matches_finite_differences(O, torch):
    """The differentiation form on the product network: the autograd
    gradient equals the oracle's and central differences of the FP64 loss
    (first-layer columns of the extra inputs included)."""
    from paper_2504_04315_amd.autograd import NPM
    net = W.TINYP
    mod = NPM(B.make_config(net, exec_mode=B.EXEC_FUSED))
    on = oracle_net(O, net)
    params = mod.model.get_state().astype(np.float64)
    b = W.make_batch("cube", 2003, seed=71)
    aux = W.make_aux(b, 71)
    loss = mod(*(dev(torch, a) for a in (b.pos, b.dir, b.radiance, b.pdf)), aux=dev(torch, aux))
    loss.backward()
    g = mod.params.grad.detach().cpu().numpy().astype(np.float64)
    ref = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, params, aux=aux)
    cond = O.backward_cond(on, b.pos, b.dir, b.radiance, b.pdf, params, aux=aux)
    print(P.check_grads("product autograd vs oracle", g, ref["grad"], cond))
    assert float(loss.item()) == pytest.approx(ref["loss"], rel=1e-5)
    w0 = on.layer_offset[0]
    pick = [w0 + o * on.n_in + k for o in range(0, net.width, 3) for k in range(4, on.n_in)]
    for j in pick:
        def f(h):
            p = params.copy(); p[j] += h
            a = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, p, with_abs=False, aux=aux)["loss"]
            p[j] -= 2 * h
            c = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, p, with_abs=False, aux=aux)["loss"]
            return (a - c) / (2 * h)
        f1, f2 = f(1e-6), f(5e-7)
        fd_err = abs(f1 - f2) * 4.0 / 3.0 + 1e-16 * abs(ref["loss"]) / 5e-7
        assert abs(g[j] - f2) <= 1e-5 * cond[j] + fd_err + 1e-12, (j, g[j], f2)
    mod.model.close()
