"""GPU parity of the learned BSDF-selection probability (the network's extra
output; the Sec. 6.3 extension) against the FP64 oracle, through the C ABI,
on the staged and the fused path.

- Query: the raw outputs (4K + 1 rows) to their forward condition scale; the
  selection probability c = sigmoid(c') to the raw tolerance carried through
  the sigmoid; the mixture outputs of npm_query_select identical to
  npm_query's on the same network.
- Backward: every gradient entry within 1e-5 of the oracle's condition scale
  (which covers the selection term; its size is pinned on the CPU), the
  mixture's loss and the selection loss; BSDF densities from the
  diffuse/glossy mix (zeros below a diffuse surface included).
- Train step: backward + Adam over three steps, from identical states.
- The plain calls on a selection network train the mixture only: the
  selection row's gradient is exactly 0.
- Edge cases: invalid densities (inf, NaN, negative) have no selection term;
  -0.0 and denormals are valid; n = 0; calls on a network without the
  output fail with NPM_ERR_STATE.
- Sizes: the tiny net at a ragged 997, cfg1 at 16,384 + 17 (several tiles
  and a ragged tail), and the paper's network at its training batch, 2^18,
  whole (fused: in spatial order); a spatially ordered fused query (staged
  slots and the un-permute carry c).
- The fused static backward (no allocation) on a selection network trains
  the mixture only.
- Precision form (fused BF16): the gradient's cosine with the oracle's
  > 0.99 for the grid, the MLP and the selection row; c within 1e-2.
"""
import math

import numpy as np
import pytest

import parity as P
from paper_2504_04315_amd import npm as B
from paper_2504_04315_amd import workload as W

pytestmark = pytest.mark.gpu
K = 8
MODES = {"staged": B.EXEC_STAGED, "fused": B.EXEC_FUSED}


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a device"
    return T


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def oracle_net(O, net):
    return O.Net(net.n_levels, net.feat, net.base_res, net.max_res, net.log2_table,
                 net.dense_only, net.n_hidden, net.width, net.n_lobes, select=net.select)


def randomize(model, on, rng, grid_sd=1.0, mlp_gain=2.0):
    p = np.zeros(on.n_params, dtype=np.float32)
    p[:on.grid_params] = rng.normal(0, grid_sd, on.grid_params)
    for i, (o, k) in enumerate(on.layer_shape):
        a = mlp_gain * math.sqrt(6.0 / (o + k)) / math.sqrt(k / 8.0)
        off = on.layer_offset[i]
        p[off:off + o * k] = rng.uniform(-a, a, o * k)
    model.set_state(p)
    return p.astype(np.float64)


def selection_row(on):
    width = on.layer_shape[-1][1]
    off = on.layer_offset[-1] + 4 * K * width
    return slice(off, off + width)


def check_query_select(O, torch, model, on, params, b, n, tag):
    pos, dirs = dev(torch, b.pos), dev(torch, b.dir)
    out = model.query_select(pos, dirs, seed=4, stream_id=2)
    plain = model.query(pos, dirs, seed=4, stream_id=2)
    raw = model.forward_raw(pos).cpu().numpy().T
    torch.cuda.synchronize()
    for k in ("lobes", "pdf", "sample_dir", "sample_pdf"):
        assert torch.equal(out[k], plain[k]), k
    q = O.query(on, b.pos, params, dirs=b.dir, seed=4, stream=2)
    rr, rs = O.mlp_forward(on, q["G"], params, with_scale=True)
    assert raw.shape == (n, 4 * K + 1)
    msgs = [P.check_scaled(f"{tag} raw (with the selection logit)", raw, rr, rs)]
    c = q["sel"]
    bound = P.RTOL * (c + c * (1 - c) * rs[:, 4 * K]) + 1e-30
    msgs.append(P.assert_within(f"{tag} selection probability", out["select_prob"].cpu().numpy(),
                                c, bound))
    assert 0.05 < np.median(c) < 0.95 and c.std() > 0.01    # a spread of probabilities
    return msgs


@pytest.mark.parametrize("mode", ["staged", "fused"])
@pytest.mark.parametrize("net,n", [(W.TINYS, 997), (W.CFG1S, 16384 + 17)])
def test_query_select_parity(O, torch, net, n, mode):
    model = B.NPM(B.make_config(net, exec_mode=MODES[mode]))
    on = oracle_net(O, net)
    params = randomize(model, on, np.random.default_rng(21), grid_sd=0.5)
    b = W.make_batch("surface", n, seed=22)
    print("\n".join(check_query_select(O, torch, model, on, params, b, n, mode)))
    model.close()


def test_query_select_spatial_order(O, torch):
    """A fused query in spatial order: c goes through the staged slots and the
    un-permute like the other outputs."""
    net = W.PAPERS
    model = B.NPM(B.make_config(net, exec_mode=B.EXEC_FUSED, batch_order=B.ORDER_SPATIAL))
    on = oracle_net(O, net)
    params = randomize(model, on, np.random.default_rng(31), grid_sd=0.5)
    n = 40001
    b = W.make_batch("surface", n, seed=32)
    print("\n".join(check_query_select(O, torch, model, on, params, b, n, "ordered")))
    model.close()


def check_backward_select(O, torch, model, on, params, batch, bsdf, tag):
    pos, dirs = dev(torch, batch.pos), dev(torch, batch.dir)
    rad, pdf = dev(torch, batch.radiance), dev(torch, batch.pdf)
    loss = torch.zeros(2, dtype=torch.float64, device="cuda")
    grad = torch.zeros(on.n_params, dtype=torch.float32, device="cuda")
    model.backward_select(pos, dirs, rad, pdf, dev(torch, bsdf), grad=grad, loss=loss)
    torch.cuda.synchronize()
    ref = O.backward(on, batch.pos, batch.dir, batch.radiance, batch.pdf, params, bsdf=bsdf)
    cond = O.backward_cond(on, batch.pos, batch.dir, batch.radiance, batch.pdf, params,
                           bsdf=bsdf)
    g = grad.cpu().numpy().astype(np.float64)
    gp, row = on.grid_params, selection_row(on)
    msgs = [P.check_grads(f"{tag} grad(grid)", g[:gp], ref["grad"][:gp], cond[:gp]),
            P.check_grads(f"{tag} grad(mlp)", g[gp:], ref["grad"][gp:], cond[gp:]),
            P.check_grads(f"{tag} grad(selection row)", g[row], ref["grad"][row], cond[row])]
    assert np.count_nonzero(ref["grad"][row]) == on.layer_shape[-1][1]
    lv = loss.cpu().numpy()
    for got, want, name in ((lv[0], ref["loss"], "loss"), (lv[1], ref["loss_sel"], "loss_sel")):
        assert abs(got - want) <= 1e-5 * max(1.0, abs(want)), (name, got, want)
        msgs.append(f"{tag} {name} {got:.9g} vs oracle {want:.9g}")
    return msgs, g, ref


@pytest.mark.parametrize("mode", ["staged", "fused"])
@pytest.mark.parametrize("net,n", [(W.TINYS, 997), (W.CFG1S, 16384 + 17)])
def test_backward_select_parity(O, torch, net, n, mode):
    model = B.NPM(B.make_config(net, exec_mode=MODES[mode]))
    on = oracle_net(O, net)
    params = randomize(model, on, np.random.default_rng(23), grid_sd=0.5)
    batch = W.make_batch("surface", n, seed=24)
    bsdf = W.make_bsdf(batch, 24)
    assert np.mean(bsdf == 0) > 0.05                # zero densities are part of the case
    msgs, _, _ = check_backward_select(O, torch, model, on, params, batch, bsdf,
                                       f"{mode} {net_name(net)}")
    print("\n".join(msgs))
    model.close()


def net_name(net):
    return {W.TINYS: "tiny", W.CFG1S: "cfg1", W.PAPERS: "paper"}[net]


@pytest.mark.parametrize("mode", ["staged", "fused"])
def test_backward_select_paper_training_batch(O, torch, mode):
    """The paper's network with the selection output at its training batch
    (2^18 vertices, surface samples), the launch configuration the benchmark
    times (fused: spatially ordered): every gradient entry and both losses."""
    model = B.NPM(B.make_config(W.PAPERS, exec_mode=MODES[mode]))
    on = oracle_net(O, W.PAPERS)
    params = randomize(model, on, np.random.default_rng(25), grid_sd=0.5)
    batch = W.make_batch("surface", W.N_PAPER_TRAIN, seed=26)
    bsdf = W.make_bsdf(batch, 26)
    msgs, _, _ = check_backward_select(O, torch, model, on, params, batch, bsdf,
                                       f"{mode} paper 2^18")
    print("\n".join(msgs))
    model.close()


@pytest.mark.parametrize("mode", ["staged", "fused"])
def test_train_step_select_against_oracle(O, torch, mode):
    """npm_train_step_select = backward (both terms) + Adam, over three steps,
    each from the GPU's own state; the bound adds the Adam update's spread
    when the gradient moves within its parity tolerance."""
    net = W.TINYS
    model = B.NPM(B.make_config(net, exec_mode=MODES[mode]))
    on = oracle_net(O, net)
    f = lambda x: float(np.float32(x))
    hp = dict(lr=f(net.lr), beta1=f(net.beta1), beta2=f(net.beta2), eps=f(net.eps))
    for t in range(1, 4):
        p0 = model.get_state().astype(np.float64)
        m0 = model.get_state(B.STATE_ADAM_M).astype(np.float64)
        v0 = model.get_state(B.STATE_ADAM_V).astype(np.float64)
        batch = W.make_batch("cube", 997, seed=200 + t)
        bsdf = W.make_bsdf(batch, 200 + t)
        stats = torch.zeros(3, dtype=torch.float64, device="cuda")
        model.train_step_select(dev(torch, batch.pos), dev(torch, batch.dir),
                                dev(torch, batch.radiance), dev(torch, batch.pdf),
                                dev(torch, bsdf), stats=stats)
        torch.cuda.synchronize()
        ref = O.backward(on, batch.pos, batch.dir, batch.radiance, batch.pdf, p0, bsdf=bsdf)
        cond = O.backward_cond(on, batch.pos, batch.dir, batch.radiance, batch.pdf, p0,
                               bsdf=bsdf)
        outs = []
        for dg in (0.0, 1e-5, -1e-5):
            p, m, v = p0.copy(), m0.copy(), v0.copy()
            O.adam(p, ref["grad"] + dg * cond, m, v, t, **hp)
            outs.append(p)
        st = stats.cpu().numpy()
        assert st[0] == pytest.approx(ref["loss"], rel=1e-5)
        assert st[1] == pytest.approx(ref["loss_sel"], rel=1e-5)
        assert st[2] == pytest.approx(float(np.sum(ref["grad"] ** 2)), rel=1e-4)
        p_gpu = model.get_state().astype(np.float64)
        bound = 1e-5 * np.abs(outs[0]) + np.abs(outs[1] - outs[2]) + 1e-9 * hp["lr"]
        print(P.assert_within(f"{mode} selection train step {t} params", p_gpu, outs[0], bound))
        assert model.step == t
    model.close()


@pytest.mark.parametrize("mode", ["staged", "fused"])
def test_plain_calls_train_the_mixture_only(O, torch, mode):
    net = W.TINYS
    model = B.NPM(B.make_config(net, exec_mode=MODES[mode]))
    on = oracle_net(O, net)
    params = randomize(model, on, np.random.default_rng(27), grid_sd=0.5)
    b = W.make_batch("cube", 777, seed=28)
    grad = torch.zeros(on.n_params, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    model.backward(dev(torch, b.pos), dev(torch, b.dir), dev(torch, b.radiance),
                   dev(torch, b.pdf), grad=grad, loss=loss)
    torch.cuda.synchronize()
    ref = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, params)
    cond = O.backward_cond(on, b.pos, b.dir, b.radiance, b.pdf, params)
    g = grad.cpu().numpy().astype(np.float64)
    print(P.check_grads(f"{mode} mixture-only grad", g, ref["grad"], cond))
    assert np.all(g[selection_row(on)] == 0.0)
    assert float(loss.cpu()[0]) == pytest.approx(ref["loss"], rel=1e-5)
    if mode == "fused":
        # the static entry point (no allocation) after a selection call: the
        # block partials of the selection row are rewritten, not left over
        model.backward_select(dev(torch, b.pos), dev(torch, b.dir), dev(torch, b.radiance),
                              dev(torch, b.pdf), dev(torch, W.make_bsdf(b, 28)),
                              grad=torch.zeros_like(grad))
        g2 = torch.zeros_like(grad)
        model.backward_static(dev(torch, b.pos), dev(torch, b.dir), dev(torch, b.radiance),
                              dev(torch, b.pdf), grad=g2)
        torch.cuda.synchronize()
        g2 = g2.cpu().numpy().astype(np.float64)
        print(P.check_grads("static mixture-only grad", g2, ref["grad"], cond))
        assert np.all(g2[selection_row(on)] == 0.0)
    model.close()


@pytest.mark.parametrize("mode", ["staged", "fused"])
def test_select_edge_cases(O, torch, mode):
    net = W.TINYS
    model = B.NPM(B.make_config(net, exec_mode=MODES[mode]))
    on = oracle_net(O, net)
    params = randomize(model, on, np.random.default_rng(29), grid_sd=0.5)
    b = W.make_batch("cube", 64, seed=30)
    bsdf = W.make_bsdf(b, 30)
    bsdf[:8] = [np.inf, np.nan, -1.0, -np.inf, -0.0, 0.0, 1e-40, 3e38]
    msgs, _, _ = check_backward_select(O, torch, model, on, params, b, bsdf,
                                       f"{mode} edge densities")
    print("\n".join(msgs))
    # n = 0 is a no-op
    empty = torch.zeros((3, 0), device="cuda")
    e1 = torch.zeros(0, device="cuda")
    model.backward_select(empty, empty, e1, e1, e1)
    model.query_select(empty, empty)
    # bsdf_pdf is required
    with pytest.raises(B.NPMError) as ei:
        model.backward_select(dev(torch, b.pos), dev(torch, b.dir), dev(torch, b.radiance),
                              dev(torch, b.pdf), None)
    assert ei.value.status == -1
    model.close()
    # a network without the output refuses the calls
    plain = B.NPM(B.make_config(W.TINY))
    with pytest.raises(B.NPMError) as ei:
        plain.query_select(dev(torch, b.pos))
    assert ei.value.status == -6
    with pytest.raises(B.NPMError) as ei:
        plain.train_step_select(dev(torch, b.pos), dev(torch, b.dir), dev(torch, b.radiance),
                                dev(torch, b.pdf), dev(torch, bsdf))
    assert ei.value.status == -6
    plain.close()


def test_select_precision_form(O, torch):
    """The fused precision form (BF16 MLP, FP16 grid) with the selection
    output, at the paper's training batch: gradient cosine with the oracle's
    (grid, MLP, selection row) > 0.99, both losses within 1e-2 relative, and
    the selection probability of a query within 1e-2."""
    net = W.PAPERS
    model = B.NPM(B.make_config(net, exec_mode=B.EXEC_FUSED, precision="bf16"))
    on = oracle_net(O, net)
    params = model.get_state().astype(np.float64)
    batch = W.make_batch("surface", W.N_PAPER_TRAIN, seed=33)
    bsdf = W.make_bsdf(batch, 33)
    loss = torch.zeros(2, dtype=torch.float64, device="cuda")
    grad = torch.zeros(on.n_params, dtype=torch.float32, device="cuda")
    model.backward_select(dev(torch, batch.pos), dev(torch, batch.dir), dev(torch, batch.radiance),
                          dev(torch, batch.pdf), dev(torch, bsdf), grad=grad, loss=loss)
    q = model.query_select(dev(torch, batch.pos[:, :4096]), None, lobes=False, sample=False)
    torch.cuda.synchronize()
    ref = O.backward(on, batch.pos, batch.dir, batch.radiance, batch.pdf, params, bsdf=bsdf,
                     with_abs=False)
    g = grad.cpu().numpy().astype(np.float64)
    gp, row = on.grid_params, selection_row(on)
    for name, sl in (("grid", slice(0, gp)), ("mlp", slice(gp, None)), ("selection row", row)):
        a, r = g[sl], ref["grad"][sl]
        cs = float(a @ r / (np.linalg.norm(a) * np.linalg.norm(r)))
        print(f"bf16 selection gradient cosine ({name}): {cs:.6f}")
        assert cs > 0.99, (name, cs)
    lv = loss.cpu().numpy()
    for got, want, name in ((lv[0], ref["loss"], "loss"), (lv[1], ref["loss_sel"], "loss_sel")):
        print(f"bf16 {name} {got:.7f} vs oracle {want:.7f}")
        assert abs(got - want) <= 1e-2 * abs(want), name
    c = O.query(on, batch.pos[:, :4096], params)["sel"]
    err = np.abs(q["select_prob"].cpu().numpy() - c)
    print(f"bf16 selection probability: max abs err {err.max():.2e}")
    assert err.max() <= 1e-2
    model.close()
