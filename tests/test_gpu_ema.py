"""Moving average of the weights for inference (Sec. 5.3), through the C ABI.

* After every optimizer step the average follows ema <- d ema + (1 - d) p,
  checked against the oracle's recursion from the GPU's previous average and
  new parameters.
* npm_query evaluates the averaged weights: its outputs equal, bit for bit,
  those of a context without an average whose parameters are set to the
  average (same kernels, same weights, same uniforms), and they match the
  FP64 oracle evaluated at the average.
* Setting the parameters restarts the average there.
"""
import numpy as np
import pytest

import parity as P
from paper_2504_04315_amd import npm as B
from paper_2504_04315_amd import workload as W
from test_gpu_parity import check_query, dev, oracle_net

pytestmark = pytest.mark.gpu

DECAY = 0.9


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


CASES = [("staged", W.CFG1, "fp32"), ("fused", W.CFG1, "fp32"), ("fused", W.CFG3, "bf16")]


@pytest.mark.parametrize("mode,net,prec", CASES, ids=[f"{m}-{p}" for m, _, p in CASES])
def test_average_follows_the_steps_and_drives_the_query(O, torch, mode, net, prec):
    ex = B.EXEC_FUSED if mode == "fused" else B.EXEC_STAGED
    model = B.NPM(B.make_config(net, exec_mode=ex, precision=prec, ema_decay=DECAY))
    e = model.get_state(B.STATE_EMA).astype(np.float64)
    assert np.array_equal(e, model.get_state().astype(np.float64))   # starts at the init
    kind = "cube" if net is W.CFG1 else "surface"
    d32 = float(np.float32(DECAY))
    for t in range(1, 4):
        b = W.make_batch(kind, 4096 + 7 * t, seed=300 + t)
        model.train_step(*(dev(torch, a) for a in (b.pos, b.dir, b.radiance, b.pdf)))
        torch.cuda.synchronize()
        p = model.get_state().astype(np.float64)
        e_gpu = model.get_state(B.STATE_EMA).astype(np.float64)
        O.ema(e, p, d32)
        # one FP32 multiply-add per entry on each side
        bound = 2 * 2.0 ** -23 * (np.abs(e) + np.abs(p)) + 1e-30
        print(P.assert_within(f"average after step {t}", e_gpu, e, bound))
        e = e_gpu
    # the query reads the average: a context without one, holding it as params
    twin = B.NPM(B.make_config(net, exec_mode=ex, precision=prec))
    twin.set_state(e.astype(np.float32))
    q = W.make_batch(kind, 3000, seed=77)
    a = model.query(dev(torch, q.pos), dev(torch, q.dir), seed=5, stream_id=2)
    b = twin.query(dev(torch, q.pos), dev(torch, q.dir), seed=5, stream_id=2)
    torch.cuda.synchronize()
    for k in ("lobes", "pdf", "sample_dir", "sample_pdf"):
        assert torch.equal(a[k], b[k]), k
    if prec == "fp32":
        on = oracle_net(O, net)
        msgs, _ = check_query(O, torch, model, on, e, q, seed=5, sid=2)
        print("\n".join(msgs))
    model.close()
    twin.close()


def test_training_uses_the_current_weights(O, torch):
    """The gradient is taken at the trained parameters, not at the average."""
    model = B.NPM(B.make_config(W.TINY, exec_mode=B.EXEC_FUSED, ema_decay=0.5))
    on = oracle_net(O, W.TINY)
    b = W.make_batch("cube", 2048, seed=8)
    args = [dev(torch, x) for x in (b.pos, b.dir, b.radiance, b.pdf)]
    for _ in range(2):
        model.train_step(*args)
    torch.cuda.synchronize()
    p = model.get_state().astype(np.float64)
    assert not np.array_equal(p, model.get_state(B.STATE_EMA).astype(np.float64))
    g = torch.zeros(on.n_params, device="cuda")
    model.backward(*args, grad=g)
    torch.cuda.synchronize()
    ref = O.backward(on, b.pos, b.dir, b.radiance, b.pdf, p)
    cond = O.backward_cond(on, b.pos, b.dir, b.radiance, b.pdf, p)
    print(P.check_grads("gradient at the trained weights", g.cpu().numpy().astype(np.float64),
                        ref["grad"], cond))
    model.close()


def test_setting_parameters_restarts_the_average(torch):
    model = B.NPM(B.make_config(W.TINY, exec_mode=B.EXEC_STAGED, ema_decay=0.9))
    p = np.random.default_rng(1).normal(size=model.n_params).astype(np.float32)
    model.set_state(p)
    assert np.array_equal(model.get_state(B.STATE_EMA), p)
    plain = B.NPM(B.make_config(W.TINY, exec_mode=B.EXEC_STAGED))
    with pytest.raises(B.NPMError):
        plain.get_state(B.STATE_EMA)
    model.close()
    plain.close()
