"""Serving form on the GPU: many sessions resident, requests batched into
persistent multi-session kernels.

* A query gives the same result (bit for bit) alone and in a mix of other
  sessions' requests, and the same as the session's own fused path.
* A training batch gives the same parameters alone and in the mix, within
  the parity tolerance (the order of atomic adds differs).
* Admission respects the HBM budget; every request completes exactly once.
* The per-session plain path agrees with the FP64 oracle.
"""
import numpy as np
import pytest

from paper_2504_04315_amd import npm as B
from paper_2504_04315_amd import serve as S
from paper_2504_04315_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()




def small_cfg(seed):
    from dataclasses import replace
    return B.make_config(replace(W.CFG5, log2_table=14, seed=seed))


def test_query_alone_equals_mix(torch):
    srv_a = S.Server(budget_bytes=4 << 30, max_sessions=8)
    srv_m = S.Server(budget_bytes=4 << 30, max_sessions=8)
    a = srv_a.create_session(small_cfg(11))
    m_sids = [srv_m.create_session(small_cfg(11 + i)) for i in range(4)]
    b = W.make_batch("surface", 3000, seed=1)
    pos, dirs = dev(torch, b.pos), dev(torch, b.dir)

    def outs(n):
        return dict(lobes=torch.empty((4, 8, n), device="cuda"), pdf=torch.empty(n, device="cuda"),
                    sdir=torch.empty((3, n), device="cuda"), spdf=torch.empty(n, device="cuda"))
    alone = outs(b.n)
    r = srv_a.submit_query(a, pos, dirs, seed=3, stream_id=1, **alone)
    srv_a.wait(r)
    # the same request in a mix with three other sessions' queries and trains
    mix = outs(b.n)
    others = []
    for i, sid in enumerate(m_sids[1:]):
        ob = W.make_batch("surface", 5000 + 977 * i, seed=10 + i)
        others.append(srv_m.submit_train(sid, dev(torch, ob.pos), dev(torch, ob.dir),
                                         dev(torch, ob.radiance), dev(torch, ob.pdf)))
        o = outs(ob.n)
        others.append(srv_m.submit_query(sid, dev(torch, ob.pos), dev(torch, ob.dir), **o))
    r2 = srv_m.submit_query(m_sids[0], pos, dirs, seed=3, stream_id=1, **mix)
    srv_m.drain()
    for k in alone:
        assert torch.equal(alone[k], mix[k]), k
    # and equal to the session's own fused path (same kernel code per tile)
    model = B.NPM(small_cfg(11))
    own = model.query(pos, dirs, seed=3, stream_id=1)
    torch.cuda.synchronize()
    assert torch.equal(own["pdf"], alone["pdf"]) and torch.equal(own["sample_dir"], alone["sdir"])
    model.close()
    srv_a.close()
    srv_m.close()


def test_train_alone_equals_mix(torch):
    cfg = small_cfg(21)
    n_params = B.layout_of(cfg).n_params
    srv_a = S.Server(budget_bytes=4 << 30, max_sessions=8)
    srv_m = S.Server(budget_bytes=4 << 30, max_sessions=8)
    a = srv_a.create_session(cfg)
    m = [srv_m.create_session(cfg)] + [srv_m.create_session(small_cfg(30 + i)) for i in range(3)]
    b = W.make_batch("surface", 20000, seed=5)
    pos, dirs, rad, pdf = dev(torch, b.pos), dev(torch, b.dir), dev(torch, b.radiance), dev(torch, b.pdf)
    st_a = torch.zeros(2, dtype=torch.float64, device="cuda")
    st_m = torch.zeros(2, dtype=torch.float64, device="cuda")
    srv_a.wait(srv_a.submit_train(a, pos, dirs, rad, pdf, stats=st_a))
    for i, sid in enumerate(m[1:]):
        ob = W.make_batch("surface", 7000 + 1000 * i, seed=40 + i)
        srv_m.submit_train(sid, dev(torch, ob.pos), dev(torch, ob.dir), dev(torch, ob.radiance),
                           dev(torch, ob.pdf))
    srv_m.submit_train(m[0], pos, dirs, rad, pdf, stats=st_m)
    srv_m.drain()
    pa = S.session_ctx_state(srv_a, a, n_params)
    pm = S.session_ctx_state(srv_m, m[0], n_params)
    ma = S.session_ctx_state(srv_a, a, n_params, B.STATE_ADAM_M)
    mm = S.session_ctx_state(srv_m, m[0], n_params, B.STATE_ADAM_M)
    # one step from the same state: the gradients differ only by the order of
    # FP32 atomic adds, so the first moments (0.1 g) agree to rounding ...
    scale = float(np.abs(ma).max())
    np.testing.assert_allclose(mm, ma, rtol=1e-5, atol=1e-6 * scale)
    # ... and the parameters agree except where a gradient within rounding of
    # zero flips the sign of the Adam step (at most 2 lr, rare)
    lr = float(np.float32(W.CFG5.lr))
    bad = np.abs(pm - pa) > 1e-5 * np.abs(pa) + 1e-7
    assert bad.mean() < 1e-3 and np.abs(pm - pa).max() <= 2.01 * lr
    assert abs(float(st_a[0]) - float(st_m[0])) <= 1e-6 * abs(float(st_a[0]))
    srv_a.close()
    srv_m.close()


def test_budget_admission(torch):
    cfg = small_cfg(1)
    per = B.layout_of(cfg).device_bytes
    srv = S.Server(budget_bytes=int(per * 2.5), max_sessions=8)
    s1 = srv.create_session(cfg)
    s2 = srv.create_session(small_cfg(2))
    with pytest.raises(B.NPMError) as e:
        srv.create_session(small_cfg(3))
    assert e.value.status == -4
    srv.destroy_session(s1)
    s3 = srv.create_session(small_cfg(3))       # fits again once memory is freed
    assert srv.stats().sessions == 2
    srv.close()


def test_every_request_completes_once(torch):
    srv = S.Server(budget_bytes=8 << 30, max_sessions=8, round_vertices=1 << 14)
    sids = [srv.create_session(small_cfg(50 + i)) for i in range(4)]
    plan = S.plan_requests(4, 6, rate_hz=2000.0, min_log2=10, max_log2=14, train_every=3, seed=1)
    S.make_request_buffers(plan, n_pools=2, pool_size=1 << 15)
    res = S.run_load(srv, sids, plan)
    st = srv.stats()
    assert st.requests_done == len(plan)
    assert st.vertices_done == sum(r["n"] for r in plan)
    assert res["latency_ms"]["p99"] >= res["latency_ms"]["p50"] > 0
    for r in plan:
        if r["kind"] == 0:
            p = r["pdf"].cpu().numpy()
            assert np.all(np.isfinite(p)) and np.all(p > 0)
    srv.close()


def test_sessions_with_a_moving_average(torch):
    """A session that keeps a moving average (ema_decay > 0) answers queries
    with it in the shared kernels, as its own context does."""
    srv = S.Server(budget_bytes=4 << 30, max_sessions=2)
    cfg = small_cfg(21)
    cfg.ema_decay = 0.9
    sid = srv.create_session(cfg)
    tb = W.make_batch("surface", 4096, seed=22)
    targs = [dev(torch, a) for a in (tb.pos, tb.dir, tb.radiance, tb.pdf)]
    for _ in range(2):
        srv.wait(srv.submit_train(sid, *targs))
    b = W.make_batch("surface", 3000, seed=23)
    pos, dirs = dev(torch, b.pos), dev(torch, b.dir)
    o = dict(lobes=torch.empty((4, 8, b.n), device="cuda"), pdf=torch.empty(b.n, device="cuda"),
             sdir=torch.empty((3, b.n), device="cuda"), spdf=torch.empty(b.n, device="cuda"))
    srv.wait(srv.submit_query(sid, pos, dirs, seed=4, **o))
    # the session's average, evaluated by a context holding it as parameters
    twin = B.NPM(small_cfg(21))
    avg = srv.session_state(sid, twin.n_params, B.STATE_EMA)
    assert not np.array_equal(avg, srv.session_state(sid, twin.n_params, B.STATE_PARAMS))
    twin.set_state(avg)
    ref = twin.query(pos, dirs, seed=4)
    torch.cuda.synchronize()
    assert torch.equal(o["pdf"], ref["pdf"]) and torch.equal(o["sdir"], ref["sample_dir"])
    twin.close()
    srv.close()


def test_product_sessions_are_refused(torch):
    srv = S.Server(budget_bytes=4 << 30, max_sessions=2)
    with pytest.raises(B.NPMError):
        srv.create_session(B.make_config(W.TINYP, exec_mode=B.EXEC_FUSED))
    srv.close()
