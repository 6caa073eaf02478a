"""End-to-end pin of the oracle's training step (Sec. 4.2 and 5.3).

The surrogate loss -(1/N) sum w log V, with samples w ~ uniform and
w = L / p, has expectation equal to the cross-entropy between the normalised
target and V, which is minimised exactly at V = target.  A one-lobe network on
a one-cell grid trained with Adam on a position-independent vMF target must
therefore recover the target's mean direction and concentration, and its loss
must approach the target's differential entropy from above.
"""
import math

import numpy as np


def _vmf_entropy(kappa):
    # H = -E[log v] = -log(kappa / (4 pi sinh kappa)) - kappa (coth kappa - 1/kappa)
    return -math.log(kappa / (4 * math.pi * math.sinh(kappa))) - kappa * (
        1 / math.tanh(kappa) - 1 / kappa)


def test_single_lobe_fit_recovers_target(O):
    net = O.Net(1, 2, 1, 1, 8, True, 1, 16, n_lobes=1)
    rng = np.random.default_rng(0)
    params = np.zeros(net.n_params)
    params[:net.grid_params] = rng.uniform(-0.1, 0.1, net.grid_params)
    for i, (o, k) in enumerate(net.layer_shape):
        a = math.sqrt(6.0 / (o + k))
        off = net.layer_offset[i]
        params[off:off + o * k] = rng.uniform(-a, a, o * k)
    m = np.zeros_like(params); v = np.zeros_like(params)
    th_t, ph_t, ka_t = 0.3, 0.6, 8.0
    T, P = math.pi * th_t, 2 * math.pi * ph_t
    mu_t = np.array([math.sin(T) * math.cos(P), math.sin(T) * math.sin(P), math.cos(T)])
    norm_t = ka_t / (4 * math.pi * math.sinh(ka_t))
    n = 2048
    losses = []
    for t in range(1, 801):
        pos = rng.random((3, n)).astype(np.float32)
        d = rng.normal(size=(n, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
        rad = (norm_t * np.exp(ka_t * (d @ mu_t))).astype(np.float32)
        pdf = np.full(n, 1 / (4 * math.pi), dtype=np.float32)
        out = O.backward(net, pos, d.T.astype(np.float32), rad, pdf, params, with_abs=False)
        losses.append(out["loss"])
        O.adam(params, out["grad"], m, v, t, lr=1e-2)
    pos = rng.random((3, 64)).astype(np.float32)
    lob = O.query(net, pos, params)["lobes"][:, 0, :]
    th, ph, ka = lob[:, 0].mean(), lob[:, 1].mean(), lob[:, 2].mean()
    assert abs(th - th_t) < 0.01 and abs(ph - ph_t) < 0.01, (th, ph)
    assert abs(ka / ka_t - 1) < 0.05, ka
    # the surrogate loss tends to the target entropy (its minimum) from above
    tail = float(np.mean(losses[-100:]))
    H = _vmf_entropy(ka_t)
    assert losses[0] > tail
    assert abs(tail - H) < 0.03 * abs(H) + 0.02, (tail, H)
