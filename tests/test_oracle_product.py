"""Pins of the oracle's NPM-product inputs (Sec. 4.3, Full Integrand
Learning): the spherical-harmonics encoding of the outgoing direction and of
the surface normal, and the network that takes them after G(x).

The basis is pinned by what defines it, not by its formulas: orthonormality
on the sphere (quadrature), the addition theorem per band, parity, the
azimuthal order and phase of each function (a Fourier analysis over phi),
and the sign convention (no Condon-Shortley phase: every function is
positive near the pole on its leading azimuth).
"""
import math

import numpy as np
import pytest

DEG = 4


def _sphere_quadrature(nz=24, nphi=48):
    x, w = np.polynomial.legendre.leggauss(nz)
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    Z, PH = np.meshgrid(x, phi, indexing="ij")
    R = np.sqrt(1 - Z * Z)
    v = np.stack([R * np.cos(PH), R * np.sin(PH), Z], -1).reshape(-1, 3)
    wt = np.outer(w, np.full(nphi, 2 * math.pi / nphi)).reshape(-1)
    return v, wt


def test_sh_orthonormal(O):
    v, wt = _sphere_quadrature()
    Y, _ = O.sh(DEG, v)
    gram = (Y * wt[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(DEG * DEG), atol=1e-12)


def test_sh_addition_theorem_and_parity(O):
    rng = np.random.default_rng(1)
    v = rng.normal(size=(200, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    Y, _ = O.sh(DEG, v)
    Yn, _ = O.sh(DEG, -v)
    for l in range(DEG):
        band = slice(l * l, (l + 1) * (l + 1))
        np.testing.assert_allclose((Y[:, band] ** 2).sum(1), (2 * l + 1) / (4 * math.pi),
                                   rtol=1e-12)
        np.testing.assert_allclose(Yn[:, band], (-1) ** l * Y[:, band], atol=1e-14)


@pytest.mark.parametrize("theta", [0.3, 1.1, 2.2])
def test_sh_azimuthal_order_and_phase(O, theta):
    """Y_lm(theta, phi) = a(theta) cos(m phi) for m > 0, a(theta) sin(|m| phi)
    for m < 0, constant in phi for m = 0; at theta = 0.3 every a > 0."""
    N = 64
    phi = 2 * math.pi * np.arange(N) / N
    v = np.stack([math.sin(theta) * np.cos(phi), math.sin(theta) * np.sin(phi),
                  np.full(N, math.cos(theta))], 1)
    Y, _ = O.sh(DEG, v)
    for l in range(DEG):
        for m in range(-l, l + 1):
            c = np.fft.rfft(Y[:, l * l + l + m]) / N
            k = abs(m)
            coef = c[k].real * (1 if k == 0 else 2) if m >= 0 else -2 * c[k].imag
            other = np.delete(np.abs(c), k)
            assert other.max() < 1e-12 * max(1.0, abs(coef)), (l, m)
            if m >= 0:
                assert abs(c[k].imag) < 1e-12
            else:
                assert abs(c[k].real) < 1e-12
            if theta == 0.3:
                assert coef > 0, (l, m, coef)


def test_sh_condition_scale_bounds_the_value(O):
    rng = np.random.default_rng(2)
    v = rng.normal(size=(50, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    Y, S = O.sh(DEG, v)
    assert np.all(S >= np.abs(Y) - 1e-15)
    assert np.all(S[:, 0] == Y[:, 0])


def _product_net(O):
    # 2-level hash grid (T = 2^8), F = 2, SH degree 2: 4 + 9 inputs, MLP 13-8-8-32
    return O.Net(2, 2, 4, 16, 8, False, 2, 8, sh_degree=2)


def _aux(rng, n):
    wo = rng.normal(size=(n, 3)); wo /= np.linalg.norm(wo, axis=1, keepdims=True)
    nn = rng.normal(size=(n, 3)); nn /= np.linalg.norm(nn, axis=1, keepdims=True)
    return np.concatenate([wo.T, nn.T, rng.random((1, n))]).astype(np.float32)


def test_product_inputs_follow_the_grid_features(O):
    net = _product_net(O)
    plain = O.Net(2, 2, 4, 16, 8, False, 2, 8)
    assert net.n_in == 4 + 2 * 4 + 1 == plain.n_in + 9
    assert net.grid_params == plain.grid_params
    assert net.n_params == plain.n_params + 8 * 9
    rng = np.random.default_rng(3)
    n = 20
    pos = rng.random((3, n)).astype(np.float32)
    aux = _aux(rng, n)
    params = rng.normal(size=net.n_params)
    G = O.encode(net, pos, params, aux=aux)
    Gp = O.encode(plain, pos, params[:plain.n_params])
    np.testing.assert_array_equal(G[:, :4], Gp)
    np.testing.assert_array_equal(G[:, 4:8], O.sh(2, aux[0:3].T.astype(np.float64))[0])
    np.testing.assert_array_equal(G[:, 8:12], O.sh(2, aux[3:6].T.astype(np.float64))[0])
    np.testing.assert_array_equal(G[:, 12], aux[6].astype(np.float64))
    with pytest.raises(AssertionError):
        O.encode(net, pos, params)


def test_product_backward_vs_finite_differences(O):
    """Every parameter of the product network, including the first layer's
    columns of the extra inputs, against central differences of the loss."""
    net = _product_net(O)
    rng = np.random.default_rng(4)
    params = rng.normal(scale=0.6, size=net.n_params)
    n = 48
    pos = rng.random((3, n)).astype(np.float32)
    aux = _aux(rng, n)
    d = rng.normal(size=(n, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    dirs = d.T.astype(np.float32)
    rad = rng.exponential(size=n).astype(np.float32)
    pdf = np.full(n, 1 / (4 * math.pi), dtype=np.float32)
    out = O.backward(net, pos, dirs, rad, pdf, params, aux=aux)
    g = out["grad"]
    h = 1e-6
    fd = np.zeros(net.n_params)
    for j in np.nonzero(out["gabs"])[0]:
        p = params.copy(); p[j] += h
        lp = O.backward(net, pos, dirs, rad, pdf, p, with_abs=False, aux=aux)["loss"]
        p[j] -= 2 * h
        lm = O.backward(net, pos, dirs, rad, pdf, p, with_abs=False, aux=aux)["loss"]
        fd[j] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=0, atol=2e-7 * np.abs(g).max())
    w0 = net.layer_offset[0]
    aux_cols = np.array([w0 + o * net.n_in + k for o in range(8) for k in range(4, 13)])
    assert np.abs(g[aux_cols]).max() > 0
    q = O.query(net, pos, params, dirs=dirs, aux=aux)
    w = rad.astype(np.float64) / pdf.astype(np.float64)
    assert out["loss"] == pytest.approx(-np.mean(w * q["logpdf"]), rel=1e-12)
