"""Pins of the oracle's vMF density, Table 1 mappings and mixture pdf.

Preliminary, "Von Mises-Fisher Mixtures": v(w|mu,kappa) = kappa/(4 pi sinh
kappa) exp(kappa mu.w); the mixture is a convex combination, so it integrates
to 1 over the sphere.  Table 1: kappa = exp(kappa'), lambda = softmax(lambda'),
theta, phi = logistic.
"""
import math

import mpmath
import numpy as np
import pytest


def lobe_raw(theta, phi, kappa, logit=0.0):
    """Raw outputs (theta', phi', kappa', lambda') that map to the given values."""
    return [math.log(theta / (1 - theta)), math.log(phi / (1 - phi)), math.log(kappa), logit]


def mu_of(theta, phi):
    T, P = math.pi * theta, 2 * math.pi * phi
    return np.array([math.sin(T) * math.cos(P), math.sin(T) * math.sin(P), math.cos(T)])


@pytest.fixture(scope="module")
def net1(O):
    return O.Net(1, 1, 1, 1, 8, True, 1, 1, n_lobes=1)


@pytest.fixture(scope="module")
def net8(O):
    return O.Net(1, 1, 1, 1, 8, True, 1, 1, n_lobes=8)


@pytest.mark.parametrize("kappa", [1e-8, 1e-4, 0.1, 1.0, 10.0, 100.0, 1e3, 1e4])
def test_single_lobe_normaliser_vs_mpmath(O, net1, kappa):
    th, ph = 0.3, 0.7
    raw = np.array([lobe_raw(th, ph, kappa)])
    mu = mu_of(th, ph)
    mpmath.mp.dps = 50
    k = mpmath.mpf(kappa)
    for sign in (+1.0, -1.0):
        want = mpmath.log(k / (4 * mpmath.pi * mpmath.sinh(k))) + sign * k
        got = O.logpdf(net1, raw, (sign * mu)[None, :])[0]
        assert abs(got - float(want)) <= 1e-12 * max(1.0, abs(float(want))), (kappa, sign)


def test_isotropic_limit(O, net8):
    rng = np.random.default_rng(3)
    raw = rng.normal(size=(5, 32))
    raw[:, 2::4] = -80.0                     # kappa = e^-80: uniform lobes
    d = rng.normal(size=(5, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    lp = O.logpdf(net8, raw, d)
    np.testing.assert_allclose(lp, -math.log(4 * math.pi), rtol=0, atol=1e-13)


def test_mapping_ranges_and_values(O, net8):
    rng = np.random.default_rng(4)
    raw = rng.normal(scale=3.0, size=(200, 32))
    lob = O.head(net8, raw)
    th, ph, ka, la = lob[..., 0], lob[..., 1], lob[..., 2], lob[..., 3]
    assert np.all((th > 0) & (th < 1) & (ph > 0) & (ph < 1) & (ka > 0) & (la > 0))
    np.testing.assert_allclose(la.sum(axis=1), 1.0, atol=1e-14)
    # logistic and exponential, spot values
    np.testing.assert_allclose(th, 1 / (1 + np.exp(-raw[:, 0::4])), rtol=1e-14)
    np.testing.assert_allclose(ka, np.exp(raw[:, 2::4]), rtol=1e-14)
    # softmax is invariant to a common shift of the logits
    raw2 = raw.copy()
    raw2[:, 3::4] += 7.5
    np.testing.assert_allclose(O.head(net8, raw2)[..., 3], la, rtol=1e-12)


def _sphere_quadrature(nz=256, nphi=512):
    z, wz = np.polynomial.legendre.leggauss(nz)
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    Z, P = np.meshgrid(z, phi, indexing="ij")
    R = np.sqrt(1 - Z * Z)
    d = np.stack([R * np.cos(P), R * np.sin(P), Z], axis=-1).reshape(-1, 3)
    w = (wz[:, None] * np.full((1, nphi), 2 * math.pi / nphi)).reshape(-1)
    return d, w


def test_mixture_integrates_to_one(O, net8):
    d, w = _sphere_quadrature()
    rng = np.random.default_rng(5)
    for trial in range(4):
        raw = rng.normal(size=32)
        raw[2::4] = rng.uniform(-3, math.log(30.0), 8)
        lp = O.logpdf(net8, np.broadcast_to(raw, (d.shape[0], 32)), d)
        integral = float(np.sum(np.exp(lp) * w))
        assert abs(integral - 1.0) < 1e-9, (trial, integral)


def test_sharp_lobe_integrates_to_one_in_its_frame(O, net1):
    # kappa = 1e4: integrate with the pole on mu, cosines clustered near 1.
    th, ph, kappa = 0.4, 0.15, 1e4
    raw = np.array(lobe_raw(th, ph, kappa))
    mu = mu_of(th, ph)
    a = np.array([0.0, 0.0, 1.0])
    t1 = np.cross(a, mu); t1 /= np.linalg.norm(t1); t2 = np.cross(mu, t1)
    x, wx = np.polynomial.legendre.leggauss(200)
    # cos = 1 - s, s in [0, 0.01] carries all but e^-100 of the mass
    s = 0.005 * (x + 1); ws = 0.005 * wx
    nphi = 64
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    c = 1 - s
    r = np.sqrt(1 - c * c)
    d = (c[:, None, None] * mu + r[:, None, None] * (np.cos(phi)[None, :, None] * t1
                                                   + np.sin(phi)[None, :, None] * t2)).reshape(-1, 3)
    wq = (ws[:, None] * np.full((1, nphi), 2 * math.pi / nphi)).reshape(-1)
    lp = O.logpdf(net1, np.broadcast_to(raw, (d.shape[0], 4)), d)
    assert abs(float(np.sum(np.exp(lp) * wq)) - 1.0) < 1e-9


def test_pdf_at_axis_closed_form(O, net1):
    # at w = mu a single lobe equals kappa / (2 pi (1 - e^{-2 kappa}))
    for kappa in (0.5, 3.0, 40.0):
        raw = np.array([lobe_raw(0.6, 0.2, kappa)])
        got = math.exp(O.logpdf(net1, raw, mu_of(0.6, 0.2)[None, :])[0])
        assert got == pytest.approx(kappa / (2 * math.pi * (1 - math.exp(-2 * kappa))), rel=1e-13)


def test_mixture_is_weighted_sum_of_lobes(O, net1, net8):
    rng = np.random.default_rng(6)
    raw = rng.normal(size=32)
    d = rng.normal(size=(10, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    lam = O.head(net8, raw[None, :])[0, :, 3]
    mix = np.exp(O.logpdf(net8, np.broadcast_to(raw, (10, 32)), d))
    parts = np.zeros(10)
    for k in range(8):
        r1 = raw[4 * k:4 * k + 4].copy()
        parts += lam[k] * np.exp(O.logpdf(net1, np.broadcast_to(r1, (10, 4)), d))
    np.testing.assert_allclose(mix, parts, rtol=1e-12)
