"""Pins of the oracle's mixture sampler (Sec. 5.3, Jakob 2012) and uniforms.

Closed forms: for one vMF lobe the cosine t = mu.w has density proportional
to e^{kappa t} on [-1, 1], so E[t] = coth(kappa) - 1/kappa, and the azimuth
about mu is uniform.  For the mixture, sample histograms must match the bin
integrals of the pdf (chi-square).
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

from test_oracle_vmf import lobe_raw, mu_of

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers(O):
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        assert O.philox(w[0:4], w[4:6]).tolist() == w[6:10]


def test_uniforms_range_and_independence(O):
    u = O.uniforms(200000, seed=123, stream=4)
    assert u.min() >= 0.0 and u.max() < 1.0
    # 24-bit grid: every value is an exact multiple of 2^-24
    assert np.all(u * 2**24 == np.floor(u * 2**24))
    for j in range(3):
        assert stats.kstest(u[:, j], "uniform").pvalue > 1e-3
    assert abs(np.corrcoef(u[:, 0], u[:, 1])[0, 1]) < 0.01
    # different stream, seed or vertex number gives different draws
    assert not np.array_equal(u[:10], O.uniforms(10, seed=123, stream=5))
    assert not np.array_equal(u[:10], O.uniforms(10, seed=124, stream=4))
    vid = np.arange(10) + 7
    np.testing.assert_array_equal(O.uniforms(10, 123, 4, vid=vid), u[7:17])


@pytest.fixture(scope="module")
def net1(O):
    return O.Net(1, 1, 1, 1, 8, True, 1, 1, n_lobes=1)


@pytest.fixture(scope="module")
def net8(O):
    return O.Net(1, 1, 1, 1, 8, True, 1, 1, n_lobes=8)


@pytest.mark.parametrize("kappa", [1e-6, 0.3, 2.0, 25.0, 400.0])
def test_single_lobe_mean_cosine(O, net1, kappa):
    n = 200000
    th, ph = 0.35, 0.8
    raw = np.broadcast_to(np.array(lobe_raw(th, ph, kappa)), (n, 4))
    u = O.uniforms(n, seed=9, stream=1)
    d, _ = O.sample_raw(net1, raw, u)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    t = d @ mu_of(th, ph)
    expect = 1.0 / math.tanh(kappa) - 1.0 / kappa if kappa > 1e-3 else kappa / 3.0
    se = t.std() / math.sqrt(n)
    assert abs(t.mean() - expect) < 5 * se + 1e-12, (t.mean(), expect)
    # the cosine marginal: CDF of t is (e^{kappa(t+1)} - 1) / (e^{2 kappa} - 1)
    if kappa < 50:
        cdf = lambda x: np.expm1(kappa * (np.asarray(x) + 1)) / math.expm1(2 * kappa)
        assert stats.kstest(t, cdf).pvalue > 1e-3


def test_single_lobe_azimuth_uniform(O, net1):
    n = 100000
    th, ph = 0.6, 0.1
    raw = np.broadcast_to(np.array(lobe_raw(th, ph, 5.0)), (n, 4))
    d, _ = O.sample_raw(net1, raw, O.uniforms(n, seed=10, stream=0))
    mu = mu_of(th, ph)
    a = np.array([1.0, 0.0, 0.0]); t1 = np.cross(mu, a); t1 /= np.linalg.norm(t1)
    t2 = np.cross(mu, t1)
    az = np.arctan2(d @ t2, d @ t1)
    assert stats.kstest((az + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3


def test_mixture_chi_square(O, net8):
    rng = np.random.default_rng(11)
    raw = rng.normal(size=32)
    raw[2::4] = rng.uniform(0.0, math.log(40.0), 8)
    n = 400000
    d, lobe = O.sample_raw(net8, np.broadcast_to(raw, (n, 32)), O.uniforms(n, seed=12, stream=0))
    lam = O.head(net8, raw[None, :])[0, :, 3]
    # lobe frequencies follow lambda
    cnt = np.bincount(lobe, minlength=8)
    assert stats.chisquare(cnt, lam * n).pvalue > 1e-3
    # direction histogram over (cos theta, phi) bins vs quadrature of the pdf
    nz, nphi = 12, 24
    zb = np.linspace(-1, 1, nz + 1)
    pb = np.linspace(-math.pi, math.pi, nphi + 1)
    H, _, _ = np.histogram2d(d[:, 2], np.arctan2(d[:, 1], d[:, 0]), bins=[zb, pb])
    x, wx = np.polynomial.legendre.leggauss(24)
    E = np.zeros((nz, nphi))
    for i in range(nz):
        z = 0.5 * (zb[i + 1] - zb[i]) * (x + 1) + zb[i]
        wz = 0.5 * (zb[i + 1] - zb[i]) * wx
        for j in range(nphi):
            p = 0.5 * (pb[j + 1] - pb[j]) * (x + 1) + pb[j]
            wp = 0.5 * (pb[j + 1] - pb[j]) * wx
            Z, P = np.meshgrid(z, p, indexing="ij")
            R = np.sqrt(1 - Z * Z)
            dd = np.stack([R * np.cos(P), R * np.sin(P), Z], -1).reshape(-1, 3)
            lp = O.logpdf(net8, np.broadcast_to(raw, (dd.shape[0], 32)), dd)
            E[i, j] = np.sum(np.exp(lp) * np.outer(wz, wp).reshape(-1))
    assert abs(E.sum() - 1.0) < 1e-3
    E *= n
    keep = E > 5
    Hk, Ek = H[keep], E[keep]
    Ek *= Hk.sum() / Ek.sum()
    chi = float(((Hk - Ek) ** 2 / Ek).sum())
    dof = keep.sum() - 1
    assert stats.chi2.sf(chi, dof) > 1e-3, (chi, dof)


def test_sample_pdf_matches_logpdf(O):
    # npmo_query's sample log-pdf is the full mixture log-density at the sample
    net = O.Net(2, 2, 2, 4, 8, True, 1, 8)
    rng = np.random.default_rng(13)
    params = rng.normal(scale=0.5, size=net.n_params)
    pos = rng.random((3, 50)).astype(np.float32)
    q = O.query(net, pos, params, seed=5, stream=2)
    np.testing.assert_allclose(q["slogpdf"], O.logpdf(net, q["raw"], q["sdir"]), rtol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(q["sdir"], axis=1), 1.0, atol=1e-12)


def test_sample_cosine_bounded_for_huge_kappa(O, net1):
    # At u1 = 0 the inverse CDF of the cosine is exactly -1 (the antipode of
    # mu); the log1p/expm1 form underflows there for large kappa.
    th, ph = 0.45, 0.3
    raw = np.array([lobe_raw(th, ph, math.exp(80.0))])
    d, _ = O.sample_raw(net1, raw, np.array([[0.5, 0.0, 0.25]]))
    np.testing.assert_allclose(d[0], -mu_of(th, ph), atol=1e-12)
    d, _ = O.sample_raw(net1, raw, np.array([[0.5, 0.5, 0.25]]))
    np.testing.assert_allclose(d[0], mu_of(th, ph), atol=1e-12)
