"""Host-side checks of the seeded synthetic input generator."""
import math

import numpy as np

from paper_2504_04315_amd import workload as W


def test_batches_are_seeded_and_shaped():
    a = W.make_batch("surface", 5000, seed=3)
    b = W.make_batch("surface", 5000, seed=3)
    c = W.make_batch("surface", 5000, seed=4)
    for x, y in ((a.pos, b.pos), (a.dir, b.dir), (a.radiance, b.radiance), (a.pdf, b.pdf)):
        np.testing.assert_array_equal(x, y)
    assert not np.array_equal(a.pos, c.pos)
    assert a.pos.shape == (3, 5000) and a.pos.dtype == np.float32 and a.pos.flags.c_contiguous
    assert a.dir.shape == (3, 5000) and a.radiance.shape == (5000,) and a.pdf.shape == (5000,)
    np.testing.assert_allclose(np.linalg.norm(a.dir.astype(np.float64), axis=0), 1, atol=1e-6)
    assert a.pos.min() > 0.0 and a.pos.max() < 1.0
    assert np.all(a.pdf > 0) and np.all(a.radiance >= 0)


def test_cube_batch_uniform_pdf():
    b = W.make_batch("cube", 4096, seed=1)
    np.testing.assert_allclose(b.pdf, 1 / (4 * math.pi), rtol=1e-7)


def test_field_density_normalised_and_sampler_consistent():
    rng = np.random.default_rng(0)
    x = rng.random((4, 3))
    z, wz = np.polynomial.legendre.leggauss(200)
    phi = (np.arange(400) + 0.5) * 2 * math.pi / 400
    Z, P = np.meshgrid(z, phi, indexing="ij")
    R = np.sqrt(1 - Z * Z)
    d = np.stack([R * np.cos(P), R * np.sin(P), Z], -1).reshape(-1, 3)
    w = (wz[:, None] * np.full((1, 400), 2 * math.pi / 400)).reshape(-1)
    for i in range(4):
        f = W.field_pdf(np.repeat(x[i:i + 1], d.shape[0], 0), d)
        assert abs(float((f * w).sum()) - 1) < 1e-6
    # sampler: mean direction of field samples matches quadrature of the pdf
    xs = np.repeat(x[:1], 200000, 0)
    s = W.field_sample(rng, xs)
    f = W.field_pdf(np.repeat(x[:1], d.shape[0], 0), d)
    mean_q = (d * (f * w)[:, None]).sum(0)
    assert np.all(np.abs(s.mean(0) - mean_q) < 5e-3)


def test_device_batch_generator_matches_numpy_field():
    """The torch restatement of the field (used for fresh device batches in
    long training runs) equals the numpy definition, and its batches follow
    the same distribution: the mean log field density of the sampled
    directions (minus the field's expected entropy) and the mean weight L/p
    agree with make_batch's within their Monte Carlo error."""
    import torch
    import field_torch as FT
    rng = np.random.default_rng(0)
    x = rng.random((4096, 3))
    w = W.uniform_sphere(rng, 4096)
    for a, b in zip(W.field_params(x, 0.0), FT.field_params(torch, torch.from_numpy(x))):
        np.testing.assert_allclose(b.numpy(), a, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(FT.field_pdf(torch, torch.from_numpy(x), torch.from_numpy(w)).numpy(),
                               W.field_pdf(x, w), rtol=1e-12)
    n = 1 << 16
    gen = FT.SurfaceBatches(torch, seed=3, tris_seed=3, device="cpu")
    pos, d, rad, pdf = (t.numpy().astype(np.float64) for t in gen.next(n))
    ref = W.make_batch("surface", n, seed=3)
    assert np.abs(np.linalg.norm(d, axis=0) - 1).max() < 1e-6
    for got, exp in ((np.log(pdf), np.log(ref.pdf.astype(np.float64))),
                     (rad / pdf, ref.radiance.astype(np.float64) / ref.pdf)):
        se = math.sqrt(got.var() / n + exp.var() / n)
        assert abs(got.mean() - exp.mean()) < 5 * se, (got.mean(), exp.mean(), se)
    assert np.allclose(pos.mean(axis=1), ref.pos.mean(axis=1), atol=0.01)


def test_product_inputs():
    """omega_o is a unit vector cosine-distributed about the unit normal
    (E[cos] = 2/3), on the triangle's side; roughness in [0.05, 1]."""
    b = W.make_batch("surface", 20000, seed=4)
    a = W.make_aux(b, 4).astype(np.float64)
    wo, nrm, r = a[0:3], a[3:6], a[6]
    assert np.abs(np.linalg.norm(wo, axis=0) - 1).max() < 1e-6
    assert np.abs(np.linalg.norm(nrm, axis=0) - 1).max() < 1e-6
    c = np.sum(wo * nrm, axis=0)
    assert c.min() >= -1e-6
    assert abs(c.mean() - 2 / 3) < 5 * math.sqrt((0.5 - 4 / 9) / c.size)
    assert r.min() >= 0.05 and r.max() <= 1.0
    assert np.array_equal(W.make_aux(b, 4), W.make_aux(b, 4))
