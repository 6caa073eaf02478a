"""Device-side generator of fresh training batches from the analytic 8-lobe
field (test infrastructure for long training runs).

It draws from the same distribution as workload.make_batch("surface", ...)
-- positions on the seeded triangle set, directions sampled from the field,
sampling pdf = field pdf, radiance = field pdf * Exp(1) -- with torch's
generator instead of numpy's, so that a 200-step run at 2^20 vertices per
step gets a new batch every step without minutes of host work.  The field's
formulas are restated here in torch; a CPU test checks them against the
numpy definitions.
"""
import math

import numpy as np

from paper_2504_04315_amd import workload as W


def field_params(torch, x, phase=0.0):
    k = torch.arange(W.FIELD_LOBES, device=x.device, dtype=x.dtype)
    a = 2.0 * math.pi * k / W.FIELD_LOBES + phase
    m = torch.as_tensor(W._fibonacci_dirs(W.FIELD_LOBES), device=x.device, dtype=x.dtype)
    pert = torch.stack([torch.sin(2 * math.pi * x[:, None, 0] + a[None, :]),
                        torch.sin(2 * math.pi * x[:, None, 1] + 2 * a[None, :]),
                        torch.sin(2 * math.pi * x[:, None, 2] + 3 * a[None, :])], dim=2)
    mu = m[None] + 0.4 * pert
    mu = mu / torch.linalg.norm(mu, dim=2, keepdim=True)
    kappa = 10.0 * torch.exp(torch.sin(2 * math.pi * (x[:, 0] + 2 * x[:, 1] + 3 * x[:, 2])[:, None]
                                       + a[None, :]))
    idx = torch.arange(W.FIELD_LOBES, device=x.device) % 3
    logits = torch.sin(2 * math.pi * x[:, idx] + a[None, :])
    lam = torch.softmax(logits, dim=1)
    return mu, kappa, lam


def field_pdf(torch, x, w, phase=0.0):
    mu, kappa, lam = field_params(torch, x, phase)
    cosv = (mu * w[:, None, :]).sum(-1)
    dens = kappa / (2 * math.pi * (-torch.expm1(-2 * kappa))) * torch.exp(kappa * (cosv - 1.0))
    return (lam * dens).sum(1)


class SurfaceBatches:
    """Fresh surface batches on the device: next(n) -> (pos, dir, rad, pdf),
    SoA float32 tensors ready for the library."""

    def __init__(self, torch, seed, tris_seed, device="cuda"):
        self.t = torch
        self.dev = device
        tris = W.triangle_soup(np.random.default_rng(1000 + tris_seed))
        e1, e2 = tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]
        area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
        self.tris = torch.as_tensor(tris, device=device, dtype=torch.float64)
        self.area = torch.as_tensor(area / area.sum(), device=device, dtype=torch.float64)
        self.g = torch.Generator(device=device)
        self.g.manual_seed(seed)

    def _rand(self, *shape):
        return self.t.rand(*shape, generator=self.g, device=self.dev, dtype=self.t.float64)

    def next(self, n):
        T = self.t
        tri = T.multinomial(self.area, n, replacement=True, generator=self.g)
        r1 = T.sqrt(self._rand(n))[:, None]
        r2 = self._rand(n)[:, None]
        t = self.tris[tri]
        x = (1 - r1) * t[:, 0] + r1 * (1 - r2) * t[:, 1] + r1 * r2 * t[:, 2]
        mu, kappa, lam = field_params(T, x)
        k = T.multinomial(lam, 1, generator=self.g)[:, 0]
        ar = T.arange(n, device=self.dev)
        m, kap = mu[ar, k], kappa[ar, k]
        v = self._rand(n)
        c = 1.0 + T.log(v + (1.0 - v) * T.exp(-2.0 * kap)) / kap
        s = T.sqrt(T.clamp(1.0 - c * c, min=0.0))
        ang = 2.0 * math.pi * self._rand(n)
        ref = T.where((m[:, 2:3].abs() < 0.9), T.tensor([0.0, 0.0, 1.0], device=self.dev,
                                                          dtype=T.float64),
                      T.tensor([1.0, 0.0, 0.0], device=self.dev, dtype=T.float64))
        t1 = T.linalg.cross(ref, m)
        t1 = t1 / T.linalg.norm(t1, dim=1, keepdim=True)
        t2 = T.linalg.cross(m, t1)
        w = c[:, None] * m + s[:, None] * (T.cos(ang)[:, None] * t1 + T.sin(ang)[:, None] * t2)
        w = w / T.linalg.norm(w, dim=1, keepdim=True)
        x32, w32 = x.float(), w.float()
        f = field_pdf(T, x32.double(), w32.double())
        e = -T.log1p(-self._rand(n))                 # Exp(1)
        soa = lambda a: a.t().contiguous()
        return soa(x32), soa(w32), (f * e).float(), f.float()
