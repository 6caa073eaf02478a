"""Seeded synthetic workloads for the NPM hot path.

This module only *generates inputs*: vertex positions, directions, Monte Carlo
radiance estimates and their sampling pdfs, standing in for the path vertices
a wavefront path tracer would hand to the guiding network (the paper's scenes
and renderer are not part of this library).  It holds none of the method's
arithmetic: no grid encoding, no MLP, no Table 1 mapping, no training step.
It is shared by the tests, the benchmark and the smoke check, on both the GPU
and the CPU-oracle side, and depends on numpy only.

The "scene" is an analytic incident-radiance field that is itself an 8-lobe
vMF mixture whose parameters vary smoothly with position, so the optimum the
network should reach is known.  It is evaluated and sampled here with its own
numpy code (the generator plays the renderer's role).

Shapes follow the paper's workload: ~2^20 path vertices per wavefront
(1280x720 = 921,600 in Sec. 6.4), training batches of 2^18..2^20 samples,
vertices on surfaces, directional lobed radiance.
"""
from dataclasses import dataclass, field, replace
import math

import numpy as np

FIELD_LOBES = 8


# ----------------------------------------------------------------------------
# Network / grid configurations of the five workloads (sizes only).
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class NetConfig:
    n_levels: int
    feat: int
    base_res: int
    max_res: int
    log2_table: int
    dense_only: bool
    n_hidden: int            # hidden ReLU layers; the output layer is extra
    width: int
    n_lobes: int = 8
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    grid_init: str = "uniform"   # "normal" (sigma) or "uniform" (+-scale)
    grid_init_scale: float = 1e-4
    precision: str = "fp32"      # "fp32" or "bf16" (BF16 MLP + FP16 grid)
    seed: int = 1
    sh_degree: int = 0           # NPM-product: SH bands of omega_o and the normal
    resolution: tuple = ()       # explicit per-level resolutions (empty: grow base..max)
    select: bool = False         # learned BSDF-selection probability (one more output)

    @property
    def n_in(self):
        return self.n_levels * self.feat


# Plain FP32, 4 dense levels 8/16/32/64 x F=4, MLP 16-64-64-32, N(0, var 1e-4)
CFG1 = NetConfig(n_levels=4, feat=4, base_res=8, max_res=64, log2_table=19, dense_only=True,
                 n_hidden=2, width=64, grid_init="normal", grid_init_scale=1e-2, seed=1)
# Plain FP32 production size: 16 levels x F=2, T=2^19, 16..2048, MLP 32-64-64-64-32
CFG2 = NetConfig(n_levels=16, feat=2, base_res=16, max_res=2048, log2_table=19, dense_only=False,
                 n_hidden=3, width=64, grid_init="uniform", grid_init_scale=1e-4, seed=2)
# Precision form of cfg2
CFG3 = replace(CFG2, precision="bf16", seed=3)
# Differentiation form of cfg2 (lr 1e-2, 200 steps)
CFG4 = replace(CFG2, seed=4)
# Serving: per-session 16-level FP16 hash grid with T=2^17
CFG5 = replace(CFG2, log2_table=17, precision="bf16", seed=5)
# Finite-difference net: 2-level hash grid, T=2^8, F=2, MLP 4-8-8-32
TINY = NetConfig(n_levels=2, feat=2, base_res=4, max_res=16, log2_table=8, dense_only=False,
                 n_hidden=2, width=8, grid_init="uniform", grid_init_scale=0.3, seed=7)

# The paper's own network (Sec. 5.3): 8 dense levels 8..86 x F=4, three linear
# layers of width 64 (MLP 32-64-64-32), lr 5e-3; query batch = one 1280x720
# wavefront, training batch 2^18 (Sec. 6.4).  Grid init is not stated: U(+-1e-4).
PAPER = NetConfig(n_levels=8, feat=4, base_res=8, max_res=86, log2_table=19, dense_only=True,
                  n_hidden=2, width=64, lr=5e-3, grid_init="uniform", grid_init_scale=1e-4,
                  seed=6)

# NPM-product (Sec. 4.3) forms: omega_o, normal and roughness after G(x), four
# SH bands each (65 inputs on the 32 grid features); two bands on TINY.
CFG2P = replace(CFG2, sh_degree=4, seed=8)
PAPERP = replace(PAPER, sh_degree=4, seed=9)
TINYP = replace(TINY, sh_degree=2, seed=10)

# Learned BSDF-selection probability (Sec. 6.3 extension): one more output.
TINYS = replace(TINY, select=True, seed=11)
CFG1S = replace(CFG1, select=True, seed=12)
PAPERS = replace(PAPER, select=True, seed=13)

N_CFG1 = 16384
N_CFG2 = 1 << 20
N_PAPER_QUERY = 1280 * 720
N_PAPER_TRAIN = 1 << 18


# ----------------------------------------------------------------------------
# The analytic field (the synthetic scene's incident radiance, normalised).
# ----------------------------------------------------------------------------
def _fibonacci_dirs(k):
    i = np.arange(k)
    z = 1.0 - (2.0 * i + 1.0) / k
    psi = i * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(1.0 - z * z)
    return np.stack([r * np.cos(psi), r * np.sin(psi), z], axis=1)


def field_params(x, phase=0.0):
    """Field mixture at positions x [n][3] (float64).

    Returns mu [n][8][3], kappa [n][8], lam [n][8].  Lobe k has
    base direction m_k (Fibonacci point), perturbed by 0.4 * sinusoids of x,
    kappa_k(x) = 10 exp(sin(2 pi (x0 + 2 x1 + 3 x2) + a_k)) in [3.7, 27.2],
    lambda = softmax_k(sin(2 pi x_{k mod 3} + a_k)), a_k = 2 pi k / 8 + phase.
    """
    x = np.asarray(x, dtype=np.float64)
    k = np.arange(FIELD_LOBES)
    a = 2.0 * math.pi * k / FIELD_LOBES + phase
    m = _fibonacci_dirs(FIELD_LOBES)
    pert = np.stack([np.sin(2 * math.pi * x[:, None, 0] + a[None, :]),
                     np.sin(2 * math.pi * x[:, None, 1] + 2 * a[None, :]),
                     np.sin(2 * math.pi * x[:, None, 2] + 3 * a[None, :])], axis=2)
    mu = m[None, :, :] + 0.4 * pert
    mu /= np.linalg.norm(mu, axis=2, keepdims=True)
    kappa = 10.0 * np.exp(np.sin(2 * math.pi * (x[:, 0] + 2 * x[:, 1] + 3 * x[:, 2])[:, None]
                                 + a[None, :]))
    logits = np.sin(2 * math.pi * x[:, k % 3] + a[None, :])
    logits -= logits.max(axis=1, keepdims=True)
    lam = np.exp(logits)
    lam /= lam.sum(axis=1, keepdims=True)
    return mu, kappa, lam


def field_pdf(x, w, phase=0.0):
    """Field density at (x [n][3], w [n][3]), float64."""
    mu, kappa, lam = field_params(x, phase)
    cosv = np.einsum("nkd,nd->nk", mu, np.asarray(w, dtype=np.float64))
    # kappa / (4 pi sinh kappa) * exp(kappa cos) = kappa/(2 pi (1-e^{-2k})) * exp(kappa (cos-1))
    dens = kappa / (2 * math.pi * (-np.expm1(-2 * kappa))) * np.exp(kappa * (cosv - 1.0))
    return (lam * dens).sum(axis=1)


def _orthonormal_frame(mu):
    # any frame; the generator's sampler does not need the network's convention
    a = np.where(np.abs(mu[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    t1 = np.cross(a, mu)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(mu, t1)
    return t1, t2


def field_sample(rng, x, phase=0.0):
    """Exact samples of the field's directional density at each x."""
    n = x.shape[0]
    mu, kappa, lam = field_params(x, phase)
    cdf = np.cumsum(lam, axis=1)
    u = rng.random(n)[:, None] * cdf[:, -1:]
    k = np.minimum((u >= cdf).sum(axis=1), FIELD_LOBES - 1)
    m = mu[np.arange(n), k]
    kap = kappa[np.arange(n), k]
    # cosine to the lobe axis from the inverse CDF of e^{kappa t} on [-1, 1]
    v = rng.random(n)
    t = 1.0 + np.log(v + (1.0 - v) * np.exp(-2.0 * kap)) / kap
    s = np.sqrt(np.clip(1.0 - t * t, 0.0, None))
    ang = 2.0 * math.pi * rng.random(n)
    t1, t2 = _orthonormal_frame(m)
    w = t[:, None] * m + s[:, None] * (np.cos(ang)[:, None] * t1 + np.sin(ang)[:, None] * t2)
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    return w


# ----------------------------------------------------------------------------
# Vertex positions: uniform in the cube (cfg1) or on a random triangle set.
# ----------------------------------------------------------------------------
def triangle_soup(rng, n_tri=4096):
    c = rng.uniform(0.1, 0.9, size=(n_tri, 1, 3))
    return c + rng.uniform(-0.08, 0.08, size=(n_tri, 3, 3))


def surface_points(rng, n, tris, return_tri=False):
    e1 = tris[:, 1] - tris[:, 0]
    e2 = tris[:, 2] - tris[:, 0]
    area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
    t = rng.choice(tris.shape[0], size=n, p=area / area.sum())
    r1 = np.sqrt(rng.random(n))[:, None]
    r2 = rng.random(n)[:, None]
    # uniform barycentrics (Osada et al. 2002)
    x = (1 - r1) * tris[t, 0] + r1 * (1 - r2) * tris[t, 1] + r1 * r2 * tris[t, 2]
    return (x, t) if return_tri else x


def triangle_normals(tris):
    nrm = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    return nrm / np.linalg.norm(nrm, axis=1, keepdims=True)


def uniform_sphere(rng, n):
    z = rng.uniform(-1.0, 1.0, n)
    a = rng.uniform(0.0, 2 * math.pi, n)
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(a), r * np.sin(a), z], axis=1)


@dataclass
class Batch:
    """One SoA batch of path vertices, float32, ready to upload."""
    pos: np.ndarray        # [3][n]
    dir: np.ndarray        # [3][n] unit vectors
    radiance: np.ndarray   # [n]  Monte Carlo radiance estimate L
    pdf: np.ndarray        # [n]  pdf the direction was sampled with
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.pos.shape[1]

    def subset(self, idx):
        return Batch(self.pos[:, idx].copy(), self.dir[:, idx].copy(), self.radiance[idx].copy(),
                     self.pdf[idx].copy(), dict(self.meta))


def _soa(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).T.astype(np.float32))


def make_batch(kind, n, seed, phase=0.0, tris_seed=None):
    """kind "cube": x ~ U[0,1]^3, w ~ U(S^2), p = 1/(4 pi), L = field(w|x) E.
    kind "surface": x on a random triangle set, w ~ field(.|x), p = field(w|x),
    L = field(w|x) E; E ~ Exp(1) in both."""
    rng = np.random.default_rng(seed)
    if kind == "cube":
        x = rng.random((n, 3))
        w = uniform_sphere(rng, n)
        p = np.full(n, 1.0 / (4 * math.pi))
    elif kind == "surface":
        trng = np.random.default_rng(1000 + (seed if tris_seed is None else tris_seed))
        tris = triangle_soup(trng)
        x, tri = surface_points(rng, n, tris, return_tri=True)
        normal = triangle_normals(tris)[tri]
        w = field_sample(rng, x, phase)
        p = None
    else:
        raise ValueError(kind)
    x32 = x.astype(np.float32).astype(np.float64)
    w32 = w.astype(np.float32).astype(np.float64)
    f = field_pdf(x32, w32, phase)
    if p is None:
        p = f
    e = rng.exponential(1.0, n)
    meta = dict(kind=kind, seed=seed, phase=phase)
    if kind == "surface":
        meta["normal"] = normal
    return Batch(_soa(x), _soa(w), (f * e).astype(np.float32), p.astype(np.float32), meta)


def make_aux(batch, seed):
    """NPM-product inputs [7][n] float32 for a batch: the outgoing direction
    omega_o (cosine-distributed about the normal, the direction a path
    arrives from), the surface normal (the triangle's, facing omega_o; a
    random unit vector for cube batches), and a roughness U(0.05, 1)."""
    rng = np.random.default_rng(50000 + seed)
    n = batch.n
    nrm = batch.meta.get("normal")
    if nrm is None:
        nrm = uniform_sphere(rng, n)
    # cosine-weighted direction about nrm (Malley's method in a local frame)
    r = np.sqrt(rng.random(n))
    phi = 2 * math.pi * rng.random(n)
    local = np.stack([r * np.cos(phi), r * np.sin(phi), np.sqrt(np.maximum(0.0, 1 - r * r))], 1)
    a = np.where(np.abs(nrm[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    t1 = np.cross(a, nrm)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(nrm, t1)
    wo = local[:, :1] * t1 + local[:, 1:2] * t2 + local[:, 2:3] * nrm
    wo /= np.linalg.norm(wo, axis=1, keepdims=True)
    rough = rng.uniform(0.05, 1.0, n)
    out = np.concatenate([wo.T, nrm.T, rough[None, :]], 0)
    return np.ascontiguousarray(out.astype(np.float32))


def make_bsdf(batch, seed):
    """BSDF sampling density [n] float32 at each sample's direction, for the
    learned selection probability: half the vertices diffuse (cos / pi about
    the normal, 0 below it), half glossy (the normalised Phong lobe
    (m + 1) / (2 pi) max(0, r . w)^m about a random unit r, with m
    log-uniform in [1, 1000], so near-specular densities reach ~160)."""
    rng = np.random.default_rng(70000 + seed)
    n = batch.n
    nrm = batch.meta.get("normal")
    if nrm is None:
        nrm = uniform_sphere(rng, n)
    w = batch.dir.T.astype(np.float64)
    diffuse = rng.random(n) < 0.5
    r = uniform_sphere(rng, n)
    m = np.exp(rng.uniform(0.0, math.log(1000.0), n))
    cos_n = np.maximum(0.0, np.sum(nrm * w, axis=1))
    cos_r = np.maximum(0.0, np.sum(r * w, axis=1))
    p = np.where(diffuse, cos_n / math.pi, (m + 1) / (2 * math.pi) * cos_r ** m)
    return np.ascontiguousarray(p.astype(np.float32))


def edge_positions(rng, n, res_list):
    """Positions that stress the lattice: exact lattice points of the given
    resolutions, 0, 1, values just inside/outside [0,1], and NaN-free randoms."""
    out = rng.random((n, 3))
    sel = rng.integers(0, 6, size=(n, 3))
    res = np.asarray(res_list)[rng.integers(0, len(res_list), size=(n, 3))]
    lattice = rng.integers(0, res + 1) / res
    out = np.where(sel == 0, lattice, out)
    out = np.where(sel == 1, 0.0, out)
    out = np.where(sel == 2, 1.0, out)
    out = np.where(sel == 3, np.nextafter(1.0, 0.0), out)
    out = np.where(sel == 4, rng.choice([-0.25, 1.25, -1e-7, 1 + 1e-7], size=(n, 3)), out)
    return np.ascontiguousarray(out.T.astype(np.float32))
