"""Tolerance policy of the GPU-vs-oracle parity tests (test infrastructure).

The plain FP32 path must match the FP64 oracle to 1e-5 relative, with
integer work (grid corner indices) bit-exact.  "Relative" is taken against the
size of the terms that produce each value (its condition scale), because
FP32 sums of terms of mixed sign have errors proportional to sum |term|, not
to the (possibly cancelled) result:

* encoding G and raw MLP outputs: |d| <= 1e-5 * max(|ref|, sum |terms|);
* mapped lobe parameters: the raw error bound propagated through the
  Table 1 mapping's derivative, plus 1e-5 relative on the value itself;
* log pdf: 1e-5 + 1e-5 * sum_j |d logV / d raw_j| * scale_j
  + 4 * kappa_max * 2^-23 (an ulp of mu.w amplified by kappa);
* sampled directions (same uniforms): |d|_inf <= 2e-5 plus the change of the
  oracle's sample when each raw output moves by its own 1e-5 tolerance,
  except samples whose CDF margin is below 1e-5, where FP32 and FP64 may
  pick different lobes;
* sample pdf: the log-pdf bound at the sample plus the sample's own move
  (its bound above) through the gradient of log V in the direction;
* gradients: |d| <= 1e-5 * cond, where cond is the oracle's condition scale
  of the entry: the first-order bound on an FP32 evaluation's error in
  units of the unit roundoff -- the sizes of all the terms it rounds,
  propagated from the KL-gradient head (its own rounding, amplified by
  kappa, plus the raw outputs' rounding through the head's Jacobian)
  through the MLP and the scatter (sums of many signed terms -- dG =
  W^T delta, the atomic sums over vertices -- have errors proportional to
  them, not to the result).  Its size against an FP32 evaluation's actual
  errors is pinned on the CPU (tests/test_oracle_cond.py).
"""
import numpy as np

RTOL = 1e-5
FP32_EPS = 2.0 ** -23


def report(name, err, bound):
    ratio = float(np.max(err / bound)) if err.size else 0.0
    return f"{name}: max err {float(np.max(err)) if err.size else 0:.3e}, max err/bound {ratio:.3f}"


def assert_within(name, got, ref, bound):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    err = np.abs(got - ref)
    bad = ~(err <= bound)
    if bad.any():
        i = np.flatnonzero(bad.ravel())[:8]
        raise AssertionError(f"{name}: {bad.sum()} of {bad.size} out of tolerance; e.g. "
                             f"got {got.ravel()[i]} ref {ref.ravel()[i]} bound {bound.ravel()[i]}")
    return report(name, err, bound)


def check_scaled(name, got, ref, scale, rtol=RTOL):
    ref = np.asarray(ref, dtype=np.float64)
    bound = rtol * np.maximum(np.abs(ref), scale) + 1e-30
    return assert_within(name, got, ref, bound)


def check_lobes(got, ref, raw_scale, rtol=RTOL):
    """got/ref: [n][K][4] (theta, phi, kappa, lambda); raw_scale [n][4K]."""
    s = raw_scale.reshape(-1, 8, 4)
    th, ph, ka, la = (ref[..., i] for i in range(4))
    msgs = []
    b = rtol * (th + th * (1 - th) * s[..., 0]) + 1e-30
    msgs.append(assert_within("theta", got[..., 0], th, b))
    b = rtol * (ph + ph * (1 - ph) * s[..., 1]) + 1e-30
    msgs.append(assert_within("phi", got[..., 1], ph, b))
    b = rtol * ka * (1 + s[..., 2])
    msgs.append(assert_within("kappa", got[..., 2], ka, b))
    b = rtol * la * (1 + 2 * s[..., 3].max(axis=1, keepdims=True))
    msgs.append(assert_within("lambda", got[..., 3], la, b))
    return msgs


def logpdf_bound(dlogv_draw, raw_scale, kappa_max, rtol=RTOL):
    sens = np.sum(np.abs(dlogv_draw) * raw_scale, axis=1)
    return rtol * (1.0 + sens) + 4.0 * kappa_max * FP32_EPS


def check_logpdf(name, got_pdf, ref_logpdf, bound):
    with np.errstate(divide="ignore"):
        lg = np.log(np.asarray(got_pdf, dtype=np.float64))
    return assert_within(name, lg, ref_logpdf, bound)


def sample_bound(O, net, raw, raw_scale, u, base=2e-5, rtol=RTOL):
    """|d omega| allowed per sample: base + sum_j |omega(raw + rtol scale_j e_j)
    - omega(raw)| (first-order effect of each raw output's tolerance)."""
    w0, _ = O.sample_raw(net, raw, u)
    b = np.full(raw.shape[0], base)
    for j in range(raw.shape[1]):
        r = raw.copy()
        r[:, j] += rtol * raw_scale[:, j]
        w1, _ = O.sample_raw(net, r, u)
        b += np.abs(w1 - w0).max(axis=1)
    return b


def sample_logpdf_bound(O, net, raw, sdir, sb, lp_bound, kappa_max, h=1e-6):
    """Bound on |log V_gpu(w_gpu) - log V_ref(w_ref)| for a sample: the
    log-density's own bound at the sample, plus the move of the sample
    itself, |w_gpu - w_ref| <= sqrt(3) sb (sb bounds each component),
    through the gradient of log V in the direction (central differences of
    the oracle's log-density in FP64), and the second-order term with the
    Hessian bounded by kappa_max^2."""
    g = np.zeros_like(sdir)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        g[:, d] = (O.logpdf(net, raw, sdir + e) - O.logpdf(net, raw, sdir - e)) / (2.0 * h)
    move = np.sqrt(3.0) * sb
    return lp_bound + np.linalg.norm(g, axis=1) * move + 0.5 * kappa_max ** 2 * move ** 2


def cond_quantiles(cond, gabs):
    """cond / sum|contributions| at the median and the 99th percentile."""
    nz = gabs > 0
    if not nz.any():
        return "cond/gabs: no contributions"
    q = np.quantile(cond[nz] / gabs[nz], [0.5, 0.99])
    return f"cond/gabs median {q[0]:.3g}, p99 {q[1]:.3g}"


def check_grads(name, got, ref, gabs, rtol=RTOL, atol=1e-12):
    bound = rtol * gabs + atol
    return assert_within(name, got, ref, bound)


def fibonacci_sphere(m):
    i = np.arange(m) + 0.5
    z = 1 - 2 * i / m
    a = i * np.pi * (3 - np.sqrt(5))
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(a), r * np.sin(a), z], 1)


def sample_chi2_pvalue(O, on, raw, samples, nz=8, nphi=8, quad=16):
    """Chi-square p-value of sampled directions [m][3] against the oracle's
    mixture pdf for the raw outputs `raw` [4K]: cells of equal width in cos
    theta and phi, expected counts by Gauss-Legendre quadrature of the pdf,
    cells expecting fewer than 5 draws dropped."""
    from scipy import stats
    m = samples.shape[0]
    zb = np.linspace(-1, 1, nz + 1)
    pb = np.linspace(-np.pi, np.pi, nphi + 1)
    H, _, _ = np.histogram2d(samples[:, 2], np.arctan2(samples[:, 1], samples[:, 0]),
                             bins=[zb, pb])
    x, wx = np.polynomial.legendre.leggauss(quad)
    E = np.zeros((nz, nphi))
    for i in range(nz):
        z = 0.5 * (zb[i + 1] - zb[i]) * (x + 1) + zb[i]
        wz = 0.5 * (zb[i + 1] - zb[i]) * wx
        for j in range(nphi):
            ph = 0.5 * (pb[j + 1] - pb[j]) * (x + 1) + pb[j]
            wp = 0.5 * (pb[j + 1] - pb[j]) * wx
            Z, PH = np.meshgrid(z, ph, indexing="ij")
            R = np.sqrt(1 - Z * Z)
            d = np.stack([R * np.cos(PH), R * np.sin(PH), Z], -1).reshape(-1, 3)
            lp = O.logpdf(on, np.broadcast_to(raw, (d.shape[0], raw.shape[0])), d)
            E[i, j] = np.sum(np.exp(lp) * np.outer(wz, wp).reshape(-1))
    E *= m / E.sum()
    keep = E > 5
    chi = float(((H[keep] - E[keep]) ** 2 / E[keep]).sum())
    return float(stats.chi2.sf(chi, keep.sum() - 1))
