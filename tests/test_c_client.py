"""The C ABI from plain C: tests/c_client/npm_client.c includes
include/npm.h, links libnpm.so and the HIP runtime, and uses nothing else
(no Python, no torch).  Without a device it must build, load and report
NPM_ERR_NO_DEVICE (exit 77); on the GPU its query and training losses are
checked against the FP64 oracle at the parameters it read back through
npm_get_state.

The client's network is the 4-level dense grid (8..64, F = 4) with MLP
16-64-64-32; it queries 4099 vertices with seed 5, stream 0, then trains
three steps on them (lr 1e-2)."""
import os
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "c_client"))
import build as cbuild  # noqa: E402

import parity as P  # noqa: E402

N = 4099


def test_client_builds_and_reports_no_device(tmp_path):
    exe = cbuild.build(str(tmp_path / "npm_client"))
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=120)
    # 77 without a device; on a GPU host the full run (checked below) exits 0
    assert r.returncode in (0, 77), r.stderr


@pytest.mark.gpu
def test_client_matches_the_oracle(O, tmp_path):
    exe = cbuild.BINARY if cbuild.up_to_date() else cbuild.build(str(tmp_path / "c"))
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    print(r.stdout.strip())

    def load(name, shape, dt=np.float32):
        return np.fromfile(tmp_path / name, dtype=dt).reshape(shape)

    pos, dirs = load("pos.f32", (3, N)), load("dir.f32", (3, N))
    rad, spdf = load("rad.f32", (N,)), load("spdf.f32", (N,))
    on = O.Net(4, 4, 8, 64, 19, True, 2, 64)
    params = load("params0.f32", (on.n_params,)).astype(np.float64)
    pdf, sdir = load("pdf.f32", (N,)), load("sdir.f32", (3, N)).T
    loss = load("loss.f64", (3,), np.float64)

    q = O.query(on, pos, params, dirs=dirs, seed=5, stream=0)
    _, raw_scale = O.mlp_forward(on, q["G"], params, with_scale=True)
    ones = np.ones(N, dtype=np.float32)
    _, d = O.loss_grad(on, q["raw"], dirs, ones, ones, n_total=1)
    kmax = q["lobes"][..., 2].max(axis=1)
    print(P.check_logpdf("C client pdf", pdf, q["logpdf"], P.logpdf_bound(d, raw_scale, kmax)))
    keep = q["margin"] > 1e-5
    assert keep.mean() > 0.999
    u = O.uniforms(N, 5, 0)
    sb = P.sample_bound(O, on, q["raw"][keep], raw_scale[keep], u[keep])
    print(P.assert_within("C client sample_dir", sdir[keep], q["sdir"][keep],
                          np.repeat(sb[:, None], 3, axis=1)))
    ref = O.backward(on, pos, dirs, rad, spdf, params, with_abs=False)
    assert loss[0] == pytest.approx(ref["loss"], rel=1e-5)
    assert np.all(np.isfinite(loss))
