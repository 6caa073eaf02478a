"""Pins of the oracle's multiresolution grid encoding (Sec. 5.1) and MLP.

Interpolation over the 8 corners of the enclosing cell is exact at lattice
points, reproduces affine fields, and its weights form a partition of unity.
Dense levels index their (D+1)^3 lattice points bijectively.  The MLP is
checked against numpy's float64 matmul.
"""
import math

import numpy as np
import pytest


def test_level_tables(O):
    n1 = O.Net(4, 4, 8, 64, 19, True, 2, 64)
    assert n1.res == [8, 16, 32, 64] and n1.hashed == [0, 0, 0, 0]
    assert n1.level_size == [(d + 1) ** 3 for d in n1.res]
    n2 = O.Net(16, 2, 16, 2048, 19, False, 3, 64)
    assert n2.res[0] == 16 and n2.res[-1] == 2048
    b = 2048 / 16
    for l, d in enumerate(n2.res):
        assert d == math.floor(16 * b ** (l / 15) + 1e-6)
    # dense exactly while (D+1)^3 fits the table
    for d, h, s in zip(n2.res, n2.hashed, n2.level_size):
        assert h == int((d + 1) ** 3 > 2 ** 19)
        assert s == (2 ** 19 if h else (d + 1) ** 3)
    assert n2.level_offset == list(np.cumsum([0] + n2.level_size[:-1]))
    assert n2.grid_entries == 6098925
    # the paper's own configuration (Sec. 5.3): D_1 = 8 ... D_8 = 86
    paper = O.Net(8, 4, 8, 86, 19, True, 2, 64)
    assert paper.res[0] == 8 and paper.res[-1] == 86 and sorted(paper.res) == paper.res


@pytest.mark.parametrize("L,base,mx", [(4, 8, 64), (16, 16, 2048), (8, 8, 86), (12, 5, 700)])
def test_level_resolutions_are_floors_of_the_exact_exponential(O, L, base, mx):
    """The reading of "grows exponentially": D_l = floor(base (max/base)^(l/(L-1)))
    of the exact real value (evaluated with 50 significant digits here), the
    last level forced to max.  Where that value is an integer (power-of-two
    ratios) the floating-point evaluation must not fall below it."""
    import mpmath
    mpmath.mp.dps = 50
    net = O.Net(L, 2, base, mx, 19, True, 1, 8)
    exact = [int(mpmath.floor(mpmath.mpf(base) * (mpmath.mpf(mx) / base) ** (mpmath.mpf(l) / (L - 1))
                              + mpmath.mpf(10) ** -30)) for l in range(L - 1)] + [mx]
    assert net.res == exact


def test_explicit_resolution_table(O):
    """An explicit table replaces the growth rule; the layout follows it
    (dense while (D+1)^3 fits the table, offsets the running sums), and the
    table equal to the derived one gives the derived layout."""
    table = [5, 7, 13, 13, 40, 97]
    net = O.Net(6, 2, 4, 64, 12, False, 2, 16, resolution=table)
    assert net.res == table
    for d, h, sz in zip(net.res, net.hashed, net.level_size):
        assert h == int((d + 1) ** 3 > 2 ** 12)
        assert sz == (2 ** 12 if h else (d + 1) ** 3)
    assert net.level_offset == list(np.cumsum([0] + net.level_size[:-1]))
    assert net.grid_params == 2 * sum(net.level_size)
    derived = O.Net(16, 2, 16, 2048, 19, False, 3, 64)
    again = O.Net(16, 2, 16, 2048, 19, False, 3, 64, resolution=derived.res)
    assert (again.res, again.level_offset, again.n_params) == \
           (derived.res, derived.level_offset, derived.n_params)
    for bad in ([5, 4, 13, 13, 40, 97], [0, 7, 13, 13, 40, 97], [5, 7, 13, 13, 40, 70000]):
        with pytest.raises(ValueError):
            O.Net(6, 2, 4, 64, 12, False, 2, 16, resolution=bad)


def _grid_net(O):
    # two dense power-of-two levels plus a hashed one (T = 2^9 < 33^3)
    return O.Net(3, 2, 4, 32, 9, False, 1, 8)


def test_partition_of_unity(O):
    net = _grid_net(O)
    rng = np.random.default_rng(1)
    pos = rng.uniform(-0.1, 1.1, (3, 5000)).astype(np.float32)
    idx, w = O.corners(net, pos)
    np.testing.assert_allclose(w.sum(axis=2), 1.0, atol=1e-14)
    assert np.all(w >= 0)


def test_exact_at_lattice_points(O):
    net = _grid_net(O)
    rng = np.random.default_rng(2)
    params = rng.normal(size=net.n_params)
    for l, D in enumerate(net.res):
        c = rng.integers(0, D + 1, size=(3, 300))
        pos = (c / D).astype(np.float32)            # exact: D is a power of two
        G = O.encode(net, pos, params)
        idx, w = O.corners(net, pos)
        # exactly one corner carries weight 1, and G equals its table entry
        assert np.all(np.sort(w[:, l, :], axis=1)[:, -1] == 1.0)
        k = np.argmax(w[:, l, :], axis=1)
        e = idx[np.arange(300), l, k]
        F = net.feat
        for f in range(F):
            np.testing.assert_array_equal(G[:, l * F + f], params[e * F + f])


def test_reproduces_affine_field(O):
    net = O.Net(3, 1, 5, 37, 30, True, 1, 8)      # dense, non power-of-two resolutions
    a = np.array([0.7, -1.3, 2.1]); b0 = 0.4
    params = np.zeros(net.n_params)
    for l, D in enumerate(net.res):
        g = np.arange(D + 1) / D
        X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
        vals = a[0] * X + a[1] * Y + a[2] * Z + b0
        # dense index = x + y (D+1) + z (D+1)^2
        off = net.level_offset[l]
        params[off:off + (D + 1) ** 3] = vals.transpose(2, 1, 0).reshape(-1)
    rng = np.random.default_rng(3)
    pos = rng.random((3, 2000)).astype(np.float32)
    G = O.encode(net, pos, params)
    want = a @ pos.astype(np.float64) + b0
    for l in range(3):
        np.testing.assert_allclose(G[:, l], want, atol=2e-6)


def test_clamping_outside_unit_cube(O):
    net = _grid_net(O)
    rng = np.random.default_rng(4)
    params = rng.normal(size=net.n_params)
    pos = rng.random((3, 100)).astype(np.float32)
    out = pos.copy()
    out[0, :50] = -0.3; out[1, 50:] = 1.7
    inn = out.copy()
    inn[0, :50] = 0.0; inn[1, 50:] = 1.0
    np.testing.assert_array_equal(O.encode(net, out, params), O.encode(net, inn, params))


def test_dense_index_bijective(O):
    net = O.Net(2, 1, 3, 6, 30, True, 1, 8)
    for l, D in enumerate(net.res):
        g = (np.arange(D) + 0.5) / D
        X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
        pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()]).astype(np.float32)
        idx, _ = O.corners(net, pos)
        seen = np.unique(idx[:, l, :])
        off = net.level_offset[l]
        np.testing.assert_array_equal(seen, np.arange(off, off + (D + 1) ** 3))


def test_hashed_indices_in_range(O):
    net = O.Net(16, 2, 16, 2048, 19, False, 3, 64)
    rng = np.random.default_rng(5)
    pos = rng.random((3, 4000)).astype(np.float32)
    idx, _ = O.corners(net, pos)
    for l in range(16):
        lo, sz = net.level_offset[l], net.level_size[l]
        assert idx[:, l, :].min() >= lo and idx[:, l, :].max() < lo + sz
    # the x term of the hash is the identity: corners differing only in x
    # land on table entries that differ only in the low bits (x XOR ...)
    l = 10
    d = (idx[:, l, 1] - net.level_offset[l]) ^ (idx[:, l, 0] - net.level_offset[l])
    cx = np.minimum(np.floor(pos[0] * np.float32(net.res[l])), net.res[l] - 1).astype(np.int64)
    assert np.all(d == (cx ^ (cx + 1)))


@pytest.mark.parametrize("feat,log2_slice", [(1, 14), (2, 13), (4, 12)])
def test_x_neighbour_pairs_share_a_slice(O, feat, log2_slice):
    """The binned grid scatter stores one item per pair of x-neighbour
    corners.  That rests on the hash taking x unmultiplied: at every hashed
    level and for every (y, z) corner pair, slot(x + 1) = slot(x) XOR
    (x XOR (x + 1)), so the two corners fall in the same table slice of
    2^log2_slice entries whenever the resolution is below the slice size
    (the slice sizes the pass uses at F = 1, 2, 4)."""
    net = O.Net(16, feat, 16, 2048, 19, False, 2, 32)
    rng = np.random.default_rng(7 + feat)
    pos = rng.random((3, 3000)).astype(np.float32)
    idx, _ = O.corners(net, pos)
    checked = 0
    for l in range(16):
        if not net.hashed[l]:
            continue
        D = net.res[l]
        assert D < (1 << log2_slice)
        off = net.level_offset[l]
        cx = np.minimum(np.floor(pos[0] * np.float32(D)), D - 1).astype(np.int64)
        for yz in range(4):                 # corners b = 2 yz (x) and 2 yz + 1 (x + 1)
            lo = idx[:, l, 2 * yz] - off
            hi = idx[:, l, 2 * yz + 1] - off
            np.testing.assert_array_equal(hi, lo ^ (cx ^ (cx + 1)))
            np.testing.assert_array_equal(hi >> log2_slice, lo >> log2_slice)
            checked += 1
    assert checked >= 4 * 10


def test_mlp_matches_numpy(O):
    net = O.Net(16, 2, 16, 2048, 19, False, 3, 64)
    rng = np.random.default_rng(6)
    params = rng.normal(scale=0.2, size=net.n_params)
    G = rng.normal(size=(300, net.n_in))
    raw, scale = O.mlp_forward(net, G, params, with_scale=True)
    h = G
    for i in range(len(net.layer_shape)):
        W = net.weights(params, i)
        z = h @ W.T
        h = np.maximum(z, 0.0) if i < len(net.layer_shape) - 1 else z
    np.testing.assert_allclose(raw, h, rtol=1e-12, atol=1e-12)
    assert np.all(scale >= np.abs(raw) - 1e-12)
