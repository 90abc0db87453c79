"""Pins of the oracle's active sites, interleave g_d (Sec. 3.3), rulebook and submanifold
convolution (Sec. 2.3), and de-interleave + threshold (Sec. 3.1, 3.3).

Each oracle function is checked against an independent route: numpy reshapes/transposes for the
permutations, O(n^2) neighbour search for the rulebook, a masked dense convolution and
torch.nn.functional.conv3d (float64, CPU) for the sparse convolution, and closed forms.
"""
import numpy as np
import pytest
import torch

import oracle
import synth


def _np_interleave(a, d):
    nz, ny, nx = a.shape[:3]
    return (a.reshape(nz // d, d, ny // d, d, nx // d, d)
            .transpose(0, 2, 4, 1, 3, 5).reshape(nz // d, ny // d, nx // d, d ** 3))


def _scene(seed=0, dims=(32, 32, 32), n_boxes=20):
    tris = synth.box_scene(seed, dims, n_boxes)
    occ, _ = oracle.froxelize(tris, dims)
    return tris, occ


# ------------------------------------------------------------------ active sites
@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_active_sites_brute_force(d):
    dims = (32, 16, 24)
    _, occ = _scene(1, dims, 8)
    keys = oracle.active_sites(occ, dims, d)
    g = oracle.unpack(occ)
    act = _np_interleave(g, d).any(axis=-1).reshape(-1)
    np.testing.assert_array_equal(keys, np.nonzero(act)[0])
    assert (np.diff(keys) > 0).all()


# ------------------------------------------------------------------ interleave
@pytest.mark.parametrize("dtype", [np.uint8, np.float16, np.float32, np.float64])
@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_interleave_roundtrip_and_count(dtype, d):
    rng = np.random.default_rng(d)
    dims = (16, 8, 24)
    a = (rng.random((dims[2], dims[1], dims[0])) * 100).astype(dtype)
    b = oracle.interleave(a, d)
    assert b.size == a.size and b.shape[-1] == d ** 3
    np.testing.assert_array_equal(oracle.deinterleave(b, dims, d), a)
    np.testing.assert_array_equal(b, _np_interleave(a, d))
    c = (rng.random(b.shape) * 100).astype(dtype)
    np.testing.assert_array_equal(oracle.interleave(oracle.deinterleave(c, dims, d), d), c)


def test_interleave_closed_form_4cube():
    a = np.arange(64, dtype=np.int32).reshape(4, 4, 4)  # value = (z*4 + y)*4 + x
    b = oracle.interleave(a, 2)
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                for oz in range(2):
                    for oy in range(2):
                        for ox in range(2):
                            want = ((bz * 2 + oz) * 4 + (by * 2 + oy)) * 4 + (bx * 2 + ox)
                            assert b[bz, by, bx, (oz * 2 + oy) * 2 + ox] == want


def test_d1_is_identity():
    a = np.arange(8 * 8 * 8, dtype=np.float32).reshape(8, 8, 8)
    np.testing.assert_array_equal(oracle.interleave(a, 1).reshape(8, 8, 8), a)


def test_gather_sites_is_sparse_interleave():
    dims = (32, 32, 32)
    _, occ = _scene(2, dims)
    keys = oracle.active_sites(occ, dims, 2)
    X = oracle.gather_sites(occ, dims, 2, keys)
    dense = _np_interleave(oracle.unpack(occ), 2).reshape(-1, 8)
    np.testing.assert_array_equal(X, dense[keys])


# ------------------------------------------------------------------ rulebook
def _brute_pairs(keys, bdims):
    Bx, By, Bz = bdims
    pos = np.stack([keys % Bx, (keys // Bx) % By, keys // (Bx * By)], 1)
    out = {}
    for k in range(27):
        dz, dy, dx = k // 9 - 1, (k // 3) % 3 - 1, k % 3 - 1
        s = []
        for r in range(len(keys)):
            for i in range(len(keys)):
                if (pos[i] == pos[r] + np.array([dx, dy, dz])).all():
                    s.append((i, r))
        out[k] = s
    return out


def test_rulebook_brute_force_and_symmetries():
    dims = (16, 16, 16)
    _, occ = _scene(3, dims, 6)
    keys = oracle.active_sites(occ, dims, 2)
    bd = (8, 8, 8)
    rb_off, pairs = oracle.rulebook(keys, bd)
    brute = _brute_pairs(keys, bd)
    total = 0
    for k in range(27):
        seg = [tuple(p) for p in pairs[rb_off[k]:rb_off[k + 1]]]
        assert seg == brute[k]  # same pairs, ascending output row
        total += len(seg)
        mirror = {(r, i) for i, r in pairs[rb_off[26 - k]:rb_off[27 - k]]}
        assert set(seg) == mirror
    assert total == rb_off[27] == len(pairs)
    centre = pairs[rb_off[13]:rb_off[14]]
    np.testing.assert_array_equal(centre[:, 0], np.arange(len(keys)))
    np.testing.assert_array_equal(centre[:, 1], np.arange(len(keys)))


# ------------------------------------------------------------------ convolution
def _dense_of(X, keys, bdims):
    Bx, By, Bz = bdims
    D = np.zeros((Bz * By * Bx, X.shape[1]))
    D[keys] = X
    act = np.zeros(Bz * By * Bx, np.uint8)
    act[keys] = 1
    return D.reshape(Bz, By, Bx, -1), act.reshape(Bz, By, Bx)


def _torch_conv3d(D, W, b):
    # W[k][c][o], k = (dz+1)*9 + (dy+1)*3 + (dx+1)  ->  torch weight [o][c][dz][dy][dx]
    cin, cout = W.shape[1:]
    w = torch.from_numpy(W.reshape(3, 3, 3, cin, cout).transpose(4, 3, 0, 1, 2).copy())
    x = torch.from_numpy(D.transpose(3, 0, 1, 2)[None].copy())
    y = torch.nn.functional.conv3d(x, w, torch.from_numpy(b), padding=1)
    return y[0].numpy().transpose(1, 2, 3, 0)


def _setup_conv(seed, cin, cout, dims=(32, 32, 32), d=2):
    _, occ = _scene(seed, dims)
    keys = oracle.active_sites(occ, dims, d)
    bd = tuple(s // d for s in dims)
    rb_off, pairs = oracle.rulebook(keys, bd)
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(len(keys), cin))
    W = rng.normal(size=(27, cin, cout)) / np.sqrt(27 * cin)
    b = rng.normal(size=cout)
    return keys, bd, rb_off, pairs, X, W, b


@pytest.mark.parametrize("relu", [False, True])
def test_sparse_equals_masked_dense(relu):
    keys, bd, rb_off, pairs, X, W, b = _setup_conv(4, 8, 16)
    Y = oracle.subm_conv(X, W, b, rb_off, pairs, relu)
    D, act = _dense_of(X, keys, bd)
    Yd = oracle.masked_dense_conv(D, act, W, b, relu).reshape(-1, W.shape[2])
    np.testing.assert_allclose(Y, Yd[keys], rtol=0, atol=1e-12)
    assert not Yd[np.setdiff1d(np.arange(len(Yd)), keys)].any()


def test_masked_dense_fully_active_equals_torch_conv3d():
    rng = np.random.default_rng(5)
    bd = (6, 5, 4)
    D = rng.normal(size=(4, 5, 6, 3))
    W = rng.normal(size=(27, 3, 5))
    b = rng.normal(size=5)
    act = np.ones((4, 5, 6), np.uint8)
    got = oracle.masked_dense_conv(D, act, W, b, False)
    np.testing.assert_allclose(got, _torch_conv3d(D, W, b), rtol=0, atol=1e-12)
    # and the sparse form on the fully active grid agrees too
    keys = np.arange(np.prod(bd), dtype=np.int32)
    rb_off, pairs = oracle.rulebook(keys, bd)
    Y = oracle.subm_conv(D.reshape(-1, 3), W, b, rb_off, pairs, False)
    np.testing.assert_allclose(Y, _torch_conv3d(D, W, b).reshape(-1, 5), rtol=0, atol=1e-12)


def test_delta_weight_shifts():
    keys, bd, rb_off, pairs, X, _, _ = _setup_conv(6, 4, 4)
    Bx, By, Bz = bd
    row_of = {int(k): r for r, k in enumerate(keys)}
    for k in [0, 5, 13, 22, 26]:
        W = np.zeros((27, 4, 4))
        W[k] = np.eye(4)
        Y = oracle.subm_conv(X, W, None, rb_off, pairs, False)
        dz, dy, dx = k // 9 - 1, (k // 3) % 3 - 1, k % 3 - 1
        for r, key in enumerate(keys):
            bx, by, bz = key % Bx + dx, (key // Bx) % By + dy, key // (Bx * By) + dz
            nb = (bz * By + by) * Bx + bx
            inside = 0 <= bx < Bx and 0 <= by < By and 0 <= bz < Bz
            want = X[row_of[nb]] if inside and nb in row_of else np.zeros(4)
            np.testing.assert_array_equal(Y[r], want)


def test_centre_only_is_rowwise_gemm_and_all_ones_counts_neighbours():
    keys, bd, rb_off, pairs, X, W, b = _setup_conv(7, 8, 6)
    Wc = np.zeros_like(W)
    Wc[13] = W[13]
    np.testing.assert_allclose(oracle.subm_conv(X, Wc, b, rb_off, pairs, False), X @ W[13] + b, atol=1e-12)
    ones = oracle.subm_conv(np.ones_like(X), np.ones_like(W), None, rb_off, pairs, False)
    nbrs = np.bincount(pairs[:, 1], minlength=len(keys))
    np.testing.assert_array_equal(ones, np.repeat((8 * nbrs)[:, None], 6, axis=1))


def test_translation_equivariance_block_aligned():
    dims = (32, 32, 32)
    tris = synth.box_scene(8, (24, 24, 24), 10)
    shift = np.array([4.0, 2.0, 6.0], np.float32)  # multiples of d = 2
    o1 = oracle.forward(tris, dims, 2, synth.he_weights(3, [8, 6, 8], 0.1))
    o2 = oracle.forward(tris + shift, dims, 2, synth.he_weights(3, [8, 6, 8], 0.1))
    np.testing.assert_allclose(o1["acts"][-1], o2["acts"][-1], atol=1e-12)
    l1 = o1["logits"]
    l2 = o2["logits"]
    np.testing.assert_array_equal(l1[:26, :30, :28], l2[6:, 2:, 4:])


# ------------------------------------------------------------------ deinterleave + threshold
def test_deinterleave_threshold_independent_route_and_subset():
    dims = (32, 32, 32)
    out = oracle.forward(synth.box_scene(0, dims, 20), dims, 2, synth.he_weights(100, [8, 16, 16, 8], 0.05))
    keys, occ = out["keys"], out["occ"]
    Y = out["acts"][-1]
    dense = np.full(((32 // 2) ** 3, 8), -np.inf)
    dense[keys] = Y
    logits = oracle.deinterleave(dense.reshape(16, 16, 16, 8), dims, 2)
    np.testing.assert_array_equal(out["logits"], logits)
    bits = (logits >= 0) & (oracle.unpack(occ) == 1)
    np.testing.assert_array_equal(out["pvs"], np.packbits(bits, axis=-1, bitorder="little"))
    assert not (oracle.unpack(out["pvs"]) & (1 - oracle.unpack(occ))).any()  # V within G
    assert 0 < oracle.unpack(out["pvs"]).sum() < oracle.unpack(occ).sum()
