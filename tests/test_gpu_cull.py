"""GPU parity of PVS culling (npvs_visible_triangles, npvs_visible_objects) against the oracle,
bit for bit, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_24677_amd as npvs
import synth
from gpu_util import DEV, to_np, upload_tris

pytestmark = pytest.mark.gpu


def _adversarial(rng, n, dims):
    out = []
    hi = np.array(dims, np.float64)
    for i in range(n):
        kind = i % 3
        if kind == 0:
            v = rng.uniform(-2, hi + 2, size=(3, 3))
        elif kind == 1:  # integer lattice: vertices, edges and faces on froxel boundaries
            v = rng.integers(0, np.array(dims) + 1, size=(3, 3)).astype(np.float64)
        else:  # long slivers across many words and rows
            a = rng.uniform(0, hi, size=3)
            b = rng.uniform(0, hi, size=3)
            v = np.stack([a, b, b + rng.uniform(-0.01, 0.01, 3)])
        out.append(v)
    return np.asarray(out, np.float32)


def _random_pvs(rng, dims, p):
    return [(rng.random((g[2], g[1], g[0] // 8, 8)) < p).astype(np.uint8) for g in dims]


def _pack(bits):
    return np.packbits(bits, axis=-1, bitorder="little").reshape(bits.shape[:-1])


@pytest.mark.parametrize("p", [0.0, 0.02, 0.3, 1.0])
def test_visible_triangles_batched_adversarial(p):
    rng = np.random.default_rng(31)
    dims = [(72, 24, 40), (32, 32, 32), (64, 8, 16)]
    tri_list = [_adversarial(rng, 400, g) for g in dims]
    tri_list[1] = np.concatenate([tri_list[1], np.full((2, 3, 3), np.nan, np.float32),
                                  np.full((1, 3, 3), 5000.0, np.float32)])
    pvs_list = [_pack(b) for b in _random_pvs(rng, dims, p)]
    tris, counts = upload_tris(tri_list)
    pvs = torch.from_numpy(np.concatenate([x.reshape(-1) for x in pvs_list])).to(DEV)
    got = to_np(npvs.visible_triangles(tris, counts, dims, pvs))
    want = np.concatenate([oracle.visible_triangles(t, g, x) for t, g, x in zip(tri_list, dims, pvs_list)])
    np.testing.assert_array_equal(got, want)
    if p == 0.0:
        assert not got.any()


def test_visible_triangles_against_a_network_pvs():
    cfg = synth.config("tiny32")
    t = synth.scene_for(cfg)
    layers = synth.net_layers(cfg)
    out = oracle.forward(t, cfg.grids[0], cfg.d, layers)
    pvs = out["pvs"]
    tris, counts = upload_tris([t])
    got = to_np(npvs.visible_triangles(tris, counts, cfg.grids, torch.from_numpy(pvs.reshape(-1)).to(DEV)))
    np.testing.assert_array_equal(got, oracle.visible_triangles(t, cfg.grids[0], pvs))
    # a sparser set (about a tenth of those bits) keeps some triangles and culls others
    sparse = pvs & synth.label_mask_bits(3, pvs.shape, p=0.1)
    got = to_np(npvs.visible_triangles(tris, counts, cfg.grids, torch.from_numpy(sparse.reshape(-1)).to(DEV)))
    np.testing.assert_array_equal(got, oracle.visible_triangles(t, cfg.grids[0], sparse))
    assert 0 < got.sum() < len(got)


def test_city_sample_against_a_pvs():
    """The 50 000 city triangles against a PVS-like subset of the city's occupancy (a seeded 35 %
    of the occupied froxels of the nearest 48 depth slices, built on the oracle side); a sample
    of 600 triangles against the oracle one by one."""
    cfg = synth.config("city256")
    t = synth.scene_for(cfg)
    occ, _ = oracle.froxelize(t, cfg.grids[0])  # [nz][ny][nx / 8]
    near = occ.copy()
    near[48:] = 0
    pvs_np = near.reshape(-1) & synth.label_mask_bits(9, (occ.size,))
    tris, counts = upload_tris([t])
    got = to_np(npvs.visible_triangles(tris, counts, cfg.grids, torch.from_numpy(pvs_np).to(DEV)))
    idx = np.random.default_rng(5).choice(len(t), 600, replace=False)
    want = oracle.visible_triangles(t[idx], cfg.grids[0], pvs_np)
    np.testing.assert_array_equal(got[idx], want)
    assert 0 < want.sum() < len(want)


def test_visible_objects_or_of_their_triangles():
    rng = np.random.default_rng(8)
    v = (rng.random(5000) < 0.05).astype(np.uint8)
    off = np.concatenate([[0], np.sort(rng.integers(0, 5001, size=300)), [5000]]).astype(np.int64)
    got = to_np(npvs.visible_objects(torch.from_numpy(v).to(DEV), torch.from_numpy(off).to(DEV)))
    np.testing.assert_array_equal(got, oracle.visible_objects(v, off))
