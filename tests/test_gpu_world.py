"""GPU parity of the world-space front end (viewcell frustum, froxelization into linear depth
slices) against the oracle, through the C ABI.  Both sides decide in float64 but do different
arithmetic (the oracle clips the polygon against every froxel, the kernels clip it once per row
of froxels and read the covered run off its X extent), so the GPU grid must contain every froxel
the oracle marks with the froxels shrunk by 1e-9 of their size, and no froxel the oracle rejects
with them grown by 1e-9; in practice it equals the oracle's grid."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2509_24677_amd as npvs
import synth
from gpu_util import DEV, to_np

pytestmark = pytest.mark.gpu


def _as_dict(v):
    return dict(eye=np.array(v.eye), right=np.array(v.right), up=np.array(v.up), fwd=np.array(v.forward),
                tx=v.tan_half_x, ty=v.tan_half_y, zn=v.z_near, zf=v.z_far)


def _check(tris, view, dims):
    """view: (the library's frustum, the oracle's frustum of the same camera)."""
    view, vd = view
    lib = _as_dict(view)  # the library's frustum equals the oracle's
    for k in vd:
        np.testing.assert_allclose(lib[k], vd[k], rtol=1e-12, atol=1e-12, err_msg=k)
    got = to_np(npvs.froxelize_view(torch.from_numpy(tris).to(DEV), view, dims)).reshape(dims[2], dims[1], -1)
    bits = lambda occ: np.unpackbits(occ, axis=-1, bitorder="little")
    exact, n = oracle.froxelize_view(tris, vd, dims)
    inner = bits(oracle.froxelize_view(tris, vd, dims, margin=-1e-9)[0])
    outer = bits(oracle.froxelize_view(tris, vd, dims, margin=1e-9)[0])
    g = bits(got)
    assert (inner <= g).all(), int((inner > g).sum())
    assert (g <= outer).all(), int((g > outer).sum())
    diff = int((g != bits(exact)).sum())
    print(f"dims {dims}: {n} froxels marked, {diff} differ from the oracle's margin-0 grid", flush=True)
    assert diff == 0
    return n


def _paper_view(c, zf=1000.0):
    """Sec. 4.3 camera: 60 degree field of view, 15 degrees of rotation (90 degree grid), near 0.3;
    the library's frustum and, computed on the oracle side, the oracle's."""
    args = (c, [0.0, 0.0, 1.0], [0.0, 1.0, 0.0], math.pi / 3, 1.0, 0.6, math.pi / 12, 0.3, zf)
    return npvs.viewcell_frustum(*args), oracle.viewcell_view(*args)


@pytest.mark.parametrize("dims", [(64, 64, 64), (96, 40, 70)])
def test_random_triangles_near_the_camera(dims):
    rng = np.random.default_rng(sum(dims))
    n = 400
    c = np.stack([rng.uniform(-8, 8, n), rng.uniform(-8, 8, n), rng.uniform(-1.5, 18, n)], 1)
    tris = (c[:, None, :] + rng.normal(0, 1.5, size=(n, 3, 3))).astype(np.float32)
    assert _check(tris, _paper_view([0.0, 0.0, 0.0], zf=20.0), dims) > 1000


def test_city_frame_in_world_space():
    cfg = synth.config("city256")
    tris = synth.scene_for(cfg)
    assert _check(tris, _paper_view([128.0, 40.0, -20.0]), (256, 256, 256)) > 100000


def test_no_triangles_and_triangles_behind_the_camera():
    view, _ = _paper_view([0.0, 0.0, 0.0], zf=20.0)
    occ = npvs.froxelize_view(torch.zeros((0, 3, 3), dtype=torch.float32, device=DEV), view, (32, 32, 32))
    assert not to_np(occ).any()
    behind = np.array([[[-1, -1, -3.0], [1, -1, -3.0], [0, 1, -2.5]]], np.float32)
    occ = npvs.froxelize_view(torch.from_numpy(behind).to(DEV), view, (32, 32, 32))
    assert not to_np(occ).any()
