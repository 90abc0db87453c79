"""Pins of the oracle's PVS culling (a triangle is kept iff it overlaps a visible froxel; an
object iff any of its triangles is kept)."""
import numpy as np

import oracle
import synth


def _tri(a, b, c):
    return np.array([a, b, c], np.float32).reshape(1, 9)


def test_empty_pvs_culls_everything_and_full_occupancy_keeps_every_accepted_triangle():
    cfg = synth.config("tiny32")
    t = synth.scene_for(cfg)
    dims = cfg.grids[0]
    occ, ign = oracle.froxelize(t, dims)
    assert ign == 0
    none = oracle.visible_triangles(t, dims, np.zeros_like(occ))
    assert not none.any()
    # every triangle overlaps its own froxels, all of which are occupied
    assert oracle.visible_triangles(t, dims, occ).all()


def test_single_visible_froxel():
    dims = (16, 16, 16)
    inside = _tri((3.2, 4.2, 5.2), (3.8, 4.3, 5.4), (3.4, 4.9, 5.6))   # within froxel (3, 4, 5)
    far = _tri((10.2, 10.2, 10.2), (10.8, 10.3, 10.4), (10.4, 10.9, 10.6))
    touch = _tri((4.0, 4.2, 5.2), (4.0, 4.8, 5.4), (4.0, 4.5, 5.9))    # on the plane x = 4 (closed boxes)
    pvs = np.zeros((16, 16, 2), np.uint8)
    pvs[5, 4, 0] = 1 << 3                                              # froxel (3, 4, 5)
    v = oracle.visible_triangles(np.concatenate([inside, far, touch]), dims, pvs)
    np.testing.assert_array_equal(v, [1, 0, 1])
    pvs[5, 4, 0] = 1 << 4                                              # froxel (4, 4, 5) instead
    v = oracle.visible_triangles(np.concatenate([inside, far, touch]), dims, pvs)
    np.testing.assert_array_equal(v, [0, 0, 1])


def test_ignored_triangles_are_never_visible():
    dims = (16, 16, 16)
    big = _tri((3.0, 4.0, 5.0), (2048.0, 4.0, 5.0), (3.0, 5.0, 5.0))  # |v| >= 2048 froxels: ignored
    nan = _tri((3.0, 4.0, 5.0), (np.nan, 4.0, 5.0), (3.0, 5.0, 5.0))
    full = np.full((16, 16, 2), 0xFF, np.uint8)
    np.testing.assert_array_equal(oracle.visible_triangles(np.concatenate([big, nan]), dims, full), [0, 0])


def test_objects_are_or_of_their_triangles():
    v = np.array([0, 0, 1, 0, 0, 0, 1], np.uint8)
    np.testing.assert_array_equal(oracle.visible_objects(v, [0, 2, 4, 4, 7]), [0, 1, 0, 1])
