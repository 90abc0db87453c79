"""Pins of the oracle's froxelization (Sec. 3.2, pre-processing; Fig. 2(b)).

The oracle decides triangle / closed-froxel overlap with an integer separating-axis test.  These
tests pin it to things other than itself: an exact rational polygon-clipping test over every
(triangle, froxel) pair, closed forms for axis-aligned boxes and in-plane triangles, sampled
points on the triangles, order invariance and the tie cases (vertices, edges and faces on froxel
boundaries), and the worst-case coordinate range of the int64 arithmetic.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

FX = 256


def _clip(poly, axis, bound, keep_ge):
    out = []
    m = len(poly)
    for i in range(m):
        p, q = poly[i], poly[(i + 1) % m]
        ip = p[axis] >= bound if keep_ge else p[axis] <= bound
        iq = q[axis] >= bound if keep_ge else q[axis] <= bound
        if ip:
            out.append(p)
        if ip != iq:
            t = (bound - p[axis]) / (q[axis] - p[axis])
            out.append(tuple(p[a] + t * (q[a] - p[a]) for a in range(3)))
    return out


def clip_overlap(q, lo, hi) -> bool:
    """Exact: the triangle's intersection with the closed box is non-empty iff clipping it by the
    six closed half-spaces in rational arithmetic leaves a (possibly degenerate) polygon."""
    poly = [tuple(Fraction(int(c)) for c in v) for v in q]
    for a in range(3):
        poly = _clip(poly, a, Fraction(int(lo[a])), True)
        if not poly:
            return False
        poly = _clip(poly, a, Fraction(int(hi[a])), False)
        if not poly:
            return False
    return True


def _unpacked(tris, dims):
    occ, ign = oracle.froxelize(np.asarray(tris, np.float32).reshape(-1, 3, 3), dims)
    return oracle.unpack(occ), ign


def _random_tris(rng, n, lo, hi):
    out = []
    for t in range(n):
        kind = t % 3
        if kind == 0:
            v = rng.uniform(lo, hi, size=(3, 3))
        elif kind == 1:
            v = rng.integers(int(lo), int(hi) + 1, size=(3, 3)).astype(np.float64)
        else:
            v = rng.integers(int(2 * lo), int(2 * hi) + 1, size=(3, 3)) / 2.0
        if t % 7 == 3:  # collinear / point-degenerate triangles
            v[2] = v[0] + (v[1] - v[0]) * rng.choice([0.0, 0.5, 2.0])
        out.append(v)
    return np.asarray(out, np.float32)


def test_matches_exact_clipping_every_pair():
    rng = np.random.default_rng(11)
    dims = (8, 6, 5)
    tris = _random_tris(rng, 45, -1.0, 8.5)
    for t in tris:
        got, _ = _unpacked(t, dims)
        q = oracle.quantize_tri(t)
        for k in range(dims[2]):
            for j in range(dims[1]):
                for i in range(dims[0]):
                    lo = (FX * i, FX * j, FX * k)
                    hi = (FX * i + FX, FX * j + FX, FX * k + FX)
                    assert got[k, j, i] == int(clip_overlap(q, lo, hi)), (t.tolist(), (i, j, k))


def test_axis_aligned_box_closed_form():
    rng = np.random.default_rng(5)
    dims = (24, 16, 16)
    for _ in range(6):
        lo = rng.integers(0, 6, size=3) + rng.uniform(0.1, 0.8, size=3)
        hi = lo + rng.integers(2, 8, size=3) + rng.uniform(0.05, 0.1)
        faces = synth.scenes._box_faces(lo, hi)
        tris = []
        for o, u, v in faces:
            tris += synth.scenes._tess_rect(o, u, v, 2, 3)
        got, _ = _unpacked(tris, dims)
        want = np.zeros((dims[2], dims[1], dims[0]), np.uint8)
        f = np.floor
        i0, j0, k0 = (int(f(c)) for c in lo)
        i1, j1, k1 = (int(f(c)) for c in hi)
        want[k0:k1 + 1, j1, i0:i1 + 1] = 1           # top y = hi.y
        want[k0, j0:j1 + 1, i0:i1 + 1] = 1           # front z = lo.z
        want[k1, j0:j1 + 1, i0:i1 + 1] = 1           # back z = hi.z
        want[k0:k1 + 1, j0:j1 + 1, i0] = 1           # left x = lo.x
        want[k0:k1 + 1, j0:j1 + 1, i1] = 1           # right x = hi.x
        np.testing.assert_array_equal(got, want)


def test_triangle_in_plane_between_layers_touches_one_layer():
    rng = np.random.default_rng(7)
    dims = (16, 16, 8)
    for _ in range(10):
        k = int(rng.integers(0, dims[2]))
        xy = rng.uniform(0.3, 15.7, size=(3, 2))
        t = np.concatenate([xy, np.full((3, 1), k + 0.5)], axis=1)
        got, _ = _unpacked(t, dims)
        layers = np.nonzero(got.reshape(dims[2], -1).any(axis=1))[0]
        assert list(layers) == [k]
        # the 2D overlap set of the layer equals the exact clip on that layer
        q = oracle.quantize_tri(t)
        for j in range(dims[1]):
            for i in range(dims[0]):
                want = clip_overlap(q, (FX * i, FX * j, FX * k), (FX * i + FX, FX * j + FX, FX * k + FX))
                assert got[k, j, i] == int(want)


def test_face_on_froxel_plane_marks_both_layers():
    dims = (8, 8, 8)
    t = np.array([[1.25, 1.5, 3.0], [6.5, 1.75, 3.0], [2.25, 6.5, 3.0]], np.float32)
    got, _ = _unpacked(t, dims)
    layers = np.nonzero(got.reshape(dims[2], -1).any(axis=1))[0]
    assert list(layers) == [2, 3]
    np.testing.assert_array_equal(got[2], got[3])


def test_vertex_on_corner_marks_eight_froxels():
    dims = (8, 8, 8)
    p = np.array([3.0, 4.0, 5.0], np.float32)
    t = np.stack([p, p, p])  # a point-degenerate triangle exactly on a froxel corner
    got, _ = _unpacked(t, dims)
    want = np.zeros((8, 8, 8), np.uint8)
    want[4:6, 3:5, 2:4] = 1
    np.testing.assert_array_equal(got, want)


def test_edge_along_froxel_edge_marks_four_columns():
    dims = (8, 8, 8)
    t = np.array([[2.0, 3.0, 1.2], [2.0, 3.0, 5.7], [2.0, 3.0, 3.3]], np.float32)  # segment on x=2,y=3
    got, _ = _unpacked(t, dims)
    want = np.zeros((8, 8, 8), np.uint8)
    want[1:6, 2:4, 1:3] = 1
    np.testing.assert_array_equal(got, want)


def test_sampled_points_lie_in_marked_froxels():
    rng = np.random.default_rng(3)
    dims = (32, 32, 16)
    tris = _random_tris(rng, 60, 0.2, 15.8)
    got, _ = _unpacked(tris, dims)
    uv = np.array([(a, b) for a in np.linspace(0, 1, 21) for b in np.linspace(0, 1, 21) if a + b <= 1])
    for t in tris.astype(np.float64):
        pts = t[0] + uv[:, :1] * (t[1] - t[0]) + uv[:, 1:] * (t[2] - t[0])
        idx = np.floor(pts).astype(int)
        ok = (idx >= 0).all(1) & (idx < np.array(dims)).all(1)
        idx = idx[ok]
        assert got[idx[:, 2], idx[:, 1], idx[:, 0]].all()


def test_order_and_vertex_rotation_invariance():
    rng = np.random.default_rng(9)
    dims = (32, 16, 16)
    tris = _random_tris(rng, 80, 0.0, 15.5)
    a, _ = _unpacked(tris, dims)
    perm = rng.permutation(len(tris))
    rot = np.roll(tris[perm], 1, axis=1)[:, ::-1]
    b, _ = _unpacked(rot, dims)
    np.testing.assert_array_equal(a, b)


def test_invalid_triangles_are_ignored():
    dims = (8, 8, 8)
    good = np.array([[1.5, 1.5, 1.5], [2.5, 1.5, 1.5], [1.5, 2.5, 1.5]], np.float32)
    bad = [good.copy() for _ in range(4)]
    bad[0][1, 0] = np.nan
    bad[1][2, 2] = np.inf
    bad[2][0, 1] = 2048.0
    bad[3][1, 2] = -2048.0
    far = good + np.float32(1500.0)  # inside the exact range, outside the grid: not ignored, marks nothing
    got, ign = _unpacked(np.stack([good] + bad + [far]), dims)
    want, _ = _unpacked(good, dims)
    assert ign == 4
    np.testing.assert_array_equal(got, want)


def test_large_triangles_crossing_the_grid_match_exact_clipping():
    # vertices in [1024, 2048): the triangle reaches far outside the grid and still marks exactly
    # the froxels it meets (G(x) = 1 iff a triangle meets x, Sec. 3.2, with no limit on where the
    # triangle lies); checked against rational clipping on whole froxel rows of a 256-wide grid
    dims = (256, 8, 8)
    tris = np.array([
        [[-1500.25, 3.5, 2.0], [1900.75, 4.25, 6.5], [200.0, 1600.5, -1300.0]],
        [[1024.0, -1024.0, 4.5], [-2047.5, 2.0, 4.5], [100.5, 2047.0, 4.5]],
        [[-1999.5, 0.5, 7.75], [1999.25, 7.5, 0.25], [64.0, -1500.0, -1800.0]],
    ], np.float32)
    rows = [(0, 0), (3, 2), (4, 4), (7, 7), (1, 6), (2, 1), (4, 6)]
    for t in tris:
        got, ign = _unpacked(t, dims)
        assert ign == 0
        q = oracle.quantize_tri(t)
        for j, k in rows:
            for i in range(dims[0]):
                want = clip_overlap(q, (FX * i, FX * j, FX * k), (FX * i + FX, FX * j + FX, FX * k + FX))
                assert got[k, j, i] == int(want), (t, i, j, k)
        assert got.any()


def test_worst_case_coordinate_range_is_exact():
    # vertices at the edge of the accepted range exercise the largest int64 products
    t = np.array([[-2047.99, -2047.5, 2047.99], [2047.99, 3.25, -2047.75], [1.5, 2047.9, 0.5]], np.float32)
    dims = (16, 16, 16)
    got, ign = _unpacked(t, dims)
    assert ign == 0
    q = oracle.quantize_tri(t)
    assert np.abs(q).max() <= 2 ** 19
    for k in range(0, 16, 3):
        for j in range(16):
            for i in range(0, 16, 2):
                want = clip_overlap(q, (FX * i, FX * j, FX * k), (FX * i + FX, FX * j + FX, FX * k + FX))
                assert got[k, j, i] == int(want)


def test_quantization_rounds_half_to_even():
    t = np.zeros((3, 3), np.float32)
    t[0] = [0.5 / 256, 1.5 / 256, 2.5 / 256]
    t[1] = [-0.5 / 256, -1.5 / 256, 3.0]
    q = oracle.quantize_tri(t)
    assert q[0].tolist() == [0, 2, 2]
    assert q[1].tolist() == [0, -2, 768]


@pytest.mark.parametrize("name", ["tiny32"])
def test_config_scene_occupancy(name):
    cfg = synth.config(name)
    occ, ign = oracle.froxelize(synth.scene_for(cfg), cfg.grids[0])
    frac = oracle.unpack(occ).mean()
    assert ign == 0 and 0.05 < frac < 0.11
