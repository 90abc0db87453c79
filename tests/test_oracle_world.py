"""Pins of the oracle's world-space front end (CPU): the viewcell frustum (Sec. 3.2) and the
froxelization of world-space triangles into linear depth slices of that frustum.

Independent routes: a hand-computed apex offset, the enclosure property the frustum is built
for, an exact rational separating-axis test (the oracle clips polygons instead), the paper's own
fragment rule (every sampled point of a triangle lands in a marked froxel), and closed-form
slices."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle

ZN, ZF = 0.3, 100.0


def _view(r=0.6):
    return oracle.viewcell_view([0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0], math.pi / 3, 1.0, r, math.pi / 12,
                                ZN, ZF)


def _bits(occ):
    return np.unpackbits(occ, axis=-1, bitorder="little")


def test_viewcell_apex_and_field_of_view():
    # the paper's camera: 60 degrees, 15 degrees of rotation, r = 0.6: apex 0.6 / tan(30 deg) =
    # 0.6 sqrt(3) behind the camera, field of view 90 degrees (half-angle tangent 1)
    v = oracle.viewcell_view([1.0, 2.0, 3.0], [0.0, 0.0, 2.0], [0.0, 5.0, 0.0], math.pi / 3, 1.0, 0.6, math.pi / 12,
                             ZN, ZF)
    np.testing.assert_allclose(v["eye"], [1.0, 2.0, 3.0 - 0.6 * math.sqrt(3.0)], rtol=0, atol=1e-15)
    assert v["tx"] == pytest.approx(1.0, abs=1e-15) and v["ty"] == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(np.stack([v["right"], v["up"], v["fwd"]]), np.eye(3), atol=1e-15)


def test_viewcell_frustum_encloses_moved_and_turned_cameras():
    rng = np.random.default_rng(0)
    theta, beta, r = math.pi / 3, math.pi / 12, 0.6
    v = oracle.viewcell_view([0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0], theta, 1.0, r, beta, ZN, ZF)
    for _ in range(4000):
        rho, phi = r * math.sqrt(rng.random()), 2 * math.pi * rng.random()
        cam = np.array([rho * math.cos(phi), rho * math.sin(phi), 0.0])
        # a ray of a camera turned by up to beta about each axis, inside its half-angle per axis
        ax = math.atan(math.tan(theta / 2) * rng.uniform(-1, 1)) + rng.uniform(-beta, beta)
        ay = math.atan(math.tan(theta / 2) * rng.uniform(-1, 1)) + rng.uniform(-beta, beta)
        d = np.array([math.tan(ax), math.tan(ay), 1.0])
        p = cam + rng.uniform(0.0, 50.0) * d - v["eye"]
        assert abs(p[0] / p[2]) <= v["tx"] + 1e-12 and abs(p[1] / p[2]) <= v["ty"] + 1e-12


# ---------------------------------------------------------------- exact rational reference
def _clip_exact(poly, zn):
    out = []
    for a in range(len(poly)):
        P, R = poly[a], poly[(a + 1) % len(poly)]
        dp, dr = P[2] - zn, R[2] - zn
        if dp >= 0:
            out.append(P)
        if (dp >= 0) != (dr >= 0):
            t = dp / (dp - dr)
            out.append(tuple(P[c] + t * (R[c] - P[c]) for c in range(3)))
    return out


def _sat_exact(tri, lo, hi):
    """Closed triangle vs closed box, separating axes, exact rationals."""
    e = [tuple(tri[(a + 1) % 3][c] - tri[a][c] for c in range(3)) for a in range(3)]
    unit = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    cross = lambda u, w: (u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0])
    axes = unit + [cross(e[0], e[1])] + [cross(ei, uj) for ei in e for uj in unit]
    corners = [(x, y, z) for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])]
    for a in axes:
        if a == (0, 0, 0):
            continue
        pt = [sum(a[c] * p[c] for c in range(3)) for p in tri]
        pb = [sum(a[c] * p[c] for c in range(3)) for p in corners]
        if max(pt) < min(pb) or min(pt) > max(pb):
            return False
    return True


def _exact_grid(tris, view, dims):
    nx, ny, nz = dims
    E = [Fr(x) for x in view["eye"]]
    B = [[Fr(x) for x in view[k]] for k in ("right", "up", "fwd")]
    tx, ty, zn, zf = Fr(view["tx"]), Fr(view["ty"]), Fr(view["zn"]), Fr(view["zf"])
    s = (zf - zn) / nz
    G = np.zeros((nz, ny, nx), np.uint8)
    for tri in tris:
        eye_pts = []
        for p in tri:
            d = [Fr(float(p[c])) - E[c] for c in range(3)]
            eye_pts.append(tuple(sum(d[c] * B[a][c] for c in range(3)) for a in range(3)))
        poly = _clip_exact(eye_pts, zn)
        if len(poly) < 3:
            continue
        P = [(p[0] / p[2], p[1] / p[2], 1 / p[2]) for p in poly]
        fans = [(P[0], P[a], P[a + 1]) for a in range(1, len(P) - 1)]
        for k in range(nz):
            qlo, qhi = 1 / (zn + (k + 1) * s), 1 / (zn + k * s)
            for j in range(ny):
                for i in range(nx):
                    lo = (tx * (Fr(2 * i, nx) - 1), ty * (Fr(2 * j, ny) - 1), qlo)
                    hi = (tx * (Fr(2 * (i + 1), nx) - 1), ty * (Fr(2 * (j + 1), ny) - 1), qhi)
                    if any(_sat_exact(f, lo, hi) for f in fans):
                        G[k, j, i] = 1
    return G


def _random_world_tris(rng, n, spread=6.0, zlo=-0.5, zhi=12.0):
    c = np.stack([rng.uniform(-spread, spread, n), rng.uniform(-spread, spread, n), rng.uniform(zlo, zhi, n)], 1)
    return (c[:, None, :] + rng.normal(0, 1.5, size=(n, 3, 3))).astype(np.float32)


@pytest.mark.parametrize("seed", [0, 1])
def test_matches_exact_separating_axis(seed):
    rng = np.random.default_rng(seed)
    dims = (8, 6, 5)
    view = _view()
    view = dict(view, zf=15.0)
    tris = _random_world_tris(rng, 6)
    exact = _exact_grid(tris, view, dims)
    got = _bits(oracle.froxelize_view(tris, view, dims)[0])
    inner = _bits(oracle.froxelize_view(tris, view, dims, margin=-1e-9)[0])
    outer = _bits(oracle.froxelize_view(tris, view, dims, margin=1e-9)[0])
    assert exact.any() and not exact.all()
    assert (inner <= exact).all() and (exact <= outer).all()
    np.testing.assert_array_equal(got, exact)


def test_sampled_points_land_in_marked_froxels():
    rng = np.random.default_rng(5)
    dims = (32, 32, 32)
    view = dict(_view(), zf=20.0)
    tris = _random_world_tris(rng, 60, spread=10.0, zhi=18.0)
    G = _bits(oracle.froxelize_view(tris, view, dims)[0])
    nx, ny, nz = dims
    B = np.stack([view["right"], view["up"], view["fwd"]])
    hits = 0
    for t in tris.astype(np.float64):
        w = rng.dirichlet(np.ones(3), size=300)
        pts = (w @ t - view["eye"]) @ B.T
        z = pts[:, 2]
        ok = (z > ZN) & (z < view["zf"])
        u = (pts[ok, 0] / z[ok] / view["tx"] + 1) / 2 * nx
        v = (pts[ok, 1] / z[ok] / view["ty"] + 1) / 2 * ny
        q = (z[ok] - ZN) / (view["zf"] - ZN) * nz
        inside = (u >= 0) & (u < nx) & (v >= 0) & (v < ny)
        for a, b, c in zip(u[inside], v[inside], q[inside]):
            # skip points within rounding distance of a froxel face
            if min(abs(a - round(a)), abs(b - round(b)), abs(c - round(c))) < 1e-9:
                continue
            assert G[int(c), int(b), int(a)], (a, b, c)
            hits += 1
    assert hits > 1000


def test_behind_the_camera_and_whole_slices():
    dims = (16, 16, 16)
    # apex at the origin (r = 0), slices exactly 1 deep: slice k covers eye depth [0.5 + k, 1.5 + k]
    view = oracle.viewcell_view([0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0], math.pi / 3, 1.0, 0.0, math.pi / 12,
                                0.5, 16.5)
    behind = np.array([[[-1, -1, -3.0], [1, -1, -3.0], [0, 1, -2.0]]], np.float32)
    assert not _bits(oracle.froxelize_view(behind, view, dims)[0]).any()

    def quad(z):  # a square at depth z reaching past the frustum's sides
        L = 4 * z
        a, b, c, d = [-L, -L, z], [L, -L, z], [L, L, z], [-L, L, z]
        return np.array([[a, b, c], [a, c, d]], np.float32)

    G = _bits(oracle.froxelize_view(quad(6.0), view, dims)[0])  # inside slice 5
    assert G[5].all() and G.sum() == 16 * 16
    G = _bits(oracle.froxelize_view(quad(6.5), view, dims)[0])  # on the face between slices 5 and 6
    assert G[5].all() and G[6].all() and G.sum() == 2 * 16 * 16
