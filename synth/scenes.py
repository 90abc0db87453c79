"""Seeded scene, weight and label generators (numpy PCG64).

Every input of the froxelize -> interleave -> sparse CNN -> deinterleave path is drawn here.
Triangles are given directly in grid space: one unit is one froxel, x runs along the grid width
(fastest axis of the packed grid), y along the height and z along the depth slices.

Scenes stand in for the paper's evaluation scenes, which are not available: they follow the
paper's grid resolution (Sec. 4.2, A = 256), its occupancy regime (Sec. 2.3: under 5 % of the
froxels) and its scene character (Sec. 4.1: boxes, walls, floors, architectural structure).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _quad(a, b, c, d):
    """Two triangles (a, b, c) and (a, c, d) of the planar quad a-b-c-d."""
    return [(a, b, c), (a, c, d)]


def _tess_rect(o, u, v, na: int, nb: int):
    """Split the rectangle o + s*u + t*v, s,t in [0,1], into na x nb quads (2*na*nb triangles)."""
    o = np.asarray(o, np.float64)
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    out = []
    for i in range(na):
        for j in range(nb):
            p00 = o + u * (i / na) + v * (j / nb)
            p10 = o + u * ((i + 1) / na) + v * (j / nb)
            p11 = o + u * ((i + 1) / na) + v * ((j + 1) / nb)
            p01 = o + u * (i / na) + v * ((j + 1) / nb)
            out += _quad(p00, p10, p11, p01)
    return out


def _box_faces(lo, hi):
    """The five faces of an axis-aligned box without its bottom (y = lo.y) face, as
    (origin, u, v) rectangles."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    return [
        ((x0, y1, z0), (x1 - x0, 0, 0), (0, 0, z1 - z0)),  # top
        ((x0, y0, z0), (x1 - x0, 0, 0), (0, y1 - y0, 0)),  # front  z = z0
        ((x0, y0, z1), (x1 - x0, 0, 0), (0, y1 - y0, 0)),  # back   z = z1
        ((x0, y0, z0), (0, 0, z1 - z0), (0, y1 - y0, 0)),  # left   x = x0
        ((x1, y0, z0), (0, 0, z1 - z0), (0, y1 - y0, 0)),  # right  x = x1
    ]


def box_scene(seed: int, dims, n_boxes: int, side_lo: int = 2, side_hi: int = 8) -> np.ndarray:
    """Axis-aligned boxes with integer side lengths U{side_lo..side_hi} froxels whose corners
    are offset by U[0,1), so faces do not lie on froxel boundaries.  Each box contributes its
    five non-bottom faces as two triangles each (10 triangles per box).

    Returns float32 [T][3][3] grid-space vertices.
    """
    rng = _rng(seed)
    nx, ny, nz = dims
    tris = []
    for _ in range(n_boxes):
        side = rng.integers(side_lo, side_hi + 1, size=3)
        lim = np.array([nx, ny, nz]) - side - 1
        base = np.array([rng.integers(0, max(int(l), 0) + 1) for l in lim], np.float64)
        lo = base + rng.random(3)
        hi = lo + side
        for o, u, v in _box_faces(lo, hi):
            tris += _tess_rect(o, u, v, 1, 1)
    return np.asarray(tris, np.float32).reshape(-1, 3, 3)


def city_scene(seed: int = 1, dims=(256, 256, 128), n_tris: int = 50_000,
               n_buildings: int = 840) -> np.ndarray:
    """City blocks on a ground plane, tessellated to exactly ``n_tris`` triangles.

    The ground plane lies at a non-integer height and spans the whole x-z extent of the grid.
    Blocks are 32 (x) by 16 (z) froxels with 4-froxel streets.  Buildings have footprints
    U[3,10]^2 and log-normal heights (median 12, sigma_ln 0.6) clamped to the grid; each has
    five faces.  Faces are split into near-square quads of a common target edge length, and the
    ground plane absorbs the remaining triangle budget so the total is exact.
    """
    rng = _rng(seed)
    nx, ny, nz = dims
    y_g = float(rng.uniform(6.0, 10.0))
    block_x = [2 + 36 * i for i in range(nx) if 2 + 36 * i + 32 <= nx]
    block_z = [2 + 20 * j for j in range(nz) if 2 + 20 * j + 16 <= nz]
    faces = []
    for _ in range(n_buildings):
        bx = block_x[int(rng.integers(len(block_x)))]
        bz = block_z[int(rng.integers(len(block_z)))]
        w, l = rng.uniform(3.0, 10.0, size=2)
        x0 = bx + rng.uniform(0.0, 32.0 - w)
        z0 = bz + rng.uniform(0.0, 16.0 - l)
        h = float(np.exp(rng.normal(math.log(12.0), 0.6)))
        h = min(max(h, 1.0), ny - y_g - 1.5)
        faces += _box_faces((x0, y_g, z0), (x0 + w, y_g + h, z0 + l))

    def count(s: float) -> int:
        tot = 0
        for _, u, v in faces:
            a = max(1, round(float(np.linalg.norm(u)) / s))
            b = max(1, round(float(np.linalg.norm(v)) / s))
            tot += 2 * a * b
        return tot

    min_ground = 2 * 2048
    budget = n_tris - min_ground
    if count(1e9) > budget:
        raise ValueError("too many buildings for the triangle budget")
    lo_s, hi_s = 0.05, 1e3  # count(lo_s) > budget >= count(hi_s)
    for _ in range(60):
        mid = math.sqrt(lo_s * hi_s)
        if count(mid) > budget:
            lo_s = mid
        else:
            hi_s = mid
    s = hi_s
    tris = []
    for o, u, v in faces:
        a = max(1, round(float(np.linalg.norm(u)) / s))
        b = max(1, round(float(np.linalg.norm(v)) / s))
        tris += _tess_rect(o, u, v, a, b)
    k = (n_tris - len(tris)) // 2  # ground quads
    assert k >= 1 and len(tris) % 2 == 0
    kx = max(1, int(round(math.sqrt(k * nx / nz))))
    kx = min(kx, k)
    x_edges = np.linspace(0.0, float(nx), kx + 1)
    for i in range(kx):
        rows = k // kx + (1 if i < k % kx else 0)
        z_edges = np.linspace(0.0, float(nz), rows + 1)
        for j in range(rows):
            tris += _quad((x_edges[i], y_g, z_edges[j]), (x_edges[i + 1], y_g, z_edges[j]),
                          (x_edges[i + 1], y_g, z_edges[j + 1]), (x_edges[i], y_g, z_edges[j + 1]))
    out = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    assert out.shape[0] == n_tris, out.shape
    return out


def he_weights(seed: int, channels, bias_std: float = 0.0):
    """He-normal weights W[27][Cin][Cout] ~ N(0, 2 / (27 Cin)) for each layer of the channel
    list, float32.  Biases are zero unless ``bias_std`` > 0 (tests use non-zero biases)."""
    rng = _rng(seed)
    out = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        w = rng.normal(0.0, math.sqrt(2.0 / (27 * cin)), size=(27, cin, cout)).astype(np.float32)
        b = (rng.normal(0.0, bias_std, size=cout) if bias_std > 0 else np.zeros(cout)).astype(np.float32)
        out.append((w, b))
    return out


def unet_params(seed: int, d: int, E: int = 64, Dc: int = 96, bias_std: float = 0.05) -> dict:
    """He-normal weights of the two-level U-Net, stage by stage: stem [27][d^3][E], enc0 2 x
    [27][E][E], down [8][E][E], enc1 3 x [27][E][E], up [8][E][Dc], dec0 [27][Dc+E][Dc] and
    [27][Dc][Dc], head [27][Dc][d^3]; biases N(0, bias_std)."""
    rng = _rng(seed)

    def conv(k, cin, cout):
        w = rng.normal(0.0, math.sqrt(2.0 / (k * cin)), size=(k, cin, cout)).astype(np.float32)
        return w, rng.normal(0.0, bias_std, size=cout).astype(np.float32)

    C = d ** 3
    return dict(stem=[conv(27, C, E)], enc0=[conv(27, E, E) for _ in range(2)], down=[conv(8, E, E)],
                enc1=[conv(27, E, E) for _ in range(3)], up=[conv(8, E, Dc)],
                dec0=[conv(27, Dc + E, Dc), conv(27, Dc, Dc)], head=[conv(27, Dc, C)])


def label_mask_bits(seed: int, shape_bytes, p: float = 0.35) -> np.ndarray:
    """Random packed bit mask (uint8, same shape as a packed froxel grid) with each bit set with
    probability p.  ANDed with an occupancy grid it gives a fixed label subset of G, used where
    label values do not affect the measurement."""
    rng = _rng(seed)
    bits = rng.random(tuple(shape_bytes) + (8,)) < p
    return np.packbits(bits, axis=-1, bitorder="little").reshape(shape_bytes)


def viewpoints(seed: int, m: int, centre, side: float) -> np.ndarray:
    """m viewpoints drawn uniformly from the axis-aligned cube of the given side centred at
    ``centre`` (the viewcell), float64 [m][3]."""
    rng = _rng(seed)
    c = np.asarray(centre, np.float64)
    return c + (rng.random((m, 3)) - 0.5) * side


# ----------------------------------------------------------------------------------------
# Workload configurations
# ----------------------------------------------------------------------------------------

@dataclass
class Config:
    name: str
    grids: list            # list of (nx, ny, nz)
    d: int
    channels: list         # conv channel list, e.g. [64]*7 for six 64->64 layers
    scene: str             # "boxes" | "city"
    seeds: list
    weight_seed: int
    scene_args: list = field(default_factory=list)  # per-grid kwargs


def _c4_grids():
    dims_cycle = [(64, 64, 64), (128, 128, 64), (128, 128, 128), (192, 192, 128), (256, 256, 128)]
    rng = _rng(4000)
    occ = rng.uniform(0.01, 0.10, size=16)
    grids, args = [], []
    for i in range(16):
        g = dims_cycle[i % len(dims_cycle)]
        grids.append(g)
        n = g[0] * g[1] * g[2]
        # about 1100 occupied froxels per box of sides U{4..24} (measured on 128^3 scenes)
        args.append(dict(n_boxes=max(1, int(round(occ[i] * n / 1100.0))), side_lo=4, side_hi=24))
    return grids, args


CONFIGS = {
    "tiny32": Config("tiny32", [(32, 32, 32)], 2, [8, 16, 16, 8], "boxes", [0], 100,
                     [dict(n_boxes=20, side_lo=2, side_hi=8)]),
    "city256": Config("city256", [(256, 256, 128)], 4, [64] * 7, "city", [1], 101, [dict()]),
    "train128x4": Config("train128x4", [(128, 128, 128)] * 4, 4, [64] * 7, "boxes",
                         [30, 31, 32, 33], 101,
                         [dict(n_boxes=80, side_lo=4, side_hi=24)] * 4),
}
_g, _a = _c4_grids()
CONFIGS["batch16"] = Config("batch16", _g, 4, [64] * 7, "boxes", list(range(40, 56)), 101, _a)
# the paper's interleave factors: first and last layers d^3 = 512 or 4096 channels wide
CONFIGS["city256_d8"] = Config("city256_d8", [(256, 256, 128)], 8, [512] + [64] * 5 + [512], "city", [1], 108,
                               [dict()])
CONFIGS["city256_d16"] = Config("city256_d16", [(256, 256, 128)], 16, [4096] + [64] * 5 + [4096], "city", [1],
                                116, [dict()])
# no interleave (d = 1, the ablation of Table 2): one input and one output channel per site
CONFIGS["tiny32_d1"] = Config("tiny32_d1", [(32, 32, 32)], 1, [1, 16, 16, 1], "boxes", [0], 201,
                              [dict(n_boxes=20, side_lo=2, side_hi=8)])
CONFIGS["city256_d1"] = Config("city256_d1", [(256, 256, 128)], 1, [1] + [64] * 5 + [1], "city", [1], 102, [dict()])
CONFIGS["city256_d2"] = Config("city256_d2", [(256, 256, 128)], 2, [8] + [64] * 5 + [8], "city", [1], 103, [dict()])
CONFIGS["boxes64_d8"] = Config("boxes64_d8", [(64, 64, 64)], 8, [512, 32, 512], "boxes", [5], 208,
                               [dict(n_boxes=12, side_lo=4, side_hi=16)])
CONFIGS["boxes64_d16"] = Config("boxes64_d16", [(64, 64, 64)], 16, [4096, 32, 4096], "boxes", [6], 216,
                                [dict(n_boxes=12, side_lo=4, side_hi=16)])


def config(name: str) -> Config:
    return CONFIGS[name]


def net_layers(cfg: Config, bias_std: float = 0.0):
    return he_weights(cfg.weight_seed, cfg.channels, bias_std)


def scene_for(cfg: Config, i: int = 0) -> np.ndarray:
    if cfg.scene == "city":
        return city_scene(cfg.seeds[i], cfg.grids[i], **cfg.scene_args[i])
    return box_scene(cfg.seeds[i], cfg.grids[i], **cfg.scene_args[i])
