"""GPU parity of the forward path against the CPU oracle, through the C ABI.

Integer stages (froxelize, sites, rulebook, interleave) must be bit-exact; float stages must sit
within the float32 accumulation bound of each layer and, for the whole network, 1e-5 max-abs on
the logits against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_24677_amd as npvs
import synth
from gpu_util import DEV, bf16_reference, bf16_round, conv_tolerance, drift_tol, oracle_batch, to_np, upload_tris

pytestmark = pytest.mark.gpu


def _frox_and_rb(tri_list, dims, d, csr=True):
    tris, counts = upload_tris(tri_list)
    occ = npvs.froxelize(tris, counts, dims)
    rb = npvs.build_rulebook(occ, dims, d, csr=csr)
    return occ, rb


# ------------------------------------------------------------------------------- froxelize
@pytest.mark.parametrize("name", ["tiny32", "city256"])
def test_froxelize_bit_exact_configs(name):
    cfg = synth.config(name)
    t = synth.scene_for(cfg)
    print(f"froxelize {name} T={len(t)}", flush=True)
    tris, counts = upload_tris([t])
    occ = npvs.froxelize(tris, counts, cfg.grids)
    want, _ = oracle.froxelize(t, cfg.grids[0])
    np.testing.assert_array_equal(to_np(occ), want.reshape(-1))


def _adversarial(rng, n, dims):
    out = []
    hi = np.array(dims, np.float64)
    for i in range(n):
        kind = i % 4
        if kind == 0:
            v = rng.uniform(-2, hi + 2, size=(3, 3))
        elif kind == 1:  # integer lattice: vertices/edges/faces on froxel boundaries
            v = rng.integers(0, np.array(dims) + 1, size=(3, 3)).astype(np.float64)
        elif kind == 2:  # small triangles near corners
            c = rng.integers(0, np.array(dims), size=3).astype(np.float64)
            v = c + rng.choice([-0.5, 0.0, 0.5, 1.0 / 256, -1.0 / 512], size=(3, 3))
        else:  # long slivers across many tiles
            a = rng.uniform(0, hi, size=3)
            b = rng.uniform(0, hi, size=3)
            v = np.stack([a, b, b + rng.uniform(-0.01, 0.01, 3)])
        if i % 9 == 4:
            v[2] = v[1]  # degenerate
        out.append(v)
    return np.asarray(out, np.float32)


def test_froxelize_adversarial_and_batched():
    rng = np.random.default_rng(21)
    dims = [(136, 24, 40), (32, 32, 32), (64, 8, 16)]
    tri_list = [_adversarial(rng, 700, g) for g in dims]
    tri_list[1] = np.concatenate([tri_list[1], np.full((2, 3, 3), np.nan, np.float32),
                                  np.full((1, 3, 3), 5000.0, np.float32)])
    tris, counts = upload_tris(tri_list)
    occ = npvs.froxelize(tris, counts, dims)
    want = np.concatenate([oracle.froxelize(t, g)[0].reshape(-1) for t, g in zip(tri_list, dims)])
    np.testing.assert_array_equal(to_np(occ), want)


def test_froxelize_tile_overflow_falls_back_to_full_scan():
    # more than 2048 triangles inside one 128x8x8 tile
    rng = np.random.default_rng(3)
    c = rng.uniform(1, 7, size=(2600, 1, 3)) * np.array([10.0, 1, 1])
    t = (c + rng.uniform(-0.7, 0.7, size=(2600, 3, 3))).astype(np.float32)
    dims = [(128, 16, 16)]
    tris, counts = upload_tris([t])
    occ = npvs.froxelize(tris, counts, dims)
    np.testing.assert_array_equal(to_np(occ), oracle.froxelize(t, dims[0])[0].reshape(-1))


def test_froxelize_parts_of_one_tile():
    # 300 to 2000 triangles in one tile are split over several 256-triangle parts
    rng = np.random.default_rng(4)
    for n in (300, 1100, 2000):
        c = rng.uniform(1, 7, size=(n, 1, 3)) * np.array([16.0, 1, 1])
        t = (c + rng.uniform(-0.9, 0.9, size=(n, 3, 3))).astype(np.float32)
        dims = [(256, 16, 8)]
        tris, counts = upload_tris([t])
        occ = npvs.froxelize(tris, counts, dims)
        np.testing.assert_array_equal(to_np(occ), oracle.froxelize(t, dims[0])[0].reshape(-1))


def test_froxelize_large_coordinates_and_ignored_count():
    # vertices in [1024, 2048) reach far outside the 256 x 256 x 128 grid and still mark exactly
    # the froxels they meet; 2048 and non-finite coordinates are ignored and counted on the device
    rng = np.random.default_rng(31)
    dims = [(256, 256, 128)]
    big = rng.uniform(-2047.9, 2047.9, size=(600, 3, 3))
    big[:, 0] = rng.uniform(0, 256, size=(600, 3)) * np.array([1.0, 1.0, 0.5])  # one vertex in the grid
    lattice = rng.integers(-2047, 2048, size=(200, 3, 3)).astype(np.float64)  # integer vertices
    bad = np.tile(np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0], [7.0, 8.0, 9.0]]), (7, 1, 1))
    bad[0, 1, 0] = 2048.0
    bad[1, 2, 2] = -2048.0
    bad[2, 0, 1] = np.nan
    bad[3, 1, 1] = np.inf
    bad[4, 0, 0] = -np.inf
    bad[5, 2, 0] = 3.0e38
    bad[6, 1, 2] = 2048.0001  # rounds to 2048 in float32: ignored
    edge = np.array([[[2047.9998, -2047.9998, 3.5], [-2047.9998, 2047.9998, 60.25], [128.5, 100.0, 2047.9998]]])
    t = np.concatenate([big, bad[:3], lattice, edge, bad[3:]]).astype(np.float32)
    want, ign = oracle.froxelize(t, dims[0])
    print(f"froxelize large coordinates T={len(t)} ignored={ign}", flush=True)
    assert ign == 7
    tris, counts = upload_tris([t])
    n_ign = torch.full((1,), -5, dtype=torch.int32, device=DEV)
    occ = npvs.froxelize(tris, counts, dims, n_ignored=n_ign)
    np.testing.assert_array_equal(to_np(occ), want.reshape(-1))
    assert int(n_ign.item()) == ign


def test_plan_counts_ignored_triangles():
    cfg = synth.config("tiny32")
    t = synth.scene_for(cfg)
    t = np.concatenate([t, np.full((3, 3, 3), np.nan, np.float32), np.full((2, 3, 3), 4096.0, np.float32)])
    tris, counts = upload_tris([t])
    plan = npvs.Plan(cfg.grids, counts, cfg.d, cfg.channels, npvs.NPVS_F32)
    plan.forward(tris)
    assert plan.counts()["n_tris_ignored"] == 5


def test_froxelize_empty_and_all_ignored():
    dims = [(64, 16, 16), (32, 32, 32)]
    tri_list = [np.zeros((0, 3, 3), np.float32), np.full((3, 3, 3), np.inf, np.float32)]
    tris, counts = upload_tris(tri_list)
    occ = torch.full((sum(g[0] * g[1] * g[2] // 8 for g in dims),), 0xAB, dtype=torch.uint8, device=DEV)
    npvs.froxelize(tris, counts, dims, occ=occ)
    assert not to_np(occ).any()


# ------------------------------------------------------------------------------- sites / rulebook
@pytest.mark.parametrize("d", [2, 4, 8, 16, 32])
def test_rulebook_bit_exact_batched(d):
    dims = [(64, 64, 64), (32, 32, 32), (128, 64, 32)]
    tri_list = [synth.box_scene(10 + i, g, 25, 2, 12) for i, g in enumerate(dims)]
    occ, rb = _frox_and_rb(tri_list, dims, d)
    ref = oracle_batch(tri_list, dims, d)
    c = rb.host_counts()
    assert c["n_sites"] == c["n_sites_needed"] == ref["n"]
    assert c["n_pairs"] == len(ref["pairs"])
    n = ref["n"]
    np.testing.assert_array_equal(to_np(rb.site_keys)[:n], ref["keys"])
    br = np.full(ref["total_blocks"], -1, np.int32)
    br[ref["keys"]] = np.arange(n)
    np.testing.assert_array_equal(to_np(rb.block_row), br)
    np.testing.assert_array_equal(to_np(rb.grid_rows), ref["grid_rows"])
    np.testing.assert_array_equal(to_np(rb.nbr)[:, :n], ref["nbr"])
    np.testing.assert_array_equal(to_np(rb.rb_off), ref["rb_off"])
    np.testing.assert_array_equal(to_np(rb.rb_pairs)[:len(ref["pairs"])], ref["pairs"])


def test_rulebook_city_and_capacity_overflow():
    cfg = synth.config("city256")
    t = synth.scene_for(cfg)
    occ, rb = _frox_and_rb([t], cfg.grids, 4)
    ref = oracle_batch([t], cfg.grids, 4)
    n = ref["n"]
    assert rb.host_counts()["n_sites"] == n
    np.testing.assert_array_equal(to_np(rb.site_keys)[:n], ref["keys"])
    np.testing.assert_array_equal(to_np(rb.nbr)[:, :n], ref["nbr"])
    np.testing.assert_array_equal(to_np(rb.rb_pairs)[:len(ref["pairs"])], ref["pairs"])
    # capacity below the site count: rows are dropped, the count reports what was needed
    small = npvs.build_rulebook(occ, cfg.grids, 4, cap=n // 2)
    c = small.host_counts()
    assert c["n_sites"] == n // 2 and c["n_sites_needed"] == n
    np.testing.assert_array_equal(to_np(small.site_keys), ref["keys"][:n // 2])


def test_empty_grid_has_no_sites():
    dims = [(32, 32, 32)]
    occ, rb = _frox_and_rb([np.zeros((0, 3, 3), np.float32)], dims, 2)
    c = rb.host_counts()
    assert c["n_sites"] == 0 and c["n_pairs"] == 0
    assert not to_np(rb.rb_off).any()
    assert (to_np(rb.block_row) == -1).all()


# ------------------------------------------------------------------------------- interleave
# (d, dims): the LDS tile holds 4096 elements, Kx = 4096 / d^3 blocks along x; (280, 8, 4) at
# d = 4 ends in a partial tile of 6 blocks, d = 16 fills one tile per block and d = 32 splits
# each block over 8 tiles of 128 rows.
@pytest.mark.parametrize("d,dims", [(1, (64, 32, 16)), (2, (64, 32, 16)), (4, (64, 32, 16)), (4, (280, 8, 4)),
                                    (8, (64, 32, 16)), (16, (96, 32, 16)), (32, (96, 64, 32))])
@pytest.mark.parametrize("dtype", [torch.uint8, torch.float16, torch.float32, torch.float64])
def test_dense_interleave_bit_exact(d, dims, dtype):
    g = torch.Generator().manual_seed(d)
    a = (torch.rand((dims[2], dims[1], dims[0]), generator=g) * 200).to(dtype)
    out = npvs.interleave(a.to(DEV), d)
    np.testing.assert_array_equal(to_np(out), oracle.interleave(a.numpy(), d))
    back = npvs.deinterleave(out, dims, d)
    np.testing.assert_array_equal(to_np(back), a.numpy())


def test_dense_interleave_logits_grid_full_size():
    """Dense g_d and its inverse on the float32 grid the benchmark times (256 x 256 x 128, 33.5 MB),
    every interleave factor, against a reshape-and-transpose of the same array (the index formula
    of g_d written with numpy), bit for bit."""
    dims = (256, 256, 128)
    a = np.random.default_rng(17).standard_normal((dims[2], dims[1], dims[0])).astype(np.float32)
    dev = torch.from_numpy(a).to(DEV)
    for d in (1, 2, 4, 8, 16, 32):
        want = a.reshape(dims[2] // d, d, dims[1] // d, d, dims[0] // d, d).transpose(0, 2, 4, 1, 3, 5)
        out = npvs.interleave(dev, d)
        np.testing.assert_array_equal(to_np(out), want.reshape(out.shape))
        np.testing.assert_array_equal(to_np(npvs.deinterleave(out, dims, d)), a)


@pytest.mark.parametrize("dt", [npvs.NPVS_F32, npvs.NPVS_BF16, npvs.NPVS_U8])
def test_sparse_gather_bit_exact(dt):
    dims = [(64, 64, 64), (32, 32, 32)]
    tri_list = [synth.box_scene(40 + i, g, 20, 2, 10) for i, g in enumerate(dims)]
    occ, rb = _frox_and_rb(tri_list, dims, 4, csr=False)
    X = npvs.gather_input(occ, rb, dt)
    ref = oracle_batch(tri_list, dims, 4)
    np.testing.assert_array_equal(to_np(X)[:ref["n"]], ref["X"])


@pytest.mark.parametrize("dt", [npvs.NPVS_F32, npvs.NPVS_BF16])
def test_sparse_gather_of_two_grids_in_one_pass(dt):
    """npvs_gather_input with a second bit grid (a training step's labels): the first output equals
    the oracle's interleave of the occupancy, the second the oracle's site labels of the second
    grid (u8), bit for bit, over two grids of different sizes."""
    dims = [(64, 64, 64), (32, 32, 32)]
    tri_list = [synth.box_scene(40 + i, g, 20, 2, 10) for i, g in enumerate(dims)]
    occ, rb = _frox_and_rb(tri_list, dims, 4, csr=False)
    mask = synth.label_mask_bits(9, (to_np(occ).size,))
    lab_bits = torch.from_numpy(to_np(occ) & mask).to(DEV)
    X, Y = npvs.gather_input(occ, rb, dt, bits2=lab_bits)
    ref = oracle_batch(tri_list, dims, 4)
    n = ref["n"]
    np.testing.assert_array_equal(to_np(X)[:n], ref["X"])
    # the oracle's labels: its own occupancy masked by the same bits, interleaved onto its sites
    lab_ref, o = [], 0
    for i, g in enumerate(dims):
        nb = g[0] * g[1] * g[2] // 8
        occ_i, _ = oracle.froxelize(tri_list[i], g)
        keys = oracle.active_sites(occ_i, g, 4)
        lab_ref.append(oracle.site_labels(occ_i.reshape(-1) & mask[o:o + nb], g, 4, keys))
        o += nb
    np.testing.assert_array_equal(to_np(Y)[:n], np.concatenate(lab_ref))


# ------------------------------------------------------------------------------- convolution
def _conv_case(cin, cout, d=2, seed=0, dims=((32, 32, 32), (64, 32, 32))):
    dims = [tuple(g) for g in dims]
    tri_list = [synth.box_scene(seed + i, g, 25, 2, 10) for i, g in enumerate(dims)]
    occ, rb = _frox_and_rb(tri_list, dims, d, csr=False)
    ref = oracle_batch(tri_list, dims, d)
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(rb.cap, cin)).astype(np.float32)
    W = (rng.normal(size=(27, cin, cout)) / np.sqrt(27 * cin)).astype(np.float32)
    b = rng.normal(size=cout).astype(np.float32)
    return rb, ref, X, W, b


@pytest.mark.parametrize("cin,cout,relu", [(8, 16, True), (16, 8, False), (64, 64, True), (24, 40, False)])
def test_conv_fwd_f32(cin, cout, relu):
    rb, ref, X, W, b = _conv_case(cin, cout)
    n = ref["n"]
    Wp = npvs.pack_weights(torch.from_numpy(W).to(DEV), npvs.NPVS_F32)
    Y = npvs.sparse_conv_fwd(torch.from_numpy(X).to(DEV), Wp, torch.from_numpy(b).to(DEV), cin, cout, rb,
                             npvs.NPVS_F32, relu)
    want = oracle.subm_conv(X[:n], W, b, ref["rb_off"], ref["pairs"], relu)
    tol = conv_tolerance(X[:n], W, ref["rb_off"], ref["pairs"])
    err = np.abs(to_np(Y)[:n] - want)
    assert (err <= tol).all(), err.max()


@pytest.mark.parametrize("cin,cout", [(8, 16), (16, 8), (64, 64), (32, 48), (512, 64)])
@pytest.mark.parametrize("variant_rows", [None])
def test_conv_fwd_bf16_mfma(cin, cout, variant_rows):
    d = 8 if cin == 512 else 2
    rb, ref, X, W, b = _conv_case(cin, cout, d=d, dims=((64, 64, 64), (32, 32, 32)))
    n = ref["n"]
    Xb = torch.from_numpy(X).to(DEV).to(torch.bfloat16)
    Wp = npvs.pack_weights(torch.from_numpy(W).to(DEV), npvs.NPVS_BF16)
    Y = npvs.sparse_conv_fwd(Xb, Wp, torch.from_numpy(b).to(DEV), cin, cout, rb, npvs.NPVS_BF16, True, out_f32=True)
    Xr, Wr = bf16_round(X[:n]), bf16_round(W)
    want = oracle.subm_conv(Xr, Wr, b, ref["rb_off"], ref["pairs"], True)
    tol = conv_tolerance(Xr, Wr, ref["rb_off"], ref["pairs"])
    err = np.abs(to_np(Y)[:n] - want)
    assert (err <= tol).all(), err.max()
    # bf16 output: the float32 result rounded to nearest even
    Yb = npvs.sparse_conv_fwd(Xb, Wp, torch.from_numpy(b).to(DEV), cin, cout, rb, npvs.NPVS_BF16, True)
    np.testing.assert_array_equal(to_np(Yb)[:n], to_np(Y[:n].to(torch.bfloat16)))


@pytest.mark.parametrize("variant", range(npvs.NPVS_CONV_VARIANTS))
@pytest.mark.parametrize("cin,cout,d", [(64, 64, 2), (16, 8, 2), (512, 64, 8)])
def test_conv_fwd_bf16_every_tile_shape(variant, cin, cout, d):
    rb, ref, X, W, b = _conv_case(cin, cout, d=d, dims=((64, 64, 64), (32, 32, 32)))
    n = ref["n"]
    Xb = torch.from_numpy(X).to(DEV).to(torch.bfloat16)
    Wp = npvs.pack_weights(torch.from_numpy(W).to(DEV), npvs.NPVS_BF16)
    Y = npvs.sparse_conv_fwd(Xb, Wp, torch.from_numpy(b).to(DEV), cin, cout, rb, npvs.NPVS_BF16, True, out_f32=True,
                             variant=variant)
    Xr, Wr = bf16_round(X[:n]), bf16_round(W)
    want = oracle.subm_conv(Xr, Wr, b, ref["rb_off"], ref["pairs"], True)
    tol = conv_tolerance(Xr, Wr, ref["rb_off"], ref["pairs"])
    err = np.abs(to_np(Y)[:n] - want)
    assert (err <= tol).all(), err.max()
    # deterministic run to run
    Y2 = npvs.sparse_conv_fwd(Xb, Wp, torch.from_numpy(b).to(DEV), cin, cout, rb, npvs.NPVS_BF16, True, out_f32=True,
                              variant=variant)
    np.testing.assert_array_equal(to_np(Y)[:n], to_np(Y2)[:n])


def test_plan_autotune_picks_valid_shapes_and_keeps_results():
    cfg = synth.config("city256")
    t = synth.scene_for(cfg)
    layers = synth.net_layers(cfg)
    tris, counts = upload_tris([t])
    plan = npvs.Plan(cfg.grids, counts, cfg.d, cfg.channels, npvs.NPVS_BF16)
    for li, (W, b) in enumerate(layers):
        plan.set_weights(li, torch.from_numpy(W).to(DEV), torch.from_numpy(b).to(DEV))
    v = plan.autotune(tris, reps=3)
    print("autotuned variants", v, flush=True)
    assert len(v) == 6 and all(0 <= x < npvs.NPVS_CONV_VARIANTS for x in v) and len(set(v[:5])) == 1
    pvs, logits = plan.forward(tris, want_logits=True)
    out = oracle.forward(t, cfg.grids[0], cfg.d, layers)
    got = to_np(logits).reshape(out["logits"].shape)
    act = np.isfinite(out["logits"])
    assert np.abs(got[act] - out["logits"][act]).max() < 0.1


def test_conv_weight_packing_flip_transpose_is_dgrad_weight():
    rb, ref, X, W, _ = _conv_case(16, 24)
    n = ref["n"]
    G = np.random.default_rng(1).normal(size=(rb.cap, 24)).astype(np.float32)
    Wt = npvs.pack_weights(torch.from_numpy(W).to(DEV), npvs.NPVS_F32, flip_transpose=True)
    dX = npvs.sparse_conv_fwd(torch.from_numpy(G).to(DEV), Wt, None, 24, 16, rb, npvs.NPVS_F32, False)
    want, _, _ = oracle.subm_conv_bwd(X[:n], W, ref["rb_off"], ref["pairs"], np.ones((n, 24)), G[:n], relu=False)
    np.testing.assert_allclose(to_np(dX)[:n], want, rtol=0, atol=2e-5)


@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
def test_batched_packing_equals_single_packings(dtype):
    rng = np.random.default_rng(7)
    shapes = [(8, 16), (64, 64), (24, 40), (512, 64), (64, 8)]
    Ws = [torch.from_numpy(rng.normal(size=(27, ci, co)).astype(np.float32)).to(DEV) for ci, co in shapes]
    items, want = [], []
    for W in Ws:
        for flip in (False, True):
            ref = npvs.pack_weights(W, dtype, flip_transpose=flip)
            items.append((W, torch.full_like(ref, 0xAB), flip))
            want.append(ref)
    npvs.pack_weights_batch(items, dtype)
    for (_, got, _), ref in zip(items, want):
        np.testing.assert_array_equal(to_np(got), to_np(ref))


def test_conv_rows_beyond_n_untouched_and_deterministic():
    rb, ref, X, W, b = _conv_case(64, 64)
    n = ref["n"]
    Wp = npvs.pack_weights(torch.from_numpy(W).to(DEV), npvs.NPVS_BF16)
    Xb = torch.from_numpy(X).to(DEV).to(torch.bfloat16)
    Y1 = torch.full((rb.cap, 64), 7.0, device=DEV)
    npvs.sparse_conv_fwd(Xb, Wp, None, 64, 64, rb, npvs.NPVS_BF16, False, out_f32=True, out=Y1)
    Y2 = npvs.sparse_conv_fwd(Xb, Wp, None, 64, 64, rb, npvs.NPVS_BF16, False, out_f32=True)
    assert (to_np(Y1)[n:] == 7.0).all()
    np.testing.assert_array_equal(to_np(Y1)[:n], to_np(Y2)[:n])


# ------------------------------------------------------------------------------- output
def test_deinterleave_threshold_exact():
    dims = [(64, 32, 32), (32, 32, 32)]
    tri_list = [synth.box_scene(60 + i, g, 20, 2, 10) for i, g in enumerate(dims)]
    occ, rb = _frox_and_rb(tri_list, dims, 2, csr=False)
    ref = oracle_batch(tri_list, dims, 2)
    n = ref["n"]
    Y = np.random.default_rng(0).normal(size=(rb.cap, 8)).astype(np.float32)
    Y[:n:7] = 0.0  # exact zeros are visible (tau = 0.5 <=> logit >= 0)
    pvs, logits = npvs.deinterleave_threshold(torch.from_numpy(Y).to(DEV), rb, occ, want_logits=True)
    wp, wl = [], []
    for b, g in enumerate(dims):
        r0, r1 = ref["grid_rows"][b], ref["grid_rows"][b + 1]
        keys = ref["keys"][r0:r1] - (0 if b == 0 else (dims[0][0] // 2) * (dims[0][1] // 2) * (dims[0][2] // 2))
        o = oracle.froxelize(tri_list[b], g)[0]
        l, p = oracle.deinterleave_threshold(Y[r0:r1], keys, o, g, 2)
        wp.append(p.reshape(-1))
        wl.append(l.reshape(-1))
    np.testing.assert_array_equal(to_np(pvs), np.concatenate(wp))
    np.testing.assert_array_equal(to_np(logits), np.concatenate(wl).astype(np.float32))


# ------------------------------------------------------------------------------- whole network
def _net_fwd_gpu(occ, rb, layers, dtype):
    X = npvs.gather_input(occ, rb, dtype)
    for li, (W, b) in enumerate(layers):
        last = li == len(layers) - 1
        Wp = npvs.pack_weights(torch.from_numpy(W).to(DEV), dtype)
        X = npvs.sparse_conv_fwd(X, Wp, torch.from_numpy(b).to(DEV), W.shape[1], W.shape[2], rb, dtype,
                                 relu=not last, out_f32=last)
    return X


@pytest.mark.parametrize("name", ["tiny32", "city256"])
def test_network_f32_logits_within_1e5_of_fp64_oracle(name):
    cfg = synth.config(name)
    t = synth.scene_for(cfg)
    layers = synth.net_layers(cfg, bias_std=0.05)
    occ, rb = _frox_and_rb([t], cfg.grids, cfg.d, csr=False)
    Y = _net_fwd_gpu(occ, rb, layers, npvs.NPVS_F32)
    out = oracle.forward(t, cfg.grids[0], cfg.d, layers)
    n = len(out["keys"])
    err = np.abs(to_np(Y)[:n] - out["acts"][-1]).max()
    print(f"{name}: n_sites={n} max|logit err|={err:.3e}", flush=True)
    assert err <= 1e-5
    pvs, _ = npvs.deinterleave_threshold(Y, rb, occ)
    # bits agree wherever the oracle's logit is farther than the error bound from the threshold
    got = np.unpackbits(to_np(pvs).reshape(out["pvs"].shape), axis=-1, bitorder="little")
    want = oracle.unpack(out["pvs"])
    near = np.abs(np.nan_to_num(out["logits"], neginf=-1e9)) <= 1e-5
    assert ((got == want) | near).all()


def test_city256_bf16_layers_at_the_rounding_points():
    """Every layer of the city network, forward and backward, on the oracle's own BF16 operands
    (its rounded weights and its bfloat16 activations of the same layer), against rigorous
    bounds: the float32 sums of exact products lie within gamma_n sum |terms| of the FP64 values,
    so each hidden output's bfloat16 bits must equal the oracle's rounding wherever the FP64
    value is farther than that from a rounding boundary, and lie between the two neighbours
    where it is not; logits, dX, dW and db lie within their gamma_n bounds."""
    cfg = synth.config("city256")
    t = synth.scene_for(cfg)
    layers = synth.net_layers(cfg, bias_std=0.05)
    occ, rb = _frox_and_rb([t], cfg.grids, cfg.d, csr=True)
    emu = oracle.forward_bf16(t, cfg.grids[0], cfg.d, layers)
    n = len(emu["keys"])
    assert rb.host_counts()["n_sites"] == n
    rb_off, pairs = emu["rb_off"], emu["pairs"]
    up = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(DEV).to(torch.bfloat16)
    rng = np.random.default_rng(17)
    dY = (rng.standard_normal((n, layers[-1][0].shape[2])) * 1e-3).astype(np.float32).astype(np.float64)
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        last = li == len(layers) - 1
        cin, cout = W.shape[1], W.shape[2]
        X = torch.zeros((rb.cap, cin), dtype=torch.bfloat16, device=DEV)
        X[:n] = up(emu["acts"][li])
        Wd = torch.from_numpy(W).to(DEV)
        Y = npvs.sparse_conv_fwd(X, npvs.pack_weights(Wd, npvs.NPVS_BF16), torch.from_numpy(b).to(DEV), cin, cout,
                                 rb, npvs.NPVS_BF16, relu=not last, out_f32=last)
        r = oracle.bf16_layer_bound(emu["acts"][li], emu["Wb"][li], b, rb_off, pairs, relu=not last)
        got = to_np(Y)[:n].astype(np.float64)
        inside = (got >= r["lo"]) & (got <= r["hi"])
        exact = (r["lo"] == r["hi"])
        print(f"layer {li}: outputs inside the bound {inside.mean():.6f}, pinned to one value {exact.mean():.4f}",
              flush=True)
        assert inside.all(), (li, np.abs(got - r["out"]).max())
        if not last:
            assert np.array_equal(got[exact], r["out"][exact])
        # backward of the same layer on the oracle's operands (dY: float32 values)
        Yo = torch.zeros((rb.cap, cout), dtype=torch.bfloat16, device=DEV)  # the ReLU mask's operand
        if not last:
            Yo[:n] = up(emu["acts"][li + 1])
        dYd = torch.zeros((rb.cap, cout), dtype=torch.float32, device=DEV)
        dYd[:n] = torch.from_numpy(dY.astype(np.float32)).to(DEV)
        Wt = npvs.pack_weights(Wd, npvs.NPVS_BF16, flip_transpose=True)
        dX, dW, db = npvs.sparse_conv_bwd(X, Wt, cin, cout, Yo, dYd, rb, npvs.NPVS_BF16, relu=not last,
                                          want_dx=li > 0)
        rb_ = oracle.bf16_layer_bwd_bound(emu["acts"][li], emu["Wb"][li], rb_off, pairs, emu["acts"][li + 1], dY,
                                          relu=not last, want_dx=li > 0)
        for nm, g, ref, bnd in (("dW", dW, rb_["dW"], rb_["E_dW"]), ("db", db, rb_["db"], rb_["E_db"])):
            e = np.abs(to_np(g).astype(np.float64) - ref)
            print(f"layer {li} {nm}: max err / bound {np.max(e / np.maximum(bnd, 1e-300)):.3e}", flush=True)
            assert (e <= bnd).all(), (li, nm)
        if li > 0:
            e = np.abs(to_np(dX)[:n].astype(np.float64) - rb_["dX"])
            assert (e <= rb_["E_dX"]).all(), li
            dY = rb_["dX"].astype(np.float32).astype(np.float64)


def test_network_bf16_c2_end_to_end():
    """C2: the city frame through the BF16 network against the oracle's BF16 network (same
    rounding points), within DRIFT_FACTOR times the oracle's own drift between two evaluation
    orders; the FP32 path within 1e-5 of FP64.  The PVS flips against the FP64 oracle are
    counted by oracle.metrics: the target (at most 0.1 % of thresholded froxels) is asserted over
    the froxels that receive a logit and go through the threshold (the active blocks); the rate
    over the occupied froxels is printed beside it."""
    cfg = synth.config("city256")
    t = synth.scene_for(cfg)
    layers = synth.net_layers(cfg)
    occ, rb = _frox_and_rb([t], cfg.grids, cfg.d, csr=False)
    Yb = _net_fwd_gpu(occ, rb, layers, npvs.NPVS_BF16)
    Yf = _net_fwd_gpu(occ, rb, layers, npvs.NPVS_F32)
    ref = bf16_reference(t, cfg.grids[0], cfg.d, layers)
    emu, o32 = ref["emu"], ref["o32"]
    out = oracle.forward(t, cfg.grids[0], cfg.d, layers, occ=emu["occ"])
    n = len(emu["keys"])
    tol = drift_tol(emu["acts"][-1], o32["acts"][-1], ref["logit_floor"])
    err_b = np.abs(to_np(Yb)[:n] - emu["acts"][-1])
    print(f"bf16 vs the oracle's BF16 network: max|err| {err_b.max():.3e}, tolerance {tol:.3e}; "
          f"vs FP64 {np.abs(to_np(Yb)[:n] - out['acts'][-1]).max():.3e}", flush=True)
    assert err_b.max() <= tol
    assert np.abs(to_np(Yf)[:n] - out["acts"][-1]).max() <= 1e-5
    pb, _ = npvs.deinterleave_threshold(Yb, rb, occ)
    active = oracle.active_froxels(emu["occ"], cfg.grids[0], cfg.d).reshape(-1)
    occ_o = emu["occ"].reshape(-1)
    m = oracle.metrics(out["pvs"].reshape(-1), to_np(pb).reshape(-1), occ_o, active)
    mb = oracle.metrics(emu["pvs"].reshape(-1), to_np(pb).reshape(-1), occ_o, active)
    print(f"bf16 vs FP64 oracle: flips {m['flips']}, over active-block froxels {m['flip_rate_active']:.5%}, "
          f"over occupied {m['flip_rate_occupied']:.5%}, over all {m['flip_rate_all']:.6%}; missing geometry "
          f"{m['missing_geometry']:.5%}, FPR {m['fpr']:.5%}; flips against the oracle's BF16 network "
          f"{mb['flips']}", flush=True)
    assert m["flip_rate_active"] <= 1e-3


# ------------------------------------------------------------------------------- plan / graph
def test_plan_forward_matches_staged_calls_and_graph_replays():
    cfg = synth.config("tiny32")
    t = synth.scene_for(cfg)
    layers = synth.net_layers(cfg, bias_std=0.05)
    for dtype in (npvs.NPVS_F32, npvs.NPVS_BF16):
        tris, counts = upload_tris([t])
        plan = npvs.Plan(cfg.grids, counts, cfg.d, cfg.channels, dtype)
        for li, (W, b) in enumerate(layers):
            plan.set_weights(li, torch.from_numpy(W).to(DEV), torch.from_numpy(b).to(DEV))
        pvs, logits = plan.forward(tris, want_logits=True)
        occ, rb = _frox_and_rb([t], cfg.grids, cfg.d, csr=False)
        Y = _net_fwd_gpu(occ, rb, layers, dtype)
        p2, l2 = npvs.deinterleave_threshold(Y, rb, occ, want_logits=True)
        np.testing.assert_array_equal(to_np(pvs), to_np(p2))
        np.testing.assert_array_equal(to_np(logits), to_np(l2))
        assert plan.counts()["n_sites"] == rb.host_counts()["n_sites"]
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            gp, gl = plan.capture(tris, want_logits=True)
            for rep in range(3):
                gp.fill_(0xFF)
                gl.fill_(123.0)
                plan.replay()
                torch.cuda.synchronize()
                np.testing.assert_array_equal(to_np(gp), to_np(pvs))
                np.testing.assert_array_equal(to_np(gl), to_np(logits))
                _ = _net_fwd_gpu(occ, rb, layers[:1], dtype)  # eager work between replays
        torch.cuda.synchronize()


def test_maximum_grid_extent_bit_exact():
    """Grids 1024 froxels long (the largest extent) with triangles spanning the whole x range:
    froxelize, the rulebook at d = 8 and culling against a random PVS, bit for bit."""
    rng = np.random.default_rng(77)
    dims = [(1024, 16, 8), (8, 1024, 8)]
    tri_list = []
    for g in dims:
        hi = np.array(g, np.float64)
        t = []
        for i in range(120):
            if i % 2 == 0:  # long slivers across the long axis
                a = rng.uniform(0, hi, size=3)
                b = rng.uniform(0, hi, size=3)
                ax = int(np.argmax(hi))
                a[ax], b[ax] = rng.uniform(0, 4), rng.uniform(hi[ax] - 4, hi[ax])
                t.append(np.stack([a, b, b + rng.uniform(-0.5, 0.5, 3)]))
            else:
                t.append(rng.uniform(-1, hi + 1, size=(3, 3)))
        tri_list.append(np.asarray(t, np.float32))
    tris, counts = upload_tris(tri_list)
    occ = npvs.froxelize(tris, counts, dims)
    want = [oracle.froxelize(t, g)[0] for t, g in zip(tri_list, dims)]
    np.testing.assert_array_equal(to_np(occ), np.concatenate([w.reshape(-1) for w in want]))
    rb = npvs.build_rulebook(occ, dims, 8, csr=True)
    ref = oracle_batch(tri_list, dims, 8)
    n = ref["n"]
    assert rb.host_counts()["n_sites"] == n
    np.testing.assert_array_equal(to_np(rb.site_keys)[:n], ref["keys"])
    np.testing.assert_array_equal(to_np(rb.rb_pairs)[:len(ref["pairs"])], ref["pairs"])
    pvs = [np.packbits((rng.random((g[2], g[1], g[0] // 8, 8)) < 0.01).astype(np.uint8), axis=-1,
                       bitorder="little").reshape(g[2], g[1], g[0] // 8) for g in dims]
    vis = npvs.visible_triangles(tris, counts, dims, torch.from_numpy(np.concatenate([p.reshape(-1) for p in pvs])).to(DEV))
    np.testing.assert_array_equal(to_np(vis), np.concatenate([oracle.visible_triangles(t, g, p)
                                                              for t, g, p in zip(tri_list, dims, pvs)]))
