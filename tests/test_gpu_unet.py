"""GPU parity of the two-level U-Net pieces (level maps, strided and inverse convolutions, the
whole encoder/decoder forward) against the oracle, through the C ABI."""
import functools

import numpy as np
import pytest
import torch

import oracle
import paper_2509_24677_amd as npvs
import synth
from gpu_util import DEV, bf16_round, drift_tol, to_np, upload_tris
from paper_2509_24677_amd.unet import UNet, unet_pvs

pytestmark = pytest.mark.gpu


def _grids(dims, seeds):
    tri_list = [synth.box_scene(s, g, 20, 2, 8) for s, g in zip(seeds, dims)]
    tris, counts = upload_tris(tri_list)
    return tri_list, npvs.froxelize(tris, counts, dims)


def _oracle_levels(tri_list, dims, d):
    """Per-grid oracle level maps in the batch's row numbering: children [8][n1], parent [n0]
    (8 * level-1 row + child index), n0, n1."""
    ch, par, n0, n1 = [], [], 0, 0
    for t, g in zip(tri_list, dims):
        occ, _ = oracle.froxelize(t, g)
        k0, k1 = oracle.active_sites(occ, g, d), oracle.active_sites(occ, g, 2 * d)
        c, p, kid = oracle.level_maps(k0, k1, (g[0] // d, g[1] // d, g[2] // d))
        ch.append(np.where(c >= 0, c + n0, -1))
        par.append((p + n1) * 8 + kid)
        n0 += len(k0)
        n1 += len(k1)
    return np.concatenate(ch, axis=1), np.concatenate(par), n0, n1


@pytest.mark.parametrize("d", [2, 4])
def test_level_maps_bit_exact(d):
    dims = [(64, 32, 32), (32, 32, 16), (128, 64, 32)]
    tri_list, occ = _grids(dims, [5, 6, 7])
    lv = npvs.build_levels(occ, dims, d)
    ch, par, n0, n1 = _oracle_levels(tri_list, dims, d)
    assert lv.rb0.host_counts()["n_sites"] == n0 and lv.rb1.host_counts()["n_sites"] == n1
    assert 0 < n1 < n0
    got_c, got_p = to_np(lv.children), to_np(lv.parent)
    np.testing.assert_array_equal(got_c[:, :n1], ch)
    assert (got_c[:, n1:] == -1).all()
    np.testing.assert_array_equal(got_p[:n0], par)
    assert (got_p[n0:] == -1).all()


@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
@pytest.mark.parametrize("up", [False, True])
@pytest.mark.parametrize("cin,cout", [(64, 64), (64, 96), (8, 24), (160, 16)])
def test_strided_conv_matches_oracle(dtype, up, cin, cout):
    dims, d = [(64, 32, 32), (32, 32, 16)], 4
    tri_list, occ = _grids(dims, [3, 4])
    lv = npvs.build_levels(occ, dims, d)
    ch, par, n0, n1 = _oracle_levels(tri_list, dims, d)
    rng = np.random.default_rng(cin * 1000 + cout + 7 * up)
    cap_in = lv.rb1.cap if up else lv.rb0.cap
    X = rng.normal(size=(cap_in, cin)).astype(np.float32)
    W = (rng.normal(size=(8, cin, cout)) / np.sqrt(8 * cin)).astype(np.float32)
    b = rng.normal(0, 0.1, size=cout).astype(np.float32)
    Xt = torch.from_numpy(X).to(DEV)
    if dtype == npvs.NPVS_BF16:
        Xt, Xr, Wr = Xt.to(torch.bfloat16), bf16_round(X), bf16_round(W)
    else:
        Xr, Wr = X.astype(np.float64), W.astype(np.float64)
    Wp = npvs.pack_weights_k(torch.from_numpy(W).to(DEV), dtype)
    bt = torch.from_numpy(b).to(DEV)
    Y = npvs.strided_conv_fwd(Xt, Wp, bt, cin, cout, lv, up, dtype, relu=True, out_f32=True)
    if up:
        want = oracle.inverse_up(Xr[:n1], par // 8, par % 8, Wr, b, True)
        mag = oracle.inverse_up(np.abs(Xr[:n1]), par // 8, par % 8, np.abs(Wr), np.zeros(cout), False)
        n_out = n0
    else:
        want = oracle.strided_down(Xr[:n0], ch, Wr, b, True)
        mag = oracle.strided_down(np.abs(Xr[:n0]), ch, np.abs(Wr), np.zeros(cout), False)
        n_out = n1
    tol = 2 * 8 * cin * 2.0 ** -24 * (mag + np.abs(b)) + 1e-30  # float32 accumulation bound
    err = np.abs(to_np(Y)[:n_out] - want)
    assert (err <= tol).all(), (err.max(), tol.max())
    if dtype == npvs.NPVS_BF16:  # bf16 output: the float32 result rounded to nearest even
        Yb = npvs.strided_conv_fwd(Xt, Wp, bt, cin, cout, lv, up, dtype, relu=True)
        np.testing.assert_array_equal(to_np(Yb)[:n_out], to_np(Y[:n_out].to(torch.bfloat16)))


def test_concat_channels_bit_exact():
    dims = [(32, 32, 32)]
    _, occ = _grids(dims, [9])
    rb = npvs.build_rulebook(occ, dims, 2)
    n = rb.host_counts()["n_sites"]
    A = torch.randn((rb.cap, 24), device=DEV).to(torch.bfloat16)
    B = torch.randn((rb.cap, 16), device=DEV).to(torch.bfloat16)
    Y = npvs.concat_channels(A, B, rb)
    np.testing.assert_array_equal(to_np(Y)[:n], np.concatenate([to_np(A)[:n], to_np(B)[:n]], axis=1))


@functools.lru_cache(maxsize=None)
def _oracle_unet(name, seed, E, Dc):
    cfg = synth.config(name)
    t = synth.scene_for(cfg)
    params = synth.unet_params(seed, cfg.d, E=E, Dc=Dc)
    return cfg, t, params, oracle.unet_forward(t, cfg.grids[0], cfg.d, params)


@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
@pytest.mark.parametrize("name,E,Dc", [("tiny32", 16, 24), ("city256", 64, 96)])
def test_unet_forward_matches_oracle(name, E, Dc, dtype):
    cfg, t, params, out = _oracle_unet(name, 11, E, Dc)
    net = UNet(params, cfg.d, dtype)
    tris, counts = upload_tris([t])
    pvs, logits, lv, occ = unet_pvs(net, tris, counts, cfg.grids)
    n = len(out["keys0"])
    assert lv.rb0.host_counts()["n_sites"] == n and lv.rb1.host_counts()["n_sites"] == len(out["keys1"])
    np.testing.assert_array_equal(to_np(occ).reshape(-1), out["occ"].reshape(-1))
    if dtype == npvs.NPVS_F32:
        ref, lg, tol = out["acts"]["Y"], out["logits"].reshape(-1), 1e-4
        pw = np.unpackbits(out["pvs"].reshape(-1), bitorder="little")
    else:  # the oracle's BF16 U-Net, within DRIFT_FACTOR times its own drift between two orders
        emu = oracle.unet_forward_bf16(t, cfg.grids[0], cfg.d, params, occ=out["occ"])
        o32 = oracle.unet_forward_bf16(t, cfg.grids[0], cfg.d, params, occ=out["occ"], accum="f32")
        ref, lg = emu["acts"]["Y"], emu["logits"].reshape(-1)
        tol = drift_tol(ref, o32["acts"]["Y"])
        pw = np.unpackbits(emu["pvs"].reshape(-1), bitorder="little")
    err = np.abs(to_np(logits)[:n] - ref).max()
    print(f"{name} dtype {dtype}: n0 {n} n1 {len(out['keys1'])} max |logit err| {err:.3e}, tolerance {tol:.3e}",
          flush=True)
    assert err <= tol, err
    # the PVS bits agree wherever the reference logit is clear of the threshold by the tolerance
    safe = np.abs(lg) > tol
    pv = np.unpackbits(to_np(pvs).reshape(-1), bitorder="little")
    np.testing.assert_array_equal(pv[safe], pw[safe])


def test_unet_forward_on_an_empty_grid():
    cfg = synth.config("tiny32")
    net = UNet(synth.unet_params(11, cfg.d, E=16, Dc=24), cfg.d, npvs.NPVS_BF16)
    tris, counts = upload_tris([np.zeros((0, 3, 3), np.float32)])
    pvs, logits, lv, occ = unet_pvs(net, tris, counts, cfg.grids)
    assert lv.rb0.host_counts()["n_sites"] == 0 and lv.rb1.host_counts()["n_sites"] == 0
    assert not to_np(pvs).any()


@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
@pytest.mark.parametrize("up", [False, True])
@pytest.mark.parametrize("cin,cout", [(64, 96), (24, 16), (136, 72)])
def test_strided_conv_bwd_matches_oracle(dtype, up, cin, cout):
    """dX, dW and db of the strided convolution and of its inverse (ReLU) against the oracle on the
    same operands (bfloat16-representable X, Y, W; the BF16 products take dZ rounded to bfloat16,
    the bias gradient the float32 dZ); also deterministic."""
    dims, d = [(64, 32, 32), (32, 32, 16)], 4
    tri_list, occ = _grids(dims, [3, 4])
    lv = npvs.build_levels(occ, dims, d)
    ch, par, n0, n1 = _oracle_levels(tri_list, dims, d)
    rng = np.random.default_rng(cin * 1000 + cout + 7 * up)
    cap_in, cap_out = (lv.rb1.cap, lv.rb0.cap) if up else (lv.rb0.cap, lv.rb1.cap)
    n_in, n_out = (n1, n0) if up else (n0, n1)
    X = bf16_round(rng.normal(size=(cap_in, cin))).astype(np.float32)
    Y = bf16_round(rng.normal(size=(cap_out, cout))).astype(np.float32)
    dY = rng.normal(size=(cap_out, cout)).astype(np.float32)
    W = bf16_round(rng.normal(size=(8, cin, cout)) / np.sqrt(8 * cin)).astype(np.float32)
    tdt = torch.float32 if dtype == npvs.NPVS_F32 else torch.bfloat16
    Wt = npvs.pack_weights_k(torch.from_numpy(W).to(DEV), dtype, transpose=True)
    args = (torch.from_numpy(X).to(DEV).to(tdt), Wt, cin, cout, torch.from_numpy(Y).to(DEV).to(tdt),
            torch.from_numpy(dY).to(DEV), lv, up, dtype)
    dX, dW, db = npvs.strided_conv_bwd(*args)
    dX, dW, db = to_np(dX)[:n_in], to_np(dW), to_np(db)
    dZ = np.where(Y[:n_out] > 0, dY[:n_out], np.float32(0)).astype(np.float64)
    dZm = dZ if dtype == npvs.NPVS_F32 else bf16_round(dZ)
    if up:
        bwd = lambda x, w, g: oracle.inverse_up_bwd(x, par // 8, par % 8, w, Y[:n_out], g, relu=False)
    else:
        bwd = lambda x, w, g: oracle.strided_down_bwd(x, ch, w, Y[:n_out], g, relu=False)
    rX, rW, rb_ = bwd(X[:n_in], W, dZm)
    aX, aW, _ = bwd(np.abs(X[:n_in]), np.abs(W), np.abs(dZm))
    u = 2.0 ** -24
    assert (np.abs(dW - rW) <= 2e-5 * aW + 1e-30).all(), np.abs(dW - rW).max()
    assert (np.abs(dX - rX) <= 2 * 8 * cout * u * aX + 1e-30).all(), np.abs(dX - rX).max()
    _, _, rdb = bwd(X[:n_in], W, dZ)
    assert (np.abs(db - rdb) <= 1e-5 * np.abs(dZ).sum(0) + 1e-30).all()
    dX2, dW2, db2 = npvs.strided_conv_bwd(*args)
    np.testing.assert_array_equal(to_np(dW2), dW)
    np.testing.assert_array_equal(to_np(db2), db)
    np.testing.assert_array_equal(to_np(dX2)[:n_in], dX)


def test_concat_channels_bwd_splits_and_adds():
    dims, d = [(64, 32, 32)], 4
    _, occ = _grids(dims, [8])
    rb = npvs.build_rulebook(occ, dims, d)
    n = rb.host_counts()["n_sites"]
    g = torch.Generator(device=DEV).manual_seed(1)
    dY = torch.randn((rb.cap, 40), device=DEV, generator=g)
    add = torch.randn((rb.cap, 16), device=DEV, generator=g)
    dA, dB = npvs.concat_channels_bwd(dY, 24, 16, rb, add_b=add)
    np.testing.assert_array_equal(to_np(dA)[:n], to_np(dY)[:n, :24])
    np.testing.assert_array_equal(to_np(dB)[:n], to_np(dY)[:n, 24:] + to_np(add)[:n])
    _, dB = npvs.concat_channels_bwd(dY, 24, 16, rb, want_a=False)
    np.testing.assert_array_equal(to_np(dB)[:n], to_np(dY)[:n, 24:])


@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
def test_unet_backward_matches_oracle(dtype):
    """Gradients of BCE + repulsive visibility loss through the whole two-level U-Net.  FP32
    against the oracle's FP64 backward: max error 1e-4 of the largest gradient.  BF16 against the
    oracle's BF16 U-Net (unet_forward_bf16 / unet_backward_bf16, the same rounding points, labels
    from the oracle's occupancy): every dW and db within DRIFT_FACTOR times the oracle's own
    drift between two evaluation orders."""
    cfg = synth.config("tiny32")
    t = synth.scene_for(cfg)
    g, d = cfg.grids[0], 2
    params = synth.unet_params(6, d, E=16, Dc=24)
    tris, counts = upload_tris([t])
    occ = npvs.froxelize(tris, counts, cfg.grids)
    lv = npvs.build_levels(occ, cfg.grids, d, csr=True)
    lab_bits = torch.from_numpy(to_np(occ) & synth.label_mask_bits(5, (to_np(occ).size,))).to(DEV)
    labels = npvs.gather_input(lab_bits, lv.rb0, npvs.NPVS_U8)
    net = UNet(params, d, dtype)
    saved = {}
    logits = net.forward(npvs.gather_input(occ, lv.rb0, dtype), lv, saved=saved)
    _, dl = npvs.loss(logits, labels, lv.rb0)
    grads = net.backward(saved, logits, dl, lv)
    torch.cuda.synchronize()
    if dtype == npvs.NPVS_F32:
        p64 = {k: [(W.astype(np.float64), b.astype(np.float64)) for W, b in v] for k, v in params.items()}
        out = oracle.unet_forward(t, g, d, p64, want_logits=False)
        o = out["occ"].reshape(-1)
        ref_lab = oracle.site_labels(o & synth.label_mask_bits(5, (o.size,)), g, d, out["keys0"])
        ref, _ = oracle.unet_backward(out, p64, oracle.loss(out["acts"]["Y"], ref_lab)["grad"])
        alt = None
    else:
        out = oracle.unet_forward_bf16(t, g, d, params)
        o32 = oracle.unet_forward_bf16(t, g, d, params, occ=out["occ"], accum="f32")
        o = out["occ"].reshape(-1)
        ref_lab = oracle.site_labels(o & synth.label_mask_bits(5, (o.size,)), g, d, out["keys0"])
        ref = oracle.unet_backward_bf16(out, oracle.loss(out["acts"]["Y"], ref_lab)["grad"])
        dl32 = oracle.loss(o32["acts"]["Y"], ref_lab)["grad"].astype(np.float32).astype(np.float64)
        alt = oracle.unet_backward_bf16(o32, dl32, accum="f32")
    for st in ref:
        for i, ((dW, db), (rW, rdb)) in enumerate(zip(grads[st], ref[st])):
            for j, (a, b, nm) in enumerate(((to_np(dW), rW, "dW"), (to_np(db), rdb, "db"))):
                scale = np.abs(b).max()
                err = np.abs(a - b).max()
                assert scale > 0
                if dtype == npvs.NPVS_F32:
                    print(f"fp32 {st}[{i}] {nm}: max rel err {err / scale:.3e}", flush=True)
                    assert err <= 1e-4 * scale, (st, i, nm)
                else:
                    tol = drift_tol(b, alt[st][i][j])
                    print(f"bf16 {st}[{i}] {nm}: max err {err:.3e}, tolerance {tol:.3e} ({tol / scale:.2e} of the "
                          f"largest entry)", flush=True)
                    assert tol > 0 and err <= tol, (st, i, nm)


@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
def test_unet_batched_weight_gradients_equal_per_layer(dtype):
    """The 3^3 layers' weight gradients deferred and batched per level (at the single-layer slice
    count) give the per-layer side-stream backward's gradients bit for bit."""
    cfg = synth.config("tiny32")
    t = synth.scene_for(cfg)
    params = synth.unet_params(6, 2, E=16, Dc=24)
    tris, counts = upload_tris([t])
    occ = npvs.froxelize(tris, counts, cfg.grids)
    lv = npvs.build_levels(occ, cfg.grids, 2, csr=True)
    lab_bits = torch.from_numpy(to_np(occ) & synth.label_mask_bits(5, (to_np(occ).size,))).to(DEV)
    labels = npvs.gather_input(lab_bits, lv.rb0, npvs.NPVS_U8)
    net = UNet(params, 2, dtype)
    saved = {}
    logits = net.forward(npvs.gather_input(occ, lv.rb0, dtype), lv, saved=saved)
    _, dl = npvs.loss(logits, labels, lv.rb0)
    per_layer = net.backward(saved, logits, dl, lv, overlap=True)
    batched = net.backward(saved, logits, dl, lv, batch_wgrad=True, wgrad_slices=16)
    torch.cuda.synchronize()
    for st in per_layer:
        for (a, b), (c, e) in zip(per_layer[st], batched[st]):
            np.testing.assert_array_equal(to_np(a), to_np(c))
            np.testing.assert_array_equal(to_np(b), to_np(e))


def test_unet_backward_on_an_empty_grid_is_zero():
    """No triangles: no active sites on either level; every gradient is zero (the strided layers'
    pair lists are empty, every slice partial is zero)."""
    cfg = synth.config("tiny32")
    d = 2
    params = synth.unet_params(6, d, E=16, Dc=24)
    tris, counts = upload_tris([np.zeros((0, 3, 3), np.float32)])
    occ = npvs.froxelize(tris, counts, cfg.grids)
    lv = npvs.build_levels(occ, cfg.grids, d, csr=True)
    assert lv.rb0.host_counts()["n_sites"] == 0 and lv.rb1.host_counts()["n_sites"] == 0
    net = UNet(params, d, npvs.NPVS_BF16)
    saved = {}
    logits = net.forward(npvs.gather_input(occ, lv.rb0, npvs.NPVS_BF16), lv, saved=saved)
    dl = torch.zeros_like(logits)
    grads = net.backward(saved, logits, dl, lv)
    for st, layer_grads in grads.items():
        for dW, db in layer_grads:
            assert not to_np(dW).any() and not to_np(db).any(), st
