"""GPU parity of the training path (loss, backward, Adam) against the oracle, through the C ABI,
and the backward against FP64 finite differences of the oracle's forward."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_24677_amd as npvs
import synth
from gpu_util import DEV, bf16_reference, drift_tol, oracle_batch, to_np, upload_tris
from paper_2509_24677_amd.train import Network

pytestmark = pytest.mark.gpu


def _oracle_labels(out, dims, d, label_seed=5):
    """The oracle's labels: the same seeded mask over the oracle's own occupancy, interleaved by
    the oracle (no GPU output enters the reference)."""
    occ = out["occ"].reshape(-1)
    return oracle.site_labels(occ & synth.label_mask_bits(label_seed, (occ.size,)), dims, d, out["keys"])


def _setup(name="tiny32", layers=None, label_seed=5):
    cfg = synth.config(name)
    t = synth.scene_for(cfg)
    layers = layers or synth.net_layers(cfg, bias_std=0.05)
    tris, counts = upload_tris([t])
    occ = npvs.froxelize(tris, counts, cfg.grids)
    rb = npvs.build_rulebook(occ, cfg.grids, cfg.d, csr=True)
    lab_bits = torch.from_numpy(to_np(occ) & synth.label_mask_bits(label_seed, (to_np(occ).size,))).to(DEV)
    return cfg, t, layers, occ, rb, lab_bits


def _gpu_forward(occ, rb, layers, dtype):
    acts = [npvs.gather_input(occ, rb, dtype)]
    for li, (W, b) in enumerate(layers):
        last = li == len(layers) - 1
        Wp = npvs.pack_weights(torch.from_numpy(W).to(DEV), dtype)
        acts.append(npvs.sparse_conv_fwd(acts[-1], Wp, torch.from_numpy(b).to(DEV), W.shape[1], W.shape[2], rb, dtype,
                                         relu=not last, out_f32=last))
    return acts


def _gpu_backward(acts, rb, layers, dtype, dlogits, dx_out=None):
    grads = [None] * len(layers)
    dY = dlogits
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        Wt = npvs.pack_weights(torch.from_numpy(W).to(DEV), dtype, flip_transpose=True)
        dX, dW, db = npvs.sparse_conv_bwd(acts[li], Wt, W.shape[1], W.shape[2], acts[li + 1], dY, rb, dtype,
                                          relu=li < len(layers) - 1, want_dx=li > 0)
        grads[li] = (to_np(dW), to_np(db))
        if dx_out is not None and dX is not None:
            dx_out[li] = to_np(dX)
        dY = dX
    return grads


def _loss_inputs(seed):
    """One tiny32 grid's rulebook and seeded logits and labels (the same arrays on both sides)."""
    cfg, t, layers, occ, rb, lab_bits = _setup()
    rng = np.random.default_rng(seed)
    C = cfg.d ** 3
    L = (3.0 * rng.normal(size=(rb.cap, C))).astype(np.float32)
    Y = (rng.random((rb.cap, C)) < 0.3).astype(np.uint8)
    return cfg, rb, L, Y


def test_loss_matches_oracle():
    cfg, rb, L, Y = _loss_inputs(11)
    stats, dl = npvs.loss(torch.from_numpy(L).to(DEV), torch.from_numpy(Y).to(DEV), rb, lam=0.99)
    n = rb.host_counts()["n_sites"]
    ref = oracle.loss(L[:n].astype(np.float64), Y[:n], lam=0.99)
    s = to_np(stats)[0]
    for i, key in enumerate(["loss", "bce", "lrv", "tp", "fn", "fp", "gtp"]):
        assert abs(s[i] - ref[key]) <= 2e-6 * max(1.0, abs(ref[key])), (key, s[i], ref[key])
    assert s[7] == n * cfg.d ** 3
    g = to_np(dl)[:n]
    assert np.abs(g - ref["grad"]).max() <= 1e-6 * np.abs(ref["grad"]).max()


def test_loss_batched_mean_over_grids():
    dims = [(32, 32, 32), (64, 32, 32), (32, 32, 64)]
    tri_list = [synth.box_scene(70 + i, g, 20, 2, 8) for i, g in enumerate(dims)]
    tris, counts = upload_tris(tri_list)
    occ = npvs.froxelize(tris, counts, dims)
    rb = npvs.build_rulebook(occ, dims, 2)
    ref = oracle_batch(tri_list, dims, 2)
    n = ref["n"]
    rng = np.random.default_rng(2)
    L = rng.normal(size=(rb.cap, 8)).astype(np.float32)
    Y = (rng.random((rb.cap, 8)) < 0.3).astype(np.uint8)
    stats, dl = npvs.loss(torch.from_numpy(L).to(DEV), torch.from_numpy(Y).to(DEV), rb)
    s = to_np(stats)
    gr = ref["grid_rows"]
    per = [oracle.loss(L[gr[b]:gr[b + 1]].astype(np.float64), Y[gr[b]:gr[b + 1]]) for b in range(3)]
    for b in range(3):
        assert abs(s[b, 0] - per[b]["loss"]) <= 2e-6 * abs(per[b]["loss"])
    assert abs(s[3, 0] - np.mean([p["loss"] for p in per])) <= 2e-6
    want = np.concatenate([p["grad"] / 3 for p in per])
    assert np.abs(to_np(dl)[:n] - want).max() <= 1e-6 * np.abs(want).max()


@pytest.mark.parametrize("alpha", [0.9, 0.5])
def test_dice_loss_matches_oracle(alpha):
    cfg, rb, L, Y = _loss_inputs(12)
    stats, dl = npvs.loss(torch.from_numpy(L).to(DEV), torch.from_numpy(Y).to(DEV), rb, lam=0.99, dice_alpha=alpha)
    n = rb.host_counts()["n_sites"]
    ref = oracle.loss_dice(L[:n].astype(np.float64), Y[:n], lam=0.99, alpha=alpha)
    s = to_np(stats)[0]
    for i, key in enumerate(["loss", "dice", "lrv", "tp", "fn", "fp", "gtp"]):
        assert abs(s[i] - ref[key]) <= 2e-6 * max(1.0, abs(ref[key])), (key, s[i], ref[key])
    g = to_np(dl)[:n]
    assert np.abs(g - ref["grad"]).max() <= 1e-5 * np.abs(ref["grad"]).max()


def test_dice_loss_batched_mean_over_grids():
    dims = [(32, 32, 32), (64, 32, 32), (32, 32, 64)]
    tri_list = [synth.box_scene(70 + i, g, 20, 2, 8) for i, g in enumerate(dims)]
    tris, counts = upload_tris(tri_list)
    occ = npvs.froxelize(tris, counts, dims)
    rb = npvs.build_rulebook(occ, dims, 2)
    ref = oracle_batch(tri_list, dims, 2)
    n = ref["n"]
    rng = np.random.default_rng(3)
    L = rng.normal(size=(rb.cap, 8)).astype(np.float32)
    Y = (rng.random((rb.cap, 8)) < 0.3).astype(np.uint8)
    stats, dl = npvs.loss(torch.from_numpy(L).to(DEV), torch.from_numpy(Y).to(DEV), rb, dice_alpha=0.8)
    s = to_np(stats)
    gr = ref["grid_rows"]
    per = [oracle.loss_dice(L[gr[b]:gr[b + 1]].astype(np.float64), Y[gr[b]:gr[b + 1]], alpha=0.8) for b in range(3)]
    for b in range(3):
        assert abs(s[b, 0] - per[b]["loss"]) <= 2e-6 * abs(per[b]["loss"])
    assert abs(s[3, 0] - np.mean([p["loss"] for p in per])) <= 2e-6
    want = np.concatenate([p["grad"] / 3 for p in per])
    assert np.abs(to_np(dl)[:n] - want).max() <= 1e-5 * np.abs(want).max()


def test_backward_f32_matches_oracle_gradient():
    cfg, t, layers, occ, rb, lab_bits = _setup()
    acts = _gpu_forward(occ, rb, layers, npvs.NPVS_F32)
    labels = npvs.gather_input(lab_bits, rb, npvs.NPVS_U8)
    _, dl = npvs.loss(acts[-1], labels, rb)
    grads = _gpu_backward(acts, rb, layers, npvs.NPVS_F32, dl)
    out = oracle.forward(t, cfg.grids[0], cfg.d, layers, want_logits=False)
    lab = _oracle_labels(out, cfg.grids[0], cfg.d)
    ref_dl = oracle.loss(out["acts"][-1], lab)["grad"]
    ref, _ = oracle.backward(out, layers, ref_dl)
    for li in range(len(layers)):
        for a, b, nm in ((grads[li][0], ref[li][0], "dW"), (grads[li][1], ref[li][1], "db")):
            scale = np.abs(b).max()
            err = np.abs(a - b).max()
            print(f"layer {li} {nm}: max|err|={err:.3e} max|g|={scale:.3e}", flush=True)
            assert err <= 1e-4 * scale + 1e-9


def test_backward_matches_fp64_finite_differences():
    cfg, t, layers, occ, rb, lab_bits = _setup(layers=synth.he_weights(7, [8, 4, 8], 0.1))
    acts = _gpu_forward(occ, rb, layers, npvs.NPVS_F32)
    labels = npvs.gather_input(lab_bits, rb, npvs.NPVS_U8)
    _, dl = npvs.loss(acts[-1], labels, rb)
    grads = _gpu_backward(acts, rb, layers, npvs.NPVS_F32, dl)
    occ_np, _ = oracle.froxelize(t, cfg.grids[0])  # the oracle's own occupancy, reused by every evaluation
    lab = _oracle_labels(oracle.forward(t, cfg.grids[0], cfg.d, layers, want_logits=False, occ=occ_np),
                         cfg.grids[0], cfg.d)
    rng = np.random.default_rng(0)
    h = 1e-5
    checked = 0
    for li, (W, b) in enumerate(layers):
        for _ in range(12):
            k, c, o = rng.integers(27), rng.integers(W.shape[1]), rng.integers(W.shape[2])
            f, masks = [], []
            for s in (+1, -1):
                L2 = [(w.astype(np.float64).copy(), bb.astype(np.float64).copy()) for w, bb in layers]
                L2[li][0][k, c, o] += s * h
                o2 = oracle.forward(t, cfg.grids[0], cfg.d, L2, want_logits=False, occ=occ_np)
                f.append(oracle.loss(o2["acts"][-1], lab, want_grad=False)["loss"])
                masks.append([a > 0 for a in o2["acts"][1:-1]])
            if any((m1 != m2).any() for m1, m2 in zip(*masks)):
                continue
            fd = (f[0] - f[1]) / (2 * h)
            g = grads[li][0][k, c, o]
            # float32 gradients against FP64 finite differences
            assert abs(g - fd) <= 1e-4 * abs(fd) + 1e-7, (li, k, c, o, g, fd)
            checked += 1
    assert checked >= 15


def test_backward_bf16_within_rigorous_bounds_and_deterministic():
    """tiny32 (three layers) through the BF16 forward and backward against the oracle's BF16
    network (forward_bf16 / backward_bf16, the same rounding points) under the rigorous bounds of
    forward_bf16_bound / loss_grad_bound / backward_bf16_bound, element by element; two runs
    give the same bits."""
    cfg, t, layers, occ, rb, lab_bits = _setup()
    acts = _gpu_forward(occ, rb, layers, npvs.NPVS_BF16)
    labels = npvs.gather_input(lab_bits, rb, npvs.NPVS_U8)
    _, dl = npvs.loss(acts[-1], labels, rb)
    g1 = _gpu_backward(acts, rb, layers, npvs.NPVS_BF16, dl)
    g2 = _gpu_backward(acts, rb, layers, npvs.NPVS_BF16, dl)
    for a, b in zip(g1, g2):
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
    emu = oracle.forward_bf16(t, cfg.grids[0], cfg.d, layers)
    n = len(emu["keys"])
    fb = oracle.forward_bf16_bound(emu, layers)
    assert np.all(np.abs(to_np(acts[-1])[:n] - emu["acts"][-1]) <= fb["D"][-1])
    lab = _oracle_labels(emu, cfg.grids[0], cfg.d)
    ref_dl = oracle.loss(emu["acts"][-1], lab)["grad"]
    e_dl = oracle.loss_grad_bound(emu["acts"][-1], lab, fb["D"][-1])
    assert np.all(np.abs(to_np(dl)[:n] - ref_dl) <= e_dl)
    ref, _ = oracle.backward_bf16(emu, layers, ref_dl)
    bnd, _ = oracle.backward_bf16_bound(emu, layers, fb, ref_dl, e_dl)
    for li in range(len(layers)):
        for j, nm in ((0, "dW"), (1, "db")):
            e = np.abs(g1[li][j] - ref[li][j])
            print(f"bf16 layer {li} {nm}: max err {e.max():.3e}, max err / bound {np.max(e / np.maximum(bnd[li][j], 1e-300)):.3e}, "
                  f"max bound / max |g| {bnd[li][j].max() / np.abs(ref[li][j]).max():.3e}", flush=True)
            assert np.all(e <= bnd[li][j]), (li, nm)


@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
def test_backward_side_streams_change_nothing(dtype):
    """npvs_sparse_conv_bwd with the weight gradient on a second stream and its reductions on a
    third gives the single-stream dX, dW and db bit for bit."""
    cfg, t, layers, occ, rb, lab_bits = _setup()
    acts = _gpu_forward(occ, rb, layers, dtype)
    labels = npvs.gather_input(lab_bits, rb, npvs.NPVS_U8)
    _, dl = npvs.loss(acts[-1], labels, rb)
    side, side2 = torch.cuda.Stream(), torch.cuda.Stream()
    W, _ = layers[-1]
    Wt = npvs.pack_weights(torch.from_numpy(W).to(DEV), dtype, flip_transpose=True)
    args = (acts[-2], Wt, W.shape[1], W.shape[2], acts[-1], dl, rb, dtype, False)
    n = rb.host_counts()["n_sites"]
    ref = npvs.sparse_conv_bwd(*args)
    for ws, rs in ((side, None), (side, side2)):
        got = npvs.sparse_conv_bwd(*args, wgrad_stream=ws, reduce_stream=rs)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.current_stream().wait_stream(side2)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(to_np(ref[0])[:n], to_np(got[0])[:n])  # rows past n_sites: undefined
        for a, b in zip(ref[1:], got[1:]):
            np.testing.assert_array_equal(to_np(a), to_np(b))


@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
def test_batched_weight_gradient_matches_per_layer(dtype):
    """Every layer's backward with the weight gradient deferred (dW = db = NULL), then one
    npvs_sparse_conv_wgrad over all layers: with the single-layer slice count (16) dX, dW and db
    equal the per-layer backward bit for bit; with other slice counts only the grouping of the
    float32 sums changes, so dW stays within 2^-15 sum_p |x_p| |dz_p| of it (each side's error is
    at most a 128-term float32 chunk sum, gamma_128 < 2^-16, of that magnitude) and db is
    unchanged."""
    cfg, t, layers, occ, rb, lab_bits = _setup()
    acts = _gpu_forward(occ, rb, layers, dtype)
    labels = npvs.gather_input(lab_bits, rb, npvs.NPVS_U8)
    _, dl = npvs.loss(acts[-1], labels, rb)
    n = rb.host_counts()["n_sites"]
    ref, pending, mags = {}, [], {}
    off = to_np(rb.rb_off).astype(np.int64)
    pairs = to_np(rb.rb_pairs).reshape(-1, 2)
    dY = dl
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        cin, cout = W.shape[1], W.shape[2]
        Wt = npvs.pack_weights(torch.from_numpy(W).to(DEV), dtype, flip_transpose=True)
        args = (acts[li], Wt, cin, cout, acts[li + 1], dY, rb, dtype)
        kw = dict(relu=li < len(layers) - 1, want_dx=li > 0)
        dX, dW, db = npvs.sparse_conv_bwd(*args, **kw)
        ws = npvs.conv_bwd_workspace(cin, cout, rb, dtype)
        dX2, dW2, db2 = npvs.sparse_conv_bwd(*args, **kw, ws=ws, want_dw=False)
        assert dW2 is None and db2 is None
        if dX is not None:
            np.testing.assert_array_equal(to_np(dX)[:n], to_np(dX2)[:n])
        ref[li] = (to_np(dW), to_np(db))
        pending.append((acts[li], cin, cout, ws, torch.empty_like(dW), torch.empty_like(db)))
        # sum over each offset's pairs of |X[i]| |dZ[r]| (|dZ| <= |dY|, bf16 rounding of dZ inside 1 %)
        ax = np.abs(to_np(acts[li][:n]).astype(np.float64))  # rows past n_sites: undefined
        ag = 1.01 * np.abs(to_np(dY[:n]).astype(np.float64))
        mags[li] = np.stack([ax[pairs[off[k]:off[k + 1], 0]].T @ ag[pairs[off[k]:off[k + 1], 1]] for k in range(27)])
        dY = dX
    order = list(range(len(layers) - 1, -1, -1))
    for slices in (16, 0, 1, 3):
        for _, _, _, _, gW, gb in pending:
            gW.fill_(float("nan"))
            gb.fill_(float("nan"))
        npvs.sparse_conv_wgrad(pending, rb, dtype, slices=slices)
        torch.cuda.synchronize()
        for li, (_, _, _, _, gW, gb) in zip(order, pending):
            if slices == 16:
                np.testing.assert_array_equal(to_np(gW), ref[li][0])
            else:
                err = np.abs(to_np(gW).astype(np.float64) - ref[li][0])
                assert np.all(err <= 2.0 ** -15 * mags[li] + 1e-30), (slices, li, float(err.max()))
            np.testing.assert_array_equal(to_np(gb), ref[li][1])


@pytest.mark.parametrize("checkpoint", [False, True])
def test_chained_backward_matches_unchained(checkpoint):
    """The BF16 network backward with each data gradient fused with the ReLU' of the layer below
    (npvs_sparse_conv_dgrad_relu) against the same backward with separate ReLU' passes and
    against the per-layer backward, all at 16 slices: dW bit for bit (the fused epilogue forms
    the same bfloat16 dZ), the top layer's db bit for bit (formed the same way), and the other
    layers' db within 2^-14 sum_r |dX[r]| (float32 sums of the same values in another grouping:
    running sums over a workgroup's tiles and a 16-row butterfly instead of per-block sums)."""
    cfg, t, layers, occ, rb, lab_bits = _setup()
    labels = npvs.gather_input(lab_bits, rb, npvs.NPVS_U8)
    net = Network(layers, cfg.d, npvs.NPVS_BF16)
    assert net._chainable()
    logits, saved = net.forward(npvs.gather_input(occ, rb, npvs.NPVS_BF16), rb, checkpoint=checkpoint)
    _, dl = npvs.loss(logits, labels, rb)
    grads = {}
    for name, kw in (("chain", dict(batch_wgrad=True, chain=True)), ("plain", dict(batch_wgrad=True, chain=False)),
                     ("layer", dict(batch_wgrad=False))):
        grads[name] = [(to_np(a), to_np(b)) for a, b in net.backward(saved, logits, dl, rb, wgrad_slices=16, **kw)]
    # |dX| of each layer from the per-layer reference path
    acts = _gpu_forward(occ, rb, layers, npvs.NPVS_BF16)
    dx = {}
    _gpu_backward(acts, rb, layers, npvs.NPVS_BF16, dl, dx_out=dx)
    n = rb.host_counts()["n_sites"]
    top = len(layers) - 1
    for li in range(len(layers)):
        np.testing.assert_array_equal(grads["chain"][li][0], grads["plain"][li][0])
        np.testing.assert_array_equal(grads["plain"][li][0], grads["layer"][li][0])
        np.testing.assert_array_equal(grads["plain"][li][1], grads["layer"][li][1])
        if li == top:
            np.testing.assert_array_equal(grads["chain"][li][1], grads["plain"][li][1])
        else:
            mag = np.abs(dx[li + 1][:n].astype(np.float64)).sum(axis=0)
            err = np.abs(grads["chain"][li][1].astype(np.float64) - grads["plain"][li][1])
            assert np.all(err <= 2.0 ** -14 * mag + 1e-30), (li, float(err.max()))


def test_fused_data_gradient_without_mask():
    """npvs_sparse_conv_dgrad_relu with M = NULL (no ReLU' below): the dZ and bias partials it leaves
    in the lower layer's workspace give that layer's weight gradient bit for bit as the per-layer
    backward of that layer with relu = 0 on the same data gradient (dX of the upper layer, in
    float32), and its bias gradient within 2^-14 sum_r |dX[r]| (another grouping of the sums)."""
    cfg, t, layers, occ, rb, lab_bits = _setup()
    acts = _gpu_forward(occ, rb, layers, npvs.NPVS_BF16)
    dY = torch.randn((rb.cap, cfg.channels[2]), device=DEV)
    n = rb.host_counts()["n_sites"]
    (W1, _), (W0, _) = layers[1], layers[0]
    c0, c1, c2 = W0.shape[1], W1.shape[1], W1.shape[2]
    Wt1 = npvs.pack_weights(torch.from_numpy(W1).to(DEV), npvs.NPVS_BF16, flip_transpose=True)
    # upper layer (1): its dZ in ws1, then its data gradient two ways
    ws1 = npvs.conv_bwd_workspace(c1, c2, rb, npvs.NPVS_BF16)
    dX, _, _ = npvs.sparse_conv_bwd(acts[1], Wt1, c1, c2, acts[2], dY, rb, npvs.NPVS_BF16, relu=True, ws=ws1,
                                    want_dw=False)
    ws0 = npvs.conv_bwd_workspace(c0, c1, rb, npvs.NPVS_BF16)
    npvs.sparse_conv_dgrad_relu(Wt1, c1, c2, None, c0, rb, ws1, ws0)
    gW, gb = torch.empty((27, c0, c1), device=DEV), torch.empty(c1, device=DEV)
    npvs.sparse_conv_wgrad([(acts[0], c0, c1, ws0, gW, gb)], rb, npvs.NPVS_BF16, slices=16)
    Wt0 = npvs.pack_weights(torch.from_numpy(W0).to(DEV), npvs.NPVS_BF16, flip_transpose=True)
    _, rW, rdb = npvs.sparse_conv_bwd(acts[0], Wt0, c0, c1, acts[1], dX, rb, npvs.NPVS_BF16, relu=False,
                                      want_dx=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(gW), to_np(rW))
    mag = np.abs(to_np(dX)[:n].astype(np.float64)).sum(axis=0)
    assert np.all(np.abs(to_np(gb).astype(np.float64) - to_np(rdb)) <= 2.0 ** -14 * mag + 1e-30)


@pytest.mark.parametrize("grids", ["one", "three"])
def test_loss_forms_the_last_layers_dz(grids):
    """npvs_loss with the last layer's backward workspace (dz_ws): the chained BF16 backward that
    starts from the dZ the loss wrote equals, bit for bit, the one that forms that dZ itself from
    dL/dlogits (every dW and db), and the loss statistics and dL/dlogits are unchanged.  Three
    grids of different sizes exercise the row-to-grid lookup of the gradient coefficients."""
    cfg = synth.config("tiny32")
    layers = synth.net_layers(cfg, bias_std=0.05)
    if grids == "one":
        dims = cfg.grids
        tri_list = [synth.scene_for(cfg)]
    else:
        dims = [(32, 32, 32), (64, 32, 32), (32, 32, 64)]
        tri_list = [synth.box_scene(70 + i, g, 20, 2, 8) for i, g in enumerate(dims)]
    tris, counts = upload_tris(tri_list)
    occ = npvs.froxelize(tris, counts, dims)
    rb = npvs.build_rulebook(occ, dims, cfg.d, csr=True)
    lab_bits = torch.from_numpy(to_np(occ) & synth.label_mask_bits(5, (to_np(occ).size,))).to(DEV)
    labels = npvs.gather_input(lab_bits, rb, npvs.NPVS_U8)
    net = Network(layers, cfg.d, npvs.NPVS_BF16)
    assert net.backward_form() == (True, True)
    logits, saved = net.forward(npvs.gather_input(occ, rb, npvs.NPVS_BF16), rb)
    stats, dl = npvs.loss(logits, labels, rb)
    ref = [(to_np(a), to_np(b)) for a, b in net.backward(saved, logits, dl, rb)]
    top = len(layers) - 1
    top_ws = npvs.conv_bwd_workspace(net.channels[top], net.channels[top + 1], rb, npvs.NPVS_BF16)
    stats2, dl2 = npvs.loss(logits, labels, rb, dz_ws=top_ws, dz_cin=net.channels[top])
    got = [(to_np(a), to_np(b)) for a, b in net.backward(saved, logits, None, rb, top_ws=top_ws)]
    n = rb.host_counts()["n_sites"]
    np.testing.assert_array_equal(to_np(stats2), to_np(stats))
    np.testing.assert_array_equal(to_np(dl2)[:n], to_np(dl)[:n])
    for (a, b), (c, d) in zip(ref, got):
        np.testing.assert_array_equal(a, c)
        np.testing.assert_array_equal(b, d)


def test_backward_on_an_empty_grid_is_zero():
    """No active sites: every gradient is zero, per layer and with the weight gradients batched
    (both forms; the outputs start as NaN, so each entry must be written)."""
    cfg = synth.config("tiny32")
    layers = synth.net_layers(cfg, bias_std=0.05)
    tris, counts = upload_tris([np.zeros((0, 3, 3), np.float32)])
    occ = npvs.froxelize(tris, counts, cfg.grids)
    rb = npvs.build_rulebook(occ, cfg.grids, cfg.d, csr=True)
    assert rb.host_counts()["n_sites"] == 0
    acts = _gpu_forward(occ, rb, layers, npvs.NPVS_BF16)
    dl = torch.zeros((rb.cap, cfg.channels[-1]), dtype=torch.float32, device=DEV)
    for dW, db in _gpu_backward(acts, rb, layers, npvs.NPVS_BF16, dl):
        assert not dW.any() and not db.any()
    W, _ = layers[1]
    cin, cout = W.shape[1], W.shape[2]
    Wt = npvs.pack_weights(torch.from_numpy(W).to(DEV), npvs.NPVS_BF16, flip_transpose=True)
    ws = npvs.conv_bwd_workspace(cin, cout, rb, npvs.NPVS_BF16)
    npvs.sparse_conv_bwd(acts[1], Wt, cin, cout, acts[2], dl[:, :cout].contiguous(), rb, npvs.NPVS_BF16, relu=True,
                         ws=ws, want_dw=False)
    for slices in (0, 3):
        gW = torch.full((27, cin, cout), float("nan"), device=DEV)
        gb = torch.full((cout,), float("nan"), device=DEV)
        npvs.sparse_conv_wgrad([(acts[1], cin, cout, ws, gW, gb)], rb, npvs.NPVS_BF16, slices=slices)
        torch.cuda.synchronize()
        assert not gW.isnan().any() and not gW.any() and not gb.any()


def test_adam_matches_oracle():
    rng = np.random.default_rng(8)
    p = rng.normal(size=5000).astype(np.float32)
    gs = [rng.normal(size=5000).astype(np.float32) for _ in range(3)]
    tp, tm, tv = (torch.from_numpy(x).to(DEV) for x in (p, np.zeros_like(p), np.zeros_like(p)))
    rp, rm, rv = p.astype(np.float64), np.zeros(5000), np.zeros(5000)
    for t, g in enumerate(gs, start=1):
        npvs.adam(tp, torch.from_numpy(g).to(DEV), tm, tv, t)
        rp, rm, rv = oracle.adam(rp, g, rm, rv, t)
    assert np.abs(to_np(tp) - rp).max() <= 1e-6


def test_adam_with_device_step_equals_host_step():
    rng = np.random.default_rng(9)
    p = rng.normal(size=3000).astype(np.float32)
    gs = [torch.from_numpy(rng.normal(size=3000).astype(np.float32)).to(DEV) for _ in range(4)]
    a = [torch.from_numpy(x).to(DEV) for x in (p, np.zeros_like(p), np.zeros_like(p))]
    b = [x.clone() for x in a]
    step = torch.zeros(16, dtype=torch.uint8, device=DEV)
    for t, g in enumerate(gs, start=1):
        npvs.adam(a[0], g, a[1], a[2], t)
        npvs.adam(b[0], g, b[1], b[2], step)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(to_np(x), to_np(y))
    assert int(step[:8].view(torch.int64).item()) == 4


def test_city256_training_gradients_at_full_size():
    """The benchmark's workload at full size (256x256x128 city frame, six 64-channel layers, the
    launch configuration of its training step: BF16 with the weight gradients of all layers in
    one balanced launch after the data gradients, FP32 per layer on side streams; BF16 per layer
    as well).  FP32 against the oracle's FP64 forward and backward: every dW and db within
    2e-4 of the largest entry.  BF16 against the oracle's BF16 network (forward_bf16 /
    backward_bf16, the same rounding points, labels from the oracle's occupancy): every dW and db
    within DRIFT_FACTOR times the oracle's own drift between two evaluation orders."""
    cfg = synth.config("city256")
    t = synth.scene_for(cfg)
    layers = synth.net_layers(cfg, bias_std=0.05)
    tris, counts = upload_tris([t])
    occ = npvs.froxelize(tris, counts, cfg.grids)
    rb = npvs.build_rulebook(occ, cfg.grids, cfg.d, csr=True)
    label_mask = synth.label_mask_bits(7, (cfg.grids[0][0] * cfg.grids[0][1] * cfg.grids[0][2] // 8,))
    out = oracle.forward(t, cfg.grids[0], cfg.d, layers, want_logits=False)
    n = len(out["keys"])
    assert n == rb.host_counts()["n_sites"] == 9706
    lab_bits = torch.from_numpy(to_np(occ) & label_mask).to(DEV)
    labels = npvs.gather_input(lab_bits, rb, npvs.NPVS_U8)
    ref_lab = oracle.site_labels(out["occ"].reshape(-1) & label_mask, cfg.grids[0], cfg.d, out["keys"])
    ref_dl = oracle.loss(out["acts"][-1], ref_lab)["grad"]
    ref, _ = oracle.backward(out, layers, ref_dl)
    rbf = bf16_reference(t, cfg.grids[0], cfg.d, layers, occ=out["occ"], labels_mask=label_mask)
    for dtype, batch in ((npvs.NPVS_F32, None), (npvs.NPVS_BF16, None), (npvs.NPVS_BF16, False)):
        net = Network(layers, cfg.d, dtype)
        logits, saved = net.forward(npvs.gather_input(occ, rb, dtype), rb)
        _, dl = npvs.loss(logits, labels, rb)
        grads = [(to_np(a), to_np(b)) for a, b in net.backward(saved, logits, dl, rb, batch_wgrad=batch)]
        for li in range(len(layers)):
            for j, nm in ((0, "dW"), (1, "db")):
                a = grads[li][j]
                if dtype == npvs.NPVS_F32:
                    assert np.abs(a - ref[li][j]).max() <= 2e-4 * np.abs(ref[li][j]).max(), (li, nm)
                    continue
                b, b32 = rbf["g"][li][j], rbf["g32"][li][j]
                tol = drift_tol(b, b32)
                err = np.abs(a - b).max()
                print(f"city256 bf16 (batched {batch is None}) layer {li} {nm}: max err {err:.3e}, tolerance {tol:.3e} "
                      f"({tol / np.abs(b).max():.2e} of the largest entry)", flush=True)
                assert tol > 0 and err <= tol, (li, nm)


@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
def test_adam_with_packing_equals_adam_then_packing(dtype):
    """npvs_adam with packings over two steps equals npvs_adam without them followed by both
    packings of each layer, bit for bit (channel counts with padded BF16 fragments included)."""
    rng = np.random.default_rng(21)
    shapes = [(24, 40), (64, 8), (16, 136)]
    sizes = [27 * a * b for a, b in shapes]
    n = sum(sizes) + 300  # a tail of parameters that are not packed weights (biases)
    p0 = rng.normal(size=n).astype(np.float32)
    offs = np.concatenate([[0], np.cumsum(sizes)])[:-1]

    def run(fused):
        p, m, v = (torch.from_numpy(x).to(DEV) for x in (p0.copy(), np.zeros(n, np.float32), np.zeros(n, np.float32)))
        step = torch.zeros(16, dtype=torch.uint8, device=DEV)
        packs = []
        for (a, b), o in zip(shapes, offs):
            W = p[o:o + 27 * a * b].view(27, a, b)
            packs.append((npvs.pack_weights(W, dtype), npvs.pack_weights(W, dtype, flip_transpose=True)))
        for t in range(2):
            g = torch.from_numpy(np.random.default_rng(30 + t).normal(size=n).astype(np.float32)).to(DEV)
            if fused:
                npvs.adam(p, g, m, v, step, [(o, a, b, wp, wt) for (a, b), o, (wp, wt) in zip(shapes, offs, packs)],
                          dtype)
            else:
                npvs.adam(p, g, m, v, step)
                for (a, b), o, (wp, wt) in zip(shapes, offs, packs):
                    W = p[o:o + 27 * a * b].view(27, a, b)
                    wp.copy_(npvs.pack_weights(W, dtype))
                    wt.copy_(npvs.pack_weights(W, dtype, flip_transpose=True))
        torch.cuda.synchronize()
        return to_np(p), [(to_np(wp), to_np(wt)) for wp, wt in packs]

    pa, ka = run(True)
    pb, kb = run(False)
    np.testing.assert_array_equal(pa, pb)
    for (wa, ta), (wb, tb) in zip(ka, kb):
        np.testing.assert_array_equal(wa, wb)
        np.testing.assert_array_equal(ta, tb)


@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
def test_autograd_function_matches_oracle(dtype):
    """Two layers through torch autograd with the hand-written backward (SubMConvFn): the input,
    weight and bias gradients of sum(Y * G) (seeded G) against the oracle's FP64 backward (rows
    past the active sites are left undefined).  FP32 within 1e-4 of the largest entry; BF16
    against the oracle's BF16 network under the rigorous bounds of backward_bf16_bound, with the
    hidden layer's incoming gradient a bfloat16 tensor as autograd hands it over."""
    from paper_2509_24677_amd.train import SubMConvFn
    cfg = synth.config("tiny32")
    t = synth.scene_for(cfg)
    layers = synth.he_weights(9, [8, 16, 8], 0.05)
    tris, counts = upload_tris([t])
    occ = npvs.froxelize(tris, counts, cfg.grids)
    rb = npvs.build_rulebook(occ, cfg.grids, cfg.d, csr=True)
    out = oracle.forward(t, cfg.grids[0], cfg.d, layers, want_logits=False)
    n = len(out["keys"])
    G = np.random.default_rng(4).normal(size=(rb.cap, 8)).astype(np.float32)
    ref, ref_dx = oracle.backward(out, layers, G[:n].astype(np.float64))
    tdt = torch.float32 if dtype == npvs.NPVS_F32 else torch.bfloat16
    X = npvs.gather_input(occ, rb, npvs.NPVS_F32).to(tdt).requires_grad_(True)
    params = [(torch.from_numpy(W).to(DEV).requires_grad_(True), torch.from_numpy(b).to(DEV).requires_grad_(True))
              for W, b in layers]
    h = SubMConvFn.apply(X, params[0][0], params[0][1], rb, dtype, True, False)
    y = SubMConvFn.apply(h, params[1][0], params[1][1], rb, dtype, False, True)
    (y[:n] * torch.from_numpy(G[:n]).to(DEV)).sum().backward()
    got = [(to_np(W.grad), to_np(b.grad)) for W, b in params]
    pairs = [(got[li][j], ref[li][j]) for li in range(2) for j in range(2)]
    pairs.append((to_np(X.grad.float())[:n], ref_dx))
    if dtype == npvs.NPVS_F32:
        for a, b in pairs:
            assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max()
        return
    # BF16: the oracle's BF16 network and its rigorous bounds (G is exact in float32)
    emu = oracle.forward_bf16(t, cfg.grids[0], cfg.d, layers)
    fb = oracle.forward_bf16_bound(emu, layers)
    Gn = G[:n].astype(np.float64)
    # autograd hands the hidden layer its gradient as bfloat16 (the dtype of its output)
    gref, dzb = oracle.backward_bf16(emu, layers, Gn, dy_bf16=True)
    bnd, e_dx0 = oracle.backward_bf16_bound(emu, layers, fb, Gn, np.zeros_like(Gn), dy_bf16=True)
    dx0, _, _ = oracle.subm_conv_bwd(emu["acts"][0], emu["Wb"][0], emu["rb_off"], emu["pairs"], None, dzb[0],
                                     relu=False)
    checks = [(got[li][j], gref[li][j], bnd[li][j]) for li in range(2) for j in range(2)]
    # X is a bfloat16 leaf, so autograd hands back its gradient rounded to bfloat16
    checks.append((to_np(X.grad.float())[:n], dx0, e_dx0 + 2.0 ** -8 * (np.abs(dx0) + e_dx0)))
    for a, b, e in checks:
        assert np.all(np.abs(a - b) <= e), np.abs(a - b).max()
