"""Pins of the oracle's loss (Sec. 3.3 repulsive visibility loss, combined loss with BCE in place
of Dice), convolution backward (chain rule), Adam, and the ray-march labeller (Sec. 3.2 ground
truth by dense sampling of the viewcell).

Independent routes: hand-derived closed forms, FP64 central finite differences, the transposed
rulebook identity, torch.optim.Adam, and a brute-force nearest-hit ray caster over all triangles.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_hparams_fixture():
    hp = json.load(open(os.path.join(GOLD, "paper_hparams.json")))
    assert hp["tau"] == 0.5 and hp["lambda"] == 0.99
    # tau = 0.5 on sigma(l) is the logit threshold l >= 0
    assert 1 / (1 + math.exp(-0.0)) == hp["tau"]
    assert int(hp["channels_for_d"]["8"]) == 8 ** 3


# ------------------------------------------------------------------ loss
def test_loss_two_froxel_hand_example():
    # l = (0, ln 3), y = (1, 0): p = (1/2, 3/4); softplus = (ln 2, ln 4)
    r = oracle.loss(np.array([0.0, math.log(3.0)]), np.array([1, 0]), lam=0.99)
    assert r["bce"] == pytest.approx(1.5 * math.log(2.0), abs=1e-15)
    assert (r["tp"], r["fn"], r["fp"], r["gtp"]) == pytest.approx((0.5, 0.5, 0.75, 1.0), abs=1e-15)
    assert r["lrv"] == pytest.approx(1.25, abs=1e-15)
    assert r["loss"] == pytest.approx(0.99 * 1.5 * math.log(2.0) + 0.01 * 1.25, abs=1e-15)
    # dL/dl = lam (p - y)/m + (1 - lam) p (1 - p)(1 - 2y)/GTP
    g = r["grad"]
    assert g[0] == pytest.approx(0.99 * (-0.5) / 2 + 0.01 * 0.25 * (-1.0), abs=1e-15)
    assert g[1] == pytest.approx(0.99 * 0.75 / 2 + 0.01 * 0.1875, abs=1e-15)


def test_perfect_prediction_has_zero_rvl():
    y = np.array([1, 0, 1, 1, 0, 0], np.uint8)
    l = np.where(y == 1, 60.0, -60.0)
    r = oracle.loss(l, y)
    assert r["lrv"] < 1e-20 and r["fn"] < 1e-20 and r["fp"] < 1e-20


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(0)
    l = rng.normal(0, 2, size=40)
    y = (rng.random(40) < 0.3).astype(np.uint8)
    g = oracle.loss(l, y)["grad"]
    h = 1e-6
    for t in range(40):
        lp, lm = l.copy(), l.copy()
        lp[t] += h
        lm[t] -= h
        fd = (oracle.loss(lp, y, want_grad=False)["loss"] - oracle.loss(lm, y, want_grad=False)["loss"]) / (2 * h)
        assert abs(fd - g[t]) <= 1e-7 * max(1.0, abs(g[t]))


def test_no_positive_labels_guard():
    r = oracle.loss(np.array([0.3, -1.0]), np.array([0, 0]))
    p = 1 / (1 + np.exp(-np.array([0.3, -1.0])))
    assert r["gtp"] == 0 and r["lrv"] == pytest.approx(p.sum(), abs=1e-15)


def test_dice_loss_three_froxel_hand_example():
    # l = (ln 3, ln 3, -ln 3), y = (1, 0, 1): p = (3/4, 3/4, 1/4); TP = 1, missed A = 1, B = 3/4,
    # GTP = 2; alpha = 0.8: den = 2 + 0.8 + 0.15 = 59/20, L_dice = 1 - 40/59 = 19/59; L_rv = 7/8
    r = oracle.loss_dice(np.array([math.log(3.0), math.log(3.0), -math.log(3.0)]), np.array([1, 0, 1]), lam=0.99,
                         alpha=0.8)
    assert (r["tp"], r["fn"], r["fp"], r["gtp"]) == pytest.approx((1.0, 1.0, 0.75, 2.0), abs=1e-15)
    assert r["dice"] == pytest.approx(19.0 / 59.0, abs=1e-15)
    assert r["lrv"] == pytest.approx(0.875, abs=1e-15)
    assert r["loss"] == pytest.approx(0.99 * 19.0 / 59.0 + 0.01 * 0.875, abs=1e-15)


def test_dice_loss_gradient_finite_differences_and_autograd():
    rng = np.random.default_rng(1)
    l = rng.normal(0, 2, size=40)
    y = (rng.random(40) < 0.3).astype(np.uint8)
    for alpha in (0.9, 0.5, 0.0):
        g = oracle.loss_dice(l, y, alpha=alpha)["grad"]
        h = 1e-6
        for t in range(40):
            lp, lm = l.copy(), l.copy()
            lp[t] += h
            lm[t] -= h
            fd = (oracle.loss_dice(lp, y, alpha=alpha, want_grad=False)["loss"]
                  - oracle.loss_dice(lm, y, alpha=alpha, want_grad=False)["loss"]) / (2 * h)
            assert abs(fd - g[t]) <= 1e-7 * max(1.0, abs(g[t]))
        # torch autograd of the soft counts (float64)
        lt = torch.tensor(l, requires_grad=True)
        yt = torch.tensor(y, dtype=torch.float64)
        p = torch.sigmoid(lt)
        tp, a, b = (yt * p).sum(), (yt * (1 - p)).sum(), ((1 - yt) * p).sum()
        val = 0.99 * (1 - 2 * tp / (2 * tp + alpha * a + (1 - alpha) * b)) + 0.01 * (a + b) / max(float(y.sum()), 1.0)
        val.backward()
        np.testing.assert_allclose(g, lt.grad.numpy(), rtol=1e-12, atol=1e-15)


def test_dice_loss_limits():
    y = np.array([1, 0, 1, 1, 0, 0], np.uint8)
    r = oracle.loss_dice(np.where(y == 1, 60.0, -60.0), y)  # perfect prediction
    assert r["dice"] < 1e-20 and r["lrv"] < 1e-20
    r = oracle.loss_dice(np.array([0.3, -1.0]), np.array([0, 0]))  # no ground truth: TP = 0
    assert r["dice"] == pytest.approx(1.0, abs=1e-15)


# ------------------------------------------------------------------ backward
def _small_net():
    dims = (32, 32, 32)
    tris = synth.box_scene(0, dims, 20)
    layers = synth.he_weights(7, [8, 4, 8], 0.1)
    return dims, tris, layers


def _scalar(out, labels_rows):
    return oracle.loss(out["acts"][-1], labels_rows, want_grad=False)["loss"]


def test_backward_matches_finite_differences():
    dims, tris, layers = _small_net()
    out = oracle.forward(tris, dims, 2, layers, want_logits=False)
    lab = oracle.site_labels(out["occ"] & synth.label_mask_bits(3, out["occ"].shape), dims, 2, out["keys"])
    dl = oracle.loss(out["acts"][-1], lab)["grad"]
    grads, _ = oracle.backward(out, layers, dl)
    rng = np.random.default_rng(1)
    h = 1e-5  # FP64 central differences: truncation ~h^2, rounding of the summed loss ~1e-14/h
    checked = 0
    for li, (W, b) in enumerate(layers):
        for _ in range(25):
            k, c, o = rng.integers(27), rng.integers(W.shape[1]), rng.integers(W.shape[2])
            res = []
            masks = []
            for s in (+1, -1):
                L2 = [(w.astype(np.float64).copy(), bb.astype(np.float64).copy()) for w, bb in layers]
                L2[li][0][k, c, o] += s * h
                o2 = oracle.forward(tris, dims, 2, L2, want_logits=False, occ=out["occ"])
                res.append(_scalar(o2, lab))
                masks.append([a > 0 for a in o2["acts"][1:-1]])
            if any((m1 != m2).any() for m1, m2 in zip(*masks)):
                continue  # the perturbation crosses a ReLU kink
            fd = (res[0] - res[1]) / (2 * h)
            an = grads[li][0][k, c, o]
            assert abs(fd - an) <= 1e-6 * abs(an) + 1e-10, (li, k, c, o, fd, an)
            checked += 1
        for o in range(b.shape[0]):
            res = []
            for s in (+1, -1):
                L2 = [(w.astype(np.float64).copy(), bb.astype(np.float64).copy()) for w, bb in layers]
                L2[li][1][o] += s * h
                res.append(_scalar(oracle.forward(tris, dims, 2, L2, want_logits=False, occ=out["occ"]), lab))
            fd = (res[0] - res[1]) / (2 * h)
            assert abs(fd - grads[li][1][o]) <= 1e-6 * abs(grads[li][1][o]) + 1e-10
    assert checked >= 30


def test_dgrad_is_forward_conv_with_flipped_transposed_weights():
    dims, tris, _ = _small_net()
    occ, _ = oracle.froxelize(tris, dims)
    keys = oracle.active_sites(occ, dims, 2)
    rb_off, pairs = oracle.rulebook(keys, (16, 16, 16))
    rng = np.random.default_rng(2)
    X = rng.normal(size=(len(keys), 6))
    W = rng.normal(size=(27, 6, 5))
    dY = rng.normal(size=(len(keys), 5))
    dX, _, _ = oracle.subm_conv_bwd(X, W, rb_off, pairs, np.ones((len(keys), 5)), dY, relu=False)
    Wf = W[::-1].transpose(0, 2, 1)
    np.testing.assert_allclose(dX, oracle.subm_conv(dY, Wf, None, rb_off, pairs, False), atol=1e-12)


def test_relu_mask_and_bias_gradient():
    dims, tris, _ = _small_net()
    occ, _ = oracle.froxelize(tris, dims)
    keys = oracle.active_sites(occ, dims, 2)
    rb_off, pairs = oracle.rulebook(keys, (16, 16, 16))
    rng = np.random.default_rng(3)
    X = rng.normal(size=(len(keys), 3))
    W = rng.normal(size=(27, 3, 4))
    Y = np.maximum(rng.normal(size=(len(keys), 4)), 0.0)
    dY = rng.normal(size=(len(keys), 4))
    _, _, db = oracle.subm_conv_bwd(X, W, rb_off, pairs, Y, dY, relu=True)
    np.testing.assert_allclose(db, (dY * (Y > 0)).sum(0), atol=1e-12)


# ------------------------------------------------------------------ Adam
def test_adam_first_step_closed_form_and_torch():
    rng = np.random.default_rng(4)
    p0 = rng.normal(size=50)
    gs = [rng.normal(size=50) for _ in range(4)]
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    p1, _, _ = oracle.adam(p, gs[0], m, v, 1, lr=1e-3, wd=0.0)
    # first step from m = v = 0: m_hat = g, v_hat = g^2, so the step is -lr g / (|g| + eps)
    np.testing.assert_allclose(p1 - p0, -1e-3 * gs[0] / (np.abs(gs[0]) + 1e-8), rtol=0, atol=1e-15)
    tp = torch.nn.Parameter(torch.tensor(p0, dtype=torch.float64))
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-10)
    for t, g in enumerate(gs, start=1):
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = oracle.adam(p, g, m, v, t, lr=1e-3, wd=1e-10)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=0, atol=1e-15)


# ------------------------------------------------------------------ labeller
def _wall_scene(nx, ny, z):
    # full-width wall in the plane z, plus boxes behind it
    w = [[(0, 0, z), (nx, 0, z), (nx, ny, z)], [(0, 0, z), (nx, ny, z), (0, ny, z)]]
    behind = synth.box_scene(5, (nx, ny, 16), 6) + np.array([0, 0, z + 2.0], np.float32)
    return np.concatenate([np.asarray(w, np.float32), behind])


def test_labeller_wall_occludes_everything_behind():
    nx, ny, nz = 16, 16, 32
    tris = _wall_scene(nx, ny, 8.5)
    views = synth.viewpoints(1, 8, (nx / 2, ny / 2, -nz / 2), 1.0)
    lab = oracle.unpack(oracle.label_raymarch(tris, (nx, ny, nz), views, s_r=2))
    assert lab[8].all()          # every froxel of the wall layer is seen
    assert not lab[9:].any()     # nothing behind the wall
    assert not lab[:8].any()


def _brute_labels(tris, dims, view, s_r):
    nx, ny, nz = dims
    T = tris.astype(np.float64)
    v0, e1, e2 = T[:, 0], T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]
    lab = np.zeros((nz, ny, nx), np.uint8)
    targets = []
    for j in range(ny * s_r):
        for i in range(nx * s_r):
            targets.append(((i + .5) / s_r, (j + .5) / s_r, nz))
    for side in (0, 1):
        for k in range(nz * s_r):
            for j in range(ny * s_r):
                targets.append((nx if side else 0.0, (j + .5) / s_r, (k + .5) / s_r))
        for k in range(nz * s_r):
            for i in range(nx * s_r):
                targets.append(((i + .5) / s_r, ny if side else 0.0, (k + .5) / s_r))
    o = np.asarray(view, np.float64)
    for tg in targets:
        d = np.asarray(tg) - o
        pv = np.cross(d, e2)
        det = (e1 * pv).sum(1)
        ok = det != 0
        inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
        tv = o - v0
        u = (tv * pv).sum(1) * inv
        qv = np.cross(tv, e1)
        v = (d * qv).sum(1) * inv
        s = (e2 * qv).sum(1) * inv
        hit = ok & (u >= 0) & (u <= 1) & (v >= 0) & (u + v <= 1)
        # segment of the ray inside the grid box
        s0, s1 = 0.0, 1.0
        for a, hi in enumerate((nx, ny, nz)):
            if d[a] != 0:
                ta, tb = sorted(((0 - o[a]) / d[a], (hi - o[a]) / d[a]))
                s0, s1 = max(s0, ta), min(s1, tb)
        hit &= (s >= s0) & (s <= s1)
        if s0 > s1 or not hit.any():
            continue
        sh = s[hit].min()
        p = o + sh * d
        c = np.clip(np.floor(p).astype(int), 0, np.array(dims) - 1)
        lab[c[2], c[1], c[0]] = 1
    return lab


def test_labeller_matches_brute_force_nearest_hit():
    dims = (16, 16, 16)
    tris = synth.box_scene(12, dims, 7, 2, 6)
    view = synth.viewpoints(2, 1, (8.0, 8.0, -8.0), 1.0)
    got = oracle.unpack(oracle.label_raymarch(tris, dims, view, s_r=1))
    want = _brute_labels(tris, dims, view[0], 1)
    np.testing.assert_array_equal(got, want)


def test_labels_subset_of_occupancy_and_deterministic():
    cfg = synth.config("tiny32")
    dims = cfg.grids[0]
    tris = synth.scene_for(cfg)
    views = synth.viewpoints(200, 64, (dims[0] / 2, dims[1] / 2, -dims[2] / 2), 1.0)
    lab = oracle.label_raymarch(tris, dims, views, 2)
    occ, _ = oracle.froxelize(tris, dims)
    assert not (lab & ~occ).any()
    assert 0 < oracle.unpack(lab).sum() < oracle.unpack(occ).sum()
    np.testing.assert_array_equal(lab, oracle.label_raymarch(tris, dims, views, 2))
    one = views[:1]
    np.testing.assert_array_equal(oracle.label_raymarch(tris, dims, np.repeat(one, 5, 0), 2),
                                  oracle.label_raymarch(tris, dims, one, 2))
