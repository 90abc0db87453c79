"""Pins of the oracle's bfloat16 rounding and of the BF16-path emulation (the rounding points of
the BF16 network: weights from float32 masters, each hidden layer's result after bias and ReLU,
the backward's dZ operand; logits and db unrounded).

bf16_round is pinned by hand values (ties to even, the subnormal quantum, overflow) and by
torch's float32 -> bfloat16 conversion (a library routine) on float32 inputs, where rounding the
float64 value directly is the same rounding.  forward_bf16 / backward_bf16 are pinned by hand on
a one-site network whose hidden value is a rounding tie, and reduce to the plain FP64 oracle when
every value is representable in bfloat16.
"""
import numpy as np
import pytest
import torch

import oracle


def test_bf16_round_hand_values():
    r = oracle.bf16_round
    assert r(1.0 + 2.0 ** -8) == 1.0                     # tie between 1 and 1 + 2^-7: even is 1
    assert r(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6     # tie between 1 + 2^-7 (odd) and 1 + 2^-6
    assert r(1.0 + 2.0 ** -8 + 2.0 ** -30) == 1.0 + 2.0 ** -7  # just above the tie
    assert r(-(3.0 + 2.0 ** -7)) == -3.0                 # quantum 2^-6 at [2, 4): below half a quantum
    assert r(0.0) == 0.0 and r(-0.0) == 0.0
    assert r(2.0 ** -133) == 2.0 ** -133                 # smallest subnormal
    assert r(1.4 * 2.0 ** -133) == 2.0 ** -133 and r(0.4 * 2.0 ** -133) == 0.0
    big = (2.0 - 2.0 ** -7) * 2.0 ** 127                  # largest finite bfloat16
    assert r(big) == big
    assert np.isinf(r((2.0 - 2.0 ** -8) * 2.0 ** 127))   # tie with 2^128: even rounds up, overflows
    assert np.isnan(r(np.nan)) and r(np.inf) == np.inf


def test_bf16_round_matches_torch_on_float32_values():
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))).astype(np.float32)
    # exact ties: float32 values whose low 16 bits are 0x8000
    ties = ((rng.integers(0x3F000000, 0x47000000, 2000, dtype=np.int64) & ~0xFFFF) | 0x8000).astype(np.uint32)
    x = np.concatenate([x, ties.view(np.float32), -ties.view(np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.bf16_round(x.astype(np.float64)), want)


def _one_site_net():
    # an 8x4x4 grid with one occupied froxel at (1, 1, 1); d = 2 gives one active site (block 0)
    # whose channel c = (1*2 + 1)*2 + 1 = 7 is 1 and the other 7 channels are 0
    tris = np.array([[[1.25, 1.25, 1.5], [1.75, 1.25, 1.5], [1.25, 1.75, 1.5]]], np.float32)
    W1 = np.zeros((27, 8, 8), np.float32)
    W1[13, 7, 0] = np.float32(1.0 + 2.0 ** -9)   # rounds to 1 in bfloat16
    b1 = np.zeros(8, np.float32)
    b1[0] = np.float32(2.0 ** -8)                # bias stays float32
    W2 = np.zeros((27, 8, 8), np.float32)
    W2[13, 0, 3] = np.float32(3.0)
    b2 = np.zeros(8, np.float32)
    b2[3] = np.float32(2.0 ** -10)               # a logit of 3 + 2^-10 is not a bfloat16 value
    return tris, [(W1, b1), (W2, b2)]


def test_forward_bf16_hand_example():
    tris, layers = _one_site_net()
    dims = (8, 4, 4)
    emu = oracle.forward_bf16(tris, dims, 2, layers)
    ref = oracle.forward(tris, dims, 2, layers)
    assert len(emu["keys"]) == 1 and emu["acts"][0][0].tolist() == [0, 0, 0, 0, 0, 0, 0, 1]
    assert emu["Wb"][0][13, 7, 0] == 1.0
    # hidden: 1 * 1 + 2^-8 = 1 + 2^-8, a tie, rounds to 1; the logit 3 * 1 + 2^-10 is not rounded
    assert emu["pre"][0][0, 0] == 1.0 + 2.0 ** -8 and emu["acts"][1][0, 0] == 1.0
    assert emu["acts"][2][0, 3] == 3.0 + 2.0 ** -10
    # the FP64 network keeps everything: 3 * (1 + 2^-9 + 2^-8) + 2^-10
    assert ref["acts"][2][0, 3] == pytest.approx(3.0 * (1.0 + 2.0 ** -9 + 2.0 ** -8) + 2.0 ** -10, abs=1e-15)


def test_backward_bf16_hand_example():
    tris, layers = _one_site_net()
    emu = oracle.forward_bf16(tris, (8, 4, 4), 2, layers)
    dl = np.zeros((1, 8))
    dl[0, 3] = 1.0 + 2.0 ** -8                    # the last layer's dZ: rounds to 1 for the products
    grads, dzb = oracle.backward_bf16(emu, layers, dl)
    dW2, db2 = grads[1]
    assert dzb[1][0, 3] == 1.0
    assert dW2[13, 0, 3] == 1.0                   # X (= 1) times dZb (= 1)
    assert db2[3] == 1.0 + 2.0 ** -8              # db sums the unrounded dZ
    # the hidden layer: dY = dZb W2^T = 3 at channel 0, its output 1 > 0 keeps it
    dW1, db1 = grads[0]
    assert dzb[0][0, 0] == 3.0 and dW1[13, 7, 0] == 3.0 and db1[0] == 3.0


def test_bf16_emulation_reduces_to_fp64_when_everything_is_representable():
    rng = np.random.default_rng(8)
    dims = (16, 16, 16)
    tris = np.concatenate([rng.uniform(0, 16, size=(40, 1, 3)) + rng.uniform(-1.5, 1.5, size=(40, 3, 3))]).astype(
        np.float32)
    # weights in {0, +-1/2, +-1}, biases 0: every hidden value is a small multiple of 1/2^6 below 64,
    # exactly representable in bfloat16, so no rounding point changes anything
    layers = []
    for cin, cout in ((8, 4), (4, 8)):
        W = (rng.integers(-2, 3, size=(27, cin, cout)) / 2.0 * (rng.random((27, cin, cout)) < 0.15)).astype(np.float32)
        layers.append((W, np.zeros(cout, np.float32)))
    emu = oracle.forward_bf16(tris, dims, 2, layers)
    ref = oracle.forward(tris, dims, 2, layers)
    for a, b in zip(emu["acts"], ref["acts"]):
        np.testing.assert_array_equal(a, b)
    assert np.all(oracle.bf16_round(emu["acts"][1]) == emu["acts"][1])
    dl = rng.integers(-4, 5, size=emu["acts"][-1].shape) / 8.0
    grads, _ = oracle.backward_bf16(emu, layers, dl)
    rgrads, _ = oracle.backward(ref, layers, dl)
    for (a, b), (c, e) in zip(grads, rgrads):
        np.testing.assert_array_equal(a, c)
        np.testing.assert_array_equal(b, e)


def test_float32_order_variants_stay_within_the_float32_bound():
    # the float32-accumulation evaluations differ from the FP64 definitions by at most the
    # float32 rounding bound gamma_n sum |x||w| (n terms per output)
    rng = np.random.default_rng(12)
    keys = np.sort(rng.choice(6 * 6 * 6, 90, replace=False)).astype(np.int32)
    rb_off, pairs = oracle.rulebook(keys, (6, 6, 6))
    X = rng.standard_normal((90, 16))
    W = rng.standard_normal((27, 16, 8))
    b = rng.standard_normal(8)
    y64 = oracle.subm_conv(X, W, b, rb_off, pairs, relu=False)
    y32 = oracle.subm_conv_f32(X.astype(np.float32), W.astype(np.float32), b, rb_off, pairs, relu=False)
    u = 2.0 ** -24
    n = 27 * 16 + 1
    x32, w32 = X.astype(np.float32).astype(np.float64), W.astype(np.float32).astype(np.float64)
    y64r = oracle.subm_conv(x32, w32, b.astype(np.float32), rb_off, pairs, relu=False)
    bound = n * u / (1 - n * u) * (oracle.subm_conv(np.abs(x32), np.abs(w32), np.abs(b.astype(np.float32)), rb_off,
                                                    pairs, relu=False))
    assert np.all(np.abs(y32 - y64r) <= bound)
    assert np.abs(y32 - y64).max() > 0  # a different evaluation, not a copy
    dZ = rng.standard_normal((90, 8)).astype(np.float32).astype(np.float64)
    dX64, dW64, _ = oracle.subm_conv_bwd(x32, w32, rb_off, pairs, None, dZ, relu=False)
    dX32, dW32 = oracle.subm_conv_bwd_f32(x32, w32, rb_off, pairs, dZ)
    bx = 27 * 8 * u * 2 * np.abs(oracle.subm_conv_bwd(np.abs(x32), np.abs(w32), rb_off, pairs, None, np.abs(dZ),
                                                      relu=False)[0])
    assert np.all(np.abs(dX32 - dX64) <= bx + 1e-300)
    bw = len(pairs) * u * 2 * np.abs(oracle.subm_conv_bwd(np.abs(x32), np.abs(w32), rb_off, pairs, None, np.abs(dZ),
                                                          relu=False)[1])
    assert np.all(np.abs(dW32 - dW64) <= bw + 1e-300)


# ------------------------------------------------------------------ error bounds of the BF16 path
# Pins of f32_sum_gamma, bf16_layer_bound, bf16_layer_bwd_bound, forward_bf16_bound,
# backward_bf16_bound and loss_grad_bound: hand values on the one-site network, containment of
# float32 evaluations in several orders (numpy's sequential and pairwise float32 sums), and
# planted mistakes that every tight bound must reject.
import synth


def _f32_orders(X, W, b, rb_off, pairs):
    """Three float32-accumulation evaluations of one layer (no ReLU): offsets in order, offsets
    reversed, and one pairwise float32 sum over all 27 cin products and the bias per output."""
    X32, W32 = np.asarray(X, np.float32), np.asarray(W, np.float32)
    b32 = np.asarray(b, np.float32)
    fwd = oracle.subm_conv_f32(X32, W32, b32, rb_off, pairs, relu=False)
    rev = np.zeros_like(fwd)
    for k in range(26, -1, -1):
        p = pairs[rb_off[k]:rb_off[k + 1]]
        if len(p):
            rev[p[:, 1]] += X32[p[:, 0]] @ W32[k]
    rev += b32
    n, cin = X32.shape
    terms = np.zeros((n, 27 * cin + 1, W32.shape[2]), np.float32)
    for k in range(27):
        p = pairs[rb_off[k]:rb_off[k + 1]]
        terms[p[:, 1], k * cin:(k + 1) * cin, :] = X32[p[:, 0]][:, :, None] * W32[k][None, :, :]
    terms[:, -1, :] = b32
    pw = terms.sum(axis=1, dtype=np.float32)
    return [np.asarray(a, np.float64) for a in (fwd, rev, pw)]


def _tiny_case():
    cfg = synth.config("tiny32")
    t = synth.scene_for(cfg)
    layers = synth.net_layers(cfg, bias_std=0.05)
    return cfg, t, layers, oracle.forward_bf16(t, cfg.grids[0], cfg.d, layers)


def test_f32_sum_gamma_closed_form_and_containment():
    u = 2.0 ** -23
    assert oracle.f32_sum_gamma(1) == u / (1 - u)
    assert oracle.f32_sum_gamma(1000) == 1000 * u / (1 - 1000 * u)
    with pytest.raises(ValueError):
        oracle.f32_sum_gamma(2 ** 23)
    rng = np.random.default_rng(3)
    for n in (2, 17, 1000, 20000):
        t = (rng.standard_normal(n) * np.exp(rng.uniform(-8, 8, n))).astype(np.float32)
        exact = np.sum(t.astype(np.float64))  # exact float32 terms; float64 error far below the bound
        g = oracle.f32_sum_gamma(n) * np.abs(t.astype(np.float64)).sum()
        seq = np.float32(0)
        for v in t:
            seq = np.float32(seq + v)
        for s in (seq, t.sum(dtype=np.float32), t[::-1].sum(dtype=np.float32)):
            assert abs(float(s) - exact) <= g


def test_layer_bound_hand_example():
    tris, layers = _one_site_net()
    emu = oracle.forward_bf16(tris, (8, 4, 4), 2, layers)
    (W1, b1), (W2, b2) = layers
    r = oracle.bf16_layer_bound(emu["acts"][0], emu["Wb"][0], b1, emu["rb_off"], emu["pairs"], relu=True)
    g = oracle.f32_sum_gamma(27 * 8 + 1)
    # z = 1 * 1 + 2^-8 (a tie); sum |x| |w| + |b| = 1 + 2^-8
    assert r["z"][0, 0] == 1.0 + 2.0 ** -8
    assert r["D"][0, 0] == pytest.approx(g * (1.0 + 2.0 ** -8), rel=1e-8)
    assert r["lo"][0, 0] == 1.0 and r["hi"][0, 0] == 1.0 + 2.0 ** -7 and r["out"][0, 0] == 1.0
    # channels with no weight and no bias: z = 0 exactly, D = 0, the output is certainly 0
    assert (r["D"][0, 1:] == 0).all() and (r["lo"][0, 1:] == 0).all() and (r["hi"][0, 1:] == 0).all()
    # the propagated bound: E_1 = the whole quantum 2^-7 at the tie, so the logit carries 3 * 2^-7
    fb = oracle.forward_bf16_bound(emu, layers)
    assert fb["E"][1][0, 0] == 2.0 ** -7 and (fb["E"][1][0, 1:] == 0).all()
    assert fb["mask_certain"][0].all()
    want = 3 * 2.0 ** -7 + g * ((1.0 + 2.0 ** -7) * 3.0 + 2.0 ** -10)
    assert fb["D"][1][0, 3] == pytest.approx(want, rel=1e-8)


def test_layer_bound_contains_float32_orders_and_rejects_planted_mistakes():
    cfg, t, layers, emu = _tiny_case()
    rb_off, pairs = emu["rb_off"], emu["pairs"]
    n_checked = 0
    for li, (_, b) in enumerate(layers):
        relu = li < len(layers) - 1
        X, Wb = emu["acts"][li], emu["Wb"][li]
        r = oracle.bf16_layer_bound(X, Wb, b, rb_off, pairs, relu)
        for z32 in _f32_orders(X, Wb, b, rb_off, pairs):
            assert np.all(np.abs(z32 - r["z"]) <= r["D"])
            if relu:
                o = oracle.bf16_round(np.maximum(z32, 0.0))
                assert np.all((o >= r["lo"]) & (o <= r["hi"]))
            n_checked += 1
        # planted mistakes: a dropped offset, the bias left out, truncation instead of RNE
        W_drop = Wb.copy()
        W_drop[4] = 0.0
        z_drop = oracle.subm_conv(X, W_drop, b, rb_off, pairs, relu=False)
        assert np.any(np.abs(z_drop - r["z"]) > r["D"])
        z_nob = oracle.subm_conv(X, Wb, None, rb_off, pairs, relu=False)
        assert np.any(np.abs(z_nob - r["z"]) > r["D"])
        if relu:
            zz = np.maximum(r["z"], 0.0).astype(np.float32)
            trunc = (zz.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
            assert np.any((trunc < r["lo"]) | (trunc > r["hi"]))
    assert n_checked == 9
    # the worst-case gamma_n bound still pins most outputs to one bfloat16 value (82 % here)
    r = oracle.bf16_layer_bound(emu["acts"][1], emu["Wb"][1], layers[1][1], rb_off, pairs, True)
    assert (r["lo"] == r["hi"]).mean() > 0.75


def test_layer_bwd_bound_contains_float32_orders_and_rejects_planted_mistakes():
    cfg, t, layers, emu = _tiny_case()
    rb_off, pairs = emu["rb_off"], emu["pairs"]
    rng = np.random.default_rng(21)
    for li in range(len(layers)):
        relu = li < len(layers) - 1
        X, Wb, Y = emu["acts"][li], emu["Wb"][li], emu["acts"][li + 1]
        dY = (rng.standard_normal(Y.shape) * 1e-2).astype(np.float32).astype(np.float64)
        r = oracle.bf16_layer_bwd_bound(X, Wb, rb_off, pairs, Y, dY, relu, want_dx=True)
        dZ = dY * (Y > 0) if relu else dY
        assert np.array_equal(r["dZb"], oracle.bf16_round(dZ))
        dX32, dW32 = oracle.subm_conv_bwd_f32(X, Wb, rb_off, pairs, r["dZb"])
        assert np.all(np.abs(dX32 - r["dX"]) <= r["E_dX"])
        assert np.all(np.abs(dW32 - r["dW"]) <= r["E_dW"])
        db32 = np.asarray(dZ, np.float32).sum(axis=0, dtype=np.float32)
        assert np.all(np.abs(db32 - r["db"]) <= r["E_db"])
        # planted: dZ not rounded to bfloat16 before the products; no ReLU mask; W not transposed
        _, dW_nr, _ = oracle.subm_conv_bwd(X, Wb, rb_off, pairs, None, dZ, relu=False, want_dx=False)
        assert np.any(np.abs(dW_nr - r["dW"]) > r["E_dW"])
        if relu:
            _, dW_nm, _ = oracle.subm_conv_bwd(X, Wb, rb_off, pairs, None, oracle.bf16_round(dY), relu=False,
                                               want_dx=False)
            assert np.any(np.abs(dW_nm - r["dW"]) > r["E_dW"])
        if Wb.shape[1] == Wb.shape[2]:
            dX_nt, _, _ = oracle.subm_conv_bwd(X, np.transpose(Wb, (0, 2, 1)), rb_off, pairs, None, r["dZb"],
                                               relu=False)
            assert np.any(np.abs(dX_nt - r["dX"]) > r["E_dX"])


def test_network_bounds_contain_a_float32_order_evaluation():
    cfg, t, layers, emu = _tiny_case()
    fb = oracle.forward_bf16_bound(emu, layers)
    o32 = oracle.forward_bf16(t, cfg.grids[0], cfg.d, layers, accum="f32")
    for li in range(1, len(layers)):
        assert np.all(np.abs(o32["acts"][li] - emu["acts"][li]) <= fb["E"][li])
    assert np.all(np.abs(o32["acts"][-1] - emu["acts"][-1]) <= fb["D"][-1])
    occ = emu["occ"].reshape(-1)
    lab = oracle.site_labels(occ & synth.label_mask_bits(5, (occ.size,)), cfg.grids[0], cfg.d, emu["keys"])
    dl = oracle.loss(emu["acts"][-1], lab)["grad"]
    e_dl = oracle.loss_grad_bound(emu["acts"][-1], lab, fb["D"][-1])
    dl32 = oracle.loss(o32["acts"][-1], lab)["grad"].astype(np.float32).astype(np.float64)
    assert np.all(np.abs(dl32 - dl) <= e_dl)
    bb, e_dx0 = oracle.backward_bf16_bound(emu, layers, fb, dl, e_dl)
    g, _ = oracle.backward_bf16(emu, layers, dl)
    g32, _ = oracle.backward_bf16(o32, layers, dl32, accum="f32")
    for li in range(len(layers)):
        assert np.all(np.abs(g32[li][0] - g[li][0]) <= bb[li][0])
        assert np.all(np.abs(g32[li][1] - g[li][1]) <= bb[li][1])
    # with the incoming gradient of each hidden layer rounded to bfloat16 as well
    gr, _ = oracle.backward_bf16(emu, layers, dl, dy_bf16=True)
    gr32, _ = oracle.backward_bf16(o32, layers, dl32, accum="f32", dy_bf16=True)
    bbr, _ = oracle.backward_bf16_bound(emu, layers, fb, dl, e_dl, dy_bf16=True)
    for li in range(len(layers)):
        assert np.all(np.abs(gr32[li][0] - gr[li][0]) <= bbr[li][0])
        assert np.all(np.abs(gr32[li][1] - gr[li][1]) <= bbr[li][1])
    # the hidden layers' db sums bfloat16 values then; the top layer's is unchanged
    assert np.array_equal(gr[-1][1], g[-1][1]) and not np.array_equal(gr[0][1], g[0][1])
    # the input gradient: products of the rounded dZ of layer 0 with its weights
    _, dzb = oracle.backward_bf16(emu, layers, dl)
    _, dzb32 = oracle.backward_bf16(o32, layers, dl32, accum="f32")
    dx0, _ = oracle.subm_conv_bwd_f32(emu["acts"][0], emu["Wb"][0], emu["rb_off"], emu["pairs"], dzb32[0])
    dx0_ref, _, _ = oracle.subm_conv_bwd(emu["acts"][0], emu["Wb"][0], emu["rb_off"], emu["pairs"], None, dzb[0],
                                         relu=False)
    assert np.all(np.abs(dx0 - dx0_ref) <= e_dx0)
    # the bound of a layer whose inputs are exact equals the one-layer bound
    r = oracle.bf16_layer_bound(emu["acts"][0], emu["Wb"][0], layers[0][1], emu["rb_off"], emu["pairs"], True)
    np.testing.assert_allclose(fb["D"][0], r["D"], rtol=1e-12, atol=0)


def test_loss_grad_bound_lipschitz_and_float32_evaluation():
    rng = np.random.default_rng(4)
    n = 4000
    l = rng.standard_normal(n) * 4
    y = (rng.random(n) < 0.2).astype(np.uint8)
    e = np.full(n, 0.05)
    bnd = oracle.loss_grad_bound(l, y, e)
    g = oracle.loss(l, y)["grad"]
    for s in range(5):
        d = rng.uniform(-1, 1, n) * e
        g2 = oracle.loss(l + d, y)["grad"]
        assert np.all(np.abs(g2 - g) <= bnd)
    # the largest slope of p (1 - p) is 1 / (6 sqrt 3), at p = 1/2 +- 1/(2 sqrt 3)
    t = np.linspace(-6, 6, 200001)
    p = 1 / (1 + np.exp(-t))
    slope = np.abs(p * (1 - p) * (1 - 2 * p))
    assert slope.max() == pytest.approx(1 / (6 * np.sqrt(3)), rel=1e-6)
    # a float32 evaluation of the gradient formula, on the same logits
    lam, g_den = 0.99, max(float(y.sum()), 1.0)
    l32 = l.astype(np.float32)
    p32 = np.float32(1) / (np.float32(1) + np.exp(-l32))
    yf = y.astype(np.float32)
    g32 = (np.float32(lam / n) * (p32 - yf) + np.float32((1 - lam) / g_den) * p32 * (np.float32(1) - p32)
           * (np.float32(1) - np.float32(2) * yf)).astype(np.float64)
    g_exact = oracle.loss(l32.astype(np.float64), y)["grad"]
    assert np.all(np.abs(g32 - g_exact) <= oracle.loss_grad_bound(l32.astype(np.float64), y, np.zeros(n)))


def _unet_exact_params(rng, d, E=4, Dc=6):
    # weights in {0, +-1/2, +-1} (sparse), zero biases: every value of the network is a small
    # multiple of a power of two, exactly representable in bfloat16
    def conv(k, cin, cout):
        W = (rng.integers(-2, 3, size=(k, cin, cout)) / 2.0 * (rng.random((k, cin, cout)) < 0.12)).astype(np.float32)
        return W, np.zeros(cout, np.float32)
    C = d ** 3
    return dict(stem=[conv(27, C, E)], enc0=[conv(27, E, E) for _ in range(2)], down=[conv(8, E, E)],
                enc1=[conv(27, E, E) for _ in range(3)], up=[conv(8, E, Dc)],
                dec0=[conv(27, Dc + E, Dc), conv(27, Dc, Dc)], head=[conv(27, Dc, C)])


def test_unet_bf16_reduces_to_fp64_when_everything_is_representable():
    rng = np.random.default_rng(31)
    dims = (16, 16, 16)
    tris = (rng.uniform(0, 16, size=(40, 1, 3)) + rng.uniform(-1.5, 1.5, size=(40, 3, 3))).astype(np.float32)
    params = _unet_exact_params(rng, 2)
    emu = oracle.unet_forward_bf16(tris, dims, 2, params)
    ref = oracle.unet_forward(tris, dims, 2, params)
    assert np.abs(ref["acts"]["Y"]).max() > 0 and np.all(oracle.bf16_round(ref["acts"]["skip"]) == ref["acts"]["skip"])
    for k in ("X", "skip", "coarse", "up", "Y"):
        np.testing.assert_array_equal(emu["acts"][k], ref["acts"][k])


def test_unet_bf16_without_its_rounding_is_the_fp64_unet(monkeypatch):
    # with bfloat16 rounding replaced by the identity, the BF16 U-Net (forward and backward, both
    # evaluation orders' wiring) is the FP64 U-Net: the rounding points are the only difference
    cfg = synth.config("tiny32")
    t = synth.scene_for(cfg)
    params = synth.unet_params(6, 2, E=16, Dc=24)
    p64 = {k: [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in v] for k, v in params.items()}
    monkeypatch.setattr(oracle, "bf16_round", lambda x: np.asarray(x, np.float64))
    emu = oracle.unet_forward_bf16(t, cfg.grids[0], 2, params)
    ref = oracle.unet_forward(t, cfg.grids[0], 2, p64)
    np.testing.assert_allclose(emu["acts"]["Y"], ref["acts"]["Y"], rtol=1e-12, atol=1e-12)
    dY = np.random.default_rng(2).standard_normal(emu["acts"]["Y"].shape)
    g = oracle.unet_backward_bf16(emu, dY)
    r, _ = oracle.unet_backward(ref, p64, dY)
    for st in r:
        for (a, b), (c, e) in zip(g[st], r[st]):
            np.testing.assert_allclose(a, c, rtol=1e-10, atol=1e-12)
            np.testing.assert_allclose(b, e, rtol=1e-10, atol=1e-12)
    g32 = oracle.unet_backward_bf16(oracle.unet_forward_bf16(t, cfg.grids[0], 2, params, accum="f32"), dY,
                                    accum="f32")
    for st in r:
        for (a, b), (c, e) in zip(g32[st], r[st]):
            np.testing.assert_allclose(a, c, rtol=1e-3, atol=1e-5 * np.abs(c).max())


def test_unet_bf16_rounds_every_hidden_value():
    cfg = synth.config("tiny32")
    t = synth.scene_for(cfg)
    params = synth.unet_params(6, 2, E=16, Dc=24)
    emu = oracle.unet_forward_bf16(t, cfg.grids[0], 2, params)
    ref = oracle.unet_forward(t, cfg.grids[0], 2, params)
    for k in ("skip", "coarse", "up"):
        a = emu["acts"][k]
        assert np.array_equal(oracle.bf16_round(a), a)
        assert not np.array_equal(a, ref["acts"][k])
        # one rounding per layer: close to the FP64 network, not equal
        assert np.abs(a - ref["acts"][k]).max() < 0.05 * np.abs(ref["acts"][k]).max()
    for st, v in emu["Wr"].items():
        for W, _ in v:
            assert np.array_equal(oracle.bf16_round(W), W)
    # logits are not rounded
    assert not np.array_equal(oracle.bf16_round(emu["acts"]["Y"]), emu["acts"]["Y"])
