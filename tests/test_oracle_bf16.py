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
