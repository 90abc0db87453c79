"""Pins of the oracle's PVS agreement metrics (Sec. 5.1: FNR = FN / GTP and FPR = FP / GTP with
the reference as the ground truth; flip rates over the occupied froxels, the froxels of the active
blocks and all froxels).

The expected values are counted by hand on an 8 x 2 x 2 grid with d = 2 (four blocks of 2 x 2 x 2
froxels along x).  Packed byte (z * 2 + y) holds froxels x = 0..7 of row (y, z), bit x.
  G     = {(0,0,0), (1,0,0), (5,0,0), (2,1,1), (5,1,1)}: bytes 0x23, 0x00, 0x00, 0x24
  blocks x//2 = 0, 1, 2 are active (3 x 8 = 24 froxels), block 3 (x = 6, 7) is not
  V_ref = {(0,0,0), (5,0,0), (2,1,1)}:                    bytes 0x21, 0x00, 0x00, 0x04
  V_tst = {(1,0,0), (5,0,0), (2,1,1), (5,1,1)}:           bytes 0x22, 0x00, 0x00, 0x24
  FN = {(0,0,0)} = 1, FP = {(1,0,0), (5,1,1)} = 2, flips = 3, GTP = 3, |G| = 5, N = 32.
"""
import numpy as np
import pytest

import oracle

DIMS = (8, 2, 2)
G = np.array([0x23, 0x00, 0x00, 0x24], np.uint8).reshape(2, 2, 1)
REF = np.array([0x21, 0x00, 0x00, 0x04], np.uint8).reshape(2, 2, 1)
TST = np.array([0x22, 0x00, 0x00, 0x24], np.uint8).reshape(2, 2, 1)


def test_active_froxels_hand_example():
    act = oracle.active_froxels(G, DIMS, 2)
    # blocks 0-2 cover x = 0..5 of every row: bits 0-5 in all four bytes
    assert act.reshape(-1).tolist() == [0x3F] * 4


def test_metrics_hand_example():
    m = oracle.metrics(REF, TST, G, oracle.active_froxels(G, DIMS, 2))
    assert (m["flips"], m["fn"], m["fp"], m["gtp"]) == (3, 1, 2, 3)
    assert (m["occupied"], m["active"], m["froxels"]) == (5, 24, 32)
    assert m["flip_rate_occupied"] == pytest.approx(3 / 5)
    assert m["flip_rate_active"] == pytest.approx(3 / 24)
    assert m["flip_rate_all"] == pytest.approx(3 / 32)
    assert m["missing_geometry"] == pytest.approx(1 / 3) and m["fnr"] == m["missing_geometry"]
    assert m["fpr"] == pytest.approx(2 / 3)


def test_metrics_roles_swap():
    # exchanging the roles of reference and tested set exchanges FN and FP (and GTP follows the
    # reference): 2 / 4 missing, 1 / 4 false positive
    m = oracle.metrics(TST, REF, G, oracle.active_froxels(G, DIMS, 2))
    assert (m["fn"], m["fp"], m["gtp"]) == (2, 1, 4)
    assert m["missing_geometry"] == pytest.approx(0.5) and m["fpr"] == pytest.approx(0.25)


def test_metrics_identical_sets_and_empty_reference():
    act = oracle.active_froxels(G, DIMS, 2)
    m = oracle.metrics(REF, REF, G, act)
    assert m["flips"] == 0 and m["flip_rate_occupied"] == 0 and m["fnr"] == 0 and m["fpr"] == 0
    z = np.zeros_like(REF)
    m = oracle.metrics(z, TST, G, act)
    assert m["gtp"] == 0 and m["fnr"] == 0.0 and m["fpr"] == 0.0 and m["fp"] == 4


def test_metrics_random_against_direct_counts():
    rng = np.random.default_rng(3)
    dims = (32, 16, 8)
    occ = np.packbits((rng.random((8, 16, 32)) < 0.1).astype(np.uint8), axis=-1, bitorder="little")
    g = oracle.unpack(occ).astype(bool)
    a = g & (rng.random(g.shape) < 0.5)
    b = g & (rng.random(g.shape) < 0.5)
    pk = lambda x: np.packbits(x.astype(np.uint8), axis=-1, bitorder="little")
    act = oracle.active_froxels(occ, dims, 4)
    m = oracle.metrics(pk(a), pk(b), occ, act)
    # brute force over every froxel
    n_fn = n_fp = n_flip = 0
    for z in range(8):
        for y in range(16):
            for x in range(32):
                n_fn += a[z, y, x] and not b[z, y, x]
                n_fp += b[z, y, x] and not a[z, y, x]
                n_flip += a[z, y, x] != b[z, y, x]
    assert (m["fn"], m["fp"], m["flips"]) == (n_fn, n_fp, n_flip)
    blk = np.zeros((2, 4, 8), bool)
    for z in range(8):
        for y in range(16):
            for x in range(32):
                blk[z // 4, y // 4, x // 4] |= g[z, y, x]
    assert m["active"] == int(blk.sum()) * 64
