"""Shared setup of the GPU parity tests: seeded scenes on the device and the oracle's per-grid
results concatenated into the batch layout of the HIP library."""
import numpy as np
import torch

import oracle
import paper_2509_24677_amd as npvs
import synth

DEV = "cuda"


def upload_tris(tri_list):
    allt = np.concatenate([np.asarray(t, np.float32).reshape(-1, 3, 3) for t in tri_list]) if tri_list else \
        np.zeros((0, 3, 3), np.float32)
    return torch.from_numpy(allt).to(DEV), [len(t) for t in tri_list]


def oracle_batch(tri_list, dims, d):
    """Per-grid oracle results merged into the batch layout (global keys, row offsets)."""
    occs, keys, nbrs, pairs_k, grid_rows = [], [], [], [[] for _ in range(27)], [0]
    X = []
    key_off = 0
    row_off = 0
    for t, g in zip(tri_list, dims):
        occ, _ = oracle.froxelize(t, g)
        k = oracle.active_sites(occ, g, d)
        bd = (g[0] // d, g[1] // d, g[2] // d)
        rb_off, pairs = oracle.rulebook(k, bd)
        occs.append(occ.reshape(-1))
        keys.append(k + key_off)
        X.append(oracle.gather_sites(occ, g, d, k))
        for kk in range(27):
            seg = pairs[rb_off[kk]:rb_off[kk + 1]] + row_off
            pairs_k[kk].append(seg)
        key_off += bd[0] * bd[1] * bd[2]
        row_off += len(k)
        grid_rows.append(row_off)
    pairs_all = [np.concatenate(p) if p else np.zeros((0, 2), np.int32) for p in pairs_k]
    rb_off = np.concatenate([[0], np.cumsum([len(p) for p in pairs_all])]).astype(np.int32)
    pairs = np.concatenate(pairs_all).astype(np.int32)
    n = row_off
    nbr = np.full((27, n), -1, np.int32)
    for kk in range(27):
        nbr[kk, pairs_all[kk][:, 1]] = pairs_all[kk][:, 0]
    return dict(occ=np.concatenate(occs), keys=np.concatenate(keys).astype(np.int32), n=n, rb_off=rb_off,
                pairs=pairs, nbr=nbr, grid_rows=np.array(grid_rows, np.int32), X=np.concatenate(X),
                total_blocks=key_off)


def to_np(t):
    if t.dtype == torch.bfloat16:
        return t.float().cpu().numpy()
    return t.cpu().numpy()


def bf16_round(a):
    """Round float64 values to bfloat16 and back (torch's round-to-nearest-even)."""
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def conv_tolerance(X, W, rb_off, pairs, n_terms_scale=2.0):
    """Float32 accumulation bound of a conv layer: 2 n u sum |x||w| per output element
    (u = 2^-24, n = 27 * cin terms at most)."""
    absY = oracle.subm_conv(np.abs(X), np.abs(W), None, rb_off, pairs, False)
    n = 27 * W.shape[1]
    return n_terms_scale * n * 2.0 ** -24 * absY + 1e-30


def scene(name, i=0):
    cfg = synth.config(name)
    return cfg, synth.scene_for(cfg, i)


# End-to-end BF16 tolerance.  Two float32 evaluation orders of the same BF16 network (same
# rounded weights, same rounding points) differ only where a float32 sum lands on the other side
# of a bfloat16 rounding boundary or of the ReLU's zero; the deviation that follows is one
# bfloat16 quantum at a few hidden values, carried on by the later layers.  The oracle measures
# how large that gets on the same input by evaluating its BF16 network a second time with
# float32 accumulation (forward_bf16 / backward_bf16 with accum="f32").  The library's order is
# a third one; its results must lie within DRIFT_FACTOR times the oracle's own drift, per tensor
# (max-abs).  The arithmetic of each layer is checked separately against rigorous bounds.
DRIFT_FACTOR = 4.0


def bf16_reference(t, dims, d, layers, occ=None, labels_mask=None):
    """The oracle's BF16 network on one grid in FP64 between the rounding points (emu) and with
    float32 accumulation (o32); with labels_mask, also the loss gradient and the backward of
    both (g, g32: [(dW, db)] per layer) from the oracle's own labels."""
    emu = oracle.forward_bf16(t, dims, d, layers, occ=occ)
    o32 = oracle.forward_bf16(t, dims, d, layers, occ=emu["occ"], accum="f32")
    # the float32 bound of the last layer alone: what remains when no rounding decision differs
    last = oracle.bf16_layer_bound(emu["acts"][-2], emu["Wb"][-1], layers[-1][1], emu["rb_off"], emu["pairs"],
                                   relu=False)
    res = dict(emu=emu, o32=o32, logit_floor=float(last["D"].max()) if last["D"].size else 0.0)
    if labels_mask is not None:
        occf = emu["occ"].reshape(-1)
        lab = oracle.site_labels(occf & labels_mask, dims, d, emu["keys"])
        dl = oracle.loss(emu["acts"][-1], lab)["grad"]
        dl32 = oracle.loss(o32["acts"][-1], lab)["grad"].astype(np.float32).astype(np.float64)
        res["g"], _ = oracle.backward_bf16(emu, layers, dl)
        res["g32"], _ = oracle.backward_bf16(o32, layers, dl32, accum="f32")
        res["labels"] = lab
    return res


def drift_tol(a_ref, a_alt, floor=0.0):
    """DRIFT_FACTOR times the max-abs distance of the oracle's two evaluation orders."""
    return DRIFT_FACTOR * max(float(np.abs(np.asarray(a_alt) - np.asarray(a_ref)).max()), floor)
