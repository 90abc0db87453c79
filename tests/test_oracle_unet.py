"""Pins of the oracle's two-level U-Net pieces (CPU): the strided convolution against torch's
dense stride-2 conv3d, the inverse convolution against conv_transpose3d, the level relation
against the active sites at interleave factor 2d, and the whole U-Net against a masked dense
evaluation built from torch conv3d / conv_transpose3d (all float64)."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import synth


def _dense(X, keys, bdims):
    """Sparse rows at block keys -> dense [C][Bz][By][Bx] (zero at inactive blocks)."""
    Bx, By, Bz = bdims
    D = np.zeros((X.shape[1], Bz * By * Bx))
    D[:, keys] = X.T
    return torch.from_numpy(D.reshape(X.shape[1], Bz, By, Bx))


def _at(D, keys):
    return D.reshape(D.shape[0], -1)[:, keys].T.numpy()


def _to_torch_w(W):
    """[8][cin][cout] with k = (dz*2 + dy)*2 + dx -> conv3d weight [cout][cin][2][2][2]."""
    cin, cout = W.shape[1], W.shape[2]
    return torch.from_numpy(np.ascontiguousarray(W.reshape(2, 2, 2, cin, cout).transpose(4, 3, 0, 1, 2)))


def _random_blocks(rng, bdims, p):
    Bx, By, Bz = bdims
    return np.flatnonzero(rng.random(Bx * By * Bz) < p).astype(np.int32)


@pytest.mark.parametrize("seed,p", [(0, 0.05), (1, 0.3), (2, 0.9)])
def test_level_maps_and_strided_convs_match_dense_torch(seed, p):
    rng = np.random.default_rng(seed)
    b0 = (8, 6, 4)
    keys0 = _random_blocks(rng, b0, p)
    b1 = (4, 3, 2)
    # level 1 = the coarse blocks that hold an active level-0 block
    bx, by, bz = keys0 % 8, (keys0 // 8) % 6, keys0 // 48
    keys1 = np.unique(((bz // 2) * 3 + by // 2) * 4 + bx // 2).astype(np.int32)
    children, parent, kid = oracle.level_maps(keys0, keys1, b0)
    assert (children >= 0).sum() == len(keys0)
    assert sorted(children[children >= 0].tolist()) == list(range(len(keys0)))
    cin, cout = 5, 7
    X0 = rng.normal(size=(len(keys0), cin))
    W = rng.normal(size=(8, cin, cout))
    b = rng.normal(size=cout)
    got = oracle.strided_down(X0, children, W, b, relu=False)
    ref = F.conv3d(_dense(X0, keys0, b0)[None], _to_torch_w(W), torch.from_numpy(b), stride=2)[0]
    np.testing.assert_allclose(got, _at(ref, keys1), rtol=1e-12, atol=1e-12)
    X1 = rng.normal(size=(len(keys1), cin))
    got = oracle.inverse_up(X1, parent, kid, W, b, relu=True)
    wt = torch.from_numpy(np.ascontiguousarray(W.reshape(2, 2, 2, cin, cout).transpose(3, 4, 0, 1, 2)))
    ref = F.conv_transpose3d(_dense(X1, keys1, b1)[None], wt, torch.from_numpy(b), stride=2)[0]
    np.testing.assert_allclose(got, np.maximum(_at(ref, keys0), 0.0), rtol=1e-12, atol=1e-12)


def test_coarse_sites_are_the_sites_of_interleave_factor_2d():
    cfg = synth.config("tiny32")
    tris = synth.scene_for(cfg)
    g = cfg.grids[0]
    occ, _ = oracle.froxelize(tris, g)
    keys0 = oracle.active_sites(occ, g, 2)
    keys1 = oracle.active_sites(occ, g, 4)
    B = g[0] // 2
    bx, by, bz = keys0 % B, (keys0 // B) % B, keys0 // (B * B)
    C = B // 2
    np.testing.assert_array_equal(np.unique(((bz // 2) * C + by // 2) * C + bx // 2), keys1)


def test_unet_forward_matches_masked_dense_torch():
    cfg = synth.config("tiny32")
    tris = synth.scene_for(cfg)
    g, d = cfg.grids[0], 2
    params = {k: [(W.astype(np.float64), b.astype(np.float64)) for W, b in v]
              for k, v in synth.unet_params(4, d, E=16, Dc=24).items()}
    out = oracle.unet_forward(tris, g, d, params, want_logits=False)
    keys0, keys1 = out["keys0"], out["keys1"]
    b0 = (g[0] // d, g[1] // d, g[2] // d)
    b1 = (b0[0] // 2, b0[1] // 2, b0[2] // 2)
    m0 = np.zeros(b0[0] * b0[1] * b0[2]); m0[keys0] = 1
    m1 = np.zeros(b1[0] * b1[1] * b1[2]); m1[keys1] = 1
    m0 = torch.from_numpy(m0.reshape(b0[2], b0[1], b0[0]))
    m1 = torch.from_numpy(m1.reshape(b1[2], b1[1], b1[0]))

    def subm(x, Wb, mask, relu=True):
        W, b = Wb
        w = torch.from_numpy(np.ascontiguousarray(W.reshape(3, 3, 3, W.shape[1], W.shape[2]).transpose(4, 3, 0, 1, 2)))
        y = (F.conv3d(x[None], w, torch.from_numpy(b), padding=1)[0]) * mask
        return torch.relu(y) if relu else y

    x = _dense(oracle.gather_sites(out["occ"], g, d, keys0), keys0, b0)
    for Wb in params["stem"] + params["enc0"]:
        x = subm(x, Wb, m0)
    skip = x
    (W, b), = params["down"]
    h = torch.relu(F.conv3d(x[None], _to_torch_w(W), torch.from_numpy(b), stride=2)[0]) * m1
    for Wb in params["enc1"]:
        h = subm(h, Wb, m1)
    (W, b), = params["up"]
    wt = torch.from_numpy(np.ascontiguousarray(W.reshape(2, 2, 2, W.shape[1], W.shape[2]).transpose(3, 4, 0, 1, 2)))
    u = torch.relu(F.conv_transpose3d(h[None], wt, torch.from_numpy(b), stride=2)[0]) * m0
    x = torch.cat([u, skip], 0)
    for Wb in params["dec0"]:
        x = subm(x, Wb, m0)
    y = subm(x, params["head"][0], m0, relu=False)
    np.testing.assert_allclose(out["acts"]["Y"], _at(y, keys0), rtol=1e-9, atol=1e-9)
    assert len(keys1) < len(keys0)


def _leaf(a):
    return torch.tensor(np.asarray(a, np.float64), requires_grad=True)


@pytest.mark.parametrize("relu", [False, True])
def test_strided_backward_matches_torch_autograd(relu):
    """The backward of the strided convolution and of its inverse against torch autograd through
    dense stride-2 conv3d / conv_transpose3d (float64): dX, dW, db."""
    rng = np.random.default_rng(5)
    b0, b1 = (8, 6, 4), (4, 3, 2)
    keys0 = _random_blocks(rng, b0, 0.4)
    bx, by, bz = keys0 % 8, (keys0 // 8) % 6, keys0 // 48
    keys1 = np.unique(((bz // 2) * 3 + by // 2) * 4 + bx // 2).astype(np.int32)
    children, parent, kid = oracle.level_maps(keys0, keys1, b0)
    cin, cout = 5, 7
    for up in (False, True):
        n_in, n_out = (len(keys1), len(keys0)) if up else (len(keys0), len(keys1))
        X = rng.normal(size=(n_in, cin))
        W = rng.normal(size=(8, cin, cout))
        b = rng.normal(size=cout)
        G = rng.normal(size=(n_out, cout))
        x, w, bb = _leaf(_dense(X, keys1 if up else keys0, b1 if up else b0).numpy()), _leaf(W), _leaf(b)
        w5 = w.reshape(2, 2, 2, cin, cout)
        if up:
            y = F.conv_transpose3d(x[None], w5.permute(3, 4, 0, 1, 2), bb, stride=2)[0]
            keys_out = keys0
        else:
            y = F.conv3d(x[None], w5.permute(4, 3, 0, 1, 2), bb, stride=2)[0]
            keys_out = keys1
        if relu:
            y = torch.relu(y)
        yr = y.reshape(cout, -1)[:, torch.from_numpy(keys_out.astype(np.int64))].T
        (yr * torch.from_numpy(G)).sum().backward()
        Yo = yr.detach().numpy()
        if up:
            dX, dW, db = oracle.inverse_up_bwd(X, parent, kid, W, Yo, G, relu)
            gx = x.grad.reshape(cin, -1)[:, torch.from_numpy(keys1.astype(np.int64))].T.numpy()
        else:
            dX, dW, db = oracle.strided_down_bwd(X, children, W, Yo, G, relu)
            gx = x.grad.reshape(cin, -1)[:, torch.from_numpy(keys0.astype(np.int64))].T.numpy()
        np.testing.assert_allclose(dX, gx, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(dW, w.grad.numpy(), rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(db, bb.grad.numpy(), rtol=1e-10, atol=1e-10)


def test_unet_backward_matches_torch_autograd_on_masked_dense():
    """The oracle's U-Net backward against torch autograd through the masked dense evaluation of
    the same network (float64), for the loss sum(Y * G) with a random G: the gradient of every
    weight and bias of every stage and of the network input."""
    cfg = synth.config("tiny32")
    tris = synth.scene_for(cfg)
    g, d = cfg.grids[0], 2
    params = {k: [(W.astype(np.float64), b.astype(np.float64)) for W, b in v]
              for k, v in synth.unet_params(6, d, E=8, Dc=12).items()}
    out = oracle.unet_forward(tris, g, d, params, want_logits=False)
    keys0, keys1 = out["keys0"], out["keys1"]
    b0 = (g[0] // d, g[1] // d, g[2] // d)
    b1 = (b0[0] // 2, b0[1] // 2, b0[2] // 2)
    m0 = np.zeros(b0[0] * b0[1] * b0[2]); m0[keys0] = 1
    m1 = np.zeros(b1[0] * b1[1] * b1[2]); m1[keys1] = 1
    m0 = torch.from_numpy(m0.reshape(b0[2], b0[1], b0[0]))
    m1 = torch.from_numpy(m1.reshape(b1[2], b1[1], b1[0]))
    leaves = {st: [(_leaf(W), _leaf(b)) for W, b in v] for st, v in params.items()}

    def subm(x, wb, mask, relu=True):
        w, b = wb
        cin, cout = w.shape[1], w.shape[2]
        y = F.conv3d(x[None], w.reshape(3, 3, 3, cin, cout).permute(4, 3, 0, 1, 2), b, padding=1)[0] * mask
        return torch.relu(y) if relu else y

    x = _leaf(_dense(oracle.gather_sites(out["occ"], g, d, keys0), keys0, b0).numpy())
    h = x
    for wb in leaves["stem"] + leaves["enc0"]:
        h = subm(h, wb, m0)
    skip = h
    (w, b), = leaves["down"]
    E = w.shape[1]
    h1 = torch.relu(F.conv3d(h[None], w.reshape(2, 2, 2, E, E).permute(4, 3, 0, 1, 2), b, stride=2)[0]) * m1
    for wb in leaves["enc1"]:
        h1 = subm(h1, wb, m1)
    (w, b), = leaves["up"]
    Dc = w.shape[2]
    u = torch.relu(F.conv_transpose3d(h1[None], w.reshape(2, 2, 2, E, Dc).permute(3, 4, 0, 1, 2), b, stride=2)[0]) * m0
    h = torch.cat([u, skip], 0)
    for wb in leaves["dec0"]:
        h = subm(h, wb, m0)
    y = subm(h, leaves["head"][0], m0, relu=False)
    G = np.random.default_rng(9).normal(size=out["acts"]["Y"].shape)
    yr = y.reshape(y.shape[0], -1)[:, torch.from_numpy(keys0.astype(np.int64))].T
    (yr * torch.from_numpy(G)).sum().backward()
    grads, dX = oracle.unet_backward(out, params, G)
    checked = 0
    for st, layer_grads in grads.items():
        for (dW, db), (w, b) in zip(layer_grads, leaves[st]):
            np.testing.assert_allclose(dW, w.grad.numpy(), rtol=1e-9, atol=1e-9, err_msg=st)
            np.testing.assert_allclose(db, b.grad.numpy(), rtol=1e-9, atol=1e-9, err_msg=st)
            assert np.abs(dW).max() > 0, st
            checked += 1
    assert checked == 11
    gx = x.grad.reshape(x.shape[0], -1)[:, torch.from_numpy(keys0.astype(np.int64))].T.numpy()
    np.testing.assert_allclose(dX, gx, rtol=1e-9, atol=1e-9)
