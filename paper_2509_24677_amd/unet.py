"""Two-level sparse U-Net forward over the C ABI.

Sec. 3.3 adopts an encoder/decoder backbone; the supplement's network settings give its shapes
(embedding and encoder channels 64, down ratio 2, decoder channels 96, encoder depths 2 and 3,
decoder depth 2).  With two levels the network here is

    stem     submanifold 3^3, d^3 -> E            level 0
    enc0     2 x submanifold 3^3, E -> E          level 0   (its output is the skip)
    down     kernel 2 stride 2, E -> E            level 0 -> 1
    enc1     3 x submanifold 3^3, E -> E          level 1
    up       its transposed convolution, E -> D   level 1 -> 0
    concat   [up | skip], D + E channels
    dec0     2 x submanifold 3^3, D + E -> D -> D level 0
    head     submanifold 3^3, D -> d^3            logits (float32, no ReLU)

with ReLU after every layer but the head.  Level 1 is the rulebook of interleave factor 2d.
The paper's adaptive relation convolutions and aggregators are not part of it.  The backward
(chain rule stage by stage) splits the concatenation's gradient into its up and skip parts and
adds to the skip's part the gradient arriving through the strided convolution.
"""
from __future__ import annotations

import torch

from . import (NPVS_BF16, NPVS_F32, Levels, build_levels, concat_channels, concat_channels_bwd, conv_bwd_workspace,
               deinterleave_threshold, froxelize, gather_input, pack_weights, pack_weights_k, sparse_conv_bwd,
               sparse_conv_fwd, sparse_conv_wgrad, strided_conv_bwd, strided_conv_fwd)
from ._lib import NPVS_MAX_WGRAD_LAYERS

STAGES = ("stem", "enc0", "down", "enc1", "up", "dec0", "head")


class UNet:
    def __init__(self, params: dict, d: int, dtype: int = NPVS_BF16, device="cuda"):
        """params: {stage: [(W, b), ...]} with W float32 [27][cin][cout] (submanifold) or
        [8][cin][cout] (down, up) and b float32 [cout], as numpy or torch."""
        self.d = d
        self.dtype = dtype
        self.layers = {}
        self.weights = {}  # float32 master weights, packed for the data gradient on first use
        self.Wt = {}
        for st in STAGES:
            out = []
            for W, b in params[st]:
                W = torch.as_tensor(W, dtype=torch.float32).to(device).contiguous()
                b = torch.as_tensor(b, dtype=torch.float32).to(device).contiguous()
                Wp = pack_weights_k(W, dtype) if W.shape[0] == 8 else pack_weights(W, dtype)
                out.append((Wp, b, W.shape[1], W.shape[2]))
                self.weights.setdefault(st, []).append(W)
            self.layers[st] = out
        (_, _, E, Dc), = self.layers["up"]
        if self.layers["dec0"][0][2] != Dc + E:
            raise ValueError("the first decoder layer must take the up output and the skip channels")

    def forward(self, X0: torch.Tensor, lv: Levels, saved: dict | None = None) -> torch.Tensor:
        """Logits float32 [rb0.cap][d^3] (rows past the level-0 count undefined).  With `saved`
        (a dict), the input of every layer (saved[stage] = [...]) and the up output (saved["u"])
        are kept for backward()."""
        dt = self.dtype
        rb0, rb1 = lv.rb0, lv.rb1

        def keep(st, x):
            if saved is not None:
                saved.setdefault(st, []).append(x)

        def subm(h, layer, rb, last=False):
            Wp, b, cin, cout = layer
            return sparse_conv_fwd(h, Wp, b, cin, cout, rb, dt, relu=not last, out_f32=last)

        h = X0
        for st in ("stem", "enc0"):
            for layer in self.layers[st]:
                keep(st, h)
                h = subm(h, layer, rb0)
        skip = h
        (Wp, b, cin, cout), = self.layers["down"]
        keep("down", skip)
        h1 = strided_conv_fwd(skip, Wp, b, cin, cout, lv, up=False, dtype=dt)
        for layer in self.layers["enc1"]:
            keep("enc1", h1)
            h1 = subm(h1, layer, rb1)
        (Wp, b, cin, cout), = self.layers["up"]
        keep("up", h1)
        u = strided_conv_fwd(h1, Wp, b, cin, cout, lv, up=True, dtype=dt)
        if saved is not None:
            saved["u"] = u
        h = concat_channels(u, skip, rb0)
        for layer in self.layers["dec0"]:
            keep("dec0", h)
            h = subm(h, layer, rb0)
        keep("head", h)
        return subm(h, self.layers["head"][0], rb0, last=True)

    def _wt(self, st, i):
        """The data-gradient packing of layer i of stage st (flipped transpose for the 3^3
        layers, per-offset transpose for the strided ones), made on first use."""
        if (st, i) not in self.Wt:
            W = self.weights[st][i]
            self.Wt[(st, i)] = (pack_weights_k(W, self.dtype, transpose=True) if W.shape[0] == 8 else
                                pack_weights(W, self.dtype, flip_transpose=True))
        return self.Wt[(st, i)]

    def backward(self, saved: dict, logits: torch.Tensor, dlogits: torch.Tensor, lv: Levels,
                 overlap: bool = True, batch_wgrad: bool = False, wgrad_slices: int = 0) -> dict:
        """Gradients {stage: [(dW, db), ...]} (float32) of the loss whose gradient with respect to
        the logits rows is `dlogits` (float32 [rb0.cap][d^3]), through the activations kept by
        forward(saved=...).  The levels must carry CSR rulebooks (build_levels(csr=True)).  With
        `batch_wgrad`, the weight gradients of the 3^3 layers are deferred and computed after the
        data gradients, those of each level's layers in one launch (up to 16 per launch;
        `wgrad_slices` pair-list slices per offset, 0 for the library's choice).  It is not the
        default: the decoder's wider layers give a level about 15 channel windows, so the
        one-round launch has a single slice per offset and window, and the per-layer form is
        faster.  Otherwise, with `overlap`, they run on a side stream (their final reductions on
        a third) while the data gradients continue; both are joined before returning."""
        dt = self.dtype
        rb0, rb1 = lv.rb0, lv.rb1
        pending = {id(rb0): [], id(rb1): []}  # deferred weight gradients per rulebook
        main = torch.cuda.current_stream()
        side = side2 = None
        if overlap and not batch_wgrad:
            if getattr(self, "_side", None) is None:
                self._side, self._side2 = torch.cuda.Stream(), torch.cuda.Stream()
            side, side2 = self._side, self._side2
        in_use = []  # tensors the side streams read: alive until they are joined
        outs = {"stem": saved["stem"][1:] + [saved["enc0"][0]], "enc0": saved["enc0"][1:] + [saved["down"][0]],
                "enc1": saved["enc1"][1:] + [saved["up"][0]], "dec0": saved["dec0"][1:] + [saved["head"][0]],
                "head": [logits]}
        grads = {st: [None] * len(self.layers[st]) for st in STAGES}

        def subm_chain(st, dY, rb, last_is_head=False, want_dx=True):
            for i in range(len(self.layers[st]) - 1, -1, -1):
                _, _, cin, cout = self.layers[st][i]
                ws = conv_bwd_workspace(cin, cout, rb, dt)
                dX, dW, db = sparse_conv_bwd(saved[st][i], self._wt(st, i), cin, cout, outs[st][i], dY, rb, dt,
                                             relu=not last_is_head, want_dx=want_dx or i > 0, ws=ws,
                                             wgrad_stream=side, reduce_stream=side2, want_dw=not batch_wgrad)
                in_use.extend((ws, saved[st][i]))
                if batch_wgrad:
                    dev = dY.device
                    dW = torch.empty((27, cin, cout), dtype=torch.float32, device=dev)
                    db = torch.empty(cout, dtype=torch.float32, device=dev)
                    pending[id(rb)].append((saved[st][i], cin, cout, ws, dW, db))
                grads[st][i] = (dW, db)
                dY = dX
            return dY

        dH = subm_chain("head", dlogits, rb0, last_is_head=True)
        dH = subm_chain("dec0", dH, rb0)
        (_, _, E, Dc), = self.layers["up"]
        dU, _ = concat_channels_bwd(dH, Dc, E, rb0, want_b=False)
        dC, dW, db = strided_conv_bwd(saved["up"][0], self._wt("up", 0), E, Dc, saved["u"], dU, lv, up=True, dtype=dt)
        grads["up"][0] = (dW, db)
        dC = subm_chain("enc1", dC, rb1)
        (_, _, cin, cout), = self.layers["down"]
        dX0, dW, db = strided_conv_bwd(saved["down"][0], self._wt("down", 0), cin, cout, saved["enc1"][0], dC, lv,
                                       up=False, dtype=dt)
        grads["down"][0] = (dW, db)
        _, dS = concat_channels_bwd(dH, Dc, E, rb0, add_b=dX0, want_a=False)
        dS = subm_chain("enc0", dS, rb0)
        subm_chain("stem", dS, rb0, want_dx=False)
        for rb in (rb0, rb1):
            todo = pending[id(rb)]
            for j in range(0, len(todo), NPVS_MAX_WGRAD_LAYERS):
                sparse_conv_wgrad(todo[j:j + NPVS_MAX_WGRAD_LAYERS], rb, dt, wgrad_slices)
        if side is not None:
            main.wait_stream(side)
            main.wait_stream(side2)
        del in_use
        return grads


def unet_pvs(net: UNet, tris: torch.Tensor, n_tris, dims):
    """Triangles -> (pvs bits, logits rows, levels): froxelize, both levels' sites and rulebooks,
    the level maps, interleave, the U-Net, de-interleave + threshold."""
    occ = froxelize(tris, n_tris, dims)
    lv = build_levels(occ, dims, net.d)
    X0 = gather_input(occ, lv.rb0, net.dtype)
    logits = net.forward(X0, lv)
    pvs, _ = deinterleave_threshold(logits, lv.rb0, occ)
    return pvs, logits, lv, occ
