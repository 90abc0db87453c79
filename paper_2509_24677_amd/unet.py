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
The paper's adaptive relation convolutions and aggregators are not part of it.
"""
from __future__ import annotations

import torch

from . import (NPVS_BF16, NPVS_F32, Levels, build_levels, concat_channels, deinterleave_threshold, froxelize,
               gather_input, pack_weights, pack_weights_k, sparse_conv_fwd, strided_conv_fwd)

STAGES = ("stem", "enc0", "down", "enc1", "up", "dec0", "head")


class UNet:
    def __init__(self, params: dict, d: int, dtype: int = NPVS_BF16, device="cuda"):
        """params: {stage: [(W, b), ...]} with W float32 [27][cin][cout] (submanifold) or
        [8][cin][cout] (down, up) and b float32 [cout], as numpy or torch."""
        self.d = d
        self.dtype = dtype
        self.layers = {}
        for st in STAGES:
            out = []
            for W, b in params[st]:
                W = torch.as_tensor(W, dtype=torch.float32).to(device).contiguous()
                b = torch.as_tensor(b, dtype=torch.float32).to(device).contiguous()
                Wp = pack_weights_k(W, dtype) if W.shape[0] == 8 else pack_weights(W, dtype)
                out.append((Wp, b, W.shape[1], W.shape[2]))
            self.layers[st] = out
        (_, _, E, Dc), = self.layers["up"]
        if self.layers["dec0"][0][2] != Dc + E:
            raise ValueError("the first decoder layer must take the up output and the skip channels")

    def forward(self, X0: torch.Tensor, lv: Levels) -> torch.Tensor:
        """Logits float32 [rb0.cap][d^3] (rows past the level-0 count undefined)."""
        dt = self.dtype
        rb0, rb1 = lv.rb0, lv.rb1

        def subm(h, layer, rb, last=False):
            Wp, b, cin, cout = layer
            return sparse_conv_fwd(h, Wp, b, cin, cout, rb, dt, relu=not last, out_f32=last)

        h = X0
        for layer in self.layers["stem"] + self.layers["enc0"]:
            h = subm(h, layer, rb0)
        skip = h
        (Wp, b, cin, cout), = self.layers["down"]
        h1 = strided_conv_fwd(skip, Wp, b, cin, cout, lv, up=False, dtype=dt)
        for layer in self.layers["enc1"]:
            h1 = subm(h1, layer, rb1)
        (Wp, b, cin, cout), = self.layers["up"]
        u = strided_conv_fwd(h1, Wp, b, cin, cout, lv, up=True, dtype=dt)
        h = concat_channels(u, skip, rb0)
        for layer in self.layers["dec0"]:
            h = subm(h, layer, rb0)
        return subm(h, self.layers["head"][0], rb0, last=True)


def unet_pvs(net: UNet, tris: torch.Tensor, n_tris, dims):
    """Triangles -> (pvs bits, logits rows, levels): froxelize, both levels' sites and rulebooks,
    the level maps, interleave, the U-Net, de-interleave + threshold."""
    occ = froxelize(tris, n_tris, dims)
    lv = build_levels(occ, dims, net.d)
    X0 = gather_input(occ, lv.rb0, net.dtype)
    logits = net.forward(X0, lv)
    pvs, _ = deinterleave_threshold(logits, lv.rb0, occ)
    return pvs, logits, lv, occ
