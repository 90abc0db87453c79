"""Forward/backward driver of the visibility network over the C ABI.

* ``Network``: float32 master weights, their packed forms for the kernels (re-packed after every
  optimizer step), the forward stack (ReLU after every layer but the last) with optional
  activation checkpointing: only every second layer input is kept and the others are recomputed
  in the backward.
* ``Trainer``: one training step on a batch of grids: froxelize, rulebook, forward, de-interleave
  + threshold, BCE + repulsive visibility loss (Sec. 3.3), hand-written backward and Adam.  Every
  step runs entirely on one stream without host synchronization, so it can be captured in a graph.
* ``SubMConvFn``: the same layer as a ``torch.autograd.Function`` for callers that want autograd.

The loss weight lambda = 0.99, the learning rate 1e-3 and the decay 1e-10 (read as weight decay)
follow Sec. 4.2.
"""
from __future__ import annotations

import torch

from . import _lib as L
from . import (NPVS_BF16, NPVS_F32, NPVS_U8, Rulebook, adam, build_rulebook, conv_bwd_workspace,
               deinterleave_threshold, froxelize, gather_input, loss, pack_weights, pack_weights_batch, sparse_conv_bwd,
               sparse_conv_dgrad_relu, sparse_conv_fwd, sparse_conv_wgrad)


class Network:
    def __init__(self, layers, d: int, dtype: int = NPVS_BF16, device="cuda"):
        """layers: list of (W float32 [27][cin][cout], b float32 [cout]) as numpy or torch."""
        self.d = d
        self.dtype = dtype
        Ws = [torch.as_tensor(W, dtype=torch.float32) for W, _ in layers]
        bs = [torch.as_tensor(b, dtype=torch.float32) for _, b in layers]
        # all parameters (and their gradients) live in one flat buffer, so one optimizer launch
        # updates every layer; W[i], b[i], gW[i], gb[i] are views into it
        sizes = [w.numel() for w in Ws] + [b.numel() for b in bs]
        self.flat = torch.empty(sum(sizes), dtype=torch.float32, device=device)
        self.gflat = torch.zeros_like(self.flat)
        views, gviews, off = [], [], 0
        for t, n in zip(Ws + bs, sizes):
            views.append(self.flat[off:off + n].view(t.shape))
            gviews.append(self.gflat[off:off + n].view(t.shape))
            views[-1].copy_(t)
            off += n
        L = len(Ws)
        self.W, self.b = views[:L], views[L:]
        self.gW, self.gb = gviews[:L], gviews[L:]
        self.channels = [self.W[0].shape[1]] + [w.shape[2] for w in self.W]
        self.Wp = [None] * len(self.W)
        self.Wt = [None] * len(self.W)
        self.variant = [None] * len(self.W)  # BF16 tile shape per layer (None = library default)
        self.repack()

    @property
    def n_layers(self):
        return len(self.W)

    def pack_descs(self):
        """[(offset in the flat buffer, cin, cout, Wp, Wt)] per layer, for the optimizer step that
        writes the packings itself."""
        out, off = [], 0
        for i, W in enumerate(self.W):
            out.append((off, W.shape[1], W.shape[2], self.Wp[i], self.Wt[i]))
            off += W.numel()
        return out

    def repack(self):
        """Packs every layer for the forward and the data-gradient convolutions in one launch,
        in place, so captured graphs keep reading the current weights."""
        for i, W in enumerate(self.W):
            if self.Wp[i] is None:
                nbytes = L.get().npvs_packed_weight_bytes(W.shape[1], W.shape[2], self.dtype)
                self.Wp[i] = torch.empty(nbytes, dtype=torch.uint8, device=W.device)
                self.Wt[i] = torch.empty(nbytes, dtype=torch.uint8, device=W.device)
        items = [(W, self.Wp[i], False) for i, W in enumerate(self.W)]
        items += [(W, self.Wt[i], True) for i, W in enumerate(self.W)]
        for j in range(0, len(items), L.NPVS_MAX_PACK):
            pack_weights_batch(items[j:j + L.NPVS_MAX_PACK], self.dtype)

    def layer(self, i: int, X: torch.Tensor, rb: Rulebook) -> torch.Tensor:
        last = i == self.n_layers - 1
        return sparse_conv_fwd(X, self.Wp[i], self.b[i], self.channels[i], self.channels[i + 1], rb, self.dtype,
                               relu=not last, out_f32=last, variant=self.variant[i])

    def autotune(self, X0: torch.Tensor, rb: Rulebook, reps: int = 20, margin: float = 0.03):
        """Times every BF16 tile shape of each distinct layer shape on the rulebook `rb` (HIP events
        on the current stream) and keeps the fastest; the library's default shape is kept unless
        another one is faster by more than `margin` (so that timing noise does not flip the choice
        between shapes of equal speed from run to run).  Synchronizes."""
        if self.dtype != NPVS_BF16:
            return self.variant
        from ._lib import NPVS_CONV_VARIANTS
        chosen = {}
        X = X0
        for i in range(self.n_layers):
            last = i == self.n_layers - 1
            key = (self.channels[i], self.channels[i + 1], last)
            if key not in chosen:
                out = self.layer(i, X, rb)
                best = None
                for v in range(NPVS_CONV_VARIANTS):
                    self.variant[i] = v
                    self.layer(i, X, rb)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):
                        sparse_conv_fwd(X, self.Wp[i], self.b[i], self.channels[i], self.channels[i + 1], rb,
                                        self.dtype, relu=not last, out_f32=last, out=out, variant=v)
                    e1.record()
                    e1.synchronize()
                    t = e0.elapsed_time(e1)
                    if v == L.NPVS_DEFAULT_CONV_VARIANT:
                        t_default = t
                    if best is None or t < best[0]:
                        best = (t, v)
                chosen[key] = best[1] if best[0] < (1.0 - margin) * t_default else L.NPVS_DEFAULT_CONV_VARIANT
            self.variant[i] = chosen[key]
            X = self.layer(i, X, rb)
        torch.cuda.synchronize()
        return list(self.variant)

    def forward(self, X0: torch.Tensor, rb: Rulebook, checkpoint: bool = False):
        """Returns (logits float32 [cap][d^3], saved inputs: dict layer -> input tensor)."""
        saved = {}
        X = X0
        for i in range(self.n_layers):
            if not checkpoint or i % 2 == 0:
                saved[i] = X
            X = self.layer(i, X, rb)
        return X, saved

    def backward(self, saved, logits: torch.Tensor, dlogits: torch.Tensor, rb: Rulebook, overlap: bool = True,
                 batch_wgrad: bool | None = None, wgrad_slices: int = 0, chain: bool | None = None,
                 top_ws: torch.Tensor | None = None):
        """Hand-written backward through the stack; recomputes the layer inputs that were not
        saved.  With `batch_wgrad` (default: for BF16, whose weight gradients are short
        latency-bound launches), the data gradients run down the stack first, all on the current
        stream, and the weight gradients of every layer follow in one launch (and one reduction
        launch; `wgrad_slices` pair-list slices per offset, 0 for the library's choice); there,
        with `chain` (default: wherever the layers allow it, see _chainable) each data gradient
        also forms the dZ of the layer below in its epilogue (npvs_sparse_conv_dgrad_relu), so no
        separate ReLU' pass runs between them (`top_ws`: the last layer's backward workspace, into
        which the loss already wrote that layer's dZ, see loss(dz_ws=...); dlogits is then unused).
        Otherwise (the FP32 default) each layer's weight gradient follows its data gradient:
        with `overlap` on a side stream while the data gradient continues down the stack (their
        final reductions on a third stream, beside the next weight gradient; the side streams
        are joined before returning).  The gradients land in the flat gradient buffer; returns
        [(dW, db)] per layer (views of it)."""
        batch_wgrad, chain = self.backward_form(batch_wgrad, chain)
        if top_ws is not None and not self.loss_forms_top_dz(batch_wgrad):
            raise ValueError("top_ws is for the chained backward with a fusable last layer")
        if batch_wgrad:
            return self._backward_batched(saved, logits, dlogits, rb, wgrad_slices, chain, top_ws)
        main = torch.cuda.current_stream()
        side = side2 = None
        if overlap:
            if getattr(self, "_side", None) is None:
                self._side, self._side2 = torch.cuda.Stream(), torch.cuda.Stream()
            side, side2 = self._side, self._side2
        grads = [None] * self.n_layers
        outputs = {self.n_layers - 1: logits}
        in_use = []  # tensors the side stream reads: alive until it is joined
        dY = dlogits
        for i in range(self.n_layers - 1, -1, -1):
            X = saved.get(i)
            if X is None:  # recompute this layer's input from the previous saved one
                X = self.layer(i - 1, saved[i - 1], rb)
            Y = outputs.get(i)
            if Y is None:
                Y = self.layer(i, X, rb)
            ws = conv_bwd_workspace(self.channels[i], self.channels[i + 1], rb, self.dtype)
            dX, dW, db = sparse_conv_bwd(X, self.Wt[i], self.channels[i], self.channels[i + 1], Y, dY, rb,
                                         self.dtype, relu=i < self.n_layers - 1, want_dx=i > 0,
                                         dW=self.gW[i], db=self.gb[i], ws=ws, wgrad_stream=side,
                                         reduce_stream=side2)
            in_use += [X, ws]
            grads[i] = (dW, db)
            if i > 0:
                outputs[i - 1] = X
            dY = dX
        if side is not None:
            main.wait_stream(side)
            main.wait_stream(side2)
        del in_use
        return grads

    def backward_form(self, batch_wgrad: bool | None = None, chain: bool | None = None):
        """(batch_wgrad, chain) as backward() resolves them."""
        if batch_wgrad is None:
            batch_wgrad = self.dtype == NPVS_BF16
        if not batch_wgrad:
            return False, False
        if chain is None:
            chain = self._chainable()
        elif chain and not self._chainable():
            raise ValueError("the chained backward needs BF16 layers of at most 64 channels above the first")
        return True, chain

    def _fusable(self, i: int) -> bool:
        """Layer i's data gradient can form the dZ of layer i - 1 in its epilogue
        (npvs_sparse_conv_dgrad_relu): BF16, at most 64 channels in and out, and the layer below
        can take that dZ in place (it is fusable itself, or it is the first layer, which needs no
        data gradient): the fused layers are a run from layer 1 upward."""
        ch = self.channels
        if self.dtype != NPVS_BF16 or i < 1 or ch[0] % 8:
            return False
        return all(max(ch[j], ch[j + 1]) <= 64 and ch[j + 1] % 8 == 0 for j in range(1, i + 1))

    def _chainable(self) -> bool:
        """Some layer's data gradient can be fused (see _fusable)."""
        return any(self._fusable(i) for i in range(1, self.n_layers))

    def loss_forms_top_dz(self, batch_wgrad: bool | None = None) -> bool:
        """The loss may write the last layer's dZ into its workspace (backward(top_ws=...)): the
        chained form runs and the last layer's data gradient is fused."""
        _, chain = self.backward_form(batch_wgrad)
        top = self.n_layers - 1
        return chain and (top == 0 or self._fusable(top)) and self.channels[top + 1] % 8 == 0

    def _backward_batched(self, saved, logits, dlogits, rb, slices, chain, top_ws=None):
        if chain:
            return self._backward_chained(saved, logits, dlogits, rb, slices, top_ws)
        outputs = {self.n_layers - 1: logits}
        pending = []  # (X, cin, cout, ws, dW, db) of each layer, for the batched weight gradient
        dY = dlogits
        for i in range(self.n_layers - 1, -1, -1):
            X = saved.get(i)
            if X is None:
                X = self.layer(i - 1, saved[i - 1], rb)
            Y = outputs.get(i)
            if Y is None:
                Y = self.layer(i, X, rb)
            cin, cout = self.channels[i], self.channels[i + 1]
            ws = conv_bwd_workspace(cin, cout, rb, self.dtype)
            dX, _, _ = sparse_conv_bwd(X, self.Wt[i], cin, cout, Y, dY, rb, self.dtype, relu=i < self.n_layers - 1,
                                       want_dx=i > 0, ws=ws, want_dw=False)
            pending.append((X, cin, cout, ws, self.gW[i], self.gb[i]))
            if i > 0:
                outputs[i - 1] = X
            dY = dX
        sparse_conv_wgrad(pending, rb, self.dtype, slices)
        return [(self.gW[i], self.gb[i]) for i in range(self.n_layers)]

    def _backward_chained(self, saved, logits, dlogits, rb, slices, top_ws=None):
        """Down the stack, each layer whose data gradient is fusable (_fusable) runs it with the
        ReLU' of the layer below fused in, writing that layer's dZ and bias partials straight
        into its workspace; any other layer forms its dZ from the float32 gradient of the layer
        above and, when the layer below needs one, its float32 data gradient as usual.  Then
        every weight gradient at once."""
        top, ch = self.n_layers - 1, self.channels
        inputs = {}

        def layer_input(i):
            if i not in inputs:
                inputs[i] = saved[i] if i in saved else self.layer(i - 1, saved[i - 1], rb)
            return inputs[i]

        ws = [conv_bwd_workspace(ch[i], ch[i + 1], rb, self.dtype) if i < top or top_ws is None else top_ws
              for i in range(self.n_layers)]
        dY = dlogits  # float32 gradient of layer i's output, when its dZ is not in ws[i] yet
        have_dz = top_ws is not None
        for i in range(top, -1, -1):
            fuse = i > 0 and self._fusable(i)
            if not have_dz:
                Y = logits if i == top else layer_input(i + 1)
                dX, _, _ = sparse_conv_bwd(layer_input(i), self.Wt[i], ch[i], ch[i + 1], Y, dY, rb, self.dtype,
                                           relu=i < top, want_dx=i > 0 and not fuse, ws=ws[i], want_dw=False)
            if fuse:
                sparse_conv_dgrad_relu(self.Wt[i], ch[i], ch[i + 1], layer_input(i), ch[i - 1], rb, ws[i], ws[i - 1])
                have_dz = True
            else:
                if have_dz and i > 0:
                    raise RuntimeError("a layer whose dZ is formed in place needs a fusable data gradient")
                have_dz, dY = False, (dX if i > 0 else None)
        layer_input(0)
        pending = [(inputs[i], ch[i], ch[i + 1], ws[i], self.gW[i], self.gb[i]) for i in range(top, -1, -1)]
        sparse_conv_wgrad(pending, rb, self.dtype, slices)
        return [(self.gW[i], self.gb[i]) for i in range(self.n_layers)]


class Trainer:
    """One training step per call; all state lives on the device."""

    def __init__(self, net: Network, dims, n_tris, lam: float = 0.99, lr: float = 1e-3, weight_decay: float = 1e-10,
                 checkpoint: bool = True, dice_alpha: float | None = None, batch_wgrad: bool | None = None):
        """dice_alpha: train on the paper's weighted Dice term (with that alpha) instead of BCE;
        batch_wgrad: the backward's weight gradients in one launch after the data gradients, or
        per layer on side streams (None: as Network.backward chooses for the precision)."""
        self.net = net
        self.dice_alpha = dice_alpha
        self.dims = [tuple(g) for g in dims]
        self.n_tris = list(n_tris)
        self.lam, self.lr, self.wd = lam, lr, weight_decay
        self.checkpoint = checkpoint
        self.batch_wgrad = batch_wgrad
        self.m = torch.zeros_like(net.flat)
        self.v = torch.zeros_like(net.flat)
        self.adam_step = torch.zeros(16, dtype=torch.uint8, device=net.flat.device)  # npvs_adam_step, t = 0
        self.step_count = 0  # host mirror of the device counter (eager calls only)

    def step(self, tris: torch.Tensor, label_bits: torch.Tensor):
        net = self.net
        occ = froxelize(tris, self.n_tris, self.dims)
        rb = build_rulebook(occ, self.dims, net.d, csr=True)
        X0, labels = gather_input(occ, rb, net.dtype, width=net.channels[0], bits2=label_bits)  # one launch
        logits, saved = net.forward(X0, rb, checkpoint=self.checkpoint)
        pvs, _ = deinterleave_threshold(logits, rb, occ)
        if net.loss_forms_top_dz(self.batch_wgrad):  # the loss forms the last layer's dZ in its workspace
            top = net.n_layers - 1
            top_ws = conv_bwd_workspace(net.channels[top], net.channels[top + 1], rb, net.dtype)
            stats, dl = loss(logits, labels, rb, self.lam, want_grad=False, dice_alpha=self.dice_alpha,
                             dz_ws=top_ws, dz_cin=net.channels[top])
            net.backward(saved, logits, dl, rb, batch_wgrad=self.batch_wgrad, top_ws=top_ws)
        else:
            stats, dl = loss(logits, labels, rb, self.lam, dice_alpha=self.dice_alpha)
            net.backward(saved, logits, dl, rb, batch_wgrad=self.batch_wgrad)  # gradients land in net.gflat
        self.step_count += 1
        # Adam, writing the updated weights straight into both packings of every layer
        adam(net.flat, net.gflat, self.m, self.v, self.adam_step, net.pack_descs(), net.dtype, lr=self.lr,
                      weight_decay=self.wd)
        return stats, pvs


class SubMConvFn(torch.autograd.Function):
    """Y = act(b + sum_k gather_k(X) W_k) over a rulebook (built with csr=True), differentiable in
    X, W and b through the hand-written backward.  Rows of dX past the active sites are left
    undefined, as are those of Y."""

    @staticmethod
    def forward(ctx, X, W, b, rb: Rulebook, dtype: int, relu: bool, out_f32: bool):
        Wp = pack_weights(W.detach(), dtype)
        Y = sparse_conv_fwd(X.detach(), Wp, b.detach(), W.shape[1], W.shape[2], rb, dtype, relu, out_f32)
        ctx.save_for_backward(X, W, Y)
        ctx.rb, ctx.dtype, ctx.relu = rb, dtype, relu
        return Y

    @staticmethod
    def backward(ctx, dY):
        X, W, Y = ctx.saved_tensors
        Wt = pack_weights(W.detach(), ctx.dtype, flip_transpose=True)
        dX, dW, db = sparse_conv_bwd(X.detach(), Wt, W.shape[1], W.shape[2], Y, dY.float().contiguous(), ctx.rb,
                                     ctx.dtype, ctx.relu, want_dx=ctx.needs_input_grad[0])
        if dX is not None and X.dtype != torch.float32:
            dX = dX.to(X.dtype)
        return dX, dW, db, None, None, None, None
