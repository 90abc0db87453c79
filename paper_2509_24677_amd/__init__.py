"""NeuralPVS hot path on MI355X (gfx950): Python binding of ``libneuralpvs.so``.

Every function here marshals torch tensors (device memory) and the current HIP stream into one
call of the C ABI declared in ``include/neuralpvs.h``; all computation runs in the library's
HIP kernels.  There is no CPU fallback: calls raise if the library is not built.

Stages (paper: NeuralPVS, arXiv 2509.24677):
  froxelize (Sec. 3.2) -> build_rulebook (Sec. 2.3 submanifold sites) -> gather_input
  (g_d of Sec. 3.3 on the active sites) -> sparse_conv_fwd x L -> deinterleave_threshold
  (g_d^-1 and V = 1[f >= tau], Sec. 3.1).  Plan runs them all as one stream of launches.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L
from ._lib import NPVS_BF16, NPVS_CONV_VARIANTS, NPVS_F32, NPVS_U8, NpvsError  # noqa: F401

__all__ = [
    "froxelize", "build_rulebook", "gather_input", "interleave", "deinterleave", "pack_weights",
    "sparse_conv_fwd", "sparse_conv_bwd", "sparse_conv_wgrad", "sparse_conv_dgrad_relu", "Levels", "build_levels",
    "pack_weights_k", "strided_conv_fwd", "concat_channels", "viewcell_frustum", "froxelize_view", "deinterleave_threshold", "loss", "adam", "Plan", "Rulebook",
    "NpvsError", "NPVS_F32", "NPVS_BF16", "NPVS_U8", "version",
]

_TORCH_DT = {NPVS_F32: torch.float32, NPVS_BF16: torch.bfloat16, NPVS_U8: torch.uint8}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _dev():
    return torch.device("cuda", torch.cuda.current_device())


def version() -> str:
    return L.get().npvs_version().decode()


def batch_sizes(dims, d: int):
    tb, tby = ctypes.c_int64(), ctypes.c_int64()
    L.call("npvs_batch_sizes", len(dims), L.dims_array(dims), d, ctypes.byref(tb), ctypes.byref(tby))
    return tb.value, tby.value


# --------------------------------------------------------------------------------- froxelize
def froxelize(tris: torch.Tensor, n_tris, dims, occ: torch.Tensor | None = None,
              n_ignored: torch.Tensor | None = None) -> torch.Tensor:
    """Packed occupancy bits of a batch of grids (uint8, grids back to back).

    tris: float32 device tensor [sum T][3][3] in grid units; n_tris: triangles per grid;
    n_ignored (optional): int32 device tensor of one element that receives the number of
    ignored triangles (a non-finite coordinate or |coordinate| >= 2048)."""
    dims = [tuple(g) for g in dims]
    n_tris = [int(t) for t in n_tris]
    tris = tris.contiguous()
    if tris.dtype != torch.float32 or tris.numel() != 9 * sum(n_tris):
        raise ValueError("tris must be float32 [sum n_tris][3][3]")
    darr, tarr = L.dims_array(dims), L.i64_array(n_tris)
    nbytes = ctypes.c_size_t()
    L.call("npvs_froxelize_workspace_size", len(dims), darr, tarr, ctypes.byref(nbytes))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=_dev())
    _, total_bytes = batch_sizes(dims, 1)
    if occ is None:
        occ = torch.empty(total_bytes, dtype=torch.uint8, device=_dev())
    elif occ.numel() != total_bytes or occ.dtype != torch.uint8:
        raise ValueError("occ must be uint8 with one byte per 8 froxels")
    if n_ignored is not None and (n_ignored.dtype != torch.int32 or n_ignored.numel() < 1):
        raise ValueError("n_ignored must be an int32 tensor of at least one element")
    L.call("npvs_froxelize", _p(tris) if tris.numel() else None, tarr, len(dims), darr, _p(occ),
           _p(n_ignored) if n_ignored is not None else None, _p(ws), nbytes.value, _stream())
    return occ


# --------------------------------------------------------------------------------- rulebook
@dataclass
class Rulebook:
    dims: list
    d: int
    cap: int
    counts: torch.Tensor      # int32 [4] device (npvs_counts)
    site_keys: torch.Tensor   # int32 [cap]
    block_row: torch.Tensor   # int32 [total_blocks]
    grid_rows: torch.Tensor   # int32 [n_grids + 1]
    nbr: torch.Tensor         # int32 [27][cap]
    rb_off: torch.Tensor | None = None    # int32 [28]
    rb_pairs: torch.Tensor | None = None  # int32 [27 cap][2]

    def host_counts(self) -> dict:
        c = self.counts.cpu().tolist()
        return dict(n_sites=c[0], n_sites_needed=c[1], n_pairs=c[2])


def build_rulebook(occ: torch.Tensor, dims, d: int, cap: int | None = None, csr: bool = False,
                   out: Rulebook | None = None, noalloc: bool = False) -> Rulebook:
    """Active sites, site table, neighbour map and (csr) the per-offset pair lists.  `out`: a
    Rulebook of the same dims, d, cap and form to write into.  noalloc: the library's
    workspace-free entry point (npvs_build_rulebook_noalloc), which allocates no device memory."""
    dims = [tuple(g) for g in dims]
    total_blocks, _ = batch_sizes(dims, d)
    cap = total_blocks if cap is None else int(cap)
    darr = L.dims_array(dims)
    dev = _dev()
    if out is not None and (out.dims != dims or out.d != d or out.cap != cap or (out.rb_off is not None) != csr):
        raise ValueError("out: a Rulebook of other dims, d, capacity or form")
    rb = out if out is not None else _new_rulebook(dims, d, cap, total_blocks, csr, dev)
    if noalloc:
        L.call("npvs_build_rulebook_noalloc", _p(occ), len(dims), darr, d, cap, _p(rb.counts), _p(rb.site_keys),
               _p(rb.block_row), _p(rb.grid_rows), _p(rb.nbr), _p(rb.rb_off), _p(rb.rb_pairs), _stream())
        return rb
    nbytes = ctypes.c_size_t()
    L.call("npvs_rulebook_workspace_size", len(dims), darr, d, cap, ctypes.byref(nbytes))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    L.call("npvs_build_rulebook", _p(occ), len(dims), darr, d, cap, _p(rb.counts), _p(rb.site_keys),
           _p(rb.block_row), _p(rb.grid_rows), _p(rb.nbr), _p(rb.rb_off), _p(rb.rb_pairs), _p(ws), nbytes.value,
           _stream())
    return rb


def _new_rulebook(dims, d, cap, total_blocks, csr, dev) -> Rulebook:
    rb = Rulebook(dims, d, cap,
                  torch.empty(4, dtype=torch.int32, device=dev),
                  torch.empty(cap, dtype=torch.int32, device=dev),
                  torch.empty(total_blocks, dtype=torch.int32, device=dev),
                  torch.empty(len(dims) + 1, dtype=torch.int32, device=dev),
                  torch.empty((27, cap), dtype=torch.int32, device=dev))
    if csr:
        rb.rb_off = torch.empty(28, dtype=torch.int32, device=dev)
        rb.rb_pairs = torch.empty((27 * cap, 2), dtype=torch.int32, device=dev)
    return rb


# --------------------------------------------------------------------------------- interleave
def gather_input(bits: torch.Tensor, rb: Rulebook, dtype: int = NPVS_F32, out: torch.Tensor | None = None,
                 width: int | None = None, bits2: torch.Tensor | None = None):
    """Sparse g_d: [cap][width] 0/1 values of `bits` on the active sites, width d^3 by default;
    channels d^3 .. width - 1 are zero (a BF16 input of fewer than 8 channels is given width 8).
    Rows >= n_sites are left as allocated.  With `bits2` (a second bit grid of the same grids),
    returns (out, out2): out2 uint8 [cap][d^3] its values, gathered in the same launch."""
    C = rb.d ** 3
    width = C if width is None else int(width)
    if out is None:
        out = torch.empty((rb.cap, width), dtype=_TORCH_DT[dtype], device=_dev())
    elif out.shape[-1] != width:
        raise ValueError("out must have `width` elements per row")
    out2 = None if bits2 is None else torch.empty((rb.cap, C), dtype=torch.uint8, device=_dev())
    L.call("npvs_gather_input", _p(bits), len(rb.dims), L.dims_array(rb.dims), rb.d, _p(rb.site_keys),
           _p(rb.counts), rb.cap, dtype, width, _p(out), _p(bits2), _p(out2), _stream())
    return out if bits2 is None else (out, out2)


def _dense_out(out, shape, x):
    if out is None:
        return torch.empty(shape, dtype=x.dtype, device=x.device)
    if out.dtype != x.dtype or out.device != x.device or not out.is_contiguous() or out.numel() != x.numel():
        raise ValueError("out must be a contiguous tensor of x's dtype, device and size")
    return out


def interleave(x: torch.Tensor, d: int, out: torch.Tensor = None) -> torch.Tensor:
    """Dense g_d of a [nz][ny][nx] tensor -> [nz/d][ny/d][nx/d][d^3] (written into `out` if given)."""
    x = x.contiguous()
    nz, ny, nx = x.shape
    out = _dense_out(out, (nz // d, ny // d, nx // d, d ** 3), x)
    L.call("npvs_interleave", _p(x), L.Dims(nx, ny, nz), d, x.element_size(), _p(out), _stream())
    return out


def deinterleave(x: torch.Tensor, dims, d: int, out: torch.Tensor = None) -> torch.Tensor:
    """Inverse of interleave: [nz/d][ny/d][nx/d][d^3] -> [nz][ny][nx] for dims (nx, ny, nz)."""
    x = x.contiguous()
    nx, ny, nz = dims
    out = _dense_out(out, (nz, ny, nx), x)
    L.call("npvs_deinterleave", _p(x), L.Dims(nx, ny, nz), d, x.element_size(), _p(out), _stream())
    return out


# --------------------------------------------------------------------------------- convolution
def pack_weights(W: torch.Tensor, dtype: int, flip_transpose: bool = False) -> torch.Tensor:
    """Kernel layout of float32 weights [27][cin][cout] (uint8 byte tensor)."""
    W = W.contiguous()
    if W.dtype != torch.float32 or W.dim() != 3 or W.shape[0] != 27:
        raise ValueError("W must be float32 [27][cin][cout]")
    cin, cout = W.shape[1], W.shape[2]
    nbytes = L.get().npvs_packed_weight_bytes(cin, cout, dtype)
    Wp = torch.empty(nbytes, dtype=torch.uint8, device=W.device)
    L.call("npvs_pack_weights", _p(W), cin, cout, dtype, int(flip_transpose), _p(Wp), _stream())
    return Wp


def pack_weights_batch(items, dtype: int):
    """Packs several weights in one launch: items = [(W float32 [27][cin][cout], Wp uint8 output,
    flip_transpose)], every Wp of npvs_packed_weight_bytes(cin, cout, dtype) bytes, written in place."""
    n = len(items)
    if n > L.NPVS_MAX_PACK:
        raise ValueError(f"at most {L.NPVS_MAX_PACK} packings per call")
    descs = (L.PackDesc * max(n, 1))()
    for i, (W, Wp, flip) in enumerate(items):
        if W.dtype != torch.float32 or W.dim() != 3 or W.shape[0] != 27 or not W.is_contiguous():
            raise ValueError("W must be contiguous float32 [27][cin][cout]")
        cin, cout = W.shape[1], W.shape[2]
        if Wp.numel() * Wp.element_size() != L.get().npvs_packed_weight_bytes(cin, cout, dtype):
            raise ValueError("Wp has the wrong size")
        descs[i] = L.PackDesc(_p(W), _p(Wp), cin, cout, int(flip), 0)
    L.call("npvs_pack_weights_batch", n, ctypes.cast(descs, ctypes.c_void_p), dtype, _stream())


def sparse_conv_fwd(X: torch.Tensor, Wp: torch.Tensor, bias: torch.Tensor | None, cin: int, cout: int,
                    rb: Rulebook, dtype: int, relu: bool, out_f32: bool = False,
                    out: torch.Tensor | None = None, variant: int | None = None) -> torch.Tensor:
    """One submanifold layer; `variant` selects the BF16 tile shape (None = library default)."""
    if out is None:
        odt = torch.float32 if (dtype == NPVS_F32 or out_f32) else torch.bfloat16
        out = torch.empty((rb.cap, cout), dtype=odt, device=X.device)
    nbytes = ctypes.c_size_t()
    L.call("npvs_conv_fwd_workspace_size", cin, cout, rb.cap, dtype, ctypes.byref(nbytes))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=X.device) if nbytes.value else None
    L.call("npvs_sparse_conv_fwd", _p(X), cin, _p(Wp), _p(bias), cout, _p(rb.nbr), _p(rb.counts), rb.cap, dtype,
           int(relu), int(out_f32), int(variant) if variant is not None else -1, _p(out), _p(ws), nbytes.value,
           _stream())
    return out


def conv_bwd_workspace(cin: int, cout: int, rb: Rulebook, dtype: int) -> torch.Tensor:
    nbytes = ctypes.c_size_t()
    L.call("npvs_conv_bwd_workspace_size", cin, cout, rb.cap, dtype, ctypes.byref(nbytes))
    return torch.empty(nbytes.value, dtype=torch.uint8, device=rb.nbr.device)


def sparse_conv_bwd(X, Wt, cin: int, cout: int, Y, dY, rb: Rulebook, dtype: int, relu: bool, want_dx: bool = True,
                    dW: torch.Tensor | None = None, db: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                    wgrad_stream: torch.cuda.Stream | None = None, reduce_stream: torch.cuda.Stream | None = None,
                    want_dw: bool = True):
    """Returns (dX float32 [cap][cin] or None, dW float32 [27][cin][cout], db float32 [cout]).
    dW / db may be given (contiguous float32 device tensors) to receive the gradients in place.
    With `wgrad_stream`, dW and db are computed on that stream, and with `reduce_stream` too their
    final reductions on that one: the caller keeps X and ws alive and joins the streams before
    reading dW / db.  With want_dw=False, dW and db are not computed (returned as None): dZ and
    the bias partials stay in `ws` (which must be given) for `sparse_conv_wgrad`."""
    if rb.rb_off is None:
        raise ValueError("the backward needs a rulebook built with csr=True")
    dev = X.device
    if ws is None:
        if not want_dw:
            raise ValueError("want_dw=False needs the workspace that sparse_conv_wgrad will read")
        ws = conv_bwd_workspace(cin, cout, rb, dtype)
        for side in (wgrad_stream, reduce_stream):  # freed here, still read by the side streams
            if side is not None:
                ws.record_stream(side)
    dX = torch.empty((rb.cap, cin), dtype=torch.float32, device=dev) if want_dx else None
    if not want_dw:
        dW = db = None
    else:
        if dW is None:
            dW = torch.empty((27, cin, cout), dtype=torch.float32, device=dev)
        if db is None:
            db = torch.empty(cout, dtype=torch.float32, device=dev)
        _check_grad_out(dW, db, cin, cout)
    side = [ctypes.c_void_p(t.cuda_stream) if t is not None else None for t in (wgrad_stream, reduce_stream)]
    L.call("npvs_sparse_conv_bwd", _p(X), cin, _p(Wt), cout, _p(Y), _p(dY.contiguous()), _p(rb.nbr), _p(rb.rb_off),
           _p(rb.rb_pairs), _p(rb.counts), rb.cap, dtype, int(relu), _p(dX), _p(dW), _p(db), _p(ws), ws.numel(),
           _stream(), side[0], side[1])
    return dX, dW, db


def _check_grad_out(dW, db, cin: int, cout: int):
    if dW.numel() != 27 * cin * cout or db.numel() != cout or not (dW.is_contiguous() and db.is_contiguous()):
        raise ValueError("dW / db must be contiguous float32 [27][cin][cout] / [cout]")


def sparse_conv_dgrad_relu(Wt, cin: int, cout: int, M, cin_below: int, rb: Rulebook, ws: torch.Tensor,
                           ws_below: torch.Tensor):
    """BF16 data gradient of a layer (cin -> cout) from the dZ its backward workspace `ws` holds,
    fused with the ReLU' of the layer below (M: that layer's output, this layer's input; None: no
    mask): writes the layer below's dZ and bias partials into `ws_below` (that layer's backward
    workspace, cin_below -> cin channels), ready for another sparse_conv_dgrad_relu and for
    sparse_conv_wgrad."""
    L.call("npvs_sparse_conv_dgrad_relu", _p(Wt), cin, cout, _p(M), cin_below, _p(rb.nbr), _p(rb.counts), rb.cap,
           _p(ws), ws.numel(), _p(ws_below), ws_below.numel(), _stream())


def sparse_conv_wgrad(layers, rb: Rulebook, dtype: int, slices: int = 0):
    """Weight and bias gradients of several layers of rulebook `rb` in one launch: `layers` is a
    list of (X, cin, cout, ws, dW, db), ws being the workspace of that layer's
    sparse_conv_bwd(..., want_dw=False) call; dW / db (contiguous float32 [27][cin][cout] /
    [cout]) are overwritten.  slices: pair-list slices per offset (0: the library's choice)."""
    if rb.rb_off is None:
        raise ValueError("the weight gradient needs a rulebook built with csr=True")
    if not 1 <= len(layers) <= L.NPVS_MAX_WGRAD_LAYERS:
        raise ValueError(f"1 to {L.NPVS_MAX_WGRAD_LAYERS} layers")
    arr = (L.WgradLayer * len(layers))()
    for i, (X, cin, cout, ws, dW, db) in enumerate(layers):
        _check_grad_out(dW, db, cin, cout)
        arr[i] = L.WgradLayer(X.data_ptr(), cin, cout, ws.data_ptr(), ws.numel(), dW.data_ptr(), db.data_ptr())
    L.call("npvs_sparse_conv_wgrad", len(layers), ctypes.cast(arr, ctypes.c_void_p), _p(rb.rb_off), _p(rb.rb_pairs),
           rb.cap, dtype, slices, _stream())


# --------------------------------------------------------------------------------- U-Net levels
@dataclass
class Levels:
    """Two levels of a sparse U-Net: rb0 at interleave factor d, rb1 at 2d, and the maps between
    them (children int32 [8][rb1.cap], parent int32 [rb0.cap] = 8 * level-1 row + child index)."""
    rb0: Rulebook
    rb1: Rulebook
    children: torch.Tensor
    parent: torch.Tensor


def build_levels(occ: torch.Tensor, dims, d: int, csr: bool = False) -> Levels:
    dims = [tuple(g) for g in dims]
    rb0 = build_rulebook(occ, dims, d, csr=csr)
    rb1 = build_rulebook(occ, dims, 2 * d, csr=csr)
    dev = occ.device
    children = torch.empty((8, rb1.cap), dtype=torch.int32, device=dev)
    parent = torch.empty(rb0.cap, dtype=torch.int32, device=dev)
    L.call("npvs_level_maps", len(dims), L.dims_array(dims), d, _p(rb0.counts), _p(rb0.site_keys), _p(rb0.block_row),
           rb0.cap, _p(rb1.counts), _p(rb1.site_keys), _p(rb1.block_row), rb1.cap, _p(children), _p(parent),
           _stream())
    return Levels(rb0, rb1, children, parent)


def pack_weights_k(W: torch.Tensor, dtype: int, transpose: bool = False) -> torch.Tensor:
    """Kernel layout of float32 weights [K][cin][cout] of K offsets (uint8 byte tensor); with
    `transpose` that of the per-offset transposes W_k^T (the strided layers' data gradient)."""
    W = W.contiguous()
    if W.dtype != torch.float32 or W.dim() != 3:
        raise ValueError("W must be float32 [K][cin][cout]")
    K, cin, cout = W.shape
    nbytes = L.get().npvs_packed_weight_bytes_k(K, cout if transpose else cin, cin if transpose else cout, dtype)
    Wp = torch.empty(nbytes, dtype=torch.uint8, device=W.device)
    L.call("npvs_pack_weights_k", _p(W), K, cin, cout, int(transpose), dtype, _p(Wp), _stream())
    return Wp


def strided_conv_fwd(X: torch.Tensor, Wp: torch.Tensor, bias: torch.Tensor | None, cin: int, cout: int, lv: Levels,
                     up: bool, dtype: int, relu: bool = True, out_f32: bool = False,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """Kernel-2 stride-2 convolution level 0 -> 1 (up=False) or its inverse level 1 -> 0 (up=True);
    Wp from pack_weights_k of a [8][cin][cout] weight."""
    rb = lv.rb0 if up else lv.rb1
    tdt = torch.float32 if (dtype == NPVS_F32 or out_f32) else _TORCH_DT[dtype]
    Y = torch.empty((rb.cap, cout), dtype=tdt, device=X.device) if out is None else out
    L.call("npvs_strided_conv_fwd", _p(X), cin, _p(Wp), _p(bias), cout, _p(lv.parent if up else lv.children),
           int(up), _p(rb.counts), rb.cap, dtype, int(relu), int(out_f32), _p(Y), _stream())
    return Y


def strided_conv_bwd(X, Wt, cin: int, cout: int, Y, dY, lv: Levels, up: bool, dtype: int, relu: bool = True,
                     want_dx: bool = True, dW: torch.Tensor | None = None, db: torch.Tensor | None = None):
    """Backward of strided_conv_fwd (npvs_strided_conv_bwd).  Wt = pack_weights_k(W, dtype,
    transpose=True).  Returns (dX float32 [input cap][cin] or None, dW float32 [8][cin][cout],
    db float32 [cout])."""
    rb_in, rb_out = (lv.rb1, lv.rb0) if up else (lv.rb0, lv.rb1)
    dev = X.device
    nbytes = ctypes.c_size_t()
    L.call("npvs_strided_bwd_workspace_size", cin, cout, rb_in.cap, rb_out.cap, int(up), dtype, ctypes.byref(nbytes))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    dX = torch.empty((rb_in.cap, cin), dtype=torch.float32, device=dev) if want_dx else None
    if dW is None:
        dW = torch.empty((8, cin, cout), dtype=torch.float32, device=dev)
    if db is None:
        db = torch.empty(cout, dtype=torch.float32, device=dev)
    if dW.numel() != 8 * cin * cout or db.numel() != cout or not (dW.is_contiguous() and db.is_contiguous()):
        raise ValueError("dW / db must be contiguous float32 [8][cin][cout] / [cout]")
    L.call("npvs_strided_conv_bwd", _p(X), cin, _p(Wt), cout, _p(Y), _p(dY.contiguous()), _p(lv.children),
           _p(lv.parent), int(up), _p(rb_in.counts), rb_in.cap, _p(rb_out.counts), rb_out.cap, dtype, int(relu),
           _p(dX), _p(dW), _p(db), _p(ws), ws.numel(), _stream())
    return dX, dW, db


def concat_channels_bwd(dY: torch.Tensor, ca: int, cb: int, rb: Rulebook, add_b: torch.Tensor | None = None,
                        want_a: bool = True, want_b: bool = True):
    """Gradient of concat_channels (float32): (dA [cap][ca] or None, dB [cap][cb] or None), with
    add_b (float32 [cap][cb]) added to dB."""
    dev = dY.device
    dA = torch.empty((dY.shape[0], ca), dtype=torch.float32, device=dev) if want_a else None
    dB = torch.empty((dY.shape[0], cb), dtype=torch.float32, device=dev) if want_b else None
    L.call("npvs_concat_channels_bwd", _p(dY.contiguous()), ca, cb, _p(add_b), _p(rb.counts), rb.cap, _p(dA), _p(dB),
           _stream())
    return dA, dB


def concat_channels(A: torch.Tensor, B: torch.Tensor, rb: Rulebook) -> torch.Tensor:
    """[A | B] row by row over the active sites (rows past the count left uninitialized)."""
    if A.dtype != B.dtype or A.shape[0] != B.shape[0]:
        raise ValueError("A and B must have the same dtype and row count")
    Y = torch.empty((A.shape[0], A.shape[1] + B.shape[1]), dtype=A.dtype, device=A.device)
    L.call("npvs_concat_channels", _p(A.contiguous()), A.shape[1], _p(B.contiguous()), B.shape[1], A.element_size(),
           _p(rb.counts), rb.cap, _p(Y), _stream())
    return Y


# --------------------------------------------------------------------------------- output
def deinterleave_threshold(Y: torch.Tensor, rb: Rulebook, occ: torch.Tensor, want_logits: bool = False):
    """(pvs bits uint8 like occ, dense float32 logits or None).  Y float32 [cap][w], w >= d^3: the
    d^3 logits first (a padded last layer's extra channels are ignored)."""
    if Y.dtype != torch.float32 or Y.dim() != 2 or Y.shape[1] < rb.d ** 3 or not Y.is_contiguous():
        raise ValueError("Y must be contiguous float32 [cap][w] with w >= d^3")
    pvs = torch.empty_like(occ)
    logits = None
    if want_logits:
        n = sum(nx * ny * nz for nx, ny, nz in rb.dims)
        logits = torch.empty(n, dtype=torch.float32, device=occ.device)
    L.call("npvs_deinterleave_threshold", _p(Y), Y.shape[1], _p(rb.block_row), _p(occ), len(rb.dims),
           L.dims_array(rb.dims), rb.d, _p(pvs), _p(logits), _stream())
    return pvs, logits


# --------------------------------------------------------------------------------- world space
def viewcell_frustum(c, forward, up, fov_y: float, aspect: float, r: float, beta: float, z_near: float,
                     z_far: float) -> L.View:
    """The frustum of a viewcell (npvs_viewcell_frustum): apex, basis, half-angle tangents, depth range."""
    arr = lambda v: (ctypes.c_double * 3)(*[float(x) for x in v])
    out = L.View()
    L.call("npvs_viewcell_frustum", ctypes.cast(arr(c), ctypes.c_void_p), ctypes.cast(arr(forward), ctypes.c_void_p),
           ctypes.cast(arr(up), ctypes.c_void_p), float(fov_y), float(aspect), float(r), float(beta), float(z_near),
           float(z_far), ctypes.byref(out))
    return out


def froxelize_view(tris: torch.Tensor, view: L.View, dims) -> torch.Tensor:
    """Packed occupancy uint8 [nz][ny][nx/8] of world-space triangles float32 [T][3][3] in the
    froxels of `view` (linear depth slices)."""
    nx, ny, nz = dims
    T = tris.shape[0] if tris.numel() else 0
    nbytes = ctypes.c_size_t()
    L.call("npvs_froxelize_view_workspace_size", T, ctypes.byref(nbytes))
    dev = tris.device
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    occ = torch.empty(nz * ny * nx // 8, dtype=torch.uint8, device=dev)
    L.call("npvs_froxelize_view", _p(tris.contiguous()) if T else None, T, ctypes.byref(view), L.Dims(nx, ny, nz),
           _p(occ), _p(ws), nbytes.value, _stream())
    return occ


# --------------------------------------------------------------------------------- culling
def visible_triangles(tris: torch.Tensor, n_tris, dims, pvs: torch.Tensor) -> torch.Tensor:
    """uint8 [total triangles]: 1 iff the triangle overlaps a froxel whose PVS bit is set."""
    dims = [tuple(g) for g in dims]
    total = int(sum(n_tris))
    vis = torch.empty(total, dtype=torch.uint8, device=pvs.device)
    L.call("npvs_visible_triangles", _p(tris), L.i64_array(list(n_tris)), len(dims), L.dims_array(dims), _p(pvs),
           _p(vis), _stream())
    return vis


def visible_objects(vis_tris: torch.Tensor, obj_off: torch.Tensor) -> torch.Tensor:
    """uint8 [n_objects]: OR of each object's triangle flags (obj_off int64 [n_objects + 1])."""
    n = obj_off.numel() - 1
    out = torch.empty(max(n, 0), dtype=torch.uint8, device=vis_tris.device)
    L.call("npvs_visible_objects", _p(vis_tris), _p(obj_off), n, _p(out), _stream())
    return out


# --------------------------------------------------------------------------------- training
def loss(logits: torch.Tensor, labels: torch.Tensor, rb: Rulebook, lam: float = 0.99, want_grad: bool = True,
         dice_alpha: float | None = None, dz_ws: torch.Tensor | None = None, dz_cin: int = 0):
    """Per-grid BCE (or, with dice_alpha, the weighted Dice term) + repulsive visibility loss.
    Returns (stats float32 [n_grids + 1][8] with columns L, BCE or Dice, L_rv, TP, FN, FP, GTP, m
    and the batch mean in the last row, dL/dlogits or None).  dz_ws: the BF16 backward workspace
    of the last layer (dz_cin -> C channels), which also receives the gradient as that layer's dZ
    and bias partials (see sparse_conv_bwd(want_dw=False))."""
    G = len(rb.dims)
    C = logits.shape[1]
    nbytes = ctypes.c_size_t()
    L.call("npvs_loss_workspace_size", G, ctypes.byref(nbytes))
    dev = logits.device
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    stats = torch.empty((G + 1, 8), dtype=torch.float32, device=dev)
    dl = torch.empty_like(logits) if want_grad else None  # rows past the active sites are never read
    term = L.NPVS_LOSS_BCE if dice_alpha is None else L.NPVS_LOSS_DICE
    L.call("npvs_loss", _p(logits), _p(labels), C, _p(rb.grid_rows), G, _p(rb.counts), rb.cap, float(lam), term,
           float(dice_alpha or 0.0), _p(stats), _p(dl), _p(dz_ws), 0 if dz_ws is None else dz_ws.numel(), dz_cin,
           _p(ws), nbytes.value, _stream())
    return stats, dl


def adam(p, g, m, v, step, layers=(), dtype: int = NPVS_F32, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
         weight_decay=1e-10):
    """npvs_adam.  `step`: a 16-byte npvs_adam_step on the device (uint8 tensor, zero to start),
    advanced by the call so that graph replays keep counting; or the step number t >= 1 counted on
    the host (a temporary counter holding t - 1 is made for the call).  layers = [(offset in p,
    cin, cout, Wp, Wt)]: weights whose forward and flipped-transpose packings (in `dtype`) are
    rewritten in the same pass."""
    if isinstance(step, int):
        if step < 1:
            raise ValueError("the step number starts at 1")
        host = torch.zeros(2, dtype=torch.int64)
        host[0] = step - 1
        step = host.view(torch.uint8).to(p.device)
    if step.numel() * step.element_size() != 16:
        raise ValueError("step must hold 16 bytes (npvs_adam_step)")
    if len(layers) > L.NPVS_MAX_ADAM_PACK:
        raise ValueError(f"at most {L.NPVS_MAX_ADAM_PACK} layers")
    descs = (L.AdamPackDesc * max(len(layers), 1))()
    for i, (off, cin, cout, Wp, Wt) in enumerate(layers):
        descs[i] = L.AdamPackDesc(int(off), int(cin), int(cout), Wp.data_ptr(), Wt.data_ptr())
    L.call("npvs_adam", _p(p), _p(g), _p(m), _p(v), p.numel(), _p(step), float(lr), float(beta1), float(beta2),
           float(eps), float(weight_decay), len(layers), descs, dtype, _stream())


# --------------------------------------------------------------------------------- plan
class Plan:
    """Library-owned plan of the whole forward pass for a fixed batch shape and network."""

    def __init__(self, dims, n_tris, d: int, channels, dtype: int = NPVS_BF16):
        self.dims = [tuple(g) for g in dims]
        self.n_tris = [int(t) for t in n_tris]
        self.d = d
        self.channels = list(channels)
        self.dtype = dtype
        h = ctypes.c_void_p()
        ch = (ctypes.c_int32 * len(self.channels))(*self.channels)
        L.call("npvs_plan_create", len(self.dims), L.dims_array(self.dims), L.i64_array(self.n_tris), d,
               len(self.channels) - 1, ch, dtype, ctypes.byref(h))
        self._h = h
        self.total_blocks, self.total_bytes = batch_sizes(self.dims, d)

    def set_weights(self, layer: int, W: torch.Tensor, b: torch.Tensor | None = None):
        L.call("npvs_plan_set_weights", self._h, layer, _p(W.contiguous()), _p(b), _stream())

    def _outs(self, pvs, logits, want_logits):
        if pvs is None:
            pvs = torch.empty(self.total_bytes, dtype=torch.uint8, device=_dev())
        if logits is None and want_logits:
            n = sum(nx * ny * nz for nx, ny, nz in self.dims)
            logits = torch.empty(n, dtype=torch.float32, device=_dev())
        return pvs, logits

    def forward(self, tris, pvs=None, occ=None, logits=None, want_logits=False):
        pvs, logits = self._outs(pvs, logits, want_logits)
        L.call("npvs_pvs_forward", self._h, _p(tris), _p(occ), _p(pvs), _p(logits), _stream())
        return pvs, logits

    def capture(self, tris, pvs=None, occ=None, logits=None, want_logits=False):
        pvs, logits = self._outs(pvs, logits, want_logits)
        L.call("npvs_plan_capture", self._h, _p(tris), _p(occ), _p(pvs), _p(logits), _stream())
        self._captured = (tris, pvs, occ, logits)  # keep the captured buffers alive
        return pvs, logits

    def replay(self):
        L.call("npvs_plan_replay", self._h, _stream())

    def autotune(self, tris, reps: int = 20) -> list:
        """Times every BF16 tile shape per distinct layer shape on the real rulebook of `tris` and
        keeps the fastest (synchronizes)."""
        v = (ctypes.c_int32 * (len(self.channels) - 1))()
        L.call("npvs_plan_autotune", self._h, _p(tris), int(reps), v, _stream())
        return list(v)

    def counts(self) -> dict:
        c = L.Counts()
        L.call("npvs_plan_counts", self._h, ctypes.byref(c), _stream())
        return dict(n_sites=c.n_sites, n_sites_needed=c.n_sites_needed, n_pairs=c.n_pairs,
                    n_tris_ignored=c.n_tris_ignored)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and L._lib is not None:
            L._lib.npvs_plan_destroy(h)
            self._h = None
