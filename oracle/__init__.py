"""NeuralPVS CPU oracle (numpy front end over ``npvs_oracle.c``).  TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct FP64 / exact-integer reference for every step of the forward
path (froxelize, active sites, interleave, rulebook, submanifold convolution, de-interleave and
threshold), the training loss and its gradient, the convolution backward, Adam, the ray-march
labeller, culling against the PVS, and the two-level U-Net (level relation, strided and inverse
convolutions, the whole encoder/decoder forward).  Each C function cites the passage of the paper it follows.  It shares no code with
the HIP library and must only be used by the tests, the smoke check and the benchmark's
CPU-baseline leg.

Pinning: every function is checked by ``tests/test_oracle_*.py`` against brute force, closed
forms, library routines (torch conv3d in float64) and the paper's stated invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "npvs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        sig = {
            "oracle_quantize_tri": (ctypes.c_int, [P, P]),
            "oracle_tri_box_overlap": (ctypes.c_int, [P, P, P]),
            "oracle_froxelize": (i64, [P, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]),
            "oracle_active_sites": (i32, [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]),
            "oracle_interleave": (None, [P] + [ctypes.c_int] * 5 + [P]),
            "oracle_deinterleave": (None, [P] + [ctypes.c_int] * 5 + [P]),
            "oracle_gather_sites": (None, [P] + [ctypes.c_int] * 4 + [i32, P, P]),
            "oracle_rulebook": (i64, [P, i32, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]),
            "oracle_subm_conv": (None, [P, i32, ctypes.c_int, P, P, ctypes.c_int, P, P, ctypes.c_int, P]),
            "oracle_masked_dense_conv": (None, [P, P] + [ctypes.c_int] * 4 + [P, P, ctypes.c_int, ctypes.c_int, P]),
            "oracle_deinterleave_threshold": (None, [P, i32, P, P] + [ctypes.c_int] * 4 + [P, P]),
            "oracle_loss": (None, [P, P, i64, f64, P, P]),
            "oracle_loss_dice": (None, [P, P, i64, f64, f64, P, P]),
            "oracle_froxelize_view": (i64, [P, i64, P, P, P, P, f64, f64, f64, f64, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, f64, P]),
            "oracle_subm_conv_bwd": (None, [P, i32, ctypes.c_int, P, ctypes.c_int, P, P, P, P, ctypes.c_int, P, P, P]),
            "oracle_adam": (None, [P, P, P, P, i64, i64, f64, f64, f64, f64, f64]),
            "oracle_label_raymarch": (i64, [P, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int,
                                            ctypes.c_int, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- froxelization
def quantize_tri(tri) -> np.ndarray | None:
    """Fixed-point (1/256 froxel, round half to even) vertices of one triangle, or None when
    the triangle is ignored (non-finite or |coordinate| >= 2048)."""
    t = _c(tri, np.float32).reshape(9)
    q = np.zeros((3, 3), np.int64)
    return q if _load().oracle_quantize_tri(_p(t), _p(q)) else None


def tri_box_overlap(q: np.ndarray, lo, hi) -> bool:
    """Exact SAT test of quantized triangle q against the closed fixed-point box [lo, hi]."""
    q = _c(q, np.int64)
    lo = _c(lo, np.int64)
    hi = _c(hi, np.int64)
    return bool(_load().oracle_tri_box_overlap(_p(q), _p(lo), _p(hi)))


def froxelize(tris, dims):
    """Packed occupancy grid uint8 [nz][ny][nx/8] and the number of ignored triangles."""
    nx, ny, nz = dims
    t = _c(tris, np.float32).reshape(-1, 9)
    occ = np.zeros((nz, ny, nx // 8), np.uint8)
    ign = _load().oracle_froxelize(_p(t), t.shape[0], nx, ny, nz, _p(occ))
    return occ, int(ign)


def visible_triangles(tris, dims, pvs) -> np.ndarray:
    """Culling against a PVS (the pipeline of Fig. 3 discards primitives whose froxels are all
    invisible; Sec. 5.6, dynamic scenes, tests a froxelized temporal bounding volume the same way):
    uint8 [T], 1 iff some froxel the triangle overlaps (the froxelization of that triangle alone)
    has its PVS bit set."""
    t = np.asarray(tris, np.float32).reshape(-1, 9)
    pvs = np.asarray(pvs, np.uint8).reshape(dims[2], dims[1], dims[0] // 8)
    out = np.zeros(t.shape[0], np.uint8)
    for i in range(t.shape[0]):
        occ, _ = froxelize(t[i:i + 1], dims)
        out[i] = 1 if (occ & pvs).any() else 0
    return out


def visible_objects(vis_tris, obj_off) -> np.ndarray:
    """An object (e.g. the triangles of a temporal bounding volume) is kept iff any of its
    triangles is visible: uint8 [n_objects], triangles obj_off[i] .. obj_off[i+1] - 1."""
    v = np.asarray(vis_tris, np.uint8)
    off = np.asarray(obj_off, np.int64)
    return np.array([1 if v[off[i]:off[i + 1]].any() else 0 for i in range(len(off) - 1)], np.uint8)


def unpack(bits: np.ndarray) -> np.ndarray:
    """Packed [nz][ny][nx/8] -> uint8 0/1 [nz][ny][nx] (bit x & 7 of byte x >> 3)."""
    return np.unpackbits(bits, axis=-1, bitorder="little")


# ---------------------------------------------------------------- sites / interleave / rulebook
def active_sites(occ, dims, d) -> np.ndarray:
    nx, ny, nz = dims
    occ = _c(occ, np.uint8)
    keys = np.zeros((nx // d) * (ny // d) * (nz // d), np.int32)
    n = _load().oracle_active_sites(_p(occ), nx, ny, nz, d, _p(keys))
    return keys[:n].copy()


def interleave(a: np.ndarray, d: int) -> np.ndarray:
    """Dense g_d of a [nz][ny][nx] array of any fixed-size dtype -> [nz/d][ny/d][nx/d][d^3]."""
    a = np.ascontiguousarray(a)
    nz, ny, nx = a.shape
    out = np.empty((nz // d, ny // d, nx // d, d ** 3), a.dtype)
    _load().oracle_interleave(_p(a), nx, ny, nz, d, a.itemsize, _p(out))
    return out


def deinterleave(a: np.ndarray, dims, d: int) -> np.ndarray:
    nx, ny, nz = dims
    a = np.ascontiguousarray(a)
    out = np.empty((nz, ny, nx), a.dtype)
    _load().oracle_deinterleave(_p(a), nx, ny, nz, d, a.itemsize, _p(out))
    return out


def gather_sites(occ, dims, d, keys) -> np.ndarray:
    nx, ny, nz = dims
    keys = _c(keys, np.int32)
    X = np.zeros((keys.shape[0], d ** 3), np.float64)
    _load().oracle_gather_sites(_p(_c(occ, np.uint8)), nx, ny, nz, d, keys.shape[0], _p(keys), _p(X))
    return X


def rulebook(keys, bdims):
    """CSR rulebook: rb_off int32[28], pairs int32[P][2] = (in_row, out_row)."""
    Bx, By, Bz = bdims
    keys = _c(keys, np.int32)
    n = keys.shape[0]
    rb_off = np.zeros(28, np.int32)
    pairs = np.zeros((27 * max(n, 1), 2), np.int32)
    P = _load().oracle_rulebook(_p(keys), n, Bx, By, Bz, _p(rb_off), _p(pairs))
    return rb_off, pairs[:P].copy()


def neighbor_map(rb_off, pairs, n) -> np.ndarray:
    """nbr[27][n]: input row feeding output row r through offset k, or -1."""
    nbr = np.full((27, n), -1, np.int32)
    for k in range(27):
        seg = pairs[rb_off[k]:rb_off[k + 1]]
        nbr[k, seg[:, 1]] = seg[:, 0]
    return nbr


# ---------------------------------------------------------------- convolution
def subm_conv(X, W, b, rb_off, pairs, relu: bool) -> np.ndarray:
    X = _c(X, np.float64)
    W = _c(W, np.float64)
    n, cin = X.shape
    cout = W.shape[2]
    b = _c(b if b is not None else np.zeros(cout), np.float64)
    Y = np.zeros((n, cout), np.float64)
    _load().oracle_subm_conv(_p(X), n, cin, _p(W), _p(b), cout, _p(_c(rb_off, np.int32)),
                             _p(_c(pairs, np.int32)), int(relu), _p(Y))
    return Y


def masked_dense_conv(dense_in, active, W, b, relu: bool) -> np.ndarray:
    """dense_in [Bz][By][Bx][cin], active [Bz][By][Bx] -> [Bz][By][Bx][cout]."""
    x = _c(dense_in, np.float64)
    Bz, By, Bx, cin = x.shape
    W = _c(W, np.float64)
    cout = W.shape[2]
    b = _c(b if b is not None else np.zeros(cout), np.float64)
    out = np.zeros((Bz, By, Bx, cout), np.float64)
    _load().oracle_masked_dense_conv(_p(x), _p(_c(active, np.uint8)), Bx, By, Bz, cin, _p(W), _p(b), cout,
                                     int(relu), _p(out))
    return out


def subm_conv_bwd(X, W, rb_off, pairs, Y, dY, relu: bool, want_dx: bool = True):
    X = _c(X, np.float64)
    W = _c(W, np.float64)
    n, cin = X.shape
    cout = W.shape[2]
    dX = np.zeros((n, cin), np.float64) if want_dx else None
    dW = np.zeros_like(W)
    db = np.zeros(cout, np.float64)
    _load().oracle_subm_conv_bwd(_p(X), n, cin, _p(W), cout, _p(_c(rb_off, np.int32)), _p(_c(pairs, np.int32)),
                                 _p(_c(Y, np.float64)), _p(_c(dY, np.float64)), int(relu), _p(dX), _p(dW), _p(db))
    return dX, dW, db


# ---------------------------------------------------------------- output, loss, optimizer
def deinterleave_threshold(Y, keys, occ, dims, d, want_logits: bool = True):
    nx, ny, nz = dims
    Y = _c(Y, np.float64)
    keys = _c(keys, np.int32)
    if Y.shape != (keys.shape[0], d ** 3):
        raise ValueError("de-interleave needs one row of d^3 logits per active site")
    logits = np.zeros((nz, ny, nx), np.float64) if want_logits else None
    pvs = np.zeros((nz, ny, nx // 8), np.uint8)
    _load().oracle_deinterleave_threshold(_p(Y), keys.shape[0], _p(keys), _p(_c(occ, np.uint8)), nx, ny, nz, d,
                                          _p(logits), _p(pvs))
    return logits, pvs


def loss(logits, labels, lam: float = 0.99, want_grad: bool = True):
    l = _c(logits, np.float64).reshape(-1)
    y = _c(labels, np.uint8).reshape(-1)
    out = np.zeros(7, np.float64)
    g = np.zeros_like(l) if want_grad else None
    _load().oracle_loss(_p(l), _p(y), l.shape[0], lam, _p(out), _p(g))
    keys = ["loss", "bce", "lrv", "tp", "fn", "fp", "gtp"]
    res = dict(zip(keys, out.tolist()))
    if want_grad:
        res["grad"] = g.reshape(np.shape(logits))
    return res


def loss_dice(logits, labels, lam: float = 0.99, alpha: float = 0.9, want_grad: bool = True):
    """The paper's combined loss lambda * L_dice + (1 - lambda) * L_rv (Sec. 3.3), weighted Dice
    with alpha on the missed ground-truth froxels.  Keys: loss, dice, lrv, tp, fn, fp, gtp[, grad]."""
    l = _c(logits, np.float64).reshape(-1)
    y = _c(labels, np.uint8).reshape(-1)
    out = np.zeros(7, np.float64)
    g = np.zeros_like(l) if want_grad else None
    _load().oracle_loss_dice(_p(l), _p(y), l.shape[0], lam, alpha, _p(out), _p(g))
    res = dict(zip(["loss", "dice", "lrv", "tp", "fn", "fp", "gtp"], out.tolist()))
    if want_grad:
        res["grad"] = g.reshape(np.shape(logits))
    return res


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=1e-10):
    """One Adam step on FP64 copies; returns (p, m, v)."""
    p = _c(p, np.float64).copy()
    m = _c(m, np.float64).copy()
    v = _c(v, np.float64).copy()
    g = _c(g, np.float64)
    _load().oracle_adam(_p(p), _p(g), _p(m), _p(v), p.size, t, lr, b1, b2, eps, wd)
    return p, m, v


def label_raymarch(tris, dims, views, s_r: int = 2) -> np.ndarray:
    nx, ny, nz = dims
    t = _c(tris, np.float32).reshape(-1, 9)
    v = _c(views, np.float64).reshape(-1, 3)
    lab = np.zeros((nz, ny, nx // 8), np.uint8)
    _load().oracle_label_raymarch(_p(t), t.shape[0], nx, ny, nz, _p(v), v.shape[0], s_r, _p(lab))
    return lab


# ---------------------------------------------------------------- bfloat16 rounding points
def bf16_round(x) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 value, ties to even, returned as float64.

    bfloat16 keeps float32's 8-bit exponent and 8 significant bits (7 stored).  For a finite x
    with x = m 2^e, 0.5 <= |m| < 1 (frexp), the representable neighbours are the multiples of
    the quantum 2^(e - 8) (2^-133 at the subnormal end), and rint rounds half to even; a result
    of 2^128 or more overflows to infinity.  Non-finite values pass through."""
    x = np.asarray(x, np.float64)
    out = x.copy()
    fin = np.isfinite(x) & (x != 0)
    _, e = np.frexp(x[fin])
    q = np.maximum(e - 8, -133)
    r = np.ldexp(np.rint(np.ldexp(x[fin], -q)), q)
    r[np.abs(r) >= 2.0 ** 128] = np.inf * np.sign(r[np.abs(r) >= 2.0 ** 128])
    out[fin] = r
    return out


def subm_conv_f32(X, W, b, rb_off, pairs, relu: bool) -> np.ndarray:
    """The submanifold convolution evaluated with float32 accumulation (numpy float32 products
    per offset, added offset by offset): a second admissible evaluation order of the same
    arithmetic, used to measure how far two orders of the float32 sums drift apart through a
    BF16 network.  Not a reference value."""
    X = np.asarray(X, np.float32)
    W = np.asarray(W, np.float32)
    Y = np.zeros((X.shape[0], W.shape[2]), np.float32)
    for k in range(27):
        p = np.asarray(pairs[rb_off[k]:rb_off[k + 1]])
        if len(p):
            Y[p[:, 1]] += X[p[:, 0]] @ W[k]  # output rows are distinct within one offset
    if b is not None:
        Y += np.asarray(b, np.float32)
    return np.maximum(Y, 0.0) if relu else Y


def subm_conv_bwd_f32(X, W, rb_off, pairs, dZ, want_dx: bool = True):
    """The products of ``subm_conv_bwd`` (no ReLU mask; dZ given) evaluated with float32
    accumulation, offset by offset: (dX, dW).  Used like subm_conv_f32, never as a reference."""
    X = np.asarray(X, np.float32)
    W = np.asarray(W, np.float32)
    dZ = np.asarray(dZ, np.float32)
    dX = np.zeros_like(X) if want_dx else None
    dW = np.zeros_like(W)
    for k in range(27):
        p = np.asarray(pairs[rb_off[k]:rb_off[k + 1]])
        if len(p):
            if want_dx:
                dX[p[:, 0]] += dZ[p[:, 1]] @ W[k].T  # input rows are distinct within one offset
            dW[k] = X[p[:, 0]].T @ dZ[p[:, 1]]
    return dX, dW


def forward_bf16(tris, dims, d, layers, occ=None, accum: str = "f64"):
    """The whole path of ``forward`` at the BF16 path's rounding points (MFMA products of
    bfloat16 operands with float32 accumulation, float32 bias and ReLU): every weight is rounded
    to bfloat16 from its float32 master, each hidden layer's result (after bias and ReLU) is
    rounded to bfloat16 before it feeds the next layer, the last layer's logits are not rounded,
    and the input (0/1) is exact.  The arithmetic between the rounding points is FP64, so this
    is the exact value of the BF16 network up to the order of the float32 accumulations.
    Returns the keys of ``forward`` plus Wb (the rounded weights), z (each layer's result before
    ReLU) and pre (each layer's unrounded result after ReLU).  accum = "f32" evaluates the sums with float32 accumulation instead
    (subm_conv_f32): a second evaluation order, for sizing end-to-end tolerances only."""
    nx, ny, nz = dims
    if occ is None:
        occ, _ = froxelize(tris, dims)
    keys = active_sites(occ, dims, d)
    rb_off, pairs = rulebook(keys, (nx // d, ny // d, nz // d))
    X = gather_sites(occ, dims, d, keys)
    conv = subm_conv if accum == "f64" else subm_conv_f32
    acts, pre, zs, Wb = [X], [], [], []
    for li, (W, b) in enumerate(layers):
        last = li == len(layers) - 1
        w = bf16_round(np.asarray(W, np.float32))
        Wb.append(w)
        z = np.asarray(conv(acts[-1], w, np.asarray(b, np.float32) if b is not None else None, rb_off, pairs,
                            relu=False), np.float64)
        y = z if last else np.maximum(z, 0.0)
        zs.append(z)
        pre.append(y)
        acts.append(y if last else bf16_round(y))
    logits, pvs = deinterleave_threshold(acts[-1], keys, occ, dims, d)
    return dict(occ=occ, keys=keys, rb_off=rb_off, pairs=pairs, acts=acts, pre=pre, z=zs, Wb=Wb, logits=logits,
                pvs=pvs)


def backward_bf16(out, layers, dlogits_rows, accum: str = "f64", dy_bf16: bool = False):
    """Backward of ``forward_bf16`` at the BF16 path's rounding points: per layer, from the top,
    dZ = dY [Y > 0] (ReLU'(0) = 0; no mask on the last layer), its bfloat16 rounding dZb is the
    operand of the products, dX = sum_k dZb W_k^T over the transposed rulebook with the rounded
    weights, dW_k = sum X^T dZb with the layer's bfloat16 input X, and db = sum dZ (unrounded).
    dX is the next layer's dY.  FP64 between the rounding points.  Returns [(dW, db)] per layer
    and the list of each layer's dZb (top layer last).  accum = "f32": float32 accumulation
    (subm_conv_bwd_f32, with dY carried in float32), for sizing end-to-end tolerances only.
    dy_bf16: the gradient arriving at each hidden layer is itself rounded to bfloat16 first (a
    chain of layers through torch autograd hands each layer the gradient in its output's dtype);
    db then sums the rounded values."""
    acts, rb_off, pairs, Wb = out["acts"], out["rb_off"], out["pairs"], out["Wb"]
    grads = [None] * len(layers)
    dzb = [None] * len(layers)
    dY = np.asarray(dlogits_rows, np.float64)
    for li in range(len(layers) - 1, -1, -1):
        relu = li < len(layers) - 1
        if relu and dy_bf16:
            dY = bf16_round(dY)
        dZ = dY * (acts[li + 1] > 0) if relu else dY
        dZb = bf16_round(dZ)
        dzb[li] = dZb
        if accum == "f64":
            dX, dW, _ = subm_conv_bwd(acts[li], Wb[li], rb_off, pairs, None, dZb, relu=False, want_dx=li > 0)
            db = dZ.sum(axis=0)
        else:
            dX, dW = subm_conv_bwd_f32(acts[li], Wb[li], rb_off, pairs, dZb, want_dx=li > 0)
            dX = None if dX is None else np.asarray(dX, np.float64)
            dW = np.asarray(dW, np.float64)
            db = np.asarray(dZ, np.float32).sum(axis=0, dtype=np.float32).astype(np.float64)
        grads[li] = (dW, db)
        dY = dX
    return grads, dzb


# ---------------------------------------------------------------- BF16 error bounds
# The BF16 path fixes its rounding points (forward_bf16 / backward_bf16); what it leaves free is
# the order of its float32 sums.  Every product it sums is exact in float32 (a product of two
# bfloat16 values has at most 16 significant bits), so a sum of n such terms, added in any order
# with a rounding after each addition, differs from the exact sum by at most
# gamma_n * sum |term|, gamma_n = n u / (1 - n u) (Higham, Accuracy and Stability of Numerical
# Algorithms, 2nd ed., Sec. 4.2).  u = 2^-23 covers both round-to-nearest and truncating adders.
# A blocked sum whose block results are added with compensation (Neumaier) stays within the same
# bound.  The functions below carry that bound through the network, with the bfloat16 rounding
# of each hidden value evaluated on the whole interval it can come from (bfloat16 rounding is
# monotone), so a value whose interval crosses a rounding boundary carries the whole quantum.
F32_UNIT = 2.0 ** -23


def f32_sum_gamma(n: int) -> float:
    """gamma_n for float32 sums of n exact terms: |computed - exact| <= gamma_n sum |terms|."""
    nu = n * F32_UNIT
    if nu >= 1.0:
        raise ValueError("sum too long for the float32 bound")
    return nu / (1.0 - nu)


def _round_interval_dev(x, lo, hi):
    """Largest |bf16(t) - x| over t in [lo, hi], with x the rounding of a point of the interval."""
    return np.maximum(bf16_round(hi) - x, x - bf16_round(lo))


def forward_bf16_bound(out, layers) -> dict:
    """Element-wise bounds on how far any float32-order evaluation of the BF16 network can lie
    from ``forward_bf16``'s values (same rounded weights, same rounding points).

    Layer l: the computed pre-activation z' = fl(sum x' w + b) with |x' - x| <= E_l satisfies
    |z' - z| <= D_l = sum E_l |w| + gamma_{27 cin + 1} (sum (|x| + E_l) |w| + |b|).  The next input
    x' = bf16(relu(z')) lies in [bf16(relu(z - D_l)), bf16(relu(z + D_l))], which gives E_{l+1};
    the ReLU mask of the layer (x' > 0) is certain where both ends agree.  E_0 = 0 (the 0/1 input
    is exact).  Returns D (per layer; the last one bounds the logits), E (per layer input) and
    mask_certain (per hidden layer).  Bounds are widened by 1e-9 of themselves for the float64
    evaluation of this function."""
    acts, Wb, zs = out["acts"], out["Wb"], out["z"]
    rb_off, pairs = out["rb_off"], out["pairs"]
    E = np.zeros_like(np.asarray(acts[0], np.float64))
    res = dict(D=[], E=[E], mask_certain=[])
    for li, (_, b) in enumerate(layers):
        aW = np.abs(Wb[li])
        ab = np.abs(np.asarray(b, np.float64)) if b is not None else None
        prop = subm_conv(E, aW, None, rb_off, pairs, relu=False)
        mag = subm_conv(np.abs(acts[li]) + E, aW, ab, rb_off, pairs, relu=False)
        D = (prop + f32_sum_gamma(27 * aW.shape[1] + 1) * mag) * (1.0 + 1e-9)
        res["D"].append(D)
        if li == len(layers) - 1:
            break
        z = zs[li]
        lo = bf16_round(np.maximum(z - D, 0.0))
        hi = bf16_round(np.maximum(z + D, 0.0))
        E = _round_interval_dev(acts[li + 1], np.maximum(z - D, 0.0), np.maximum(z + D, 0.0))
        res["E"].append(E)
        res["mask_certain"].append((lo > 0) == (hi > 0))
    return res


def bf16_layer_bound(X, Wb, b, rb_off, pairs, relu: bool) -> dict:
    """One BF16 layer on exact operands (X and the rounded weights Wb as float64 values of
    bfloat16 numbers): the exact pre-activation z, the bound D = gamma_{27 cin + 1} (sum |x| |w| + |b|)
    on any float32-order evaluation of it, and the interval [lo, hi] that the layer's rounded
    output bf16(relu(z')) must lie in (lo == hi == bf16(relu(z)) unless z lies within D of a
    rounding boundary).  Without relu (a last layer) lo / hi bound the float32 output itself."""
    aW = np.abs(np.asarray(Wb, np.float64))
    ab = np.abs(np.asarray(b, np.float64)) if b is not None else None
    z = subm_conv(X, Wb, b, rb_off, pairs, relu=False)
    D = f32_sum_gamma(27 * aW.shape[1] + 1) * subm_conv(np.abs(X), aW, ab, rb_off, pairs, relu=False)
    D *= 1.0 + 1e-9
    if relu:
        lo, hi = bf16_round(np.maximum(z - D, 0.0)), bf16_round(np.maximum(z + D, 0.0))
        x = bf16_round(np.maximum(z, 0.0))
    else:
        lo, hi, x = z - D, z + D, z
    return dict(z=z, D=D, lo=lo, hi=hi, out=x)


def bf16_layer_bwd_bound(X, Wb, rb_off, pairs, Y, dY, relu: bool, want_dx: bool = True) -> dict:
    """Backward of one BF16 layer on exact operands: X (the layer's bfloat16 input), Wb (rounded
    weights), Y (its bfloat16 output, for the ReLU mask) and dY (float32 values).  The path forms
    dZ = dY [Y > 0] exactly, rounds it to dZb = bf16(dZ) (both sides round the same float32
    value, so dZb is exact too) and sums exact products in float32.  Returns dX, dW, db with the
    bounds E_dX = gamma_{27 cout} sum |dZb| |W|, E_dW = gamma_P sum |X| |dZb| (P the largest pair
    count of an offset) and E_db = gamma_n sum |dZ|, plus dZb."""
    dY = np.asarray(dY, np.float64)
    dZ = dY * (np.asarray(Y) > 0) if relu else dY
    dZb = bf16_round(dZ)
    dX, dW, _ = subm_conv_bwd(X, Wb, rb_off, pairs, None, dZb, relu=False, want_dx=want_dx)
    aW = np.abs(np.asarray(Wb, np.float64))
    n = dZ.shape[0]
    adx, adW, _ = subm_conv_bwd(np.abs(X), aW, rb_off, pairs, None, np.abs(dZb), relu=False, want_dx=want_dx)
    P = int(np.diff(rb_off).max()) if len(pairs) else 1
    w = 1.0 + 1e-9
    return dict(dX=dX, dW=dW, db=dZ.sum(axis=0), dZb=dZb,
                E_dX=None if adx is None else f32_sum_gamma(27 * aW.shape[2]) * adx * w,
                E_dW=f32_sum_gamma(max(P, 1)) * adW * w,
                E_db=f32_sum_gamma(max(n, 1)) * np.abs(dZ).sum(axis=0) * w)


def loss_grad_bound(logits_rows, labels_rows, e_logits, lam: float = 0.99):
    """Element-wise bound on the loss gradient's deviation when the logits deviate by at most
    e_logits and the gradient is evaluated in float32 (one grid).

    dL/dl = lam (p - y) / n + (1 - lam) p (1 - p) (1 - 2y) / max(GTP, 1) with p = sigmoid(l) (the
    loss ``loss``); its derivative in l is at most lam / (4 n) + (1 - lam) / (6 sqrt 3) / max(GTP, 1)
    in size (p (1 - p) <= 1/4 and |d/dl p (1 - p)| = p (1 - p) |1 - 2p| <= 1 / (6 sqrt 3)).  The float32
    evaluation (sigmoid through exp, a few operations) is allowed 8 units of 2^-23 of each term's
    scale and of the result."""
    l = np.asarray(logits_rows, np.float64)
    y = np.asarray(labels_rows, np.float64)
    n = l.size
    g_den = max(float(y.sum()), 1.0)
    lip = lam / (4.0 * n) + (1.0 - lam) / (6.0 * np.sqrt(3.0)) / g_den
    g = loss(l, np.asarray(labels_rows, np.uint8))["grad"]
    return lip * np.asarray(e_logits, np.float64) + 8 * F32_UNIT * (lam / n + (1.0 - lam) / g_den + np.abs(g))


def backward_bf16_bound(out, layers, fwd_bound, dlogits_rows, e_dlogits, dy_bf16: bool = False):
    """Element-wise bounds on how far any float32-order evaluation of the BF16 backward can lie
    from ``backward_bf16``'s gradients, given its forward deviation bounds (forward_bf16_bound)
    and a bound e_dlogits on the deviation of the incoming dL/dlogits.

    Per layer from the top, with E_dY the bound on dY: dZ = dY [x' > 0] deviates by E_dY where
    the mask is certain and by |dY| + E_dY where it is not; dZb = bf16(dZ) by its interval's
    rounding; the data gradient by sum E_dZb |W| + gamma_{27 cout} sum (|dZb| + E_dZb) |W| (the
    next layer's E_dY); dW by sum (|X| + E_X)(|dZb| + E_dZb)(1 + gamma_P) - sum |X| |dZb| with P
    the largest pair count of an offset; db by sum E_dZ + gamma_n sum (|dZ| + E_dZ).  Returns
    [(E_dW, E_db)] per layer and the bound on the network input's gradient, widened by 1e-9 of
    themselves.  dy_bf16 as in backward_bf16: the incoming gradient of each hidden layer is
    rounded first, its deviation taken over its interval like the other rounding points."""
    acts, Wb, rb_off, pairs = out["acts"], out["Wb"], out["rb_off"], out["pairs"]
    n = np.asarray(acts[0]).shape[0]
    g_p = f32_sum_gamma(int(np.diff(rb_off).max()) if len(pairs) else 1)
    g_n = f32_sum_gamma(max(n, 1))
    bounds = [None] * len(layers)
    dY = np.asarray(dlogits_rows, np.float64)
    E_dY = np.asarray(e_dlogits, np.float64)
    for li in range(len(layers) - 1, -1, -1):
        if li < len(layers) - 1 and dy_bf16:
            dYr = bf16_round(dY)
            E_dY = _round_interval_dev(dYr, dY - E_dY, dY + E_dY)
            dY = dYr
        if li < len(layers) - 1:
            m = acts[li + 1] > 0
            dZ = dY * m
            E_dZ = np.where(fwd_bound["mask_certain"][li], m * E_dY, np.abs(dY) + E_dY)
        else:
            dZ, E_dZ = dY, E_dY
        dZb = bf16_round(dZ)
        E_dZb = _round_interval_dev(dZb, dZ - E_dZ, dZ + E_dZ)
        X, E_X = np.abs(acts[li]), fwd_bound["E"][li]
        aW = np.abs(Wb[li])
        dxa, dWa, _ = subm_conv_bwd(X + E_X, aW, rb_off, pairs, None, np.abs(dZb) + E_dZb, relu=False,
                                    want_dx=li > 0)
        _, dWb, _ = subm_conv_bwd(X, aW, rb_off, pairs, None, np.abs(dZb), relu=False, want_dx=False)
        E_dW = np.maximum((1.0 + g_p) * dWa - dWb, 0.0) * (1.0 + 1e-9)
        E_db = (E_dZ.sum(axis=0) + g_n * (np.abs(dZ) + E_dZ).sum(axis=0)) * (1.0 + 1e-9)
        bounds[li] = (E_dW, E_db)
        if li == 0:
            dxa, _, _ = subm_conv_bwd(X + E_X, aW, rb_off, pairs, None, np.abs(dZb) + E_dZb, relu=False,
                                      want_dx=True)
        dxc, _, _ = subm_conv_bwd(X, aW, rb_off, pairs, None, E_dZb, relu=False, want_dx=True)
        E_dY = (dxc + f32_sum_gamma(27 * aW.shape[2]) * dxa) * (1.0 + 1e-9)
        if li > 0:
            dY, _, _ = subm_conv_bwd(acts[li], Wb[li], rb_off, pairs, None, dZb, relu=False, want_dx=True)
    return bounds, E_dY


# ---------------------------------------------------------------- evaluation metrics
def active_froxels(occ, dims, d) -> np.ndarray:
    """Packed mask [nz][ny][nx/8] of the froxels that lie in active blocks (a block of d^3
    froxels is active iff one of its froxels is occupied): the froxels that receive a logit and
    are thresholded (Sec. 3.1, 3.3)."""
    nx, ny, nz = dims
    g = unpack(np.asarray(occ, np.uint8).reshape(nz, ny, nx // 8)).astype(bool)
    blk = g.reshape(nz // d, d, ny // d, d, nx // d, d).any(axis=(1, 3, 5))
    full = np.repeat(np.repeat(np.repeat(blk, d, axis=0), d, axis=1), d, axis=2)
    return np.packbits(full.astype(np.uint8), axis=-1, bitorder="little")


def metrics(v_ref, v_test, occ, active) -> dict:
    """Agreement of a tested PVS with a reference PVS (packed bits of the same grid).

    Sec. 5.1 evaluates a PVS by its false negative rate FNR = FN / GTP and false positive rate
    FPR = FP / GTP, counted over froxels with the reference as the ground truth: FN = #{ref 1,
    test 0}, FP = #{ref 0, test 1}, GTP = #{ref 1}.  missing_geometry is that FNR (geometry the
    reference keeps and the tested set drops).  The flip rate is #{ref != test} over three
    denominators: the occupied froxels (supp G; both sets lie inside G, so only these can
    differ), the froxels of the active blocks (`active`, the froxels that are thresholded) and
    all froxels.  Counts are returned beside the rates; a zero denominator gives a rate of 0."""
    a = unpack(np.asarray(v_ref, np.uint8)).astype(bool)
    b = unpack(np.asarray(v_test, np.uint8)).astype(bool)
    g = unpack(np.asarray(occ, np.uint8)).astype(bool)
    m = unpack(np.asarray(active, np.uint8)).astype(bool)
    if not (a.shape == b.shape == g.shape == m.shape):
        raise ValueError("all four grids must have the same shape")
    flips = int((a != b).sum())
    fn = int((a & ~b).sum())
    fp = int((~a & b).sum())
    gtp = int(a.sum())
    n_occ, n_act, n_all = int(g.sum()), int(m.sum()), int(g.size)
    rate = lambda x, y: x / y if y else 0.0
    return dict(flips=flips, fn=fn, fp=fp, gtp=gtp, occupied=n_occ, active=n_act, froxels=n_all,
                flip_rate_occupied=rate(flips, n_occ), flip_rate_active=rate(flips, n_act),
                flip_rate_all=rate(flips, n_all), missing_geometry=rate(fn, gtp), fnr=rate(fn, gtp),
                fpr=rate(fp, gtp))


# ---------------------------------------------------------------- composition
def forward(tris, dims, d, layers, want_logits: bool = True, occ=None):
    """Whole path on one grid (Sec. 3: V = g_d^-1(f(g_d(G))) thresholded), FP64.

    layers: list of (W [27][cin][cout], b [cout]); ReLU after every layer but the last.
    Returns a dict of every intermediate."""
    nx, ny, nz = dims
    if occ is None:
        occ, _ = froxelize(tris, dims)
    keys = active_sites(occ, dims, d)
    rb_off, pairs = rulebook(keys, (nx // d, ny // d, nz // d))
    X = gather_sites(occ, dims, d, keys)
    acts = [X]
    for li, (W, b) in enumerate(layers):
        acts.append(subm_conv(acts[-1], W, b, rb_off, pairs, relu=li < len(layers) - 1))
    logits, pvs = deinterleave_threshold(acts[-1], keys, occ, dims, d, want_logits)
    return dict(occ=occ, keys=keys, rb_off=rb_off, pairs=pairs, acts=acts, logits=logits, pvs=pvs)


def backward(out, layers, dlogits_rows):
    """Backward through the whole layer stack of ``forward`` (chain rule on each layer, FP64).

    dlogits_rows: dL/dY of the last layer [n][d^3].  Returns [(dW, db)] per layer and dX of the
    network input."""
    acts, rb_off, pairs = out["acts"], out["rb_off"], out["pairs"]
    grads = [None] * len(layers)
    dY = dlogits_rows
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        dX, dW, db = subm_conv_bwd(acts[li], W, rb_off, pairs, acts[li + 1], dY, relu=li < len(layers) - 1)
        grads[li] = (dW, db)
        dY = dX
    return grads, dY


def site_labels(label_bits, dims, d, keys) -> np.ndarray:
    """Labels of the froxels of the active blocks, in the interleaved [n][d^3] row layout."""
    return gather_sites(label_bits, dims, d, keys).astype(np.uint8)


# ---------------------------------------------------------------- two-level sparse U-Net
# The backbone of Sec. 3.3 is an encoder/decoder (Suppl. A.2: embedding 64 channels, encoder
# channels 64, down ratio 2, decoder channels 96, encoder depths 2 and 3, decoder depth 2).  Its
# coarse level holds the blocks of the grid at interleave factor 2d, i.e. the 2x2x2 groups of
# level-0 blocks; a coarse block is active iff one of its eight children is.
def level_maps(keys0, keys1, bdims0):
    """Child / parent relation between the active blocks of level 0 (block grid bdims0 =
    (Bx, By, Bz)) and of level 1 (the grid halved along each axis).  Child index
    k = ((bz & 1) * 2 + (by & 1)) * 2 + (bx & 1).  Returns children int32 [8][n1] (level-0 row
    or -1), parent int32 [n0] (level-1 row) and kid int32 [n0] (child index)."""
    Bx, By, Bz = bdims0
    Cx, Cy = Bx // 2, By // 2
    row1 = {int(key): r for r, key in enumerate(keys1)}
    children = np.full((8, len(keys1)), -1, np.int32)
    parent = np.zeros(len(keys0), np.int32)
    kid = np.zeros(len(keys0), np.int32)
    for f, key in enumerate(keys0):
        key = int(key)
        bx, by, bz = key % Bx, (key // Bx) % By, key // (Bx * By)
        c = row1[((bz >> 1) * Cy + (by >> 1)) * Cx + (bx >> 1)]
        k = ((bz & 1) * 2 + (by & 1)) * 2 + (bx & 1)
        children[k, c] = f
        parent[f] = c
        kid[f] = k
    return children, parent, kid


def strided_down(X0, children, W, b, relu: bool) -> np.ndarray:
    """Sparse convolution with kernel 2 and stride 2 (down ratio 2): coarse row c gets
    b + sum_k X0[child k of c] W[k] over its active children; W [8][cin][cout]."""
    X0 = np.asarray(X0, np.float64)
    W = np.asarray(W, np.float64)
    Y = np.zeros((children.shape[1], W.shape[2])) + np.asarray(b, np.float64)
    for k in range(8):
        has = children[k] >= 0
        Y[has] += X0[children[k, has]] @ W[k]
    return np.maximum(Y, 0.0) if relu else Y


def inverse_up(X1, parent, kid, W, b, relu: bool) -> np.ndarray:
    """The inverse (transposed) convolution of strided_down on the same blocks: level-0 row f
    gets b + X1[parent f] W[kid f]; W [8][cin][cout]."""
    X1 = np.asarray(X1, np.float64)
    W = np.asarray(W, np.float64)
    Y = np.zeros((len(parent), W.shape[2])) + np.asarray(b, np.float64)
    for k in range(8):
        sel = kid == k
        Y[sel] += X1[parent[sel]] @ W[k]
    return np.maximum(Y, 0.0) if relu else Y


def unet_forward(tris, dims, d, params, want_logits: bool = True, occ=None):
    """Whole path with the two-level U-Net in place of the plain stack, FP64.  params: dict of
    lists of (W, b): stem [1] (d^3 -> E), enc0, down [1] (W [8][E][E]), enc1, up [1]
    (W [8][E][D]), dec0 (first one takes D + E channels: the up output, then the level-0 skip),
    head [1] (-> d^3, no ReLU).  ReLU after every other layer."""
    nx, ny, nz = dims
    if occ is None:
        occ, _ = froxelize(tris, dims)
    b0 = (nx // d, ny // d, nz // d)
    keys0 = active_sites(occ, dims, d)
    keys1 = active_sites(occ, dims, 2 * d)
    rb0 = rulebook(keys0, b0)
    rb1 = rulebook(keys1, (b0[0] // 2, b0[1] // 2, b0[2] // 2))
    children, parent, kid = level_maps(keys0, keys1, b0)
    acts = {"X": gather_sites(occ, dims, d, keys0)}
    inputs = {st: [] for st in params}  # the input of every layer, kept for the backward
    h = acts["X"]
    for st in ("stem", "enc0"):
        for W, b in params[st]:
            inputs[st].append(h)
            h = subm_conv(h, W, b, *rb0, relu=True)
    acts["skip"] = h
    (W, b), = params["down"]
    inputs["down"].append(h)
    h1 = strided_down(h, children, W, b, relu=True)
    for W, b in params["enc1"]:
        inputs["enc1"].append(h1)
        h1 = subm_conv(h1, W, b, *rb1, relu=True)
    acts["coarse"] = h1
    (W, b), = params["up"]
    inputs["up"].append(h1)
    u = inverse_up(h1, parent, kid, W, b, relu=True)
    acts["up"] = u
    h = np.concatenate([u, acts["skip"]], axis=1)
    for W, b in params["dec0"]:
        inputs["dec0"].append(h)
        h = subm_conv(h, W, b, *rb0, relu=True)
    (W, b), = params["head"]
    inputs["head"].append(h)
    Y = subm_conv(h, W, b, *rb0, relu=False)
    acts["Y"] = Y
    acts["inputs"] = inputs
    logits, pvs = deinterleave_threshold(Y, keys0, occ, dims, d, want_logits)
    return dict(occ=occ, keys0=keys0, keys1=keys1, children=children, parent=parent, kid=kid, acts=acts,
                rb0=rb0, rb1=rb1, logits=logits, pvs=pvs)


def strided_down_bwd(X0, children, W, Y, dY, relu: bool, want_dx: bool = True):
    """Chain rule on strided_down: dZ = dY [Y > 0] (ReLU'(0) = 0) or dY; every level-0 row is the
    child k of exactly one coarse row c, so dX0[child k of c] = dZ[c] W[k]^T; dW[k] = sum over
    coarse rows c of X0[child k of c]^T dZ[c]; db = sum_c dZ[c].  FP64."""
    X0 = np.asarray(X0, np.float64)
    W = np.asarray(W, np.float64)
    dZ = np.asarray(dY, np.float64) * (np.asarray(Y) > 0) if relu else np.asarray(dY, np.float64)
    dX0 = np.zeros_like(X0) if want_dx else None
    dW = np.zeros_like(W)
    for k in range(8):
        has = children[k] >= 0
        rows = children[k, has]
        if want_dx:
            dX0[rows] = dZ[has] @ W[k].T
        dW[k] = X0[rows].T @ dZ[has]
    return dX0, dW, dZ.sum(0)


def inverse_up_bwd(X1, parent, kid, W, Y, dY, relu: bool, want_dx: bool = True):
    """Chain rule on inverse_up: dZ as in strided_down_bwd; coarse row c collects the products of
    its children, dX1[c] = sum over children f of c of dZ[f] W[kid f]^T; dW[k] = sum over level-0
    rows f with kid k of X1[parent f]^T dZ[f]; db = sum_f dZ[f].  FP64."""
    X1 = np.asarray(X1, np.float64)
    W = np.asarray(W, np.float64)
    dZ = np.asarray(dY, np.float64) * (np.asarray(Y) > 0) if relu else np.asarray(dY, np.float64)
    dX1 = np.zeros_like(X1) if want_dx else None
    dW = np.zeros_like(W)
    for k in range(8):
        sel = kid == k
        if want_dx:
            np.add.at(dX1, parent[sel], dZ[sel] @ W[k].T)
        dW[k] = X1[parent[sel]].T @ dZ[sel]
    return dX1, dW, dZ.sum(0)


def unet_backward(out, params, dY_rows):
    """Backward through the U-Net of ``unet_forward`` (chain rule stage by stage, FP64), from dL/dY
    of the head [n0][d^3].  The gradient of the concatenation splits into its up and skip parts;
    the skip's gradient adds the one arriving through the strided convolution.  Returns
    {stage: [(dW, db), ...]} and dX of the network input."""
    acts = out["acts"]
    inp = acts["inputs"]
    rb0, rb1 = out["rb0"], out["rb1"]
    grads = {st: [None] * len(v) for st, v in params.items()}

    def subm_chain(st, dY, rb, relu_top=True):
        # layers of stage st in reverse; a layer's output is the next layer's input (or the
        # stage's given output for the last one)
        ins = inp[st]
        for i in range(len(ins) - 1, -1, -1):
            W, _ = params[st][i]
            Y = outs[st][i]
            relu = relu_top or i < len(ins) - 1
            dX, dW, db = subm_conv_bwd(ins[i], W, *rb, Y, dY, relu=relu)
            grads[st][i] = (dW, db)
            dY = dX
        return dY

    def stage_outputs(st, last):
        return inp[st][1:] + [last]

    u = acts["up"]
    outs = {"stem": stage_outputs("stem", inp["enc0"][0]), "enc0": stage_outputs("enc0", acts["skip"]),
            "enc1": stage_outputs("enc1", acts["coarse"]), "dec0": stage_outputs("dec0", inp["head"][0]),
            "head": [acts["Y"]]}
    dH = subm_chain("head", dY_rows, rb0, relu_top=False)
    dH = subm_chain("dec0", dH, rb0)
    Dc = u.shape[1]
    dU, dS = dH[:, :Dc], dH[:, Dc:]
    (W, _), = params["up"]
    dC, dW, db = inverse_up_bwd(inp["up"][0], out["parent"], out["kid"], W, u, dU, relu=True)
    grads["up"][0] = (dW, db)
    dC = subm_chain("enc1", dC, rb1)
    (W, _), = params["down"]
    dX0, dW, db = strided_down_bwd(inp["down"][0], out["children"], W, inp["enc1"][0], dC, relu=True)
    grads["down"][0] = (dW, db)
    dS = dS + dX0
    dS = subm_chain("enc0", dS, rb0)
    dX = subm_chain("stem", dS, rb0)
    return grads, dX


# ---------------------------------------------------------------- the U-Net at the BF16 rounding points
def _strided_down_f32(X0, children, W, b, relu: bool):
    X0, W = np.asarray(X0, np.float32), np.asarray(W, np.float32)
    Y = np.zeros((children.shape[1], W.shape[2]), np.float32)
    for k in range(8):
        has = children[k] >= 0
        Y[has] += X0[children[k, has]] @ W[k]
    Y += np.asarray(b, np.float32)
    return np.maximum(Y, 0.0) if relu else Y


def _inverse_up_f32(X1, parent, kid, W, b, relu: bool):
    X1, W = np.asarray(X1, np.float32), np.asarray(W, np.float32)
    Y = np.zeros((len(parent), W.shape[2]), np.float32)
    for k in range(8):
        sel = kid == k
        Y[sel] = X1[parent[sel]] @ W[k]
    Y += np.asarray(b, np.float32)
    return np.maximum(Y, 0.0) if relu else Y


def unet_forward_bf16(tris, dims, d, params, occ=None, accum: str = "f64"):
    """``unet_forward`` at the BF16 path's rounding points: every weight rounded to bfloat16 from
    its float32 master, each layer's result after bias and ReLU (stem, enc0, down, enc1, up,
    dec0) rounded to bfloat16, the concatenation joining rounded values, the head's logits not
    rounded.  FP64 between the rounding points; accum = "f32" evaluates every sum with float32
    accumulation instead (a second evaluation order, for sizing tolerances only).  Returns the
    keys of ``unet_forward`` plus Wr (the rounded weights by stage)."""
    nx, ny, nz = dims
    if occ is None:
        occ, _ = froxelize(tris, dims)
    f32 = accum == "f32"
    b0 = (nx // d, ny // d, nz // d)
    keys0 = active_sites(occ, dims, d)
    keys1 = active_sites(occ, dims, 2 * d)
    rb0 = rulebook(keys0, b0)
    rb1 = rulebook(keys1, (b0[0] // 2, b0[1] // 2, b0[2] // 2))
    children, parent, kid = level_maps(keys0, keys1, b0)
    Wr = {st: [(bf16_round(np.asarray(W, np.float32)), np.asarray(b, np.float32)) for W, b in v]
          for st, v in params.items()}

    def sub(h, W, b, rb, relu=True):
        y = np.asarray((subm_conv_f32 if f32 else subm_conv)(h, W, b, *rb, relu=relu), np.float64)
        return bf16_round(y) if relu else y

    acts = {"X": gather_sites(occ, dims, d, keys0)}
    inputs = {st: [] for st in params}
    h = acts["X"]
    for st in ("stem", "enc0"):
        for W, b in Wr[st]:
            inputs[st].append(h)
            h = sub(h, W, b, rb0)
    acts["skip"] = h
    (W, b), = Wr["down"]
    inputs["down"].append(h)
    h1 = bf16_round(np.asarray((_strided_down_f32 if f32 else strided_down)(h, children, W, b, True), np.float64))
    for W, b in Wr["enc1"]:
        inputs["enc1"].append(h1)
        h1 = sub(h1, W, b, rb1)
    acts["coarse"] = h1
    (W, b), = Wr["up"]
    inputs["up"].append(h1)
    u = bf16_round(np.asarray((_inverse_up_f32 if f32 else inverse_up)(h1, parent, kid, W, b, True), np.float64))
    acts["up"] = u
    h = np.concatenate([u, acts["skip"]], axis=1)
    for W, b in Wr["dec0"]:
        inputs["dec0"].append(h)
        h = sub(h, W, b, rb0)
    (W, b), = Wr["head"]
    inputs["head"].append(h)
    Y = sub(h, W, b, rb0, relu=False)
    acts["Y"] = Y
    acts["inputs"] = inputs
    logits, pvs = deinterleave_threshold(Y, keys0, occ, dims, d)
    return dict(occ=occ, keys0=keys0, keys1=keys1, children=children, parent=parent, kid=kid, acts=acts,
                rb0=rb0, rb1=rb1, logits=logits, pvs=pvs, Wr=Wr)


def unet_backward_bf16(out, dY_rows, accum: str = "f64"):
    """Backward of ``unet_forward_bf16`` at the BF16 path's rounding points: per layer,
    dZ = dY [Y > 0] (no mask on the head), its bfloat16 rounding dZb is the operand of the
    products (dX = dZb W^T through the layer's pairs or children, dW = X^T dZb with the layer's
    bfloat16 input), db = sum dZ unrounded; the concatenation's gradient splits into its up and
    skip parts, and the skip's part adds the gradient through the strided convolution (one
    addition of two values).  FP64 between the rounding points, or float32 accumulation with
    accum = "f32".  Returns {stage: [(dW, db), ...]}."""
    f32 = accum == "f32"
    acts, Wr = out["acts"], out["Wr"]
    inp = acts["inputs"]
    rb0, rb1 = out["rb0"], out["rb1"]
    children, parent, kid = out["children"], out["parent"], out["kid"]
    grads = {st: [None] * len(v) for st, v in Wr.items()}
    cast = (lambda a: np.asarray(np.asarray(a, np.float32), np.float64)) if f32 else (lambda a: a)

    def layer_bwd(kind, X, W, Y, dY, relu, rb=None):
        dZ = dY * (Y > 0) if relu else dY
        dZb = bf16_round(dZ)
        if kind == "subm":
            if f32:
                dX, dW = subm_conv_bwd_f32(X, W, *rb, dZb)
            else:
                dX, dW, _ = subm_conv_bwd(X, W, *rb, None, dZb, relu=False)
        else:
            X32, W32, dZ32 = (np.asarray(a, np.float32 if f32 else np.float64) for a in (X, W, dZb))
            dX = np.zeros_like(X32)
            dW = np.zeros_like(W32)
            for k in range(8):
                if kind == "down":
                    has = children[k] >= 0
                    rows = children[k, has]
                    dX[rows] = dZ32[has] @ W32[k].T
                    dW[k] = X32[rows].T @ dZ32[has]
                else:
                    sel = kid == k
                    np.add.at(dX, parent[sel], dZ32[sel] @ W32[k].T)
                    dW[k] = X32[parent[sel]].T @ dZ32[sel]
        db = np.asarray(dZ, np.float32).sum(0, dtype=np.float32) if f32 else dZ.sum(0)
        return cast(dX), np.asarray(dW, np.float64), np.asarray(db, np.float64)

    def chain(st, dY, rb, last_out, relu_top=True):
        ins = inp[st]
        outs = ins[1:] + [last_out]
        for i in range(len(ins) - 1, -1, -1):
            dY, dW, db = layer_bwd("subm", ins[i], Wr[st][i][0], outs[i], dY, relu_top or i < len(ins) - 1, rb)
            grads[st][i] = (dW, db)
        return dY

    dH = chain("head", cast(dY_rows), rb0, acts["Y"], relu_top=False)
    dH = chain("dec0", dH, rb0, inp["head"][0])
    Dc = acts["up"].shape[1]
    dU, dS = dH[:, :Dc], dH[:, Dc:]
    dC, dW, db = layer_bwd("up", inp["up"][0], Wr["up"][0][0], acts["up"], dU, True)
    grads["up"][0] = (dW, db)
    dC = chain("enc1", dC, rb1, acts["coarse"])
    dX0, dW, db = layer_bwd("down", inp["down"][0], Wr["down"][0][0], inp["enc1"][0], dC, True)
    grads["down"][0] = (dW, db)
    dS = cast(dS + dX0)
    dS = chain("enc0", dS, rb0, acts["skip"])
    chain("stem", dS, rb0, inp["enc0"][0])
    return grads


# ---------------------------------------------------------------- world-space front end
def viewcell_view(c, forward, up, fov_y, aspect, r, beta, z_near, z_far):
    """The frustum F of a viewcell (Sec. 3.2): a camera at c looking along `forward` with
    vertical field of view fov_y (radians) may move laterally by up to r and turn by up to beta;
    F has its apex at c' = c - r / tan(fov_y / 2) * forward and the field of view fov_y + 2 beta
    (horizontal: aspect times its tangent).  Returns a dict: eye, right, up, fwd (orthonormal;
    right = up x forward), tx, ty (half-angle tangents), zn, zf (linear depth range)."""
    f = np.asarray(forward, np.float64)
    f = f / np.linalg.norm(f)
    rt = np.cross(np.asarray(up, np.float64), f)
    rt = rt / np.linalg.norm(rt)
    u = np.cross(f, rt)
    eye = np.asarray(c, np.float64) - r / np.tan(fov_y / 2.0) * f
    ty = np.tan((fov_y + 2.0 * beta) / 2.0)
    return dict(eye=eye, right=rt, up=u, fwd=f, tx=aspect * ty, ty=ty, zn=float(z_near), zf=float(z_far))


def froxelize_view(tris_world, view, dims, margin: float = 0.0):
    """Packed occupancy [nz][ny][nx/8] of world-space triangles in the froxels of `view` (linear
    depth slices); `margin` widens (> 0) or shrinks (< 0) every froxel by that fraction of its
    extent per axis in (x/z, y/z, 1/z).  Returns (occ, number of marked froxels)."""
    nx, ny, nz = dims
    t = _c(tris_world, np.float32).reshape(-1, 3, 3)
    occ = np.zeros((nz, ny, nx // 8), np.uint8)
    v = {k: _c(view[k], np.float64) for k in ("eye", "right", "up", "fwd")}
    n = _load().oracle_froxelize_view(_p(t), t.shape[0], _p(v["eye"]), _p(v["right"]), _p(v["up"]), _p(v["fwd"]),
                                      view["tx"], view["ty"], view["zn"], view["zf"], nx, ny, nz, margin, _p(occ))
    return occ, n
