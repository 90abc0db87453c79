"""ctypes loader of ``libneuralpvs.so`` (the gfx950 HIP library).

Argument marshalling only.  There is no fallback: if the library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libneuralpvs.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "neuralpvs.h")

NPVS_OK = 0
NPVS_ERR_INVALID_ARG = -1
NPVS_ERR_CAPACITY = -2
NPVS_ERR_HIP = -3
NPVS_ERR_UNSUPPORTED = -4
NPVS_F32, NPVS_BF16, NPVS_U8 = 0, 1, 2
NPVS_MAX_GRIDS = 32
NPVS_CONV_VARIANTS = 16
NPVS_DEFAULT_CONV_VARIANT = 15
NPVS_MAX_PACK = 64
NPVS_MAX_ADAM_PACK = 32
NPVS_MAX_WGRAD_LAYERS = 16
NPVS_LOSS_BCE = 0
NPVS_LOSS_DICE = 1


class NpvsError(RuntimeError):
    def __init__(self, code: int, fn: str, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


class Dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class Counts(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("n_sites_needed", ctypes.c_int32),
                ("n_pairs", ctypes.c_int32), ("n_tris_ignored", ctypes.c_int32)]


class PackDesc(ctypes.Structure):
    _fields_ = [("W", ctypes.c_void_p), ("Wp", ctypes.c_void_p), ("cin", ctypes.c_int32), ("cout", ctypes.c_int32),
                ("flip_transpose", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class View(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("right", ctypes.c_double * 3), ("up", ctypes.c_double * 3),
                ("forward", ctypes.c_double * 3), ("tan_half_x", ctypes.c_double), ("tan_half_y", ctypes.c_double),
                ("z_near", ctypes.c_double), ("z_far", ctypes.c_double)]


class WgradLayer(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("cin", ctypes.c_int32), ("cout", ctypes.c_int32), ("ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_size_t), ("dW", ctypes.c_void_p), ("db", ctypes.c_void_p)]


class AdamPackDesc(ctypes.Structure):
    _fields_ = [("off", ctypes.c_int64), ("cin", ctypes.c_int32), ("cout", ctypes.c_int32), ("Wp", ctypes.c_void_p),
                ("Wt", ctypes.c_void_p)]


P = ctypes.c_void_p
i32, i64, f32, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
f64 = ctypes.c_double
PS = ctypes.POINTER(ctypes.c_size_t)
PI64 = ctypes.POINTER(ctypes.c_int64)

SIGNATURES = {
    "npvs_version": (ctypes.c_char_p, []),
    "npvs_source_hash": (ctypes.c_char_p, []),
    "npvs_last_error": (ctypes.c_char_p, []),
    "npvs_batch_sizes": (i32, [i32, P, i32, PI64, PI64]),
    "npvs_froxelize_workspace_size": (i32, [i32, P, P, PS]),
    "npvs_froxelize": (i32, [P, P, i32, P, P, P, P, sz, P]),
    "npvs_rulebook_workspace_size": (i32, [i32, P, i32, i32, PS]),
    "npvs_build_rulebook": (i32, [P, i32, P, i32, i32, P, P, P, P, P, P, P, P, sz, P]),
    "npvs_build_rulebook_noalloc": (i32, [P, i32, P, i32, i32, P, P, P, P, P, P, P, P]),
    "npvs_interleave": (i32, [P, Dims, i32, i32, P, P]),
    "npvs_deinterleave": (i32, [P, Dims, i32, i32, P, P]),
    "npvs_gather_input": (i32, [P, i32, P, i32, P, P, i32, i32, i32, P, P, P, P]),
    "npvs_packed_weight_bytes": (sz, [i32, i32, i32]),
    "npvs_pack_weights": (i32, [P, i32, i32, i32, i32, P, P]),
    "npvs_pack_weights_batch": (i32, [i32, P, i32, P]),
    "npvs_sparse_conv_fwd": (i32, [P, i32, P, P, i32, P, P, i32, i32, i32, i32, i32, P, P, sz, P]),
    "npvs_conv_fwd_workspace_size": (i32, [i32, i32, i32, i32, PS]),
    "npvs_conv_bwd_workspace_size": (i32, [i32, i32, i32, i32, PS]),
    "npvs_sparse_conv_bwd": (i32, [P, i32, P, i32, P, P, P, P, P, P, i32, i32, i32, P, P, P, P, sz, P, P, P]),
    "npvs_sparse_conv_wgrad": (i32, [i32, P, P, P, i32, i32, i32, P]),
    "npvs_sparse_conv_dgrad_relu": (i32, [P, i32, i32, P, i32, P, P, i32, P, sz, P, sz, P]),
    "npvs_level_maps": (i32, [i32, P, i32, P, P, P, i32, P, P, P, i32, P, P, P]),
    "npvs_packed_weight_bytes_k": (sz, [i32, i32, i32, i32]),
    "npvs_pack_weights_k": (i32, [P, i32, i32, i32, i32, i32, P, P]),
    "npvs_strided_conv_fwd": (i32, [P, i32, P, P, i32, P, i32, P, i32, i32, i32, i32, P, P]),
    "npvs_concat_channels": (i32, [P, i32, P, i32, i32, P, i32, P, P]),
    "npvs_strided_bwd_workspace_size": (i32, [i32, i32, i32, i32, i32, i32, PS]),
    "npvs_strided_conv_bwd": (i32, [P, i32, P, i32, P, P, P, P, i32, P, i32, P, i32, i32, i32, P, P, P, P, sz, P]),
    "npvs_concat_channels_bwd": (i32, [P, i32, i32, P, P, i32, P, P, P]),
    "npvs_viewcell_frustum": (i32, [P, P, P, f64, f64, f64, f64, f64, f64, P]),
    "npvs_froxelize_view_workspace_size": (i32, [i64, PS]),
    "npvs_froxelize_view": (i32, [P, i64, P, Dims, P, P, sz, P]),
    "npvs_visible_triangles": (i32, [P, PI64, i32, P, P, P, P]),
    "npvs_visible_objects": (i32, [P, P, i64, P, P]),
    "npvs_deinterleave_threshold": (i32, [P, i32, P, P, i32, P, i32, P, P, P]),
    "npvs_loss_workspace_size": (i32, [i32, PS]),
    "npvs_loss": (i32, [P, P, i32, P, i32, P, i32, f32, i32, f32, P, P, P, sz, i32, P, sz, P]),
    "npvs_adam": (i32, [P, P, P, P, i64, P, f32, f32, f32, f32, f32, i32, P, i32, P]),
    "npvs_plan_create": (i32, [i32, P, P, i32, i32, P, i32, ctypes.POINTER(P)]),
    "npvs_plan_destroy": (i32, [P]),
    "npvs_plan_set_weights": (i32, [P, i32, P, P, P]),
    "npvs_pvs_forward": (i32, [P, P, P, P, P, P]),
    "npvs_plan_capture": (i32, [P, P, P, P, P, P]),
    "npvs_plan_replay": (i32, [P, P]),
    "npvs_plan_counts": (i32, [P, ctypes.POINTER(Counts), P]),
    "npvs_plan_autotune": (i32, [P, P, i32, P, P]),
}

_lib = None


def header_functions() -> list[str]:
    """Names of the functions declared in include/neuralpvs.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(npvs_[a-z0-9_]+)\s*\(", text)))


def get() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built, or if it was built from sources other
    than the ones in this tree (its compiled-in source hash differs)."""
    global _lib
    if _lib is None:
        from . import build
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        built, want = L.npvs_source_hash().decode(), build.source_hash()
        if built != want:
            raise RuntimeError(f"{LIB_PATH} was built from other sources (hash {built}, the tree's sources hash to "
                               f"{want}): rebuild it (python -c 'import __graft_entry__ as g; g.build()')")
        _lib = L
    return _lib


def call(name: str, *args):
    st = getattr(get(), name)(*args)
    if st != NPVS_OK:
        raise NpvsError(st, name, get().npvs_last_error().decode(errors="replace"))
    return st


def dims_array(dims) -> ctypes.Array:
    arr = (Dims * len(dims))()
    for i, (nx, ny, nz) in enumerate(dims):
        arr[i] = Dims(int(nx), int(ny), int(nz))
    return arr


def i64_array(vals) -> ctypes.Array:
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])
