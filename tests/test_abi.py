"""The C ABI library loads on any host and exports every function include/neuralpvs.h declares;
host-side argument checks answer without a GPU (nothing is enqueued on these paths)."""
import ctypes

import pytest

from paper_2509_24677_amd import _lib as L


@pytest.fixture(scope="module")
def lib():
    return L.get()


def test_exports_every_declared_function(lib):
    names = L.header_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(L.SIGNATURES) == names  # the binding covers exactly the header


def test_version_and_sizes(lib):
    assert lib.npvs_version().decode().startswith("neuralpvs-gfx950")
    tb, tby = ctypes.c_int64(), ctypes.c_int64()
    L.call("npvs_batch_sizes", 2, L.dims_array([(256, 256, 128), (64, 64, 64)]), 4, ctypes.byref(tb), ctypes.byref(tby))
    assert tb.value == 64 * 64 * 32 + 16 ** 3
    assert tby.value == 128 * 256 * 32 + 64 * 64 * 8
    assert lib.npvs_packed_weight_bytes(64, 64, L.NPVS_F32) == 27 * 64 * 64 * 4
    assert lib.npvs_packed_weight_bytes(64, 64, L.NPVS_BF16) == 27 * 4 * 2 * 1024
    n = ctypes.c_size_t()
    L.call("npvs_froxelize_workspace_size", 1, L.dims_array([(256, 256, 128)]), L.i64_array([50000]), ctypes.byref(n))
    assert n.value > 50000 * 48


def test_header_constants_match_binding():
    text = open(L.HEADER).read()
    for name in ("NPVS_MAX_GRIDS", "NPVS_MAX_PACK", "NPVS_CONV_VARIANTS", "NPVS_DEFAULT_CONV_VARIANT",
                 "NPVS_LOSS_BCE", "NPVS_LOSS_DICE", "NPVS_MAX_ADAM_PACK", "NPVS_MAX_WGRAD_LAYERS"):
        assert f"#define {name} {getattr(L, name)}" in text, name
    assert ctypes.sizeof(L.PackDesc) == 32 and ctypes.sizeof(L.Counts) == 16 and ctypes.sizeof(L.AdamPackDesc) == 32
    assert ctypes.sizeof(L.WgradLayer) == 48
    assert "int64_t t;\n  float c1, c2;\n} npvs_adam_step;" in text  # 16 bytes, as the binding assumes


def test_conv_workspace_sizes_and_checks(lib):
    n = ctypes.c_size_t()
    L.call("npvs_conv_fwd_workspace_size", 4096, 64, 1000, L.NPVS_BF16, ctypes.byref(n))
    assert n.value == 16 * 1000 * 64 * 4  # 128 chunks of 32 channels split 16 ways, float32 partials
    for cin, cout, dt in ((64, 64, L.NPVS_BF16), (512, 64, L.NPVS_BF16), (4096, 64, L.NPVS_F32)):
        L.call("npvs_conv_fwd_workspace_size", cin, cout, 1000, dt, ctypes.byref(n))
        assert n.value == 0
    fake = ctypes.c_void_p(16)  # never dereferenced: the argument checks answer first

    def fwd(variant=-1, ws=None, ws_bytes=0, cin=4096):
        return lib.npvs_sparse_conv_fwd(fake, cin, fake, None, 64, fake, fake, 1000, L.NPVS_BF16, 1, 0, variant,
                                        ctypes.c_void_p(32), ws, ws_bytes, None)

    # a workspace given, but smaller than the split needs
    assert fwd(ws=fake, ws_bytes=16) == L.NPVS_ERR_INVALID_ARG and b"workspace" in lib.npvs_last_error()
    for v in (-2, L.NPVS_CONV_VARIANTS):
        assert fwd(variant=v) == L.NPVS_ERR_INVALID_ARG and b"variant" in lib.npvs_last_error()
    assert lib.npvs_sparse_conv_fwd(fake, 64, fake, None, 64, fake, fake, 1000, L.NPVS_BF16, 1, 0, -1, fake, None, 0,
                                    None) == L.NPVS_ERR_INVALID_ARG  # X aliases Y
    L.call("npvs_conv_bwd_workspace_size", 64, 64, 1000, L.NPVS_BF16, ctypes.byref(n))
    bwd = [fake, 64, fake, 64, fake, fake, fake, fake, fake, fake, 1000, L.NPVS_BF16, 1, fake, fake, fake, fake,
           n.value, None, None, None]
    bad = list(bwd)
    bad[17] = n.value - 1
    assert lib.npvs_sparse_conv_bwd(*bad) == L.NPVS_ERR_INVALID_ARG and b"workspace" in lib.npvs_last_error()
    bad = list(bwd)
    bad[1] = 60  # BF16 needs multiples of 8
    assert lib.npvs_sparse_conv_bwd(*bad) == L.NPVS_ERR_UNSUPPORTED
    bad = list(bwd)
    bad[15] = None  # dW given, db null
    assert lib.npvs_sparse_conv_bwd(*bad) == L.NPVS_ERR_INVALID_ARG and b"both" in lib.npvs_last_error()


def test_gather_argument_checks(lib):
    fake = ctypes.c_void_p(16)  # never dereferenced: the argument checks answer first
    dims = L.dims_array([(32, 32, 32)])
    assert lib.npvs_gather_input(fake, 1, dims, 4, fake, fake, 100, L.NPVS_BF16, 0, fake, fake, None,
                                 None) == L.NPVS_ERR_INVALID_ARG and b"both" in lib.npvs_last_error()
    assert lib.npvs_gather_input(fake, 1, dims, 4, fake, fake, 100, L.NPVS_BF16, 32, fake, None, None,
                                 None) == L.NPVS_ERR_INVALID_ARG and b"row_stride" in lib.npvs_last_error()


def test_loss_argument_checks(lib):
    fake = ctypes.c_void_p(16)  # never dereferenced: the argument checks answer first
    nl = ctypes.c_size_t()
    L.call("npvs_loss_workspace_size", 1, ctypes.byref(nl))
    n = ctypes.c_size_t()
    L.call("npvs_conv_bwd_workspace_size", 64, 64, 1000, L.NPVS_BF16, ctypes.byref(n))

    def call(C=64, dz_ws=ctypes.c_void_p(4096), dz_bytes=None, dz_cin=64, term=L.NPVS_LOSS_BCE):
        return lib.npvs_loss(ctypes.c_void_p(1024), fake, C, fake, 1, fake, 1000, 0.99, term, 0.0, fake, None, dz_ws,
                             n.value if dz_bytes is None else dz_bytes, dz_cin, fake, nl.value, None)

    assert call(term=7) == L.NPVS_ERR_INVALID_ARG and b"term" in lib.npvs_last_error()
    assert call(C=60) == L.NPVS_ERR_UNSUPPORTED and b"multiples of 8" in lib.npvs_last_error()
    assert call(dz_cin=12) == L.NPVS_ERR_UNSUPPORTED
    assert call(dz_bytes=n.value - 1) == L.NPVS_ERR_INVALID_ARG and b"dZ workspace" in lib.npvs_last_error()


def test_fused_data_gradient_argument_checks(lib):
    fake = ctypes.c_void_p(16)  # never dereferenced: the argument checks answer first
    n = ctypes.c_size_t()
    L.call("npvs_conv_bwd_workspace_size", 64, 64, 1000, L.NPVS_BF16, ctypes.byref(n))

    def call(cin=64, cout=64, cin_below=64, ws=fake, ws_bytes=None, ws_below=ctypes.c_void_p(32), wsb_bytes=None,
             Wt=fake):
        return lib.npvs_sparse_conv_dgrad_relu(Wt, cin, cout, fake, cin_below, fake, fake, 1000, ws,
                                               n.value if ws_bytes is None else ws_bytes, ws_below,
                                               n.value if wsb_bytes is None else wsb_bytes, None)

    assert call(Wt=None) == L.NPVS_ERR_INVALID_ARG and b"null" in lib.npvs_last_error()
    assert call(ws_below=fake) == L.NPVS_ERR_INVALID_ARG and b"differ" in lib.npvs_last_error()
    assert call(cin=96) == L.NPVS_ERR_UNSUPPORTED
    assert call(cout=60) == L.NPVS_ERR_UNSUPPORTED
    assert call(cin_below=12) == L.NPVS_ERR_UNSUPPORTED
    assert call(ws_bytes=n.value - 1) == L.NPVS_ERR_INVALID_ARG and b"workspace too small" in lib.npvs_last_error()
    assert call(wsb_bytes=16) == L.NPVS_ERR_INVALID_ARG and b"layer below" in lib.npvs_last_error()


def test_batched_weight_gradient_argument_checks(lib):
    fake = ctypes.c_void_p(16)  # never dereferenced: the argument checks answer first
    n = ctypes.c_size_t()
    L.call("npvs_conv_bwd_workspace_size", 64, 64, 1000, L.NPVS_BF16, ctypes.byref(n))

    def call(descs, nl=None, dtype=L.NPVS_BF16, slices=0, rb=fake):
        arr = (L.WgradLayer * len(descs))(*descs) if descs else None
        return lib.npvs_sparse_conv_wgrad(len(descs) if nl is None else nl, arr, rb, fake, 1000, dtype, slices, None)

    good = L.WgradLayer(16, 64, 64, 16, n.value, 16, 16)
    assert call([], nl=0) == L.NPVS_ERR_INVALID_ARG
    assert call([good] * (L.NPVS_MAX_WGRAD_LAYERS + 1)) == L.NPVS_ERR_INVALID_ARG
    assert call([good], rb=None) == L.NPVS_ERR_INVALID_ARG and b"null" in lib.npvs_last_error()
    assert call([good], dtype=L.NPVS_U8) == L.NPVS_ERR_INVALID_ARG and b"dtype" in lib.npvs_last_error()
    assert call([good], slices=-1) == L.NPVS_ERR_INVALID_ARG
    assert call([good, L.WgradLayer(16, 64, 64, 16, n.value, 16, None)]) == L.NPVS_ERR_INVALID_ARG
    assert call([L.WgradLayer(16, 64, 64, 16, n.value - 1, 16, 16)]) == L.NPVS_ERR_INVALID_ARG
    assert b"workspace" in lib.npvs_last_error()
    assert call([L.WgradLayer(16, 60, 64, 16, n.value, 16, 16)]) == L.NPVS_ERR_UNSUPPORTED


def test_batched_packing_argument_checks(lib):
    assert lib.npvs_pack_weights_batch(0, None, L.NPVS_BF16, None) == L.NPVS_OK
    assert lib.npvs_pack_weights_batch(L.NPVS_MAX_PACK + 1, None, L.NPVS_BF16, None) == L.NPVS_ERR_INVALID_ARG
    d = (L.PackDesc * 1)(L.PackDesc(None, None, 8, 8, 0, 0))
    assert lib.npvs_pack_weights_batch(1, ctypes.cast(d, ctypes.c_void_p), L.NPVS_BF16, None) == L.NPVS_ERR_INVALID_ARG
    assert b"null pointer" in lib.npvs_last_error()


def test_adam_pack_argument_checks(lib):
    fake = ctypes.c_void_p(0x1000)

    def call(descs, n=1000, nl=None):
        arr = (L.AdamPackDesc * len(descs))(*descs) if descs else None
        return lib.npvs_adam(fake, fake, fake, fake, n, fake, 1e-3, 0.9, 0.999, 1e-8, 0.0,
                             len(descs) if nl is None else nl, arr, L.NPVS_BF16, None)

    assert call([], nl=L.NPVS_MAX_ADAM_PACK + 1) == L.NPVS_ERR_INVALID_ARG
    # a layer reaching past the parameter buffer (27 * 8 * 8 = 1728 > 1000)
    assert call([L.AdamPackDesc(0, 8, 8, 0x2000, 0x3000)]) == L.NPVS_ERR_INVALID_ARG
    assert b"outside" in lib.npvs_last_error()
    # overlapping layers
    d = [L.AdamPackDesc(0, 4, 4, 0x2000, 0x3000), L.AdamPackDesc(100, 4, 4, 0x4000, 0x5000)]
    assert call(d) == L.NPVS_ERR_INVALID_ARG and b"overlapping" in lib.npvs_last_error()
    # missing packing buffer
    assert call([L.AdamPackDesc(0, 4, 4, 0x2000, None)]) == L.NPVS_ERR_INVALID_ARG


@pytest.mark.parametrize("dims,d,msg", [
    ([(250, 256, 128)], 4, "multiple of 8"),
    ([(256, 256, 126)], 4, "multiples of d"),
    ([(2048, 256, 128)], 4, "1024"),
    ([(256, 256, 128)], 3, "power of two"),
])
def test_bad_dims_rejected(lib, dims, d, msg):
    tb, tby = ctypes.c_int64(), ctypes.c_int64()
    st = lib.npvs_batch_sizes(len(dims), L.dims_array(dims), d, ctypes.byref(tb), ctypes.byref(tby))
    assert st == L.NPVS_ERR_INVALID_ARG
    assert msg in lib.npvs_last_error().decode()


def test_too_many_grids_and_null_pointers(lib):
    tb, tby = ctypes.c_int64(), ctypes.c_int64()
    dims = L.dims_array([(64, 64, 64)] * 33)
    assert lib.npvs_batch_sizes(33, dims, 4, ctypes.byref(tb), ctypes.byref(tby)) == L.NPVS_ERR_INVALID_ARG
    one = L.dims_array([(64, 64, 64)])
    st = lib.npvs_froxelize(None, L.i64_array([1]), 1, one, None, None, None, 0, None)
    assert st == L.NPVS_ERR_INVALID_ARG
    st = lib.npvs_sparse_conv_fwd(None, 64, None, None, 64, None, None, 10, 0, 1, 0, -1, None, None, 0, None)
    assert st == L.NPVS_ERR_INVALID_ARG
    st = lib.npvs_build_rulebook(ctypes.c_void_p(16), 1, one, 4, 10, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                 ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                 None, ctypes.c_void_p(16), 1 << 20, None)
    assert st == L.NPVS_ERR_INVALID_ARG and "rb_off and rb_pairs" in lib.npvs_last_error().decode()


def test_workspace_too_small_is_rejected(lib):
    one = L.dims_array([(64, 64, 64)])
    p = ctypes.c_void_p(256)
    st = lib.npvs_froxelize(p, L.i64_array([10]), 1, one, p, None, p, 16, None)
    assert st == L.NPVS_ERR_INVALID_ARG and "workspace" in lib.npvs_last_error().decode()


def test_unsupported_bf16_shape_reported(lib):
    p = ctypes.c_void_p(256)
    st = lib.npvs_sparse_conv_fwd(p, 12, p, None, 64, p, p, 10, L.NPVS_BF16, 1, 0, -1, ctypes.c_void_p(512), None, 0,
                                  None)
    assert st == L.NPVS_ERR_UNSUPPORTED


def test_viewcell_frustum_matches_oracle_and_rejects_bad_cameras(lib):
    import math

    import numpy as np

    import oracle
    import paper_2509_24677_amd as npvs

    rng = np.random.default_rng(4)
    for _ in range(20):
        c, f, u = rng.normal(size=3) * 10, rng.normal(size=3), rng.normal(size=3)
        fov, asp, r, beta = rng.uniform(0.3, 1.5), rng.uniform(0.5, 2), rng.uniform(0, 1), rng.uniform(0, 0.4)
        v = npvs.viewcell_frustum(c, f, u, fov, asp, r, beta, 0.3, 1000.0)
        w = oracle.viewcell_view(c, f, u, fov, asp, r, beta, 0.3, 1000.0)
        for key, wk in (("eye", "eye"), ("right", "right"), ("up", "up"), ("forward", "fwd")):
            np.testing.assert_allclose(list(getattr(v, key)), w[wk], rtol=0, atol=1e-12)
        assert v.tan_half_x == pytest.approx(w["tx"], rel=1e-14) and v.tan_half_y == pytest.approx(w["ty"], rel=1e-14)
    arr = lambda x: (ctypes.c_double * 3)(*x)
    out = L.View()
    p = lambda x: ctypes.cast(arr(x), ctypes.c_void_p)
    st = lib.npvs_viewcell_frustum(p([0, 0, 0]), p([0, 0, 1]), p([0, 0, 2]), math.pi / 3, 1.0, 0.6, 0.2, 0.3, 100.0,
                                   ctypes.byref(out))
    assert st == L.NPVS_ERR_INVALID_ARG and b"parallel" in lib.npvs_last_error()
    st = lib.npvs_viewcell_frustum(p([0, 0, 0]), p([0, 0, 1]), p([0, 1, 0]), math.pi / 3, 1.0, 0.6, 0.2, 100.0, 50.0,
                                   ctypes.byref(out))
    assert st == L.NPVS_ERR_INVALID_ARG


def test_noalloc_rulebook_refuses_a_batch_beyond_its_scratch(lib):
    # a 1024^3 grid at d = 4 needs 1.7 MiB of rulebook workspace, beyond the 1 MiB static scratch:
    # refused with NPVS_ERR_CAPACITY before any device call (none is made on this host)
    dims = L.dims_array([(1024, 1024, 1024)])
    cap = 256 * 256 * 256
    need = ctypes.c_size_t()
    L.call("npvs_rulebook_workspace_size", 1, dims, 4, cap, ctypes.byref(need))
    assert need.value > (1 << 20)
    assert "#define NPVS_RULEBOOK_SCRATCH_BYTES (1u << 20)" in open(L.HEADER).read()
    st = lib.npvs_build_rulebook_noalloc(None, 1, dims, 4, cap, None, None, None, None, None, None, None, None)
    assert st == L.NPVS_ERR_CAPACITY and b"scratch" in lib.npvs_last_error()
    # 32 city-size grids fit
    L.call("npvs_rulebook_workspace_size", 32, L.dims_array([(256, 256, 128)] * 32), 4, 32 * 64 * 64 * 32,
           ctypes.byref(need))
    assert need.value <= (1 << 20)
