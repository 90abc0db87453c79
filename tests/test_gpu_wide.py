"""GPU parity of the general BF16 convolution (channel counts the tuned tile shapes do not cover)
and of whole networks at the paper's interleave factors d = 8 and 16, whose first and last layers
are d^3 = 512 or 4096 channels wide, against the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_24677_amd as npvs
import synth
from gpu_util import DEV, bf16_round, conv_tolerance, oracle_batch, to_np, upload_tris

pytestmark = pytest.mark.gpu


def _case(cin, cout, d, seed=3):
    dims = [(64, 64, 64), (32, 32, 32)]
    tri_list = [synth.box_scene(seed + i, g, 25, 2, 10) for i, g in enumerate(dims)]
    tris, counts = upload_tris(tri_list)
    occ = npvs.froxelize(tris, counts, dims)
    rb = npvs.build_rulebook(occ, dims, d)
    ref = oracle_batch(tri_list, dims, d)
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(rb.cap, cin)).astype(np.float32)
    W = (rng.normal(size=(27, cin, cout)) / np.sqrt(27 * cin)).astype(np.float32)
    b = rng.normal(size=cout).astype(np.float32)
    return rb, ref, X, W, b


@pytest.mark.parametrize("variant", [0, 5, 12, 13])
@pytest.mark.parametrize("cin,cout,d", [(128, 64, 4), (96, 24, 4), (64, 200, 4), (32, 64, 4), (512, 512, 8),
                                        (4096, 64, 16), (64, 4096, 16)])
def test_conv_fwd_bf16_general_shapes(cin, cout, d, variant):
    rb, ref, X, W, b = _case(cin, cout, d)
    n = ref["n"]
    Xb = torch.from_numpy(X).to(DEV).to(torch.bfloat16)
    Wp = npvs.pack_weights(torch.from_numpy(W).to(DEV), npvs.NPVS_BF16)
    bt = torch.from_numpy(b).to(DEV)
    Y = torch.full((rb.cap, cout), 7.0, device=DEV)
    npvs.sparse_conv_fwd(Xb, Wp, bt, cin, cout, rb, npvs.NPVS_BF16, True, out_f32=True, out=Y, variant=variant)
    Xr, Wr = bf16_round(X[:n]), bf16_round(W)
    want = oracle.subm_conv(Xr, Wr, b, ref["rb_off"], ref["pairs"], True)
    tol = conv_tolerance(Xr, Wr, ref["rb_off"], ref["pairs"])
    got = to_np(Y)
    err = np.abs(got[:n] - want)
    assert (err <= tol).all(), (err.max(), tol.max())
    assert (got[n:] == 7.0).all()  # rows past the active sites are untouched
    # bf16 output: the float32 result rounded to nearest even
    Yb = npvs.sparse_conv_fwd(Xb, Wp, bt, cin, cout, rb, npvs.NPVS_BF16, True, variant=variant)
    np.testing.assert_array_equal(to_np(Yb)[:n], to_np(Y[:n].to(torch.bfloat16)))


@pytest.mark.parametrize("name", ["boxes64_d8", "boxes64_d16"])
@pytest.mark.parametrize("dtype", [npvs.NPVS_F32, npvs.NPVS_BF16])
def test_network_at_paper_interleave_factors(name, dtype):
    cfg = synth.config(name)
    t = synth.scene_for(cfg)
    layers = synth.net_layers(cfg, bias_std=0.05)
    tris, counts = upload_tris([t])
    plan = npvs.Plan(cfg.grids, counts, cfg.d, cfg.channels, dtype)
    for li, (W, b) in enumerate(layers):
        plan.set_weights(li, torch.from_numpy(W).to(DEV), torch.from_numpy(b).to(DEV))
    pvs, logits = plan.forward(tris, want_logits=True)
    out = oracle.forward(t, cfg.grids[0], cfg.d, layers)
    ref = out["logits"].reshape(-1)
    act = np.isfinite(ref)
    got = to_np(logits)
    assert act.any()
    assert (got[~act] == -np.inf).all()
    err = np.abs(got[act] - ref[act]).max()
    assert err <= (1e-5 if dtype == npvs.NPVS_F32 else 0.1), err
    if dtype == npvs.NPVS_F32:  # the thresholded bits agree wherever the logit is not within the error
        pv = np.unpackbits(to_np(pvs), bitorder="little")
        pw = np.unpackbits(out["pvs"].reshape(-1), bitorder="little")
        safe = np.abs(np.nan_to_num(ref, neginf=-1e9)) > 1e-5
        np.testing.assert_array_equal(pv[safe], pw[safe])
