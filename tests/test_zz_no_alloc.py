"""The workspace-free rulebook entry point (npvs_build_rulebook_noalloc): its output equals
npvs_build_rulebook's bit for bit on two calls in a row (a 256x256x128 city frame, then a
smaller 32^3 grid, so the second call runs over scratch contents left by the first).  The
refusal of a batch beyond the scratch is checked without a GPU in test_abi.py."""
import numpy as np
import pytest
import torch

import paper_2509_24677_amd as npvs
import synth
from gpu_util import DEV, to_np, upload_tris

pytestmark = pytest.mark.gpu


def _compare(rb_a, rb_b):
    ca, cb = rb_a.host_counts(), rb_b.host_counts()
    assert ca == cb
    n, P = ca["n_sites"], ca["n_pairs"]
    np.testing.assert_array_equal(to_np(rb_a.site_keys)[:n], to_np(rb_b.site_keys)[:n])
    np.testing.assert_array_equal(to_np(rb_a.block_row), to_np(rb_b.block_row))
    np.testing.assert_array_equal(to_np(rb_a.grid_rows), to_np(rb_b.grid_rows))
    np.testing.assert_array_equal(to_np(rb_a.nbr)[:, :n], to_np(rb_b.nbr)[:, :n])
    np.testing.assert_array_equal(to_np(rb_a.rb_off), to_np(rb_b.rb_off))
    np.testing.assert_array_equal(to_np(rb_a.rb_pairs)[:P], to_np(rb_b.rb_pairs)[:P])
    return n, P


def test_noalloc_rulebook_equals_workspace_rulebook_on_two_calls():
    sizes = []
    for name, d in (("city256", 4), ("tiny32", 2)):
        cfg = synth.config(name)
        tris, counts = upload_tris([synth.scene_for(cfg)])
        occ = npvs.froxelize(tris, counts, cfg.grids)
        want = npvs.build_rulebook(occ, cfg.grids, d, csr=True)
        # the output buffers are filled with a pattern first, so stale values cannot pass
        got = npvs.build_rulebook(occ, cfg.grids, d, csr=True)
        for t in (got.counts, got.site_keys, got.block_row, got.grid_rows, got.nbr, got.rb_off, got.rb_pairs):
            t.fill_(-7)
        npvs.build_rulebook(occ, cfg.grids, d, csr=True, out=got, noalloc=True)
        torch.cuda.synchronize()
        n, P = _compare(got, want)
        print(f"{name}: {n} sites, {P} pairs equal", flush=True)
        assert n > 0 and P > 0
        sizes.append(n)
    assert sizes[1] < sizes[0]
