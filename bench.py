#!/usr/bin/env python3
"""Benchmark of the NeuralPVS hot path on one MI355X.

Workload: the 256x256x128 froxel grid of a seeded synthetic city (50 000 triangles, about 3 %
occupied froxels), interleave factor d = 4 (64 channels), six submanifold 3x3x3 convolutions
64 -> 64, batch 1.  One step is one frame through the whole path: froxelize -> active sites and
rulebook -> interleave -> 6 convolutions -> de-interleave + threshold -> BCE + repulsive
visibility loss -> hand-written backward (weight gradients on a second stream) -> Adam,
in BF16 on MFMA with FP32 accumulation and FP32 master weights.  Each step is replayed from a
HIP graph captured once; inputs are resident in HBM before the timed region.

Also reported: forward-only and FP32 variants, the step with activation checkpointing, the
per-stage breakdown, the roofline of the
dominant kernel (its launches timed with HIP events on the stream they run on), accuracy of the
BF16 path against the FP32 path and the FP64 oracle, and the CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/sec + ms/frame fwd and fwd+bwd, BF16 vs FP32, 256x256x128 froxel grid"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default tile shape for every layer (for profiler runs, whose "
                         "per-launch overhead skews the autotuner's timings)")
    ap.add_argument("--profile-only", action="store_true", help="run warmup + timed steps only (for rocprofv3)")
    ap.add_argument("--counters", action="store_true",
                    help="for rocprofv3 --pmc: a plain 256 MiB copy (counter calibration), then --steps eager "
                         "(not graph-replayed) BF16 training steps; prints one JSON line and exits")
    return ap.parse_args()


def conv_traffic(variant):
    """HBM bytes per launch of the timed hidden-layer conv in tile shape `variant`, from the counter
    summary under profiles/ (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy of known size);
    None when that summary is missing or was taken on other kernel sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "conv_fwd_bf16_city256_traffic.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    for src in ("conv.hip", "conv_common.hpp", "npvs_common.hpp"):
        h = hashlib.sha256(open(os.path.join(ROOT, "paper_2509_24677_amd", "csrc", src), "rb").read()).hexdigest()
        if f"{src} {h}" not in text:
            return None
    shapes = {0: (1, 9), 1: (2, 1), 2: (1, 3), 3: (2, 3), 4: (1, 1), 5: (2, 9)}
    lds = {6: (1, 4), 7: (1, 2), 8: (2, 2), 9: (1, 8), 10: (2, 4), 11: (2, 8)}
    if variant in shapes:
        name = f"conv_fwd_bf16_kernel<2, 4, {shapes[variant][0]}, {shapes[variant][1]}>"
    elif variant in lds:
        name = f"conv_fwd_bf16_lds_kernel<2, 4, {lds[variant][0]}, {lds[variant][1]}>"
    elif variant == 14:
        name = "conv_fwd_bf16_wsta_kernel<2, 1, 4>"
    elif variant == 15:
        name = "conv_fwd_bf16_wsred_kernel<2>"
    else:
        name = f"conv_fwd_bf16_wsta_kernel<2, {variant - 11}, 2>"
    for line in text.splitlines():
        if line.startswith("## batch16"):  # the first table is the city256 one
            break
        parts = line.rsplit(None, 3)
        if len(parts) == 4 and parts[0] == name:
            return int(parts[3])
    return None


def bench_batch16(args, dev, timed_launches):
    """16 viewcell grids of uneven size (64^3 .. 256x256x128) and occupancy (1-10 %) through the
    BF16 forward as one plan (one concatenated site table and rulebook, autotuned tile shapes, one
    captured graph), against the same 16 grids as 16 single-grid plans replayed one after another.
    Also times one hidden conv launch on the batched rulebook (MFMA roofline at this size)."""
    import numpy as np
    import torch

    import paper_2509_24677_amd as npvs
    import synth

    cfg = synth.config("batch16")
    tri_list = [synth.scene_for(cfg, i) for i in range(len(cfg.grids))]
    layers = synth.net_layers(cfg)
    flat = np.concatenate([t.reshape(-1) for t in tri_list]).astype(np.float32)
    tris = torch.from_numpy(flat).to(dev)
    counts = [len(t) for t in tri_list]

    def plan_for(dims, cnts, tr):
        p = npvs.Plan(dims, cnts, cfg.d, cfg.channels, npvs.NPVS_BF16)
        for li, (W, b) in enumerate(layers):
            p.set_weights(li, torch.from_numpy(W).to(dev), torch.from_numpy(b).to(dev))
        return p, p.autotune(tr, reps=5)

    def time_replays(plans, steps):
        for p in plans:
            p.replay()
        torch.cuda.current_stream().synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            for p in plans:
                p.replay()
        e1.record()
        torch.cuda.current_stream().synchronize()
        return e0.elapsed_time(e1) / steps

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan, tuned = plan_for(cfg.grids, counts, tris)
        plan.capture(tris)
        ms_batched = time_replays([plan], args.steps)
        singles, off = [], 0
        for g, t in zip(cfg.grids, tri_list):
            tr = tris[off:off + t.size]
            off += t.size
            p, _ = plan_for([g], [len(t)], tr)
            p.capture(tr)
            singles.append(p)
        ms_separate = time_replays(singles, args.steps)
    torch.cuda.synchronize()
    c = plan.counts()
    # one hidden layer on the batched rulebook, launch by launch
    occ = npvs.froxelize(tris, counts, cfg.grids)
    rb = npvs.build_rulebook(occ, cfg.grids, cfg.d, csr=True)
    X0 = npvs.gather_input(occ, rb, npvs.NPVS_BF16)
    W1 = npvs.pack_weights(torch.from_numpy(layers[1][0]).to(dev), npvs.NPVS_BF16)
    b1 = torch.from_numpy(layers[1][1]).to(dev)
    W0 = npvs.pack_weights(torch.from_numpy(layers[0][0]).to(dev), npvs.NPVS_BF16)
    H = npvs.sparse_conv_fwd(X0, W0, torch.from_numpy(layers[0][1]).to(dev), 64, 64, rb, npvs.NPVS_BF16, True)
    out = torch.empty_like(H)
    var = tuned[1]
    ts = timed_launches(lambda: npvs.sparse_conv_fwd(H, W1, b1, 64, 64, rb, npvs.NPVS_BF16, True, out=out,
                                                     variant=var), 40)
    conv_ms = float(np.mean(ts))
    n_pairs = rb.host_counts()["n_pairs"]
    flops = 2.0 * n_pairs * 64 * 64
    n = len(cfg.grids)
    # balance: the conv's 16-row tiles are cut from the concatenated sites of all grids and dealt
    # to the XCDs in contiguous ranges, then over each XCD's workgroups (the default shape runs
    # 256 workgroups); tiles per workgroup, whatever the grids' sizes
    grid_rows = rb.grid_rows.cpu().numpy().astype(np.int64)
    ntiles = (int(grid_rows[-1]) + 15) // 16
    G = 256
    per = (ntiles + 7) // 8
    per_wg = [sum(1 for j in range(per) if (i // 8) + j * (G // 8) < per and (i % 8) * per + (i // 8) + j * (G // 8)
                  < ntiles) for i in range(G)]
    balance = {"sites_per_grid": np.diff(grid_rows).tolist(), "tiles": ntiles,
               "tiles_per_workgroup_min": min(per_wg), "tiles_per_workgroup_max": max(per_wg),
               "tiles_spanning_two_grids": int(sum(1 for r in grid_rows[1:-1] if r % 16))}
    return {"grids": n, "n_sites": c["n_sites"], "n_pairs": n_pairs, "tile_variants": tuned, "balance": balance,
            "batched_ms": ms_batched, "batched_frames_per_s": 1000.0 * n / ms_batched,
            "separate_ms": ms_separate, "separate_frames_per_s": 1000.0 * n / ms_separate,
            "speedup": ms_separate / ms_batched,
            "conv_fwd_bf16_avg_launch_ms": conv_ms,
            "conv_fwd_bf16_tflops": flops / (conv_ms * 1e-3) / 1e12,
            "conv_fwd_bf16_frac_of_peak": flops / (conv_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS}


def bench_train4(args, dev):
    """The batch-of-four training configuration: one training step (froxelize, rulebook, forward
    with every second layer input recomputed in the backward, loss, backward, Adam) over four
    128^3 grids of seeded boxes (3.5-4.1 % occupied), captured as one graph, in BF16 and FP32.
    Labels are a fixed subset of the occupied froxels (timing does not depend on their values)."""
    import numpy as np
    import torch

    import paper_2509_24677_amd as npvs
    import synth
    from paper_2509_24677_amd.train import Network, Trainer

    cfg = synth.config("train128x4")
    tri_list = [synth.scene_for(cfg, i) for i in range(len(cfg.grids))]
    tris = torch.from_numpy(np.concatenate([t.reshape(-1) for t in tri_list]).astype(np.float32)).to(dev)
    counts = [len(t) for t in tri_list]
    layers = synth.net_layers(cfg)
    occ = npvs.froxelize(tris, counts, cfg.grids)
    lab = occ & torch.from_numpy(synth.label_mask_bits(7, (occ.numel(),))).to(dev)
    rb = npvs.build_rulebook(occ, cfg.grids, cfg.d, csr=True)
    c = rb.host_counts()
    r = {"grids": len(cfg.grids), "grid": list(cfg.grids[0]), "n_sites": c["n_sites"], "n_pairs": c["n_pairs"],
         "checkpoint": "every second layer input recomputed"}
    for dtype, tag, steps in ((npvs.NPVS_BF16, "bf16", args.steps), (npvs.NPVS_F32, "fp32", 5)):
        net = Network(layers, cfg.d, dtype)
        tr = Trainer(net, cfg.grids, counts, checkpoint=True)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(2):
                tr.step(tris, lab)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            tr.step(tris, lab)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        r[f"{tag}_step_ms"], r[f"{tag}_frames_per_s"] = ms, 1000.0 * len(cfg.grids) / ms
        del g
    r["bf16_speedup_vs_fp32"] = r["fp32_step_ms"] / r["bf16_step_ms"]
    return r


def bench_stage_table(args, dev):
    """The city frame at every interleave factor d in {1, 2, 4, 8, 16} (d = 1: no interleave, the
    ablation of Table 2), BF16, with the stages of the paper's speed figure: froxelize, active
    sites + neighbour map (rulebook), interleave (sparse g_d), the six convolutions (CNN), and
    de-interleave + threshold; each stage timed as 20 back-to-back calls in a captured graph, plus
    the whole pass (library plan graph).  Channels: d^3 -> 64 x 5 -> d^3, He-normal weights."""
    import numpy as np
    import torch

    import paper_2509_24677_amd as npvs
    import synth

    def graph_ms(fn, reps=20, loops=10):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(2):
                fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                fn()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(loops):
            g.replay()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / (reps * loops)
        del g
        return ms

    out = {}
    for name in ("city256_d1", "city256_d2", "city256", "city256_d8", "city256_d16"):
        cfg = synth.config(name)
        t = synth.scene_for(cfg)
        layers = synth.net_layers(cfg)
        tris = torch.from_numpy(t).to(dev)
        dims, d = cfg.grids, cfg.d
        occ = npvs.froxelize(tris, [len(t)], dims)
        rb = npvs.build_rulebook(occ, dims, d)
        c = rb.host_counts()
        C = d ** 3
        w0 = (C + 7) // 8 * 8  # BF16 rows of fewer than 8 channels are padded
        X = npvs.gather_input(occ, rb, npvs.NPVS_BF16, width=w0)
        chans = [w0] + [64] * 5 + [w0]
        Wp = [npvs.pack_weights(torch.from_numpy(W).to(dev), npvs.NPVS_BF16) for W, _ in layers]
        bias = [torch.zeros(co, dtype=torch.float32, device=dev) for co in chans[1:]]
        for i, (_, b) in enumerate(layers):
            bias[i][:b.shape[0]] = torch.from_numpy(b).to(dev)
        acts = [X] + [torch.empty((rb.cap, co), dtype=torch.bfloat16 if i < 5 else torch.float32, device=dev)
                      for i, co in enumerate(chans[1:])]

        def cnn():
            for i in range(6):
                npvs.sparse_conv_fwd(acts[i], Wp[i], bias[i], chans[i], chans[i + 1], rb, npvs.NPVS_BF16, relu=i < 5,
                                     out_f32=i == 5, out=acts[i + 1])

        r = {"d": d, "channels": [C] + [64] * 5 + [C], "n_sites": c["n_sites"]}
        r["froxelize_ms"] = graph_ms(lambda: npvs.froxelize(tris, [len(t)], dims, occ=occ))
        rbo = npvs.build_rulebook(occ, dims, d)
        r["rulebook_ms"] = graph_ms(lambda: npvs.build_rulebook(occ, dims, d, out=rbo))
        r["interleave_ms"] = graph_ms(lambda: npvs.gather_input(occ, rb, npvs.NPVS_BF16, out=X, width=w0))
        r["cnn_ms"] = graph_ms(cnn, reps=5 if d == 1 else 20)
        r["deinterleave_ms"] = graph_ms(lambda: npvs.deinterleave_threshold(acts[6], rb, occ))
        plan = npvs.Plan(dims, [len(t)], d, [C] + [64] * 5 + [C], npvs.NPVS_BF16)
        for li, (W, b) in enumerate(layers):
            plan.set_weights(li, torch.from_numpy(W).to(dev), torch.from_numpy(b).to(dev))
        r["n_pairs"] = npvs.build_rulebook(occ, dims, d, csr=True).host_counts()["n_pairs"]
        plan.forward(tris)
        reps = 5 if d == 1 else 20
        s = torch.cuda.Stream()  # a capture needs a stream of its own
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.capture(tris)
            plan.replay()
            s.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                plan.replay()
            e1.record(s)
            e1.synchronize()
        r["forward_ms"] = e0.elapsed_time(e1) / reps
        r["forward_frames_per_s"] = 1000.0 / r["forward_ms"]
        out[f"d{d}"] = r
        del plan, acts, X, rb, rbo
        torch.cuda.empty_cache()
    return out


def bench_dense_interleave(dev):
    """Dense g_d and its inverse on the logits grid of the 256x256x128 frame (33.5 MB of float32):
    mean time per launch from graph replays and the HBM rate of its algorithmic bytes (every
    element read once and written once)."""
    import numpy as np
    import torch

    import paper_2509_24677_amd as npvs

    def graph_ms(fn, reps=20, loops=10):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(2):
                fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                fn()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(loops):
            g.replay()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / (reps * loops)

    dims = (256, 256, 128)
    gen = torch.Generator(device=dev).manual_seed(11)
    res = {}
    for name, dt, ds in (("f32", torch.float32, (1, 2, 4, 8, 16, 32)), ("bf16", torch.bfloat16, (4,)),
                         ("u8", torch.uint8, (4,))):
        if dt == torch.uint8:
            x = torch.randint(0, 256, (dims[2], dims[1], dims[0]), device=dev, dtype=torch.uint8, generator=gen)
        else:
            x = torch.randn((dims[2], dims[1], dims[0]), device=dev, generator=gen).to(dt)
        nbytes = 2 * x.numel() * x.element_size()
        for d in ds:
            y = npvs.interleave(x, d)
            back = npvs.deinterleave(y, dims, d)
            exact = bool(torch.equal(back.reshape(-1), x.reshape(-1)))
            out_y, out_x = torch.empty_like(y), torch.empty_like(back)
            ms_i = graph_ms(lambda: npvs.interleave(x, d, out=out_y))
            ms_d = graph_ms(lambda: npvs.deinterleave(y, dims, d, out=out_x))
            res[f"{name}_d{d}"] = {"bytes": nbytes, "interleave_ms": ms_i, "deinterleave_ms": ms_d,
                                   "interleave_GB_per_s": nbytes / ms_i / 1e6,
                                   "deinterleave_GB_per_s": nbytes / ms_d / 1e6,
                                   "frac_of_hbm_peak": nbytes / min(ms_i, ms_d) / 1e6 / HBM_PEAK_GBS,
                                   "round_trip_exact": exact}
    return res


def bench_wide(args, dev, timed_launches):
    """The city frame at the paper's interleave factors d = 8 and 16: forward (froxelize -> PVS) as a
    library-captured graph in BF16 and FP32, the training step (forward, loss, backward, Adam) as
    a captured graph in BF16 (and FP32 at d = 8), and the wide first and last layers (Cin or Cout
    = d^3 = 512 / 4096) timed launch by launch against the BF16 MFMA peak."""
    import numpy as np
    import torch

    import paper_2509_24677_amd as npvs
    import synth
    from paper_2509_24677_amd.train import Network, Trainer

    def train_ms(cfg, layers, tris, nt, dtype, steps):
        net = Network(layers, cfg.d, dtype)
        tr = Trainer(net, cfg.grids, nt, checkpoint=False)
        occ = npvs.froxelize(tris, nt, cfg.grids)
        lab = occ & torch.from_numpy(synth.label_mask_bits(7, (occ.numel(),))).to(dev)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(2):
                tr.step(tris, lab)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            tr.step(tris, lab)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    res = {}
    for name in ("city256_d8", "city256_d16"):
        cfg = synth.config(name)
        t = synth.scene_for(cfg)
        layers = synth.net_layers(cfg)
        tris = torch.from_numpy(t).to(dev)
        nt = [len(t)]
        r = {"d": cfg.d, "channels": cfg.channels}
        for dtype, tag in ((npvs.NPVS_BF16, "bf16"), (npvs.NPVS_F32, "fp32")):
            plan = npvs.Plan(cfg.grids, nt, cfg.d, cfg.channels, dtype)
            for li, (W, b) in enumerate(layers):
                plan.set_weights(li, torch.from_numpy(W).to(dev), torch.from_numpy(b).to(dev))
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                plan.capture(tris)
                for _ in range(3):
                    plan.replay()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                for _ in range(args.steps):
                    plan.replay()
                e1.record(s)
                s.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            r[f"{tag}_fwd_ms"] = ms
            r[f"{tag}_fwd_frames_per_s"] = 1000.0 / ms
        r["bf16_fwd_speedup_vs_fp32"] = r["fp32_fwd_ms"] / r["bf16_fwd_ms"]
        ms = train_ms(cfg, layers, tris, nt, npvs.NPVS_BF16, args.steps)
        r["bf16_fwd_bwd_ms"], r["bf16_fwd_bwd_frames_per_s"] = ms, 1000.0 / ms
        if cfg.d == 8:  # the FP32 step at d = 16 takes about 0.1 s: left out to keep the run short
            ms = train_ms(cfg, layers, tris, nt, npvs.NPVS_F32, 5)
            r["fp32_fwd_bwd_ms"], r["fp32_fwd_bwd_frames_per_s"] = ms, 1000.0 / ms
            r["bf16_fwd_bwd_speedup_vs_fp32"] = r["fp32_fwd_bwd_ms"] / r["bf16_fwd_bwd_ms"]
        occ = npvs.froxelize(tris, nt, cfg.grids)
        rb = npvs.build_rulebook(occ, cfg.grids, cfg.d, csr=True)
        c = rb.host_counts()
        r["n_sites"], r["n_pairs"] = c["n_sites"], c["n_pairs"]
        C, H = cfg.channels[0], cfg.channels[1]
        X0 = npvs.gather_input(occ, rb, npvs.NPVS_BF16)
        Wf = npvs.pack_weights(torch.from_numpy(layers[0][0]).to(dev), npvs.NPVS_BF16)
        bf = torch.from_numpy(layers[0][1]).to(dev)
        Hd = npvs.sparse_conv_fwd(X0, Wf, bf, C, H, rb, npvs.NPVS_BF16, True)
        Wl = npvs.pack_weights(torch.from_numpy(layers[-1][0]).to(dev), npvs.NPVS_BF16)
        bl = torch.from_numpy(layers[-1][1]).to(dev)
        Lo = torch.empty((rb.cap, C), dtype=torch.float32, device=dev)
        flops = 2.0 * c["n_pairs"] * C * H
        for key, launch in (("first_layer", lambda: npvs.sparse_conv_fwd(X0, Wf, bf, C, H, rb, npvs.NPVS_BF16, True,
                                                                          out=Hd)),
                            ("last_layer", lambda: npvs.sparse_conv_fwd(Hd, Wl, bl, H, C, rb, npvs.NPVS_BF16, False,
                                                                         out_f32=True, out=Lo))):
            ms = float(np.mean(timed_launches(launch, 20)))
            r[key] = {"shape": [C, H] if key == "first_layer" else [H, C], "ms": ms,
                      "tflops": flops / (ms * 1e-3) / 1e12, "frac_of_bf16_peak": flops / (ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS}
        res[name] = r
    return res


def bench_unet(args, dev, timed_launches):
    """The city frame through the two-level U-Net (d = 4; embedding / encoder 64 and decoder 96
    channels): the whole path froxelize -> PVS captured as one graph in BF16 and FP32, the
    training pass (froxelize -> loss -> backward of every stage) as one graph in BF16 and FP32,
    and the strided down and inverse up convolutions timed launch by launch."""
    import numpy as np
    import torch

    import paper_2509_24677_amd as npvs
    import synth
    from paper_2509_24677_amd.unet import UNet, unet_pvs

    cfg = synth.config("city256")
    t = synth.scene_for(cfg)
    params = synth.unet_params(11, cfg.d)
    tris = torch.from_numpy(t).to(dev)
    nt = [len(t)]
    r = {"d": cfg.d, "channels": {"embed": 64, "encoder": 64, "decoder": 96}}
    for dtype, tag in ((npvs.NPVS_BF16, "bf16"), (npvs.NPVS_F32, "fp32")):
        net = UNet(params, cfg.d, dtype)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(3):
                unet_pvs(net, tris, nt, cfg.grids)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            unet_pvs(net, tris, nt, cfg.grids)
        torch.cuda.synchronize()
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            g.replay()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        r[f"{tag}_fwd_ms"] = ms
        r[f"{tag}_fwd_frames_per_s"] = 1000.0 / ms
        del g
    r["bf16_fwd_speedup_vs_fp32"] = r["fp32_fwd_ms"] / r["bf16_fwd_ms"]
    # forward + loss + backward (every stage's weight and bias gradient), captured as one graph;
    # labels: a fixed subset of the occupied froxels (timing does not depend on their values)
    lab = npvs.froxelize(tris, nt, cfg.grids)
    lab &= torch.from_numpy(synth.label_mask_bits(7, (lab.numel(),))).to(dev)
    for dtype, tag, steps in ((npvs.NPVS_BF16, "bf16", args.steps), (npvs.NPVS_F32, "fp32", 5)):
        net = UNet(params, cfg.d, dtype)

        def train_pass():
            occ_ = npvs.froxelize(tris, nt, cfg.grids)
            lv_ = npvs.build_levels(occ_, cfg.grids, cfg.d, csr=True)
            saved = {}
            logits = net.forward(npvs.gather_input(occ_, lv_.rb0, dtype), lv_, saved=saved)
            _, dl = npvs.loss(logits, npvs.gather_input(lab, lv_.rb0, npvs.NPVS_U8), lv_.rb0)
            return net.backward(saved, logits, dl, lv_)

        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(2):
                train_pass()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            train_pass()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        r[f"{tag}_fwd_bwd_ms"], r[f"{tag}_fwd_bwd_frames_per_s"] = ms, 1000.0 / ms
        del g
    r["bf16_fwd_bwd_speedup_vs_fp32"] = r["fp32_fwd_bwd_ms"] / r["bf16_fwd_bwd_ms"]
    occ = npvs.froxelize(tris, nt, cfg.grids)
    lv = npvs.build_levels(occ, cfg.grids, cfg.d, csr=True)
    c0, c1 = lv.rb0.host_counts(), lv.rb1.host_counts()
    r.update(n_sites_level0=c0["n_sites"], n_sites_level1=c1["n_sites"], n_pairs_level0=c0["n_pairs"],
             n_pairs_level1=c1["n_pairs"])
    n0 = c0["n_sites"]
    X0 = torch.randn((lv.rb0.cap, 64), device=dev).to(torch.bfloat16)
    (Wd, bd), = params["down"]
    (Wu, bu), = params["up"]
    Wdp = npvs.pack_weights_k(torch.from_numpy(Wd).to(dev), npvs.NPVS_BF16)
    Wup = npvs.pack_weights_k(torch.from_numpy(Wu).to(dev), npvs.NPVS_BF16)
    bdt, but = torch.from_numpy(bd).to(dev), torch.from_numpy(bu).to(dev)
    H1 = npvs.strided_conv_fwd(X0, Wdp, bdt, 64, 64, lv, False, npvs.NPVS_BF16)
    U = npvs.strided_conv_fwd(H1, Wup, but, 64, 96, lv, True, npvs.NPVS_BF16)
    for key, cin, cout, launch in (
            ("down_layer", 64, 64, lambda: npvs.strided_conv_fwd(X0, Wdp, bdt, 64, 64, lv, False, npvs.NPVS_BF16, out=H1)),
            ("up_layer", 64, 96, lambda: npvs.strided_conv_fwd(H1, Wup, but, 64, 96, lv, True, npvs.NPVS_BF16, out=U))):
        ms = float(np.mean(timed_launches(launch, 20)))
        flops = 2.0 * n0 * cin * cout  # every level-0 site enters exactly one product
        r[key] = {"shape": [cin, cout], "ms": ms, "tflops": flops / (ms * 1e-3) / 1e12,
                  "frac_of_bf16_peak": flops / (ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS}
    return r


def bench_world(args, dev, timed_launches):
    """The city frame in world space: froxelization into the viewcell frustum of the paper's camera
    (60 degree field of view widened by 2 x 15 degrees, near 0.3, far 1000, 256^3 froxels, linear
    depth slices), timed launch by launch, and the whole pass world triangles -> PVS through the
    BF16 network of the benchmark (d = 4, six 64-channel layers) captured as one graph."""
    import math

    import numpy as np
    import torch

    import paper_2509_24677_amd as npvs
    import synth
    from paper_2509_24677_amd.train import Network

    cfg = synth.config("city256")
    t = synth.scene_for(cfg)
    tris = torch.from_numpy(t).to(dev)
    view = npvs.viewcell_frustum([128.0, 40.0, -20.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0], math.pi / 3, 1.0, 0.6,
                                 math.pi / 12, 0.3, 1000.0)
    dims = (256, 256, 256)
    occ = npvs.froxelize_view(tris, view, dims)
    r = {"grid": list(dims), "scene_triangles": len(t),
         "occupied": int(np.unpackbits(occ.cpu().numpy()).sum())}
    r["froxelize_ms"] = float(np.median(timed_launches(lambda: npvs.froxelize_view(tris, view, dims), 20)))
    net = Network(synth.net_layers(cfg), cfg.d, npvs.NPVS_BF16)

    def frame():
        o = npvs.froxelize_view(tris, view, dims)
        rb = npvs.build_rulebook(o, [dims], cfg.d)
        logits, _ = net.forward(npvs.gather_input(o, rb, npvs.NPVS_BF16), rb)
        return npvs.deinterleave_threshold(logits, rb, o)[0]

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(3):
            frame()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        frame()
    torch.cuda.synchronize()
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    rb = npvs.build_rulebook(occ, [dims], cfg.d)
    r.update(bf16_fwd_ms=ms, bf16_fwd_frames_per_s=1000.0 / ms, n_sites=rb.host_counts()["n_sites"])
    return r


def bench_cull(args, dev, timed_launches, tris, n_tris, dims, pvs):
    """Culling against the city's BF16 PVS: every scene triangle (npvs_visible_triangles), and 2048
    box-shaped temporal bounding volumes of 10 triangles each as objects (npvs_visible_objects)."""
    import numpy as np
    import torch

    import paper_2509_24677_amd as npvs
    import synth

    vis = npvs.visible_triangles(tris, n_tris, dims, pvs)
    ms_t = float(np.median(timed_launches(lambda: npvs.visible_triangles(tris, n_tris, dims, pvs), 20)))
    boxes = synth.box_scene(77, dims[0], 2048, 4, 24)
    tb = torch.from_numpy(boxes).to(dev)
    off = torch.arange(0, len(boxes) + 1, 10, dtype=torch.int64, device=dev)

    def tbv():
        v = npvs.visible_triangles(tb, [len(boxes)], dims, pvs)
        return npvs.visible_objects(v, off)
    kept = tbv()
    ms_o = float(np.median(timed_launches(lambda: (tbv(),), 20)))  # two launches per call
    return {"scene_triangles": int(sum(n_tris)), "kept_triangles": int(vis.sum().item()),
            "triangles_ms": ms_t, "triangles_per_s": sum(n_tris) / (ms_t * 1e-3),
            "tbv_objects": 2048, "kept_objects": int(kept.sum().item()), "tbv_ms": ms_o,
            "objects_per_s": 2048 / (ms_o * 1e-3)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_frame(job):
    """One full frame of the FP64 oracle (forward, loss, backward); returns its wall time."""
    import numpy as np

    import oracle
    import synth
    tris_np, dims, d, layers, total_bytes = job
    t0 = time.perf_counter()
    out = oracle.forward(tris_np, dims, d, layers)
    lab_np = out["occ"] & synth.label_mask_bits(7, (total_bytes,)).reshape(out["occ"].shape)
    site_lab = oracle.site_labels(lab_np, dims, d, out["keys"])
    dl = oracle.loss(out["acts"][-1], site_lab)["grad"]
    oracle.backward(out, layers, dl)
    return time.perf_counter() - t0, out


def _trained_layers(dev, steps=300):
    """The city network (d = 4, six 64-channel layers, He init) after `steps` BF16 training steps
    on the four 128^3 grids with their ray-march labels (the oracle's labeller, stored by
    tests/golden/make_train_labels.py), Adam at the paper's learning rate."""
    import numpy as np
    import torch

    import paper_2509_24677_amd as npvs
    import synth
    from paper_2509_24677_amd.train import Network, Trainer

    cfg = synth.config("train128x4")
    tri_list = [synth.scene_for(cfg, i) for i in range(len(cfg.grids))]
    tris = torch.from_numpy(np.concatenate([t.reshape(-1) for t in tri_list]).astype(np.float32)).to(dev)
    counts = [len(t) for t in tri_list]
    gold = np.load(os.path.join(ROOT, "tests", "golden", "train128x4_labels.npz"))
    lab = torch.from_numpy(np.concatenate([gold[f"labels{i}"].reshape(-1) for i in range(len(cfg.grids))])).to(dev)
    net = Network(synth.net_layers(synth.config("city256")), cfg.d, npvs.NPVS_BF16)
    tr = Trainer(net, cfg.grids, counts, checkpoint=True)
    tr_first, _ = tr.step(tris, lab)
    tr_first = tr_first.clone()
    stats = tr_first
    for _ in range(steps - 1):
        stats, _ = tr.step(tris, lab)
    torch.cuda.synchronize()
    layers = [(W.detach().cpu().numpy(), b.detach().cpu().numpy()) for W, b in zip(net.W, net.b)]
    first = float(tr_first[-1, 0].item())
    return layers, (first, float(stats[-1, 0].item())), (cfg, tri_list, tris, counts)


def cpu_baseline_and_accuracy(args, dev, cfg, tris_np, dims, layers, occ_np, pvs_b, pvs_f, logits_b, logits_f,
                              n_sites, total_bytes):
    """The CPU oracle baseline (one frame single-threaded, then one frame per host core in
    parallel processes; the oracle itself is single-threaded) and the accuracy of the BF16 path:
    flips, missing geometry and FPR against the FP64 oracle and the FP32 path (oracle.metrics),
    with the He-initialised weights and after 300 BF16 training steps."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    import paper_2509_24677_amd as npvs
    from paper_2509_24677_amd.train import Network
    oracle.build(force=False)
    acc = {}
    cpu_s, out = _oracle_frame((tris_np, dims[0], cfg.d, layers, total_bytes))
    try:
        n_cores = len(os.sched_getaffinity(0))
    except AttributeError:
        n_cores = os.cpu_count() or 1
    n_cores = max(1, min(n_cores, 16))
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(n_cores) as ex:
        list(ex.map(_oracle_frame_time, [(tris_np, dims[0], cfg.d, layers, total_bytes)] * n_cores))
    wall = time.perf_counter() - t0
    cpu = {"value": n_cores / wall, "unit": "frames/s", "cores": n_cores, "kind": "oracle",
           "cpu_model": _cpu_model(), "single_thread_value": 1.0 / cpu_s,
           "sample": f"the 256x256x128 city frame (froxelize, sites, rulebook, interleave, 6 conv layers, "
                     f"de-interleave + threshold, loss and backward) in the FP64 C oracle: {n_cores} frames in "
                     f"{n_cores} processes in {wall:.2f} s; one frame single-threaded {cpu_s:.2f} s"}
    ref = out["acts"][-1]
    lf = logits_f[:n_sites].cpu().numpy()
    lb = logits_b[:n_sites].cpu().numpy()
    acc["max_abs_logit_err_fp32_vs_fp64_oracle"] = float(np.abs(lf - ref).max())
    acc["max_abs_logit_err_bf16_vs_fp64_oracle"] = float(np.abs(lb - ref).max())
    pf_bits = pvs_f.cpu().numpy()
    acc["pvs_bits_fp32_equal_oracle_outside_1e-5_band"] = bool(
        ((np.unpackbits(out["pvs"].reshape(-1), bitorder="little") == np.unpackbits(pf_bits, bitorder="little")) |
         (np.abs(np.nan_to_num(out["logits"].reshape(-1), neginf=-1e9)) <= 1e-5)).all())
    occ = out["occ"].reshape(-1)
    active = oracle.active_froxels(out["occ"], dims[0], cfg.d).reshape(-1)
    keep = ("flips", "flip_rate_active", "flip_rate_occupied", "flip_rate_all", "missing_geometry", "fpr")
    m = oracle.metrics(out["pvs"].reshape(-1), pvs_b.cpu().numpy(), occ, active)
    acc["bf16_vs_fp64_oracle"] = {k: m[k] for k in keep}
    m = oracle.metrics(pf_bits, pvs_b.cpu().numpy(), occ, active)
    acc["bf16_vs_fp32_path"] = {k: m[k] for k in keep}
    acc["flip_target"] = ("at most 0.1 % of thresholded froxels: flip_rate_active (froxels of active blocks, "
                          "the ones that receive a logit and are thresholded); flip_rate_occupied beside it")
    # after training: the same comparisons with the trained weights, on the city frame and on
    # the four training grids
    trained, final_loss, (tcfg, tri_list, ttris, tcounts) = _trained_layers(dev)
    tr_acc = {"training": "300 BF16 steps (Adam, lr 1e-3) on the four 128^3 grids with ray-march labels",
              "loss_first_step": final_loss[0], "loss_last_step": final_loss[1]}
    import torch
    nets = {dt: Network(trained, cfg.d, dt) for dt in (npvs.NPVS_BF16, npvs.NPVS_F32)}
    for name, (t_np, g) in [("city256", (tris_np, dims[0]))] + [(f"train{i}", (tri_list[i], tcfg.grids[i]))
                                                                 for i in range(len(tri_list))]:
        tt = torch.from_numpy(np.asarray(t_np, np.float32)).to(dev)
        occ_d = npvs.froxelize(tt, [len(t_np)], [g])
        rb = npvs.build_rulebook(occ_d, [g], cfg.d)
        pv = {}
        for dt, net in nets.items():
            lg, _ = net.forward(npvs.gather_input(occ_d, rb, dt), rb)
            pv[dt], _ = npvs.deinterleave_threshold(lg, rb, occ_d)
        o = oracle.forward(t_np, g, cfg.d, trained, want_logits=False)
        act_m = oracle.active_froxels(o["occ"], g, cfg.d).reshape(-1)
        ma = oracle.metrics(o["pvs"].reshape(-1), pv[npvs.NPVS_BF16].cpu().numpy(), o["occ"].reshape(-1), act_m)
        mf = oracle.metrics(pv[npvs.NPVS_F32].cpu().numpy(), pv[npvs.NPVS_BF16].cpu().numpy(), o["occ"].reshape(-1),
                            act_m)
        tr_acc[name] = {"bf16_vs_fp64_oracle": {k: ma[k] for k in keep}, "bf16_vs_fp32_path": {k: mf[k] for k in keep}}
    acc["after_training"] = tr_acc
    return cpu, acc


def _oracle_frame_time(job):
    return _oracle_frame(job)[0]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(grids are independent frames; see the sharding note in the design document)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2509_24677_amd as npvs
    import synth
    from paper_2509_24677_amd.train import Network, Trainer

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    cfg = synth.config("city256")
    dims = cfg.grids
    tris_np = synth.scene_for(cfg)
    layers = synth.net_layers(cfg)
    tris = torch.from_numpy(tris_np).to(dev)
    n_tris = [len(tris_np)]
    total_bytes = dims[0][0] * dims[0][1] * dims[0][2] // 8
    occ_np = None

    # label subset of G for the training step (timing does not depend on label values)
    def label_bits_for(occ):
        mask = torch.from_numpy(synth.label_mask_bits(7, (total_bytes,))).to(dev)
        return occ & mask

    torch.cuda.synchronize()
    occ0 = npvs.froxelize(tris, n_tris, dims)
    labels = label_bits_for(occ0)
    rb0 = npvs.build_rulebook(occ0, dims, cfg.d, csr=True)
    counts = rb0.host_counts()
    n_sites, n_pairs = counts["n_sites"], counts["n_pairs"]
    occ_np = occ0.cpu().numpy()
    occupied = int(np.unpackbits(occ_np).sum())
    print(f"# workload: T={n_tris[0]} occupied={occupied} ({occupied / (8 * total_bytes):.4f}) "
          f"sites={n_sites} pairs={n_pairs}", file=sys.stderr, flush=True)

    # ------------------------------------------------------------------ step functions
    X0_b = npvs.gather_input(occ0, rb0, npvs.NPVS_BF16)
    tuned = {}

    def make(dtype, checkpoint=False):
        net = Network(layers, cfg.d, dtype)
        if dtype == npvs.NPVS_BF16:  # autotuned tile shapes, chosen once on the real rulebook
            if "v" not in tuned:
                tuned["v"] = ([npvs._lib.NPVS_DEFAULT_CONV_VARIANT] * net.n_layers if args.no_autotune
                              else net.autotune(X0_b, rb0))
            net.variant = list(tuned["v"])
        tr = Trainer(net, dims, n_tris, checkpoint=checkpoint)
        return net, tr

    def fwd_fn(net):
        def f():
            occ = npvs.froxelize(tris, n_tris, dims)
            rb = npvs.build_rulebook(occ, dims, cfg.d)
            X0 = npvs.gather_input(occ, rb, net.dtype)
            logits, _ = net.forward(X0, rb)
            pvs, _ = npvs.deinterleave_threshold(logits, rb, occ)
            return pvs, logits
        return f

    def infer_fn(net, occ):
        """Inference from a froxelized grid: sites and rulebook, interleave, convolutions,
        de-interleave + threshold (everything after froxelization)."""
        def f():
            rb = npvs.build_rulebook(occ, dims, cfg.d)
            X0 = npvs.gather_input(occ, rb, net.dtype)
            logits, _ = net.forward(X0, rb)
            pvs, _ = npvs.deinterleave_threshold(logits, rb, occ)
            return pvs, logits
        return f

    def train_fn(tr):
        return lambda: tr.step(tris, labels)

    def capture(fn, warm):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warm):
                fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            out = fn()
        torch.cuda.synchronize()
        return g, out

    def time_graph(g, steps, per_step=None):
        """Mean ms per replay over `steps` back-to-back replays (one event pair around all of
        them); with `per_step` (a dict), also the median / p10 / p90 of per-replay event pairs
        from a second run of the same length."""
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if per_step is not None:
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
            evs[0].record()
            for i in range(steps):
                g.replay()
                evs[i + 1].record()
            torch.cuda.synchronize()
            d = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
            per_step.update(median_ms=float(np.median(d)), p10_ms=float(np.percentile(d, 10)),
                            p90_ms=float(np.percentile(d, 90)))
        return e0.elapsed_time(e1) / steps, wall

    net_b, tr_b = make(npvs.NPVS_BF16)
    if args.counters:
        # calibration: an elementwise kernel that reads and writes exactly 256 MiB each
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        step = train_fn(tr_b)
        for _ in range(args.steps):
            step()
        # last: 10 launches of the timed hidden layer in each tile shape (the kernel whose roofline
        # the benchmark line reports is one of them)
        rbc = npvs.build_rulebook(occ0, dims, cfg.d, csr=True)
        hid = net_b.layer(0, npvs.gather_input(occ0, rbc, npvs.NPVS_BF16), rbc)
        out = torch.empty_like(hid)
        for v in range(npvs.NPVS_CONV_VARIANTS):
            for _ in range(10):
                npvs.sparse_conv_fwd(hid, net_b.Wp[1], net_b.b[1], 64, 64, rbc, npvs.NPVS_BF16, True, out=out, variant=v)
        # then (after a marker copy) the same layer on the batch of 16 grids, 5 launches per shape
        torch.mul(a[:1024], 1.0, out=b[:1024])  # marker
        c16 = synth.config("batch16")
        t16 = [synth.scene_for(c16, i) for i in range(len(c16.grids))]
        tr16 = torch.from_numpy(np.concatenate([x.reshape(-1) for x in t16]).astype(np.float32)).to(dev)
        occ16 = npvs.froxelize(tr16, [len(x) for x in t16], c16.grids)
        rb16 = npvs.build_rulebook(occ16, c16.grids, c16.d)
        h16 = net_b.layer(0, npvs.gather_input(occ16, rb16, npvs.NPVS_BF16), rb16)
        o16 = torch.empty_like(h16)
        for v in (14, 15, 9, 12, 3, 0):
            for _ in range(5):
                npvs.sparse_conv_fwd(h16, net_b.Wp[1], net_b.b[1], 64, 64, rb16, npvs.NPVS_BF16, True, out=o16,
                                     variant=v)
        torch.cuda.synchronize()
        print(json.dumps({"counters": True, "steps": args.steps, "calibration_bytes_each_way": a.numel() * 4}))
        return
    g_train_b, _ = capture(train_fn(tr_b), max(args.warmup, 2))
    print("# captured bf16 training step", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        g_train_b.replay()
    torch.cuda.synchronize()
    # ------------------------------------------------------------------ timed region (primary)
    step_dist = {}
    ms_step, wall = time_graph(g_train_b, args.steps, step_dist)
    print(f"# bf16 fwd+bwd: {ms_step:.4f} ms/frame over {args.steps} steps (wall {wall:.3f} s)",
          file=sys.stderr, flush=True)
    if args.profile_only:
        print(json.dumps({"profile_only": True, "ms_per_step": ms_step}))
        return

    # ------------------------------------------------------------------ variants
    variants = {"bf16_fwd_bwd": {"ms_per_frame": ms_step, "frames_per_s": 1000.0 / ms_step, **step_dist}}

    def variant(name, g):
        dist = {}
        ms, _ = time_graph(g, args.steps, dist)
        variants[name] = {"ms_per_frame": ms, "frames_per_s": 1000.0 / ms, **dist}

    # end to end (froxelize -> PVS) and inference only (after froxelization), BF16 and FP32
    net_bf, _ = make(npvs.NPVS_BF16)
    g_fb, (pvs_b, logits_b) = capture(fwd_fn(net_bf), 2)
    variant("bf16_fwd", g_fb)
    g_ib, _ = capture(infer_fn(net_bf, occ0), 2)
    variant("bf16_infer", g_ib)
    net_ff, _ = make(npvs.NPVS_F32)
    g_ff, (pvs_f, logits_f) = capture(fwd_fn(net_ff), 2)
    variant("fp32_fwd", g_ff)
    g_if, _ = capture(infer_fn(net_ff, occ0), 2)
    variant("fp32_infer", g_if)
    net_f, tr_f = make(npvs.NPVS_F32)
    g_train_f, _ = capture(train_fn(tr_f), 2)
    variant("fp32_fwd_bwd", g_train_f)
    # the same BF16 step with activation checkpointing (every second layer input recomputed)
    _, tr_c = make(npvs.NPVS_BF16, checkpoint=True)
    g_train_c, _ = capture(train_fn(tr_c), 2)
    variant("bf16_fwd_bwd_checkpointed", g_train_c)
    # the whole forward as one library-captured graph (npvs_plan_capture / npvs_plan_replay)
    plan = npvs.Plan(dims, n_tris, cfg.d, cfg.channels, npvs.NPVS_BF16)
    for li, (W, b) in enumerate(layers):
        plan.set_weights(li, torch.from_numpy(W).to(dev), torch.from_numpy(b).to(dev))
    ps = torch.cuda.Stream()
    with torch.cuda.stream(ps):
        plan.capture(tris)
        for _ in range(3):
            plan.replay()
        ps.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ps)
        for _ in range(args.steps):
            plan.replay()
        e1.record(ps)
        ps.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    variants["bf16_fwd_plan_graph"] = {"ms_per_frame": ms, "frames_per_s": 1000.0 / ms}
    variants["bf16_fwd_speedup_vs_fp32_fwd"] = variants["fp32_fwd"]["ms_per_frame"] / variants["bf16_fwd"]["ms_per_frame"]
    variants["bf16_infer_speedup_vs_fp32_infer"] = (variants["fp32_infer"]["ms_per_frame"] /
                                                   variants["bf16_infer"]["ms_per_frame"])
    print("# variants " + json.dumps(variants), file=sys.stderr, flush=True)

    # ------------------------------------------------------------------ device memory per frame
    # Transient: the largest amount of torch-allocated memory one eager frame holds on top of what
    # was allocated before it (activations, rulebook, workspaces; freed when the frame ends).
    # Persistent: what a network with its Adam state and its autotuned shapes keeps between
    # frames.  The library plan allocates through HIP directly, so its footprint is the drop in
    # free device memory over its creation and capture.
    def transient_mb(fn):
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        fn()
        torch.cuda.synchronize()
        return (torch.cuda.max_memory_allocated() - base) / 2 ** 20

    base = torch.cuda.memory_allocated()
    net_m, tr_m = make(npvs.NPVS_BF16)
    tr_m.step(tris, labels)
    torch.cuda.synchronize()
    persistent = (torch.cuda.memory_allocated() - base) / 2 ** 20
    memory = {"bf16_fwd_bwd_transient_MiB": transient_mb(train_fn(tr_m)),
              "bf16_fwd_bwd_persistent_MiB": persistent,
              "bf16_fwd_bwd_checkpointed_transient_MiB": transient_mb(train_fn(tr_c)),
              "bf16_fwd_transient_MiB": transient_mb(fwd_fn(net_bf)),
              "fp32_fwd_bwd_transient_MiB": transient_mb(train_fn(tr_f))}
    del net_m, tr_m
    torch.cuda.synchronize()
    pvs_m = torch.empty(total_bytes, dtype=torch.uint8, device=dev)
    wts_m = [(torch.from_numpy(W).to(dev), torch.from_numpy(b).to(dev)) for W, b in layers]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    plan_m = npvs.Plan(dims, n_tris, cfg.d, cfg.channels, npvs.NPVS_BF16)
    for li, (W, b) in enumerate(wts_m):
        plan_m.set_weights(li, W, b)
    with torch.cuda.stream(ps):
        plan_m.capture(tris, pvs=pvs_m)
        ps.synchronize()
    memory["bf16_fwd_plan_MiB"] = (free0 - torch.cuda.mem_get_info()[0]) / 2 ** 20
    del plan_m
    print("# device memory " + json.dumps(memory), file=sys.stderr, flush=True)

    # ------------------------------------------------------------------ per-launch kernel timing
    # A GPU-side spin first lets the host enqueue the instrumented launches ahead of the GPU, so
    # each event pair brackets exactly one kernel on the stream it runs on.
    def timed_launches(launch, reps):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        torch.cuda.synchronize()
        torch.cuda._sleep(50_000_000)
        for a, b in evs:
            a.record()
            launch()
            b.record()
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs]

    def streamed_launches(launch, reps):
        """Mean ms per launch of `reps` launches back to back between one pair of events on the
        launching stream: the GPU runs them one after another, with no event inside the region."""
        for _ in range(3):
            launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            launch()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    occ = npvs.froxelize(tris, n_tris, dims)
    rb = npvs.build_rulebook(occ, dims, cfg.d, csr=True)
    Xb = npvs.gather_input(occ, rb, npvs.NPVS_BF16)
    hid_b = net_b.layer(0, Xb, rb)
    out_b = torch.empty_like(hid_b)
    Xf = npvs.gather_input(occ, rb, npvs.NPVS_F32)
    hid_f = net_f.layer(0, Xf, rb)
    out_f = torch.empty_like(hid_f)
    reps = 60
    stage = {}
    stage["froxelize"] = timed_launches(lambda: npvs.froxelize(tris, n_tris, dims, occ=occ), 20)
    stage["rulebook"] = timed_launches(lambda: npvs.build_rulebook(occ, dims, cfg.d, csr=True), 20)
    stage["gather_bf16"] = timed_launches(lambda: npvs.gather_input(occ, rb, npvs.NPVS_BF16, out=Xb), 20)
    stage["conv_fwd_bf16"] = timed_launches(
        lambda: npvs.sparse_conv_fwd(hid_b, net_b.Wp[1], net_b.b[1], 64, 64, rb, npvs.NPVS_BF16, True, out=out_b,
                                     variant=net_b.variant[1]), reps)
    stage["conv_fwd_fp32"] = timed_launches(
        lambda: npvs.sparse_conv_fwd(hid_f, net_f.Wp[1], net_f.b[1], 64, 64, rb, npvs.NPVS_F32, True, out=out_f), reps)
    dY = torch.randn((rb.cap, 64), device=dev)
    stage["conv_bwd_bf16"] = timed_launches(
        lambda: npvs.sparse_conv_bwd(hid_b, net_b.Wt[1], 64, 64, out_b, dY, rb, npvs.NPVS_BF16, True), 20)
    # the training step's form: each layer's dZ and data gradient, then the weight gradients of
    # all six layers in one launch (here six copies of the hidden layer's operands)
    ws_b = npvs.conv_bwd_workspace(64, 64, rb, npvs.NPVS_BF16)
    stage["conv_bwd_bf16_without_wgrad"] = timed_launches(
        lambda: npvs.sparse_conv_bwd(hid_b, net_b.Wt[1], 64, 64, out_b, dY, rb, npvs.NPVS_BF16, True, ws=ws_b,
                                     want_dw=False), 20)
    # the chained form's data gradient: dZ of the hidden layer -> the layer below's dZ and bias
    # partials, its ReLU' fused in
    ws_b2 = npvs.conv_bwd_workspace(64, 64, rb, npvs.NPVS_BF16)
    stage["dgrad_relu_bf16"] = timed_launches(
        lambda: npvs.sparse_conv_dgrad_relu(net_b.Wt[1], 64, 64, hid_b, 64, rb, ws_b, ws_b2), 20)
    wg_ws = [npvs.conv_bwd_workspace(64, 64, rb, npvs.NPVS_BF16) for _ in range(6)]
    for w in wg_ws:
        npvs.sparse_conv_bwd(hid_b, net_b.Wt[1], 64, 64, out_b, dY, rb, npvs.NPVS_BF16, True, ws=w, want_dw=False)
    wg_out = [(torch.empty((27, 64, 64), device=dev), torch.empty(64, device=dev)) for _ in range(6)]
    wg_layers = [(hid_b, 64, 64, w, gW, gb) for w, (gW, gb) in zip(wg_ws, wg_out)]
    stage["wgrad_bf16_six_layers_batched"] = timed_launches(
        lambda: npvs.sparse_conv_wgrad(wg_layers, rb, npvs.NPVS_BF16), 20)
    stage["deinterleave_threshold"] = timed_launches(lambda: npvs.deinterleave_threshold(logits_b, rb, occ), 20)
    stage_ms = {k: float(np.median(v)) for k, v in stage.items()}
    # algorithmic bytes of the memory-bound stages and the HBM rate they reach (peak 8 TB/s)
    N = dims[0][0] * dims[0][1] * dims[0][2]
    nblocks = N // cfg.d ** 3
    stage_bytes = {
        "froxelize": 36 * n_tris[0] + N // 8,                        # triangles in, bits out
        "rulebook": N // 8 + 4 * nblocks + 4 * n_sites + 27 * 4 * n_sites + 8 * n_pairs,
        "gather_bf16": N // 8 + n_sites * 64 * 2,                  # bits in, rows out
        "deinterleave_threshold": n_sites * 64 * 4 + 2 * (N // 8),  # logits and G in, PVS out
    }
    stage_gbs = {k: {"bytes": b, "GB_per_s": b / (stage_ms[k] * 1e-3) / 1e9,
                     "frac_of_hbm_peak": b / (stage_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                 for k, b in stage_bytes.items()}
    # froxelize's integer work: one separating-axis test per froxel of each triangle's clipped
    # range (vertices in 1/256-froxel fixed point, rounded to nearest even; closed froxels, so a
    # coordinate on a froxel face also meets the froxel below)
    q = np.rint(tris_np.astype(np.float64).reshape(-1, 3, 3) * 256.0).astype(np.int64)
    ext = np.array([dims[0][0], dims[0][1], dims[0][2]])
    lo = np.maximum((q.min(axis=1) - 1) >> 8, 0)
    hi = np.minimum(q.max(axis=1) >> 8, ext - 1)
    sat_tests = int(np.prod(np.maximum(hi - lo + 1, 0), axis=1).sum())
    stage_gbs["froxelize"].update(sat_tests=sat_tests, sat_tests_per_s=sat_tests / (stage_ms["froxelize"] * 1e-3))
    print("# stages (median ms per call) " + json.dumps(stage_ms), file=sys.stderr, flush=True)

    # dominant kernel: the BF16 MFMA gather-GEMM (6 forward and 5 data-gradient launches per
    # frame); its average launch duration from 200 launches back to back (the isolated,
    # event-bracketed launch of the stage table also counts the events' own overhead)
    conv_bf16 = lambda: npvs.sparse_conv_fwd(hid_b, net_b.Wp[1], net_b.b[1], 64, 64, rb, npvs.NPVS_BF16, True,
                                            out=out_b, variant=net_b.variant[1])
    conv_ms = streamed_launches(conv_bf16, 200)
    flops = 2.0 * n_pairs * 64 * 64
    achieved = flops / (conv_ms * 1e-3) / 1e12
    shapes = {0: "<2,4,1,9>", 1: "<2,4,2,1>", 2: "<2,4,1,3>", 3: "<2,4,2,3>", 4: "<2,4,1,1>", 5: "<2,4,2,9>",
              6: "_lds<2,4,1,4>", 7: "_lds<2,4,1,2>", 8: "_lds<2,4,2,2>", 9: "_lds<2,4,1,8>",
              10: "_lds<2,4,2,4>", 11: "_lds<2,4,2,8>", 12: "_wsta<2,1>", 13: "_wsta<2,2>", 14: "_wsta<2,1,4>",
              15: "_wsred<2>"}
    alg_bytes = n_sites * 64 * 2 * 2 + 27 * n_sites * 4 + 27 * 64 * 64 * 2  # X in, Y out, neighbour map, weights
    roofline = {"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / BF16_PEAK_TFLOPS, "traffic": conv_traffic(net_b.variant[1]),
                "algorithmic_bytes_per_launch": alg_bytes,
                "kernel": "conv_fwd_bf16" + shapes[net_b.variant[1]], "avg_launch_ms": conv_ms,
                "isolated_launch_ms": float(np.mean(stage["conv_fwd_bf16"])),
                "algorithmic_flops_per_launch": flops, "autotuned_variants": net_b.variant}
    conv32_ms = streamed_launches(
        lambda: npvs.sparse_conv_fwd(hid_f, net_f.Wp[1], net_f.b[1], 64, 64, rb, npvs.NPVS_F32, True, out=out_f), 50)
    roofline_fp32 = {"achieved": flops / (conv32_ms * 1e-3) / 1e12, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "avg_launch_ms": conv32_ms}
    roofline_fp32["frac"] = roofline_fp32["achieved"] / FP32_PEAK_TFLOPS

    # ------------------------------------------------------------------ batching (16 uneven grids)
    batch16 = bench_batch16(args, dev, timed_launches)
    print("# batch16 " + json.dumps(batch16), file=sys.stderr, flush=True)
    train4 = bench_train4(args, dev)
    print("# batch of four 128^3 grids, training " + json.dumps(train4), file=sys.stderr, flush=True)
    wide = bench_wide(args, dev, timed_launches)
    print("# interleave factors 8 and 16 " + json.dumps(wide), file=sys.stderr, flush=True)
    dense = bench_dense_interleave(dev)
    print("# dense interleave " + json.dumps(dense), file=sys.stderr, flush=True)
    stage_table = bench_stage_table(args, dev)
    print("# stages by interleave factor " + json.dumps(stage_table), file=sys.stderr, flush=True)
    cull = bench_cull(args, dev, timed_launches, tris, n_tris, dims, pvs_b)
    print("# culling " + json.dumps(cull), file=sys.stderr, flush=True)
    unet = bench_unet(args, dev, timed_launches)
    print("# two-level U-Net " + json.dumps(unet), file=sys.stderr, flush=True)
    world = bench_world(args, dev, timed_launches)
    print("# world space " + json.dumps(world), file=sys.stderr, flush=True)

    # ------------------------------------------------------------------ accuracy + CPU oracle baseline
    # Both use the oracle (test infrastructure), so both run in this leg only.
    torch.cuda.synchronize()
    acc = {"max_abs_logit_diff_bf16_vs_fp32": float(np.abs(logits_b[:n_sites].cpu().numpy()
                                                               - logits_f[:n_sites].cpu().numpy()).max())}
    cpu = None
    if not args.no_cpu_baseline:
        cpu, acc_o = cpu_baseline_and_accuracy(args, dev, cfg, tris_np, dims, layers, occ_np, pvs_b, pvs_f,
                                               logits_b, logits_f, n_sites, total_bytes)
        acc.update(acc_o)

    line = {
        "metric": METRIC,
        "value": 1000.0 / ms_step,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "city256: 256x256x128 froxel grid, 50000 triangles, d=4 (64 ch), "
                               "6 submanifold 3^3 convs 64->64, batch 1, fwd+bwd+Adam per frame",
                   "global_batch": 1, "grid": [256, 256, 128], "n_sites": n_sites, "n_pairs": n_pairs,
                   "occupancy": occupied / (8 * total_bytes), "parallelism": "single GPU"},
        "roofline": roofline,
        "roofline_fp32_conv": roofline_fp32,
        "cpu_baseline": cpu,
        "variants": variants,
        "stages_ms": stage_ms,
        "stages_hbm": stage_gbs,
        "batch16": batch16,
        "train128x4": train4,
        "interleave_8_16": wide,
        "stages_by_interleave_factor": stage_table,
        "dense_interleave_logits_grid": dense,
        "device_memory": memory,
        "culling": cull,
        "unet": unet,
        "world_space": world,
        "accuracy": acc,
        "library_source_hash": npvs._lib.get().npvs_source_hash().decode(),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
