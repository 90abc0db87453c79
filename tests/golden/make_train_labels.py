"""Writes tests/golden/train128x4_labels.npz: ground-truth PVS labels of the four 128^3 training
grids (seeds 30-33), computed by the oracle's ray-march labeller (the dense viewcell sampling of
Sec. 3.2: M = 64 viewpoints from a unit viewcell cube centred at (64, 64, -64), 2 x 2 rays per
froxel face of the grid box).  Calls only synth/ and oracle/.

Usage: python tests/golden/make_train_labels.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

M, S_R, VIEW_SEED = 64, 2, 200


def main():
    cfg = synth.config("train128x4")
    out = {}
    for i, g in enumerate(cfg.grids):
        tris = synth.scene_for(cfg, i)
        views = synth.viewpoints(VIEW_SEED + i, M, (g[0] / 2, g[1] / 2, -g[2] / 2), 1.0)
        out[f"labels{i}"] = oracle.label_raymarch(tris, g, views, S_R)
        print(i, int(oracle.unpack(out[f"labels{i}"]).sum()), flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "train128x4_labels.npz"),
                        m=M, s_r=S_R, view_seed=VIEW_SEED, **out)


if __name__ == "__main__":
    main()
