#!/usr/bin/env python3
"""Trains the learned merge proposal's network on the GPU and writes a checkpoint.

1. Merge traces: the plain partitioner (hgp_partition_traced) runs on seeded
   training hypergraphs whose shapes and seeds differ from every evaluation
   instance; each unordered candidate pair of each coarsening level becomes a
   row (16 input codes, label = the pair ended in one part).
2. Training: hgp_mlp_train (hand-written forward / backward / Adam kernels),
   FP32 master weights, seeded initialisation and shuffles.
3. Quantisation: hgp_mlp_quantize to the integer network (BF16-exact on MFMA).

    python -m paper_2604_14411_amd.learn --out mlp.json [--epochs 6]

The checkpoint holds the float weights, the integer network, the score shift
and the training record (graphs, rows, positive rate, loss per epoch).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2604_14411_amd import hgp  # noqa: E402
from paper_2604_14411_amd import synth  # noqa: E402

# Training hypergraphs: layered conv-like networks of other shapes and seeds
# than the evaluation instances (8 x 96x16x17 seed 3; 8 x 42x30x30 seed 5),
# and random SNNs of other sizes and seeds.
TRAIN_SET = [
    ("conv 8x(32x12x12) 3x3", lambda: synth.layered_conv(8, 32, 12, 12, 3, 0.1, 1101), 4096, 65536),
    ("conv 6x(24x14x14) 5x5", lambda: synth.layered_conv(6, 24, 14, 14, 5, 0.1, 1102), 4096, 65536),
    ("conv 8x(48x10x11) 3x3", lambda: synth.layered_conv(8, 48, 10, 11, 3, 0.1, 1103), 4096, 65536),
    ("rand 8192 mu 64", lambda: synth.random_snn(8192, 64.0, 1104), 1024, 4096),
    ("rand 12000 mu 127", lambda: synth.random_snn(12000, 127.0, 1105), 1024, 4096),
]


# v2 adds layered networks with the evaluation instances' channel widths
# (96 and 42 channels) on other spatial shapes and seeds.
TRAIN_SET_V2 = TRAIN_SET + [
    ("conv 8x(96x10x10) 3x3", lambda: synth.layered_conv(8, 96, 10, 10, 3, 0.1, 1201), 4096, 65536),
    ("conv 8x(42x18x18) 5x5", lambda: synth.layered_conv(8, 42, 18, 18, 5, 0.1, 1202), 4096, 65536),
]
TRAIN_SETS = {"v1": TRAIN_SET, "v2": TRAIN_SET_V2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def collect(ctx, train_set, max_rows_per_graph: int, seed: int):
    rng = np.random.default_rng(seed)
    xs, ys, info = [], [], []
    for name, make, omega, delta in train_set:
        g = make()
        t = time.perf_counter()
        parts, res, tr = hgp.partition_traced(ctx, g, omega, delta)
        rows = len(tr["label"])
        keep = np.arange(rows)
        if rows > max_rows_per_graph:
            keep = np.sort(rng.choice(rows, max_rows_per_graph, replace=False))
        xs.append(tr["xq"][keep])
        ys.append(tr["label"][keep])
        info.append(dict(graph=name, n=g.n_nodes, pins=g.n_pins, omega=omega, delta=delta, rows=int(rows),
                         kept=int(len(keep)), positive=float(tr["label"].mean()) if rows else 0.0,
                         levels=res["n_levels"], connectivity=res["connectivity"]))
        log(f"[learn] {name}: {rows} rows, {len(keep)} kept, positive {info[-1]['positive']:.3f}, "
            f"{time.perf_counter() - t:.1f} s")
    return np.concatenate(xs), np.concatenate(ys), info


def train(out: str, epochs: int = 6, batch: int = 2048, lr: float = 2e-3, seed: int = 7,
          max_rows_per_graph: int = 400_000, k: int = 8, train_set=None):
    import torch

    ctx = hgp.Context(0)
    x, y, info = collect(ctx, train_set or TRAIN_SET, max_rows_per_graph, seed)
    log(f"[learn] {len(y)} rows, positive rate {y.mean():.3f}")
    xd = torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32)).to("cuda:0")
    yd = torch.as_tensor(np.ascontiguousarray(y, dtype=np.float32)).to("cuda:0")
    w0 = hgp.mlp_init(seed)
    t = time.perf_counter()
    w, losses = hgp.mlp_train(ctx, w0, xd, yd, epochs=epochs, batch=batch, lr=lr, seed=seed)
    log(f"[learn] trained {epochs} epochs in {time.perf_counter() - t:.1f} s, loss {losses}")
    calib = x[np.random.default_rng(seed + 1).choice(len(x), min(len(x), 20000), replace=False)]
    q, shift = hgp.mlp_quantize(w, calib, k=k)
    ck = dict(format="hgp-mlp-1", k=k, score_shift=shift,
              float={kk: (np.asarray(v).tolist() if not np.isscalar(v) else float(v)) for kk, v in w.items()},
              int={kk: (np.asarray(v).tolist() if not np.isscalar(v) else int(v)) for kk, v in q.items()},
              train=dict(set=[name for name, *_ in (train_set or TRAIN_SET)], graphs=info, rows=int(len(y)),
                         positive=float(y.mean()), epochs=epochs, batch=batch, lr=lr, seed=seed, loss=losses))
    with open(out, "w") as f:
        json.dump(ck, f)
    log(f"[learn] wrote {out}")
    ctx.close()
    return ck


def load_checkpoint(path: str):
    """Returns (integer network dict, float weights dict, checkpoint dict)."""
    with open(path) as f:
        ck = json.load(f)
    q = {k: (np.asarray(v, dtype=np.int32) if isinstance(v, list) else int(v)) for k, v in ck["int"].items()}
    q["w1"] = q["w1"].reshape(16, 64)
    q["w2"] = q["w2"].reshape(64, 64)
    w = {k: (np.asarray(v, dtype=np.float32) if isinstance(v, list) else float(v)) for k, v in ck["float"].items()}
    w["w1"] = w["w1"].reshape(16, 64)
    w["w2"] = w["w2"].reshape(64, 64)
    return q, w, ck


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--max-rows", type=int, default=400_000)
    ap.add_argument("--set", default="v1", choices=sorted(TRAIN_SETS))
    a = ap.parse_args()
    train(a.out, a.epochs, a.batch, a.lr, a.seed, a.max_rows, train_set=TRAIN_SETS[a.set])


if __name__ == "__main__":
    main()
