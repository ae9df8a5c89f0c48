"""GPU training kernels and merge traces vs the CPU references.

* hgp_mlp_grad (hand-written forward/backward kernels, FP32) against the
  float64 back-propagation of oracle/mlp_ref.py;
* hgp_mlp_train lowers the loss and is deterministic for a seed;
* hgp_partition_traced returns the plain partition, and its rows (candidate
  pairs, codes, labels) match the oracle's candidate records, with labels
  recomputed here from the oracle's cluster maps and final parts.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp_ref
from paper_2604_14411_amd import synth
from paper_2604_14411_amd.synth import feature_codes

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2604_14411_amd import hgp

    assert torch.cuda.is_available()
    c = hgp.Context(0)
    yield c
    c.close()


def _dev(a, dt):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=dt)).to("cuda:0")


@pytest.mark.parametrize("n,seed", [(1, 0), (63, 1), (3001, 2), (20000, 3)])
def test_gradient_matches_float64_reference(ctx, n, seed):
    from paper_2604_14411_amd import hgp

    w = hgp.mlp_init(seed)
    rng = np.random.default_rng(seed)
    w["b3"] = 0.3
    w["w3"] = w["w3"] * 2
    x = feature_codes(10 + seed, n)
    y = (rng.random(n) < 0.4).astype(np.float32)
    say(f"[grad] n={n}")
    g, L = hgp.mlp_grad(ctx, w, _dev(x, np.int32), _dev(y, np.float32))
    Lr, gr = mlp_ref.grad(w, x, y)
    assert abs(L - Lr) <= 1e-5 * max(1.0, abs(Lr))
    for k in ("w1", "b1", "w2", "b2", "w3"):
        a, b = np.asarray(g[k], np.float64), np.asarray(gr[k], np.float64)
        scale = max(np.abs(b).max(), 1e-6)
        assert np.abs(a - b).max() <= 2e-4 * scale, (k, np.abs(a - b).max(), scale)
    assert abs(g["b3"] - gr["b3"]) <= 2e-4 * max(abs(gr["b3"]), 1e-6)


def test_training_lowers_loss_and_is_deterministic(ctx):
    from paper_2604_14411_amd import hgp

    n = 30000
    x = feature_codes(21, n)
    # a learnable rule: pairs with a large first code and a small fifth code
    y = ((x[:, 0] > 128) & (x[:, 4] < 160)).astype(np.float32)
    xd, yd = _dev(x, np.int32), _dev(y, np.float32)
    w0 = hgp.mlp_init(5)
    L0 = mlp_ref.loss(w0, x, y)
    say("[train] run 1")
    w1, losses1 = hgp.mlp_train(ctx, w0, xd, yd, epochs=6, batch=1024, lr=3e-3, seed=9)
    say("[train] run 2")
    w2, losses2 = hgp.mlp_train(ctx, w0, xd, yd, epochs=6, batch=1024, lr=3e-3, seed=9)
    for k in ("w1", "b1", "w2", "b2", "w3"):
        assert np.array_equal(w1[k], w2[k]), k
    assert losses1 == losses2
    L1 = mlp_ref.loss(w1, x, y)
    assert L1 < 0.5 * L0 and L1 < 0.25, (L0, L1, losses1)
    assert losses1[-1] < losses1[0]


def _labels_from_oracle(tr, parts, level, node, cand):
    # rep_l(c): smallest level-0 member of cluster c of level l
    gams = []
    l = 0
    while True:
        g = tr.get(oracle.LV_GAMMA, l)
        if g is None:
            break
        gams.append(g)
        l += 1
    reps = [np.arange(len(parts))]
    for g in gams:
        nn = int(g.max()) + 1 if len(g) else 0
        r = np.full(nn, np.iinfo(np.int64).max)
        np.minimum.at(r, g, reps[-1])
        reps.append(r)
    return np.array([float(parts[reps[lv][a]] == parts[reps[lv][b]]) for lv, a, b in zip(level, node, cand)],
                    np.float32)


TRACE_CASES = [
    ("rand1500", lambda: synth.random_snn(1500, 24.0, 61), 64, 200),
    ("conv", lambda: synth.layered_conv(4, 6, 8, 8, 3, 0.1, 62), 64, 2000),
]


@pytest.mark.parametrize("name,make,omega,delta", TRACE_CASES, ids=[c[0] for c in TRACE_CASES])
def test_traced_partition_rows_match_oracle(ctx, name, make, omega, delta):
    from paper_2604_14411_amd import hgp

    g = make()
    say(f"[trace] {name}")
    parts, res, t = hgp.partition_traced(ctx, g, omega, delta)
    p2, r2 = hgp.partition_host(ctx, g, omega, delta)
    assert np.array_equal(parts, p2) and res["connectivity"] == r2["connectivity"]
    rc, ref, rres, tr = oracle.partition(g, omega, delta, trace=True)
    assert rc == 0 and np.array_equal(parts, ref)
    rows = []
    for l in range(tr.levels):
        coff, cand, feat = tr.get(oracle.LV_COFF, l), tr.get(oracle.LV_CAND, l), tr.get(oracle.LV_FEAT, l)
        feat = feat.reshape(-1, 16)
        for v in range(len(coff) - 1):
            for j in range(coff[v], coff[v + 1]):
                if v < cand[j]:
                    rows.append((l, v, int(cand[j]), tuple(feat[j])))
    assert len(rows) == len(t["node"])
    got = list(zip(t["level"].tolist(), t["node"].tolist(), t["cand"].tolist(), map(tuple, t["xq"].tolist())))
    assert got == rows
    lab = _labels_from_oracle(tr, ref, t["level"], t["node"], t["cand"])
    assert np.array_equal(lab, t["label"])
    assert 0 < t["label"].mean() < 1


def test_training_resumed_from_checkpoint_is_bit_identical(ctx, tmp_path):
    """3 epochs, a binary checkpoint (weights, Adam moments, step, shuffle
    state), a fresh state loaded from it, 3 more epochs: the same bits as 6
    epochs in one run."""
    from paper_2604_14411_amd import hgp

    n = 12000
    x = feature_codes(31, n)
    y = ((x[:, 1] > 100) ^ (x[:, 6] < 90)).astype(np.float32)
    xd, yd = _dev(x, np.int32), _dev(y, np.float32)
    w0 = hgp.mlp_init(6)
    say("[resume] uninterrupted")
    w_full, loss_full = hgp.mlp_train(ctx, w0, xd, yd, epochs=6, batch=1000, lr=3e-3, seed=13)
    st = hgp.train_state(w0, seed=13)
    say("[resume] first half")
    la = hgp.mlp_train_state(ctx, st, xd, yd, 3, batch=1000, lr=3e-3)
    path = str(tmp_path / "half.hgpmlp")
    hgp.mlp_save(path, st)
    del st
    st2, _, _ = hgp.mlp_load(path, network=False)
    assert st2.epoch == 3 and st2.step == 3 * 12
    say("[resume] second half")
    lb = hgp.mlp_train_state(ctx, st2, xd, yd, 3, batch=1000, lr=3e-3)
    w_res = hgp.f32_to_dict(st2.w)
    for k in ("w1", "b1", "w2", "b2", "w3"):
        assert np.array_equal(w_res[k], w_full[k]), k
    assert w_res["b3"] == w_full["b3"]
    assert la + lb == loss_full


def test_host_connectivity_matches_oracle(ctx):
    from paper_2604_14411_amd import hgp

    g = synth.random_snn(1800, 20.0, 71)
    rng = np.random.default_rng(72)
    for k in (1, 5, 250, g.n_nodes):
        part = rng.integers(0, k, size=g.n_nodes).astype(np.int32)
        say(f"[connectivity host] k={k}")
        assert hgp.connectivity_host(ctx, g, part) == oracle.connectivity(g, part)
    with pytest.raises(hgp.HgpError) as e:
        hgp.connectivity_host(ctx, g, np.full(g.n_nodes, g.n_nodes, np.int32))
    assert e.value.code == hgp.EBADCSR
