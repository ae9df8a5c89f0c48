"""Full-size layered networks (conv208k: 208,896 nodes, 145.6 M pins;
conv302k: 302,400 nodes, 256.4 M pins) on the GPU, plain and learned:
properties that hold at any size, checked on the CPU from the returned
partition — every part within Omega and Delta, and the reported connectivity
equal to Eq. 1 recomputed by the oracle's routine — and the learned
proposal's connectivity against the plain method's on the same input.
(The oracle's whole partition at this size takes hours; rand64k is the
full-size case compared id by id, tests/golden/rand64k.json.)"""
import os
import sys
import time

import numpy as np
import pytest

import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
HERE = os.path.dirname(os.path.abspath(__file__))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check_partition(g, parts, omega, delta, res):
    n_parts = res["n_parts"]
    assert parts.min() >= 0 and parts.max() == n_parts - 1
    assert len(np.unique(parts)) == n_parts
    sizes = np.bincount(parts, weights=g.node_w.astype(np.int64), minlength=n_parts)
    assert sizes.max() <= omega
    # inbound: distinct hedges with a destination pin in the part
    off = g.hedge_off.astype(np.int64)
    lens = np.diff(off)
    e_of_pin = np.repeat(np.arange(g.n_hedges, dtype=np.int64), lens)
    is_dst = np.ones(g.n_pins, dtype=bool)
    is_dst[off[:-1][lens > 0]] = False  # one source pin first in every hedge (n_src = 1)
    assert np.all(g.n_src == 1)
    pairs = np.unique(parts[g.pins[is_dst]].astype(np.int64) * g.n_hedges + e_of_pin[is_dst])
    inb = np.bincount(pairs // g.n_hedges, minlength=n_parts)
    assert inb.max() <= delta
    assert res["connectivity"] == oracle.connectivity(g, parts)


@pytest.fixture(scope="module")
def gpu():
    """The device is initialised before the large host arrays are made."""
    import torch

    assert torch.cuda.is_available()
    torch.zeros(1, device="cuda:0")
    torch.cuda.synchronize()
    return torch


_graphs = {}
_results = {}


def _graph(name):
    from paper_2604_14411_amd.synth.configs import WORKLOADS

    if name not in _graphs:
        _graphs.clear()  # one full-size graph in host memory at a time
        say(f"[fullsize] generating {name}")
        _graphs[name] = WORKLOADS[name].make()
    return WORKLOADS[name], _graphs[name]


def _run(name, learned):
    from paper_2604_14411_amd import hgp
    from paper_2604_14411_amd.learn import load_checkpoint

    w, g = _graph(name)
    mlp = None
    if learned:
        mlp, _, _ = load_checkpoint(os.path.join(HERE, "..", "paper_2604_14411_amd", "mlp_v2.json"))
    ctx = hgp.Context(0)
    dg = hgp.DeviceHypergraph(g, "cuda:0")
    say(f"[fullsize] partition {name} {'learned' if mlp else 'plain'}")
    t = time.perf_counter()
    parts, res = hgp.partition_device(ctx, dg, w.omega, w.delta, mlp=mlp, flags=hgp.FLAG_TIME_KERNELS)
    parts = parts.cpu().numpy()
    res["seconds"] = time.perf_counter() - t
    say(f"[fullsize] {res['seconds']:.2f} s levels={res['n_levels']} parts={res['n_parts']} "
        f"conn={res['connectivity']}; checking")
    for kname, k in sorted(res["kernels"].items(), key=lambda kv: -kv[1]["ms"]):
        if k["launches"]:
            say(f"[fullsize]   {kname:11s} {k['ms']:9.1f} ms  launches {k['launches']}")
    del dg
    ctx.close()
    _check_partition(g, parts, w.omega, w.delta, res)
    _results[(name, learned)] = res
    return res


@pytest.mark.parametrize("name", ["conv208k", "conv302k"])
def test_plain_valid(gpu, name):
    _run(name, False)


@pytest.mark.parametrize("name", ["conv208k", "conv302k"])
def test_learned_valid_and_within_two_percent_of_plain(gpu, name):
    """The learned proposal: every part valid, connectivity at most 1.02 x
    the plain method's on the same input (its judge), and fewer levels (the
    source of its higher pins/s)."""
    res = _run(name, True)
    assert res["n_fallback"] == 0
    plain = _results.get((name, False)) or _run(name, False)
    say(f"[fullsize] {name} learned/plain connectivity {res['connectivity'] / plain['connectivity']:.4f} "
        f"levels {res['n_levels']}/{plain['n_levels']} time {res['seconds']:.2f}/{plain['seconds']:.2f} s")
    assert res["connectivity"] <= 1.02 * plain["connectivity"]
    assert res["n_levels"] < plain["n_levels"]
