"""Full-size layered network (conv208k: 208,896 nodes, 145.6 M pins) on the
GPU, plain and learned: properties that hold at any size, checked on the CPU
from the returned partition — every part within Omega and Delta, and the
reported connectivity equal to Eq. 1 recomputed by the oracle's routine.
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


@pytest.fixture(scope="module")
def conv208k(gpu):
    from paper_2604_14411_amd.synth.configs import WORKLOADS

    w = WORKLOADS["conv208k"]
    say("[fullsize] generating conv208k")
    return w, w.make()


def _run(conv208k, mlp):
    from paper_2604_14411_amd import hgp

    w, g = conv208k
    ctx = hgp.Context(0)
    dg = hgp.DeviceHypergraph(g, "cuda:0")
    say(f"[fullsize] partition conv208k {'learned' if mlp else 'plain'}")
    t = time.perf_counter()
    parts, res = hgp.partition_device(ctx, dg, w.omega, w.delta, mlp=mlp, flags=hgp.FLAG_TIME_KERNELS)
    parts = parts.cpu().numpy()
    say(f"[fullsize] {time.perf_counter() - t:.2f} s levels={res['n_levels']} parts={res['n_parts']} "
        f"conn={res['connectivity']}; checking")
    for name, k in sorted(res["kernels"].items(), key=lambda kv: -kv[1]["ms"]):
        if k["launches"]:
            say(f"[fullsize]   {name:11s} {k['ms']:9.1f} ms  launches {k['launches']}")
    _check_partition(g, parts, w.omega, w.delta, res)
    ctx.close()
    return res


def test_conv208k_plain_valid(conv208k):
    _run(conv208k, None)


def test_conv208k_learned_valid_and_close_to_plain(conv208k):
    from paper_2604_14411_amd.learn import load_checkpoint

    q, _, _ = load_checkpoint(os.path.join(HERE, "..", "paper_2604_14411_amd", "mlp_v2.json"))
    res = _run(conv208k, q)
    assert res["n_fallback"] == 0
