"""Batches of independent hypergraphs: every schedule gives each graph the
result of a single call (and of the oracle)."""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2604_14411_amd import synth

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


def _batch():
    gs, om, de = [], [], []
    for i in range(9):
        g, n, mu = synth.random_snn_family(7000 + i, 8.0, 11.0, 8.0, 48.0)
        gs.append(g)
        om.append(64 if i % 3 else 1024)
        de.append(256 if i % 2 else 4096)
    gs.append(synth.layered_conv(4, 6, 8, 8, 3, 0.1, 7100))
    om.append(64)
    de.append(2000)
    gs.append(synth.from_lists(3, [([0], [1, 2])]))
    om.append(2)
    de.append(1)
    return gs, om, de


@pytest.fixture(scope="module")
def singles(ctx):
    from paper_2604_14411_amd import hgp

    gs, om, de = _batch()
    dgs = [hgp.DeviceHypergraph(g, "cuda:0") for g in gs]
    ref = []
    for i, d in enumerate(dgs):
        say(f"[batch] single {i} n={gs[i].n_nodes} pins={gs[i].n_pins}")
        p, r = hgp.partition_device(ctx, d, om[i], de[i])
        ref.append((p.cpu().numpy().copy(), r["connectivity"], r["n_parts"]))
    return gs, om, de, dgs, ref


SCHEDS = [None, dict(workers=1, order=2), dict(workers=8, rate_tile=256, late_levels=2), dict(workers=3, order=1)]


@pytest.mark.parametrize("sched", SCHEDS, ids=["default", "w1_input", "w8_tile256_full", "w3_lpt"])
def test_batch_matches_single_calls(ctx, singles, sched):
    from paper_2604_14411_amd import hgp

    gs, om, de, dgs, ref = singles
    say(f"[batch] schedule {sched}")
    wall = time.perf_counter()
    parts, res, t0, t1 = hgp.partition_batch_device(ctx, dgs, om, de, sched=sched)
    wall = (time.perf_counter() - wall) * 1e3
    for i in range(len(gs)):
        assert np.array_equal(parts[i].cpu().numpy(), ref[i][0]), i
        assert res[i]["connectivity"] == ref[i][1] and res[i]["n_parts"] == ref[i][2]
        if res[i]["n_levels"] >= 3:
            assert res[i]["n_kept"] > 0, i  # the workers keep coarse levels
    # device-clock stamps: inside the call, and one after another on one worker
    assert np.all(t0 >= 0) and np.all(t1 > t0) and t1.max() <= wall * 1.05 + 5.0
    if sched and sched.get("workers") == 1 and sched.get("order") == 2:
        assert np.all(t0[1:] >= t1[:-1])


def test_batch_matches_oracle(singles):
    gs, om, de, dgs, ref = singles
    for i in (0, 4, 9, 10):
        rc, p, r, _ = oracle.partition(gs[i], om[i], de[i])
        assert rc == 0 and np.array_equal(p, ref[i][0]) and r["connectivity"] == ref[i][1]


def test_autotuner_picks_a_valid_schedule(ctx, singles):
    from paper_2604_14411_amd import hgp

    gs, om, de, dgs, ref = singles
    say("[batch] tune")
    best, ms = hgp.batch_tune(ctx, dgs, om, de)
    assert best["workers"] in (1, 2, 4, 8, 16) and best["rate_tile"] in (256, 512, 1024)
    assert best["order"] in (1, 2) and best["late_levels"] in (1, 2) and ms > 0
    parts, res, _, _ = hgp.partition_batch_device(ctx, dgs, om, de)  # tuned schedule
    for i in range(len(gs)):
        assert np.array_equal(parts[i].cpu().numpy(), ref[i][0]), i


def test_learned_batch_matches_single_calls_and_oracle(ctx, singles):
    """The learned proposal in a batch: every graph gets the result of a
    single learned call, under two schedules and the tuned one, and the
    oracle's on three of them."""
    import os

    from paper_2604_14411_amd import hgp
    from paper_2604_14411_amd.learn import load_checkpoint

    q, _, _ = load_checkpoint(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                           "paper_2604_14411_amd", "mlp_v2.json"))
    gs, om, de, dgs, _ = singles
    ref = []
    for i, d in enumerate(dgs):
        p, r = hgp.partition_device(ctx, d, om[i], de[i], mlp=q)
        ref.append((p.cpu().numpy().copy(), r["connectivity"], r["n_parts"], r["n_levels"]))
    for i in (0, 9, 10):
        rc, p, r, _ = oracle.partition_learned(gs[i], om[i], de[i], q)
        assert rc == 0 and np.array_equal(p, ref[i][0]) and r["connectivity"] == ref[i][1], i
    say("[batch] learned tune")
    best, ms = hgp.batch_tune(ctx, dgs, om, de, mlp=q)
    assert best["workers"] in (1, 2, 4, 8, 16) and ms > 0
    for sched in (dict(workers=1, order=2), dict(workers=4, order=1), None):
        say(f"[batch] learned schedule {sched}")
        parts, res, t0, t1 = hgp.partition_batch_device(ctx, dgs, om, de, sched=sched, mlp=q)
        for i in range(len(gs)):
            assert np.array_equal(parts[i].cpu().numpy(), ref[i][0]), (sched, i)
            assert res[i]["connectivity"] == ref[i][1] and res[i]["n_levels"] == ref[i][3], (sched, i)
        assert np.all(t1 > t0)


def test_batch_rejects_bad_member(ctx, singles):
    from paper_2604_14411_amd import hgp

    gs, om, de, dgs, ref = singles
    bad = list(om)
    bad[3] = 0
    with pytest.raises(hgp.HgpError) as e:
        hgp.partition_batch_device(ctx, dgs, bad, de)
    assert e.value.code == hgp.EINVAL
    with pytest.raises(hgp.HgpError):
        hgp.partition_batch_device(ctx, dgs, om, de, sched=dict(workers=17))
