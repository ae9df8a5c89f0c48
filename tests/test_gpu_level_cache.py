"""The device memory that keeps coarse levels for refinement (hgp_set_level_cache).

The partition is the same, id by id, whatever the budget, and equals the
oracle's: all levels kept, none, a budget below the first coarse levels (they
are rebuilt from level 0 when refinement reaches them) and budgets of about
one and three levels, under which the ring wraps around many times and
evicts levels while coarsening.  The number of levels refinement found kept
(n_kept) is predicted exactly by replaying the ring's placement rule on the
level sizes of the oracle's trace, with the capacity the context reports."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2604_14411_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
HERE = os.path.dirname(os.path.abspath(__file__))
LV_HOFF, LV_SIZE = 0, 2  # oracle trace records: hedge offsets and node sizes of a level


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
    c.set_level_cache(-1)
    c.close()


def _a256(b):
    return (b + 255) // 256 * 256


def _level_bytes(n, E, P):
    """hoff, hpin, inc, perm, ioff, indeg and total, each on a 256-byte boundary."""
    return _a256(4 * (E + 1)) + 3 * _a256(4 * P) + 3 * _a256(4 * (n + 1))


def _replay(sizes, E, cap):
    """Levels 1 .. L-1 placed in order in a ring of `cap` bytes: each goes
    after the newest (back to the start when it would pass the end, dropping
    the levels between the newest and the end), evicting the oldest levels it
    overlaps; a level larger than the ring is not kept.  Returns the levels
    1 .. L-2 kept at the end (the ones refinement looks up), wraps and levels
    too large."""
    kept, head, wraps, skipped = [], 0, 0, 0
    for lvl in range(1, len(sizes)):
        b = _level_bytes(sizes[lvl][0], E, sizes[lvl][1])
        if b > cap:
            skipped += 1
            continue
        off = head
        if off + b > cap:
            wraps += 1
            while kept and kept[0][1] >= head:
                kept.pop(0)
            off = 0
        while kept and kept[0][1] < off + b and kept[0][1] + kept[0][2] > off:
            kept.pop(0)
        kept.append((lvl, off, b))
        head = off + b
    L = len(sizes)
    return sum(1 for k in kept if 1 <= k[0] <= L - 2), wraps, skipped


CASES = [
    ("rand2500_tail", lambda: synth.random_snn(2500, 30.0, 31), 1024, 400, False),
    ("conv_tail", lambda: synth.layered_conv(6, 8, 8, 8, 3, 0.1, 34), 256, 3000, False),
    ("rand4000", lambda: synth.random_snn(4000, 40.0, 103), 128, 600, False),
    ("learned_rand3000", lambda: synth.random_snn(3000, 30.0, 35), 256, 600, True),
]
_paths = {"wrapped": 0, "too large": 0, "partly kept": 0}


@pytest.mark.parametrize("name,make,omega,delta,learned", CASES, ids=[c[0] for c in CASES])
def test_partition_independent_of_level_budget(ctx, name, make, omega, delta, learned):
    from paper_2604_14411_amd import hgp
    from paper_2604_14411_amd.learn import load_checkpoint

    g = make()
    mlp = None
    if learned:
        mlp, _, _ = load_checkpoint(os.path.join(HERE, "..", "paper_2604_14411_amd", "mlp_v2.json"))
        rc, ref, rres, tr = oracle.partition_learned(g, omega, delta, mlp, trace=True)
    else:
        rc, ref, rres, tr = oracle.partition(g, omega, delta, trace=True)
    assert rc == 0
    sizes = [(len(tr.get(LV_SIZE, lvl)), int(tr.get(LV_HOFF, lvl)[-1])) for lvl in range(tr.levels)]
    L = len(sizes)
    assert L == rres["n_levels"] >= 6, "the case needs several coarse levels"
    b0 = _level_bytes(g.n_nodes, g.n_hedges, g.n_pins)
    dg = hgp.DeviceHypergraph(g, "cuda:0")
    for budget, what in [(-1, "default"), (0, "none"), (b0 // 2, "half of level 0"), (5 * b0 // 4, "about one level"),
                         (3 * b0, "about three levels"), (-1, "default again")]:
        held = ctx.set_level_cache(budget)
        if budget >= 0:
            assert held <= budget
        for rep in range(2):
            say(f"[level cache] {name}: budget {budget} ({what}), run {rep}")
            parts, res = hgp.partition_device(ctx, dg, omega, delta, mlp=mlp)
            assert np.array_equal(parts.cpu().numpy(), ref), what
            for key in ("connectivity", "n_parts", "n_levels", "n_rounds"):
                assert res[key] == rres[key], (what, key)
            cap = ctx.set_level_cache(budget)  # the ring the run used (nothing released)
            want, wraps, skipped = _replay(sizes, g.n_hedges, cap)
            say(f"[level cache]   n_kept {res['n_kept']} of {L - 2} (ring {cap} B, {wraps} wraps, "
                f"{skipped} levels too large)")
            assert res["n_kept"] == want, (what, rep, res["n_kept"], want)
            _paths["wrapped"] += wraps > 0
            _paths["too large"] += skipped > 0
            _paths["partly kept"] += 0 < want < L - 2
        if budget < 0:
            assert res["n_kept"] == L - 2  # the second run sizes the ring for every level


def test_every_ring_path_ran():
    """The cases above wrapped the ring, met levels larger than it and kept
    only some levels (run after them, in file order)."""
    if not any(_paths.values()):
        pytest.skip("the level-budget cases did not run")
    assert all(v > 0 for v in _paths.values()), _paths
