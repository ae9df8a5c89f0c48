"""Exact pseudo-forest matching (the tree recursion; HGP_MATCH_EXACT and
HGP_FLAG_EXACT_MATCHING) on the GPU against the CPU oracle, through the
C-ABI.  Integer method: every comparison is exact.  The oracle's rule is
pinned to brute-force maximum-weight matching in
tests/test_oracle_exact_matching.py."""
import random
import sys

import numpy as np
import pytest

import oracle
from paper_2604_14411_amd import synth
from test_oracle_exact_matching import _case, random_pseudo_forest

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


def _check_match(ctx, pair, score, label):
    from paper_2604_14411_amd import hgp

    say(f"[exact match] {label} n={len(pair)}")
    m, gam, nn = hgp.level_match(ctx, _dev(pair, np.int32), _dev(score, np.int64), hgp.MATCH_EXACT)
    ref = oracle.match(pair, score, oracle.MATCH_EXACT)
    assert np.array_equal(m.cpu().numpy(), ref)
    reps = np.flatnonzero(ref >= np.arange(len(ref)))
    assert nn == len(reps)
    # gamma: rank of each cluster's smaller member
    rank = np.empty(len(ref), np.int64)
    rank[reps] = np.arange(len(reps))
    assert np.array_equal(gam.cpu().numpy(), rank[np.minimum(ref, np.arange(len(ref)))])


@pytest.mark.parametrize("seed", range(6))
def test_random_pseudo_forests(ctx, seed):
    rng = random.Random(90_000 + seed)
    n = [1, 2, 13, 1000, 60_000, 200_000][seed]
    pair, score = random_pseudo_forest(rng, n)
    _check_match(ctx, pair, score, f"random seed={seed}")


def test_long_chain_and_wide_star(ctx):
    # a chain of 5000 nodes hanging from a 2-cycle, then a star of 3000 leaves
    n_chain, n_star = 5000, 3000
    pair = [1, 0] + [i - 1 for i in range(2, n_chain)]
    score = [7, 7] + [1 + (i * 37) % 11 for i in range(2, n_chain)]
    base = len(pair)
    pair += [-1] + [base] * n_star
    score += [0] + [1 + (i * 13) % 5 for i in range(n_star)]
    _check_match(ctx, pair, score, "chain + star")


def test_pairs_of_a_real_rating(ctx):
    g = synth.random_snn(4000, 30.0, 91)
    rc, _, _, tr = oracle.partition(g, 128, 600, trace=True)
    assert rc == 0
    for l in (0, tr.levels // 2, tr.levels - 1):
        _check_match(ctx, tr.get(oracle.LV_PAIR, l), tr.get(oracle.LV_SCORE, l), f"rating level {l}")


def _compare(ctx, g, omega, delta, k=0, rounds=8, flags=0, label=""):
    from paper_2604_14411_amd import hgp

    say(f"[exact partition] {label} n={g.n_nodes} P={g.n_pins} omega={omega} delta={delta}")
    rc, ref, rres, _ = oracle.partition(g, omega, delta, k=k, max_rounds=rounds, matching=oracle.MATCH_EXACT)
    dg = hgp.DeviceHypergraph(g, "cuda:0")
    try:
        parts, res = hgp.partition_device(ctx, dg, omega, delta, k=k, max_refine_rounds=rounds,
                                          flags=hgp.FLAG_EXACT_MATCHING | flags)
        grc = 0
    except hgp.HgpError as e:
        grc = e.code
    assert grc == rc
    if rc:
        return
    assert np.array_equal(parts.cpu().numpy(), ref)
    for key in ("connectivity", "n_parts", "n_levels", "n_rounds"):
        assert res[key] == rres[key], key


@pytest.mark.parametrize("seed", range(60))
def test_tiny_end_to_end(ctx, seed):
    g, omega, delta, k, rounds = _case(95_000 + seed)
    _compare(ctx, g, omega, delta, k, rounds, label=f"tiny seed={seed}")


MEDIUM = [
    ("rand1500", lambda: synth.random_snn(1500, 24.0, 102), 64, 200),
    ("rand4000", lambda: synth.random_snn(4000, 40.0, 103), 128, 600),
    ("rand2500_tail", lambda: synth.random_snn(2500, 30.0, 31), 1024, 400),
    ("conv_small", lambda: synth.layered_conv(4, 6, 8, 8, 3, 0.1, 105), 64, 2000),
    ("conv_tail", lambda: synth.layered_conv(6, 8, 8, 8, 3, 0.1, 34), 256, 3000),
]


@pytest.mark.parametrize("incremental", [True, False], ids=["incremental", "full"])
@pytest.mark.parametrize("name,make,omega,delta", MEDIUM, ids=[c[0] for c in MEDIUM])
def test_medium_end_to_end(ctx, name, make, omega, delta, incremental):
    from paper_2604_14411_amd import hgp

    _compare(ctx, make(), omega, delta, flags=0 if incremental else hgp.FLAG_NO_INCREMENTAL, label=name)


def test_exact_matching_rejects_the_learned_proposal(ctx):
    from paper_2604_14411_amd import hgp

    g = synth.random_snn(300, 8.0, 5)
    dg = hgp.DeviceHypergraph(g, "cuda:0")
    with pytest.raises(hgp.HgpError) as e:
        hgp.partition_device(ctx, dg, 16, 80, flags=hgp.FLAG_EXACT_MATCHING, mlp=synth.random_int_mlp(1))
    assert e.value.code == hgp.EINVAL
