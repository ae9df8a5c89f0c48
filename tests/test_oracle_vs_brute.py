"""Pin every step of the CPU oracle to the brute-force set definitions.

On tiny random directed hypergraphs the oracle runs with its tracer on; each
recorded level and refinement round is recomputed from scratch by
``brute.py`` (literal sets, Eq. 1 from scratch, the matching procedure of
Sec. III-B simulated step by step) and must agree exactly.
"""
import random

import numpy as np
import pytest

import brute
import oracle
from paper_2604_14411_amd.synth import from_lists

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _feasible(L, omega, delta):
    return all(L.size[v] <= omega and len(L.inb(v)) <= delta for v in range(L.n))


def _case(seed):
    rng = random.Random(seed)
    n = rng.randint(2, 12)
    hedges, w, nw = brute.random_tiny(rng, n, rng.randint(1, 10), 5, wmax=5, node_wmax=rng.choice([1, 1, 3]))
    g = from_lists(n, hedges, w, nw)
    omega = rng.randint(1, 9)
    delta = rng.randint(0, 7)
    k = rng.choice([0, 0, 0, 1, 2])
    rounds = rng.choice([1, 2, 8])
    return g, omega, delta, k, rounds


def _check_case(g, omega, delta, k, rounds, role=0):
    L0 = brute.level_from_input(g, role)
    rc, parts, res, tr = oracle.partition(g, omega, delta, k=k, max_rounds=rounds, trace=True, role=role)
    if not _feasible(L0, omega, delta):
        assert rc == oracle.EINFEASIBLE
        return
    assert rc == oracle.OK
    w = [int(x) for x in g.hedge_w]
    levels = []
    for l in range(tr.levels):
        L = brute.level_from_trace(tr.get(oracle.LV_HOFF, l), tr.get(oracle.LV_HPIN, l), tr.get(oracle.LV_SIZE, l), w)
        levels.append(L)
    # level 0 is the input, canonicalised
    assert levels[0].hedges == L0.hedges and levels[0].size == L0.size
    for l, L in enumerate(levels):
        pair, score = brute.rate_select(L, omega, delta)
        assert list(tr.get(oracle.LV_PAIR, l)) == pair, f"pair level {l}"
        assert list(tr.get(oracle.LV_SCORE, l)) == score, f"score level {l}"
        match = brute.match_procedural(pair, score)
        assert list(tr.get(oracle.LV_MATCH, l)) == match, f"match level {l}"
        gam = tr.get(oracle.LV_GAMMA, l)
        if any(match[v] != v for v in range(L.n)):
            gamma, C = brute.contract(L, match)
            assert list(gam) == gamma
            if l + 1 < len(levels):
                assert levels[l + 1].hedges == C.hedges and levels[l + 1].size == C.size
        else:
            assert gam is None and l == len(levels) - 1
    for r in range(tr.rounds):
        info = tr.get(oracle.RD_INFO, r)
        lv, S, istar, gstar, applied, n_parts = (int(x) for x in info)
        L = levels[lv]
        rho = [int(x) for x in tr.get(oracle.RD_RHO, r)]
        b = brute.refine_round(L, rho, n_parts, omega, delta)
        assert list(tr.get(oracle.RD_PDEST, r)) == b["dest"]
        assert list(tr.get(oracle.RD_PGAIN, r)) == b["gain"]
        assert list(tr.get(oracle.RD_SEQ, r)) == b["seq"]
        assert list(tr.get(oracle.RD_GP, r)) == b["gp"]
        assert list(tr.get(oracle.RD_G, r)) == b["G"]
        assert list(tr.get(oracle.RD_VIOL, r)) == b["viol"]
        assert istar == b["istar"] and bool(applied) == b["applied"]
    # output: every part valid, reported connectivity = Eq. 1 from scratch
    parts = [int(x) for x in parts]
    n_parts = res["n_parts"]
    assert sorted(set(parts)) == list(range(n_parts))
    assert brute.part_valid_all(L0, parts, n_parts, omega, delta) == 0
    assert res["connectivity"] == brute.conn(L0, parts)
    return res


@pytest.mark.parametrize("seed", range(400))
def test_oracle_steps_match_brute_force(seed):
    _check_case(*_case(seed))


@pytest.mark.parametrize("role", [1, 2])
@pytest.mark.parametrize("seed", range(150))
def test_oracle_constraint_variants_match_brute_force(seed, role):
    # outbound (source pins) and incident (all pins) variants of the Delta bound
    _check_case(*_case(20_000 + seed), role=role)


@pytest.mark.parametrize("seed", range(40))
def test_oracle_not_below_exhaustive_optimum(seed):
    rng = random.Random(10_000 + seed)
    n = rng.randint(2, 8)
    hedges, w, nw = brute.random_tiny(rng, n, rng.randint(1, 8), 4, wmax=4)
    g = from_lists(n, hedges, w, nw)
    omega, delta = rng.randint(1, 5), rng.randint(1, 6)
    L0 = brute.level_from_input(g)
    rc, parts, res, _ = oracle.partition(g, omega, delta)
    if not _feasible(L0, omega, delta):
        assert rc == oracle.EINFEASIBLE
        return
    assert rc == oracle.OK
    opt = brute.exhaustive_optimum(L0, omega, delta)
    assert res["connectivity"] >= opt


def test_graph_case_hist_is_edge_weight():
    # all hedges have two pins: hist(n, m) is the weight of the edge(s) joining them
    rng = random.Random(5)
    n = 9
    hedges, w = [], []
    for a, b in brute.combos(n):
        if rng.random() < 0.5:
            hedges.append(([a], [b]))
            w.append(rng.randint(1, 9))
    g = from_lists(n, hedges, w)
    _, _, _, tr = oracle.partition(g, 100, 100, trace=True)
    pair = tr.get(oracle.LV_PAIR, 0)
    score = tr.get(oracle.LV_SCORE, 0)
    for v in range(n):
        best = None
        for (s, d), x in zip(hedges, w):
            if v in (s[0], d[0]):
                m = d[0] if s[0] == v else s[0]
                wt = sum(xx for (ss, dd), xx in zip(hedges, w) if {ss[0], dd[0]} == {v, m})
                if best is None or (wt, m) > best:
                    best = (wt, m)
        if best is None:
            assert pair[v] == -1
        else:
            assert (int(score[v]), int(pair[v])) == best
