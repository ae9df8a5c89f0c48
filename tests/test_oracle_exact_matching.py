"""Exact matching on the pairing pseudo-forest (the dynamic-programming
formulation of Sec. VI) pinned by brute force: on every tiny pseudo-forest
its weight equals the maximum over all subsets of pairing edges, it never
weighs less than the two-traversal matching of Sec. III-A, and a whole
partition with it passes the same per-step and output checks as the plain
method."""
import random

import numpy as np
import pytest

import brute
import oracle
from paper_2604_14411_amd.synth import from_lists

pytestmark = pytest.mark.usefixtures("oracle_lib")


def random_pseudo_forest(rng, n):
    """Components hanging from 2-cycles or from nodes without candidate; every
    other node points to a node of its own component created before it."""
    pair = [-1] * n
    score = [0] * n
    comp_nodes = []
    v = 0
    while v < n:
        if v + 1 < n and rng.random() < 0.5:
            w = rng.randint(1, 9)
            pair[v], pair[v + 1] = v + 1, v
            score[v] = score[v + 1] = w
            comp_nodes.append([v, v + 1])
            v += 2
        else:
            comp_nodes.append([v])
            v += 1
        # grow the component with a few tree nodes
        for _ in range(rng.randint(0, 3)):
            if v >= n:
                break
            comp = comp_nodes[-1]
            pair[v] = rng.choice(comp)
            score[v] = rng.randint(1, 9)
            comp.append(v)
            v += 1
    # shuffle ids so that children need not follow their parents
    perm = list(range(n))
    rng.shuffle(perm)
    inv = {perm[i]: i for i in range(n)}
    p2 = [-1] * n
    s2 = [0] * n
    for i in range(n):
        p2[perm[i]] = perm[pair[i]] if pair[i] >= 0 else -1
        s2[perm[i]] = score[i]
    return p2, s2


@pytest.mark.parametrize("seed", range(300))
def test_exact_matching_is_maximum_weight(seed):
    rng = random.Random(70_000 + seed)
    n = rng.randint(1, 13)
    pair, score = random_pseudo_forest(rng, n)
    ex = oracle.match(pair, score, oracle.MATCH_EXACT)
    tr = oracle.match(pair, score, oracle.MATCH_TRAVERSAL)
    w_ex = brute.matching_weight(pair, score, ex)
    w_tr = brute.matching_weight(pair, score, tr)
    assert w_ex == brute.max_weight_matching(pair, score)
    assert w_ex >= w_tr


def test_exact_matching_special_cases():
    # a chain a <- b <- c hanging from the 2-cycle {a, d}: the heuristic
    # matches the cycle (weight 1); the exact rule takes a-b and nothing else
    # would beat it: with scores 1 (cycle), 5 (b->a), 5 (c->b) the best is
    # {a,d} + {b,c} = 6 against {a,b} = 5
    pair = [3, 0, 1, 0]
    score = [1, 5, 5, 1]
    ex = oracle.match(pair, score, oracle.MATCH_EXACT)
    assert list(ex) == [3, 2, 1, 0]
    # a star: the centre matches its heaviest child, larger id on ties
    pair = [-1, 0, 0, 0]
    score = [0, 4, 7, 7]
    assert list(oracle.match(pair, score, oracle.MATCH_EXACT)) == [3, 1, 2, 0]
    # no candidates at all
    assert list(oracle.match([-1, -1], [0, 0], oracle.MATCH_EXACT)) == [0, 1]


def _case(seed):
    rng = random.Random(seed)
    n = rng.randint(2, 12)
    hedges, w, nw = brute.random_tiny(rng, n, rng.randint(1, 10), 5, wmax=5, node_wmax=rng.choice([1, 1, 3]))
    return from_lists(n, hedges, w, nw), rng.randint(1, 9), rng.randint(0, 7), rng.choice([0, 0, 1]), \
        rng.choice([1, 8])


@pytest.mark.parametrize("seed", range(200))
def test_partition_with_exact_matching_matches_brute_force(seed):
    g, omega, delta, k, rounds = _case(80_000 + seed)
    L0 = brute.level_from_input(g)
    rc, parts, res, tr = oracle.partition(g, omega, delta, k=k, max_rounds=rounds, trace=True,
                                          matching=oracle.MATCH_EXACT)
    feasible = all(L0.size[v] <= omega and len(L0.inb(v)) <= delta for v in range(L0.n))
    if not feasible:
        assert rc == oracle.EINFEASIBLE
        return
    assert rc == oracle.OK
    w = [int(x) for x in g.hedge_w]
    levels = [brute.level_from_trace(tr.get(oracle.LV_HOFF, l), tr.get(oracle.LV_HPIN, l),
                                     tr.get(oracle.LV_SIZE, l), w) for l in range(tr.levels)]
    for l, L in enumerate(levels):
        pair, score = brute.rate_select(L, omega, delta)
        assert list(tr.get(oracle.LV_PAIR, l)) == pair and list(tr.get(oracle.LV_SCORE, l)) == score
        match = tr.get(oracle.LV_MATCH, l)
        assert brute.matching_weight(pair, score, match) == brute.max_weight_matching(pair, score)
        if any(int(match[v]) != v for v in range(L.n)):
            gamma, C = brute.contract(L, [int(x) for x in match])
            assert list(tr.get(oracle.LV_GAMMA, l)) == gamma
            if l + 1 < len(levels):
                assert levels[l + 1].hedges == C.hedges and levels[l + 1].size == C.size
    for r in range(tr.rounds):
        lv, S, istar, gstar, applied, n_parts = (int(x) for x in tr.get(oracle.RD_INFO, r))
        rho = [int(x) for x in tr.get(oracle.RD_RHO, r)]
        b = brute.refine_round(levels[lv], rho, n_parts, omega, delta)
        assert list(tr.get(oracle.RD_G, r)) == b["G"] and list(tr.get(oracle.RD_VIOL, r)) == b["viol"]
        assert istar == b["istar"] and bool(applied) == b["applied"]
    parts = [int(x) for x in parts]
    assert brute.part_valid_all(L0, parts, res["n_parts"], omega, delta) == 0
    assert res["connectivity"] == brute.conn(L0, parts)


def test_traversal_rule_is_the_default():
    g, omega, delta, k, rounds = _case(80_001)
    a = oracle.partition(g, omega, delta, k=k, max_rounds=rounds)
    b = oracle.partition(g, omega, delta, k=k, max_rounds=rounds, matching=oracle.MATCH_TRAVERSAL)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and a[2] == b[2]
