"""Pins of the oracle's learned merge proposal (CPU only).

The feature code, the integer network, the top-K candidate sets, their
symmetric union, the (score, id) selection, the plain fallback and the whole
learned partition are checked against closed forms, hand-computed networks,
explicit-set brute force and the plain oracle (which is itself pinned by brute
force): with a network that is strictly increasing in hist alone, the learned
proposal must reproduce the plain method exactly.
"""
import random

import numpy as np
import pytest

import brute
import oracle
from paper_2604_14411_amd.synth import from_lists, random_int_mlp

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _zero_mlp(k=8, r1=0, r2=0, b3=0):
    return dict(k=k, r1=r1, r2=r2, b3=b3, w1=np.zeros((16, 64), np.int32), b1=np.zeros(64, np.int32),
                w2=np.zeros((64, 64), np.int32), b2=np.zeros(64, np.int32), w3=np.zeros(64, np.int32))


def _identity_on(feature, k=8):
    """score = code of one feature (unit 0 copies it through both layers)."""
    q = _zero_mlp(k)
    q["w1"][feature, 0] = 1
    q["w2"][0, 0] = 1
    q["w3"][0] = 1
    return q


def test_qlog_known_values_and_closed_form():
    known = {0: 0, 1: 8, 2: 12, 3: 16, 4: 18, 7: 24, 14: 31, 15: 32, 16: 32, 255: 64, 2 ** 32 - 2: 255,
             2 ** 32 - 1: 255, 2 ** 40: 255}
    for f, c in known.items():
        assert oracle.qlog(f) == c, f
    rng = random.Random(3)
    vals = list(range(0, 5000)) + [rng.randrange(0, 2 ** 31) for _ in range(3000)]
    for f in vals:
        assert oracle.qlog(f) == brute.qlog_closed(f), f
    # monotone, injective below 15
    codes = [oracle.qlog(f) for f in range(0, 15)]
    assert codes == sorted(set(codes))


def test_network_special_cases():
    x = np.zeros((4, 16), np.int32)
    x[:, 0] = [0, 3, 5, 7]
    # zero network: the output bias
    assert list(oracle.mlp_score(_zero_mlp(b3=-17), x)) == [-17] * 4
    # identity on code 0
    assert list(oracle.mlp_score(_identity_on(0), x)) == [0, 3, 5, 7]
    # halving with ties to even: 0, 1.5 -> 2, 2.5 -> 2, 3.5 -> 4
    q = _identity_on(0)
    q["r1"] = 1
    assert list(oracle.mlp_score(q, x)) == [0, 2, 2, 4]
    # ReLU clamp at 0 and saturation at 255
    q = _identity_on(0)
    q["w1"][0, 0] = -1
    assert list(oracle.mlp_score(q, x)) == [0, 0, 0, 0]
    q = _identity_on(0)
    q["w1"][0, 0] = 100
    assert list(oracle.mlp_score(q, x)) == [0, 255, 255, 255]
    # output layer is linear in w3 and b3
    q = _identity_on(0)
    q["w3"][0] = -3
    q["b3"] = 10
    assert list(oracle.mlp_score(q, x)) == [10, 1, -5, -11]
    # two units summed, second fed by code 1
    q = _identity_on(0)
    q["w1"][1, 1] = 2
    q["w2"][1, 1] = 1
    q["w3"][1] = 1
    x2 = x.copy()
    x2[:, 1] = [1, 2, 3, 4]
    assert list(oracle.mlp_score(q, x2)) == [2, 7, 11, 15]


def test_network_rejects_out_of_range():
    q = _identity_on(0)
    q["w2"][3, 4] = 256
    with pytest.raises(ValueError):
        oracle.mlp_score(q, np.zeros((1, 16), np.int32))
    q = _identity_on(0)
    with pytest.raises(ValueError):
        oracle.mlp_score(q, np.full((1, 16), 256, np.int32))


def _case(seed):
    rng = random.Random(seed)
    n = rng.randint(2, 12)
    hedges, w, nw = brute.random_tiny(rng, n, rng.randint(1, 10), 5, wmax=5, node_wmax=rng.choice([1, 1, 3]))
    g = from_lists(n, hedges, w, nw)
    return g, rng.randint(2, 9), rng.randint(1, 7), rng.choice([0, 0, 1]), rng.choice([1, 8]), rng


def _feasible(L, omega, delta):
    return all(L.size[v] <= omega and len(L.inb(v)) <= delta for v in range(L.n))


def _check_learned(g, omega, delta, k, rounds, mlp):
    L0 = brute.level_from_input(g)
    rc, parts, res, tr = oracle.partition_learned(g, omega, delta, mlp, k=k, max_rounds=rounds, trace=True)
    if not _feasible(L0, omega, delta):
        assert rc == oracle.EINFEASIBLE
        return None
    assert rc == oracle.OK
    w = [int(x) for x in g.hedge_w]
    K = int(mlp["k"])
    fallbacks = 0
    for l in range(tr.levels):
        L = brute.level_from_trace(tr.get(oracle.LV_HOFF, l), tr.get(oracle.LV_HPIN, l), tr.get(oracle.LV_SIZE, l), w)
        top, C = brute.candidates(L, omega, delta, K)
        coff = tr.get(oracle.LV_COFF, l)
        cand = tr.get(oracle.LV_CAND, l)
        csc = tr.get(oracle.LV_CSCORE, l)
        feat = tr.get(oracle.LV_FEAT, l).reshape(-1, 16)
        assert len(coff) == L.n + 1
        sc = {}
        for n in range(L.n):
            ids = [int(x) for x in cand[coff[n]:coff[n + 1]]]
            assert ids == sorted(C[n]), f"candidates level {l} node {n}"
            for j, m in enumerate(ids):
                h, c = C[n][m]
                assert list(feat[coff[n] + j]) == brute.pair_features(L, l, omega, delta, n, m, h, c)
                sc[(n, m)] = int(csc[coff[n] + j])
        if len(feat):
            assert list(oracle.mlp_score(mlp, feat)) == [int(x) for x in csc]
        for (n, m), s in sc.items():
            assert sc[(m, n)] == s, "scores of an unordered pair differ"
        pair, score = [-1] * L.n, [0] * L.n
        for n in range(L.n):
            best = max(((sc[(n, m)], m) for m in C[n]), default=None)
            if best is not None:
                score[n], pair[n] = best
        assert list(tr.get(oracle.LV_PAIR, l)) == pair
        assert list(tr.get(oracle.LV_SCORE, l)) == score
        ppair, pscore = brute.rate_select(L, omega, delta)
        assert list(tr.get(oracle.LV_PPAIR, l)) == ppair
        lm = brute.match_procedural(pair, score)
        pm = brute.match_procedural(ppair, pscore)
        ml = sum(1 for v in range(L.n) if lm[v] > v)
        mp = sum(1 for v in range(L.n) if pm[v] > v)
        fb = 2 * ml < mp
        assert int(tr.get(oracle.LV_FALLBACK, l)[0]) == int(fb)
        fallbacks += fb
        used = pm if fb else lm
        assert list(tr.get(oracle.LV_MATCH, l)) == used
        gam = tr.get(oracle.LV_GAMMA, l)
        if any(used[v] != v for v in range(L.n)):
            gamma, _ = brute.contract(L, used)
            assert list(gam) == gamma
    assert res["n_fallback"] == fallbacks
    parts = [int(x) for x in parts]
    n_parts = res["n_parts"]
    assert sorted(set(parts)) == list(range(n_parts))
    assert brute.part_valid_all(L0, parts, n_parts, omega, delta) == 0
    assert res["connectivity"] == brute.conn(L0, parts)
    return res


@pytest.mark.parametrize("seed", range(150))
def test_learned_steps_match_brute_force(seed):
    g, omega, delta, k, rounds, rng = _case(seed)
    mlp = random_int_mlp(seed, k=rng.choice([1, 2, 3, 8]))
    _check_learned(g, omega, delta, k, rounds, mlp)


def test_learned_fallback_is_exercised():
    # constant scores: every node takes its largest-id candidate; long chains
    # leave few 2-cycles and the plain matching must take over on some level
    total = 0
    for seed in range(60):
        g, omega, delta, k, rounds, _ = _case(1000 + seed)
        res = _check_learned(g, omega, delta, k, rounds, _zero_mlp(k=8))
        total += res["n_fallback"] if res else 0
    assert total > 0


@pytest.mark.parametrize("seed", range(80))
def test_identity_on_hist_reproduces_plain(seed):
    # unit hedge weights and at most 14 hedges keep hist <= 14, where the code
    # is strictly increasing: (score, id) then orders candidates as (hist, id)
    rng = random.Random(5000 + seed)
    n = rng.randint(2, 12)
    hedges, _, nw = brute.random_tiny(rng, n, rng.randint(1, 14), 5, wmax=1, node_wmax=rng.choice([1, 2]))
    g = from_lists(n, hedges, None, nw)
    omega, delta = rng.randint(2, 9), rng.randint(1, 7)
    rc_p, parts_p, res_p, _ = oracle.partition(g, omega, delta)
    rc_l, parts_l, res_l, _ = oracle.partition_learned(g, omega, delta, _identity_on(0, k=rng.choice([1, 3, 8])))
    assert rc_p == rc_l
    if rc_p == oracle.OK:
        assert list(parts_p) == list(parts_l)
        assert res_l["n_fallback"] == 0
        for key in ("connectivity", "n_parts", "n_levels", "n_rounds"):
            assert res_p[key] == res_l[key]


def test_learned_medium_random_network_valid():
    from paper_2604_14411_amd.synth import random_snn
    g = random_snn(600, 12.0, 7)
    L0 = brute.level_from_input(g)
    for seed in range(2):
        rc, parts, res, _ = oracle.partition_learned(g, 64, 96, random_int_mlp(seed))
        assert rc == oracle.OK
        assert brute.part_valid_all(L0, list(parts), res["n_parts"], 64, 96) == 0
        assert res["connectivity"] == oracle.connectivity(g, parts)
