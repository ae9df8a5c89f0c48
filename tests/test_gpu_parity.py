"""GPU path vs CPU oracle, end to end and step by step (through the C-ABI).

Integer method: every comparison is exact.
"""
import hashlib
import json
import os
import random
import sys

import numpy as np
import pytest

import badinputs
import brute
import oracle
from paper_2604_14411_amd import synth
from paper_2604_14411_amd.synth import from_lists

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

HERE = os.path.dirname(os.path.abspath(__file__))


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


def _gpu_partition(ctx, g, omega, delta, k=0, rounds=8, flags=0, role=0):
    from paper_2604_14411_amd import hgp

    dg = hgp.DeviceHypergraph(g, "cuda:0")
    try:
        parts, res = hgp.partition_device(ctx, dg, omega, delta, k=k, max_refine_rounds=rounds, flags=flags,
                                          constraint=role)
        return 0, parts.cpu().numpy(), res
    except hgp.HgpError as e:
        return e.code, None, None


def _compare(ctx, g, omega, delta, k=0, rounds=8, label="", role=0):
    say(f"[parity] {label} n={g.n_nodes} E={g.n_hedges} P={g.n_pins} omega={omega} delta={delta} k={k} R={rounds} "
        f"role={role}")
    rc, ref, rres, _ = oracle.partition(g, omega, delta, k=k, max_rounds=rounds, role=role)
    grc, got, gres = _gpu_partition(ctx, g, omega, delta, k, rounds, role=role)
    assert grc == rc, (grc, rc)
    if rc != 0:
        return
    assert np.array_equal(got, ref), "part ids differ"
    for key in ("connectivity", "n_parts", "n_levels", "n_rounds"):
        assert gres[key] == rres[key], (key, gres[key], rres[key])


def _tiny(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 14)
    hedges, w, nw = brute.random_tiny(rng, n, rng.randint(0, 12), 6, wmax=6, node_wmax=rng.choice([1, 1, 3]))
    return from_lists(n, hedges, w, nw), rng.randint(1, 9), rng.randint(0, 8), rng.choice([0, 0, 1, 3]), \
        rng.choice([0, 1, 8])


@pytest.mark.parametrize("seed", range(120))
def test_tiny_random_end_to_end(ctx, seed):
    g, omega, delta, k, rounds = _tiny(seed)
    _compare(ctx, g, omega, delta, k, rounds, label=f"tiny seed={seed}")


@pytest.mark.parametrize("role", [1, 2])
@pytest.mark.parametrize("seed", range(40))
def test_tiny_constraint_variants_end_to_end(ctx, seed, role):
    g, omega, delta, k, rounds = _tiny(300 + seed)
    _compare(ctx, g, omega, delta, k, rounds, label=f"tiny seed={300 + seed}", role=role)


@pytest.mark.parametrize("role", [1, 2])
def test_medium_constraint_variants_end_to_end(ctx, role):
    _compare(ctx, synth.random_snn(2000, 24.0, 111), 64, 40 if role == 1 else 400, label="rand2000", role=role)
    _compare(ctx, synth.layered_conv(4, 6, 8, 8, 3, 0.1, 112), 64, 300, label="conv", role=role)


MEDIUM = [
    ("rand300", lambda: synth.random_snn(300, 9.0, 101), 12, 60),
    ("rand1500", lambda: synth.random_snn(1500, 24.0, 102), 64, 200),
    ("rand4000", lambda: synth.random_snn(4000, 40.0, 103), 128, 600),
    ("rand3000_tightD", lambda: synth.random_snn(3000, 30.0, 104), 1024, 120),
    ("conv_small", lambda: synth.layered_conv(4, 6, 8, 8, 3, 0.1, 105), 64, 2000),
    ("conv_wide", lambda: synth.layered_conv(5, 4, 10, 9, 5, 0.2, 106), 96, 500),
]


@pytest.mark.parametrize("name,make,omega,delta", MEDIUM, ids=[m[0] for m in MEDIUM])
def test_medium_end_to_end(ctx, name, make, omega, delta):
    _compare(ctx, make(), omega, delta, label=name)


INCR = [
    ("rand2500_tail", lambda: synth.random_snn(2500, 30.0, 31), 1024, 400),
    ("rand6000_tail", lambda: synth.random_snn(6000, 60.0, 32), 1024, 1500),
    ("rand3000_omega", lambda: synth.random_snn(3000, 20.0, 33), 48, 100000),
    ("conv_tail", lambda: synth.layered_conv(6, 8, 8, 8, 3, 0.1, 34), 256, 3000),
]


@pytest.mark.parametrize("name,make,omega,delta", INCR + MEDIUM[4:], ids=[c[0] for c in INCR + MEDIUM[4:]])
def test_grouped_ratings_match_oracle(ctx, monkeypatch, name, make, omega, delta):
    """Every top-K rating grouped by inbound hedge set (HGP_GROUP_MIN=1 and HGP_GROUP_LISTS=1; by
    default only levels of 16384 nodes or more): id-by-id equal to the oracle."""
    monkeypatch.setenv("HGP_GROUP_MIN", "1")
    monkeypatch.setenv("HGP_GROUP_LISTS", "1")
    _compare(ctx, make(), omega, delta, label=f"{name} grouped")


@pytest.mark.parametrize("name,make,omega,delta", INCR, ids=[c[0] for c in INCR])
def test_incremental_late_levels_match_full_recompute(ctx, name, make, omega, delta):
    from paper_2604_14411_amd import hgp

    g = make()
    say(f"[incremental] {name} full recompute")
    rc1, p1, r1 = _gpu_partition(ctx, g, omega, delta, flags=hgp.FLAG_NO_INCREMENTAL)
    say(f"[incremental] {name} incremental")
    rc2, p2, r2 = _gpu_partition(ctx, g, omega, delta)
    assert rc1 == rc2 == 0
    assert np.array_equal(p1, p2)
    for key in ("connectivity", "n_parts", "n_levels", "n_rounds"):
        assert r1[key] == r2[key], key
    say(f"[incremental] {name} oracle")
    rc, ref, rres, _ = oracle.partition(g, omega, delta)
    assert rc == 0 and np.array_equal(p2, ref) and rres["connectivity"] == r2["connectivity"]


def test_host_entry_matches_device_entry(ctx):
    from paper_2604_14411_amd import hgp

    g = synth.random_snn(2000, 20.0, 7)
    say("[parity] host entry rand2000")
    p1, r1 = hgp.partition_host(ctx, g, 64, 300)
    rc, p2, r2 = _gpu_partition(ctx, g, 64, 300)
    assert rc == 0 and np.array_equal(p1, p2) and r1["connectivity"] == r2["connectivity"]


def test_repeat_runs_identical(ctx):
    g = synth.random_snn(2500, 30.0, 8)
    outs = []
    for i in range(3):
        say(f"[determinism] run {i}")
        rc, p, r = _gpu_partition(ctx, g, 80, 400)
        assert rc == 0
        outs.append((p.tobytes(), r["connectivity"]))
    assert outs[0] == outs[1] == outs[2]


def test_seed_does_not_change_plain_result(ctx):
    from paper_2604_14411_amd import hgp

    g = synth.random_snn(1200, 16.0, 9)
    dg = hgp.DeviceHypergraph(g, "cuda:0")
    say("[seed] two seeds")
    import ctypes

    outs = []
    for seed in (1, 987654321):
        o, _ = hgp.options(0, 8, seed)
        import torch

        out = torch.empty(g.n_nodes, dtype=torch.int32, device="cuda:0")
        res = hgp.Result_t()
        hgp._check(hgp.load().hgp_partition_device(ctx.handle, ctypes.byref(dg.struct()), 64, 256, ctypes.byref(o),
                                                   hgp._stream(), out.data_ptr(), ctypes.byref(res)))
        outs.append(out.cpu().numpy().tobytes())
    assert outs[0] == outs[1]


# --------------------------------------------------------------- step parity
def _t(a, dt=None):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a) if dt is None else np.ascontiguousarray(a, dtype=dt)).to("cuda:0")


STEP_CASES = [
    ("rand1200", lambda: synth.random_snn(1200, 16.0, 21), 48, 220),
    ("conv", lambda: synth.layered_conv(4, 5, 7, 7, 3, 0.1, 22), 40, 900),
]


@pytest.mark.parametrize("name,make,omega,delta", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_each_step_matches_oracle_trace(ctx, name, make, omega, delta):
    from paper_2604_14411_amd import hgp

    g = make()
    rc, parts, res, tr = oracle.partition(g, omega, delta, trace=True)
    assert rc == 0
    hw = _t(g.hedge_w, np.int32)
    # canonical level 0
    say(f"[steps] {name} canonical")
    dg = hgp.DeviceHypergraph(g, "cuda:0")
    hoff0, hpin0 = hgp.level_canonical(ctx, dg, omega, delta)
    assert np.array_equal(hoff0.cpu().numpy(), tr.get(oracle.LV_HOFF, 0).astype(np.int32))
    assert np.array_equal(hpin0.cpu().numpy(), tr.get(oracle.LV_HPIN, 0))
    for l in range(tr.levels):
        hoff = _t(tr.get(oracle.LV_HOFF, l), np.int32)
        hpin = _t(tr.get(oracle.LV_HPIN, l), np.int32)
        size = _t(tr.get(oracle.LV_SIZE, l), np.int32)
        n = size.numel()
        say(f"[steps] {name} level {l} rate n={n}")
        pair, score = hgp.level_rate(ctx, n, hoff, hpin, size, hw, omega, delta)
        assert np.array_equal(pair.cpu().numpy(), tr.get(oracle.LV_PAIR, l)), f"pair level {l}"
        assert np.array_equal(score.cpu().numpy(), tr.get(oracle.LV_SCORE, l)), f"score level {l}"
        say(f"[steps] {name} level {l} match")
        match, gamma, n_next = hgp.level_match(ctx, pair, score)
        assert np.array_equal(match.cpu().numpy(), tr.get(oracle.LV_MATCH, l)), f"match level {l}"
        gam = tr.get(oracle.LV_GAMMA, l)
        if gam is not None:
            assert np.array_equal(gamma.cpu().numpy(), gam)
        if l + 1 < tr.levels:
            say(f"[steps] {name} level {l} contract")
            h2, p2, s2 = hgp.level_contract(ctx, n, hoff, hpin, size, hw, gamma, n_next)
            assert np.array_equal(h2.cpu().numpy(), tr.get(oracle.LV_HOFF, l + 1).astype(np.int32))
            assert np.array_equal(p2.cpu().numpy(), tr.get(oracle.LV_HPIN, l + 1))
            assert np.array_equal(s2.cpu().numpy(), tr.get(oracle.LV_SIZE, l + 1).astype(np.int32))
    for r in range(tr.rounds):
        info = [int(x) for x in tr.get(oracle.RD_INFO, r)]
        l, S, istar, gstar, applied, n_parts = info
        hoff = _t(tr.get(oracle.LV_HOFF, l), np.int32)
        hpin = _t(tr.get(oracle.LV_HPIN, l), np.int32)
        size = _t(tr.get(oracle.LV_SIZE, l), np.int32)
        rho = _t(tr.get(oracle.RD_RHO, r), np.int32)
        say(f"[steps] {name} round {r} level {l} S={S}")
        out = hgp.level_refine_round(ctx, size.numel(), hoff, hpin, size, hw, rho, n_parts, omega, delta)
        assert np.array_equal(out["dest"].cpu().numpy(), tr.get(oracle.RD_PDEST, r)), f"dest round {r}"
        assert np.array_equal(out["gain"].cpu().numpy(), tr.get(oracle.RD_PGAIN, r)), f"gain round {r}"
        assert out["S"] == S
        assert np.array_equal(out["seq"].cpu().numpy(), tr.get(oracle.RD_SEQ, r)), f"seq round {r}"
        assert np.array_equal(out["G"].cpu().numpy(), tr.get(oracle.RD_G, r)), f"G round {r}"
        assert np.array_equal(out["viol"].cpu().numpy(), tr.get(oracle.RD_VIOL, r)), f"viol round {r}"
        assert out["istar"] == istar and out["gstar"] == gstar and out["applied"] == bool(applied)
        rho_after = tr.get(oracle.RD_RHO, r + 1) if r + 1 < tr.rounds and \
            int(tr.get(oracle.RD_INFO, r + 1)[0]) == l else None
        if rho_after is not None:
            assert np.array_equal(out["rho"].cpu().numpy(), rho_after)


# --------------------------------------------------------------- errors
@pytest.mark.parametrize("case", badinputs.cases(), ids=[c[0] for c in badinputs.cases()])
def test_error_codes(ctx, case):
    """The library rejects malformed and infeasible inputs with the oracle's codes."""
    name, g, omega, delta, want = case
    say(f"[errors] {name}")
    rc, _, _ = _gpu_partition(ctx, g, omega, delta)
    assert rc == want, (name, rc, want)
    orc, _, _, _ = oracle.partition(g, omega, delta)
    assert orc == want


def test_empty_inputs(ctx):
    say("[empty]")
    for n, hedges in [(0, []), (3, []), (3, [([], [])]), (5, [([0], []), ([1], [2])])]:
        g = from_lists(n, hedges)
        _compare(ctx, g, 2, 2, label=f"empty n={n} E={len(hedges)}")


# --------------------------------------------------------------- full-size
def test_rand16k_matches_oracle_golden(ctx):
    path = os.path.join(HERE, "golden", "rand16k.json")
    if not os.path.exists(path):
        pytest.skip("golden not generated")
    gold = json.load(open(path))
    from paper_2604_14411_amd.synth.configs import WORKLOADS

    w = WORKLOADS["rand16k"]
    g = w.make()
    assert g.digest() == gold["input_sha256"]
    say("[golden] rand16k")
    rc, parts, res = _gpu_partition(ctx, g, w.omega, w.delta)
    assert rc == 0
    assert hashlib.sha256(np.ascontiguousarray(parts, dtype="<i4").tobytes()).hexdigest() == gold["parts_sha256"]
    assert res["connectivity"] == gold["connectivity"]
    assert res["n_parts"] == gold["n_parts"] and res["n_levels"] == gold["n_levels"]
    assert res["n_rounds"] == gold["n_rounds"]


def _with_big_hedges(n, mu, n_big, big_len, seed):
    """Random SNN plus a few hub hedges longer than one wave's sort capacity."""
    import random as _r

    g = synth.random_snn(n, mu, seed)
    rng = _r.Random(seed)
    hedges = []
    for e in range(g.n_hedges):
        b, en, ns = int(g.hedge_off[e]), int(g.hedge_off[e + 1]), int(g.n_src[e])
        pins = [int(x) for x in g.pins[b:en]]
        hedges.append((pins[:ns], pins[ns:]))
    w = [int(x) for x in g.hedge_w]
    for _ in range(n_big):
        pins = rng.sample(range(n), big_len)
        hedges.append((pins[:1], pins[1:]))
        w.append(rng.randint(1, 16))
    return from_lists(n, hedges, w)


def test_hedges_longer_than_a_wave(ctx):
    g = _with_big_hedges(2500, 20.0, 6, 1500, 41)
    _compare(ctx, g, 64, 2000, label="big hedges")
    from paper_2604_14411_amd import hgp

    # one hedge just past the LDS kernels' capacity (4096 pins), and the
    # supported maximum (32767 pins) exceeded by one
    base = synth.random_snn(5000, 10.0, 5)
    hedges = []
    for e in range(base.n_hedges):
        b, en, ns = int(base.hedge_off[e]), int(base.hedge_off[e + 1]), int(base.n_src[e])
        pins = [int(x) for x in base.pins[b:en]]
        hedges.append((pins[:ns], pins[ns:]))
    hedges.append(([0], list(range(1, 4098))))
    g = from_lists(5000, hedges, [int(x) for x in base.hedge_w] + [7])
    _compare(ctx, g, 64, 4500, label="4097-pin hedge")
    too_big = from_lists(33000, [([0], list(range(1, 32768)))])
    rc, _, _ = _gpu_partition(ctx, too_big, 64, 4000)
    assert rc == hgp.EUNSUPPORTED


def test_hedges_of_ten_thousand_pins(ctx):
    """Hub hedges of 10,000 pins (above the LDS kernels' 4096): ingest,
    contraction, part tables and in-sequence events run in global scratch.
    The oracle's trace shows rounds where more than 256 pins of such a hedge
    move (the workgroup event path for long hedges)."""
    g = _with_big_hedges(12000, 12.0, 3, 10000, 77)
    rc, ref, rres, tr = oracle.partition(g, 256, 20000, trace=True)
    assert rc == 0
    heavy = 0
    first_hub = g.n_hedges - 3
    for r in range(tr.rounds):
        info = tr.get(oracle.RD_INFO, r)
        lv, S = int(info[0]), int(info[1])
        if S == 0:
            continue
        hoff = tr.get(oracle.LV_HOFF, lv)
        hpin = tr.get(oracle.LV_HPIN, lv) & 0x7FFFFFFF
        moving = np.zeros(len(tr.get(oracle.LV_SIZE, lv)), bool)
        moving[tr.get(oracle.RD_SEQ, r)] = True
        for e in range(first_hub, g.n_hedges):
            pins = hpin[hoff[e]:hoff[e + 1]]
            if len(pins) > 4096 and moving[pins].sum() > 256:
                heavy += 1
    say(f"[parity] 10k-pin hubs: {heavy} rounds x hubs with more than 256 moving pins")
    assert heavy > 0
    grc, got, gres = _gpu_partition(ctx, g, 256, 20000)
    assert grc == 0
    assert np.array_equal(got, ref), "part ids differ"
    for key in ("connectivity", "n_parts", "n_levels", "n_rounds"):
        assert gres[key] == rres[key], (key, gres[key], rres[key])


def test_connectivity_entry_point(ctx):
    from paper_2604_14411_amd import hgp

    g = _with_big_hedges(1500, 15.0, 2, 1200, 43)
    dg = hgp.DeviceHypergraph(g, "cuda:0")
    rng = np.random.default_rng(5)
    import torch

    for k in (1, 7, 300, g.n_nodes):
        part = rng.integers(0, k, size=g.n_nodes).astype(np.int32)
        say(f"[connectivity] k={k}")
        got = hgp.connectivity_device(ctx, dg, torch.as_tensor(part).to("cuda:0"))
        assert got == oracle.connectivity(g, part)


def test_rand64k_matches_oracle_golden(ctx):
    """The benchmark workload at full size: part ids and statistics bit-exact."""
    path = os.path.join(HERE, "golden", "rand64k.json")
    if not os.path.exists(path):
        pytest.skip("golden not generated")
    gold = json.load(open(path))
    from paper_2604_14411_amd.synth.configs import WORKLOADS

    w = WORKLOADS["rand64k"]
    g = w.make()
    assert g.digest() == gold["input_sha256"]
    say("[golden] rand64k")
    rc, parts, res = _gpu_partition(ctx, g, w.omega, w.delta)
    assert rc == 0
    assert hashlib.sha256(np.ascontiguousarray(parts, dtype="<i4").tobytes()).hexdigest() == gold["parts_sha256"]
    assert res["connectivity"] == gold["connectivity"]
    assert res["n_parts"] == gold["n_parts"] and res["n_levels"] == gold["n_levels"]
    assert res["n_rounds"] == gold["n_rounds"]
