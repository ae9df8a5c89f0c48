"""CPU checks of the learned proposal's float reference and quantiser.

* the float64 back-propagation of oracle/mlp_ref.py against central finite
  differences of its own forward loss, and closed-form special cases;
* the library's quantiser (host code, no GPU): the integer network it
  produces tracks the float model, score ~ z * 2^shift, within a bound that
  follows from the rounding of weights, biases and activations;
* plain oracle traces: the recorded candidate sets and codes against brute force.
"""
import os
import random

import numpy as np
import pytest

import brute
import oracle
from oracle import mlp_ref
from paper_2604_14411_amd.synth import feature_codes, from_lists

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _rand_w(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    w = dict(w1=rng.normal(0, scale, (16, 64)), b1=rng.normal(0, 0.1, 64), w2=rng.normal(0, scale, (64, 64)),
             b2=rng.normal(0, 0.1, 64), w3=rng.normal(0, scale, 64), b3=float(rng.normal()))
    w["w1"][10:] = 0
    return w


def test_backprop_matches_finite_differences():
    w = _rand_w(1)
    x = feature_codes(2, 40)
    y = (np.arange(40) % 3 == 0).astype(np.float64)
    L, g = mlp_ref.grad(w, x, y)
    assert abs(L - mlp_ref.loss(w, x, y)) < 1e-12
    rng = np.random.default_rng(3)
    h = 1e-6
    for name in ("w1", "b1", "w2", "b2", "w3", "b3"):
        for _ in range(6):
            wp = {k: (np.array(v, copy=True) if not np.isscalar(v) else v) for k, v in w.items()}
            wm = {k: (np.array(v, copy=True) if not np.isscalar(v) else v) for k, v in w.items()}
            if name == "b3":
                wp[name] = w[name] + h
                wm[name] = w[name] - h
                num = (mlp_ref.loss(wp, x, y) - mlp_ref.loss(wm, x, y)) / (2 * h)
                assert abs(num - g[name]) < 1e-6
                break
            idx = tuple(rng.integers(0, s) for s in np.shape(w[name]))
            if name == "w1":
                idx = (int(rng.integers(0, 10)), idx[1])
            wp[name][idx] += h
            wm[name][idx] -= h
            num = (mlp_ref.loss(wp, x, y) - mlp_ref.loss(wm, x, y)) / (2 * h)
            assert abs(num - g[name][idx]) < 1e-6, (name, idx, num, g[name][idx])


def test_zero_network_loss_closed_form():
    w = dict(w1=np.zeros((16, 64)), b1=np.zeros(64), w2=np.zeros((64, 64)), b2=np.zeros(64), w3=np.zeros(64),
             b3=0.7)
    x = feature_codes(4, 25)
    y = (np.arange(25) % 2).astype(np.float64)
    L, g = mlp_ref.grad(w, x, y)
    assert abs(L - (np.log1p(np.exp(0.7)) - y.mean() * 0.7)) < 1e-12
    assert abs(g["b3"] - (1 / (1 + np.exp(-0.7)) - y.mean())) < 1e-12
    assert not np.any(g["w1"]) and not np.any(g["w2"])


def _lib_or_skip():
    from paper_2604_14411_amd import hgp

    if not os.path.exists(hgp.LIB_PATH):
        pytest.skip("libhgp.so not built")
    return hgp


def test_quantized_network_tracks_float_model():
    hgp = _lib_or_skip()
    w = _rand_w(5, 0.2)
    x = feature_codes(6, 4000)
    q, shift = hgp.mlp_quantize(w, x[:2000], k=8)
    for key in ("w1", "w2", "w3"):
        assert np.abs(q[key]).max() <= 255
    z = mlp_ref.forward(w, x)["z"]
    s = oracle.mlp_score(q, x).astype(np.float64) / 2.0 ** shift
    err = np.abs(s - z)
    spread = z.max() - z.min()
    # weight steps 2^-s (<= max|w| / 128) and activation steps 2^-t propagate
    # through two layers: a few percent of the output's range
    assert np.max(err) < 0.05 * spread, (np.max(err), spread)
    # the ranking the selection uses is preserved for pairs not within the error
    i, j = np.triu_indices(200, 1)
    zi, zj, si, sj = z[i], z[j], s[i], s[j]
    clear = np.abs(zi - zj) > 2 * np.max(err)
    assert np.all(np.sign(zi - zj)[clear] == np.sign(si - sj)[clear])


def test_quantizer_rejects_bad_inputs():
    hgp = _lib_or_skip()
    w = _rand_w(7)
    with pytest.raises(hgp.HgpError):
        hgp.mlp_quantize(w, np.full((2, 16), 300, np.int32), k=8)
    with pytest.raises(hgp.HgpError):
        hgp.mlp_quantize(w, feature_codes(1, 4), k=0)


@pytest.mark.parametrize("seed", range(40))
def test_plain_trace_candidates_match_brute(seed):
    rng = random.Random(700 + seed)
    n = rng.randint(2, 12)
    hedges, w, nw = brute.random_tiny(rng, n, rng.randint(1, 10), 5, wmax=5, node_wmax=rng.choice([1, 3]))
    g = from_lists(n, hedges, w, nw)
    omega, delta = rng.randint(2, 9), rng.randint(1, 7)
    rc, parts, res, tr = oracle.partition(g, omega, delta, trace=True)
    if rc != oracle.OK:
        return
    wl = [int(v) for v in g.hedge_w]
    for l in range(tr.levels):
        L = brute.level_from_trace(tr.get(oracle.LV_HOFF, l), tr.get(oracle.LV_HPIN, l), tr.get(oracle.LV_SIZE, l),
                                   wl)
        _, C = brute.candidates(L, omega, delta, 8)
        coff = tr.get(oracle.LV_COFF, l)
        cand = tr.get(oracle.LV_CAND, l)
        feat = tr.get(oracle.LV_FEAT, l).reshape(-1, 16)
        for v in range(L.n):
            ids = [int(t) for t in cand[coff[v]:coff[v + 1]]]
            assert ids == sorted(C[v])
            for j, m in enumerate(ids):
                h, c = C[v][m]
                assert list(feat[coff[v] + j]) == brute.pair_features(L, l, omega, delta, v, m, h, c)


def test_trained_checkpoint_score_error_on_held_out_rows():
    """The committed network (mlp_v2.json): its integer scores against its own
    float weights (float64 forward of oracle/mlp_ref.py) on candidate rows of
    a held-out layered network (8 x (16x10x10), 5x5 window, seed 302; no
    training graph has this shape or seed), every level's candidates as the
    plain oracle records them."""
    from paper_2604_14411_amd import synth
    from paper_2604_14411_amd.learn import load_checkpoint

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    q, w, ck = load_checkpoint(os.path.join(root, "paper_2604_14411_amd", "mlp_v2.json"))
    g = synth.layered_conv(8, 16, 10, 10, 5, 0.1, 302)
    rc, _, _, tr = oracle.partition(g, 4096, 65536, trace=True)
    assert rc == 0
    rows = [tr.get(oracle.LV_FEAT, l).reshape(-1, 16) for l in range(0, tr.levels, 25)]
    x = np.concatenate(rows)
    x = np.unique(x, axis=0)
    assert len(x) > 1000
    z = mlp_ref.forward(w, x)["z"]
    s = oracle.mlp_score(q, x).astype(np.float64) / 2.0 ** ck["score_shift"]
    err = np.abs(s - z)
    spread = z.max() - z.min()
    print(f"held-out rows {len(x)}: max |int - float| {err.max():.4f} (mean {err.mean():.4f}), "
          f"float score range {spread:.3f}, relative {err.max() / spread:.4f}")
    rng = np.random.default_rng(3)
    i = rng.integers(0, len(x), 20000)
    j = rng.integers(0, len(x), 20000)
    differ = z[i] != z[j]
    agree = np.mean(np.sign(z[i] - z[j])[differ] == np.sign(s[i] - s[j])[differ])
    print(f"pairs ordered alike by the integer and float scores: {agree:.4f}")
    # measured: max error 7.9% of the float range, mean 1.1%; 97.3% of pairs ordered alike
    assert err.max() < 0.09 * spread and err.mean() < 0.02 * spread
    assert agree > 0.97
    clear = np.abs(z[i] - z[j]) > 2 * err.max()
    assert np.all(np.sign(z[i] - z[j])[clear] == np.sign(s[i] - s[j])[clear])
