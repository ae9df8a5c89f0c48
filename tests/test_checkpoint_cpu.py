"""The committed network checkpoint is a valid integer network (CPU only)."""
import os

import numpy as np

from paper_2604_14411_amd.learn import load_checkpoint

HERE = os.path.dirname(os.path.abspath(__file__))


def test_checkpoint_is_a_valid_integer_network():
    q, w, ck = load_checkpoint(os.path.join(HERE, "..", "paper_2604_14411_amd", "mlp_v2.json"))
    assert ck["format"] == "hgp-mlp-1" and 1 <= q["k"] <= 8
    for key in ("w1", "w2", "w3"):
        assert np.abs(q[key]).max() <= 255
    for key in ("b1", "b2"):
        assert np.abs(q[key]).max() <= 2 ** 22
    assert abs(q["b3"]) <= 2 ** 22 and 0 <= q["r1"] <= 30 and 0 <= q["r2"] <= 30
    assert np.all(q["w1"][10:] == 0)
    # the training record names graphs that are not evaluation instances
    names = [g["graph"] for g in ck["train"]["graphs"]]
    assert names and all("8x(96x16x17)" not in n and "8x(42x30x30)" not in n for n in names)
    assert ck["train"]["loss"][-1] < ck["train"]["loss"][0]
