"""Float64 reference of the learned proposal's float model (test infrastructure).

Written from the model's definition: inputs x = code / 8, two ReLU layers of
64 units, a linear output z, and the mean binary cross-entropy on logits
L = (1/n) sum softplus(z) - y z.  Gradients by the chain rule.  Used by the
tests to check the GPU training kernels and to state the error of the
integer network against the float model.
"""
from __future__ import annotations

import numpy as np


def forward(w: dict, xq):
    x = np.asarray(xq, dtype=np.float64) / 8.0
    pre1 = x @ np.asarray(w["w1"], np.float64) + np.asarray(w["b1"], np.float64)
    h1 = np.maximum(pre1, 0.0)
    pre2 = h1 @ np.asarray(w["w2"], np.float64) + np.asarray(w["b2"], np.float64)
    h2 = np.maximum(pre2, 0.0)
    z = h2 @ np.asarray(w["w3"], np.float64) + float(w["b3"])
    return dict(x=x, pre1=pre1, h1=h1, pre2=pre2, h2=h2, z=z)


def loss(w: dict, xq, y) -> float:
    z = forward(w, xq)["z"]
    y = np.asarray(y, np.float64)
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def grad(w: dict, xq, y):
    """(mean loss, gradient dict) by back-propagation."""
    f = forward(w, xq)
    y = np.asarray(y, np.float64)
    n = len(y)
    z = f["z"]
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n
    g = {}
    g["w3"] = f["h2"].T @ dz
    g["b3"] = float(dz.sum())
    d2 = np.outer(dz, np.asarray(w["w3"], np.float64)) * (f["pre2"] > 0)
    g["w2"] = f["h1"].T @ d2
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ np.asarray(w["w2"], np.float64).T) * (f["pre1"] > 0)
    g["w1"] = f["x"].T @ d1
    g["b1"] = d1.sum(axis=0)
    return float(np.mean(np.logaddexp(0.0, z) - y * z)), g
