"""Seeded synthetic spiking-network hypergraphs (input generation only).

The generators live in ``synth.c`` (built to ``libhgpsynth.so``); this module
wraps them with ctypes and returns plain numpy arrays.  They hold none of the
partitioner's arithmetic: the GPU library and the CPU oracle both consume the
bytes produced here.

A hypergraph is returned as a :class:`Hypergraph` with int32 arrays in the
CSR layout of the C-ABI: ``hedge_off[E+1]``, ``pins[P]`` (source pins first),
``n_src[E]``, ``hedge_w[E]``, ``node_w[N]``.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgpsynth.so")


class _SynthGraph(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int32),
        ("n_hedges", ctypes.c_int32),
        ("n_pins", ctypes.c_int64),
        ("hedge_off", ctypes.POINTER(ctypes.c_int32)),
        ("pins", ctypes.POINTER(ctypes.c_int32)),
        ("n_src", ctypes.POINTER(ctypes.c_int32)),
        ("hedge_w", ctypes.POINTER(ctypes.c_int32)),
        ("node_w", ctypes.POINTER(ctypes.c_int32)),
    ]


_lib = None


def build(force: bool = True) -> str:
    """Compile libhgpsynth.so with gcc (host code only)."""
    import subprocess

    src = os.path.join(_HERE, "synth.c")
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(_SynthGraph)
        lib.synth_random_snn.restype = P
        lib.synth_random_snn.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32,
                                         ctypes.c_int32]
        lib.synth_layered_conv.restype = P
        lib.synth_layered_conv.argtypes = [ctypes.c_int32] * 5 + [ctypes.c_double, ctypes.c_uint64]
        lib.synth_random_snn_family.restype = P
        lib.synth_random_snn_family.argtypes = [ctypes.c_uint64] + [ctypes.c_double] * 4 + [
            ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
        lib.synth_free.restype = None
        lib.synth_free.argtypes = [P]
        _lib = lib
    return _lib


@dataclass
class Hypergraph:
    """Directed weighted hypergraph in int32 CSR form (Sec. II-A, II-C)."""

    hedge_off: np.ndarray  # int32 [E+1]
    pins: np.ndarray  # int32 [P], source pins first within each hedge
    n_src: np.ndarray  # int32 [E]
    hedge_w: np.ndarray  # int32 [E]
    node_w: np.ndarray  # int32 [N]

    @property
    def n_nodes(self) -> int:
        return int(self.node_w.shape[0])

    @property
    def n_hedges(self) -> int:
        return int(self.hedge_off.shape[0] - 1)

    @property
    def n_pins(self) -> int:
        return int(self.hedge_off[-1]) if self.hedge_off.shape[0] else 0

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.hedge_off, self.pins, self.n_src, self.hedge_w, self.node_w):
            h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
        return h.hexdigest()

    def sum_sq(self) -> int:
        """Q = sum over hedges of |e|^2 (pin-pair visits of one rating pass)."""
        sz = np.diff(self.hedge_off.astype(np.int64))
        return int((sz * sz).sum())


def _take(gp) -> Hypergraph:
    lib = _load()
    if not gp:
        raise ValueError("synth: invalid generator arguments or out of memory")
    g = gp.contents
    n, e, p = g.n_nodes, g.n_hedges, g.n_pins

    def arr(ptr, k):
        if k == 0:
            return np.zeros(0, dtype=np.int32)
        return np.ctypeslib.as_array(ptr, shape=(k,)).copy()

    out = Hypergraph(arr(g.hedge_off, e + 1), arr(g.pins, p), arr(g.n_src, e), arr(g.hedge_w, e),
                     arr(g.node_w, n))
    lib.synth_free(gp)
    return out


def random_snn(n: int, mu: float, seed: int, wmin: int = 1, wmax: int = 16) -> Hypergraph:
    """Random SNN: each v owns {v} + T_v, |T_v| = min(Poisson(mu)+1, n-1)."""
    return _take(_load().synth_random_snn(n, mu, seed, wmin, wmax))


def layered_conv(layers: int, C: int, H: int, W: int, k: int, p_geo: float, seed: int) -> Hypergraph:
    """Layered conv-like SNN with k x k windows across all channels."""
    return _take(_load().synth_layered_conv(layers, C, H, W, k, p_geo, seed))


def random_snn_family(seed: int, log2_lo: float = 11.0, log2_hi: float = 15.0, mu_lo: float = 32.0,
                      mu_hi: float = 256.0, wmin: int = 1, wmax: int = 16):
    """One member of the log-uniform random-SNN family; returns (graph, n, mu)."""
    n = ctypes.c_int32()
    mu = ctypes.c_double()
    g = _take(_load().synth_random_snn_family(seed, log2_lo, log2_hi, mu_lo, mu_hi, wmin, wmax,
                                              ctypes.byref(n), ctypes.byref(mu)))
    return g, n.value, mu.value


def from_lists(n_nodes: int, hedges, hedge_w=None, node_w=None) -> Hypergraph:
    """Build a Hypergraph from python lists: hedges = [(src_list, dst_list), ...]."""
    off = [0]
    pins, nsrc = [], []
    for src, dst in hedges:
        pins.extend(int(x) for x in src)
        pins.extend(int(x) for x in dst)
        nsrc.append(len(src))
        off.append(len(pins))
    e = len(hedges)
    hw = np.ones(e, dtype=np.int32) if hedge_w is None else np.asarray(hedge_w, dtype=np.int32)
    nw = np.ones(n_nodes, dtype=np.int32) if node_w is None else np.asarray(node_w, dtype=np.int32)
    return Hypergraph(np.asarray(off, dtype=np.int32), np.asarray(pins, dtype=np.int32),
                      np.asarray(nsrc, dtype=np.int32), hw, nw)


def random_int_mlp(seed: int, k: int = 8, r1: int = 7, r2: int = 9, wmax: int = 255, bmax: int = 4096) -> dict:
    """Seeded random integer network for the learned merge proposal (test input):
    weights uniform in [-wmax, wmax], biases in [-bmax, bmax], codes 10..15 of
    the first layer zero (padding inputs)."""
    rng = np.random.default_rng(seed)
    w1 = rng.integers(-wmax, wmax + 1, size=(16, 64), dtype=np.int64)
    w1[10:, :] = 0
    return dict(k=int(k), r1=int(r1), r2=int(r2), b3=int(rng.integers(-bmax, bmax + 1)),
                w1=w1.astype(np.int32),
                b1=rng.integers(-bmax, bmax + 1, size=64).astype(np.int32),
                w2=rng.integers(-wmax, wmax + 1, size=(64, 64)).astype(np.int32),
                b2=rng.integers(-bmax, bmax + 1, size=64).astype(np.int32),
                w3=rng.integers(-wmax, wmax + 1, size=64).astype(np.int32))


def feature_codes(seed: int, n: int) -> np.ndarray:
    """Seeded rows of 16 input codes in 0..255 (first 10 random, rest zero)."""
    rng = np.random.default_rng(seed)
    x = np.zeros((n, 16), dtype=np.int32)
    x[:, :10] = rng.integers(0, 256, size=(n, 10))
    return x


def with_node_weights(g: Hypergraph, seed: int, wmax: int) -> Hypergraph:
    """The same hypergraph with seeded node weights uniform in [1, wmax]."""
    rng = np.random.default_rng(seed)
    nw = rng.integers(1, wmax + 1, size=g.n_nodes).astype(np.int32)
    return Hypergraph(g.hedge_off.copy(), g.pins.copy(), g.n_src.copy(), g.hedge_w.copy(), nw)
