"""CPU oracle for the constrained multilevel partitioner (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg use this package; the GPU library never calls it.  ``hgpo.cpp`` is a
plain sequential restatement of the paper's method (see its header); this
module builds it with g++ and exposes it through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgpo.so")

OK, EINVAL, EBADCSR, EINFEASIBLE, ENOMEM, EUNSUPPORTED = 0, -1, -2, -3, -4, -6

(LV_HOFF, LV_HPIN, LV_SIZE, LV_PAIR, LV_SCORE, LV_MATCH, LV_GAMMA, LV_RHO0, LV_RHO1, LV_COFF, LV_CAND, LV_CSCORE,
 LV_FEAT, LV_PPAIR, LV_FALLBACK) = range(15)
MLP_F, MLP_H, MLP_NFEAT = 16, 64, 10
(RD_INFO, RD_RHO, RD_PDEST, RD_PGAIN, RD_SEQ, RD_GP, RD_G, RD_VIOL, RD_PTOFF, RD_PT, RD_PSIZE,
 RD_PINB) = range(20, 32)


class _HG(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_hedges", ctypes.c_int32),
                ("hedge_off", ctypes.c_void_p), ("pins", ctypes.c_void_p), ("n_src", ctypes.c_void_p),
                ("hedge_w", ctypes.c_void_p), ("node_w", ctypes.c_void_p)]


class _Res(ctypes.Structure):
    _fields_ = [("connectivity", ctypes.c_int64), ("n_parts", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("n_rounds", ctypes.c_int32), ("n_fallback", ctypes.c_int32)]


class _MLP(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("r1", ctypes.c_int32), ("r2", ctypes.c_int32), ("b3", ctypes.c_int32),
                ("w1", ctypes.c_int32 * (MLP_F * MLP_H)), ("b1", ctypes.c_int32 * MLP_H),
                ("w2", ctypes.c_int32 * (MLP_H * MLP_H)), ("b2", ctypes.c_int32 * MLP_H),
                ("w3", ctypes.c_int32 * MLP_H)]


def _mlp(q) -> _MLP:
    """Packs an integer network given as a dict (k, r1, r2, b3, w1[16,64], b1[64], w2[64,64], b2[64], w3[64])."""
    m = _MLP()
    m.k, m.r1, m.r2, m.b3 = int(q["k"]), int(q["r1"]), int(q["r2"]), int(q["b3"])
    for name, n in (("w1", MLP_F * MLP_H), ("b1", MLP_H), ("w2", MLP_H * MLP_H), ("b2", MLP_H), ("w3", MLP_H)):
        a = np.ascontiguousarray(np.asarray(q[name]).reshape(-1), dtype=np.int32)
        assert a.size == n, name
        ctypes.memmove(getattr(m, name), a.ctypes.data, 4 * n)
    return m


_lib = None


def build(force: bool = True) -> str:
    """Compile libhgpo.so (g++ -O3, OpenMP over independent per-node loops)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                               os.path.join(_HERE, "hgpo.cpp")])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        lib.hgpo_partition.restype = ctypes.c_int
        lib.hgpo_partition.argtypes = [ctypes.POINTER(_HG), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(_Res), ctypes.c_void_p]
        lib.hgpo_partition_role.restype = ctypes.c_int
        lib.hgpo_partition_role.argtypes = [ctypes.POINTER(_HG), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(_Res),
                                            ctypes.c_void_p]
        lib.hgpo_partition_ex.restype = ctypes.c_int
        lib.hgpo_partition_ex.argtypes = [ctypes.POINTER(_HG), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.POINTER(_Res), ctypes.c_void_p]
        lib.hgpo_match.restype = ctypes.c_int
        lib.hgpo_match.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        lib.hgpo_partition_learned.restype = ctypes.c_int
        lib.hgpo_partition_learned.argtypes = [ctypes.POINTER(_HG), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.POINTER(_MLP), ctypes.c_void_p,
                                               ctypes.POINTER(_Res), ctypes.c_void_p]
        lib.hgpo_mlp_score.restype = ctypes.c_int
        lib.hgpo_mlp_score.argtypes = [ctypes.POINTER(_MLP), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        lib.hgpo_qlog.restype = ctypes.c_int32
        lib.hgpo_qlog.argtypes = [ctypes.c_int64]
        lib.hgpo_connectivity.restype = ctypes.c_int
        lib.hgpo_connectivity.argtypes = [ctypes.POINTER(_HG), ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
        lib.hgpo_trace_new.restype = ctypes.c_void_p
        lib.hgpo_trace_free.argtypes = [ctypes.c_void_p]
        lib.hgpo_trace_levels.restype = ctypes.c_int32
        lib.hgpo_trace_levels.argtypes = [ctypes.c_void_p]
        lib.hgpo_trace_rounds.restype = ctypes.c_int32
        lib.hgpo_trace_rounds.argtypes = [ctypes.c_void_p]
        lib.hgpo_trace_get.restype = ctypes.c_int64
        lib.hgpo_trace_get.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int32)]
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Set the OpenMP thread count used by the oracle's per-node loops."""
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(int(n))
    except OSError:
        os.environ["OMP_NUM_THREADS"] = str(int(n))


def _hg(g, keep):
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (g.hedge_off, g.pins, g.n_src, g.hedge_w, g.node_w)]
    keep.extend(arrs)
    p = [a.ctypes.data if a.size else None for a in arrs]
    return _HG(g.n_nodes, g.n_hedges, arrs[0].ctypes.data, p[1], p[2], p[3], p[4])


class Trace:
    """Per-level / per-round records captured during one oracle run."""

    def __init__(self):
        self._lib = _load()
        self.ptr = self._lib.hgpo_trace_new()

    def __del__(self):
        if getattr(self, "ptr", None):
            self._lib.hgpo_trace_free(self.ptr)
            self.ptr = None

    @property
    def levels(self) -> int:
        return int(self._lib.hgpo_trace_levels(self.ptr))

    @property
    def rounds(self) -> int:
        return int(self._lib.hgpo_trace_rounds(self.ptr))

    def get(self, kind: int, index: int):
        data = ctypes.c_void_p()
        eb = ctypes.c_int32()
        n = self._lib.hgpo_trace_get(self.ptr, kind, index, ctypes.byref(data), ctypes.byref(eb))
        if n < 0:
            return None
        dt = np.int32 if eb.value == 4 else np.int64
        if n == 0:
            return np.zeros(0, dtype=dt)
        buf = (ctypes.c_char * (int(n) * eb.value)).from_address(data.value)
        return np.frombuffer(buf, dtype=dt).copy()


INBOUND, OUTBOUND, INCIDENT = 0, 1, 2
MATCH_TRAVERSAL, MATCH_EXACT = 0, 1


def partition(g, omega: int, delta: int, k: int = 0, max_rounds: int = 8, trace: bool = False, role: int = INBOUND,
              matching: int = MATCH_TRAVERSAL):
    """Run the oracle (role: which pins' hedges count toward Delta; matching:
    the paper's two traversals or the exact tree recursion).
    Returns (rc, parts, result dict, Trace or None)."""
    lib = _load()
    keep = []
    hg = _hg(g, keep)
    parts = np.zeros(max(g.n_nodes, 1), dtype=np.int32)
    res = _Res()
    tr = Trace() if trace else None
    rc = lib.hgpo_partition_ex(ctypes.byref(hg), omega, delta, k, max_rounds, role, matching, parts.ctypes.data,
                               ctypes.byref(res), tr.ptr if tr else None)
    out = dict(connectivity=res.connectivity, n_parts=res.n_parts, n_levels=res.n_levels, n_rounds=res.n_rounds)
    return rc, parts[:g.n_nodes], out, tr


def partition_learned(g, omega: int, delta: int, mlp, k: int = 0, max_rounds: int = 8, trace: bool = False):
    """The oracle with the learned merge proposal (mlp: integer network dict).
    Returns (rc, parts, result dict, Trace or None)."""
    lib = _load()
    keep = []
    hg = _hg(g, keep)
    m = _mlp(mlp)
    parts = np.zeros(max(g.n_nodes, 1), dtype=np.int32)
    res = _Res()
    tr = Trace() if trace else None
    rc = lib.hgpo_partition_learned(ctypes.byref(hg), omega, delta, k, max_rounds, ctypes.byref(m),
                                    parts.ctypes.data, ctypes.byref(res), tr.ptr if tr else None)
    out = dict(connectivity=res.connectivity, n_parts=res.n_parts, n_levels=res.n_levels, n_rounds=res.n_rounds,
               n_fallback=res.n_fallback)
    return rc, parts[:g.n_nodes], out, tr


def match(pair, score, matching: int = MATCH_TRAVERSAL) -> np.ndarray:
    """One matching of the pairing pseudo-forest (pair: -1 = none)."""
    lib = _load()
    p = np.ascontiguousarray(pair, dtype=np.int32)
    sc = np.ascontiguousarray(score, dtype=np.int64)
    out = np.zeros(max(len(p), 1), dtype=np.int32)
    rc = lib.hgpo_match(len(p), p.ctypes.data, sc.ctypes.data, matching, out.ctypes.data)
    if rc != OK:
        raise ValueError(f"hgpo_match rc={rc}")
    return out[:len(p)]


def mlp_score(mlp, xq) -> np.ndarray:
    """The integer network on rows of 16 input codes; returns int64 scores."""
    lib = _load()
    m = _mlp(mlp)
    x = np.ascontiguousarray(xq, dtype=np.int32).reshape(-1, MLP_F)
    out = np.zeros(max(len(x), 1), dtype=np.int64)
    rc = lib.hgpo_mlp_score(ctypes.byref(m), x.ctypes.data if x.size else None, len(x), out.ctypes.data)
    if rc != OK:
        raise ValueError(f"hgpo_mlp_score rc={rc}")
    return out[:len(x)]


def qlog(f: int) -> int:
    """The 8-bit feature code of f >= 0."""
    return int(_load().hgpo_qlog(int(f)))


def connectivity(g, part) -> int:
    """Eq. 1 for an arbitrary partition vector."""
    lib = _load()
    keep = []
    hg = _hg(g, keep)
    p = np.ascontiguousarray(part, dtype=np.int32)
    out = ctypes.c_int64()
    rc = lib.hgpo_connectivity(ctypes.byref(hg), p.ctypes.data if p.size else None, ctypes.byref(out))
    if rc != OK:
        raise ValueError(f"hgpo_connectivity rc={rc}")
    return int(out.value)
