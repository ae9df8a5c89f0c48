"""Thin ctypes binding of libhgp (argument marshalling only).

Every step runs in the HIP library; torch is used only to hold device
memory and to name the stream.  Importing this module never falls back to
anything: if ``libhgp.so`` is missing, :func:`load` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgp.so")

OK, EINVAL, EBADCSR, EINFEASIBLE, ENOMEM, EDEVICE, EUNSUPPORTED, EINTERNAL = 0, -1, -2, -3, -4, -5, -6, -7
EIO, EFORMAT = -8, -9
NOALLOC_MAX_ROWS = 1 << 22
PLAIN, LEARNED = 0, 1
INBOUND, OUTBOUND, INCIDENT = 0, 1, 2
MLP_F, MLP_H = 16, 64
FLAG_TIME_KERNELS = 1
FLAG_NO_INCREMENTAL = 2
FLAG_EXACT_MATCHING = 4
MATCH_TRAVERSAL, MATCH_EXACT = 0, 1
KERNEL_CLASSES = ["rate", "propose", "part_table", "seq_events", "contract", "incidence", "sort", "match",
                  "rate_tail", "mlp"]
NK = len(KERNEL_CLASSES)


class HgpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hgp error {code}: {msg}")
        self.code = code


class Hypergraph_t(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_hedges", ctypes.c_int32), ("hedge_off", ctypes.c_void_p),
                ("pins", ctypes.c_void_p), ("n_src", ctypes.c_void_p), ("hedge_w", ctypes.c_void_p),
                ("node_w", ctypes.c_void_p)]


class Mlp_t(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("r1", ctypes.c_int32), ("r2", ctypes.c_int32), ("b3", ctypes.c_int32),
                ("w1", ctypes.c_int32 * (MLP_F * MLP_H)), ("b1", ctypes.c_int32 * MLP_H),
                ("w2", ctypes.c_int32 * (MLP_H * MLP_H)), ("b2", ctypes.c_int32 * MLP_H),
                ("w3", ctypes.c_int32 * MLP_H)]


def mlp_struct(q) -> Mlp_t:
    """Packs an integer network given as a dict (k, r1, r2, b3, w1[16,64], b1, w2[64,64], b2, w3)."""
    m = Mlp_t()
    m.k, m.r1, m.r2, m.b3 = int(q["k"]), int(q["r1"]), int(q["r2"]), int(q["b3"])
    for name, n in (("w1", MLP_F * MLP_H), ("b1", MLP_H), ("w2", MLP_H * MLP_H), ("b2", MLP_H), ("w3", MLP_H)):
        a = np.ascontiguousarray(np.asarray(q[name]).reshape(-1), dtype=np.int32)
        if a.size != n:
            raise ValueError(f"network field {name} has {a.size} values, expected {n}")
        ctypes.memmove(getattr(m, name), a.ctypes.data, 4 * n)
    return m


class MlpF32_t(ctypes.Structure):
    _fields_ = [("w1", ctypes.c_float * (MLP_F * MLP_H)), ("b1", ctypes.c_float * MLP_H),
                ("w2", ctypes.c_float * (MLP_H * MLP_H)), ("b2", ctypes.c_float * MLP_H),
                ("w3", ctypes.c_float * MLP_H), ("b3", ctypes.c_float)]


class TrainOpts_t(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class TrainState_t(ctypes.Structure):
    _fields_ = [("w", MlpF32_t), ("m", MlpF32_t), ("v", MlpF32_t), ("step", ctypes.c_int64),
                ("epoch", ctypes.c_int64), ("rng", ctypes.c_uint64)]


def f32_to_dict(w: MlpF32_t) -> dict:
    """Float weights as numpy arrays (w1[16,64], b1, w2[64,64], b2, w3, b3)."""
    return dict(w1=np.ctypeslib.as_array(w.w1).reshape(MLP_F, MLP_H).copy(), b1=np.ctypeslib.as_array(w.b1).copy(),
                w2=np.ctypeslib.as_array(w.w2).reshape(MLP_H, MLP_H).copy(), b2=np.ctypeslib.as_array(w.b2).copy(),
                w3=np.ctypeslib.as_array(w.w3).copy(), b3=float(w.b3))


def f32_from_dict(d) -> MlpF32_t:
    w = MlpF32_t()
    for name, n in (("w1", MLP_F * MLP_H), ("b1", MLP_H), ("w2", MLP_H * MLP_H), ("b2", MLP_H), ("w3", MLP_H)):
        a = np.ascontiguousarray(np.asarray(d[name]).reshape(-1), dtype=np.float32)
        if a.size != n:
            raise ValueError(f"float network field {name} has {a.size} values, expected {n}")
        ctypes.memmove(getattr(w, name), a.ctypes.data, 4 * n)
    w.b3 = float(d["b3"])
    return w


def mlp_to_dict(m: Mlp_t) -> dict:
    """Integer network as a dict of numpy arrays."""
    return dict(k=m.k, r1=m.r1, r2=m.r2, b3=m.b3, w1=np.ctypeslib.as_array(m.w1).reshape(MLP_F, MLP_H).copy(),
                b1=np.ctypeslib.as_array(m.b1).copy(), w2=np.ctypeslib.as_array(m.w2).reshape(MLP_H, MLP_H).copy(),
                b2=np.ctypeslib.as_array(m.b2).copy(), w3=np.ctypeslib.as_array(m.w3).copy())


ORDER_LPT, ORDER_INPUT = 1, 2
LATE_INCREMENTAL, LATE_FULL = 1, 2


class BatchSched_t(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("order", ctypes.c_int32), ("rate_tile", ctypes.c_int32),
                ("late_levels", ctypes.c_int32)]


class Options_t(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("max_refine_rounds", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("proposal", ctypes.c_int32), ("flags", ctypes.c_int32), ("mlp", ctypes.POINTER(Mlp_t)),
                ("constraint", ctypes.c_int32), ("time_classes", ctypes.c_int32)]


class Result_t(ctypes.Structure):
    _fields_ = [("connectivity", ctypes.c_int64), ("n_parts", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("n_rounds", ctypes.c_int32), ("n_fallback", ctypes.c_int32), ("n_kept", ctypes.c_int32),
                ("ms_coarsen", ctypes.c_double),
                ("ms_refine", ctypes.c_double), ("ms_kernel", ctypes.c_double * NK),
                ("n_kernel", ctypes.c_int64 * NK), ("units_kernel", ctypes.c_int64 * NK)]


class Level_t(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_hedges", ctypes.c_int32), ("hoff", ctypes.c_void_p),
                ("hpin", ctypes.c_void_p), ("size", ctypes.c_void_p), ("hedge_w", ctypes.c_void_p)]


EXPORTS = [
    "hgp_ctx_create", "hgp_ctx_destroy", "hgp_set_level_cache", "hgp_options_default", "hgp_partition", "hgp_partition_device",
    "hgp_connectivity_device", "hgp_strerror", "hgp_last_error", "hgp_level_canonical", "hgp_level_rate",
    "hgp_level_match", "hgp_level_contract", "hgp_level_refine_round", "hgp_level_learned",
    "hgp_mlp_score_device", "hgp_mlp_init", "hgp_mlp_grad", "hgp_mlp_train", "hgp_mlp_quantize",
    "hgp_trace_create", "hgp_trace_destroy", "hgp_partition_traced", "hgp_trace_rows", "hgp_trace_read",
    "hgp_partition_batch_device", "hgp_batch_tune", "hgp_connectivity", "hgp_train_state_init",
    "hgp_mlp_train_state", "hgp_mlp_save", "hgp_mlp_load", "hgp_mlp_score_device_noalloc", "hgp_level_match_ex",
]

_lib = None


def load():
    """Load libhgp.so (built in-tree); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    HG = ctypes.POINTER(Hypergraph_t)
    LV = ctypes.POINTER(Level_t)
    lib.hgp_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.hgp_ctx_destroy.argtypes = [vp]
    lib.hgp_ctx_destroy.restype = None
    lib.hgp_options_default.argtypes = [ctypes.POINTER(Options_t)]
    lib.hgp_set_level_cache.argtypes = [vp, ctypes.c_int64, i64p]
    lib.hgp_options_default.restype = None
    lib.hgp_partition.argtypes = [vp, HG, i32, i32, ctypes.POINTER(Options_t), vp, ctypes.POINTER(Result_t)]
    lib.hgp_partition_device.argtypes = [vp, HG, i32, i32, ctypes.POINTER(Options_t), vp, vp,
                                         ctypes.POINTER(Result_t)]
    lib.hgp_connectivity_device.argtypes = [vp, HG, vp, vp, i64p]
    lib.hgp_strerror.restype = ctypes.c_char_p
    lib.hgp_strerror.argtypes = [ctypes.c_int]
    lib.hgp_last_error.restype = ctypes.c_char_p
    lib.hgp_last_error.argtypes = []
    lib.hgp_level_canonical.argtypes = [vp, HG, i32, i32, vp, vp, vp]
    lib.hgp_level_rate.argtypes = [vp, LV, i32, i32, vp, vp, vp]
    lib.hgp_level_match.argtypes = [vp, i32, vp, vp, vp, vp, vp, ctypes.POINTER(i32)]
    lib.hgp_level_match_ex.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, ctypes.POINTER(i32)]
    lib.hgp_level_contract.argtypes = [vp, LV, vp, i32, vp, vp, vp, vp]
    lib.hgp_level_refine_round.argtypes = [vp, LV, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, i64p]
    MP = ctypes.POINTER(Mlp_t)
    lib.hgp_level_learned.argtypes = [vp, LV, i32, i32, i32, MP, vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp,
                                      i64p]
    lib.hgp_mlp_score_device.argtypes = [vp, MP, vp, ctypes.c_int64, vp, vp]
    lib.hgp_mlp_score_device_noalloc.argtypes = [vp, MP, vp, ctypes.c_int64, vp, vp]
    FP = ctypes.POINTER(MlpF32_t)
    lib.hgp_mlp_init.argtypes = [FP, ctypes.c_uint64]
    lib.hgp_mlp_grad.argtypes = [vp, FP, vp, vp, ctypes.c_int64, FP, ctypes.POINTER(ctypes.c_double), vp]
    lib.hgp_mlp_train.argtypes = [vp, FP, vp, vp, ctypes.c_int64, ctypes.POINTER(TrainOpts_t), vp, vp]
    lib.hgp_mlp_quantize.argtypes = [FP, vp, ctypes.c_int64, i32, MP, ctypes.POINTER(i32)]
    SP = ctypes.POINTER(TrainState_t)
    lib.hgp_train_state_init.argtypes = [SP, FP, ctypes.POINTER(TrainOpts_t)]
    lib.hgp_mlp_train_state.argtypes = [vp, SP, vp, vp, ctypes.c_int64, ctypes.POINTER(TrainOpts_t), i32, vp, vp]
    lib.hgp_mlp_save.argtypes = [ctypes.c_char_p, SP, MP, i32]
    lib.hgp_mlp_load.argtypes = [ctypes.c_char_p, SP, MP, ctypes.POINTER(i32)]
    lib.hgp_connectivity.argtypes = [vp, HG, vp, i64p]
    lib.hgp_trace_create.argtypes = [ctypes.POINTER(vp)]
    lib.hgp_trace_destroy.argtypes = [vp]
    lib.hgp_partition_traced.argtypes = [vp, HG, i32, i32, ctypes.POINTER(Options_t), vp, vp,
                                         ctypes.POINTER(Result_t)]
    lib.hgp_trace_rows.argtypes = [vp]
    lib.hgp_trace_read.argtypes = [vp, vp, vp, vp, vp, vp]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.hgp_partition_batch_device.argtypes = [vp, i32, HG, vp, vp, ctypes.POINTER(Options_t),
                                               ctypes.POINTER(BatchSched_t), vp, vp, ctypes.POINTER(Result_t), dp, dp]
    lib.hgp_batch_tune.argtypes = [vp, i32, HG, vp, vp, ctypes.POINTER(Options_t), vp, vp,
                                   ctypes.POINTER(BatchSched_t), dp]
    for name in EXPORTS:
        if name not in ("hgp_ctx_destroy", "hgp_options_default", "hgp_strerror", "hgp_last_error",
                        "hgp_mlp_init", "hgp_trace_destroy", "hgp_trace_rows", "hgp_train_state_init"):
            getattr(lib, name).restype = ctypes.c_int
    lib.hgp_mlp_init.restype = None
    lib.hgp_train_state_init.restype = None
    lib.hgp_trace_destroy.restype = None
    lib.hgp_trace_rows.restype = ctypes.c_int64
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise HgpError(rc, load().hgp_last_error().decode())


def _ptr(t):
    return None if t is None else (t.data_ptr() if t.numel() else None)


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A libhgp context on one HIP device (owns its device scratch)."""

    def __init__(self, device: int = 0):
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.hgp_ctx_create(ctypes.byref(h), device))
        self.handle = h
        self.device = device

    def set_level_cache(self, nbytes: int) -> int:
        """Device bytes the context may keep coarse levels in (0: none, -1:
        the default); returns the bytes it holds for them now."""
        held = ctypes.c_int64(0)
        _check(self._lib.hgp_set_level_cache(self.handle, int(nbytes), ctypes.byref(held)))
        return held.value

    def close(self):
        if getattr(self, "handle", None):
            self._lib.hgp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def options(k: int = 0, max_refine_rounds: int = 8, seed: int = 0, flags: int = 0, mlp=None, constraint: int = 0,
            time_classes: int = 0):
    """hgp_options; with an integer network dict `mlp` the learned proposal is selected.
    Returns (Options_t, keep-alive object)."""
    o = Options_t()
    load().hgp_options_default(ctypes.byref(o))
    o.k, o.max_refine_rounds, o.seed, o.flags = k, max_refine_rounds, seed, flags
    o.constraint = constraint
    o.time_classes = time_classes
    m = None
    if mlp is not None:
        m = mlp if isinstance(mlp, Mlp_t) else mlp_struct(mlp)
        o.proposal = LEARNED
        o.mlp = ctypes.pointer(m)
    return o, m


def _result_dict(r: Result_t) -> dict:
    return dict(connectivity=r.connectivity, n_parts=r.n_parts, n_levels=r.n_levels, n_rounds=r.n_rounds,
                n_fallback=r.n_fallback, n_kept=r.n_kept, ms_coarsen=r.ms_coarsen, ms_refine=r.ms_refine,
                kernels={name: dict(ms=r.ms_kernel[i], launches=r.n_kernel[i], units=r.units_kernel[i])
                         for i, name in enumerate(KERNEL_CLASSES)})


class DeviceHypergraph:
    """Hypergraph arrays resident on the GPU as int32 torch tensors."""

    def __init__(self, g, device="cuda"):
        import torch

        def t(a):
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).to(device)

        self.hedge_off, self.pins, self.n_src = t(g.hedge_off), t(g.pins), t(g.n_src)
        self.hedge_w, self.node_w = t(g.hedge_w), t(g.node_w)
        self.n_nodes, self.n_hedges = g.n_nodes, g.n_hedges

    def struct(self) -> Hypergraph_t:
        return Hypergraph_t(self.n_nodes, self.n_hedges, self.hedge_off.data_ptr(), _ptr(self.pins),
                            _ptr(self.n_src), _ptr(self.hedge_w), _ptr(self.node_w))


def partition_host(ctx: Context, g, omega: int, delta: int, k: int = 0, max_refine_rounds: int = 8, mlp=None,
                   constraint: int = 0):
    """hgp_partition on numpy arrays; returns (parts ndarray, result dict)."""
    lib = load()
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (g.hedge_off, g.pins, g.n_src, g.hedge_w, g.node_w)]
    p = [a.ctypes.data if a.size else None for a in arrs]
    hg = Hypergraph_t(g.n_nodes, g.n_hedges, arrs[0].ctypes.data, p[1], p[2], p[3], p[4])
    parts = np.zeros(max(g.n_nodes, 1), dtype=np.int32)
    res = Result_t()
    o, _keep = options(k, max_refine_rounds, mlp=mlp, constraint=constraint)
    _check(lib.hgp_partition(ctx.handle, ctypes.byref(hg), omega, delta, ctypes.byref(o), parts.ctypes.data,
                             ctypes.byref(res)))
    return parts[:g.n_nodes], _result_dict(res)


def partition_device(ctx: Context, dg: DeviceHypergraph, omega: int, delta: int, k: int = 0,
                     max_refine_rounds: int = 8, out=None, flags: int = 0, mlp=None, constraint: int = 0,
                     time_classes: int = 0):
    """hgp_partition_device; returns (parts tensor on device, result dict)."""
    import torch

    lib = load()
    if out is None:
        out = torch.empty(max(dg.n_nodes, 1), dtype=torch.int32, device=dg.hedge_off.device)
    hg = dg.struct()
    res = Result_t()
    o, _keep = options(k, max_refine_rounds, 0, flags, mlp=mlp, constraint=constraint, time_classes=time_classes)
    _check(lib.hgp_partition_device(ctx.handle, ctypes.byref(hg), omega, delta, ctypes.byref(o), _stream(),
                                    out.data_ptr(), ctypes.byref(res)))
    return out[:dg.n_nodes], _result_dict(res)


def connectivity_device(ctx: Context, dg: DeviceHypergraph, part) -> int:
    lib = load()
    hg = dg.struct()
    out = ctypes.c_int64()
    _check(lib.hgp_connectivity_device(ctx.handle, ctypes.byref(hg), _ptr(part), _stream(), ctypes.byref(out)))
    return int(out.value)


# ---------------------------------------------------------------- level API
def connectivity_host(ctx: Context, g, part) -> int:
    """hgp_connectivity: Eq. 1 of a host partition vector on a host hypergraph
    (copied to the device and computed there)."""
    lib = load()
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (g.hedge_off, g.pins, g.n_src, g.hedge_w, g.node_w)]
    p = [a.ctypes.data if a.size else None for a in arrs]
    hg = Hypergraph_t(g.n_nodes, g.n_hedges, arrs[0].ctypes.data, p[1], p[2], p[3], p[4])
    pa = np.ascontiguousarray(part, dtype=np.int32)
    out = ctypes.c_int64()
    _check(lib.hgp_connectivity(ctx.handle, ctypes.byref(hg), pa.ctypes.data if pa.size else None,
                                ctypes.byref(out)))
    return int(out.value)


def level_canonical(ctx: Context, dg: DeviceHypergraph, omega: int, delta: int):
    import torch

    lib = load()
    hoff = torch.empty(dg.n_hedges + 1, dtype=torch.int32, device=dg.hedge_off.device)
    hpin = torch.empty(max(dg.pins.numel(), 1), dtype=torch.int32, device=dg.hedge_off.device)
    hg = dg.struct()
    _check(lib.hgp_level_canonical(ctx.handle, ctypes.byref(hg), omega, delta, _stream(), hoff.data_ptr(),
                                   hpin.data_ptr()))
    return hoff, hpin[:dg.pins.numel()]


def _level(n, hoff, hpin, size, hw) -> Level_t:
    return Level_t(n, hoff.numel() - 1, hoff.data_ptr(), _ptr(hpin), _ptr(size), _ptr(hw))


def level_rate(ctx: Context, n, hoff, hpin, size, hw, omega: int, delta: int):
    import torch

    lib = load()
    dev = hoff.device
    pair = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    score = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    lv = _level(n, hoff, hpin, size, hw)
    _check(lib.hgp_level_rate(ctx.handle, ctypes.byref(lv), omega, delta, _stream(), pair.data_ptr(),
                              score.data_ptr()))
    return pair[:n], score[:n]


def level_match(ctx: Context, pair, score, rule: int = MATCH_TRAVERSAL):
    """hgp_level_match_ex on device pair (int32) and score (int64) tensors;
    returns (match, gamma, number of clusters)."""
    import torch

    lib = load()
    n = pair.numel()
    match = torch.empty(max(n, 1), dtype=torch.int32, device=pair.device)
    gamma = torch.empty(max(n, 1), dtype=torch.int32, device=pair.device)
    nn = ctypes.c_int32()
    _check(lib.hgp_level_match_ex(ctx.handle, n, _ptr(pair), _ptr(score), rule, _stream(), match.data_ptr(),
                                  gamma.data_ptr(), ctypes.byref(nn)))
    return match[:n], gamma[:n], nn.value


def level_contract(ctx: Context, n, hoff, hpin, size, hw, gamma, n_next: int):
    import torch

    lib = load()
    dev = hoff.device
    E = hoff.numel() - 1
    hoff2 = torch.empty(E + 1, dtype=torch.int32, device=dev)
    hpin2 = torch.empty(max(hpin.numel(), 1), dtype=torch.int32, device=dev)
    size2 = torch.empty(max(n_next, 1), dtype=torch.int32, device=dev)
    lv = _level(n, hoff, hpin, size, hw)
    _check(lib.hgp_level_contract(ctx.handle, ctypes.byref(lv), _ptr(gamma), n_next, _stream(), hoff2.data_ptr(),
                                  hpin2.data_ptr(), size2.data_ptr()))
    P2 = int(hoff2[-1].item())
    return hoff2, hpin2[:P2], size2[:n_next]


def level_refine_round(ctx: Context, n, hoff, hpin, size, hw, rho, n_parts: int, omega: int, delta: int):
    import torch

    lib = load()
    dev = hoff.device
    m = max(n, 1)
    pdest = torch.empty(m, dtype=torch.int32, device=dev)
    pgain = torch.empty(m, dtype=torch.int64, device=dev)
    seq = torch.empty(m, dtype=torch.int32, device=dev)
    gsum = torch.empty(m + 1, dtype=torch.int64, device=dev)
    viol = torch.empty(m + 1, dtype=torch.int32, device=dev)
    rho_out = torch.empty(m, dtype=torch.int32, device=dev)
    info = (ctypes.c_int64 * 4)()
    lv = _level(n, hoff, hpin, size, hw)
    _check(lib.hgp_level_refine_round(ctx.handle, ctypes.byref(lv), _ptr(rho), n_parts, omega, delta, _stream(),
                                      pdest.data_ptr(), pgain.data_ptr(), seq.data_ptr(), gsum.data_ptr(),
                                      viol.data_ptr(), rho_out.data_ptr(), info))
    S = int(info[0])
    return dict(dest=pdest[:n], gain=pgain[:n], seq=seq[:S], G=gsum[:S + 1], viol=viol[:S + 1], rho=rho_out[:n],
                S=S, istar=int(info[1]), gstar=int(info[2]), applied=bool(info[3]))


def level_learned(ctx: Context, n, hoff, hpin, size, hw, level: int, omega: int, delta: int, mlp, codes=True):
    """hgp_level_learned: candidate sets, codes, scores and pairs of one level."""
    import torch

    lib = load()
    dev = hoff.device
    m = max(n, 1)
    cap = 16 * m
    coff = torch.empty(m + 1, dtype=torch.int64, device=dev)
    cand = torch.empty(cap, dtype=torch.int32, device=dev)
    xq = torch.empty(cap * MLP_F, dtype=torch.int32, device=dev) if codes else None
    cscore = torch.empty(cap, dtype=torch.int64, device=dev)
    pair = torch.empty(m, dtype=torch.int32, device=dev)
    score = torch.empty(m, dtype=torch.int64, device=dev)
    ppair = torch.empty(m, dtype=torch.int32, device=dev)
    cnt = ctypes.c_int64()
    lv = _level(n, hoff, hpin, size, hw)
    q = mlp if isinstance(mlp, Mlp_t) else mlp_struct(mlp)
    _check(lib.hgp_level_learned(ctx.handle, ctypes.byref(lv), level, omega, delta, ctypes.byref(q), _stream(), cap,
                                 coff.data_ptr(), cand.data_ptr(), xq.data_ptr() if codes else None,
                                 cscore.data_ptr(), pair.data_ptr(), score.data_ptr(), ppair.data_ptr(),
                                 ctypes.byref(cnt)))
    C = int(cnt.value)
    return dict(coff=coff[:n + 1], cand=cand[:C], xq=xq[:C * MLP_F].view(C, MLP_F) if codes else None,
                cscore=cscore[:C], pair=pair[:n], score=score[:n], ppair=ppair[:n])


def mlp_score_device(ctx: Context, mlp, xq):
    """hgp_mlp_score_device on a device int32 tensor of shape [n, 16]; returns int64 scores."""
    import torch

    lib = load()
    n = xq.shape[0]
    out = torch.empty(max(n, 1), dtype=torch.int64, device=xq.device)
    q = mlp if isinstance(mlp, Mlp_t) else mlp_struct(mlp)
    _check(lib.hgp_mlp_score_device(ctx.handle, ctypes.byref(q), _ptr(xq.contiguous()), n, out.data_ptr(),
                                    _stream()))
    return out[:n]


# ---------------------------------------------------------------- training
def mlp_score_device_noalloc(ctx: Context, mlp, xq, out=None):
    """hgp_mlp_score_device_noalloc: the network on device rows xq [n,16]
    without device allocation in the library (out: int64 [n] device tensor;
    allocated here by torch when not given)."""
    import torch

    m = mlp if isinstance(mlp, Mlp_t) else mlp_struct(mlp)
    n = int(xq.shape[0])
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.int64, device=xq.device)
    _check(load().hgp_mlp_score_device_noalloc(ctx.handle, ctypes.byref(m), _ptr(xq.contiguous()), n, _ptr(out),
                                               _stream()))
    return out[:n]


def mlp_init(seed: int) -> dict:
    """Seeded initial float weights (hgp_mlp_init)."""
    w = MlpF32_t()
    load().hgp_mlp_init(ctypes.byref(w), seed)
    return f32_to_dict(w)


def mlp_grad(ctx: Context, w: dict, xq, y):
    """Mean loss and gradient on device rows (xq int32 [n,16], y float32 [n])."""
    lib = load()
    wf = f32_from_dict(w)
    g = MlpF32_t()
    loss = ctypes.c_double()
    _check(lib.hgp_mlp_grad(ctx.handle, ctypes.byref(wf), _ptr(xq.contiguous()), _ptr(y.contiguous()), xq.shape[0],
                            ctypes.byref(g), ctypes.byref(loss), _stream()))
    return f32_to_dict(g), float(loss.value)


def mlp_train(ctx: Context, w: dict, xq, y, epochs=4, batch=4096, lr=2e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              seed=0):
    """Adam training on device rows; returns (trained float weights, per-epoch mean loss)."""
    lib = load()
    wf = f32_from_dict(w)
    o = TrainOpts_t(epochs, batch, lr, beta1, beta2, eps, seed)
    losses = (ctypes.c_float * max(epochs, 1))()
    _check(lib.hgp_mlp_train(ctx.handle, ctypes.byref(wf), _ptr(xq.contiguous()), _ptr(y.contiguous()),
                             xq.shape[0], ctypes.byref(o), losses, _stream()))
    return f32_to_dict(wf), [float(losses[i]) for i in range(epochs)]


def train_state(w: dict, seed: int = 0) -> TrainState_t:
    """Fresh resumable training state (hgp_train_state_init) from float weights."""
    st = TrainState_t()
    wf = f32_from_dict(w)
    o = TrainOpts_t(0, 1, 1e-3, 0.9, 0.999, 1e-8, seed)
    load().hgp_train_state_init(ctypes.byref(st), ctypes.byref(wf), ctypes.byref(o))
    return st


def mlp_train_state(ctx: Context, st: TrainState_t, xq, y, epochs, batch=4096, lr=2e-3, beta1=0.9, beta2=0.999,
                    eps=1e-8):
    """`epochs` more epochs from a training state (updated in place); returns the per-epoch mean loss."""
    lib = load()
    o = TrainOpts_t(epochs, batch, lr, beta1, beta2, eps, 0)
    losses = (ctypes.c_float * max(epochs, 1))()
    _check(lib.hgp_mlp_train_state(ctx.handle, ctypes.byref(st), _ptr(xq.contiguous()), _ptr(y.contiguous()),
                                   xq.shape[0], ctypes.byref(o), epochs, losses, _stream()))
    return [float(losses[i]) for i in range(epochs)]


def mlp_save(path: str, state: TrainState_t = None, q=None, score_shift: int = 0) -> None:
    """hgp_mlp_save: versioned binary checkpoint (training state and/or integer network)."""
    m = None if q is None else (q if isinstance(q, Mlp_t) else mlp_struct(q))
    _check(load().hgp_mlp_save(os.fsencode(path), None if state is None else ctypes.byref(state),
                               None if m is None else ctypes.byref(m), int(score_shift)))


def mlp_load(path: str, state: bool = True, network: bool = True):
    """hgp_mlp_load; returns (TrainState_t or None, integer network dict or None, score_shift)."""
    st = TrainState_t() if state else None
    m = Mlp_t() if network else None
    sh = ctypes.c_int32()
    _check(load().hgp_mlp_load(os.fsencode(path), None if st is None else ctypes.byref(st),
                               None if m is None else ctypes.byref(m), ctypes.byref(sh)))
    return st, (None if m is None else mlp_to_dict(m)), int(sh.value)


def mlp_quantize(w: dict, xq_calib, k: int = 8):
    """Integer network from float weights and host calibration codes; returns (dict, score_shift)."""
    lib = load()
    wf = f32_from_dict(w)
    x = np.ascontiguousarray(xq_calib, dtype=np.int32).reshape(-1, MLP_F)
    q = Mlp_t()
    sh = ctypes.c_int32()
    _check(lib.hgp_mlp_quantize(ctypes.byref(wf), x.ctypes.data if x.size else None, len(x), k, ctypes.byref(q),
                                ctypes.byref(sh)))
    return mlp_to_dict(q), int(sh.value)


def partition_traced(ctx: Context, g, omega: int, delta: int, k: int = 0, max_refine_rounds: int = 8):
    """Plain partition of a host hypergraph with merge traces.  Returns
    (parts, result dict, trace dict with xq[rows,16], label, level, node, cand)."""
    lib = load()
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (g.hedge_off, g.pins, g.n_src, g.hedge_w, g.node_w)]
    p = [a.ctypes.data if a.size else None for a in arrs]
    hg = Hypergraph_t(g.n_nodes, g.n_hedges, arrs[0].ctypes.data, p[1], p[2], p[3], p[4])
    parts = np.zeros(max(g.n_nodes, 1), dtype=np.int32)
    res = Result_t()
    o, _keep = options(k, max_refine_rounds)
    t = ctypes.c_void_p()
    _check(lib.hgp_trace_create(ctypes.byref(t)))
    try:
        _check(lib.hgp_partition_traced(ctx.handle, ctypes.byref(hg), omega, delta, ctypes.byref(o), t,
                                        parts.ctypes.data, ctypes.byref(res)))
        rows = int(lib.hgp_trace_rows(t))
        xq = np.zeros((max(rows, 1), MLP_F), np.int32)
        label = np.zeros(max(rows, 1), np.float32)
        level = np.zeros(max(rows, 1), np.int32)
        node = np.zeros(max(rows, 1), np.int32)
        cand = np.zeros(max(rows, 1), np.int32)
        _check(lib.hgp_trace_read(t, xq.ctypes.data, label.ctypes.data, level.ctypes.data, node.ctypes.data,
                                  cand.ctypes.data))
    finally:
        lib.hgp_trace_destroy(t)
    tr = dict(xq=xq[:rows], label=label[:rows], level=level[:rows], node=node[:rows], cand=cand[:rows])
    return parts[:g.n_nodes], _result_dict(res), tr


# ---------------------------------------------------------------- batches
def _batch_args(dgs, omegas, deltas, outs):
    import torch

    n = len(dgs)
    hg = (Hypergraph_t * max(n, 1))()
    for i, d in enumerate(dgs):
        hg[i] = d.struct()
    om = np.ascontiguousarray(omegas, dtype=np.int32)
    de = np.ascontiguousarray(deltas, dtype=np.int32)
    if outs is None:
        outs = [torch.empty(max(d.n_nodes, 1), dtype=torch.int32, device=d.hedge_off.device) for d in dgs]
    po = (ctypes.c_void_p * max(n, 1))()
    for i, o in enumerate(outs):
        po[i] = o.data_ptr()
    return n, hg, om, de, outs, po


def partition_batch_device(ctx: Context, dgs, omegas, deltas, sched=None, outs=None, k: int = 0,
                           max_refine_rounds: int = 8, flags: int = 0, mlp=None):
    """hgp_partition_batch_device on a list of DeviceHypergraph.  sched: dict of
    BatchSched_t fields (missing = tuned/default).  Returns (parts list,
    result dicts, t_start_ms, t_end_ms)."""
    lib = load()
    n, hg, om, de, outs, po = _batch_args(dgs, omegas, deltas, outs)
    o, _keep = options(k, max_refine_rounds, 0, flags, mlp=mlp)
    sc = BatchSched_t(**(sched or {}))
    res = (Result_t * max(n, 1))()
    t0 = (ctypes.c_double * max(n, 1))()
    t1 = (ctypes.c_double * max(n, 1))()
    _check(lib.hgp_partition_batch_device(ctx.handle, n, hg, om.ctypes.data, de.ctypes.data, ctypes.byref(o),
                                          ctypes.byref(sc), _stream(), po, res, t0, t1))
    return ([outs[i][:dgs[i].n_nodes] for i in range(n)], [_result_dict(res[i]) for i in range(n)],
            np.array(t0[:n]), np.array(t1[:n]))


def batch_tune(ctx: Context, dgs, omegas, deltas, outs=None, flags: int = 0, mlp=None):
    """hgp_batch_tune (with the learned proposal when an integer network
    `mlp` is given); returns (schedule dict, wall ms of the best schedule)."""
    lib = load()
    n, hg, om, de, outs, po = _batch_args(dgs, omegas, deltas, outs)
    o, _keep = options(0, 8, 0, flags, mlp=mlp)
    best = BatchSched_t()
    ms = ctypes.c_double()
    _check(lib.hgp_batch_tune(ctx.handle, n, hg, om.ctypes.data, de.ctypes.data, ctypes.byref(o), _stream(), po,
                              ctypes.byref(best), ctypes.byref(ms)))
    return dict(workers=best.workers, order=best.order, rate_tile=best.rate_tile,
                late_levels=best.late_levels), float(ms.value)
