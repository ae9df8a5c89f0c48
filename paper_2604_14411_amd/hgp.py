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
PLAIN = 0
FLAG_TIME_KERNELS = 1
FLAG_NO_INCREMENTAL = 2
KERNEL_CLASSES = ["rate", "propose", "part_table", "seq_events", "contract", "incidence", "sort", "match",
                  "rate_tail"]


class HgpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hgp error {code}: {msg}")
        self.code = code


class Hypergraph_t(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_hedges", ctypes.c_int32), ("hedge_off", ctypes.c_void_p),
                ("pins", ctypes.c_void_p), ("n_src", ctypes.c_void_p), ("hedge_w", ctypes.c_void_p),
                ("node_w", ctypes.c_void_p)]


class Options_t(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("max_refine_rounds", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("proposal", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Result_t(ctypes.Structure):
    _fields_ = [("connectivity", ctypes.c_int64), ("n_parts", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("n_rounds", ctypes.c_int32), ("pad", ctypes.c_int32), ("ms_coarsen", ctypes.c_double),
                ("ms_refine", ctypes.c_double), ("ms_kernel", ctypes.c_double * 9),
                ("n_kernel", ctypes.c_int64 * 9), ("units_kernel", ctypes.c_int64 * 9)]


class Level_t(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_hedges", ctypes.c_int32), ("hoff", ctypes.c_void_p),
                ("hpin", ctypes.c_void_p), ("size", ctypes.c_void_p), ("hedge_w", ctypes.c_void_p)]


EXPORTS = [
    "hgp_ctx_create", "hgp_ctx_destroy", "hgp_options_default", "hgp_partition", "hgp_partition_device",
    "hgp_connectivity_device", "hgp_strerror", "hgp_last_error", "hgp_level_canonical", "hgp_level_rate",
    "hgp_level_match", "hgp_level_contract", "hgp_level_refine_round",
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
    lib.hgp_level_contract.argtypes = [vp, LV, vp, i32, vp, vp, vp, vp]
    lib.hgp_level_refine_round.argtypes = [vp, LV, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, i64p]
    for name in EXPORTS:
        if name not in ("hgp_ctx_destroy", "hgp_options_default", "hgp_strerror", "hgp_last_error"):
            getattr(lib, name).restype = ctypes.c_int
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

    def close(self):
        if getattr(self, "handle", None):
            self._lib.hgp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def options(k: int = 0, max_refine_rounds: int = 8, seed: int = 0, flags: int = 0) -> Options_t:
    o = Options_t()
    load().hgp_options_default(ctypes.byref(o))
    o.k, o.max_refine_rounds, o.seed, o.flags = k, max_refine_rounds, seed, flags
    return o


def _result_dict(r: Result_t) -> dict:
    return dict(connectivity=r.connectivity, n_parts=r.n_parts, n_levels=r.n_levels, n_rounds=r.n_rounds,
                ms_coarsen=r.ms_coarsen, ms_refine=r.ms_refine,
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


def partition_host(ctx: Context, g, omega: int, delta: int, k: int = 0, max_refine_rounds: int = 8):
    """hgp_partition on numpy arrays; returns (parts ndarray, result dict)."""
    lib = load()
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (g.hedge_off, g.pins, g.n_src, g.hedge_w, g.node_w)]
    p = [a.ctypes.data if a.size else None for a in arrs]
    hg = Hypergraph_t(g.n_nodes, g.n_hedges, arrs[0].ctypes.data, p[1], p[2], p[3], p[4])
    parts = np.zeros(max(g.n_nodes, 1), dtype=np.int32)
    res = Result_t()
    o = options(k, max_refine_rounds)
    _check(lib.hgp_partition(ctx.handle, ctypes.byref(hg), omega, delta, ctypes.byref(o), parts.ctypes.data,
                             ctypes.byref(res)))
    return parts[:g.n_nodes], _result_dict(res)


def partition_device(ctx: Context, dg: DeviceHypergraph, omega: int, delta: int, k: int = 0,
                     max_refine_rounds: int = 8, out=None, flags: int = 0):
    """hgp_partition_device; returns (parts tensor on device, result dict)."""
    import torch

    lib = load()
    if out is None:
        out = torch.empty(max(dg.n_nodes, 1), dtype=torch.int32, device=dg.hedge_off.device)
    hg = dg.struct()
    res = Result_t()
    o = options(k, max_refine_rounds, 0, flags)
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


def level_match(ctx: Context, pair, score):
    import torch

    lib = load()
    n = pair.numel()
    match = torch.empty(max(n, 1), dtype=torch.int32, device=pair.device)
    gamma = torch.empty(max(n, 1), dtype=torch.int32, device=pair.device)
    nn = ctypes.c_int32()
    _check(lib.hgp_level_match(ctx.handle, n, _ptr(pair), _ptr(score), _stream(), match.data_ptr(),
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
