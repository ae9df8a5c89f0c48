"""Malformed and infeasible inputs with the error code each must produce
(0 = accepted).  The same list is run through the CPU oracle (tests marked
not gpu) and through the GPU library (tests marked gpu), so both sides
reject the same inputs with the same codes (HGP_E* of include/hgp.h).
"""
import numpy as np

from paper_2604_14411_amd.synth import from_lists

OK, EINVAL, EBADCSR, EINFEASIBLE, EUNSUPPORTED = 0, -1, -2, -3, -6


def _g(n=4, hedges=(([0], [1, 2]), ([3], [0])), w=(1, 2), nw=None):
    return from_lists(n, list(hedges), list(w), nw)


def cases():
    """(name, hypergraph, omega, delta, expected code)."""
    out = [("good", _g(), 4, 4, OK)]
    g = _g()
    g.hedge_off = np.array([0, 3, 2], dtype=np.int32)
    out.append(("offsets not monotone", g, 4, 4, EBADCSR))
    g = _g()
    g.hedge_off = np.array([1, 3, 5], dtype=np.int32)
    g.pins = np.array([0, 0, 1, 2, 3, 0], dtype=np.int32)
    out.append(("offsets not starting at 0", g, 4, 4, EBADCSR))
    out.append(("pin above range", _g(hedges=(([0], [1, 7]), ([3], [0]))), 4, 4, EBADCSR))
    out.append(("negative pin", _g(hedges=(([0], [1, -1]), ([3], [0]))), 4, 4, EBADCSR))
    out.append(("duplicate pin", _g(hedges=(([0], [1, 1]), ([3], [0]))), 4, 4, EBADCSR))
    g = _g()
    g.n_src = np.array([4, 1], dtype=np.int32)
    out.append(("n_src above |e|", g, 4, 4, EBADCSR))
    g = _g()
    g.n_src = np.array([-1, 1], dtype=np.int32)
    out.append(("negative n_src", g, 4, 4, EBADCSR))
    out.append(("hedge weight 0", _g(w=(1, 0)), 4, 4, EINVAL))
    out.append(("node weight 0", _g(nw=[1, 0, 1, 1]), 4, 4, EINVAL))
    out.append(("Omega 0", _g(), 0, 4, EINVAL))
    out.append(("Delta -1", _g(), 4, -1, EINVAL))
    out.append(("node heavier than Omega", _g(nw=[1, 5, 1, 1]), 4, 4, EINFEASIBLE))
    out.append(("|in(n)| above Delta", _g(4, (([0], [1, 2]), ([3], [1]), ([2], [1])), (1, 1, 1)), 4, 1,
                EINFEASIBLE))
    out.append(("total hedge weight above 2^31-1", _g(w=(2 ** 31 - 1, 1)), 4, 4, EUNSUPPORTED))
    out.append(("total node weight above 2^31-1", _g(nw=[2 ** 30, 2 ** 30, 1, 1]), 2 ** 31 - 1, 4, EUNSUPPORTED))
    return out
