"""Named synthetic workloads standing in for the spiking networks of Tab. I.

Each entry gives the generator call and the size/incidence bounds (Omega,
Delta) it is partitioned under.  Sizes follow Tab. I: 16k-rand, 64k-rand,
alexnet, the rand family and the 302k-neuron model.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional, Tuple

from . import Hypergraph, layered_conv, random_snn, random_snn_family


@dataclass(frozen=True)
class Workload:
    name: str
    omega: int
    delta: int
    make: Callable[[], Hypergraph]
    note: str
    # a reduced instance of the same generator and bounds (for timing the CPU
    # oracle in seconds), its description, and an optional smaller one for a
    # single-thread run: (make, description)
    sample: Optional[Callable[[], Hypergraph]] = None
    sample_note: str = ""
    single_sample: Optional[Tuple[Callable[[], Hypergraph], str]] = None


def _rand(n, mu, seed):
    return lambda: random_snn(n, mu, seed, 1, 16)


WORKLOADS = {
    "rand16k": Workload("rand16k", 1024, 4096, _rand(16384, 127.0, 1),
                        "random SNN, 16,384 nodes, |T_v| ~ Poisson(127)+1, w in [1,16], seed 1",
                        _rand(3072, 127.0, 1), "a random SNN of 3,072 nodes, |T_v| ~ Poisson(127)+1, seed 1"),
    "rand64k": Workload("rand64k", 1024, 4096, _rand(65536, 191.0, 2),
                        "random SNN, 65,536 nodes, |T_v| ~ Poisson(191)+1, w in [1,16], seed 2",
                        _rand(3072, 191.0, 2), "a random SNN of 3,072 nodes, |T_v| ~ Poisson(191)+1, seed 2",
                        (_rand(1024, 191.0, 2), "a random SNN of 1,024 nodes, |T_v| ~ Poisson(191)+1, seed 2")),
    "conv208k": Workload("conv208k", 4096, 65536, lambda: layered_conv(8, 96, 16, 17, 3, 0.1, 3),
                         "layered conv SNN, 8 x (96x16x17), 3x3 window, Geometric(0.1) weights, seed 3",
                         lambda: layered_conv(8, 96, 4, 4, 3, 0.1, 3),
                         "a layered conv SNN of 8 x (96x4x4), 3x3 window, Geometric(0.1) weights, seed 3"),
    "conv302k": Workload("conv302k", 4096, 65536, lambda: layered_conv(8, 42, 30, 30, 5, 0.1, 5),
                         "layered conv SNN, 8 x (42x30x30), 5x5 window, Geometric(0.1) weights, seed 5",
                         lambda: layered_conv(8, 42, 5, 5, 5, 0.1, 5),
                         "a layered conv SNN of 8 x (42x5x5), 5x5 window, Geometric(0.1) weights, seed 5",
                         (lambda: layered_conv(2, 42, 5, 5, 5, 0.1, 5),
                          "a layered conv SNN of 2 x (42x5x5), 5x5 window, seed 5")),
}


def family_member(g: int):
    """Graph g of the 256-graph random-SNN batch (seed 4000+g)."""
    return random_snn_family(4000 + g, 11.0, 15.0, 32.0, 256.0, 1, 16)
