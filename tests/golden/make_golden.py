"""Write expected results of the CPU oracle for named inputs.

Calls only the oracle and the seeded input generators (the learned cases
also read the integer network of a checkpoint file as plain JSON input).
Usage:
    python tests/golden/make_golden.py NAME [threads]
writes tests/golden/NAME.json with the partition's sha256 (int32
little-endian part ids), connectivity, part/level/round counts and the
input digest.  NAME is a benchmark workload (rand16k, rand64k, ...) or one
of CASES below.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2604_14411_amd import synth  # noqa: E402
from paper_2604_14411_amd.synth.configs import WORKLOADS  # noqa: E402

MLP_V2 = os.path.join(ROOT, "paper_2604_14411_amd", "mlp_v2.json")

# Layered conv-like networks under the bounds of the two large layered
# workloads (Omega = 4096, Delta = 65,536), small enough for the oracle:
# 8 layers of 16 x 10 x 10 neurons, 3x3 and 5x5 windows, Geometric(0.1)
# spike-count weights.  Their coarse clusters reach the 64-bit rating
# counters (bits(total) + bits(|in|) > 32).
CASES = {
    "conv12k_3x3": (lambda: synth.layered_conv(8, 16, 10, 10, 3, 0.1, 301), 4096, 65536, None,
                    "layered conv SNN, 8 x (16x10x10), 3x3 window, Geometric(0.1) weights, seed 301"),
    "conv12k_5x5": (lambda: synth.layered_conv(8, 16, 10, 10, 5, 0.1, 302), 4096, 65536, None,
                    "layered conv SNN, 8 x (16x10x10), 5x5 window, Geometric(0.1) weights, seed 302"),
    "conv12k_3x3_learned": (lambda: synth.layered_conv(8, 16, 10, 10, 3, 0.1, 301), 4096, 65536, MLP_V2,
                            "as conv12k_3x3, learned proposal with the integer network of mlp_v2.json"),
    "conv12k_5x5_learned": (lambda: synth.layered_conv(8, 16, 10, 10, 5, 0.1, 302), 4096, 65536, MLP_V2,
                            "as conv12k_5x5, learned proposal with the integer network of mlp_v2.json"),
}


def load_int_network(path):
    """The integer network stored in a checkpoint (key "int"), as plain arrays."""
    with open(path) as f:
        d = json.load(f)["int"]
    return {k: (np.asarray(v, dtype=np.int32) if isinstance(v, list) else int(v)) for k, v in d.items()}


def spec(name):
    """(make, omega, delta, mlp checkpoint or None, note) of a golden input."""
    if name in CASES:
        return CASES[name]
    w = WORKLOADS[name]
    return w.make, w.omega, w.delta, None, w.note


def main():
    name = sys.argv[1]
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else os.cpu_count()
    make, omega, delta, mlp_path, note = spec(name)
    g = make()
    oracle.set_threads(threads)
    t = time.time()
    extra = {}
    if mlp_path:
        q = load_int_network(mlp_path)
        rc, parts, res, _ = oracle.partition_learned(g, omega, delta, q, k=0, max_rounds=8)
        extra = dict(mlp=os.path.basename(mlp_path), n_fallback=int(res["n_fallback"]))
    else:
        rc, parts, res, _ = oracle.partition(g, omega, delta, k=0, max_rounds=8)
    dt = time.time() - t
    assert rc == 0, rc
    out = dict(workload=name, note=note, omega=omega, delta=delta, max_rounds=8, input_sha256=g.digest(),
               parts_sha256=hashlib.sha256(np.ascontiguousarray(parts, dtype="<i4").tobytes()).hexdigest(),
               connectivity=int(res["connectivity"]), n_parts=int(res["n_parts"]), n_levels=int(res["n_levels"]),
               n_rounds=int(res["n_rounds"]), oracle_seconds=round(dt, 1), oracle_threads=threads, **extra)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
