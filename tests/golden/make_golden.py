"""Write expected results of the CPU oracle for named workloads.

Calls only the oracle (and the seeded input generator).  Usage:
    python tests/golden/make_golden.py rand16k [threads]
writes tests/golden/<name>.json with the partition's sha256 (int32
little-endian part ids), connectivity, part/level/round counts and the
input digest.
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
from paper_2604_14411_amd.synth.configs import WORKLOADS  # noqa: E402


def main():
    name = sys.argv[1]
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else os.cpu_count()
    w = WORKLOADS[name]
    g = w.make()
    oracle.set_threads(threads)
    t = time.time()
    rc, parts, res, _ = oracle.partition(g, w.omega, w.delta, k=0, max_rounds=8)
    dt = time.time() - t
    assert rc == 0, rc
    out = dict(workload=name, note=w.note, omega=w.omega, delta=w.delta, max_rounds=8, input_sha256=g.digest(),
               parts_sha256=hashlib.sha256(np.ascontiguousarray(parts, dtype="<i4").tobytes()).hexdigest(),
               connectivity=int(res["connectivity"]), n_parts=int(res["n_parts"]), n_levels=int(res["n_levels"]),
               n_rounds=int(res["n_rounds"]), oracle_seconds=round(dt, 1), oracle_threads=threads)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
