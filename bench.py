#!/usr/bin/env python3
"""Throughput of the constrained multilevel partitioner on one MI355X.

One step = one full hgp_partition_device call (coarsening + refinement +
connectivity) on a device-resident synthetic spiking-network hypergraph.
Prints one JSON line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--workload conv302k] [--mlp CHECKPOINT | --plain]

By default the timed steps use the learned merge proposal (the committed
checkpoint) on the 302,400-node layered network; the plain method is then
timed on the same input (--plain-steps runs) as the judge of its
connectivity, and the line reports both.  --plain times the plain method.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published HBM peak and the LDS-atomic peak derived from unit counts:
# 256 CUs x 2.4 GHz x 16 atomic lanes per clock per CU
HBM_PEAK_GBS = 8000.0
CUS, CLOCK_GHZ, LDS_ATOMIC_LANES_PER_CLK = 256, 2.4, 16
LDS_ATOMIC_PEAK_TOPS = CUS * CLOCK_GHZ * 1e9 * LDS_ATOMIC_LANES_PER_CLK / 1e12

# Algorithmic cost model per kernel class: (bound, bytes or ops per unit).
# rate / propose: one LDS read-modify-write per unit (pin-pair visit, part-table
# entry visit); the pin-streaming kernels: compulsory HBM bytes per pin.
COST = {
    "rate": ("alu", 1.0),
    "rate_tail": ("alu", 1.0),
    "propose": ("alu", 1.0),
    "part_table": ("hbm", 16.0),
    "seq_events": ("hbm", 1.0),  # units are algorithmic bytes: 4 per pin, 16 per event
    "contract": ("hbm", 16.0),
    "incidence": ("hbm", 12.0),  # pins read, incidences and their pin positions written
    "sort": ("hbm", 32.0),
    "match": ("hbm", 20.0),
    "mlp": ("hbm", 52.0),
}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(cls: str):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known
    size), or None when there is none or a source it was taken from changed."""
    import hashlib

    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get("classes", {}).get(cls)
    if not e:
        return None
    for rel, digest in e.get("sources", {}).items():
        try:
            with open(os.path.join(ROOT, rel), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != digest:
                    return None
        except OSError:
            return None
    return e["bytes_per_launch"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, mlp, threads_multi: int):
    """The CPU oracle on a bounded sample of the benchmarked workload: the same
    generator and bounds at a reduced size (Workload.sample), with the same
    proposal as the timed steps; all host threads, then one thread on a
    smaller sample.  The oracle is test infrastructure and runs only here."""
    import oracle

    sample, note, single = w.sample, w.sample_note, w.single_sample
    g = sample()
    oracle.set_threads(threads_multi)

    def run(graph):
        t = time.perf_counter()
        if mlp is not None:
            rc, _, res, _ = oracle.partition_learned(graph, w.omega, w.delta, mlp)
        else:
            rc, _, res, _ = oracle.partition(graph, w.omega, w.delta)
        dt = time.perf_counter() - t
        assert rc == 0, rc
        return dt, res

    dt, res = run(g)
    out = dict(value=g.n_pins / dt, unit="pins/s", cores=threads_multi, kind="oracle",
               proposal="learned" if mlp is not None else "plain",
               sample=f"CPU oracle, whole partition of {note}: {g.n_nodes} nodes, {g.n_pins} pins, "
                      f"sum|e|^2 {g.sum_sq():.3e}, Omega={w.omega}, Delta={w.delta}; {res['n_levels']} levels, "
                      f"{dt:.1f} s on {threads_multi} threads",
               seconds=dt, levels=res["n_levels"], sample_pins=g.n_pins, sample_sum_e_sq=g.sum_sq(),
               nproc=os.cpu_count(), cpu_model=_cpu_model())
    if single is not None:
        g1 = single[0]()
        oracle.set_threads(1)
        dt1, res1 = run(g1)
        out["single_thread"] = dict(value=g1.n_pins / dt1, unit="pins/s", cores=1, seconds=dt1,
                                    sample=f"{single[1]}: {g1.n_nodes} nodes, {g1.n_pins} pins, "
                                           f"{res1['n_levels']} levels")
        oracle.set_threads(threads_multi)
    return out


def bench_batch(args):
    """256 random SNNs (node counts log-uniform in [2048, 32768], |T_v| ~
    Poisson(mu)+1 with mu uniform in [32, 256], w in [1,16], seeds 4000+g),
    partitioned as one batch with the learned proposal (--plain: the plain
    method); the schedule is tuned once, on a 16-graph sample, before timing.
    --plain-steps > 0 adds one plain batch under its own tuned schedule, as
    the judge of the learned connectivity."""
    import numpy as np
    import torch

    # one line per finished graph and per tuned schedule (the batch calls are long)
    os.environ.setdefault("HGP_LOG_BATCH", "1")
    from paper_2604_14411_amd import hgp, synth

    t = time.perf_counter()
    gs = []
    for i in range(256):
        gs.append(synth.random_snn_family(4000 + i)[0])
        if i % 32 == 31:
            log(f"[bench] generated {i + 1} graphs")
    pins = sum(g.n_pins for g in gs)
    log(f"[bench] batch of {len(gs)} graphs, {pins} pins, generated in {time.perf_counter() - t:.1f} s")
    mlp = None
    if not args.plain:
        from paper_2604_14411_amd.learn import load_checkpoint

        mlp, _, _ = load_checkpoint(args.mlp)
    ctx = hgp.Context(0)
    dgs = [hgp.DeviceHypergraph(g, "cuda:0") for g in gs]
    outs = [torch.empty(max(g.n_nodes, 1), dtype=torch.int32, device="cuda:0") for g in gs]
    om, de = [1024] * len(gs), [4096] * len(gs)
    # tune on every 16th graph (16 graphs spanning the size range)
    sample = list(range(0, len(gs), 16))

    def tune(q):
        torch.cuda.synchronize()
        t = time.perf_counter()
        sched, tune_ms = hgp.batch_tune(ctx, [dgs[i] for i in sample], [om[i] for i in sample],
                                        [de[i] for i in sample], outs=[outs[i] for i in sample], mlp=q)
        log(f"[bench] tuned schedule {sched} ({tune_ms:.0f} ms for the 16-graph sample) in "
            f"{time.perf_counter() - t:.1f} s")
        return sched

    def timed(q, steps, tag):
        lat, done = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            _, res, ts, te = hgp.partition_batch_device(ctx, dgs, om, de, outs=outs, mlp=q)
            lat.append(te - ts)
            done.append(te)
            log(f"[bench] {tag} batch step {i}: {te.max():.0f} ms")
        torch.cuda.synchronize()
        return time.perf_counter() - t0, res, np.concatenate(lat), np.concatenate(done)

    sched = tune(mlp)
    elapsed, res, lat, done = timed(mlp, args.steps, "plain" if mlp is None else "learned")
    line = dict(metric="pins/s (sum |e| per second), batch of independent partitions", value=pins * args.steps / elapsed,
                unit="pins/s", n_gpus=1, steps=args.steps, warmup=0, ms_per_step=1e3 * elapsed / args.steps,
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="int32", data="synthetic",
                config=dict(workload="batch256", graphs=len(gs), pins=pins, omega=1024, delta=4096,
                            proposal="plain" if mlp is None else "learned", schedule=sched,
                            conn_sum=int(sum(r["connectivity"] for r in res)),
                            n_fallback=int(sum(r["n_fallback"] for r in res))),
                latency_ms=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                                completion_p50=float(np.percentile(done, 50)),
                                completion_p99=float(np.percentile(done, 99))))
    if mlp is not None and args.plain_steps > 0:
        psched = tune(None)
        pel, pres, _, _ = timed(None, 1, "plain")
        pconn = int(sum(r["connectivity"] for r in pres))
        line["learned_vs_plain"] = dict(plain=dict(value=pins / pel, ms_per_step=1e3 * pel, schedule=psched,
                                                   conn_sum=pconn),
                                        conn_ratio=line["config"]["conn_sum"] / pconn,
                                        speed_ratio=line["value"] / (pins / pel))
    print(json.dumps(line), flush=True)


DEFAULT_MLP = os.path.join(ROOT, "paper_2604_14411_amd", "mlp_v2.json")
METRIC = "pins/s (\u03a3|e|/s) partition throughput + connectivity, learned vs plain at \u03a9,\u0394"


def lds_probe():
    """The LDS atomic-add rate of the whole device (the peak that the ratings'
    and proposals' histograms are priced against): 512 workgroups of 1024
    threads, 8 adds per thread and iteration.  The counters are checked
    against their closed forms."""
    import ctypes

    import numpy as np
    import torch

    path = os.path.join(ROOT, "paper_2604_14411_amd", "libhgp_probe.so")
    if not os.path.exists(path):
        raise SystemExit(f"{path} is not built (python __graft_entry__.py build)")
    lib = ctypes.CDLL(path)
    lib.hgp_probe_lds_atomics.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_float)]
    lib.hgp_probe_lds_atomics.restype = ctypes.c_int
    grid, iters, words = 512, 8192, 8192
    out = torch.empty(grid * words, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    torch.cuda.synchronize()
    res = {}
    for random in (0, 1):
        ms = ctypes.c_float(0.0)
        best = None
        for _ in range(4):  # the first launch also loads the code object
            rc = lib.hgp_probe_lds_atomics(random, grid, iters, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream),
                                           ctypes.byref(ms))
            if rc != 0:
                raise SystemExit(f"hgp_probe_lds_atomics returned {rc}")
            best = ms.value if best is None else min(best, ms.value)
        cnt = out.cpu().numpy().view(np.uint32).reshape(grid, words)
        tri = (iters * (iters + 1) // 2) % 2**32
        if random:
            ok = bool(np.all(cnt.astype(np.uint64).sum(axis=1) % 2**32 == (words * tri) % 2**32))
        else:
            ok = bool(np.all(cnt == tri))
        ops = grid * 1024 * 8 * iters
        key = "random" if random else "conflict_free"
        res[key] = dict(ms=best, tops=ops / best / 1e9, frac=ops / best / 1e9 / LDS_ATOMIC_PEAK_TOPS, counters_ok=ok)
        log(f"[bench] LDS atomics {key}: {best:.3f} ms for {ops:.3e} adds, {ops / best / 1e9:.2f} T/s, counters ok={ok}")
    print(json.dumps(dict(probe="LDS atomic add (u32, no return)", grid=grid, threads=1024, iters=iters,
                          adds_per_launch=grid * 1024 * 8 * iters, peak_tops=LDS_ATOMIC_PEAK_TOPS, **res)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="conv302k")
    ap.add_argument("--plain", action="store_true", help="time the plain method only (no learned proposal)")
    ap.add_argument("--plain-steps", type=int, default=1,
                    help="timed runs of the plain method, the judge of the learned result, on the same input")
    ap.add_argument("--exact", action="store_true",
                    help="with --plain: the exact maximum-weight matching of the pairing pseudo-forest "
                         "instead of the two traversals")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, help="only copy this many bytes on the device (profiling)")
    ap.add_argument("--lds-probe", action="store_true",
                    help="only measure the device's LDS atomic-add rate (libhgp_probe.so), conflict-free and random")
    ap.add_argument("--mlp", default=DEFAULT_MLP, help="checkpoint of the learned proposal (paper_2604_14411_amd/learn.py)")
    args = ap.parse_args()
    if args.workload == "batch256":
        # one hardware queue per batch worker stream (HIP's default is 4);
        # set before the first HIP call of the process
        os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")
    if args.copy_probe:
        # a plain device-to-device copy of known size: reference for the HBM
        # byte counters (FETCH_SIZE / WRITE_SIZE) of a profiled kernel
        import torch

        a = torch.ones(args.copy_probe // 4, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_probe} bytes 3 times")
        # achieved copy bandwidth (read + write), HIP events on the copies' stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps(dict(probe="device copy", bytes=args.copy_probe, ms_per_copy=ms,
                              read_write_gbs=2 * args.copy_probe / ms / 1e6, peak_gbs=HBM_PEAK_GBS)))
        return
    if args.lds_probe:
        lds_probe()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X and has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_14411_amd import hgp
    from paper_2604_14411_amd.synth.configs import WORKLOADS

    if args.workload == "batch256":
        return bench_batch(args)

    w = WORKLOADS[args.workload]
    t = time.perf_counter()
    g = w.make()
    log(f"[bench] workload {w.name}: {w.note}; n={g.n_nodes} pins={g.n_pins} "
        f"(generated in {time.perf_counter() - t:.1f} s)")
    ctx = hgp.Context(0)
    dg = hgp.DeviceHypergraph(g, "cuda:0")
    out = torch.empty(g.n_nodes, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()

    match_flags = hgp.FLAG_EXACT_MATCHING if args.exact else 0
    if args.exact and not args.plain:
        log("[bench] --exact applies to the plain method: add --plain")
        sys.exit(2)

    def run(mlp, tag, warmup, steps, time_classes=0):
        for i in range(warmup):
            t = time.perf_counter()
            _, res = hgp.partition_device(ctx, dg, w.omega, w.delta, out=out, mlp=mlp, flags=match_flags)
            log(f"[bench] {tag} warmup {i}: {time.perf_counter() - t:.3f} s levels={res['n_levels']} "
                f"rounds={res['n_rounds']} parts={res['n_parts']} conn={res['connectivity']}")
        results = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            _, res = hgp.partition_device(ctx, dg, w.omega, w.delta, out=out,
                                          flags=hgp.FLAG_TIME_KERNELS | match_flags, mlp=mlp,
                                          time_classes=time_classes)
            results.append(res)
            log(f"[bench] {tag} step {i}: levels={res['n_levels']} rounds={res['n_rounds']} parts={res['n_parts']} "
                f"conn={res['connectivity']} fallback={res['n_fallback']}")
        torch.cuda.synchronize()
        return time.perf_counter() - t0, results

    def classes(results, steps, show):
        agg = {}
        for res in results:
            for name, k in res["kernels"].items():
                a = agg.setdefault(name, dict(ms=0.0, launches=0, units=0))
                a["ms"] += k["ms"]
                a["launches"] += k["launches"]
                a["units"] += k["units"]
        if show:
            for name, a in sorted(agg.items(), key=lambda kv: -kv[1]["ms"]):
                if a["launches"]:
                    log(f"[bench] kernel {name:11s} {a['ms'] / steps:9.2f} ms/step  launches/step "
                        f"{a['launches'] / steps:8.1f}  avg {a['ms'] / a['launches'] * 1e3:9.1f} us  "
                        f"units/step {a['units'] / steps:.3e}")
        return agg

    q = None
    if not args.plain:
        from paper_2604_14411_amd.learn import load_checkpoint

        q, _, _ = load_checkpoint(args.mlp)
    tag = "learned" if q is not None else "plain"
    # one untimed profiling run with every kernel class timed: the per-class
    # table and the dominant class.  The timed steps then record HIP events
    # around that class's launches only (events around every launch of every
    # class would slow the run down by a fifth).
    _, prof = run(q, f"{tag} (all classes timed, not in the timed region)", args.warmup, 1)
    log("[bench] kernel classes of one partition (every class timed):")
    pagg = classes(prof, 1, True)
    dom = max(pagg, key=lambda k: pagg[k]["ms"])
    dom_bit = 1 << hgp.KERNEL_CLASSES.index(dom)
    elapsed, results = run(q, tag, 0, args.steps, time_classes=dom_bit)
    ms_step = 1e3 * elapsed / args.steps
    value = g.n_pins * args.steps / elapsed
    plain_cmp = None
    if q is not None and args.plain_steps > 0:
        # the plain method on the same input: the judge of the learned result
        pel, pres = run(None, "plain", 0, args.plain_steps, time_classes=dom_bit)
        plain_cmp = dict(value=g.n_pins * args.plain_steps / pel, ms_per_step=1e3 * pel / args.plain_steps,
                         steps=args.plain_steps, connectivity=pres[-1]["connectivity"],
                         n_parts=pres[-1]["n_parts"], levels=pres[-1]["n_levels"], rounds=pres[-1]["n_rounds"])

    # the dominant class over the timed steps
    agg = classes(results, args.steps, False)
    a = agg[dom]
    bound, per_unit = COST[dom]
    avg_s = a["ms"] / a["launches"] / 1e3
    units_per_launch = a["units"] / a["launches"]
    if bound == "hbm":
        achieved = per_unit * units_per_launch / avg_s / 1e9
        tb = measured_traffic(dom)
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=None if tb is None else tb / avg_s / 1e9)
    else:
        achieved = per_unit * units_per_launch / avg_s / 1e12
        tb = measured_traffic(dom)
        roof = dict(bound="alu", achieved=achieved, peak=LDS_ATOMIC_PEAK_TOPS, unit="TOP/s",
                    frac=achieved / LDS_ATOMIC_PEAK_TOPS, traffic=None if tb is None else tb / avg_s / 1e9)
    roof.update(kernel=dom, traffic_unit="GB/s", avg_launch_us=avg_s * 1e6,
                launches_per_step=a["launches"] / args.steps,
                units_per_launch=units_per_launch, share_of_step=a["ms"] / args.steps / ms_step,
                classes_ms_per_step={k: round(v["ms"], 2) for k, v in sorted(pagg.items(), key=lambda kv: -kv[1]["ms"])
                                     if v["launches"]})

    line = dict(metric=METRIC, value=value, unit="pins/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                ms_per_step=ms_step, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="int32",
                data="synthetic",
                config=dict(workload=w.name, description=w.note, n_nodes=g.n_nodes, pins=g.n_pins,
                            sum_e_sq=g.sum_sq(), omega=w.omega, delta=w.delta, max_refine_rounds=8,
                            levels=results[-1]["n_levels"], rounds=results[-1]["n_rounds"],
                            n_parts=results[-1]["n_parts"], connectivity=results[-1]["connectivity"],
                            proposal="learned" if q is not None else "plain",
                            matching="exact" if args.exact else "two traversals"),
                roofline=roof)
    if plain_cmp:
        line["learned_vs_plain"] = dict(plain=plain_cmp, learned_connectivity=results[-1]["connectivity"],
                                        conn_ratio=results[-1]["connectivity"] / max(plain_cmp["connectivity"], 1),
                                        speed_ratio=value / plain_cmp["value"],
                                        n_fallback=results[-1]["n_fallback"], checkpoint=os.path.basename(args.mlp))
    if not args.no_cpu_baseline and w.sample is not None:
        log(f"[bench] cpu baseline: the oracle on {w.sample_note} ...")
        line["cpu_baseline"] = cpu_baseline(w, q, min(os.cpu_count() or 1, 16))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
